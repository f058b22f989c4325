"""Jacobi + DIIS amplitude iterations (oracle).

The paper does not describe its solver; any solver that drives the residual
to zero reaches the same amplitudes.  The one used on both sides:

* start from T = 0;
* iteration k: R = residual(T); stop if max|R| <= tol;
  T_new = T + R / (D - s - shift)   (no step where R = 0 exactly; D = f_ii + f_jj - f_aa - f_bb from the
  diagonal of the reference Fock matrix; s = 0, or with
  ``precond="en"`` the two-electron (Epstein-Nesbet) part of the diagonal of
  dR/dT at T = 0; shift >= 0 only damps the step);
* Pulay DIIS on (T_new, e = T_new - T) with at most ``diis_dim`` vectors,
  used once ``k >= diis_start``: minimise |sum c_i e_i| with sum c_i = 1 and
  take T = sum c_i T_new_i.

Besides the last step's T the result holds ``T_best``, the evaluated amplitudes
with the smallest max |R|, which is what the device solver returns when it
does not converge.

The fixed point does not depend on the shift or on the DIIS settings; the
iteration path does, so per-iteration comparisons use the same settings.
"""
from __future__ import annotations

import numpy as np


def diis_coefficients(errors) -> np.ndarray:
    m = len(errors)
    Bm = np.empty((m + 1, m + 1), np.result_type(*errors))
    for i in range(m):
        for j in range(i + 1):
            Bm[i, j] = Bm[j, i] = np.dot(errors[i], errors[j])  # no conjugation (complex-step safe)
    Bm[m, :m] = Bm[:m, m] = -1.0
    Bm[m, m] = 0.0
    rhs = np.zeros(m + 1)
    rhs[m] = -1.0
    return np.linalg.solve(Bm, rhs)[:m]


def solve(model, tol: float = 1e-10, max_iter: int = 200, diis_dim: int = 8,
          diis_start: int = 2, shift: float = 0.0, precond: str = "mp", T0=None, callback=None) -> dict:
    D = model.denominators() - shift
    if precond == "en":
        D = D - model.en_shift()
    T = np.zeros(model.size) if T0 is None else np.array(T0, dtype=np.float64)
    hist_T, hist_e, records = [], [], []
    converged = False
    T_best, best = None, None  # the evaluated amplitudes with the smallest max |R|
    for it in range(max_iter):
        R, W = model.residual(T)
        rmax = float(np.max(np.abs(R)))
        e = model.energies(T, W)
        rec = {"iter": it, "res_max": rmax, **e}
        records.append(rec)
        if np.isfinite(rmax) and (best is None or rmax < best["res_max"]):
            T_best, best = T.copy(), rec
        if callback is not None:
            callback(rec)
        if not np.isfinite(rmax):
            break
        if rmax <= tol:
            converged = True
            break
        # an element with R = 0 exactly takes no step: the A->B double, whose
        # residual is zero by definition and whose Epstein-Nesbet denominator
        # vanishes as well (both determinants have the same diagonal)
        Tn = T + np.divide(R, D, out=np.zeros_like(R), where=R != 0.0)
        err = Tn - T
        if diis_dim > 0:
            hist_T.append(Tn)
            hist_e.append(err)
            if len(hist_T) > diis_dim:
                hist_T.pop(0)
                hist_e.pop(0)
            if it >= diis_start and len(hist_T) >= 2:
                c = diis_coefficients(hist_e)
                Tn = sum(ci * ti for ci, ti in zip(c, hist_T))
        T = Tn
    return {"T": T, "converged": converged, "iterations": len(records), "records": records,
            "T_best": T_best, "best": best, **records[-1]}
