"""Writes adjoint.json: oracle derivatives of the converged 2D-DCSD / 2D-CCSD
energies of the tiny configuration with respect to entries of B and F.

Each derivative is the linear response of the converged solution T*:
dT solves (dR/dT) dT = -(dR/dB) dB (GMRES, denominator-preconditioned, to
1e-11 of the preconditioned right-hand side, about its rounding floor), and dE = Im E(T* + i h dT; B + i h dB) / h.  Every product with a
derivative of the oracle's residual or energy is a complex-step derivative
(perturbation i*h, h = 1e-20, exact to rounding), taken at the converged real
amplitudes.  (Running the whole Jacobi/DIIS solve in complex arithmetic is
not used: near convergence the DIIS coefficients come from an ill-conditioned
Gram matrix and the imaginary part of the iterate keeps oscillating at the
1e-4 level after the real residual has converged.)  dB moves the mirrored
entries B[P,p,q] and B[P,q,p] by h/2 each (one entry by h on the diagonal),
so the value is the gradient with respect to a symmetric B[P] as the library
reports it.  Calls only oracle/, the input generator and SciPy's GMRES.

    python tests/golden/make_adjoint_golden.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import dcsd_synth as synth  # noqa: E402
from oracle.solver import solve  # noqa: E402
from oracle.twodet import TwoDet  # noqa: E402

H = 1e-20
TOL = 1e-13
ENTRY_SEED = 5


def entries(cfg):
    """Seeded B entries (p <= q) plus ones that touch t, u and a diagonal, and F entries."""
    rng = np.random.default_rng(ENTRY_SEED)
    n, nc = cfg.n, cfg.nc
    B = set()
    while len(B) < 9:
        P, p, q = int(rng.integers(cfg.naux)), int(rng.integers(n)), int(rng.integers(n))
        B.add((P, min(p, q), max(p, q)))
    B = sorted(B) + [(1, nc, nc + 1), (2, 0, nc + 2), (4, nc + 3, nc + 3)]
    F = [(nc, nc + 1), (0, 0), (1, nc + 3), (nc + 1, nc + 1)]
    return B, F


def direction(shape, idx):
    d = np.zeros(shape)
    if len(set(idx[-2:])) == 1:
        d[idx] = 1.0
    else:
        d[idx] = 0.5
        d[idx[:-2] + (idx[-1], idx[-2])] = 0.5
    return d


def linear_response(model, T, dB, dF, B0, F0, nc, method, rtol=1e-11):
    """(dE_S, dE_T) along (dB, dF) at converged amplitudes T of `model`."""
    from scipy.sparse.linalg import LinearOperator, gmres
    pert = TwoDet(B0 + 1j * H * dB, F0 + 1j * H * dF, nc, method)
    rhs = -np.imag(pert.residual(T)[0]) / H
    D = model.denominators()
    n = T.size
    A = LinearOperator((n, n), matvec=lambda x: np.imag(model.residual(T + 1j * H * x)[0]) / H, dtype=np.float64)
    M = LinearOperator((n, n), matvec=lambda x: -x / D, dtype=np.float64)
    dT, info = gmres(A, rhs, M=M, rtol=rtol, atol=0.0, restart=300, maxiter=5)
    assert info == 0, info
    res = np.abs(A @ dT - rhs).max()
    print(f"  true residual {res:.2e}, |rhs| {np.abs(rhs).max():.2e}", flush=True)
    assert res <= 1e-10 * np.abs(rhs).max()
    e = pert.energies(T + 1j * H * dT)
    return float(np.imag(e["E_S"]) / H), float(np.imag(e["E_T"]) / H)


def main():
    cfg = synth.TINY
    B0, F0 = synth.make_config_inputs(cfg)
    Bs, Fs = entries(cfg)
    out = {"config": {"nc": cfg.nc, "nv": cfg.nv, "naux": cfg.naux, "seed": cfg.seed},
           "h": H, "tol": TOL, "entry_seed": ENTRY_SEED}
    for method in ("dcsd", "ccsd"):
        model = TwoDet(B0, F0, cfg.nc, method)
        r = solve(model, tol=TOL, max_iter=400)
        assert r["converged"]
        rec = {"E_S": r["E_S"], "E_T": r["E_T"], "entries": []}
        for kind, lst in (("B", Bs), ("F", Fs)):
            for idx in lst:
                t0 = time.time()
                d = direction(B0.shape if kind == "B" else F0.shape, idx)
                dB, dF = (d, np.zeros_like(F0)) if kind == "B" else (np.zeros_like(B0), d)
                dS, dT = linear_response(model, r["T"], dB, dF, B0, F0, cfg.nc, method)
                rec["entries"].append({"kind": kind, "index": list(idx), "dE_S": dS, "dE_T": dT})
                print(method, kind, idx, dS, dT, f"{time.time() - t0:.1f}s", flush=True)
        out[method] = rec
    with open(os.path.join(HERE, "adjoint.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
