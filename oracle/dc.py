"""Distinguishable-cluster modification of the doubles equations (oracle).

The paper applies the DC approximation to the single-reference doubles
equations "in the usual way" and leaves the coupling (M) terms unchanged
(Theory section).  The usual way keeps the singles through the T1-dressed
Hamiltonian and changes only the quadratic T2*T2 terms, which use the
<kl||cd> integrals (unchanged by T1 dressing).  In spin-orbital form the
CCSD doubles contain the four quadratic terms

    Q_a =  1/4        sum <kl||cd> t_ij^cd t_kl^ab
    Q_b =  P(ij)      sum <kl||cd> t_ik^ac t_jl^bd
    Q_c = -1/2 P(ij)  sum <kl||cd> t_ik^dc t_lj^ab
    Q_d = -1/2 P(ab)  sum <kl||cd> t_lk^ac t_ij^db

and Q_b splits into a direct part (with <kl|cd> = (kc|ld)) and an exchange
part.  DCSD keeps Q_b(direct), 1/2 Q_c and 1/2 Q_d and drops the rest:

    dropped = Q_a + Q_b(exchange) + 1/2 Q_c + 1/2 Q_d.

This is the one selection that keeps particle-hole symmetry (Q_c and Q_d
treated alike), keeps only the direct ring, and stays exact for any
two-electron system (where Q_a = E t, Q_b = 2B, Q_c = -2E t, Q_d = -2B, so the
dropped terms cancel).  The reading is listed among the readings of the
paper in the design notes.

Pinned by: the dropped terms vanish identically for every two-electron
input and random T2, and beyond two electrons the four terms add up to the
T2*T2 part of the CCSD residual (tests/test_oracle_dc.py); on a closed-shell
state the kept T2*T2 terms reduce to the closed-shell distinguishable-cluster
form (Coulomb-type (kc|ld) only, contravariant 2T - T^T amplitudes, the direct
ring whole and the two Fock-like terms halved), which fixes which half of Q_b
is kept; converged 2D-DCSD reproduces two-electron FCI and is size consistent
(tests/test_oracle_size_consistency.py).
"""
from __future__ import annotations

import numpy as np

from .ccsd import p_ab, p_ij
from .hamiltonian import Hamiltonian

es = lambda *a: np.einsum(*a, optimize=True)  # noqa: E731


def quadratic_terms(I_asym: np.ndarray, I_direct: np.ndarray, t2: np.ndarray) -> dict:
    """The four CCSD T2*T2 doubles terms and the direct half of Q_b."""
    Qa = 0.25 * es("ijkl,klab->ijab", es("klcd,ijcd->ijkl", I_asym, t2), t2)
    Qb = p_ij(es("ikac,jlbd,klcd->ijab", t2, t2, I_asym))
    Qb_dir = p_ij(es("ikac,jlbd,klcd->ijab", t2, t2, I_direct))
    Qc = -0.5 * p_ij(es("ikdc,klcd,ljab->ijab", t2, I_asym, t2))
    Qd = -0.5 * p_ab(es("lkac,klcd,ijdb->ijab", t2, I_asym, t2))
    return {"Qa": Qa, "Qb": Qb, "Qb_dir": Qb_dir, "Qc": Qc, "Qd": Qd}


def dropped_terms(ham: Hamiltonian, t2: np.ndarray, I_asym: np.ndarray | None = None) -> np.ndarray:
    """D(T2) = Q_a + Q_b(exchange) + 1/2 Q_c + 1/2 Q_d (spin-orbital doubles)."""
    O, V = ham.O, ham.V
    Ia = I_asym if I_asym is not None else ham.asym(O, O, V, V)
    Id = ham.direct(O, O, V, V)
    q = quadratic_terms(Ia, Id, t2)
    return q["Qa"] + (q["Qb"] - q["Qb_dir"]) + 0.5 * q["Qc"] + 0.5 * q["Qd"]
