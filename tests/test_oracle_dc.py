"""Pins the distinguishable-cluster term selection.

For any two-electron system (occupied spin-orbitals 0 and 1) and any T2 the
four CCSD quadratic doubles terms reduce to closed forms in
E = 1/2 sum_cd <01||cd> t^cd and B_ab = sum_cd <01||cd> t^ac t^bd:
Q_a = E t, Q_b = 2B with a direct half B, Q_c = -2E t, Q_d = -2B.  A dropped
term, a wrong factor, sign or index in any Q fails one of these, and the DC
selection (drop Q_a + Q_b(exch) + Q_c/2 + Q_d/2) must vanish identically."""
import numpy as np
import pytest

import dcsd_synth as synth
from oracle.dc import dropped_terms, quadratic_terms
from oracle.hamiltonian import Hamiltonian


@pytest.mark.parametrize("nv,seed", [(3, 1), (6, 2), (9, 3)])
def test_two_electron_closed_forms(nv, seed):
    B, F = synth.make_inputs(0, nv, 20, seed)
    ham = Hamiltonian(B, F, 0)
    vec = synth.random_amplitudes(0, nv, seed + 10, 0.2)
    _, t2 = ham.to_so(vec)
    O, V = ham.O, ham.V
    Ia = ham.asym(O, O, V, V)
    q = quadratic_terms(Ia, ham.direct(O, O, V, V), t2)
    t = t2[0, 1]
    E = 0.5 * np.einsum("cd,cd->", Ia[0, 1], t)
    Bm = np.einsum("cd,ac,bd->ab", Ia[0, 1], t, t)
    tol = 1e-14
    assert np.abs(q["Qa"][0, 1] - E * t).max() < tol
    assert np.abs(q["Qb"][0, 1] - 2 * Bm).max() < tol
    assert np.abs(q["Qb_dir"][0, 1] - Bm).max() < tol
    assert np.abs(q["Qc"][0, 1] + 2 * E * t).max() < tol
    assert np.abs(q["Qd"][0, 1] + 2 * Bm).max() < tol
    assert np.abs(dropped_terms(ham, t2)).max() < tol
    assert np.abs(Bm).max() > 1e-3 and abs(E) > 1e-3


def test_dropped_terms_nonzero_beyond_two_electrons():
    B, F = synth.make_inputs(2, 5, 20, 4)
    ham = Hamiltonian(B, F, 2)
    _, t2 = ham.to_so(synth.random_amplitudes(2, 5, 8, 0.1))
    D = dropped_terms(ham, t2)
    assert np.abs(D).max() > 1e-3
    # antisymmetric like any doubles residual
    assert np.abs(D + D.swapaxes(0, 1)).max() < 1e-15
    assert np.abs(D + D.swapaxes(2, 3)).max() < 1e-15
