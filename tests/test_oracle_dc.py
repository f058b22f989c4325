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


@pytest.mark.parametrize("nc,nv,seed", [(2, 5, 5), (3, 4, 6)])
def test_quadratic_terms_are_the_ccsd_t2_t2_part(nc, nv, seed):
    """Beyond two electrons: with T1 = 0 the CCSD doubles residual is quadratic in T2,
    so R(2t) - 2R(t) + R(0) = 2 (its T2*T2 part), and that part is Q_a + Q_b + Q_c + Q_d.
    The CCSD residual is pinned to brute force, so this ties the four terms the DC
    selection splits to the exact equations where an index or factor error in one of
    them need not show with two electrons; a planted half factor in Q_c fails it."""
    from oracle.ccsd import SlabSource, ccsd_residual, integrals
    B, F = synth.make_inputs(nc, nv, 20, seed)
    ham = Hamiltonian(B, F, nc)
    ints, slabs = integrals(ham), SlabSource(ham)
    vec = synth.random_amplitudes(nc, nv, seed + 20, 0.1)
    blocks = synth.unpack(vec, nc, nv)
    blocks["t1a"][:] = 0.0
    blocks["t1b"][:] = 0.0
    t1, t2 = ham.to_so(vec)
    R2 = lambda s: ccsd_residual(ham, t1, s * t2, ints, slabs)[1]  # noqa: E731
    quad = 0.5 * (R2(2.0) - 2.0 * R2(1.0) + R2(0.0))
    q = quadratic_terms(ints["oovv"], ham.direct(ham.O, ham.O, ham.V, ham.V), t2)
    total = q["Qa"] + q["Qb"] + q["Qc"] + q["Qd"]
    assert np.abs(total).max() > 1e-3
    assert np.abs(quad - total).max() < 1e-12
    planted = q["Qa"] + q["Qb"] + 0.5 * q["Qc"] + q["Qd"]
    assert np.abs(quad - planted).max() > 1e-4
