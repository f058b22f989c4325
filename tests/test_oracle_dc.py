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


def _closed_shell_problem(no: int, nv: int, seed: int):
    """A closed-shell system in spin orbitals, written out from the definitions:
    spatial integrals (pq|rs) = sum_P B[P,p,q] B[P,r,s] with B symmetric in p,q;
    spin-orbital lists occ = [alpha 0..no-1, beta 0..no-1], vir likewise;
    <kl|cd> = (kc|ld) delta(s_k,s_c) delta(s_l,s_d).  The spin-orbital doubles of a
    closed-shell state follow from one spatial T with T_ij^ab = T_ji^ba:
    t(i s, j s', a s, b s') = T_ij^ab and t(i s, j s', a s', b s) = -T_ij^ba."""
    rng = np.random.default_rng(seed)
    n = no + nv
    B = rng.normal(0.0, 0.3, (12, n, n))
    B = B + B.transpose(0, 2, 1)
    ovov = np.einsum("Pkc,Pld->kcld", B[:, :no, no:], B[:, :no, no:])
    T = rng.normal(0.0, 0.1, (no, no, nv, nv))
    T = T + T.transpose(1, 0, 3, 2)
    so = np.array([0] * no + [1] * no)
    sv = np.array([0] * nv + [1] * nv)
    occ = np.concatenate([np.arange(no), np.arange(no)])
    vir = np.concatenate([np.arange(nv), np.arange(nv)])
    direct = (ovov[occ][:, vir][:, :, occ][:, :, :, vir].transpose(0, 2, 1, 3)
              * (so[:, None, None, None] == sv[None, None, :, None])
              * (so[None, :, None, None] == sv[None, None, None, :]))
    asym = direct - direct.transpose(0, 1, 3, 2)
    same = lambda x, y: (x[:, None] == y[None, :])  # noqa: E731
    t2 = (T[occ][:, occ][:, :, vir][:, :, :, vir]
          * same(so, sv)[:, None, :, None] * same(so, sv)[None, :, None, :]
          - T[occ][:, occ][:, :, vir][:, :, :, vir].transpose(0, 1, 3, 2)
          * same(so, sv)[:, None, None, :] * same(so, sv)[None, :, :, None])
    return T, ovov, direct, asym, t2


class _ClosedShellIntegrals:
    """The two integral lists dropped_terms reads, for the closed-shell system."""

    def __init__(self, direct, asym):
        self._d, self._a = direct, asym
        self.O = self.V = None

    def direct(self, *_):
        return self._d

    def asym(self, *_):
        return self._a


@pytest.mark.parametrize("no,nv,seed", [(3, 4, 1), (4, 5, 2)])
def test_closed_shell_reduction_fixes_the_kept_ring(no, nv, seed):
    """Beyond two electrons: on a closed-shell state the T2*T2 part of the DCSD doubles
    residual must reduce to the closed-shell distinguishable-cluster form, with the
    contravariant amplitudes T~_ij^ab = 2 T_ij^ab - T_ij^ba and only Coulomb-type
    (kc|ld) integrals joining the two amplitudes, each term symmetrised by
    P(ia,jb) X_ij^ab = X_ij^ab + X_ji^ba:

        1/2 P(ia,jb) [ sum T~_ik^ac (kc|ld) T~_lj^db            (the direct ring)
                      - sum T~_il^cd (kc|ld) T_kj^ab            (half the hole Fock-like term)
                      - sum T~_kl^ca (kc|ld) T_ij^db ]          (half the particle one)

    while CCSD also has sum (kc|ld) T_ij^cd T_kl^ab and the exchange ring.  The
    two-electron identities cannot tell the direct ring from the exchange one (both
    equal B there); this reduction can: keeping the exchange half of Q_b instead
    gives a different closed-shell form, so a swap in the DC selection fails here."""
    T, ovov, direct, asym, t2 = _closed_shell_problem(no, nv, seed)
    q = quadratic_terms(asym, direct, t2)
    dropped = dropped_terms(_ClosedShellIntegrals(direct, asym), t2)
    kept = q["Qa"] + q["Qb"] + q["Qc"] + q["Qd"] - dropped
    ab = lambda X: X[:no, no:, :nv, nv:]  # noqa: E731  alpha-beta block
    aa = lambda X: X[:no, :no, :nv, :nv]  # noqa: E731

    Tt = 2.0 * T - T.transpose(0, 1, 3, 2)
    sym = lambda X: X + X.transpose(1, 0, 3, 2)  # noqa: E731  P(ia,jb)
    ring = np.einsum("ikac,kcld,ljdb->ijab", Tt, ovov, Tt)
    hole = np.einsum("ilcd,kcld,kjab->ijab", Tt, ovov, T)
    part = np.einsum("klca,kcld,ijdb->ijab", Tt, ovov, T)
    expect = 0.5 * sym(ring - hole - part)
    scale = np.abs(expect).max()
    assert scale > 1e-2
    assert np.abs(ab(kept) - expect).max() < 1e-13 * scale
    # the same-spin block is the antisymmetrised opposite-spin one (a singlet)
    assert np.abs(aa(kept) - (ab(kept) - ab(kept).transpose(0, 1, 3, 2))).max() < 1e-13 * scale
    # the direct half of Q_b alone is the closed-shell ring
    assert np.abs(ab(q["Qb_dir"]) - 0.5 * sym(ring)).max() < 1e-13 * scale
    # planted swap: keep the exchange half of Q_b and drop the direct one
    swapped = q["Qa"] + q["Qb"] + q["Qc"] + q["Qd"] - (q["Qa"] + q["Qb_dir"] + 0.5 * q["Qc"] + 0.5 * q["Qd"])
    assert np.abs(ab(swapped) - expect).max() > 1e-2 * scale
    # and CCSD: the full four terms carry the (kc|ld) T_ij^cd T_kl^ab ladder-like term
    assert np.abs(ab(q["Qa"]) - np.einsum("ijcd,kcld,klab->ijab", T, ovov, T)).max() < 1e-13 * scale
