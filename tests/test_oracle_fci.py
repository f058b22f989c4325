"""Pins the full 2D equations: two-electron FCI, MP2 start, invariances."""
import numpy as np
import pytest

import dcsd_synth as synth
from oracle.brute import DeterminantSpace
from oracle.hamiltonian import Hamiltonian
from oracle.solver import solve
from oracle.twodet import TwoDet


@pytest.mark.parametrize("method", ["ccsd", "dcsd"])
@pytest.mark.parametrize("nv", [4, 7])
def test_two_electron_cas_equals_fci(method, nv):
    """Complete active space (t, u in different irreps): 2D-CC is exact for
    two electrons, and so is 2D-DC (its dropped terms vanish)."""
    B, F, _ = synth.make_z2_inputs(0, nv, 30, 4 + nv)
    ham = Hamiltonian(B, F, 0)
    ES, ET, _, _ = DeterminantSpace(ham).fci_pair()
    r = solve(TwoDet(B, F, 0, method), tol=1e-11)
    assert r["converged"]
    eref = ham.e_ref()
    assert abs(eref + r["E_S"] - ES) < 1e-10
    assert abs(eref + r["E_T"] - ET) < 1e-10
    assert abs(r["W"]) > 1e-3


def test_cas_internal_singles_vanish():
    B, F, _ = synth.make_z2_inputs(2, 6, 24, 5)
    r = solve(TwoDet(B, F, 2, "dcsd"), tol=1e-10)
    assert r["converged"]
    blk = synth.unpack(r["T"], 2, 6)
    assert abs(blk["t1a"][2, 0]) < 1e-14 and abs(blk["t1b"][2, 0]) < 1e-14


def test_first_iteration_is_mp2_with_singles():
    B, F = synth.make_inputs(2, 6, 20, 6)
    model = TwoDet(B, F, 2, "dcsd")
    D = model.denominators()
    R0, W0 = model.residual(np.zeros(model.size))
    T1 = R0 / D
    ham = model.ham
    O, V = ham.O, ham.V
    fov = ham.fock(O, V)
    oovv = ham.asym(O, O, V, V)
    fo, fv = np.diag(ham.fock(O, O)), np.diag(ham.fock(V, V))
    d1 = fo[:, None] - fv[None, :]
    d2 = fo[:, None, None, None] + fo[None, :, None, None] - fv[None, None, :, None] - fv[None, None, None, :]
    t1 = fov / d1
    t2 = oovv / d2
    i, j, a, b = ham.ab_index()
    for (p, q, r, s) in ((i, j, a, b), (j, i, b, a)):
        t2[p, q, r, s] = 0.0
    for (p, q, r, s) in ((j, i, a, b), (i, j, b, a)):
        t2[p, q, r, s] = 0.0
    e_closed = (np.sum(fov * t1) + 0.25 * np.sum(oovv * t2)
                + 0.5 * np.einsum("ijab,ia,jb->", oovv, t1, t1))
    assert abs(model.energy_A(T1) - e_closed) < 1e-13
    assert abs(W0 - float(np.sum(B[:, 2, 3] ** 2))) < 1e-14


def _small(seed=11, nc=2, nv=6, naux=24):
    return synth.make_inputs(nc, nv, naux, seed)


def test_reference_choice_invariance():
    """Choosing Phi_B instead of Phi_A (swap t and u) changes nothing."""
    nc, nv = 2, 6
    B, F = _small()
    perm = np.arange(nc + 2 + nv)
    perm[nc], perm[nc + 1] = nc + 1, nc
    B2, F2 = B[:, perm][:, :, perm], F[np.ix_(perm, perm)]
    for method in ("dcsd", "ccsd"):
        r1 = solve(TwoDet(B, F, nc, method), tol=1e-11)
        r2 = solve(TwoDet(B2, F2, nc, method), tol=1e-11)
        assert r1["converged"] and r2["converged"]
        assert abs(r1["E_S"] - r2["E_S"]) < 1e-9
        assert abs(r1["E_T"] - r2["E_T"]) < 1e-9
        # the amplitudes of the swapped run are the spin flip of the original
        a, b = synth.unpack(r1["T"], nc, nv), synth.unpack(r2["T"], nc, nv)
        assert np.abs(a["t1a"] - b["t1b"]).max() < 1e-8
        assert np.abs(a["t2aa"] - b["t2bb"]).max() < 1e-8
        assert np.abs(a["t2ab"] - b["t2ab"].transpose(1, 0, 3, 2)).max() < 1e-8


def test_orbital_rotation_invariance():
    """Energies are invariant under rotations among core and among virtual
    orbitals (the open-shell orbitals stay fixed)."""
    nc, nv = 2, 6
    B, F = _small(seed=12)
    n = nc + 2 + nv
    rng = np.random.default_rng(3)
    U = np.eye(n)
    for blk in (np.arange(nc), np.arange(nc + 2, n)):
        Q, _ = np.linalg.qr(rng.normal(size=(len(blk), len(blk))))
        U[np.ix_(blk, blk)] = Q
    B2 = np.einsum("pi,Ppq,qj->Pij", U, B, U)
    F2 = U.T @ F @ U
    for method in ("dcsd", "ccsd"):
        r1 = solve(TwoDet(B, F, nc, method), tol=1e-11)
        r2 = solve(TwoDet(B2, F2, nc, method), tol=1e-11)
        assert r1["converged"] and r2["converged"]
        assert abs(r1["E_S"] - r2["E_S"]) < 1e-9
        assert abs(r1["E_T"] - r2["E_T"]) < 1e-9


def test_fixed_point_independent_of_solver_settings():
    B, F = _small(seed=13)
    a = solve(TwoDet(B, F, 2, "dcsd"), tol=1e-11)
    b = solve(TwoDet(B, F, 2, "dcsd"), tol=1e-11, diis_dim=4, shift=0.3)
    assert a["converged"] and b["converged"]
    assert np.abs(a["T"] - b["T"]).max() < 1e-9
    assert abs(a["E_S"] - b["E_S"]) < 1e-10


def test_residual_symmetries():
    B, F = _small(seed=14)
    model = TwoDet(B, F, 2, "dcsd")
    R, _ = model.residual(synth.random_amplitudes(2, 6, 3, 0.05))
    blk = synth.unpack(R, 2, 6)
    for k in ("t2aa", "t2bb"):
        assert np.abs(blk[k] + blk[k].transpose(1, 0, 2, 3)).max() < 1e-15
        assert np.abs(blk[k] + blk[k].transpose(0, 1, 3, 2)).max() < 1e-15
    assert blk["t2ab"][2, 2, 0, 0] == 0.0


def _antisym_unit(model, x):
    """Unit perturbation of packed element x respecting the antisymmetry of
    same-spin doubles."""
    nc, nv = model.nc, model.nv
    blk = synth.block_offsets(nc, nv)
    e = np.zeros(model.size)
    for name in ("t2aa", "t2bb"):
        off, shp = blk[name]
        if off <= x < off + int(np.prod(shp)):
            i, j, a, b = np.unravel_index(x - off, shp)
            for (p, q, r, s_, sg) in ((i, j, a, b, 1), (j, i, a, b, -1), (i, j, b, a, -1), (j, i, b, a, 1)):
                e[off + np.ravel_multi_index((p, q, r, s_), shp)] = sg
            return e
    e[x] = 1.0
    return e


@pytest.mark.parametrize("method", ["ccsd", "dcsd"])
def test_en_shift_is_the_jacobian_diagonal(method):
    """The Epstein-Nesbet preconditioner equals the diagonal of dR/dT at T = 0
    (coupling and DC terms are quadratic or higher there), checked by central
    differences on random elements of every block."""
    B, F = synth.make_inputs(2, 4, 12, 3)
    m = TwoDet(B, F, 2, method)
    D, s = m.denominators(), m.en_shift()
    rng = np.random.default_rng(0)
    h = 1e-5
    for name, (off, shp) in synth.block_offsets(2, 4).items():
        for x in off + rng.choice(int(np.prod(shp)), 8, replace=False):
            if x == m.ab:
                continue
            if name in ("t2aa", "t2bb"):
                i, j, a, b = np.unravel_index(x - off, shp)
                if i == j or a == b:
                    continue
            e = _antisym_unit(m, x) * h
            d = (m.connected(e)[x] - m.connected(-e)[x]) / (2 * h)
            assert abs(d - (-D[x] + s[x])) < 1e-8
