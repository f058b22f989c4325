"""Pins the tensor oracle to exact determinant algebra on small systems.

The determinant engine evaluates <A^x| e^-T H e^T |A>, <A^x| e^-T_A e^T_B |B>,
W and E_ref from their definitions; the tensor oracle must agree for random
amplitudes (including the internal t <-> u singles of the incomplete active
space case)."""
import numpy as np
import pytest

import dcsd_synth as synth
from oracle.brute import DeterminantSpace
from oracle.ccsd import ccsd_residual
from oracle.coupling import coupling
from oracle.fixedref import FixedRef
from oracle.hamiltonian import Hamiltonian
from oracle.twodet import TwoDet

CASES = [(0, 4), (1, 3), (2, 3)]


def _setup(nc, nv, seed=7):
    B, F = synth.make_inputs(nc, nv, 12, seed)
    ham = Hamiltonian(B, F, nc)
    vec = synth.random_amplitudes(nc, nv, seed + 4, scale=0.1)
    return B, F, ham, vec


@pytest.mark.parametrize("nc,nv", CASES)
def test_connected_residual_equals_similarity_transformed_projection(nc, nv):
    B, F, ham, vec = _setup(nc, nv)
    t1, t2 = ham.to_so(vec)
    ds = DeterminantSpace(ham)
    r1b, r2b = ds.projections(ds.connected(t1, t2))
    R1, R2 = ccsd_residual(ham, t1, t2)
    assert np.abs(R1 - r1b).max() < 1e-12
    assert np.abs(R2 - r2b).max() < 1e-12
    assert np.abs(r2b).max() > 0.1          # non-trivial


@pytest.mark.parametrize("nc,nv", CASES)
def test_coupling_equals_definition(nc, nv):
    B, F, ham, vec = _setup(nc, nv)
    t1, t2 = ham.to_so(vec)
    ds = DeterminantSpace(ham)
    k1, k2 = ds.projections(ds.coupling_vector(t1, t2))
    ref = ham.from_so(k1, k2)
    ref[ham.ab_packed_position()] = 0.0
    got = synth.pack(coupling(synth.unpack(vec, nc, nv), nc, nv), nc, nv)
    assert np.abs(got - ref).max() < 1e-13
    assert np.abs(ref).max() > 0.05


@pytest.mark.parametrize("nc,nv", CASES)
def test_W_and_reference_energy(nc, nv):
    B, F, ham, vec = _setup(nc, nv)
    t1, t2 = ham.to_so(vec)
    ds = DeterminantSpace(ham)
    y = ds.connected(t1, t2)
    model = TwoDet(B, F, nc, "ccsd")
    _, W = model.residual(vec)
    assert abs(W - ds.read_B(y)) < 1e-13
    a = ds.vector(ds.mask_A())
    assert abs(ham.e_ref() - ds.read_A(ds.apply_H(a))) < 1e-12
    # <A| e^-T H e^T |A> = E_ref + Delta E_A
    assert abs(ds.read_A(y) - ham.e_ref() - model.energy_A(vec)) < 1e-12


@pytest.mark.parametrize("nc,nv", CASES)
@pytest.mark.parametrize("state", ["singlet", "triplet"])
def test_fixed_reference_residual_and_energy_equal_projection(nc, nv, state):
    """Fixed reference: the projection of e^-T H e^T |A> with the A->B double
    held at +-1 (the element itself then set to zero), and <A| e^-T H e^T |A>."""
    B, F, ham, vec = _setup(nc, nv)
    model = FixedRef(B, F, nc, "ccsd", state)
    t1, t2 = ham.to_so(model.fixed(vec))
    ds = DeterminantSpace(ham)
    y = ds.connected(t1, t2)
    r1b, r2b = ds.projections(y)
    ref = ham.from_so(r1b, r2b)
    ref[model.ab] = 0.0
    R, W = model.residual(vec)
    assert W == 0.0
    assert np.abs(R - ref).max() < 1e-12
    assert abs(ds.read_A(y) - ham.e_ref() - model.energy_A(vec)) < 1e-12


def test_W_at_zero_amplitudes_is_exchange_integral():
    B, F = synth.make_inputs(2, 5, 20, 3)
    model = TwoDet(B, F, 2, "dcsd")
    _, W = model.residual(np.zeros(model.size))
    t, u = 2, 3
    assert abs(W - float(np.sum(B[:, t, u] ** 2))) < 1e-14


def test_spin_fock_closed_form():
    B, F = synth.make_inputs(3, 7, 25, 2)
    ham = Hamiltonian(B, F, 3)
    fa, fb = ham.spin_fock_closed_form()
    O, V = ham.O, ham.V
    allso = (np.concatenate([O[0], V[0]]), np.concatenate([O[1], V[1]]))
    f = ham.fock(allso, allso)
    sp, sm = allso
    for i in range(len(sp)):
        for j in range(len(sp)):
            if sm[i] != sm[j]:
                assert f[i, j] == 0.0
            else:
                ref = (fa if sm[i] == 0 else fb)[sp[i], sp[j]]
                assert abs(f[i, j] - ref) < 1e-13


def test_fci_states_are_pure_spin_states():
    B, F = synth.make_inputs(1, 3, 15, 9)
    ham = Hamiltonian(B, F, 1)
    ds = DeterminantSpace(ham)
    w, U = np.linalg.eigh(ds.H_matrix())
    s2 = np.einsum("kn,kn->n", U, ds.S2(U))
    allowed = np.array([0.0, 2.0, 6.0])     # S = 0, 1, 2 with M_s = 0
    assert np.all(np.min(np.abs(s2[:, None] - allowed[None, :]), axis=1) < 1e-9)
