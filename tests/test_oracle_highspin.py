"""Pins the M_s = 1 high-spin oracle (oracle/highspin.py).

* brute force: the tensor residual equals <x| e^-T H e^T |T> of the determinant
  engine in the M_s = 1 sector, for random T (singles and doubles, both spins);
* two electrons: CCSD is exact, and DCSD too (its dropped terms vanish), so the
  converged energies equal the M_s = 1 FCI triplet, which is also the M_s = 0
  triplet root of the same spin-free Hamiltonian (and, on complete-active-space
  inputs, 2D-CCSD's E_T);
* first iteration: from T = 0 the residual gives the MP2-with-singles energy of
  Phi_T in closed form;
* size consistency: a non-interacting closed-shell two-electron fragment shifts
  the converged triplet energy by exactly its FCI correlation energy.
"""
import numpy as np
import pytest

import dcsd_synth as synth
from oracle.brute import DeterminantSpace
from oracle.ccsd import ccsd_residual
from oracle.hamiltonian import Hamiltonian
from oracle.highspin import HighSpin, HighSpinHamiltonian
from oracle.solver import solve
from oracle.twodet import TwoDet
from test_oracle_size_consistency import fragment_correlation


@pytest.mark.parametrize("nc,nv", [(0, 4), (1, 3), (2, 3)])
def test_residual_equals_similarity_transformed_projection(nc, nv):
    B, F = synth.make_inputs(nc, nv, 12, 17)
    ham = HighSpinHamiltonian(B, F, nc)
    vec = synth.hs_random_amplitudes(nc, nv, 23, 0.1)
    t1, t2 = ham.to_so(vec)
    ds = DeterminantSpace(ham)
    r1b, r2b = ds.projections(ds.connected(t1, t2))
    R1, R2 = ccsd_residual(ham, t1, t2)
    assert np.abs(R1 - r1b).max() < 1e-12
    assert np.abs(R2 - r2b).max() < 1e-12
    assert np.abs(r2b).max() > 0.05
    # the packed round trip keeps every independent amplitude
    assert np.array_equal(ham.from_so(t1, t2), vec)
    # E_ref is <T|H|T>
    assert abs(ham.e_ref() - ds.read_A(ds.apply_H(ds.vector(ds.mask_A())))) < 1e-12


@pytest.mark.parametrize("method", ["ccsd", "dcsd"])
@pytest.mark.parametrize("nv,seed", [(4, 3), (7, 5)])
def test_two_electrons_give_the_fci_triplet(method, nv, seed):
    B, F = synth.make_inputs(0, nv, 25, seed)
    ham = HighSpinHamiltonian(B, F, 0)
    ds = DeterminantSpace(ham)
    w, U = np.linalg.eigh(ds.H_matrix())
    k = int(np.argmax(np.abs(U[ds.index[ds.mask_A()]])))   # root of Phi_T
    r = solve(HighSpin(B, F, 0, method), tol=1e-11)
    assert r["converged"]
    assert abs(ham.e_ref() + r["E_T"] - w[k]) < 1e-10
    # the same energy is the M_s = 0 triplet root of the Hamiltonian
    _, ET0, _, _ = DeterminantSpace(Hamiltonian(B, F, 0)).fci_pair()
    assert abs(w[k] - ET0) < 1e-10
    assert abs(r["E_T"]) > 1e-4  # (same-spin pair: small but non-zero)


def test_cas_two_electrons_match_the_two_determinant_triplet():
    B, F, _ = synth.make_z2_inputs(0, 6, 24, 9)
    r_hs = solve(HighSpin(B, F, 0, "ccsd"), tol=1e-11)
    model = TwoDet(B, F, 0, "ccsd")
    r_2d = solve(model, tol=1e-11)
    e_hs = HighSpinHamiltonian(B, F, 0).e_ref() + r_hs["E_T"]
    e_2d = model.ham.e_ref() + r_2d["E_T"]
    assert abs(e_hs - e_2d) < 1e-10


def test_first_iteration_is_mp2_with_singles():
    B, F = synth.make_inputs(2, 6, 20, 6)
    model = HighSpin(B, F, 2, "dcsd")
    D = model.denominators()
    R0, _ = model.residual(np.zeros(model.size))
    T1 = R0 / D
    ham = model.ham
    O, V = ham.O, ham.V
    fov, oovv = ham.fock(O, V), ham.asym(O, O, V, V)
    fo, fv = np.diag(ham.fock(O, O)), np.diag(ham.fock(V, V))
    d1 = fo[:, None] - fv[None, :]
    d2 = fo[:, None, None, None] + fo[None, :, None, None] - fv[None, None, :, None] - fv[None, None, None, :]
    t1, t2 = fov / d1, oovv / d2
    e_closed = (np.sum(fov * t1) + 0.25 * np.sum(oovv * t2) + 0.5 * np.einsum("ijab,ia,jb->", oovv, t1, t1))
    assert abs(model.energy(T1) - e_closed) < 1e-13
    assert abs(e_closed) > 1e-3


@pytest.mark.parametrize("method", ["dcsd", "ccsd"])
def test_noninteracting_fragment_shifts_the_triplet_by_its_fci(method):
    nc, nv = 1, 4
    B, F = synth.make_inputs(nc, nv, 20, 7)
    r = solve(HighSpin(B, F, nc, method), tol=1e-11)
    B2, F2, nc2, frag = synth.add_fragment(B, F, nc, 3, 107)
    r2 = solve(HighSpin(B2, F2, nc2, method), tol=1e-11)
    assert r["converged"] and r2["converged"]
    ec = fragment_correlation(frag["B"], frag["F"])
    assert abs(r2["E_T"] - (r["E_T"] + ec)) < 1e-11
