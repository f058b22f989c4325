"""Pins the (T) oracle (oracle/triples.py) on the M_s = 1 high-spin reference.

* determinant engine: for random t1, t2 every numerator is a projection onto
  the triple excitations X of Phi_T, N^c = <X|H T2|Phi> - <X|F_ov T2|Phi> and
  N^c + N^d = <X|H (T1 + T2)|Phi>, so E_(T) and each of its three parts are
  sums over triple determinants that use no tensor formula;
* a planted sign error in the connected numerator fails that comparison;
* two electrons have no triples;
* the triple-by-triple sum (used for sampled checks of large inputs) equals
  the dense sum.
"""
import numpy as np
import pytest

import dcsd_synth as synth
from oracle.brute import DeterminantSpace
from oracle.highspin import HighSpin, HighSpinHamiltonian
from oracle.solver import solve
from oracle.triples import _integrals, numerators, triples_by_triple, triples_energy


def brute_parts(ham, t1, t2):
    """E_(T) parts as sums over the triple determinants of the reference."""
    ds = DeterminantSpace(ham)
    ref_mask = ds.mask_A()
    ref = ds.vector(ref_mask)
    occ = [ds.so(s, m) for s, m in zip(ham.occ_sp, ham.occ_spin)]
    vir = [ds.so(s, m) for s, m in zip(ham.vir_sp, ham.vir_spin)]
    zero1, zero2 = np.zeros_like(t1), np.zeros_like(t2)
    t2phi = ds.apply_T(ds.cluster_terms(zero1, t2, flip=False), ref)
    t12phi = ds.apply_T(ds.cluster_terms(t1, t2, flip=False), ref)
    h2 = ds.apply_H(t2phi)
    h12 = ds.apply_H(t12phi)
    fov = ham.fock(ham.O, ham.V)
    f2 = np.zeros_like(t2phi)
    for i, ki in enumerate(occ):
        for a, ka in enumerate(vir):
            if fov[i, a] != 0.0:
                f2 += fov[i, a] * (ds.ex(ka, ki, t2phi) + ds.ex(ki, ka, t2phi))
    fo = np.diag(ham.fock(ham.O, ham.O))
    fv = np.diag(ham.fock(ham.V, ham.V))
    e4 = e5 = edt = 0.0
    count = 0
    for x, mask in enumerate(ds.dets):
        mask = int(mask)
        holes = ref_mask & ~mask
        parts = mask & ~ref_mask
        if bin(holes).count("1") != 3:
            continue
        count += 1
        D = sum(fo[i] for i, k in enumerate(occ) if holes >> k & 1) - sum(fv[a] for a, k in enumerate(vir)
                                                                          if parts >> k & 1)
        nc = h2[x] - f2[x]
        e4 += nc * nc / D
        edt += nc * f2[x] / D
        e5 += nc * (h12[x] - h2[x]) / D
    return {"E_T4": e4, "E_ST5": e5, "E_DT": edt, "E_T": e4 + e5 + edt, "triples": count}


@pytest.mark.parametrize("nc,nv,seed", [(1, 3, 5), (2, 3, 7), (1, 4, 11)])
def test_parts_equal_projections_on_triple_determinants(nc, nv, seed):
    B, F = synth.make_inputs(nc, nv, 14, seed)
    ham = HighSpinHamiltonian(B, F, nc)
    t1, t2 = ham.to_so(synth.hs_random_amplitudes(nc, nv, seed + 1, 0.1))
    ref = brute_parts(ham, t1, t2)
    got = triples_energy(ham, t1, t2)
    assert ref["triples"] > 0
    for k in ("E_T4", "E_ST5", "E_DT", "E_T"):
        assert abs(got[k] - ref[k]) <= 1e-13 + 1e-11 * abs(ref[k]), (k, got[k], ref[k])
    assert abs(ref["E_T4"]) > 1e-6 and abs(ref["E_ST5"]) > 1e-8 and abs(ref["E_DT"]) > 1e-8


def test_planted_sign_error_is_caught():
    nc, nv = 1, 4
    B, F = synth.make_inputs(nc, nv, 14, 3)
    ham = HighSpinHamiltonian(B, F, nc)
    t1, t2 = ham.to_so(synth.hs_random_amplitudes(nc, nv, 4, 0.1))
    ref = brute_parts(ham, t1, t2)
    g = _integrals(ham)
    g["ovoo"] = -g["ovoo"]   # wrong sign of the sum over m
    ncv, d1, d2, D = numerators(ham, t1, t2, g)
    with np.errstate(divide="ignore", invalid="ignore"):
        w = np.where(np.abs(ncv) > 0.0, ncv / D, 0.0)
    e4 = float(np.sum(w * ncv)) / 36.0
    assert abs(e4 - ref["E_T4"]) > 1e-3 * abs(ref["E_T4"])


def test_two_electrons_have_no_triples():
    B, F = synth.make_inputs(0, 5, 14, 2)
    ham = HighSpinHamiltonian(B, F, 0)
    t1, t2 = ham.to_so(synth.hs_random_amplitudes(0, 5, 3, 0.1))
    assert triples_energy(ham, t1, t2)["E_T"] == 0.0
    assert brute_parts(ham, t1, t2)["triples"] == 0


def test_triple_by_triple_sum_equals_dense_sum():
    nc, nv = 2, 6
    B, F = synth.make_inputs(nc, nv, 20, 8)
    model = HighSpin(B, F, nc, "ccsd")
    r = solve(model, tol=1e-10)
    assert r["converged"]
    t1, t2 = model.ham.to_so(r["T"])
    dense = triples_energy(model.ham, t1, t2)["E_T"]
    assert abs(triples_by_triple(model.ham, t1, t2) - dense) <= 1e-14 + 1e-12 * abs(dense)
    assert abs(dense) > 1e-6
    # the direct form (integrals of the three orbitals only) gives the same per-triple sums
    from oracle.triples import triple_contribution
    for ijk in ((0, 1, 2), (1, 4, 5), (3, 4, 5), (0, 2, 5)):
        a = triple_contribution(model.ham, t1, t2, *ijk)
        b = triple_contribution(model.ham, t1, t2, *ijk, direct=True)
        assert abs(a - b) <= 1e-15 + 1e-12 * abs(a)
