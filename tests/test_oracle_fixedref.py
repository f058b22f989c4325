"""Pins the fixed-reference (FR-CCSD / FR-DCSD) oracle: two-electron FCI in a
complete active space, and the energy of the fixed amplitude alone."""
import numpy as np
import pytest

import dcsd_synth as synth
from oracle.brute import DeterminantSpace
from oracle.fixedref import FixedRef
from oracle.hamiltonian import Hamiltonian
from oracle.solver import solve
from oracle.twodet import TwoDet


@pytest.mark.parametrize("method", ["ccsd", "dcsd"])
@pytest.mark.parametrize("nv", [4, 7])
def test_two_electron_cas_fixed_reference_equals_fci(method, nv):
    """With t and u in different irreps the internal singles vanish, so the
    coefficient of Phi_B is the fixed amplitude itself; the exact singlet has
    it equal to that of Phi_A and the triplet opposite.  CC (and DC, whose
    dropped terms vanish for two electrons) is exact for the other amplitudes."""
    B, F, _ = synth.make_z2_inputs(0, nv, 30, 4 + nv)
    ham = Hamiltonian(B, F, 0)
    ES, ET, _, _ = DeterminantSpace(ham).fci_pair()
    rs = solve(FixedRef(B, F, 0, method, "singlet"), tol=1e-11)
    rt = solve(FixedRef(B, F, 0, method, "triplet"), tol=1e-11)
    assert rs["converged"] and rt["converged"]
    eref = ham.e_ref()
    assert abs(eref + rs["E_S"] - ES) < 1e-10
    assert abs(eref + rt["E_T"] - ET) < 1e-10
    assert np.isnan(rs["E_T"]) and np.isnan(rt["E_S"]) and rs["W"] == 0.0
    # the same states as 2D-CC, reached without the coupling terms
    r2 = solve(TwoDet(B, F, 0, method), tol=1e-11)
    assert abs(r2["E_S"] - rs["E_S"]) < 1e-10 and abs(r2["E_T"] - rt["E_T"]) < 1e-10


def test_fixed_amplitude_alone_gives_plus_minus_exchange_integral():
    """At T = 0 apart from the fixed double, Delta E = +-<t u||u t> = +-(tu|ut)."""
    B, F = synth.make_inputs(2, 5, 20, 3)
    t, u = 2, 3
    K = float(np.sum(B[:, t, u] ** 2))
    for state, sign in (("singlet", 1.0), ("triplet", -1.0)):
        m = FixedRef(B, F, 2, "dcsd", state)
        assert abs(m.energy_A(np.zeros(m.size)) - sign * K) < 1e-14


def test_fixed_reference_residual_differs_from_two_determinant_residual():
    """Beyond two electrons FR and 2D are different equations (no coupling,
    a non-zero A->B amplitude)."""
    B, F = synth.make_inputs(2, 5, 20, 3)
    vec = synth.random_amplitudes(2, 5, 9, 0.05)
    R_fr, W_fr = FixedRef(B, F, 2, "dcsd", "singlet").residual(vec)
    R_2d, _ = TwoDet(B, F, 2, "dcsd").residual(vec)
    assert W_fr == 0.0
    assert np.abs(R_fr - R_2d).max() > 1e-2
