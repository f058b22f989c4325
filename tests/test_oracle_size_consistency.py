"""Size consistency of the full 2D equations (oracle pin).

A closed-shell two-electron fragment that shares no integral with the open-shell
system is added (``dcsd_synth.add_fragment``).  Its amplitudes are spin-flip
symmetric, so flip(T_fragment) = T_fragment and its factors cancel between
e^-T_A and e^T_B in every coupling coefficient; its own equations are then
single-reference CCSD of a two-electron system, which is exact (and the dropped
DC terms vanish for two electrons).  Hence the converged 2D-DCSD and 2D-CCSD
singlet and triplet correlation energies must shift by exactly the fragment's
FCI correlation energy, and W must stay as it was.  This ties the coupling terms,
the e^-T_A factor and the DC selection to a property the method must have; a
term that leaks between the fragments (an unlinked product in K_x, a wrong
e^-T_A subtraction) breaks it.
"""
import numpy as np
import pytest

import dcsd_synth as synth
from oracle.solver import solve
from oracle.twodet import TwoDet


def fragment_correlation(Bf: np.ndarray, Ff: np.ndarray) -> float:
    """FCI minus reference energy of a two-electron closed-shell fragment, orbital
    0 doubly occupied.  h = F - (2 J_0 - K_0) (the spin-averaged Fock reading with
    the fragment's occupied orbital as a core orbital); the singlet two-electron
    wavefunction sum_pq C_pq phi_p(1) phi_q(2) has C symmetric, and
    <pq|H|rs> = h_pr d_qs + d_pr h_qs + (pr|qs)."""
    nf = Ff.shape[0]
    eri = np.einsum("Ppq,Prs->pqrs", Bf, Bf)
    h = Ff - (2.0 * eri[:, :, 0, 0] - eri[:, 0, 0, :])
    one = np.eye(nf)
    H = (np.einsum("pr,qs->pqrs", h, one) + np.einsum("pr,qs->pqrs", one, h)
         + eri.transpose(0, 2, 1, 3)).reshape(nf * nf, nf * nf)
    swap = np.eye(nf * nf).reshape(nf, nf, nf, nf).transpose(1, 0, 2, 3).reshape(nf * nf, nf * nf)
    w, U = np.linalg.eigh(0.5 * (np.eye(nf * nf) + swap))
    Us = U[:, w > 0.5]                       # symmetric (singlet) C
    e0 = np.linalg.eigvalsh(Us.T @ H @ Us)[0]
    return float(e0 - (2.0 * h[0, 0] + eri[0, 0, 0, 0]))


def test_fragment_fci_of_a_single_orbital_pair():
    """With no virtuals the fragment has one configuration: zero correlation."""
    rng = np.random.default_rng(3)
    Bf = rng.normal(0, 0.2, (4, 1, 1))
    assert fragment_correlation(Bf, np.array([[-1.0]])) == pytest.approx(0.0, abs=1e-15)


@pytest.mark.parametrize("method", ["dcsd", "ccsd"])
@pytest.mark.parametrize("nc,nv,nf_vir,seed", [(1, 4, 3, 7), (2, 3, 2, 8)])
def test_noninteracting_fragment_shifts_energies_by_its_fci(method, nc, nv, nf_vir, seed):
    B, F = synth.make_inputs(nc, nv, 20, seed)
    r = solve(TwoDet(B, F, nc, method), tol=1e-11)
    B2, F2, nc2, frag = synth.add_fragment(B, F, nc, nf_vir, seed + 100)
    r2 = solve(TwoDet(B2, F2, nc2, method), tol=1e-11)
    assert r["converged"] and r2["converged"]
    ec = fragment_correlation(frag["B"], frag["F"])
    assert abs(ec) > 1e-3
    assert abs(r2["E_S"] - (r["E_S"] + ec)) < 1e-11
    assert abs(r2["E_T"] - (r["E_T"] + ec)) < 1e-11
    assert abs(r2["W"] - r["W"]) < 1e-11
