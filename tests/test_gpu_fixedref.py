"""GPU: the fixed-reference methods (FR-DCSD, FR-CCSD; singlet and M_s = 0
triplet) through the C ABI against the oracle (oracle/fixedref.py).

Bars: residual 1e-9 absolute and energy 1e-10 Eh against the oracle at the
same amplitudes; two-electron complete-active-space solves equal the FCI
roots to 1e-9 Eh; the gradient of the converged state energy (dcsd_backward)
against central differences of re-converged solves to 1e-6 relative.
"""
import sys

import numpy as np
import pytest

import dcsd_synth as synth

pytestmark = pytest.mark.gpu

FR = ["fr-dcsd-singlet", "fr-dcsd-triplet", "fr-ccsd-singlet", "fr-ccsd-triplet"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2401_11935_amd import libdcsd
    libdcsd.load()


def _oracle(B, F, nc, name):
    from oracle.fixedref import FixedRef
    _, method, state = name.split("-")
    return FixedRef(B, F, nc, method, state)


def _keys(name):
    return ("E_S", "E_T") if name.endswith("singlet") else ("E_T", "E_S")


@pytest.mark.parametrize("name", FR)
@pytest.mark.parametrize("nc,nv,naux,lb", [(2, 5, 13, 0), (3, 7, 11, 4), (1, 9, 17, 2), (5, 40, 37, 16),
                                           (6, 33, 70, 0)])
def test_fixed_reference_residual_and_energy_match_oracle(name, nc, nv, naux, lb):
    from gpu_util import GpuProblem
    say("fr residual", name, nc, nv, naux, lb)
    B, F = synth.make_inputs(nc, nv, naux, nc + nv)
    T = synth.random_amplitudes(nc, nv, nc + nv + 5, 0.05)
    p = GpuProblem(B, F, nc, name, ladder_block=lb)
    R, W = p.residual(T)
    e = p.energy(T)
    p.close()
    m = _oracle(B, F, nc, name)
    Ro, _ = m.residual(T)
    eo = m.energies(T)
    err = float(np.abs(R - Ro).max())
    key, other = _keys(name)
    say(f"  max|dR| = {err:.3e}  |d{key}| = {abs(e[key] - eo[key]):.3e}")
    assert W == 0.0
    assert R[m.ab] == 0.0
    assert err <= 1e-9
    assert abs(e[key] - eo[key]) <= 1e-10
    assert abs(e["dE_A"] - eo["dE_A"]) <= 1e-10
    assert np.isnan(e[other])


@pytest.mark.parametrize("method", ["dcsd", "ccsd"])
def test_fixed_reference_two_electron_cas_solves_equal_fci(method):
    from gpu_util import GpuProblem
    from oracle.brute import DeterminantSpace
    from oracle.hamiltonian import Hamiltonian
    B, F, _ = synth.make_z2_inputs(0, 7, 30, 11)
    ham = Hamiltonian(B, F, 0)
    ES, ET, _, _ = DeterminantSpace(ham).fci_pair()
    for state, key, ref in (("singlet", "E_S", ES), ("triplet", "E_T", ET)):
        name = f"fr-{method}-{state}"
        say("fr 2e CAS solve", name)
        p = GpuProblem(B, F, 0, name, tol_residual=1e-11)
        rep, _ = p.solve()
        p.close()
        say(f"  {rep['status']} iterations {rep['iterations']}  |E - FCI| = {abs(ham.e_ref() + rep[key] - ref):.2e}")
        assert rep["status"] == "OK"
        assert abs(ham.e_ref() + rep[key] - ref) <= 1e-9


@pytest.mark.parametrize("name", ["fr-dcsd-singlet", "fr-ccsd-triplet"])
def test_fixed_reference_gradient_matches_finite_differences(name):
    """dcsd_backward for the state energy of a converged FR solve against central
    differences of re-converged solves, on 16 seeded entries of B and on F."""
    import torch
    from paper_2401_11935_amd import libdcsd as L
    from gpu_util import stream, to_dev
    B, F, _ = synth.make_z2_inputs(0, 5, 13, 8)
    nc, n = 0, B.shape[1]
    key = _keys(name)[0]
    eS, eT = (1.0, 0.0) if key == "E_S" else (0.0, 1.0)

    def ctx_for(Bx, Fx):
        Bd, Fd = to_dev(Bx), to_dev(Fx)
        cfg = L.default_config(nc=nc, nv=n - 2, naux=Bx.shape[0], method=name, tol_residual=1e-12, max_iter=400,
                               adjoint=1)
        return L.Context(cfg, Bd.data_ptr(), Fd.data_ptr(), stream()), Bd, Fd

    def solve_E(Bx, Fx):
        ctx, Bd, Fd = ctx_for(Bx, Fx)  # B, F borrowed: keep the tensors alive
        T = torch.zeros(ctx.size, dtype=torch.float64, device="cuda:0")
        r = ctx.solve(T.data_ptr())
        ctx.close()
        assert r["status"] == "OK"
        return r[key]

    say("fr backward vs finite differences", name)
    ctx, Bd, Fd = ctx_for(B, F)
    T = torch.zeros(ctx.size, dtype=torch.float64, device="cuda:0")
    rep = ctx.solve(T.data_ptr())
    assert rep["status"] == "OK"
    Bb, Fb, lam = torch.empty_like(Bd), torch.empty_like(Fd), torch.zeros_like(T)
    lrep = ctx.backward(T.data_ptr(), eS, eT, Bb.data_ptr(), Fb.data_ptr(), lam.data_ptr())
    ctx.close()
    assert lrep["status"] == "OK", lrep
    Bb, Fb = Bb.cpu().numpy(), Fb.cpu().numpy()
    rng = np.random.default_rng(6)
    h = 1e-5
    worst = 0.0
    picks = set()
    while len(picks) < 16:
        P, p, q = int(rng.integers(B.shape[0])), int(rng.integers(n)), int(rng.integers(n))
        picks.add((P, min(p, q), max(p, q)))
    cases = [("B", P, p, q) for (P, p, q) in sorted(picks)] + [("F", 0, 1, 2), ("F", 0, 3, 3)]
    for kind, P, p, q in cases:
        dB, dF = np.zeros_like(B), np.zeros_like(F)
        d = dB[P] if kind == "B" else dF
        if p == q:
            d[p, p] = 1.0
        else:
            d[p, q] = d[q, p] = 0.5
        fd = (solve_E(B + h * dB, F + h * dF) - solve_E(B - h * dB, F - h * dF)) / (2 * h)
        an = Bb[P, p, q] if kind == "B" else Fb[p, q]
        worst = max(worst, abs(fd - an) / max(abs(fd), 1e-3))
        assert abs(fd - an) <= 1e-6 * abs(fd) + 1e-9, (kind, P, p, q, fd, an)
    say(f"  worst |fd - adjoint| / max(|fd|, 1e-3) = {worst:.1e}")


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_fixed_reference_mixed_precision_solve_reaches_fci(precision):
    """The low-precision ladder and rings with FP64 refreshes converge to the
    same FP64 fixed point: within 1 microhartree of the FCI roots."""
    from gpu_util import GpuProblem
    from oracle.brute import DeterminantSpace
    from oracle.hamiltonian import Hamiltonian
    B, F, _ = synth.make_z2_inputs(0, 7, 30, 11)
    ham = Hamiltonian(B, F, 0)
    ES, ET, _, _ = DeterminantSpace(ham).fci_pair()
    for name, key, ref in (("fr-dcsd-singlet", "E_S", ES), ("fr-ccsd-triplet", "E_T", ET)):
        say("fr mixed solve", name, precision)
        p = GpuProblem(B, F, 0, name, tol_residual=1e-10, precision=precision)
        rep, _ = p.solve()
        p.close()
        err = abs(ham.e_ref() + rep[key] - ref)
        say(f"  {rep['status']} iterations {rep['iterations']}  |E - FCI| = {err:.2e}")
        assert rep["status"] == "OK"
        assert err <= 1e-6
