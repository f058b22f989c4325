"""GPU: the library on inputs read from an FCIDUMP file (pivoted Cholesky
factors, reordered orbitals) against the oracle on the same loaded inputs
(residual 1e-9, W and energies 1e-10), and against the library on the original
factors, since B enters only through (pq|rs) (residual 1e-10, W and energies
1e-11)."""
import sys

import numpy as np
import pytest

import dcsd_synth as synth

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("method", ["dcsd", "fr-ccsd-singlet"])
def test_library_on_fcidump_inputs_matches_original_factors(tmp_path, method):
    from gpu_util import GpuProblem
    from oracle.hamiltonian import Hamiltonian
    from paper_2401_11935_amd import fcidump as fd
    cfg = synth.TINY
    nc, nv = cfg.nc, cfg.nv
    B, F = synth.make_config_inputs(cfg)
    n = nc + 2 + nv
    h = Hamiltonian(B, F, nc).h
    eri = np.einsum("Ppq,Prs->pqrs", B, B)
    perm = np.random.default_rng(3).permutation(n)
    inv = np.argsort(perm)
    path = tmp_path / "FCIDUMP"
    fd.write_fcidump(str(path), h[np.ix_(perm, perm)], eri[np.ix_(perm, perm, perm, perm)], nelec=2 * nc + 2)
    prob = fd.load_problem(str(path), core=[int(inv[k]) for k in range(nc)], t=int(inv[nc]), u=int(inv[nc + 1]),
                           virt=[int(inv[k]) for k in range(nc + 2, n)], tol=1e-12)
    say("fcidump inputs", method, "naux", B.shape[0], "->", prob["naux"])
    T = synth.random_amplitudes(nc, nv, 17, 0.05)
    out = []
    for Bx, Fx in ((B, F), (prob["B"], prob["F"])):
        p = GpuProblem(Bx, Fx, nc, method)
        R, W = p.residual(T)
        e = p.energy(T)
        p.close()
        out.append((R, W, e))
    (Ra, Wa, ea), (Rb, Wb, eb) = out
    # parity with the oracle on the loaded factors
    from oracle.fixedref import FixedRef
    from oracle.twodet import TwoDet
    if method.startswith("fr"):
        _, m, state = method.split("-")
        model = FixedRef(prob["B"], prob["F"], nc, m, state)
    else:
        model = TwoDet(prob["B"], prob["F"], nc, method)
    Ro, Wo = model.residual(T)
    eo = model.energies(T, Wo)
    say(f"  oracle on the loaded factors: max|dR| = {np.abs(Rb - Ro).max():.2e}  |dW| = {abs(Wb - Wo):.2e}")
    assert np.abs(Rb - Ro).max() <= 1e-9
    assert abs(Wb - Wo) <= 1e-10
    for k in ("dE_A", "E_ref_A"):
        assert abs(eb[k] - eo[k]) <= 1e-10
    say(f"  original factors: max|dR| = {np.abs(Ra - Rb).max():.2e}  |dW| = {abs(Wa - Wb):.2e}")
    assert np.abs(Ra - Rb).max() <= 1e-10
    assert abs(Wa - Wb) <= 1e-11
    for k in ("dE_A", "E_ref_A"):
        assert abs(ea[k] - eb[k]) <= 1e-11
