"""GPU parity: libdcsd (HIP, gfx950) against the CPU oracle.

Bars (FP64 path): residual max-norm error <= 1e-9, |dE| <= 1e-8 Eh for the
converged energies; the FP64 GEMM itself agrees with NumPy to a relative
1e-13.  All inputs are seeded; every case prints its name before the GPU
call."""
import json
import os
import sys

import numpy as np
import pytest

import dcsd_synth as synth
from oracle.twodet import TwoDet

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


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


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (17, 33, 5), (64, 64, 16), (129, 257, 31), (300, 70, 1000),
                                   (128, 128, 128), (513, 200, 77)])
def test_gemm_matches_numpy(M, N, K):
    import torch
    from paper_2401_11935_amd import libdcsd as L
    from gpu_util import stream, to_dev
    say("gemm", M, N, K)
    rng = np.random.default_rng(M * 1000 + N + K)
    A = rng.normal(size=(M, K))
    B = rng.normal(size=(K, N))
    Ad, Bd = to_dev(A), to_dev(B)
    Cd = torch.full((M, N), np.nan, dtype=torch.float64, device="cuda:0")
    L.selftest_gemm(M, N, K, Ad.data_ptr(), Bd.data_ptr(), Cd.data_ptr(), stream())
    ref = A @ B
    err = float(np.abs(Cd.cpu().numpy() - ref).max())
    tol = 1e-13 * max(1.0, float(np.abs(ref).max())) * np.sqrt(K)
    assert err <= tol, f"max |C - A B| = {err:.3e} > {tol:.3e}"


# (M, N, K, a_mc, b_nc, ksplit, alpha, beta, pad, shift): outputs of at least 128 tiles of
# 128 x 128 take the direct-to-LDS kernel, which streams every operand row in 16-byte chunks
# along its contiguous extent (M or N for a K-major operand, K for a K-contiguous one): an
# operand with an odd extent or leading dimension or an 8-byte shifted base is first copied,
# zero-padded (odd M or K, the shifted bases below); where the copy would cost more than the
# product gains (the 16384 x 128 row) it takes the register-staged kernel, and small outputs
# take the 64-wide kernels
LAYOUTS = [(1536, 1536, 37, 1, 1, 1, 1.0, 0.0, 0, 0), (1536, 1408, 100, 1, 1, 3, 0.5, 1.0, 0, 0),
           (1530, 1542, 8, 1, 1, 1, -1.0, 1.0, 0, 0), (1536, 1536, 24, 1, 1, 1, 1.0, 0.0, 6, 0),
           (1535, 1536, 20, 1, 1, 1, 1.0, 0.0, 0, 0), (1536, 1536, 20, 1, 1, 1, 1.0, 0.0, 0, 1),
           (100, 60, 7, 1, 1, 1, 1.0, 0.0, 0, 0), (1536, 1536, 33, 0, 1, 1, 1.0, 0.5, 0, 0),
           (1536, 1536, 33, 0, 0, 2, 1.0, 0.0, 0, 0), (1536, 1280, 33, 1, 0, 1, 2.0, 0.0, 2, 0),
           (1536, 1536, 40, 0, 1, 1, 1.0, 0.5, 0, 0), (1536, 1536, 64, 0, 0, 3, 1.0, 0.0, 0, 0),
           (1536, 1280, 34, 1, 0, 1, 2.0, 0.0, 2, 0), (1501, 1527, 50, 0, 0, 1, -0.5, 1.0, 4, 0),
           (1500, 1530, 26, 0, 1, 2, 1.0, 1.0, 0, 0), (1500, 1530, 120, 1, 1, 8, 0.5, 1.0, 0, 0),
           (338, 1024, 1000, 0, 0, 16, 1.0, 0.0, 0, 0),
           # both operands padded: odd K in K-contiguous rows with odd leading dimensions, split
           (1537, 1281, 45, 0, 0, 3, 1.0, 0.5, 1, 0), (16384, 128, 33, 0, 1, 1, 1.0, 0.0, 0, 0),
           # small outputs over a long K (split dot products): full, ragged, single row and
           # column, padded rows, an 8-byte shifted base, K not a multiple of the 2048 chunk
           (16, 16, 65536, 0, 0, 1, 1.0, 0.0, 0, 0), (13, 13, 67769, 0, 0, 1, 1.0, 1.0, 0, 0),
           (1, 16, 100003, 0, 0, 1, -0.5, 0.0, 3, 1), (16, 1, 70001, 0, 0, 1, 2.0, 0.5, 0, 1),
           (7, 11, 131073, 0, 0, 1, 1.0, 0.0, 5, 0)]


@pytest.mark.parametrize("M,N,K,a_mc,b_nc,ks,alpha,beta,pad,shift", LAYOUTS)
def test_gemm_layouts_match_numpy(M, N, K, a_mc, b_nc, ks, alpha, beta, pad, shift):
    from paper_2401_11935_amd import libdcsd as L
    from gpu_util import stream, to_dev
    say("gemm layout", M, N, K, a_mc, b_nc, ks, alpha, beta, pad, shift)
    rng = np.random.default_rng(M + 7 * N + 11 * K + a_mc + 2 * b_nc + 3 * ks)
    Am, Bm, C0 = rng.normal(size=(M, K)), rng.normal(size=(K, N)), rng.normal(size=(M, N))
    lda, ldb = (M if a_mc else K) + pad, (N if b_nc else K) + pad
    As = np.zeros((K, lda) if a_mc else (M, lda))
    if a_mc:
        As[:, :M] = Am.T  # element (m, k) at m + k*lda
    else:
        As[:, :K] = Am  # element (m, k) at m*lda + k
    Bs = np.zeros((K, ldb) if b_nc else (N, ldb))
    if b_nc:
        Bs[:, :N] = Bm  # element (k, n) at n + k*ldb
    else:
        Bs[:, :K] = Bm.T  # element (k, n) at n*ldb + k
    Ad = to_dev(np.concatenate([np.zeros(shift), As.ravel()]))
    Bd = to_dev(np.concatenate([np.zeros(shift), Bs.ravel()]))
    Cd = to_dev(C0)
    L.selftest_gemm_layout(M, N, K, Ad.data_ptr() + 8 * shift, lda, bool(a_mc), Bd.data_ptr() + 8 * shift, ldb,
                           bool(b_nc), Cd.data_ptr(), N, alpha, beta, ks, stream())
    ref = alpha * (Am @ Bm) + beta * C0
    err = float(np.abs(Cd.cpu().numpy() - ref).max())
    tol = 1e-13 * max(1.0, float(np.abs(ref).max())) * np.sqrt(K)
    assert err <= tol, f"max |C - ref| = {err:.3e} > {tol:.3e}"


SMALL = [(2, 5, 13, "dcsd", 0), (2, 5, 13, "ccsd", 0), (0, 4, 7, "dcsd", 0), (0, 6, 9, "ccsd", 3),
         (3, 7, 11, "dcsd", 4), (3, 7, 11, "ccsd", 5), (1, 9, 17, "dcsd", 2), (4, 3, 5, "ccsd", 1),
         (5, 40, 37, "dcsd", 16), (6, 33, 70, "ccsd", 0),
         (32, 2, 10, "dcsd", 0)]  # o = 33: more occupied orbitals than the T1-dressing kernel takes


@pytest.mark.parametrize("nc,nv,naux,method,lb", SMALL)
def test_residual_matches_oracle(nc, nv, naux, method, lb):
    from gpu_util import GpuProblem
    say("residual", nc, nv, naux, method, lb)
    B, F = synth.make_inputs(nc, nv, naux, nc + nv)
    T = synth.random_amplitudes(nc, nv, nc + nv + 5, 0.05)
    p = GpuProblem(B, F, nc, method, ladder_block=lb)
    R, W = p.residual(T)
    e = p.energy(T)
    p.close()
    model = TwoDet(B, F, nc, method)
    Ro, Wo = model.residual(T)
    err = float(np.abs(R - Ro).max())
    say(f"  max|dR| = {err:.3e}  |dW| = {abs(W - Wo):.3e}")
    assert err <= 1e-9, f"max |R_gpu - R_oracle| = {err:.3e}"
    assert abs(W - Wo) <= 1e-10
    assert abs(e["dE_A"] - model.energy_A(T)) <= 1e-10
    assert abs(e["E_ref_A"] - model.ham.e_ref()) <= 1e-10
    assert R[model.ab] == 0.0


@pytest.mark.parametrize("method", ["dcsd", "ccsd"])
def test_tiny_residual_and_determinism(method):
    from gpu_util import GpuProblem
    cfg = synth.TINY
    say("tiny residual", method)
    B, F = synth.make_config_inputs(cfg)
    T = synth.random_amplitudes(cfg.nc, cfg.nv, 77, 0.03)
    p = GpuProblem(B, F, cfg.nc, method)
    R1, W1 = p.residual(T)
    R2, W2 = p.residual(T)
    p.close()
    Ro, Wo = TwoDet(B, F, cfg.nc, method).residual(T)
    err = float(np.abs(R1 - Ro).max())
    say(f"  max|dR| = {err:.3e}  |dW| = {abs(W1 - Wo):.3e}")
    assert err <= 1e-9, f"max |R_gpu - R_oracle| = {err:.3e}"
    assert abs(W1 - Wo) <= 1e-10
    assert np.array_equal(R1, R2) and W1 == W2     # bitwise repeatable


def test_tiny_golden_residual_samples():
    from gpu_util import GpuProblem
    gold = json.load(open(os.path.join(HERE, "golden", "tiny.json")))
    cfg = synth.TINY
    for method in ("dcsd", "ccsd"):
        g = gold[method]["residual"]
        say("tiny golden samples", method)
        B, F = synth.make_config_inputs(cfg)
        T = synth.random_amplitudes(cfg.nc, cfg.nv, g["amp_seed"], g["amp_scale"])
        p = GpuProblem(B, F, cfg.nc, method)
        R, W = p.residual(T)
        p.close()
        err = float(np.abs(R[np.array(g["positions"])] - np.array(g["values"])).max())
        assert err <= 1e-9, f"sampled max |dR| = {err:.3e}"
        assert abs(W - g["W"]) <= 1e-10


@pytest.mark.parametrize("method", ["dcsd", "ccsd"])
def test_tiny_solve_matches_oracle_energies(method):
    from gpu_util import GpuProblem
    gold = json.load(open(os.path.join(HERE, "golden", "tiny.json")))[method]["solve"]
    cfg = synth.TINY
    say("tiny solve", method)
    B, F = synth.make_config_inputs(cfg)
    p = GpuProblem(B, F, cfg.nc, method, tol_residual=1e-10)
    rep, T = p.solve()
    p.close()
    assert rep["converged"], rep
    assert abs(rep["E_S"] - gold["E_S"]) <= 1e-8
    assert abs(rep["E_T"] - gold["E_T"]) <= 1e-8
    assert abs(rep["W"] - gold["W"]) <= 1e-8
    # Same Jacobi/DIIS settings as the oracle's solver: the first iterations
    # agree to rounding; later ones may drift (DIIS amplifies 1e-15 differences
    # while the residual is large) but reach the same fixed point.
    traj = gold["trajectory"]
    for a, b in zip(rep["records"][:6], traj[:6]):
        assert abs(a["E_S"] - b["E_S"]) <= 1e-9 and abs(a["res_max"] - b["res_max"]) <= 1e-9
    say(f"  iterations gpu {rep['iterations']} oracle {gold['iterations']}; "
        f"|dE_S| = {abs(rep['E_S'] - gold['E_S']):.2e} |dE_T| = {abs(rep['E_T'] - gold['E_T']):.2e}")


@pytest.mark.parametrize("precond", ["orbital", "en"])
def test_solver_iterations_match_oracle(precond):
    """Four Jacobi/DIIS iterations with either preconditioner follow the
    oracle's iterations (same settings) to rounding."""
    from gpu_util import GpuProblem
    from oracle.solver import solve
    nc, nv, naux = 3, 8, 20
    say("solver iterations", precond)
    B, F = synth.make_inputs(nc, nv, naux, 21)
    p = GpuProblem(B, F, nc, "dcsd", precond=1 if precond == "en" else 0, max_iter=4)
    rep, T = p.solve()
    p.close()
    r = solve(TwoDet(B, F, nc, "dcsd"), max_iter=4, precond="en" if precond == "en" else "mp")
    rel = lambda x, y: abs(x - y) / max(1.0, abs(y))  # noqa: E731
    for a, b in zip(rep["records"], r["records"]):
        assert rel(a["E_S"], b["E_S"]) <= 1e-10 and rel(a["res_max"], b["res_max"]) <= 1e-10
    # without convergence both hand back the evaluated amplitudes with the smallest max |R|
    # (the orbital-energy iteration grows |R| to ~1e2 here, which scales the rounding)
    assert rep["status"] == "ERR_NOCONV"
    assert np.abs(T - r["T_best"]).max() <= 1e-9
    assert rel(rep["res_max"], r["best"]["res_max"]) <= 1e-10


def test_small_convergent_config_matches_oracle():
    """nc=8, nv=20, naux=60: converged energies against the oracle's (stored)."""
    from gpu_util import GpuProblem
    path = os.path.join(HERE, "golden", "small.json")
    if not os.path.exists(path):
        pytest.skip("small.json not generated")
    gold = json.load(open(path))
    c = gold["config"]
    B, F = synth.make_inputs(c["nc"], c["nv"], c["naux"], c["seed"])
    methods = [m for m in ("dcsd", "ccsd") if m in gold and gold[m]["solve"]["converged"]]
    assert "dcsd" in methods
    for method in methods:
        say("small solve", method)
        g = gold[method]["solve"]
        p = GpuProblem(B, F, c["nc"], method, tol_residual=g["tol"], max_iter=400)
        rep, T = p.solve()
        p.close()
        assert rep["converged"]
        say(f"  |dE_S| = {abs(rep['E_S'] - g['E_S']):.2e}  |dE_T| = {abs(rep['E_T'] - g['E_T']):.2e}")
        assert abs(rep["E_S"] - g["E_S"]) <= 1e-8 and abs(rep["E_T"] - g["E_T"]) <= 1e-8


def test_medium_residual_matches_oracle_samples():
    """nc=8, nv=200, naux=600 (the oracle needs ~12 min per residual here):
    4096 seeded positions, W, dE_A and the max- and 2-norms of the full
    residual against the stored oracle values."""
    from gpu_util import GpuProblem
    path = os.path.join(HERE, "golden", "medium.json")
    if not os.path.exists(path):
        pytest.skip("medium.json not generated")
    gold = json.load(open(path))
    c = gold["config"]
    B, F = synth.make_inputs(c["nc"], c["nv"], c["naux"], c["seed"])
    for method in [m for m in ("dcsd", "ccsd") if m in gold]:
        g = gold[method]["residual"]
        say("medium residual", method)
        T = synth.random_amplitudes(c["nc"], c["nv"], g["amp_seed"], g["amp_scale"])
        p = GpuProblem(B, F, c["nc"], method)
        R, W = p.residual(T)
        e = p.energy(T)
        p.close()
        err = float(np.abs(R[np.array(g["positions"])] - np.array(g["values"])).max())
        say(f"  sampled max|dR| = {err:.3e}  |dW| = {abs(W - g['W']):.2e}")
        assert err <= 1e-9
        assert abs(W - g["W"]) <= 1e-10
        assert abs(e["dE_A"] - g["dE_A"]) <= 1e-9
        assert abs(float(np.abs(R).max()) - g["res_max"]) <= 1e-9
        assert abs(float(np.dot(R, R)) - g["res_norm2"]) <= 1e-9 * g["res_norm2"]


@pytest.mark.timeout(400)
@pytest.mark.parametrize("cfg", [synth.MIXED, synth.LARGEST], ids=lambda c: c.name)
def test_full_size_ladder_samples(cfg):
    """The particle-particle ladder alone (term mask), singles zero, at the metric
    (12, 400, 1200) and the largest (20, 600, 1800) sizes with the bench's
    launch configuration: 16 seeded elements per doubles block against the
    oracle's single-element ladder (bar 1e-9); the largest size also with BF16
    ladder GEMMs (bar 1e-2 of the sampled magnitude)."""
    from oracle.ccsd import ladder_element
    from gpu_util import GpuProblem
    say("full-size ladder samples", cfg.name, "inputs")
    B, F = synth.make_config_inputs(cfg)
    say("full-size ladder samples", cfg.name, "amplitudes")
    T = synth.random_amplitudes(cfg.nc, cfg.nv, cfg.seed + 11, 0.05)
    blocks = synth.unpack(T, cfg.nc, cfg.nv)
    blocks["t1a"][:] = 0.0
    blocks["t1b"][:] = 0.0
    o, v = cfg.nc + 1, cfg.nv + 1
    rng = np.random.default_rng(cfg.seed + 13)
    samples = []
    for blk, name in enumerate(("t2aa", "t2bb", "t2ab")):
        while sum(1 for s_ in samples if s_[1] == name) < 16:
            i, j, a, b = (int(x) for x in rng.integers(0, (o, o, v, v)))
            if (blk < 2 and (i == j or a == b)) or (blk == 2 and (i, j, a, b) == (cfg.nc, cfg.nc, 0, 0)):
                continue
            samples.append((blk, name, i, j, a, b))
    say("full-size ladder samples", cfg.name, "oracle elements")
    ref = np.array([ladder_element(B, cfg.nc, blocks[name], blk, i, j, a, b) for blk, name, i, j, a, b in samples])
    precisions = ["fp64", "bf16"] if cfg.name == "largest" else ["fp64"]
    for prec in precisions:
        say("full-size ladder samples", cfg.name, prec, "residual")
        p = GpuProblem(B, F, cfg.nc, "dcsd", precision=prec, term_mask=1 << 3)
        R, _ = p.residual(T)
        p.close()
        Rb = synth.unpack(R, cfg.nc, cfg.nv)
        got = np.array([Rb[name][i, j, a, b] for _, name, i, j, a, b in samples])
        err = float(np.abs(got - ref).max())
        scale = max(1.0, float(np.abs(ref).max()))
        bar = 1e-9 if prec == "fp64" else 1e-2 * scale
        say(f"  {prec}: sampled max|dR| = {err:.3e} (bar {bar:.1e}), max|R| sampled {np.abs(ref).max():.3e}")
        assert err <= bar


def test_internal_amplitude_ignored_on_input():
    from gpu_util import GpuProblem
    nc, nv, naux = 2, 5, 13
    B, F = synth.make_inputs(nc, nv, naux, 4)
    T = synth.random_amplitudes(nc, nv, 9, 0.05)
    p = GpuProblem(B, F, nc)
    R1, W1 = p.residual(T)
    T2 = T.copy()
    T2[TwoDet(B, F, nc).ab] = 0.37
    R2, W2 = p.residual(T2)
    p.close()
    assert np.array_equal(R1, R2) and W1 == W2, "residual changed with the ignored Phi_A->Phi_B amplitude"


def test_nonfinite_amplitudes_are_reported():
    from gpu_util import GpuProblem
    from paper_2401_11935_amd import libdcsd as L
    nc, nv, naux = 1, 4, 9
    B, F = synth.make_inputs(nc, nv, naux, 2)
    p = GpuProblem(B, F, nc)
    T0 = np.zeros(p.size)
    T0[3] = np.nan
    with pytest.raises(L.DcsdError) as e:
        p.solve(T0)
    assert e.value.status == L.DCSD_ERR_NONFINITE
    p.close()
