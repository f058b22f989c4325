"""GPU: the low-precision ladder and ring GEMMs (FP32 or BF16 MFMA inputs,
FP32 accumulation) and the mixed-precision solver.

Bars:
* GEMM: against the exact product of the *rounded* inputs (rounded here by
  NumPy to nearest even), elementwise within the FP32 summation bound
  (K + 2) 2^-24 (|A~| |B~|); this also pins the rounding mode of the inputs.
* Residual with low-precision ladder/ring GEMMs against the FP64 oracle:
  max |dR| and |dW| within 2e-6 s (FP32) or 1e-2 s (BF16), s = max(1, max|R|).
  BF16 errors come from the input rounding (2^-9 relative), FP32 errors mostly
  from FP32 accumulation over the (nv+2)^2-term ladder sums; the measured
  worst cases on these shapes are 1.8e-7 s and 6.6e-4 s (4-5x below the bars).
* Mixed solve: converges, and only on an FP64 residual, to the FP64 fixed
  point: |dE_S|, |dE_T| <= 1e-8 Eh against the oracle's converged energies.
"""
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


def round_to(x: np.ndarray, precision: str) -> np.ndarray:
    """FP64 -> FP32 (nearest even) -> BF16 (nearest even), back in FP64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    if precision == "fp32":
        return f.astype(np.float64)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def test_round_to_bf16_is_nearest_even():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to the even 1.0
    assert round_to(np.array([1.0 + 2.0 ** -8]), "bf16")[0] == 1.0
    assert round_to(np.array([1.0 + 3 * 2.0 ** -8]), "bf16")[0] == 1.0 + 2.0 ** -6
    assert round_to(np.array([1.0 + 2.0 ** -8 + 2.0 ** -20]), "bf16")[0] == 1.0 + 2.0 ** -7


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (17, 33, 5), (128, 128, 64), (129, 257, 31), (300, 70, 1000),
                                   (513, 200, 77), (64, 64, 4100), (4100, 4200, 1032)])
def test_lowp_gemm_within_fp32_summation_bound(precision, M, N, K):
    import torch
    from paper_2401_11935_amd import libdcsd as L
    from gpu_util import stream, to_dev
    say("lowp gemm", precision, M, N, K)
    rng = np.random.default_rng(M * 7919 + N * 31 + K)
    A = rng.normal(size=(M, K))
    B = rng.normal(size=(K, N))
    Ad, Bd = to_dev(A), to_dev(B)  # keep the tensors alive while their addresses are in use
    Cd = torch.full((M, N), np.nan, dtype=torch.float64, device="cuda:0")
    L.selftest_gemm(M, N, K, Ad.data_ptr(), Bd.data_ptr(), Cd.data_ptr(), stream(), precision=precision)
    Ar, Br = round_to(A, precision), round_to(B, precision)
    ref = Ar @ Br
    bound = (K + 2) * 2.0 ** -24 * (np.abs(Ar) @ np.abs(Br)) + 1e-300
    C = Cd.cpu().numpy()
    ratio = float((np.abs(C - ref) / bound).max())
    say(f"  max |C - A~B~| / bound = {ratio:.3f}")
    assert ratio <= 1.0
    # the rounding really happened (not an FP64 product)
    if K >= 31:
        assert np.abs(C - A @ B).max() > 1e-12


# naux a multiple of 8 takes the direct-to-LDS pair assembly (K in whole 16-byte chunks);
# the others take the register-staged kernel.  (3, 48, 40): the ladder contraction has
# K = (nv+2)^2 = 2500 split in two, on the direct-to-LDS kernel; in BF16, K is not a multiple
# of 8 and its last 16-byte chunk runs into the zeroed row padding.
MIXED_SHAPES = [(2, 5, 13, "dcsd", 0), (3, 7, 11, "ccsd", 5), (5, 40, 37, "dcsd", 16), (6, 33, 70, "ccsd", 0),
                (4, 30, 48, "dcsd", 8), (5, 41, 64, "ccsd", 0), (3, 48, 40, "dcsd", 0)]
BARS = {"fp32": 2e-6, "bf16": 1e-2}


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("nc,nv,naux,method,lb", MIXED_SHAPES)
def test_lowp_residual_error_against_oracle(precision, nc, nv, naux, method, lb):
    from gpu_util import GpuProblem
    say("lowp residual", precision, nc, nv, naux, method, lb)
    B, F = synth.make_inputs(nc, nv, naux, nc + nv)
    T = synth.random_amplitudes(nc, nv, nc + nv + 5, 0.05)
    p = GpuProblem(B, F, nc, method, ladder_block=lb, precision=precision)
    R, W = p.residual(T)
    p.close()
    model = TwoDet(B, F, nc, method)
    Ro, Wo = model.residual(T)
    s = max(1.0, float(np.abs(Ro).max()))
    err = float(np.abs(R - Ro).max())
    say(f"  max|dR| = {err:.3e} (bar {BARS[precision] * s:.1e})  |dW| = {abs(W - Wo):.3e}")
    assert err <= BARS[precision] * s
    assert abs(W - Wo) <= BARS[precision] * s
    assert err > 1e-13  # the low-precision path ran
    assert R[model.ab] == 0.0


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("method", ["dcsd", "ccsd"])
def test_mixed_solve_reaches_fp64_fixed_point_tiny(precision, method):
    from gpu_util import GpuProblem
    gold = json.load(open(os.path.join(HERE, "golden", "tiny.json")))[method]["solve"]
    cfg = synth.TINY
    say("tiny mixed solve", precision, method)
    B, F = synth.make_config_inputs(cfg)
    p = GpuProblem(B, F, cfg.nc, method, tol_residual=1e-10, precision=precision)
    rep, T = p.solve()
    p.close()
    recs = rep["records"]
    nfp = sum(r["fp64"] for r in recs)
    say(f"  {rep['status']} iterations {rep['iterations']} (oracle FP64 {gold['iterations']}), FP64 refreshes {nfp}, "
        f"|dE_S| = {abs(rep['E_S'] - gold['E_S']):.2e} |dE_T| = {abs(rep['E_T'] - gold['E_T']):.2e}")
    assert rep["converged"] and recs[-1]["fp64"] and recs[-1]["res_max"] <= 1e-10
    assert nfp < len(recs)  # most iterations ran in low precision
    assert abs(rep["E_S"] - gold["E_S"]) <= 1e-8
    assert abs(rep["E_T"] - gold["E_T"]) <= 1e-8


def test_mixed_solve_reaches_fp64_fixed_point_small_bf16():
    """nc=8, nv=20, naux=60, 2D-DCSD in BF16 with FP64 refreshes."""
    from gpu_util import GpuProblem
    gold = json.load(open(os.path.join(HERE, "golden", "small.json")))
    c = gold["config"]
    g = gold["dcsd"]["solve"]
    say("small mixed solve bf16")
    B, F = synth.make_inputs(c["nc"], c["nv"], c["naux"], c["seed"])
    p = GpuProblem(B, F, c["nc"], "dcsd", tol_residual=g["tol"], max_iter=400, precision="bf16")
    rep, T = p.solve()
    p.close()
    nfp = sum(r["fp64"] for r in rep["records"])
    say(f"  iterations {rep['iterations']} (FP64 {g['iterations']}), FP64 refreshes {nfp}, "
        f"|dE_S| = {abs(rep['E_S'] - g['E_S']):.2e}")
    assert rep["converged"] and rep["records"][-1]["fp64"]
    assert abs(rep["E_S"] - g["E_S"]) <= 1e-8 and abs(rep["E_T"] - g["E_T"]) <= 1e-8


def test_refresh_every_forces_fp64_iterations():
    from gpu_util import GpuProblem
    say("refresh_every")
    B, F = synth.make_inputs(2, 5, 13, 3)
    p = GpuProblem(B, F, 2, "dcsd", precision="bf16", max_iter=6, refresh_every=2)
    rep, _ = p.solve()
    p.close()
    flags = [r["fp64"] for r in rep["records"]]
    say("  fp64 flags", flags)
    # every second iteration at the latest is an FP64 refresh
    assert all(flags[i] or flags[i + 1] for i in range(len(flags) - 1))


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp64"])
@pytest.mark.parametrize("nc,nv,naux,lb", [(2, 5, 13, 3), (3, 16, 60, 5), (4, 40, 64, 0)])
def test_ladder_cache_is_bitwise_the_assembly(precision, nc, nv, naux, lb):
    """The cached ladder integrals (low precision: ladder_cache 1; FP64 and, in a
    low-precision context, its FP64 refreshes too: ladder_cache 2) give bitwise the
    residuals of the assembly on every evaluation, and the solves take identical steps."""
    from gpu_util import GpuProblem
    say("ladder cache", precision, nc, nv, naux, lb)
    B, F = synth.make_inputs(nc, nv, naux, 70 + nv)
    Ts = [synth.random_amplitudes(nc, nv, 71 + k, 0.05) for k in range(3)]
    modes = (0, 1, 2) if precision != "fp64" else (0, 2)
    out = {}
    for cache in modes:
        p = GpuProblem(B, F, nc, "dcsd", ladder_block=lb, precision=precision, ladder_cache=cache)
        out[cache] = [p.residual(T) for T in Ts + Ts[:1]]
        p.close()
    for cache in modes[1:]:
        for (Ra, Wa), (Rb, Wb) in zip(out[0], out[cache]):
            assert np.array_equal(Ra, Rb) and Wa == Wb
        assert np.array_equal(out[cache][0][0], out[cache][3][0])   # the same T again, from the cache
    reps = {}
    for cache in modes:
        p = GpuProblem(B, F, nc, "dcsd", ladder_block=lb, precision=precision, ladder_cache=cache, max_iter=12)
        reps[cache], _ = p.solve()
        p.close()
    for cache in modes[1:]:
        assert [r["res_max"] for r in reps[0]["records"]] == [r["res_max"] for r in reps[cache]["records"]]
