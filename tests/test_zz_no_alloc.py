"""GPU: dcsd_selftest_gemm_layout_noalloc, the FP64 layout GEMM that allocates
nothing (its split-K and small-output partial sums and its zero-padded operand
copies live in a per-GPU static array), against dcsd_selftest_gemm_layout,
which allocates the same scratch.

Two calls in a row per path, the second with a smaller input, each compared
bitwise with the allocating entry point (the same kernels in the same order);
the device's free memory is unchanged across the second call (the first may
load the code object that holds the array); a call that needs more
scratch than the array holds is refused before anything is launched."""
import sys

import numpy as np
import pytest

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


def _operands(M, N, K, a_mc, b_nc, pad, seed):
    from gpu_util import to_dev
    rng = np.random.default_rng(seed)
    Am, Bm, C0 = rng.normal(size=(M, K)), rng.normal(size=(K, N)), rng.normal(size=(M, N))
    lda, ldb = (M if a_mc else K) + pad, (N if b_nc else K) + pad
    As = np.zeros((K, lda) if a_mc else (M, lda))
    if a_mc:
        As[:, :M] = Am.T
    else:
        As[:, :K] = Am
    Bs = np.zeros((K, ldb) if b_nc else (N, ldb))
    if b_nc:
        Bs[:, :N] = Bm
    else:
        Bs[:, :K] = Bm.T
    return to_dev(As), lda, to_dev(Bs), ldb, C0, Am @ Bm


# (M, N, K, a_mc, b_nc, ksplit, alpha, beta, pad): per path, a call and then a smaller one
CASES = {
    "split-K": [(1280, 1152, 700, 1, 1, 2, 0.5, 1.0, 0), (900, 700, 300, 0, 1, 2, -1.0, 0.5, 4)],
    "small outputs over a long K": [(16, 16, 200000, 0, 0, 1, 1.0, 0.0, 0), (7, 11, 70001, 0, 0, 1, 2.0, 0.5, 3)],
    "no scratch": [(1536, 1536, 40, 0, 1, 1, 1.0, 0.5, 0), (300, 200, 20, 1, 0, 1, 1.0, 0.0, 2)],
    "zero-padded operand copies": [(1536, 1280, 33, 0, 1, 1, 1.0, 0.0, 0), (1300, 1400, 21, 1, 0, 2, -1.0, 0.5, 1)],
}


@pytest.mark.parametrize("path", list(CASES))
def test_noalloc_gemm_equals_the_allocating_entry_point(path):
    import torch
    from gpu_util import stream, to_dev
    from paper_2401_11935_amd import libdcsd as L
    for i, (M, N, K, a_mc, b_nc, ks, alpha, beta, pad) in enumerate(CASES[path]):
        say("noalloc gemm", path, M, N, K, a_mc, b_nc, ks, alpha, beta, pad)
        Ad, lda, Bd, ldb, C0, AB = _operands(M, N, K, a_mc, b_nc, pad, 97 + i)
        C1, C2 = to_dev(C0), to_dev(C0)
        L.selftest_gemm_layout(M, N, K, Ad.data_ptr(), lda, bool(a_mc), Bd.data_ptr(), ldb, bool(b_nc),
                               C1.data_ptr(), N, alpha, beta, ks, stream())
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        L.selftest_gemm_layout_noalloc(M, N, K, Ad.data_ptr(), lda, bool(a_mc), Bd.data_ptr(), ldb, bool(b_nc),
                                       C2.data_ptr(), N, alpha, beta, ks, stream())
        torch.cuda.synchronize()
        if i > 0:  # the first call may load the code object that holds the array
            assert torch.cuda.mem_get_info()[0] == free0
        assert torch.equal(C1, C2)
        ref = alpha * AB + beta * C0
        err = float(np.abs(C2.cpu().numpy() - ref).max())
        assert err <= 1e-13 * max(1.0, float(np.abs(ref).max())) * np.sqrt(K)


def test_noalloc_gemm_refuses_more_scratch_than_it_has():
    from gpu_util import stream, to_dev
    from paper_2401_11935_amd import libdcsd as L
    say("noalloc gemm oversize")
    M = N = 2048
    K = 64
    A, B, C = to_dev(np.zeros((M, K))), to_dev(np.zeros((K, N))), to_dev(np.ones((M, N)))
    # ksplit * M * ldc = 2 * 2048 * 2048 doubles > 4194304: refused on the host
    with pytest.raises(L.DcsdError) as e:
        L.selftest_gemm_layout_noalloc(M, N, K, A.data_ptr(), K, False, B.data_ptr(), N, True, C.data_ptr(), N,
                                       1.0, 0.0, 2, stream())
    assert e.value.status == L.DCSD_ERR_ARG and "32 MiB" in str(e.value)
    assert float(C.min()) == 1.0 and float(C.max()) == 1.0  # nothing ran
