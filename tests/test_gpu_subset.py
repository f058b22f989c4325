"""GPU: every term of the residual at full size, element by element, through
virtual-subset locality.

With T zero outside a subset S of the virtuals, the residual elements whose
virtual indices lie in {t, u} and S, and W and the energies, equal those of the
problem restricted to core, t, u and S (each summed virtual index of the
singles and doubles equations is an amplitude index; pinned on the oracle in
tests/test_oracle_subset.py).  The library runs at the full sizes, in the
benchmark's launch configuration (automatic ladder blocking). The oracle runs
on the reduced problem, which takes seconds. S holds the first and last
virtuals, those at the 128-wide tile edges of the pair dimension, and random
ones.  Bars: residual 1e-9 absolute and 1e-10 relative to max(1, max|R|); W and
energies 1e-11 relative to max(1, |value|)."""
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


def _keep(nv: int, seed: int) -> list[int]:
    # virt position k is pair-dimension index k + 2 (t, u first): tile edges at 128 m
    edges = [k for m in range(1, nv // 128 + 1) for k in (128 * m - 3, 128 * m - 2) if k < nv]
    rng = np.random.default_rng(seed)
    extra = rng.choice(nv, size=18, replace=False).tolist()
    return sorted(set([0, 1, nv - 2, nv - 1] + edges + extra))


def _oracle(method, B, F, nc):
    if method.startswith("fr-"):
        from oracle.fixedref import FixedRef
        _, m, state = method.split("-")
        return FixedRef(B, F, nc, m, state)
    from oracle.twodet import TwoDet
    return TwoDet(B, F, nc, method)


CASES = [(synth.MIXED, "dcsd"), (synth.MIXED, "ccsd"), (synth.MIXED, "fr-ccsd-singlet"),
         (synth.LARGEST, "dcsd"), (synth.LARGEST, "ccsd")]


@pytest.mark.timeout(400)
@pytest.mark.parametrize("cfg,method", CASES, ids=[f"{c.name}-{m}" for c, m in CASES])
def test_full_size_residual_on_virtual_subset(cfg, method):
    from gpu_util import GpuProblem
    nc, nv = cfg.nc, cfg.nv
    say("subset residual", cfg.name, method, "inputs")
    B, F = synth.make_config_inputs(cfg)
    keep = _keep(nv, cfg.seed + 31)
    Bs, Fs = synth.subset_inputs(B, F, nc, keep)
    Ts = synth.random_amplitudes(nc, len(keep), cfg.seed + 32, 0.05)
    say("subset residual", cfg.name, method, f"oracle on {len(keep)} virtuals")
    orc = _oracle(method, Bs, Fs, nc)
    Rs, Ws = orc.residual(Ts)
    es = orc.energies(Ts, Ws)
    T = synth.embed_amplitudes(Ts, nc, keep, nv)
    say("subset residual", cfg.name, method, "library")
    p = GpuProblem(B, F, nc, method)
    R, W = p.residual(T)
    e = p.energy(T)
    if method == "dcsd":
        # run to run, the full-size launches (split-K, skipped diagonal tiles and their mirror,
        # fixed-order reductions) give the same bits
        R2, W2 = p.residual(T)
        assert np.array_equal(R, R2) and W == W2
        del R2
    p.close()
    del T
    Rsub = synth.restrict_amplitudes(R, nc, nv, keep)
    err = float(np.abs(Rsub - Rs).max())
    say(f"  max|dR| = {err:.3e} over {Rs.size} elements (max|R| {np.abs(Rs).max():.3e}), |dW| = {abs(W - Ws):.2e}")
    assert err <= 1e-9  # the stated FP64 bar: residual max-norm within 1e-9
    assert err <= 1e-10 * max(1.0, float(np.abs(Rs).max()))
    close = lambda a, b: abs(a - b) <= 1e-11 * max(1.0, abs(b))  # noqa: E731
    assert close(W, Ws)
    for k in ("dE_A", "E_ref_A"):
        assert close(e[k], es[k]), k
    for k in ("E_S", "E_T"):
        assert (np.isnan(e[k]) and np.isnan(es[k])) or close(e[k], es[k]), k


LOWP_BARS = {"fp32": 2e-6, "bf16": 1e-2}


@pytest.mark.timeout(400)
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_full_size_lowp_residual_on_virtual_subset(precision):
    """The residual with FP32 or BF16 ladder and ring GEMMs at the metric size (as
    the benchmark times it), on the virtual subset, against the FP64 oracle of the
    reduced problem.  Bars as for the low-precision residual at small sizes:
    2e-6 s (FP32) and 1e-2 s (BF16), s = max(1, max|R|)."""
    from gpu_util import GpuProblem
    cfg = synth.MIXED
    nc, nv = cfg.nc, cfg.nv
    say("subset lowp residual", precision, "inputs")
    B, F = synth.make_config_inputs(cfg)
    keep = _keep(nv, cfg.seed + 41)
    Bs, Fs = synth.subset_inputs(B, F, nc, keep)
    Ts = synth.random_amplitudes(nc, len(keep), cfg.seed + 42, 0.05)
    say("subset lowp residual", precision, f"oracle on {len(keep)} virtuals")
    Rs, Ws = _oracle("dcsd", Bs, Fs, nc).residual(Ts)
    T = synth.embed_amplitudes(Ts, nc, keep, nv)
    say("subset lowp residual", precision, "library")
    p = GpuProblem(B, F, nc, "dcsd", precision=precision)
    R, W = p.residual(T)
    p.close()
    del T
    err = float(np.abs(synth.restrict_amplitudes(R, nc, nv, keep) - Rs).max())
    s = max(1.0, float(np.abs(Rs).max()))
    say(f"  max|dR| = {err:.3e} (bar {LOWP_BARS[precision] * s:.1e}), |dW| = {abs(W - Ws):.2e}")
    assert err <= LOWP_BARS[precision] * s
    assert abs(W - Ws) <= LOWP_BARS[precision] * s
    assert err > 1e-13  # the low-precision path ran


VJP_CASES = [(synth.MIXED, "dcsd"), (synth.MIXED, "fr-ccsd-triplet")]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("cfg,method", VJP_CASES, ids=[f"{c.name}-{m}" for c, m in VJP_CASES])
def test_full_size_residual_vjp_on_virtual_subset(cfg, method):
    """The residual VJP (dcsd_residual_vjp) at the metric size with T and Rbar on the
    virtual subset.  The objective Rbar.R + Wbar W + Ebar dE_A then depends on the
    reduced B, F and T only, so (1) Bbar and Fbar vanish outside the reduced orbital
    block (bar 1e-10 of their largest entry), and (2) along random directions in the
    reduced space, Tbar.dT, Bbar.dB and Fbar.dF equal the oracle's complex-step
    derivatives of the reduced objective (h = 1e-20; relative bar 1e-9)."""
    import torch
    from paper_2401_11935_amd import libdcsd as L
    from gpu_util import stream, to_dev
    nc, nv = cfg.nc, cfg.nv
    say("subset vjp", cfg.name, method, "inputs")
    B, F = synth.make_config_inputs(cfg)
    keep = _keep(nv, cfg.seed + 51)
    idx = np.concatenate([np.arange(nc + 2), nc + 2 + np.asarray(keep)])
    Bs, Fs = synth.subset_inputs(B, F, nc, keep)
    Ts = synth.random_amplitudes(nc, len(keep), cfg.seed + 52, 0.05)
    orc = _oracle(method, Bs, Fs, nc)
    rng = np.random.default_rng(cfg.seed + 53)
    Rbar_s = rng.normal(size=Ts.size)
    Rbar_s[orc.ab] = 0.0
    Wbar, Ebar = 0.7, -1.3

    say("subset vjp", cfg.name, method, "library")
    Bd, Fd = to_dev(B), to_dev(F)
    ctx = L.Context(L.default_config(nc=nc, nv=nv, naux=cfg.naux, method=method, adjoint=1), Bd.data_ptr(),
                    Fd.data_ptr(), stream())
    Td = to_dev(synth.embed_amplitudes(Ts, nc, keep, nv))
    Rb = to_dev(synth.embed_amplitudes(Rbar_s, nc, keep, nv))
    Tb, Bb, Fb = torch.empty_like(Td), torch.empty_like(Bd), torch.empty_like(Fd)
    ctx.residual_vjp(Td.data_ptr(), Rb.data_ptr(), Wbar, Ebar, Tb.data_ptr(), Bb.data_ptr(), Fb.data_ptr())
    ctx.close()
    Tb_s = synth.restrict_amplitudes(Tb.cpu().numpy(), nc, nv, keep)
    Bb, Fb = Bb.cpu().numpy(), Fb.cpu().numpy()
    del Td, Rb, Tb, Bd, Fd
    Bb_s, Fb_s = Bb[:, idx][:, :, idx], Fb[np.ix_(idx, idx)]
    Bb[:, idx[:, None], idx[None, :]] = 0.0
    Fb[np.ix_(idx, idx)] = 0.0
    say(f"  outside the reduced block: max|Bbar| {np.abs(Bb).max():.2e} (inside {np.abs(Bb_s).max():.2e}), "
        f"max|Fbar| {np.abs(Fb).max():.2e} (inside {np.abs(Fb_s).max():.2e})")
    assert np.abs(Bb).max() <= 1e-10 * np.abs(Bb_s).max()
    assert np.abs(Fb).max() <= 1e-10 * np.abs(Fb_s).max()
    del Bb, Fb

    def objective(p, T):
        R, W = p.residual(T)
        return Rbar_s @ R + Wbar * W + Ebar * p.energy_A(T)

    h = 1e-20
    # a direction of amplitudes: same-spin doubles antisymmetric, the A->B double zero (Tbar is
    # the derivative with respect to the packed entries, which include both (i,j) and (j,i))
    dT = synth.random_amplitudes(nc, len(keep), cfg.seed + 54, 1.0)
    dB = rng.normal(size=Bs.shape)
    dB = 0.5 * (dB + dB.transpose(0, 2, 1))
    dF = rng.normal(size=Fs.shape)
    dF = 0.5 * (dF + dF.T)
    for name, an, make in (("T", float(Tb_s @ dT), lambda: objective(orc, Ts + 1j * h * dT)),
                           ("B", float((Bb_s * dB).sum()), lambda: objective(_oracle(method, Bs + 1j * h * dB, Fs, nc), Ts)),
                           ("F", float((Fb_s * dF).sum()), lambda: objective(_oracle(method, Bs + 0j, Fs + 1j * h * dF, nc), Ts))):
        say("subset vjp", cfg.name, method, "oracle complex step", name)
        cs = float(np.imag(make())) / h
        rel = abs(cs - an) / max(abs(cs), 1e-12)
        say(f"  {name}: oracle {cs:.12e} vjp {an:.12e} rel {rel:.1e}")
        assert rel <= 1e-9
