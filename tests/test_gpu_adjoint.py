"""GPU: the hand-written adjoint (dcsd_residual_vjp, dcsd_backward) and its
torch.autograd bindings.

Bars:
* residual VJP against central directional differences of the GPU residual
  (h = 1e-5; T, B and F directions separately): relative 1e-7;
* gradient of the converged E_S, E_T against the oracle's derivatives
  (tests/golden/adjoint.json, tiny configuration: linear response of the
  converged oracle solution with complex-step products): relative 1e-7
  (absolute 1e-11 for entries below 1e-4);
* against central differences of re-converged GPU solves (h = 1e-5,
  tolerance 1e-12; nc=2, nv=5, naux=13) on 64 seeded entries: relative 1e-6
  of each entry, with the differences' own noise floor 1e-9 absolute.
"""
import json
import os
import sys

import numpy as np
import pytest

import dcsd_synth as synth

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


def _ctx(B, F, nc, method, **kw):
    from paper_2401_11935_amd import libdcsd as L
    from gpu_util import stream, to_dev
    Bd, Fd = to_dev(B), to_dev(F)
    cfg = L.default_config(nc=nc, nv=B.shape[1] - nc - 2, naux=B.shape[0], method=method, **kw)
    return L.Context(cfg, Bd.data_ptr(), Fd.data_ptr(), stream()), Bd, Fd


def _objective(B, F, T, nc, method, Rbar, Wbar, Ebar, lb):
    import torch
    from gpu_util import to_dev
    ctx, Bd, Fd = _ctx(B, F, nc, method, ladder_block=lb)
    Td = to_dev(T)
    Rd = torch.empty_like(Td)
    W = ctx.residual(Td.data_ptr(), Rd.data_ptr())
    e = ctx.energy(Td.data_ptr())["dE_A"]
    ctx.close()
    return float(Rbar @ Rd.cpu().numpy() + Wbar * W + Ebar * e)


@pytest.mark.parametrize("nc,nv,naux,method,lb", [(2, 5, 13, "dcsd", 0), (3, 7, 11, "ccsd", 3), (0, 6, 9, "ccsd", 2),
                                                  (3, 16, 60, "dcsd", 5), (4, 20, 30, "ccsd", 0),
                                                  (2, 5, 13, "fr-dcsd-singlet", 0), (3, 7, 11, "fr-ccsd-triplet", 3)])
def test_residual_vjp_matches_directional_differences(nc, nv, naux, method, lb):
    import torch
    from gpu_util import to_dev
    say("vjp", nc, nv, naux, method, lb)
    B, F = synth.make_inputs(nc, nv, naux, 30 + nc + nv)
    T = synth.random_amplitudes(nc, nv, 31, 0.05)
    size = T.size
    o, v = nc + 1, nv + 1
    ab = 2 * o * v + 2 * (o * v) ** 2 + (nc * o + nc) * v * v
    rng = np.random.default_rng(32)
    Rbar = rng.normal(size=size)
    Rbar[ab] = 0.0
    Wbar, Ebar = 0.7, -1.3
    ctx, Bd, Fd = _ctx(B, F, nc, method, ladder_block=lb, adjoint=1)
    Td, Rb = to_dev(T), to_dev(Rbar)
    Tb, Bb, Fb = torch.empty_like(Td), torch.empty_like(Bd), torch.empty_like(Fd)
    ctx.residual_vjp(Td.data_ptr(), Rb.data_ptr(), Wbar, Ebar, Tb.data_ptr(), Bb.data_ptr(), Fb.data_ptr())
    ctx.close()
    Tb, Bb, Fb = Tb.cpu().numpy(), Bb.cpu().numpy(), Fb.cpu().numpy()
    assert Tb[ab] == 0.0
    h = 1e-5
    for name in ("T", "B", "F"):
        dT, dB, dF = np.zeros(size), np.zeros_like(B), np.zeros_like(F)
        if name == "T":
            dT = rng.normal(size=size)
            dT[ab] = 0.0
        elif name == "B":
            dB = rng.normal(size=B.shape)
        else:
            dF = rng.normal(size=F.shape)
        fp = _objective(B + h * dB, F + h * dF, T + h * dT, nc, method, Rbar, Wbar, Ebar, lb)
        fm = _objective(B - h * dB, F - h * dF, T - h * dT, nc, method, Rbar, Wbar, Ebar, lb)
        fd = (fp - fm) / (2 * h)
        an = float(Tb @ dT + (Bb * dB).sum() + (Fb * dF).sum())
        rel = abs(fd - an) / max(abs(fd), 1e-12)
        say(f"  {name}: fd {fd:.10e} vjp {an:.10e} rel {rel:.1e}")
        assert rel <= 1e-7


def _gradients(B, F, nc, method, tol):
    import torch
    ctx, Bd, Fd = _ctx(B, F, nc, method, tol_residual=tol, max_iter=400, adjoint=1)
    T = torch.zeros(ctx.size, dtype=torch.float64, device="cuda:0")
    rep = ctx.solve(T.data_ptr())
    assert rep["status"] == "OK", rep["status"]
    out = {}
    for key, (eS, eT) in (("E_S", (1.0, 0.0)), ("E_T", (0.0, 1.0))):
        Bb, Fb, lam = torch.empty_like(Bd), torch.empty_like(Fd), torch.zeros_like(T)
        lrep = ctx.backward(T.data_ptr(), eS, eT, Bb.data_ptr(), Fb.data_ptr(), lam.data_ptr())
        assert lrep["status"] == "OK", lrep
        out[key] = (Bb.cpu().numpy(), Fb.cpu().numpy(), lam.cpu().numpy(), lrep)
    ctx.close()
    return rep, out


@pytest.mark.parametrize("method", ["dcsd", "ccsd"])
def test_backward_matches_oracle_derivatives(method):
    path = os.path.join(HERE, "golden", "adjoint.json")
    gold = json.load(open(path))
    c = gold["config"]
    B, F = synth.make_inputs(c["nc"], c["nv"], c["naux"], c["seed"])
    say("backward vs oracle", method)
    rep, g = _gradients(B, F, c["nc"], method, 1e-11)
    say(f"  E_S {rep['E_S']:.12f} (oracle {gold[method]['E_S']:.12f}); lambda iterations "
        f"{g['E_S'][3]['iterations']}, {g['E_T'][3]['iterations']}")
    worst = 0.0
    for ent in gold[method]["entries"]:
        idx = tuple(ent["index"])
        for key in ("E_S", "E_T"):
            ref = ent["d" + key]
            val = g[key][0][idx] if ent["kind"] == "B" else g[key][1][idx]
            err = abs(val - ref)
            worst = max(worst, err / max(abs(ref), 1e-4))
            assert err <= 1e-7 * max(abs(ref), 1e-4), (ent, key, val, ref)
    say(f"  worst relative difference {worst:.1e}")


def test_backward_matches_finite_differences_64_entries():
    """nc=2, nv=5, naux=13: its iterations reach max|R| <= 1e-12 in ~15 steps (the
    tiny configuration stalls near 1e-12), which the differences need."""
    cfg = synth.Config("fd", nc=2, nv=5, naux=13, seed=4)
    B, F = synth.make_config_inputs(cfg)
    nc, n = cfg.nc, cfg.n
    say("backward vs finite differences")
    rep, g = _gradients(B, F, nc, "dcsd", 1e-12)
    rng = np.random.default_rng(5)
    picks = set()
    while len(picks) < 64:
        P, p, q = int(rng.integers(cfg.naux)), int(rng.integers(n)), int(rng.integers(n))
        picks.add((P, min(p, q), max(p, q)))
    import torch
    h = 1e-5
    worst = 0.0

    def solve_E(Bx):
        ctx, Bxd, Fxd = _ctx(Bx, F, nc, "dcsd", tol_residual=1e-12, max_iter=400)  # B, F borrowed: keep
        T = torch.zeros(ctx.size, dtype=torch.float64, device="cuda:0")
        r = ctx.solve(T.data_ptr())
        ctx.close()
        assert r["status"] == "OK"
        return r["E_S"], r["E_T"]

    for (P, p, q) in sorted(picks):
        dB = np.zeros_like(B)
        if p == q:
            dB[P, p, p] = 1.0
        else:
            dB[P, p, q] = dB[P, q, p] = 0.5
        ep, em = solve_E(B + h * dB), solve_E(B - h * dB)
        for k, key in enumerate(("E_S", "E_T")):
            fd = (ep[k] - em[k]) / (2 * h)
            an = g[key][0][P, p, q]
            worst = max(worst, abs(fd - an) / max(abs(fd), 1e-3))
            assert abs(fd - an) <= 1e-6 * abs(fd) + 1e-9, ((P, p, q), key, fd, an)
    say(f"  64 entries: worst |fd - adjoint| / max(|fd|, 1e-3) = {worst:.1e}")


def test_lambda_is_antisymmetric_and_zero_at_the_internal_double():
    cfg = synth.TINY
    B, F = synth.make_config_inputs(cfg)
    say("lambda structure")
    _, g = _gradients(B, F, cfg.nc, "ccsd", 1e-10)
    lam = g["E_S"][2]
    o, v = cfg.nc + 1, cfg.nv + 1
    blocks = synth.unpack(lam, cfg.nc, cfg.nv)
    for k in ("t2aa", "t2bb"):
        x = blocks[k]
        assert np.abs(x + x.transpose(1, 0, 2, 3)).max() <= 1e-14
        assert np.abs(x + x.transpose(0, 1, 3, 2)).max() <= 1e-14
    assert blocks["t2ab"][cfg.nc, cfg.nc, 0, 0] == 0.0
    assert np.abs(lam).max() > 0.0 and o * v > 0


def test_torch_autograd_energy_and_residual():
    import torch
    from paper_2401_11935_amd.autograd import Problem
    cfg = synth.TINY
    B, F = synth.make_config_inputs(cfg)
    say("autograd")
    Bd = torch.from_numpy(B).cuda().requires_grad_(True)
    Fd = torch.from_numpy(F).cuda().requires_grad_(True)
    prob = Problem(Bd.detach(), Fd.detach(), cfg.nc, tol_residual=1e-11, max_iter=400)
    # route gradients to the leaf tensors that share storage with the problem's
    ES, ET = prob.energies(prob.B.requires_grad_(True), prob.F.requires_grad_(True))
    gB, gF = torch.autograd.grad(ES - 0.5 * ET, [prob.B, prob.F])
    _, g = _gradients(B, F, cfg.nc, "dcsd", 1e-11)
    ref_B = g["E_S"][0] - 0.5 * g["E_T"][0]
    ref_F = g["E_S"][1] - 0.5 * g["E_T"][1]
    assert np.abs(gB.cpu().numpy() - ref_B).max() <= 1e-10 * max(1.0, np.abs(ref_B).max())
    assert np.abs(gF.cpu().numpy() - ref_F).max() <= 1e-10 * max(1.0, np.abs(ref_F).max())
    # residual: d/dT of (R . c) through autograd equals the VJP with cotangent c
    T = torch.from_numpy(synth.random_amplitudes(cfg.nc, cfg.nv, 41, 0.03)).cuda().requires_grad_(True)
    R, W, E = prob.residual(T, prob.B, prob.F)
    c = torch.from_numpy(np.random.default_rng(42).normal(size=T.numel())).cuda()
    (gT,) = torch.autograd.grad((R * c).sum() + 2.0 * W - E, [T])
    Tb = torch.empty_like(T)
    prob.ctx.residual_vjp(T.detach().data_ptr(), c.data_ptr(), 2.0, -1.0, Tb.data_ptr())
    # (the coupling adjoint accumulates with atomics: equal up to summation order)
    assert torch.allclose(gT, Tb, rtol=1e-12, atol=1e-13)
    prob.close()


def test_residual_vjp_at_adjoint_size():
    """nc=8, nv=200, naux=600 (the adjoint configuration; its amplitude
    equations do not converge on these inputs, so the VJP of one residual is
    checked, with the ladder batches recomputed in the sweep)."""
    import torch
    from gpu_util import to_dev
    c = synth.ADJOINT
    B, F = synth.make_config_inputs(c)
    T = synth.random_amplitudes(c.nc, c.nv, 51, 0.01)
    rng = np.random.default_rng(52)
    size = T.size
    o, v = c.nc + 1, c.nv + 1
    ab = 2 * o * v + 2 * (o * v) ** 2 + (c.nc * o + c.nc) * v * v
    Rbar = rng.normal(size=size)
    Rbar[ab] = 0.0
    say("vjp adjoint size")
    ctx, Bd, Fd = _ctx(B, F, c.nc, "dcsd", adjoint=1)
    Td, Rb = to_dev(T), to_dev(Rbar)
    Tb, Bb = torch.empty_like(Td), torch.empty_like(Bd)
    ctx.residual_vjp(Td.data_ptr(), Rb.data_ptr(), 0.3, 0.9, Tb.data_ptr(), Bb.data_ptr(), 0)
    Tb, Bb = Tb.cpu().numpy(), Bb.cpu().numpy()
    h = 1e-5
    dT = rng.normal(size=size)
    dT[ab] = 0.0
    dB = rng.normal(size=B.shape)

    def obj(Bx, Tx):
        cx, Bxd, Fxd = _ctx(Bx, F, c.nc, "dcsd")  # the context borrows B and F: keep both alive
        Txd = to_dev(Tx)
        Rx = torch.empty_like(Txd)
        W = cx.residual(Txd.data_ptr(), Rx.data_ptr())
        e = cx.energy(Txd.data_ptr())["dE_A"]
        cx.close()
        return float(Rbar @ Rx.cpu().numpy() + 0.3 * W + 0.9 * e)

    ctx.close()
    for name, (dTx, dBx) in (("T", (dT, 0 * dB)), ("B", (0 * dT, dB))):
        fd = (obj(B + h * dBx, T + h * dTx) - obj(B - h * dBx, T - h * dTx)) / (2 * h)
        an = float(Tb @ dTx + (Bb * dBx).sum())
        rel = abs(fd - an) / max(abs(fd), 1e-12)
        say(f"  {name}: fd {fd:.10e} vjp {an:.10e} rel {rel:.1e}")
        assert rel <= 1e-6


def test_backward_at_the_adjoint_shape_with_weak_integrals():
    """The adjoint configuration's shape (nc=8, nv=200, naux=600, seed 1) with weak
    integrals (naux sigma^2 = 0.015 Eh), on which the amplitude equations converge:
    dcsd_backward against central differences (h = 1e-5) of re-converged solves
    (tol 1e-14, started from the converged amplitudes) on 64 seeded entries of B and
    8 of F, for E_S and E_T, to 1e-6 relative plus 2e-10 (the differences' noise:
    energies converged to ~1e-15, over 2h).  The B entries have a core or open-shell
    row (B[P, i, q], q any): entries with two virtual indices have gradients of
    ~4e-7 (median), below what the differences resolve at 1e-6."""
    import torch
    from gpu_util import to_dev
    cfg = synth.MEDIUM_WEAK
    B, F = synth.make_config_inputs(cfg)
    nc, n = cfg.nc, cfg.n
    say("backward vs finite differences, nc=8 nv=200 naux=600 weak integrals")
    ctx, Bd, Fd = _ctx(B, F, nc, "dcsd", tol_residual=1e-14, max_iter=400, adjoint=1)
    T = torch.zeros(ctx.size, dtype=torch.float64, device="cuda:0")
    rep = ctx.solve(T.data_ptr())
    assert rep["status"] == "OK", rep
    g = {}
    for key, (eS, eT) in (("E_S", (1.0, 0.0)), ("E_T", (0.0, 1.0))):
        Bb, Fb, lam = torch.empty_like(Bd), torch.empty_like(Fd), torch.zeros_like(T)
        lrep = ctx.backward(T.data_ptr(), eS, eT, Bb.data_ptr(), Fb.data_ptr(), lam.data_ptr())
        assert lrep["status"] == "OK", lrep
        g[key] = (Bb.cpu().numpy(), Fb.cpu().numpy())
    ctx.close()
    T0 = T.cpu().numpy()
    say(f"  converged in {rep['iterations']} iterations, E_S {rep['E_S']:.12f}")
    rng = np.random.default_rng(5)
    picks = set()
    while len(picks) < 64:
        P, p, q = int(rng.integers(cfg.naux)), int(rng.integers(nc + 2)), int(rng.integers(n))
        picks.add(("B", P, min(p, q), max(p, q)))
    fpicks = set()
    while len(fpicks) < 8:
        p, q = int(rng.integers(n)), int(rng.integers(n))
        fpicks.add(("F", 0, min(p, q), max(p, q)))
    h = 1e-5

    def solve_E(Bx, Fx):
        cx, Bxd, Fxd = _ctx(Bx, Fx, nc, "dcsd", tol_residual=1e-14, max_iter=400)  # borrowed: keep alive
        Tx = to_dev(T0)
        r = cx.solve(Tx.data_ptr())
        cx.close()
        assert r["status"] == "OK", r["status"]
        return r["E_S"], r["E_T"]

    worst = 0.0
    for (kind, P, p, q) in sorted(picks) + sorted(fpicks):
        d = np.zeros_like(B[0] if kind == "F" else B)
        tgt = d if kind == "F" else d[P]
        if p == q:
            tgt[p, p] = 1.0
        else:
            tgt[p, q] = tgt[q, p] = 0.5
        if kind == "B":
            ep, em = solve_E(B + h * d, F), solve_E(B - h * d, F)
        else:
            ep, em = solve_E(B, F + h * d), solve_E(B, F - h * d)
        for k, key in enumerate(("E_S", "E_T")):
            fd = (ep[k] - em[k]) / (2 * h)
            an = g[key][0][P, p, q] if kind == "B" else g[key][1][p, q]
            worst = max(worst, abs(fd - an) / max(abs(fd), 1e-3))
            assert abs(fd - an) <= 1e-6 * abs(fd) + 2e-10, ((kind, P, p, q), key, fd, an)
    say(f"  72 entries: worst |fd - adjoint| / max(|fd|, 1e-3) = {worst:.1e}")
