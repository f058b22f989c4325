"""Writes the stored expected values under tests/golden/ by calling only the
CPU oracle (``oracle/``) on the seeded synthetic inputs of ``dcsd_synth``.

    python tests/golden/make_golden.py tiny        # seconds
    python tests/golden/make_golden.py medium      # hours on a few CPU cores

tiny:   converged 2D-DCSD and 2D-CCSD energies (tol 1e-10) at nc=3, nv=16,
        naux=60, seed 0, plus the per-iteration trajectory.
small:  converged energies at nc=8, nv=20, naux=60, seed 1 (the largest of
        these synthetic inputs on which the iterations converge from zero).
medium: nc=8, nv=200, naux=600, seed 1: residual at seeded random amplitudes
        sampled at 4096 seeded positions (for both methods), and the converged
        energies of both methods.
medium-weak: the medium shape and seed with weak integrals (DF factors with
        naux sigma^2 = 0.015 Eh, dcsd_synth.MEDIUM_WEAK), on which the iterations
        converge: converged energies and trajectory of both methods (tol 1e-10)
        and the converged amplitudes at 4096 seeded positions.  Hours on a few
        CPU cores (about 20 oracle residuals per method).

medium-half-weak: the same with nv=100, naux=300 (dcsd_synth.MEDIUM_HALF_WEAK): converged
        energies, trajectory and sampled amplitudes of both methods; minutes per method.

    python tests/golden/make_golden.py medium-weak [dcsd|ccsd]
    python tests/golden/make_golden.py medium-half-weak [dcsd|ccsd]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import dcsd_synth as synth  # noqa: E402
from oracle.solver import solve  # noqa: E402
from oracle.twodet import TwoDet  # noqa: E402

AMP_SEED = 101        # seed of the random amplitudes used for residual parity
AMP_SCALE = 0.02
SAMPLE_SEED = 202
NSAMPLE = 4096


def converged(cfg, method, tol):
    B, F = synth.make_config_inputs(cfg)
    model = TwoDet(B, F, cfg.nc, method)
    t0 = time.time()
    r = solve(model, tol=tol, max_iter=300,
              callback=lambda rec: print(method, rec["iter"], "%.3e" % rec["res_max"], rec["E_S"], flush=True))
    return {
        "converged": r["converged"], "iterations": r["iterations"], "tol": tol,
        "E_S": r["E_S"], "E_T": r["E_T"], "dE_A": r["dE_A"], "W": r["W"], "E_ref_A": r["E_ref_A"],
        "res_max": r["res_max"], "seconds": time.time() - t0,
        "trajectory": [{k: rec[k] for k in ("iter", "res_max", "E_S", "E_T", "W")} for rec in r["records"]],
    }


def sampled_residual(cfg, method):
    B, F = synth.make_config_inputs(cfg)
    model = TwoDet(B, F, cfg.nc, method)
    T = synth.random_amplitudes(cfg.nc, cfg.nv, AMP_SEED, AMP_SCALE)
    t0 = time.time()
    R, W = model.residual(T)
    idx = synth.sample_indices(NSAMPLE, R.size, SAMPLE_SEED)
    return {"amp_seed": AMP_SEED, "amp_scale": AMP_SCALE, "sample_seed": SAMPLE_SEED,
            "positions": idx.tolist(), "values": R[idx].tolist(), "W": W,
            "dE_A": model.energy_A(T), "res_max": float(np.abs(R).max()),
            "res_norm2": float(np.dot(R, R)), "seconds": time.time() - t0}


SMALL = synth.Config("small", nc=8, nv=20, naux=60, seed=1)


def converged_with_amplitudes(cfg, method, tol):
    B, F = synth.make_config_inputs(cfg)
    model = TwoDet(B, F, cfg.nc, method)
    t0 = time.time()
    r = solve(model, tol=tol, max_iter=300,
              callback=lambda rec: print(method, rec["iter"], "%.3e" % rec["res_max"], rec["E_S"],
                                         "%.0f s" % (time.time() - t0), flush=True))
    idx = synth.sample_indices(NSAMPLE, r["T"].size, SAMPLE_SEED)
    return {
        "converged": r["converged"], "iterations": r["iterations"], "tol": tol,
        "E_S": r["E_S"], "E_T": r["E_T"], "dE_A": r["dE_A"], "W": r["W"], "E_ref_A": r["E_ref_A"],
        "res_max": r["res_max"], "seconds": time.time() - t0,
        "trajectory": [{k: rec[k] for k in ("iter", "res_max", "E_S", "E_T", "W")} for rec in r["records"]],
        "sample_seed": SAMPLE_SEED, "positions": idx.tolist(), "T": r["T"][idx].tolist(),
        "T_max": float(np.abs(r["T"]).max()),
    }


def main_weak(methods, cfg=synth.MEDIUM_WEAK, name="medium_weak.json"):
    path = os.path.join(HERE, name)
    out = json.load(open(path)) if os.path.exists(path) else {}
    out["config"] = {"nc": cfg.nc, "nv": cfg.nv, "naux": cfg.naux, "seed": cfg.seed, "sigma": cfg.sigma}
    for method in methods:
        out[method] = converged_with_amplitudes(cfg, method, 1e-10)
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print("wrote", path, flush=True)


def main(which):
    if which in ("medium-weak", "medium-half-weak"):
        methods = [m for m in ("dcsd", "ccsd") if m in sys.argv[2:]] or ["dcsd", "ccsd"]
        if which == "medium-weak":
            return main_weak(methods)
        return main_weak(methods, synth.MEDIUM_HALF_WEAK, "medium_half_weak.json")
    cfg = {"tiny": synth.TINY, "small": SMALL, "medium": synth.MEDIUM}[which]
    out = {"config": {"nc": cfg.nc, "nv": cfg.nv, "naux": cfg.naux, "seed": cfg.seed}}
    for method in ("dcsd", "ccsd"):
        out[method] = {"residual": sampled_residual(cfg, method)}
        if which != "medium" or "--no-solve" not in sys.argv:
            out[method]["solve"] = converged(cfg, method, 1e-9 if which == "medium" else 1e-10)
        path = os.path.join(HERE, f"{which}.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print("wrote", path, flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "tiny")
