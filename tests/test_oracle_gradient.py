"""The oracle's energy derivatives (linear response of the converged solution
with complex-step products, as written into tests/golden/adjoint.json, the
reference for the adjoint) against central finite differences of converged
real solves."""
import importlib.util
import os

import numpy as np
import pytest

import dcsd_synth as synth
from oracle.solver import solve
from oracle.twodet import TwoDet

NC, NV, NAUX, SEED = 2, 5, 13, 4
HERE = os.path.dirname(os.path.abspath(__file__))


def golden_module():
    spec = importlib.util.spec_from_file_location("make_adjoint_golden",
                                                  os.path.join(HERE, "golden", "make_adjoint_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def energies(B, F, method):
    r = solve(TwoDet(B, F, NC, method), tol=1e-12, max_iter=300)
    assert r["converged"]
    return r["E_S"], r["E_T"]


@pytest.mark.parametrize("method", ["dcsd", "ccsd"])
@pytest.mark.parametrize("kind,idx", [("B", (8, 7, 0)), ("B", (10, 4, 4)), ("F", (5, 3))])
def test_linear_response_matches_central_differences(method, kind, idx):
    g = golden_module()
    B0, F0 = synth.make_inputs(NC, NV, NAUX, SEED)
    d = g.direction(B0.shape if kind == "B" else F0.shape, idx)
    dB, dF = (d, np.zeros_like(F0)) if kind == "B" else (np.zeros_like(B0), d)
    model = TwoDet(B0, F0, NC, method)
    r = solve(model, tol=1e-13, max_iter=300)
    lr = g.linear_response(model, r["T"], dB, dF, B0, F0, NC, method)
    h = 1e-4
    p = energies(B0 + h * dB, F0 + h * dF, method)
    m = energies(B0 - h * dB, F0 - h * dF, method)
    for k in range(2):
        fd = (p[k] - m[k]) / (2 * h)
        # O(h^2) truncation and the 1e-12 solve tolerance leave ~1e-7 of the derivative
        assert abs(lr[k] - fd) <= 1e-6 * max(abs(fd), 1e-3), (k, lr[k], fd)
