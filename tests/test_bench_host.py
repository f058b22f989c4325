"""Host-side logic of bench.py (no GPU): the one-GPU contract and the flop
counts that the roofline and TFLOP/s figures use."""
import json
import os
import subprocess
import sys

import bench

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_algorithmic_flops_at_the_metric_shape():
    # naux V_u^4 over the distinct (ac),(bd) pairs; 2 o^2 v^4 + 4 P_o P_v^2; ten 2 (ov)^3
    a = bench.algorithmic_flops(12, 400, 1200)
    vu, o, v = 402, 13, 401
    assert a["assembly"] == 1200.0 * vu ** 4
    po, pv = o * (o - 1) / 2, v * (v - 1) / 2
    assert a["contraction"] == 2.0 * o * o * v ** 4 + 4.0 * po * pv * pv
    assert a["rings"] == 10 * 2.0 * (o * v) ** 3
    assert abs(a["total"] - 4.49e13) < 0.01e13
    # per assembly launch (91 batches of 32 orbitals) as the roofline uses it
    assert abs(a["assembly"] / 91 - 3.444e11) < 0.001e11


def test_executed_flops_exceed_the_algorithmic_count():
    ex = bench.flop_model(12, 400, 1200, 32)
    al = bench.algorithmic_flops(12, 400, 1200)
    assert ex["assembly"] > al["assembly"] and ex["contraction"] > al["contraction"]
    assert abs(sum(ex.values()) - 5.36e13) < 0.01e13


def test_triples_flops_count_only_spin_allowed_blocks():
    # nc = 1: occupied [3 alpha | 1 beta]. The alpha^3 triple has, per order, one block of va rows;
    # each of the three triples with the beta orbital has two orders (y, z of different spin)
    # with blocks of va and vb rows and one (y, z both alpha) with va rows: 12 va + 6 vb rows
    # in all, each a GEMM of rows x nV^2 x n.
    nc, nv = 1, 4
    va, vb, n, nV = nv, nv + 2, nc + 2 + nv, 2 * nv + 2
    assert bench.triples_flops(nc, nv) == 2.0 * (12 * va + 6 * vb) * nV * nV * n
