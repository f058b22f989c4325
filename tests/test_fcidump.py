"""FCIDUMP ingestion (paper_2401_11935_amd/fcidump.py), on the CPU.

Pins: the parser against a hand-written file (eight-fold symmetry, one-electron
and core-energy lines); the pivoted Cholesky factors reproduce the integrals
to their tolerance; and a round trip synthetic (B, F) -> FCIDUMP in shuffled
orbital order -> load_problem gives back F and, since B enters only through
(pq|rs), the oracle's residual and energies unchanged."""
import numpy as np
import pytest

import dcsd_synth as synth
from oracle.hamiltonian import Hamiltonian
from oracle.twodet import TwoDet
from paper_2401_11935_amd import fcidump as fd

TEXT = """&FCI NORB=  2,NELEC= 2,MS2= 0,
 ORBSYM=1,1,
 ISYM=1,
&END
  0.5  1  1  1  1
  0.25D0  2  1  1  1
  0.125  2  1  2  1
  0.375  2  2  1  1
  0.75  2  2  2  2
  -1.5  1  1  0  0
  0.1  2  1  0  0
  -0.5  2  2  0  0
  0.7  0  0  0  0
"""


def test_parser_fills_eight_fold_symmetry(tmp_path):
    p = tmp_path / "FCIDUMP"
    p.write_text(TEXT)
    d = fd.read_fcidump(str(p))
    assert (d["norb"], d["nelec"], d["ms2"]) == (2, 2, 0)
    assert d["e_core"] == 0.7
    assert np.array_equal(d["h"], np.array([[-1.5, 0.1], [0.1, -0.5]]))
    e = d["eri"]
    assert e[0, 0, 0, 0] == 0.5 and e[1, 1, 1, 1] == 0.75
    for x in [e[1, 0, 0, 0], e[0, 1, 0, 0], e[0, 0, 1, 0], e[0, 0, 0, 1]]:
        assert x == 0.25
    for x in [e[1, 0, 1, 0], e[0, 1, 0, 1], e[1, 0, 0, 1], e[0, 1, 1, 0]]:
        assert x == 0.125
    assert e[1, 1, 0, 0] == 0.375 and e[0, 0, 1, 1] == 0.375
    assert e[1, 1, 1, 0] == 0.0  # absent from the file


def test_pivoted_cholesky_reproduces_the_integrals():
    B, _ = synth.make_inputs(2, 6, 14, 3)
    eri = np.einsum("Ppq,Prs->pqrs", B, B)
    L = fd.pivoted_cholesky(eri, tol=1e-12)
    assert L.shape[0] <= B.shape[0]
    assert np.abs(np.einsum("Ppq,Prs->pqrs", L, L) - eri).max() < 1e-10
    assert np.abs(L - L.transpose(0, 2, 1)).max() == 0.0


@pytest.mark.parametrize("nc,nv,naux,seed", [(2, 5, 12, 4), (1, 6, 30, 9)])
def test_round_trip_keeps_fock_residual_and_energies(tmp_path, nc, nv, naux, seed):
    B, F = synth.make_inputs(nc, nv, naux, seed)
    n = nc + 2 + nv
    h = Hamiltonian(B, F, nc).h  # the oracle's h = F - G_avg[B]
    eri = np.einsum("Ppq,Prs->pqrs", B, B)
    perm = np.random.default_rng(seed).permutation(n)  # file orbital i = model orbital perm[i]
    inv = np.argsort(perm)
    path = tmp_path / "FCIDUMP"
    fd.write_fcidump(str(path), h[np.ix_(perm, perm)], eri[np.ix_(perm, perm, perm, perm)], nelec=2 * nc + 2,
                     e_core=1.25)
    core = [int(inv[k]) for k in range(nc)]
    virt = [int(inv[k]) for k in range(nc + 2, n)]
    prob = fd.load_problem(str(path), core=core, t=int(inv[nc]), u=int(inv[nc + 1]), virt=virt, tol=1e-12)
    assert (prob["nc"], prob["nv"], prob["e_core"], prob["nelec"]) == (nc, nv, 1.25, 2 * nc + 2)
    assert np.abs(prob["F"] - F).max() < 1e-10
    T = synth.random_amplitudes(nc, nv, seed + 1, 0.05)
    for method in ("dcsd", "ccsd"):
        a, b = TwoDet(B, F, nc, method), TwoDet(prob["B"], prob["F"], nc, method)
        Ra, Wa = a.residual(T)
        Rb, Wb = b.residual(T)
        assert np.abs(Ra - Rb).max() < 1e-10 and abs(Wa - Wb) < 1e-12
        assert abs(a.energy_A(T) - b.energy_A(T)) < 1e-12
        assert abs(a.ham.e_ref() - b.ham.e_ref()) < 1e-10


def test_bad_inputs_are_rejected(tmp_path):
    p = tmp_path / "bad"
    p.write_text("not a dump\n")
    with pytest.raises(ValueError):
        fd.read_fcidump(str(p))
    with pytest.raises(ValueError):
        fd.reorder(np.eye(3), np.zeros((3, 3, 3, 3)), [0, 0, 1])
