"""The oracle's single-element particle-particle ladder (used for sampled
checks at the full problem sizes) against the slab-batched ladder of the full
CCSD residual, which the brute-force determinant tests pin, on every element
of small systems; and the antisymmetry it inherits in the same-spin blocks."""
import numpy as np
import pytest

import dcsd_synth as synth
from oracle.ccsd import SlabSource, ladder_element
from oracle.hamiltonian import Hamiltonian


@pytest.mark.parametrize("nc,nv,naux,seed", [(2, 5, 13, 1), (3, 7, 11, 2), (0, 6, 9, 3)])
def test_ladder_element_matches_slab_ladder(nc, nv, naux, seed):
    B, F = synth.make_inputs(nc, nv, naux, seed)
    vec = synth.random_amplitudes(nc, nv, seed + 7, 0.1)
    blocks = synth.unpack(vec, nc, nv)
    blocks["t1a"][:] = 0.0
    blocks["t1b"][:] = 0.0
    ham = Hamiltonian(B, F, nc)
    _, t2 = ham.to_so(vec)
    L = synth.unpack(ham.from_so(np.zeros((2 * ham.o, 2 * ham.v)), SlabSource(ham).ladder(t2)), nc, nv)
    o, v = nc + 1, nv + 1
    for blk, name in enumerate(("t2aa", "t2bb", "t2ab")):
        ref = L[name]
        got = np.array([[[[ladder_element(B, nc, blocks[name], blk, i, j, a, b) for b in range(v)] for a in range(v)]
                         for j in range(o)] for i in range(o)])
        assert np.abs(got - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max()), name
        if blk < 2:  # antisymmetric amplitudes give an antisymmetric ladder
            assert np.abs(got + got.transpose(0, 1, 3, 2)).max() <= 1e-13
