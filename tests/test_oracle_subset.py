"""Oracle: virtual-subset locality of the residual.

In every term of the singles and doubles equations (Theory section) a summed
virtual index is an index of an amplitude, and the one-electron part sums over
occupied orbitals only.  So if T vanishes outside a subset S of the virtuals,
each residual element whose external virtual indices lie in {t, u} and S
equals the residual of the problem restricted to the orbitals core, t, u and S,
and so do W and the energies.  A summed virtual index that is not an
amplitude's (for example a term with a full virtual trace, or a wrong index
that runs over the integrals' virtual range) breaks this.

This is what lets the GPU tests check every term at full size against the
oracle on the reduced problem."""
import numpy as np
import pytest

import dcsd_synth as synth
from oracle.fixedref import FixedRef
from oracle.twodet import TwoDet

NC, NV, NAUX = 2, 9, 30
KEEP = [1, 4, 8]


def _problem(method, B, F):
    if method.startswith("fr-"):
        _, m, state = method.split("-")
        return FixedRef(B, F, NC, m, state)
    return TwoDet(B, F, NC, method)


@pytest.mark.parametrize("method", ["dcsd", "ccsd", "fr-dcsd-triplet"])
def test_residual_on_virtual_subset_equals_reduced_problem(method):
    B, F = synth.make_inputs(NC, NV, NAUX, 21)
    Bs, Fs = synth.subset_inputs(B, F, NC, KEEP)
    Ts = synth.random_amplitudes(NC, len(KEEP), 22, 0.1)
    T = synth.embed_amplitudes(Ts, NC, KEEP, NV)
    full, red = _problem(method, B, F), _problem(method, Bs, Fs)
    R, W = full.residual(T)
    Rs, Ws = red.residual(Ts)
    assert np.abs(synth.restrict_amplitudes(R, NC, NV, KEEP) - Rs).max() <= 1e-13
    assert abs(W - Ws) <= 1e-14
    e, es_ = full.energies(T, W), red.energies(Ts, Ws)
    for k in ("dE_A", "E_ref_A"):
        assert abs(e[k] - es_[k]) <= 1e-13
    # the elements outside the subset are not trivially zero (the driver term alone fills them)
    outside = np.abs(R).sum() - np.abs(synth.restrict_amplitudes(R, NC, NV, KEEP)).sum()
    assert outside > 1e-3


def test_subset_locality_detects_a_virtual_trace():
    """A planted term with a free virtual sum (trace of f_vv times t2) breaks the
    property: the check above is sensitive to that class of mistake."""
    B, F = synth.make_inputs(NC, NV, NAUX, 21)
    Bs, Fs = synth.subset_inputs(B, F, NC, KEEP)
    Ts = synth.random_amplitudes(NC, len(KEEP), 22, 0.1)
    T = synth.embed_amplitudes(Ts, NC, KEEP, NV)

    def planted(p, vec):
        R, _ = p.residual(vec)
        _, t2 = p.ham.to_so(vec)
        fvv = p.ints["fvv"]
        R1, R2 = p.ham.to_so(R)
        return p.ham.from_so(R1, R2 + 1e-2 * np.trace(fvv) * t2)

    full, red = TwoDet(B, F, NC, "dcsd"), TwoDet(Bs, Fs, NC, "dcsd")
    d = np.abs(synth.restrict_amplitudes(planted(full, T), NC, NV, KEEP) - planted(red, Ts)).max()
    assert d > 1e-6
