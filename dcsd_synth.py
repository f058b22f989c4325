"""Seeded synthetic inputs for the two-determinant DCSD/CCSD residual.

This module is shared by the CPU oracle, the tests and the benchmark. It only
draws random numbers and lays them out; it contains none of the method's
arithmetic.

Orbital order (spatial): ``[core 0..nc-1 | t = nc | u = nc+1 | virt nc+2..n-1]``
with ``n = nc + 2 + nv``.  ``t`` and ``u`` are the two singly occupied orbitals
of the open-shell singlet (Theory section, the two determinants of Fig. 1).

Packed amplitude / residual layout (FP64, row-major), relative to
``Phi_A = |core, t alpha, u beta>``::

    [ t1a (o,v) | t1b (o,v) | t2aa (o,o,v,v) | t2bb (o,o,v,v) | t2ab (o,o,v,v) ]

with ``o = nc + 1`` and ``v = nv + 1`` per spin.  Per-spin index order:
alpha-occ = [core, t], alpha-vir = [u, virt], beta-occ = [core, u],
beta-vir = [t, virt].  Same-spin doubles are stored in full and are
antisymmetric in (i,j) and in (a,b).  The element t2ab[nc, nc, 0, 0] is the
excitation of Phi_A into Phi_B and is always zero.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SIGMA_B = 0.05          # standard deviation of the DF factors
SIGMA_F_OFF = 1.0e-3    # standard deviation of off-diagonal Fock elements
# Weak-integral variants: DF factors with naux * sigma^2 = 0.015 Eh, the mean
# exchange integral (pq|qp).  With sigma = 0.05 that mean is 1.5 Eh (nc=8, nv=200)
# or 3 Eh (nc=12, nv=400): far stronger correlation than a molecule's, and the
# amplitude iterations diverge.  At 0.015 Eh the correlation energies are
# molecule-sized (about -0.4 and -1.7 Eh) and the iterations converge.
WEAK_EXCHANGE = 0.015


def weak_sigma(naux: int) -> float:
    return float(np.sqrt(WEAK_EXCHANGE / naux))


@dataclass(frozen=True)
class Config:
    name: str
    nc: int
    nv: int
    naux: int
    seed: int
    sigma: float = SIGMA_B

    @property
    def n(self) -> int:
        return self.nc + 2 + self.nv

    @property
    def o(self) -> int:
        return self.nc + 1

    @property
    def v(self) -> int:
        return self.nv + 1


# The five workloads (sizes and seeds).
TINY = Config("tiny", nc=3, nv=16, naux=60, seed=0)
MEDIUM = Config("medium", nc=8, nv=200, naux=600, seed=1)
ADJOINT = Config("adjoint", nc=8, nv=200, naux=600, seed=1)
MIXED = Config("mixed", nc=12, nv=400, naux=1200, seed=2)
LARGEST = Config("largest", nc=20, nv=600, naux=1800, seed=3)
CONFIGS = {c.name: c for c in (TINY, MEDIUM, ADJOINT, MIXED, LARGEST)}
# The same shapes and seeds with weak integrals (added configurations).
MEDIUM_WEAK = Config("medium-weak", nc=8, nv=200, naux=600, seed=1, sigma=weak_sigma(600))
# the medium core count and seed with half its virtuals (converged solves of the oracle in minutes)
MEDIUM_HALF_WEAK = Config("medium-half-weak", nc=8, nv=100, naux=300, seed=1, sigma=weak_sigma(300))
MIXED_WEAK = Config("mixed-weak", nc=12, nv=400, naux=1200, seed=2, sigma=weak_sigma(1200))
LARGEST_WEAK = Config("largest-weak", nc=20, nv=600, naux=1800, seed=3, sigma=weak_sigma(1800))
WEAK_CONFIGS = {c.name: c for c in (MEDIUM_HALF_WEAK, MEDIUM_WEAK, MIXED_WEAK, LARGEST_WEAK)}


def amplitude_count(nc: int, nv: int) -> int:
    o, v = nc + 1, nv + 1
    return 2 * o * v + 3 * o * o * v * v


def block_offsets(nc: int, nv: int) -> dict:
    """Offsets and shapes of the five blocks in the packed vector."""
    o, v = nc + 1, nv + 1
    out, off = {}, 0
    for name, shape in (("t1a", (o, v)), ("t1b", (o, v)), ("t2aa", (o, o, v, v)),
                        ("t2bb", (o, o, v, v)), ("t2ab", (o, o, v, v))):
        size = int(np.prod(shape))
        out[name] = (off, shape)
        off += size
    return out


def unpack(vec: np.ndarray, nc: int, nv: int) -> dict:
    """Views of the five blocks of a packed vector (no copy)."""
    return {k: vec[off:off + int(np.prod(shape))].reshape(shape)
            for k, (off, shape) in block_offsets(nc, nv).items()}


def pack(blocks: dict, nc: int, nv: int) -> np.ndarray:
    dt = np.result_type(np.float64, *[np.asarray(b) for b in blocks.values()])
    out = np.zeros(amplitude_count(nc, nv), dt)
    for k, (off, shape) in block_offsets(nc, nv).items():
        out[off:off + int(np.prod(shape))] = np.asarray(blocks[k], dtype=dt).ravel()
    return out


def _symmetric_draw(rng, naux: int, n: int, sigma: float) -> np.ndarray:
    """Upper triangle (q >= p) drawn iid N(0, sigma^2) in C order over
    (P, p, q), then mirrored, so every entry keeps the stated marginal."""
    iu = np.triu_indices(n)
    B = np.empty((naux, n, n))
    draws = rng.normal(0.0, sigma, size=(naux, iu[0].size))
    for P in range(naux):
        M = np.zeros((n, n))
        M[iu] = draws[P]
        B[P] = M + np.triu(M, 1).T
    return B


def _fock(rng, nc: int, nv: int) -> np.ndarray:
    n = nc + 2 + nv
    d = np.concatenate([rng.uniform(-2.0, -0.5, nc),
                        rng.uniform(-0.4, -0.2, 2),
                        rng.uniform(0.2, 3.0, nv)])
    iu = np.triu_indices(n, 1)
    off = rng.normal(0.0, SIGMA_F_OFF, size=iu[0].size)
    F = np.zeros((n, n))
    F[iu] = off
    F = F + F.T
    F[np.diag_indices(n)] = d
    return F


def make_inputs(nc: int, nv: int, naux: int, seed: int, sigma: float = SIGMA_B):
    """DF factors B[P,p,q] (naux, n, n) and spin-averaged Fock F (n, n).

    B entries ~ N(0, sigma^2) (0.05 unless given), symmetric in (p,q); F
    diagonal: core U[-2,-0.5], t and u U[-0.4,-0.2], virtuals U[0.2,3];
    off-diagonal N(0, 1e-3^2), symmetric.  Generator: numpy PCG64 seeded with
    ``seed``; B is drawn first.
    """
    rng = np.random.default_rng(seed)
    n = nc + 2 + nv
    B = _symmetric_draw(rng, naux, n, sigma)
    F = _fock(rng, nc, nv)
    return B, F


def make_config_inputs(cfg: Config):
    return make_inputs(cfg.nc, cfg.nv, cfg.naux, cfg.seed, cfg.sigma)


def make_z2_inputs(nc: int, nv: int, naux: int, seed: int):
    """Inputs with a Z2 point-group symmetry in which t and u belong to
    different irreducible representations (complete active space case).

    Orbital irreps alternate (core and virtuals), t is even and u is odd;
    each auxiliary function gets an irrep too.  B[P,p,q] vanishes unless
    g(P)+g(p)+g(q) is even, F[p,q] vanishes unless g(p) == g(q).
    """
    B, F = make_inputs(nc, nv, naux, seed)
    n = nc + 2 + nv
    g = np.zeros(n, dtype=int)
    g[:nc] = np.arange(nc) % 2
    g[nc] = 0
    g[nc + 1] = 1
    g[nc + 2:] = np.arange(nv) % 2
    gP = np.arange(naux) % 2
    mask = ((gP[:, None, None] + g[None, :, None] + g[None, None, :]) % 2) == 0
    F = np.where(g[:, None] == g[None, :], F, 0.0)
    return B * mask, F, g


def add_fragment(B: np.ndarray, F: np.ndarray, nc: int, nf_vir: int, seed: int):
    """Append a non-interacting closed-shell two-electron fragment.

    The fragment has one doubly occupied orbital (placed as the last core
    orbital) and ``nf_vir`` virtuals (placed after the original virtuals).
    Its DF factors live on their own auxiliary functions, so no integral
    couples it to the original system.  Returns (B', F', nc+1, frag) where
    ``frag`` holds the fragment's own B and F (orbital order [occ | virt]).
    """
    rng = np.random.default_rng(seed)
    naux, n, _ = B.shape
    nv = n - nc - 2
    nfa = max(4, 2 * (nf_vir + 1))
    nf = 1 + nf_vir
    Bf = _symmetric_draw(rng, nfa, nf, SIGMA_B * 3)
    Ff = np.zeros((nf, nf))
    Ff[0, 0] = rng.uniform(-2.0, -0.5)
    Ff[np.arange(1, nf), np.arange(1, nf)] = rng.uniform(0.2, 3.0, nf_vir)
    # new orbital order: [core (nc) | frag occ | t | u | virt (nv) | frag virt]
    n2 = n + nf
    old = np.concatenate([np.arange(nc), np.arange(nc + 1, nc + 3 + nv)])
    frag = np.concatenate([[nc], np.arange(nc + 3 + nv, n2)])
    B2 = np.zeros((naux + nfa, n2, n2))
    B2[np.ix_(np.arange(naux), old, old)] = B
    B2[np.ix_(np.arange(naux, naux + nfa), frag, frag)] = Bf
    F2 = np.zeros((n2, n2))
    F2[np.ix_(old, old)] = F
    F2[np.ix_(frag, frag)] = Ff
    return B2, F2, nc + 1, {"B": Bf, "F": Ff}


# ---- high-spin (M_s = 1) triplet reference Phi_T = |core, t alpha, u alpha> ----------
# Per-spin orders: alpha-occ = [core, t, u], beta-occ = [core], alpha-vir = [virt],
# beta-vir = [t, u, virt]; packed [t1a | t1b | t2aa | t2bb | t2ab] with
# oa = nc + 2, ob = nc, va = nv, vb = nv + 2.
def hs_dims(nc: int, nv: int):
    return nc + 2, nc, nv, nv + 2


def hs_block_offsets(nc: int, nv: int) -> dict:
    oa, ob, va, vb = hs_dims(nc, nv)
    out, off = {}, 0
    for name, shape in (("t1a", (oa, va)), ("t1b", (ob, vb)), ("t2aa", (oa, oa, va, va)),
                        ("t2bb", (ob, ob, vb, vb)), ("t2ab", (oa, ob, va, vb))):
        size = int(np.prod(shape))
        out[name] = (off, shape)
        off += size
    return out


def hs_amplitude_count(nc: int, nv: int) -> int:
    oa, ob, va, vb = hs_dims(nc, nv)
    return oa * va + ob * vb + oa * oa * va * va + ob * ob * vb * vb + oa * ob * va * vb


def hs_unpack(vec: np.ndarray, nc: int, nv: int) -> dict:
    return {k: vec[off:off + int(np.prod(shape))].reshape(shape)
            for k, (off, shape) in hs_block_offsets(nc, nv).items()}


def hs_pack(blocks: dict, nc: int, nv: int) -> np.ndarray:
    dt = np.result_type(np.float64, *[np.asarray(b) for b in blocks.values()])
    out = np.zeros(hs_amplitude_count(nc, nv), dt)
    for k, (off, shape) in hs_block_offsets(nc, nv).items():
        out[off:off + int(np.prod(shape))] = np.asarray(blocks[k], dtype=dt).ravel()
    return out


def hs_random_amplitudes(nc: int, nv: int, seed: int, scale: float = 0.05) -> np.ndarray:
    """Random packed high-spin amplitudes, same-spin doubles antisymmetric."""
    rng = np.random.default_rng(seed)
    oa, ob, va, vb = hs_dims(nc, nv)
    blocks = {"t1a": rng.normal(0, scale, (oa, va)), "t1b": rng.normal(0, scale, (ob, vb))}
    for name, (o, v) in (("t2aa", (oa, va)), ("t2bb", (ob, vb))):
        x = rng.normal(0, scale, (o, o, v, v))
        x = x - x.transpose(1, 0, 2, 3)
        blocks[name] = x - x.transpose(0, 1, 3, 2)
    blocks["t2ab"] = rng.normal(0, scale, (oa, ob, va, vb))
    return hs_pack(blocks, nc, nv)


def random_amplitudes(nc: int, nv: int, seed: int, scale: float = 0.05) -> np.ndarray:
    """Random packed amplitudes with the layout's symmetries: same-spin
    doubles antisymmetric in (i,j) and (a,b); the Phi_A -> Phi_B element zero."""
    rng = np.random.default_rng(seed)
    o, v = nc + 1, nv + 1
    t1a = rng.normal(0, scale, (o, v))
    t1b = rng.normal(0, scale, (o, v))
    x = rng.normal(0, scale, (o, o, v, v))
    t2aa = x - x.transpose(1, 0, 2, 3)
    t2aa = t2aa - t2aa.transpose(0, 1, 3, 2)
    x = rng.normal(0, scale, (o, o, v, v))
    t2bb = x - x.transpose(1, 0, 2, 3)
    t2bb = t2bb - t2bb.transpose(0, 1, 3, 2)
    t2ab = rng.normal(0, scale, (o, o, v, v))
    t2ab[nc, nc, 0, 0] = 0.0
    return pack({"t1a": t1a, "t1b": t1b, "t2aa": t2aa, "t2bb": t2bb, "t2ab": t2ab}, nc, nv)


def sample_indices(count: int, total: int, seed: int) -> np.ndarray:
    """Distinct sorted sample positions of a packed vector (for sampled parity)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(total, size=min(count, total), replace=False))


def subset_inputs(B: np.ndarray, F: np.ndarray, nc: int, keep) -> tuple[np.ndarray, np.ndarray]:
    """B and F restricted to the orbitals [core | t | u | virt[keep]], where keep
    holds sorted positions among the nv virtuals."""
    idx = np.concatenate([np.arange(nc + 2), nc + 2 + np.asarray(keep, dtype=np.int64)])
    return np.ascontiguousarray(B[:, idx][:, :, idx]), np.ascontiguousarray(F[np.ix_(idx, idx)])


def _vir_positions(keep) -> np.ndarray:
    """Per-spin virtual index (u or t first, then virt) of each virtual of a subset."""
    return np.concatenate([[0], 1 + np.asarray(keep, dtype=np.int64)])


def embed_amplitudes(vec_sub: np.ndarray, nc: int, keep, nv: int) -> np.ndarray:
    """Packed full-space amplitudes equal to vec_sub (amplitudes over the subset
    [core | t | u | virt[keep]]) on the kept virtuals and zero elsewhere."""
    sub = unpack(vec_sub, nc, len(keep))
    m = _vir_positions(keep)
    out = np.zeros(amplitude_count(nc, nv))
    for k, blk in unpack(out, nc, nv).items():
        if k.startswith("t1"):
            blk[:, m] = sub[k]
        else:
            for i in range(blk.shape[0]):
                blk[i][:, m[:, None], m[None, :]] = sub[k][i]
    return out


def restrict_amplitudes(vec: np.ndarray, nc: int, nv: int, keep) -> np.ndarray:
    """The elements of a packed full-space vector whose virtual indices lie on the
    subset [t | u | virt[keep]], packed for that subset."""
    full = unpack(vec, nc, nv)
    m = _vir_positions(keep)
    return pack({k: (b[:, m] if k.startswith("t1") else b[:, :, m[:, None], m[None, :]]) for k, b in full.items()},
                nc, len(keep))
