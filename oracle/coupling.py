"""Coupling coefficients between the two reference determinants (oracle).

The 2D amplitude equations (Theory section, singles and doubles equations)
add to the connected single-reference residual a renormalisation term M_x W.
Following the Bloch equation with the Jeziorski-Monkhorst wave operator the
paper starts from, projecting

    H e^{T_A}|A> = e^{T_A}|A> H_AA + e^{T_B}|B> H_BA

onto <A^x| e^{-T_A} gives M_x = -K_x with

    K_x = <A^x| e^{-T_A} e^{T_B} |B>,

T_B being the spin flip of T_A (the amplitudes of Phi_B are those of Phi_A
with every spin label flipped).  |A^x> = a+_a a+_b a_j a_i |A> for doubles and
a+_a a_i |A> for singles; |B> = a+_{u alpha} a+_{t beta} a_{u beta} a_{t alpha} |A>.
Its expansion contains the disconnected products the paper writes out with
the antisymmetriser and the restriction operator, and in the incomplete
active space case the products of the internal (t <-> u) singles.  Terms
with the same spin-orbital twice never arise in exact fermion algebra, which
is how they are omitted here.

K_x only involves amplitudes whose spin-orbitals lie in L(x) = {t alpha,
u beta, u alpha, t beta} + the orbitals of x, so it is evaluated exactly in
the Fock space of those at most eight spin-orbitals: e^{T_B} is applied to
|B> and then e^{-T_A} to the result (nilpotent Taylor series), and the
coefficient of A^x is read off.  Excitations x are grouped by which of their
indices are the open-shell orbitals t, u; inside a group every amplitude is
an array over the remaining (core or virtual) indices, so one local
calculation serves the whole group.

Pinned by: the determinant engine's <A^x| e^-T_A e^T_B |B> for random T
(tests/test_oracle_brute.py) and two-electron FCI of the converged
equations.
"""
from __future__ import annotations

import itertools

import numpy as np

ALPHA, BETA = 0, 1


class Amplitudes:
    """Lookup of T_A and T_B amplitudes for symbolic spin-orbitals.

    A spin-orbital is (spin, kind, axis) with kind in {'core','t','u','virt'};
    'core' and 'virt' carry the grid axis they range over."""

    def __init__(self, blocks: dict, nc: int, nv: int, ndim: int):
        self.b = blocks
        self.nc, self.nv, self.ndim = nc, nv, ndim

    def _axis(self, values, axis):
        shape = [1] * self.ndim
        shape[axis] = len(values)
        return np.asarray(values).reshape(shape)

    def occ_pos(self, d):
        spin, kind, ax = d
        if kind == "core":
            return self._axis(np.arange(self.nc), ax)
        if (kind, spin) in (("t", ALPHA), ("u", BETA)):
            return self.nc
        raise ValueError("not occupied in Phi_A")

    def vir_pos(self, d):
        spin, kind, ax = d
        if kind == "virt":
            return self._axis(1 + np.arange(self.nv), ax)
        if (kind, spin) in (("u", ALPHA), ("t", BETA)):
            return 0
        raise ValueError("not virtual in Phi_A")

    def t1(self, h, p):
        if h[0] != p[0]:
            return 0.0
        blk = self.b["t1a"] if h[0] == ALPHA else self.b["t1b"]
        return blk[self.occ_pos(h), self.vir_pos(p)]

    def t2(self, h1, h2, p1, p2):
        s = (h1[0], h2[0], p1[0], p2[0])
        if s == (ALPHA, ALPHA, ALPHA, ALPHA):
            return self.b["t2aa"][self.occ_pos(h1), self.occ_pos(h2), self.vir_pos(p1), self.vir_pos(p2)]
        if s == (BETA, BETA, BETA, BETA):
            return self.b["t2bb"][self.occ_pos(h1), self.occ_pos(h2), self.vir_pos(p1), self.vir_pos(p2)]
        if s == (ALPHA, BETA, ALPHA, BETA):
            return self.b["t2ab"][self.occ_pos(h1), self.occ_pos(h2), self.vir_pos(p1), self.vir_pos(p2)]
        if s == (ALPHA, BETA, BETA, ALPHA):
            return -self.b["t2ab"][self.occ_pos(h1), self.occ_pos(h2), self.vir_pos(p2), self.vir_pos(p1)]
        if h1[0] == BETA and h2[0] == ALPHA:
            return -self.t2(h2, h1, p1, p2)
        return 0.0

    @staticmethod
    def flip(d):
        return (1 - d[0], d[1], d[2])

    def t1_B(self, h, p):
        return self.t1(self.flip(h), self.flip(p))

    def t2_B(self, h1, h2, p1, p2):
        f = self.flip
        return self.t2(f(h1), f(h2), f(p1), f(p2))


def occupied_in(d, ref: str) -> bool:
    spin, kind, _ = d
    if kind == "core":
        return True
    if kind == "virt":
        return False
    if ref == "A":
        return (kind, spin) in (("t", ALPHA), ("u", BETA))
    return (kind, spin) in (("u", ALPHA), ("t", BETA))


def _apply(mask: int, ops):
    """Apply a string of creation ('c', k) / annihilation ('a', k) operators,
    rightmost first, to a local determinant bitmask.  Returns (mask, sign) or
    None if the result vanishes."""
    sign = 1
    for kind, k in reversed(ops):
        bit = 1 << k
        below = bin(mask & (bit - 1)).count("1")
        if kind == "a":
            if not mask & bit:
                return None
            mask ^= bit
        else:
            if mask & bit:
                return None
            mask |= bit
        if below % 2:
            sign = -sign
    return mask, sign


def _excitation_terms(L, amps: Amplitudes, ref: str):
    """T (relative to reference ref) restricted to the local orbitals L:
    list of (amplitude, operator string)."""
    occ = [k for k, d in enumerate(L) if occupied_in(d, ref)]
    vir = [k for k, d in enumerate(L) if not occupied_in(d, ref)]
    t1 = amps.t1 if ref == "A" else amps.t1_B
    t2 = amps.t2 if ref == "A" else amps.t2_B
    terms = []
    for h in occ:
        for p in vir:
            a = t1(L[h], L[p])
            if not (np.isscalar(a) and a == 0.0):
                terms.append((a, [("c", p), ("a", h)]))
    for h1, h2 in itertools.combinations(occ, 2):
        for p1, p2 in itertools.combinations(vir, 2):
            a = t2(L[h1], L[h2], L[p1], L[p2])
            if not (np.isscalar(a) and a == 0.0):
                terms.append((a, [("c", p1), ("c", p2), ("a", h2), ("a", h1)]))
    return terms


def _apply_terms(vec: dict, terms) -> dict:
    out = {}
    for mask, c in vec.items():
        for amp, ops in terms:
            r = _apply(mask, ops)
            if r is None:
                continue
            m2, s = r
            val = (s * amp) * c
            out[m2] = out[m2] + val if m2 in out else val
    return out


def _exp_apply(vec: dict, terms, factor: float) -> dict:
    """e^{factor T} vec by its (finite) Taylor series."""
    result = dict(vec)
    cur = vec
    for k in range(1, 64):
        cur = _apply_terms(cur, terms)
        if not cur:
            break
        cur = {m: c * (factor / k) for m, c in cur.items()}
        for m, c in cur.items():
            result[m] = result[m] + c if m in result else c
    return result


T_A = (ALPHA, "t", None)
U_B = (BETA, "u", None)
U_A = (ALPHA, "u", None)
T_B = (BETA, "t", None)
ACTIVE = [T_A, U_B, U_A, T_B]


def local_coupling(holes, parts, amps: Amplitudes, grid_shape):
    """K_x for x = holes -> parts (1 or 2 of each), as an array over the grid.

    |A^x> = a+_{p1} (a+_{p2}) (a_{h2}) a_{h1} |A>."""
    L = list(ACTIVE)
    for d in list(holes) + list(parts):
        if d not in L:
            L.append(d)
    idx = {d: k for k, d in enumerate(L)}
    a_mask = sum(1 << k for k, d in enumerate(L) if occupied_in(d, "A"))
    b = _apply(a_mask, [("c", idx[U_A]), ("c", idx[T_B]), ("a", idx[U_B]), ("a", idx[T_A])])
    if len(holes) == 1:
        xops = [("c", idx[parts[0]]), ("a", idx[holes[0]])]
    else:
        xops = [("c", idx[parts[0]]), ("c", idx[parts[1]]), ("a", idx[holes[1]]), ("a", idx[holes[0]])]
    x = _apply(a_mask, xops)
    vec = {b[0]: float(b[1])}
    vec = _exp_apply(vec, _excitation_terms(L, amps, "B"), 1.0)
    vec = _exp_apply(vec, _excitation_terms(L, amps, "A"), -1.0)
    val = vec.get(x[0], 0.0)
    return np.broadcast_to(x[1] * np.asarray(val), grid_shape).copy()


def coupling(blocks: dict, nc: int, nv: int) -> dict:
    """K_x for every single and double of Phi_A, in the packed block layout.

    The element of the Phi_A -> Phi_B double is set to zero (its residual is
    W itself, and that element is not solved for)."""
    o, v = nc + 1, nv + 1
    dt = np.result_type(*blocks.values())
    K = {"t1a": np.zeros((o, v), dt), "t1b": np.zeros((o, v), dt),
         "t2aa": np.zeros((o, o, v, v), dt), "t2bb": np.zeros((o, o, v, v), dt), "t2ab": np.zeros((o, o, v, v), dt)}

    def occ_choices(spin, axis):
        act = T_A if spin == ALPHA else U_B
        return [((spin, "core", axis), slice(0, nc), nc), (act, slice(nc, nc + 1), 1)]

    def vir_choices(spin, axis):
        act = U_A if spin == ALPHA else T_B
        return [((spin, "virt", axis), slice(1, v), nv), (act, slice(0, 1), 1)]

    # singles
    for spin, name in ((ALPHA, "t1a"), (BETA, "t1b")):
        for (hi, si, ni), (pa, sa, na) in itertools.product(occ_choices(spin, 0), vir_choices(spin, 1)):
            amps = Amplitudes(blocks, nc, nv, 2)
            if ni == 0 or na == 0:
                continue
            K[name][si, sa] = local_coupling([hi], [pa], amps, (ni, na))
    # doubles
    for s1, s2, name in ((ALPHA, ALPHA, "t2aa"), (BETA, BETA, "t2bb"), (ALPHA, BETA, "t2ab")):
        for (hi, si, ni), (hj, sj, nj), (pa, sa, na), (pb, sb, nb) in itertools.product(
                occ_choices(s1, 0), occ_choices(s2, 1), vir_choices(s1, 2), vir_choices(s2, 3)):
            if 0 in (ni, nj, na, nb):
                continue
            if hi == hj or pa == pb:      # same open-shell spin-orbital twice
                continue
            if name == "t2ab" and (hi, hj, pa, pb) == (T_A, U_B, U_A, T_B):
                continue                  # the Phi_A -> Phi_B double
            amps = Amplitudes(blocks, nc, nv, 4)
            K[name][si, sj, sa, sb] = local_coupling([hi, hj], [pa, pb], amps, (ni, nj, na, nb))
    # a repeated core or virtual index is not an excitation
    for name in ("t2aa", "t2bb"):
        idx = np.arange(nc)
        K[name][idx, idx] = 0.0
        iv = np.arange(1, v)
        K[name][:, :, iv, iv] = 0.0
    return K
