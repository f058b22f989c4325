"""Perturbative triples correction (T) of a single-determinant reference (oracle).

Test infrastructure only: nothing on the product path imports this module.

The paper places its method among two-determinant CC variants and mentions
perturbative-triples extensions of 2D-CCSD only as other work (Introduction);
it gives no triples formula of its own.  This module therefore follows the
standard (T) correction of single-reference CCSD, applied to the one
single-determinant reference this code treats, the M_s = 1 high-spin
determinant Phi_T (highspin.py), with the converged CCSD or DCSD amplitudes
of that reference (DCSD(T) uses the same expression with DC amplitudes).

In spin orbitals, with the spin-orbital Fock matrix f of the reference and
the antisymmetrised integrals <pq||rs>:

  connected numerator
    N^c_ijk^abc = P(i/jk) P(a/bc) [ sum_e t_jk^ae <ei||bc> - sum_m t_im^bc <ma||jk> ]
  disconnected numerator
    N^d_ijk^abc = P(i/jk) P(a/bc) [ t_i^a <jk||bc> + f_ia t_jk^bc ]
  denominator
    D_ijk^abc = f_ii + f_jj + f_kk - f_aa - f_bb - f_cc      (Fock diagonal)
  energy
    E_(T) = 1/36 sum_{ijkabc} N^c (N^c + N^d) / D

with P(i/jk) g(ijk) = g(ijk) - g(jik) - g(kji) and P(a/bc) likewise.  The
three parts are reported separately: E[4]_T (N^c N^c), E[5]_ST (N^c times the
t1 term) and E_DT (N^c times the f_ov t2 term, which vanishes for a
Hartree-Fock reference and is kept because Phi_T's Fock matrix has an
occupied-virtual block).  Readings where the paper is silent: the Fock
diagonal in the denominators (no semicanonical rotation; the off-diagonal
occupied-occupied and virtual-virtual elements are left out of the
perturbation denominators), and the f_ov t2 disconnected term.

Pinned by (tests/test_oracle_triples.py): the determinant engine -- for
random t1, t2 the numerators are projections <X| H T2 |Phi>, <X| F_ov T2 |Phi>
and <X| H (T1 + T2) |Phi> onto the triple excitations X, so that E_(T) is a
sum over triple determinants computed without any tensor formula; two
electrons have no triples (E_(T) = 0); the per-triple sum equals the dense
sum.
"""
from __future__ import annotations

import itertools

import numpy as np

from .hamiltonian import Hamiltonian


def _p_i_jk(x: np.ndarray) -> np.ndarray:
    """P(i/jk) on the first three axes: g(ijk) - g(jik) - g(kji)."""
    return x - x.transpose(1, 0, 2, 3, 4, 5) - x.transpose(2, 1, 0, 3, 4, 5)


def _p_a_bc(x: np.ndarray) -> np.ndarray:
    """P(a/bc) on the last three axes: g(abc) - g(bac) - g(cba)."""
    return x - x.transpose(0, 1, 2, 4, 3, 5) - x.transpose(0, 1, 2, 5, 4, 3)


def _integrals(ham: Hamiltonian) -> dict:
    O, V = ham.O, ham.V
    f_oo, f_vv = ham.fock(O, O), ham.fock(V, V)
    return {
        "vovv": ham.asym(V, O, V, V),   # <ei||bc>
        "ovoo": ham.asym(O, V, O, O),   # <ma||jk>
        "oovv": ham.asym(O, O, V, V),   # <jk||bc>
        "fov": ham.fock(O, V),
        "fo": np.diag(f_oo).copy(),
        "fv": np.diag(f_vv).copy(),
    }


def numerators(ham: Hamiltonian, t1: np.ndarray, t2: np.ndarray, ints: dict | None = None):
    """Dense N^c, the two disconnected numerators and D over all (ijk, abc)."""
    g = ints or _integrals(ham)
    x = np.einsum("jkae,eibc->ijkabc", t2, g["vovv"], optimize=True)
    y = np.einsum("imbc,majk->ijkabc", t2, g["ovoo"], optimize=True)
    nc = _p_a_bc(_p_i_jk(x - y))
    d1 = _p_a_bc(_p_i_jk(np.einsum("ia,jkbc->ijkabc", t1, g["oovv"], optimize=True)))
    d2 = _p_a_bc(_p_i_jk(np.einsum("ia,jkbc->ijkabc", g["fov"], t2, optimize=True)))
    fo, fv = g["fo"], g["fv"]
    D = (fo[:, None, None, None, None, None] + fo[None, :, None, None, None, None]
         + fo[None, None, :, None, None, None] - fv[None, None, None, :, None, None]
         - fv[None, None, None, None, :, None] - fv[None, None, None, None, None, :])
    return nc, d1, d2, D


def triples_energy(ham: Hamiltonian, t1: np.ndarray, t2: np.ndarray) -> dict:
    """E_(T) and its parts for spin-orbital amplitudes of the reference of ``ham``."""
    nc, d1, d2, D = numerators(ham, t1, t2)
    if nc.size == 0:
        return {"E_T4": 0.0, "E_ST5": 0.0, "E_DT": 0.0, "E_T": 0.0}
    # D vanishes only where every numerator does (an index repeated in ijk or abc)
    with np.errstate(divide="ignore", invalid="ignore"):
        w = np.where(np.abs(nc) > 0.0, nc / D, 0.0)
    e4 = float(np.sum(w * nc)) / 36.0
    e5 = float(np.sum(w * d1)) / 36.0
    edt = float(np.sum(w * d2)) / 36.0
    return {"E_T4": e4, "E_ST5": e5, "E_DT": edt, "E_T": e4 + e5 + edt}


class _DirectIntegrals:
    """The integral slices one occupied triple needs, formed on demand from the DF
    factors (for inputs whose dense <ei||bc> array would not fit in host memory)."""

    def __init__(self, ham: Hamiltonian):
        self.ham = ham
        O, V = ham.O, ham.V
        f_oo, f_vv = ham.fock(O, O), ham.fock(V, V)
        self.fov, self.fo, self.fv = ham.fock(O, V), np.diag(f_oo).copy(), np.diag(f_vv).copy()

    def vovv_slab(self, p):   # <ep||bc> as [e][b][c]
        ham = self.ham
        return ham.asym(ham.V, ham.sub(ham.O, p), ham.V, ham.V)[:, 0]

    def ovoo_pair(self, q, r):   # <ma||qr> as [m][a]
        ham = self.ham
        return ham.asym(ham.O, ham.V, ham.sub(ham.O, q), ham.sub(ham.O, r))[:, :, 0, 0]

    def oovv_pair(self, q, r):   # <qr||bc> as [b][c]
        ham = self.ham
        return ham.asym(ham.sub(ham.O, q), ham.sub(ham.O, r), ham.V, ham.V)[0, 0]


class _DenseIntegrals:
    def __init__(self, g: dict):
        self.g = g
        self.fov, self.fo, self.fv = g["fov"], g["fo"], g["fv"]

    def vovv_slab(self, p):
        return self.g["vovv"][:, p]

    def ovoo_pair(self, q, r):
        return self.g["ovoo"][:, :, q, r]

    def oovv_pair(self, q, r):
        return self.g["oovv"][q, r]


def triple_contribution(ham: Hamiltonian, t1: np.ndarray, t2: np.ndarray, i: int, j: int, k: int,
                        ints: dict | None = None, direct: bool = False) -> float:
    """Contribution of one occupied triple i < j < k, summed over all virtual
    (a, b, c): 1/6 sum_abc N^c (N^c + N^d) / D.  Each step is one matrix
    product or elementwise operation for the three orderings of (i, j, k), so
    that large inputs can be sampled triple by triple; with direct=True only
    the integrals of i, j and k are formed."""
    src = _DirectIntegrals(ham) if direct else _DenseIntegrals(ints or _integrals(ham))
    g = {"fov": src.fov, "fo": src.fo, "fv": src.fv}
    nv = t2.shape[2]

    def z(p, q, r):   # sum_e t_qr^ae <ep||bc> - sum_m t_pm^bc <ma||qr>, as [a][b][c]
        xa = t2[q, r] @ src.vovv_slab(p).reshape(nv, nv * nv)
        ya = src.ovoo_pair(q, r).T @ t2[p].reshape(-1, nv * nv)
        return (xa - ya).reshape(nv, nv, nv)

    zt = z(i, j, k) - z(j, i, k) - z(k, j, i)
    ncv = zt - zt.transpose(1, 0, 2) - zt.transpose(2, 1, 0)

    def s(p, q, r):   # t_p^a <qr||bc> + f_pa t_qr^bc, as [a][b][c]
        return src.oovv_pair(q, r)[None] * t1[p][:, None, None] + t2[q, r][None] * g["fov"][p][:, None, None]

    st = s(i, j, k) - s(j, i, k) - s(k, j, i)
    ndv = st - st.transpose(1, 0, 2) - st.transpose(2, 1, 0)
    fo, fv = g["fo"], g["fv"]
    D = fo[i] + fo[j] + fo[k] - fv[:, None, None] - fv[None, :, None] - fv[None, None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        w = np.where(np.abs(ncv) > 0.0, ncv / D, 0.0)
    return float(np.sum(w * (ncv + ndv))) / 6.0


def triples_by_triple(ham: Hamiltonian, t1: np.ndarray, t2: np.ndarray) -> float:
    """E_(T) as the sum of triple_contribution over all i < j < k."""
    g = _integrals(ham)
    no = t2.shape[0]
    return sum(triple_contribution(ham, t1, t2, i, j, k, g) for i, j, k in itertools.combinations(range(no), 3))
