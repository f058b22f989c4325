"""Single-reference CCSD residual of Phi_A, spin-orbital, explicit T1 (oracle).

The 2D amplitude equations (Theory section, singles and doubles equations)
start from the connected single-reference term <x| H_N e^{T_A} |A>_C, which is
exactly the CCSD residual R_x = <x| e^{-T} H e^{T} |A> for x a single or a
double.  This module writes that residual in the textbook spin-orbital form
with Stanton-Gauss intermediates (non-canonical Fock matrix, so f_ov, f_oo and
f_vv off-diagonal terms are kept; the residual equals right-hand side minus
D*t with D from the diagonal of f).

Integrals with three or four virtual indices are never stored: they are
formed one occupied (respectively one virtual) index at a time from the DF
factors, and the spatial integral of each slab is shared by both spins.

Pinned by: brute-force <x| e^-T H e^T |A> of the determinant engine for
random T (tests/test_oracle_brute.py); the MP2 closed form after one
iteration; orbital-rotation invariance of converged energies.
"""
from __future__ import annotations

import numpy as np

from .hamiltonian import Hamiltonian

es = lambda *a: np.einsum(*a, optimize=True)  # noqa: E731


def p_ij(x):
    return x - x.swapaxes(0, 1)


def p_ab(x):
    return x - x.swapaxes(2, 3)


class SlabSource:
    """Three- and four-virtual antisymmetrised integrals, one slab at a time."""

    def __init__(self, ham: Hamiltonian):
        self.ham = ham
        self.vu = np.arange(ham.nc, ham.n)             # spatial t, u, virt
        self.vmap = ham.vir_sp - ham.nc                # spin-orbital vir -> position in vu
        self.Bvv = ham.B[:, self.vu][:, :, self.vu]    # (naux, Vu, Vu)

    def ovvv(self, m: int) -> np.ndarray:
        """G[a,e,f] = <m a||e f> for occupied spin-orbital m."""
        ham = self.ham
        ms, mm = ham.occ_sp[m], ham.occ_spin[m]
        S = es("Pe,Paf->eaf", ham.B[:, ms, self.vu], self.Bvv)   # (m e|a f)
        vm, vs = self.vmap, ham.vir_spin
        Se = S[vm][:, vm][:, :, vm]                               # S[e,a,f] on spin-orbital V
        direct = Se.transpose(1, 0, 2) * ((vs[None, :, None] == mm) & (vs[:, None, None] == vs[None, None, :]))
        # <ma|fe> = (mf|ae): S[f, a, e]
        exch = Se.transpose(1, 2, 0) * ((vs[None, None, :] == mm) & (vs[:, None, None] == vs[None, :, None]))
        return direct - exch

    def ladder(self, tau: np.ndarray) -> np.ndarray:
        """sum_ef tau_ij^ef <ab|ef>  ( = 1/2 sum_ef tau_ij^ef <ab||ef> )."""
        ham = self.ham
        no, nv = tau.shape[0], tau.shape[2]
        out = np.zeros((no, no, nv, nv), np.result_type(tau, ham.B))
        vs = ham.vir_spin
        spins = [np.where(vs == s)[0] for s in (0, 1)]
        for a_sp in np.unique(ham.vir_sp):
            pos_u = a_sp - ham.nc
            S = es("Pe,Pbf->ebf", self.Bvv[:, pos_u, :], self.Bvv)   # (a e|b f) on vu
            for a in np.where(ham.vir_sp == a_sp)[0]:
                E = spins[vs[a]]
                for Fb in spins:
                    blk = S[self.vmap[E]][:, self.vmap[Fb]][:, :, self.vmap[Fb]]  # [e, b, f]
                    out[:, :, a, Fb] += es("ijef,ebf->ijb", tau[:, :, E][:, :, :, Fb], blk)
        return out


def ladder_element(B: np.ndarray, nc: int, t2_block: np.ndarray, block: int, i: int, j: int, a: int, b: int) -> float:
    """One element of the particle-particle ladder sum_ef t_ij^ef <ab|ef> of the
    doubles residual (Theory section, doubles equations; tau = t2 when the
    singles vanish), written out for a single (i, j, a, b) of a packed doubles
    block (0 alpha-alpha, 1 beta-beta, 2 alpha-beta, indices in the per-spin
    orders alpha-vir = [u, virt], beta-vir = [t, virt]).  With e of a's spin and
    f of b's spin, <ab|ef> = (ae|bf) and (pq|rs) = sum_P B[P,p,q] B[P,r,s].
    For checking sampled elements at sizes where the full residual is too costly.

    Pinned by: every element against the slab-batched ladder of the full
    residual on small systems (tests/test_oracle_ladder_element.py).
    """
    n = B.shape[1]
    virt = np.arange(nc + 2, n)
    vir = (np.concatenate([[nc + 1], virt]), np.concatenate([[nc], virt]))  # alpha, beta
    sa, sb = ((0, 0), (1, 1), (0, 1))[block]
    E, Fv = vir[sa], vir[sb]
    I = B[:, E[a], E].T @ B[:, Fv[b], Fv]  # [e, f] = (a e | b f)
    return float(np.sum(I * t2_block[i, j]))


def integrals(ham: Hamiltonian) -> dict:
    O, V = ham.O, ham.V
    return {
        "foo": ham.fock(O, O), "fov": ham.fock(O, V), "fvv": ham.fock(V, V),
        "oooo": ham.asym(O, O, O, O), "ooov": ham.asym(O, O, O, V),
        "oovv": ham.asym(O, O, V, V), "ovvo": ham.asym(O, V, V, O),
        "ovov": ham.asym(O, V, O, V), "oovo": ham.asym(O, O, V, O),
        "ovoo": ham.asym(O, V, O, O),
    }


def ccsd_residual(ham: Hamiltonian, t1: np.ndarray, t2: np.ndarray, ints: dict | None = None,
                  slabs: SlabSource | None = None):
    """(R1, R2) = <x| e^-T H e^T |A> for singles and doubles (spin-orbital)."""
    I = ints if ints is not None else integrals(ham)
    src = slabs if slabs is not None else SlabSource(ham)
    foo, fov, fvv = I["foo"], I["fov"], I["fvv"]
    no, nv = t1.shape
    t1t1 = es("ia,jb->ijab", t1, t1)
    tau_t = t2 + 0.5 * (t1t1 - t1t1.swapaxes(2, 3))
    tau = t2 + t1t1 - t1t1.swapaxes(2, 3)

    # terms with one occupied and three virtual indices, one occupied slab at a time
    dt = np.result_type(t2, src.ham.B)
    Fae_3v = np.zeros((nv, nv), dt)
    Wmbej_3v = np.zeros((no, nv, nv, no), dt)
    R1_3v = np.zeros((no, nv), dt)
    X_3v = np.zeros((no, no, nv, nv), dt)
    Y_3v = np.zeros((no, no, nv, nv), dt)
    for m in range(no):
        G = src.ovvv(m)                                   # <ma||ef>
        Fae_3v += es("f,afe->ae", t1[m], G)
        Wmbej_3v[m] = es("jf,bef->bej", t1, G)
        R1_3v += es("ief,aef->ia", t2[:, m], G)
        X_3v += es("ija,b->ijab", es("ijef,aef->ija", tau, G), t1[m])
        Y_3v[:, m] = -es("ie,eab->iab", t1, G)             # sum_e t_i^e <ab||e m>

    Fae = fvv - 0.5 * es("me,ma->ae", fov, t1) + Fae_3v - 0.5 * es("mnaf,mnef->ae", tau_t, I["oovv"])
    Fmi = foo + 0.5 * es("ie,me->mi", t1, fov) + es("ne,mnie->mi", t1, I["ooov"]) \
        + 0.5 * es("inef,mnef->mi", tau_t, I["oovv"])
    Fme = fov + es("nf,mnef->me", t1, I["oovv"])
    W = es("je,mnie->mnij", t1, I["ooov"])
    Wmnij = I["oooo"] + (W - W.swapaxes(2, 3)) + 0.25 * es("ijef,mnef->mnij", tau, I["oovv"])
    Wmbej = I["ovvo"] + Wmbej_3v - es("nb,mnej->mbej", t1, I["oovo"]) \
        - es("jnfb,mnef->mbej", 0.5 * t2 + es("jf,nb->jnfb", t1, t1), I["oovv"])

    R1 = (fov + es("ie,ae->ia", t1, Fae) - es("ma,mi->ia", t1, Fmi) + es("imae,me->ia", t2, Fme)
          - es("nf,naif->ia", t1, I["ovov"]) - 0.5 * R1_3v - 0.5 * es("mnae,nmei->ia", t2, I["oovo"]))

    R2 = I["oovv"].astype(np.result_type(I["oovv"], t2))
    R2 += p_ab(es("ijae,be->ijab", t2, Fae - 0.5 * es("mb,me->be", t1, Fme)))
    R2 -= p_ij(es("imab,mj->ijab", t2, Fmi + 0.5 * es("je,me->mj", t1, Fme)))
    R2 += 0.5 * es("mnab,mnij->ijab", tau, Wmnij)
    R2 += src.ladder(tau)
    R2 += 0.5 * p_ab(X_3v)
    R2 += 0.125 * es("ijmn,mnab->ijab", es("ijef,mnef->ijmn", tau, I["oovv"]), tau)
    R2 += p_ij(p_ab(es("imae,mbej->ijab", t2, Wmbej) - es("ie,ma,mbej->ijab", t1, t1, I["ovvo"])))
    R2 += p_ij(Y_3v)
    R2 -= p_ab(es("ma,mbij->ijab", t1, I["ovoo"]))
    return R1, R2


def ccsd_energy(ints: dict, t1: np.ndarray, t2: np.ndarray) -> float:
    """Delta E_A = sum f_ia t_i^a + 1/4 sum <ij||ab> t_ij^ab + 1/2 sum <ij||ab> t_i^a t_j^b."""
    fov, oovv = ints["fov"], ints["oovv"]
    return (es("ia,ia->", fov, t1) + 0.25 * es("ijab,ijab->", oovv, t2)
            + 0.5 * es("ijab,ia,jb->", oovv, t1, t1))[()]
