"""Spin-orbital Hamiltonian of the open-shell reference Phi_A (oracle).

Theory section (the two determinants of Fig. 1): Phi_A has the core orbitals
doubly occupied, t with an alpha and u with a beta electron; Phi_B is its
spin flip (u alpha, t beta).  Spatial orbital order is
``[core | t | u | virt]``.

Inputs are DF factors B[P,p,q] (the two-electron integrals are *defined* as
(pq|rs) = sum_P B[P,p,q] B[P,r,s]) and one spatial Fock matrix F.  The paper
works from a spin-free molecular Hamiltonian; a single spatial F is read as
the spin-averaged (ROHF-like) Fock operator of the open shell, so that the
one-electron Hamiltonian is

    h = F - G_avg[B],
    G_avg_pq = sum_{k in core} [2 (pq|kk) - (pk|kq)] + sum_{x in t,u} [(pq|xx) - 1/2 (px|xq)].

This keeps H spin free, which is what makes Phi_B's amplitudes the spin flip
of Phi_A's.  Spin-orbital integrals: <pq|rs> = (pr|qs) delta(sp,sr) delta(sq,ss),
<pq||rs> = <pq|rs> - <pq|sr>.  Fock of Phi_A: f_pq = h_pq + sum_k <pk||qk>.

Pins (tests/test_oracle_*.py): E_ref equals <A|H|A> of the determinant
engine; f^alpha, f^beta equal the closed form F -/+ 1/2 (K_t - K_u); the
determinant engine's FCI states of this H are pure spin states.
"""
from __future__ import annotations

import numpy as np


class Hamiltonian:
    """Spin-orbital view of (B, F) relative to Phi_A.

    Spin-orbital occupied list: [alpha core..., t alpha, beta core..., u beta]
    (2o entries); virtual list: [u alpha, alpha virt..., t beta, beta virt...]
    (2v entries).  This matches the per-spin order of the packed amplitude
    layout.
    """

    def __init__(self, B: np.ndarray, F: np.ndarray, nc: int):
        # FP64 (complex FP64 only for complex-step derivatives in the tests)
        self.B = np.asarray(B, dtype=np.result_type(B, np.float64))
        self.F = np.asarray(F, dtype=np.result_type(F, np.float64))
        self.naux, self.n, _ = self.B.shape
        self.nc = nc
        self.nv = self.n - nc - 2
        self.t, self.u = nc, nc + 1
        n, t, u = self.n, self.t, self.u
        core = np.arange(nc)
        virt = np.arange(nc + 2, n)
        self.o = nc + 1
        self.v = self.nv + 1
        self.occ_sp = np.concatenate([core, [t], core, [u]]).astype(int)
        self.occ_spin = np.concatenate([np.zeros(self.o), np.ones(self.o)]).astype(int)
        self.vir_sp = np.concatenate([[u], virt, [t], virt]).astype(int)
        self.vir_spin = np.concatenate([np.zeros(self.v), np.ones(self.v)]).astype(int)
        self.h = self.F - self._g_avg()

    # ---- spatial integrals -------------------------------------------------
    def spatial(self, p, q, r, s) -> np.ndarray:
        """(pq|rs) for index arrays p, q, r, s -> array [p, q, r, s]."""
        B = self.B
        L = B[:, p][:, :, q]
        R = B[:, r][:, :, s]
        return np.einsum("Ppq,Prs->pqrs", L, R, optimize=True)

    def _g_avg(self) -> np.ndarray:
        B, nc, t, u = self.B, self.nc, self.t, self.u
        G = np.zeros((self.n, self.n), B.dtype)
        for k in range(nc):
            J = np.einsum("P,Ppq->pq", B[:, k, k], B)
            K = np.einsum("Ppk,Pkq->pq", B[:, :, k:k + 1], B[:, k:k + 1, :])
            G += 2.0 * J - K
        for x in (t, u):
            J = np.einsum("P,Ppq->pq", B[:, x, x], B)
            K = np.einsum("Ppk,Pkq->pq", B[:, :, x:x + 1], B[:, x:x + 1, :])
            G += J - 0.5 * K
        return G

    def exchange(self, x: int) -> np.ndarray:
        """(K_x)_pq = (px|xq)."""
        return np.einsum("Pp,Pq->pq", self.B[:, :, x], self.B[:, x, :])

    # ---- spin-orbital integrals ---------------------------------------------
    def asym(self, P, Q, R, S) -> np.ndarray:
        """<pq||rs> for four spin-orbital lists, each a (spatial, spin) pair of
        index arrays.  Returns an array [len P, len Q, len R, len S]."""
        (ps, pm), (qs, qm), (rs, rm), (ss, sm) = P, Q, R, S
        B = self.B
        # <pq|rs> = (pr|qs) [sp = sr][sq = ss]
        A1 = B[:, ps][:, :, rs] * (pm[:, None] == rm[None, :])
        A2 = B[:, qs][:, :, ss] * (qm[:, None] == sm[None, :])
        direct = np.einsum("Ppr,Pqs->pqrs", A1, A2, optimize=True)
        # <pq|sr> = (ps|qr) [sp = ss][sq = sr]
        E1 = B[:, ps][:, :, ss] * (pm[:, None] == sm[None, :])
        E2 = B[:, qs][:, :, rs] * (qm[:, None] == rm[None, :])
        exch = np.einsum("Pps,Pqr->pqrs", E1, E2, optimize=True)
        return direct - exch

    def direct(self, P, Q, R, S) -> np.ndarray:
        """<pq|rs> (not antisymmetrised)."""
        (ps, pm), (qs, qm), (rs, rm), (ss, sm) = P, Q, R, S
        B = self.B
        A1 = B[:, ps][:, :, rs] * (pm[:, None] == rm[None, :])
        A2 = B[:, qs][:, :, ss] * (qm[:, None] == sm[None, :])
        return np.einsum("Ppr,Pqs->pqrs", A1, A2, optimize=True)

    @property
    def O(self):
        return (self.occ_sp, self.occ_spin)

    @property
    def V(self):
        return (self.vir_sp, self.vir_spin)

    def sub(self, lst, idx):
        sp, sm = lst
        idx = np.atleast_1d(idx)
        return (sp[idx], sm[idx])

    # ---- Fock matrix and reference energy -----------------------------------
    def h_so(self, P, Q) -> np.ndarray:
        (ps, pm), (qs, qm) = P, Q
        return self.h[np.ix_(ps, qs)] * (pm[:, None] == qm[None, :])

    def fock(self, P, Q) -> np.ndarray:
        """f_pq = h_pq + sum_{k in occ(A)} <pk||qk>."""
        O = self.O
        f = self.h_so(P, Q)
        (ps, pm), (qs, qm) = P, Q
        ks, km = O
        B = self.B
        # sum_k <pk|qk> = sum_k (pq|kk) [sp=sq]
        jk = B[:, ks, ks].sum(axis=1)
        J = np.einsum("P,Ppq->pq", jk, B[:, ps][:, :, qs]) * (pm[:, None] == qm[None, :])
        # sum_k <pk|kq> = sum_k (pk|kq) [sp=sk][sk=sq]
        Bpk = B[:, ps][:, :, ks] * (pm[:, None] == km[None, :])
        Bkq = B[:, ks][:, :, qs] * (km[:, None] == qm[None, :])
        K = np.einsum("Ppk,Pkq->pq", Bpk, Bkq)
        return f + J - K

    def e_ref(self) -> float:
        O = self.O
        hk = self.h_so(O, O)
        oooo = self.asym(O, O, O, O)
        no = len(O[0])
        idx = np.arange(no)
        return (np.trace(hk) + 0.5 * oooo[idx[:, None], idx[None, :], idx[:, None], idx[None, :]].sum())[()]

    def spin_fock_closed_form(self):
        """f^alpha, f^beta = F -/+ 1/2 (K_t - K_u) (spatial, full n x n)."""
        d = 0.5 * (self.exchange(self.t) - self.exchange(self.u))
        return self.F - d, self.F + d

    # ---- packing between the packed vector and spin-orbital tensors ---------
    def to_so(self, vec: np.ndarray):
        o, v = self.o, self.v
        off = 0
        t1a = vec[off:off + o * v].reshape(o, v); off += o * v
        t1b = vec[off:off + o * v].reshape(o, v); off += o * v
        s = o * o * v * v
        t2aa = vec[off:off + s].reshape(o, o, v, v); off += s
        t2bb = vec[off:off + s].reshape(o, o, v, v); off += s
        t2ab = vec[off:off + s].reshape(o, o, v, v)
        dt = np.result_type(vec, self.B)
        t1 = np.zeros((2 * o, 2 * v), dt)
        t1[:o, :v] = t1a
        t1[o:, v:] = t1b
        t2 = np.zeros((2 * o, 2 * o, 2 * v, 2 * v), dt)
        t2[:o, :o, :v, :v] = t2aa
        t2[o:, o:, v:, v:] = t2bb
        t2[:o, o:, :v, v:] = t2ab
        t2[o:, :o, :v, v:] = -t2ab.transpose(1, 0, 2, 3)
        t2[:o, o:, v:, :v] = -t2ab.transpose(0, 1, 3, 2)
        t2[o:, :o, v:, :v] = t2ab.transpose(1, 0, 3, 2)
        return t1, t2

    def from_so(self, r1: np.ndarray, r2: np.ndarray) -> np.ndarray:
        o, v = self.o, self.v
        parts = [r1[:o, :v], r1[o:, v:], r2[:o, :o, :v, :v], r2[o:, o:, v:, v:], r2[:o, o:, :v, v:]]
        return np.concatenate([np.ascontiguousarray(p).ravel() for p in parts])

    def ab_index(self):
        """Spin-orbital indices (i, j, a, b) of the Phi_A -> Phi_B double:
        t alpha, u beta -> u alpha, t beta."""
        o, v = self.o, self.v
        return (self.nc, o + self.nc, 0, v + 0)

    def ab_packed_position(self) -> int:
        o, v = self.o, self.v
        base = 2 * o * v + 2 * o * o * v * v
        return base + ((self.nc * o + self.nc) * v + 0) * v + 0
