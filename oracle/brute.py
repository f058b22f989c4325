"""Determinant-space engine: exact second quantisation on small systems (oracle).

Everything is evaluated from its definition in the full determinant space of
the reference's N_alpha and N_beta (nc + 1 each for Phi_A; nc + 2 and nc for
the M_s = 1 determinant Phi_T):

* H = sum h_pq E_pq + 1/2 sum (pq|rs) (E_pq E_rs - delta_qr E_ps), the
  spin-free Hamiltonian of the DF integrals (spin-summed E_pq);
* T_A (excitations of Phi_A) and T_B (the same amplitudes with every spin
  label flipped, acting on Phi_B) as operators; e^{+-T} by the finite Taylor
  series (T is nilpotent);
* the connected residual <A^x| e^-T_A H e^T_A |A>, the coupling
  <A^x| e^-T_A e^T_B |B>, W = <B| e^-T_A H e^T_A |A>, E_ref = <A|H|A>;
* full configuration interaction, S^2 and the singlet/triplet roots of the
  M_s = 0 open-shell pair.

Spin-orbital k = sigma*n + p; a determinant is a bitmask and
|D> = prod_{k ascending} a+_k |vac>.  Used only for systems with at most a
few thousand determinants.
"""
from __future__ import annotations

import itertools

import numpy as np

from .hamiltonian import Hamiltonian


def _apply_ops(mask: int, ops):
    """Apply ('c'|'a', k) operators rightmost first; (mask, sign) or None."""
    sign = 1
    for kind, k in reversed(ops):
        bit = 1 << k
        if bin(mask & (bit - 1)).count("1") % 2:
            sign = -sign
        if kind == "a":
            if not mask & bit:
                return None
            mask ^= bit
        else:
            if mask & bit:
                return None
            mask |= bit
    return mask, sign


class DeterminantSpace:
    def __init__(self, ham: Hamiltonian):
        self.ham = ham
        n = ham.n
        self.n = n
        self.nso = 2 * n
        # electrons of each spin in the reference (Phi_A: nc + 1 each; Phi_T: nc + 2 and nc)
        na = int(np.sum(np.asarray(ham.occ_spin) == 0))
        nb = int(np.sum(np.asarray(ham.occ_spin) == 1))
        dets = []
        for occa in itertools.combinations(range(n), na):
            for occb in itertools.combinations(range(n), nb):
                dets.append(sum(1 << p for p in occa) | sum(1 << (n + p) for p in occb))
        self.dets = np.array(dets, dtype=np.int64)
        self.index = {int(d): k for k, d in enumerate(dets)}
        self.ndet = len(dets)
        # single-excitation tables a+_p a_q for every spin-orbital pair
        self.eri = ham.spatial(np.arange(n), np.arange(n), np.arange(n), np.arange(n))
        self.tab = {}
        for p in range(self.nso):
            for q in range(self.nso):
                src, dst, sgn = [], [], []
                for k, d in enumerate(dets):
                    r = _apply_ops(d, [("c", p), ("a", q)])
                    if r is None:
                        continue
                    j = self.index.get(r[0])
                    if j is None:
                        continue
                    src.append(k)
                    dst.append(j)
                    sgn.append(r[1])
                self.tab[(p, q)] = (np.array(src, dtype=np.int64), np.array(dst, dtype=np.int64),
                                    np.array(sgn, dtype=np.float64))

    # ---- basic operators ----------------------------------------------------
    def ex(self, p: int, q: int, vec: np.ndarray) -> np.ndarray:
        """a+_p a_q vec."""
        src, dst, sgn = self.tab[(p, q)]
        out = np.zeros_like(vec)
        if src.size:
            out[dst] = (sgn.reshape((-1,) + (1,) * (vec.ndim - 1))) * vec[src]
        return out

    def E(self, p: int, q: int, vec: np.ndarray) -> np.ndarray:
        n = self.n
        return self.ex(p, q, vec) + self.ex(n + p, n + q, vec)

    def basis(self, ops, ref_mask: int):
        r = _apply_ops(ref_mask, ops)
        if r is None or int(r[0]) not in self.index:
            return None
        return self.index[int(r[0])], r[1]

    def vector(self, mask: int, sign: float = 1.0) -> np.ndarray:
        v = np.zeros(self.ndet)
        v[self.index[mask]] = sign
        return v

    # ---- Hamiltonian --------------------------------------------------------
    def apply_H(self, vec: np.ndarray) -> np.ndarray:
        ham, n = self.ham, self.n
        eri = self.eri
        X = np.stack([self.E(r, s, vec) for r in range(n) for s in range(n)])   # (n^2, ...)
        Z = np.tensordot(eri.reshape(n * n, n * n), X, axes=(1, 0))
        kps = np.einsum("pqqs->ps", eri)
        out = np.zeros_like(vec)
        for p in range(n):
            for q in range(n):
                c = ham.h[p, q] * vec + 0.5 * Z[p * n + q] - 0.5 * kps[p, q] * vec
                out += self.E(p, q, c)
        return out

    def H_matrix(self) -> np.ndarray:
        return self.apply_H(np.eye(self.ndet))

    def S2(self, vec: np.ndarray) -> np.ndarray:
        """S^2 vec for M_s = 0 states: S- S+ vec."""
        n = self.n
        sp = sum(self.ex(p, n + p, vec) for p in range(n))
        return sum(self.ex(n + p, p, sp) for p in range(n))

    # ---- references and cluster operators ------------------------------------
    def so(self, spatial: int, spin: int) -> int:
        return spin * self.n + spatial

    def mask_A(self) -> int:
        ham = self.ham
        return sum(1 << self.so(s, m) for s, m in zip(ham.occ_sp, ham.occ_spin))

    def ops_B(self):
        """Operator string taking |A> to |B> = a+_{u a} a+_{t b} a_{u b} a_{t a} |A>."""
        t, u = self.ham.t, self.ham.u
        return [("c", self.so(u, 0)), ("c", self.so(t, 1)), ("a", self.so(u, 1)), ("a", self.so(t, 0))]

    def cluster_terms(self, t1: np.ndarray, t2: np.ndarray, flip: bool):
        """Excitation operator from spin-orbital amplitudes of Phi_A; with
        flip=True every spin label is exchanged (T_B)."""
        ham = self.ham
        def so_of(sp, sm):
            return self.so(sp, 1 - sm if flip else sm)
        occ = [so_of(s, m) for s, m in zip(ham.occ_sp, ham.occ_spin)]
        vir = [so_of(s, m) for s, m in zip(ham.vir_sp, ham.vir_spin)]
        no, nv = len(occ), len(vir)
        singles = [(t1[i, a], vir[a], occ[i]) for i in range(no) for a in range(nv) if t1[i, a] != 0.0]
        doubles = []
        for i, j in itertools.combinations(range(no), 2):
            for a, b in itertools.combinations(range(nv), 2):
                if t2[i, j, a, b] != 0.0:
                    doubles.append((t2[i, j, a, b], vir[a], occ[i], vir[b], occ[j]))
        return singles, doubles

    def apply_T(self, terms, vec: np.ndarray) -> np.ndarray:
        singles, doubles = terms
        out = np.zeros_like(vec)
        for amp, p, q in singles:
            out += amp * self.ex(p, q, vec)
        for amp, a, i, b, j in doubles:
            # a+_a a+_b a_j a_i = (a+_a a_i)(a+_b a_j) since i != b
            out += amp * self.ex(a, i, self.ex(b, j, vec))
        return out

    def exp_T(self, terms, vec: np.ndarray, factor: float = 1.0) -> np.ndarray:
        out = vec.copy()
        cur = vec
        for k in range(1, 4 * (self.ham.nc + 1) + 2):
            cur = factor * self.apply_T(terms, cur) / k
            if not np.any(cur):
                break
            out += cur
        return out

    # ---- projections ----------------------------------------------------------
    def projections(self, vec: np.ndarray) -> tuple:
        """Read <A^x|vec> for every single and double of Phi_A, returned as
        spin-orbital arrays (r1[i,a], r2[i,j,a,b])."""
        ham = self.ham
        A = self.mask_A()
        occ = [self.so(s, m) for s, m in zip(ham.occ_sp, ham.occ_spin)]
        vir = [self.so(s, m) for s, m in zip(ham.vir_sp, ham.vir_spin)]
        no, nv = len(occ), len(vir)
        r1 = np.zeros((no, nv))
        r2 = np.zeros((no, no, nv, nv))
        for i in range(no):
            for a in range(nv):
                b = self.basis([("c", vir[a]), ("a", occ[i])], A)
                if b is not None:
                    r1[i, a] = b[1] * vec[b[0]]
        for i in range(no):
            for j in range(no):
                for a in range(nv):
                    for b_ in range(nv):
                        b = self.basis([("c", vir[a]), ("c", vir[b_]), ("a", occ[j]), ("a", occ[i])], A)
                        if b is not None:
                            r2[i, j, a, b_] = b[1] * vec[b[0]]
        return r1, r2

    def connected(self, t1, t2):
        """e^-T_A H e^T_A |A> as a vector."""
        TA = self.cluster_terms(t1, t2, flip=False)
        v = self.exp_T(TA, self.vector(self.mask_A()))
        return self.exp_T(TA, self.apply_H(v), -1.0)

    def coupling_vector(self, t1, t2):
        """e^-T_A e^T_B |B> as a vector."""
        TA = self.cluster_terms(t1, t2, flip=False)
        TB = self.cluster_terms(t1, t2, flip=True)
        bidx, bsign = self.basis(self.ops_B(), self.mask_A())
        v = np.zeros(self.ndet)
        v[bidx] = bsign
        return self.exp_T(TA, self.exp_T(TB, v), -1.0)

    def read_B(self, vec) -> float:
        bidx, bsign = self.basis(self.ops_B(), self.mask_A())
        return float(bsign * vec[bidx])

    def read_A(self, vec) -> float:
        return float(vec[self.index[self.mask_A()]])

    def fci_pair(self):
        """FCI roots with largest weight on the singlet (A+B)/sqrt2 and the
        M_s = 0 triplet (A-B)/sqrt2 combinations; returns (E_S, E_T, evals)."""
        H = self.H_matrix()
        w, U = np.linalg.eigh(H)
        a = self.vector(self.mask_A())
        bidx, bsign = self.basis(self.ops_B(), self.mask_A())
        b = np.zeros(self.ndet)
        b[bidx] = bsign
        s = (a + b) / np.sqrt(2.0)
        tr = (a - b) / np.sqrt(2.0)
        kS = int(np.argmax(np.abs(U.T @ s)))
        kT = int(np.argmax(np.abs(U.T @ tr)))
        return float(w[kS]), float(w[kT]), w, U
