"""High-spin (M_s = 1) triplet reference: single-reference DCSD / CCSD (oracle).

The paper obtains singlet-triplet gaps from single-reference calculations of
the M_s = 1 component of the triplet, whose reference Phi_T has t and u both
singly occupied with alpha spin (Computational Details; the spin splittings of
the diradicals in the Results), and compares them with the M_s = 0 triplet
E_T = dE_A - W of the two-determinant treatment.  Phi_T is a single
determinant, so its equations are the plain single-reference CCSD equations
<x| e^-T H e^T |T> = 0 for singles and doubles, minus the
distinguishable-cluster dropped terms for DCSD (the same selection as for
Phi_A), with no coupling and no fixed amplitude; the state's correlation
energy is the CC energy expression of Phi_T.

The Hamiltonian is the same spin-free H as for the open-shell singlet
(hamiltonian.py: h = F - G_avg[B]); only the occupation changes:
alpha occupied = [core, t, u], beta occupied = [core];
alpha virtual = [virt], beta virtual = [t, u, virt].

Packed layout (``dcsd_synth.hs_*``), per spin in those orders:
    [ t1a (oa,va) | t1b (ob,vb) | t2aa (oa,oa,va,va) | t2bb (ob,ob,vb,vb) | t2ab (oa,ob,va,vb) ]
with oa = nc + 2, ob = nc, va = nv, vb = nv + 2.

Pinned by: brute-force <x| e^-T H e^T |T> of the determinant engine (in the
M_s = 1 sector) for random T; two-electron inputs, where converged CCSD and
DCSD equal the M_s = 1 FCI triplet, which is also the M_s = 0 triplet root of
the same Hamiltonian; the MP2-with-singles closed form after the first
iteration; size consistency with a non-interacting closed-shell fragment
(tests/test_oracle_highspin.py).
"""
from __future__ import annotations

import numpy as np

import dcsd_synth as synth

from .ccsd import SlabSource, ccsd_energy, ccsd_residual, integrals
from .dc import dropped_terms
from .hamiltonian import Hamiltonian

METHODS = ("dcsd", "ccsd")


class HighSpinHamiltonian(Hamiltonian):
    """Spin-orbital view of (B, F) relative to Phi_T = |core, t alpha, u alpha>."""

    def __init__(self, B: np.ndarray, F: np.ndarray, nc: int):
        super().__init__(B, F, nc)
        n, t, u = self.n, self.t, self.u
        core = np.arange(nc)
        virt = np.arange(nc + 2, n)
        self.oa, self.ob = nc + 2, nc
        self.va, self.vb = self.nv, self.nv + 2
        self.occ_sp = np.concatenate([core, [t, u], core]).astype(int)
        self.occ_spin = np.concatenate([np.zeros(self.oa), np.ones(self.ob)]).astype(int)
        self.vir_sp = np.concatenate([virt, [t, u], virt]).astype(int)
        self.vir_spin = np.concatenate([np.zeros(self.va), np.ones(self.vb)]).astype(int)

    def to_so(self, vec: np.ndarray):
        oa, ob, va, vb = self.oa, self.ob, self.va, self.vb
        blk = synth.hs_unpack(vec, self.nc, self.nv)
        dt = np.result_type(vec, self.B)
        no, nv = oa + ob, va + vb
        t1 = np.zeros((no, nv), dt)
        t1[:oa, :va] = blk["t1a"]
        t1[oa:, va:] = blk["t1b"]
        t2 = np.zeros((no, no, nv, nv), dt)
        t2[:oa, :oa, :va, :va] = blk["t2aa"]
        t2[oa:, oa:, va:, va:] = blk["t2bb"]
        ab = blk["t2ab"]
        t2[:oa, oa:, :va, va:] = ab
        t2[oa:, :oa, :va, va:] = -ab.transpose(1, 0, 2, 3)
        t2[:oa, oa:, va:, :va] = -ab.transpose(0, 1, 3, 2)
        t2[oa:, :oa, va:, :va] = ab.transpose(1, 0, 3, 2)
        return t1, t2

    def from_so(self, r1: np.ndarray, r2: np.ndarray) -> np.ndarray:
        oa, va = self.oa, self.va
        parts = [r1[:oa, :va], r1[oa:, va:], r2[:oa, :oa, :va, :va], r2[oa:, oa:, va:, va:], r2[:oa, oa:, :va, va:]]
        return np.concatenate([np.ascontiguousarray(p).ravel() for p in parts])


class HighSpin:
    """Single-reference DCSD or CCSD of the M_s = 1 triplet determinant Phi_T.

    The interface follows TwoDet (residual returns (R, W) with W = 0, energies
    a dict) so that solver.solve drives it; E_T is the triplet's correlation
    energy dE and E_S is NaN."""

    def __init__(self, B, F, nc: int, method: str = "dcsd"):
        if method not in METHODS:
            raise ValueError(method)
        self.method = method
        self.ham = HighSpinHamiltonian(B, F, nc)
        self.ints = integrals(self.ham)
        self.slabs = SlabSource(self.ham)
        self.nc, self.nv = nc, self.ham.nv

    @property
    def size(self) -> int:
        return synth.hs_amplitude_count(self.nc, self.nv)

    def residual(self, vec: np.ndarray):
        vec = np.asarray(vec, dtype=np.result_type(vec, np.float64))
        t1, t2 = self.ham.to_so(vec)
        R1, R2 = ccsd_residual(self.ham, t1, t2, self.ints, self.slabs)
        if self.method == "dcsd":
            R2 = R2 - dropped_terms(self.ham, t2, self.ints["oovv"])
        return self.ham.from_so(R1, R2), 0.0

    def energy(self, vec: np.ndarray) -> float:
        t1, t2 = self.ham.to_so(vec)
        return ccsd_energy(self.ints, t1, t2)

    def energies(self, vec: np.ndarray, W: float | None = None) -> dict:
        dE = self.energy(vec)
        return {"dE_A": dE, "W": 0.0, "E_S": float("nan"), "E_T": dE, "E_ref_A": self.ham.e_ref()}

    def triples(self, vec: np.ndarray) -> dict:
        """(T) correction at the amplitudes vec (triples.py), with its parts."""
        from .triples import triples_energy
        t1, t2 = self.ham.to_so(vec)
        return triples_energy(self.ham, t1, t2)

    def denominators(self) -> np.ndarray:
        """D_x = sum f_ii - sum f_aa from the spin-orbital Fock diagonal (packed)."""
        fo = np.diag(self.ints["foo"])
        fv = np.diag(self.ints["fvv"])
        d1 = fo[:, None] - fv[None, :]
        d2 = fo[:, None, None, None] + fo[None, :, None, None] - fv[None, None, :, None] - fv[None, None, None, :]
        return self.ham.from_so(d1, d2)

    def en_shift(self) -> np.ndarray:
        """Two-electron part of the Jacobian diagonal at T = 0 (Epstein-Nesbet), as for TwoDet."""
        B = self.ham.B
        J = np.einsum("Ppp,Pqq->pq", B, B)
        K = np.einsum("Ppq,Ppq->pq", B, B)
        O, V = self.ham.O, self.ham.V

        def P(X, Y):
            (xs, xm), (ys, ym) = X, Y
            return J[np.ix_(xs, ys)] - (xm[:, None] == ym[None, :]) * K[np.ix_(xs, ys)]
        Poo, Pvv, Pov = P(O, O), P(V, V), P(O, V)
        s1 = -Pov
        s2 = (Pvv[None, None, :, :] + Poo[:, :, None, None] - Pov[:, None, :, None] - Pov[:, None, None, :]
              - Pov[None, :, :, None] - Pov[None, :, None, :])
        return self.ham.from_so(s1, s2)
