"""2D-DCSD / 2D-CCSD residual and energies (oracle).

Theory section (energy, singles and doubles equations, effective Hamiltonian
W, and the statements that follow them):

* R_x = <x| e^-T_A H e^T_A |A>  - dropped_x  - K_x W       (x != A->B double)
  where the first term is the CCSD residual (ccsd.py), dropped_x the terms
  the distinguishable-cluster approximation removes from the doubles
  (dc.py; zero for 2D-CCSD) and K_x the coupling coefficient (coupling.py),
  so that M_x W = -K_x W.
* The amplitude of the Phi_A -> Phi_B double is fixed at zero; the value of
  the corresponding element of the (DC or CC) doubles residual is W, and the
  element itself is then set to zero.
* Delta E_A is the single-reference CC energy expression; the 2x2 effective
  Hamiltonian [[dE_A, W], [W, dE_A]] gives the open-shell singlet
  E_S = dE_A + W and the M_s = 0 triplet E_T = dE_A - W (correlation
  energies relative to E_ref = <A|H|A>; Phi_A + Phi_B is the singlet with
  Phi_B = a+_{u alpha} a+_{t beta} |core>).

Pinned by: two-electron FCI singlet and triplet roots (complete active
space inputs), brute-force K_x and W, the t <-> u exchange invariance.
"""
from __future__ import annotations

import numpy as np

import dcsd_synth as synth

from .ccsd import SlabSource, ccsd_energy, ccsd_residual, integrals
from .coupling import coupling
from .dc import dropped_terms
from .hamiltonian import Hamiltonian

METHODS = ("dcsd", "ccsd")


class TwoDet:
    def __init__(self, B, F, nc: int, method: str = "dcsd"):
        if method not in METHODS:
            raise ValueError(method)
        self.method = method
        self.ham = Hamiltonian(B, F, nc)
        self.ints = integrals(self.ham)
        self.slabs = SlabSource(self.ham)
        self.nc, self.nv = nc, self.ham.nv
        self.ab = self.ham.ab_packed_position()

    @property
    def size(self) -> int:
        return synth.amplitude_count(self.nc, self.nv)

    def connected(self, vec: np.ndarray) -> np.ndarray:
        """Single-reference residual minus the DC-dropped terms, packed."""
        t1, t2 = self.ham.to_so(vec)
        R1, R2 = ccsd_residual(self.ham, t1, t2, self.ints, self.slabs)
        if self.method == "dcsd":
            R2 = R2 - dropped_terms(self.ham, t2, self.ints["oovv"])
        return self.ham.from_so(R1, R2)

    def coupling(self, vec: np.ndarray) -> np.ndarray:
        K = coupling(synth.unpack(vec, self.nc, self.nv), self.nc, self.nv)
        return synth.pack(K, self.nc, self.nv)

    def residual(self, vec: np.ndarray):
        """(R, W): the packed 2D residual and the effective coupling W."""
        vec = np.array(vec, dtype=np.result_type(vec, np.float64))
        vec[self.ab] = 0.0
        Rc = self.connected(vec)
        W = Rc[self.ab]
        R = Rc - self.coupling(vec) * W
        R[self.ab] = 0.0
        return R, W

    def energy_A(self, vec: np.ndarray) -> float:
        t1, t2 = self.ham.to_so(vec)
        return ccsd_energy(self.ints, t1, t2)

    def energies(self, vec: np.ndarray, W: float | None = None) -> dict:
        if W is None:
            W = self.residual(vec)[1]
        dEA = self.energy_A(vec)
        return {"dE_A": dEA, "W": W, "E_S": dEA + W, "E_T": dEA - W, "E_ref_A": self.ham.e_ref()}

    def en_shift(self) -> np.ndarray:
        """Two-electron part of the diagonal of the residual's Jacobian at T=0
        (Epstein-Nesbet), packed: with P(p,q) = <pq||pq>,
        singles s_ia = -P(i,a); doubles s_ijab = P(a,b) + P(i,j) - P(i,a)
        - P(i,b) - P(j,a) - P(j,b).  Used only to precondition the Jacobi step."""
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

    def denominators(self) -> np.ndarray:
        """D_x = sum f_ii - sum f_aa from the spin-orbital Fock diagonal (packed)."""
        o, v = self.ham.o, self.ham.v
        fo = np.diag(self.ints["foo"])
        fv = np.diag(self.ints["fvv"])
        d1 = fo[:, None] - fv[None, :]
        d2 = fo[:, None, None, None] + fo[None, :, None, None] - fv[None, None, :, None] - fv[None, None, None, :]
        return self.ham.from_so(d1, d2)
