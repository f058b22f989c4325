"""Fixed-reference DCSD / CCSD (oracle; test infrastructure only).

Introduction (the fixed-reference approach): a normal single-reference
coupled-cluster calculation from Phi_A in which the doubles amplitude of the
Phi_A -> Phi_B excitation is held at one while all other amplitudes relax.

* With Phi_B = a+_{u alpha} a+_{t beta} |core> = +Phi_{t alpha, u beta}^{u alpha, t beta}
  (the phase used throughout this oracle), the open-shell singlet
  Phi_A + Phi_B has that amplitude at +1.  The M_s = 0 triplet Phi_A - Phi_B
  has it at -1, which is this oracle's reading for the triplet (the paper
  states the singlet case only).
* There are no coupling terms.  The residual is the connected CC residual
  minus the DC-dropped terms (DCSD), evaluated with the fixed amplitude
  present; its A->B element is not an unknown and is set to zero.
* The state's correlation energy is the single-reference CC energy expression
  of Phi_A with the fixed amplitude included.  One calculation gives one state.

Pinned by: the brute-force similarity-transformed projection with the fixed
amplitude present (tests/test_oracle_brute.py), and two-electron
complete-active-space FCI (tests/test_oracle_fixedref.py).  There the exact
singlet has equal weights on Phi_A and Phi_B and the triplet opposite ones,
and the internal singles vanish by symmetry, so FR-CCSD and FR-DCSD reproduce
both roots.
"""
from __future__ import annotations

import numpy as np

from .twodet import TwoDet

STATES = ("singlet", "triplet")


class FixedRef(TwoDet):
    def __init__(self, B, F, nc: int, method: str = "dcsd", state: str = "singlet"):
        super().__init__(B, F, nc, method)
        if state not in STATES:
            raise ValueError(state)
        self.state = state
        self.sign = 1.0 if state == "singlet" else -1.0

    def fixed(self, vec: np.ndarray) -> np.ndarray:
        """Amplitudes with the A->B double set to +1 (singlet) or -1 (triplet)."""
        out = np.array(vec, dtype=np.result_type(vec, np.float64))
        out[self.ab] = self.sign
        return out

    def residual(self, vec: np.ndarray):
        """(R, 0): the packed residual (A->B element zero) and W = 0."""
        R = self.connected(self.fixed(vec))
        R[self.ab] = 0.0
        return R, 0.0

    def energy_A(self, vec: np.ndarray) -> float:
        return super().energy_A(self.fixed(vec))

    def energies(self, vec: np.ndarray, W: float | None = None) -> dict:
        dEA = self.energy_A(vec)
        nan = float("nan")
        singlet = self.state == "singlet"
        return {"dE_A": dEA, "W": 0.0, "E_S": dEA if singlet else nan, "E_T": nan if singlet else dEA,
                "E_ref_A": self.ham.e_ref()}
