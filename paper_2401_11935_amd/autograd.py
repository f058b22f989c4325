"""torch.autograd bindings of libdcsd's hand-written adjoint.

``Problem(B, F, nc, **config)`` binds a libdcsd context to the device tensors
B (naux, n, n) and F (n, n) (FP64, contiguous, on the GPU; borrowed for the
life of the problem).  Two differentiable maps:

* ``problem.residual(T, B, F) -> (R, W, dE_A)`` (``DCSDResidual``): one
  residual evaluation; backward is ``dcsd_residual_vjp`` (cotangents of T and
  of every stored entry of B and F).  The gradient of T is taken entry by
  entry over the packed vector, which stores every same-spin double in its
  four signed copies: ``T.grad . dT`` is the derivative of the loss only along
  changes dT with that antisymmetry (and with dT = 0 at the A->B double), the
  directions that are amplitude changes.  Project it onto that subspace (the
  mean of the four signed copies) before using it along any other direction;
* ``problem.energies(B, F) -> (E_S, E_T)`` (``DCSDEnergy``): the converged
  correlation energies of the singlet and triplet; backward is
  ``dcsd_backward`` (the lambda equations of the energy Lagrangian, then
  dE/dB and dE/dF as symmetric matrices).  With a fixed-reference method the
  state not computed comes back as NaN (E_T of a singlet run, E_S of a
  triplet run) and its gradient weight is ignored: build the loss from the
  computed state only.

B and F are passed again to each call so that autograd can route gradients
to them; they must be the tensors the problem was built on.  The library
works on the torch stream that was current when the problem was built; every
call checks that it is still the current stream, so torch's own work on the
inputs (zero fills, copies) is ordered before the library's.  The context
reserves the adjoint's memory at construction (``adjoint=1``), so backward
passes allocate no device memory in the library.
"""
from __future__ import annotations

import torch

from . import libdcsd as L


class Problem:
    def __init__(self, B: torch.Tensor, F: torch.Tensor, nc: int, **config):
        if B.dtype != torch.float64 or F.dtype != torch.float64 or not B.is_cuda or not F.is_cuda:
            raise ValueError("B and F must be float64 CUDA tensors")
        if not (B.is_contiguous() and F.is_contiguous()):
            raise ValueError("B and F must be contiguous")
        naux, n, _ = B.shape
        self.B, self.F, self.nc = B, F, nc
        self.stream = torch.cuda.current_stream(B.device).cuda_stream
        config.setdefault("adjoint", 1)
        cfg = L.default_config(nc=nc, nv=n - nc - 2, naux=naux, **config)
        self.ctx = L.Context(cfg, B.data_ptr(), F.data_ptr(), self.stream)
        self.size = self.ctx.size
        self.last_solve = None
        self.last_lambda = None

    def _check(self, B, F):
        if B.data_ptr() != self.B.data_ptr() or F.data_ptr() != self.F.data_ptr():
            raise ValueError("B and F must be the tensors the problem was built on")
        self.check_stream()

    def check_stream(self):
        if torch.cuda.current_stream(self.B.device).cuda_stream != self.stream:
            raise RuntimeError("the current torch stream differs from the one the problem was built on")

    def residual(self, T: torch.Tensor, B: torch.Tensor, F: torch.Tensor):
        self._check(B, F)
        return DCSDResidual.apply(T, B, F, self)

    def energies(self, B: torch.Tensor, F: torch.Tensor):
        self._check(B, F)
        return DCSDEnergy.apply(B, F, self)

    def close(self):
        self.ctx.close()


class DCSDResidual(torch.autograd.Function):
    @staticmethod
    def forward(ctx, T, B, F, problem):
        T = T.detach().contiguous()
        R = torch.empty_like(T)
        W = problem.ctx.residual(T.data_ptr(), R.data_ptr())
        e = problem.ctx.energy(T.data_ptr())["dE_A"]
        ctx.problem = problem
        ctx.save_for_backward(T)
        scal = dict(dtype=torch.float64, device=T.device)
        return R, torch.tensor(W, **scal), torch.tensor(e, **scal)

    @staticmethod
    def backward(ctx, gR, gW, gE):
        (T,) = ctx.saved_tensors
        p = ctx.problem
        gR = torch.zeros_like(T) if gR is None else gR.contiguous()
        wbar = 0.0 if gW is None else float(gW)
        ebar = 0.0 if gE is None else float(gE)
        Tb = torch.empty_like(T) if ctx.needs_input_grad[0] else None
        Bb = torch.empty_like(p.B) if ctx.needs_input_grad[1] else None
        Fb = torch.empty_like(p.F) if ctx.needs_input_grad[2] else None
        ptr = lambda x: 0 if x is None else x.data_ptr()  # noqa: E731
        p.check_stream()
        p.ctx.residual_vjp(T.data_ptr(), gR.data_ptr(), wbar, ebar, ptr(Tb), ptr(Bb), ptr(Fb))
        return Tb, Bb, Fb, None


class DCSDEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, B, F, problem):
        T = torch.zeros(problem.size, dtype=torch.float64, device=B.device)
        rep = problem.ctx.solve(T.data_ptr())
        if rep["status"] != "OK":
            raise RuntimeError(f"amplitude equations not solved: {rep['status']}")
        problem.last_solve = rep
        ctx.problem = problem
        ctx.save_for_backward(T)
        scal = dict(dtype=torch.float64, device=B.device)
        return torch.tensor(rep["E_S"], **scal), torch.tensor(rep["E_T"], **scal)

    @staticmethod
    def backward(ctx, gS, gT):
        (T,) = ctx.saved_tensors
        p = ctx.problem
        p.check_stream()
        Bb, Fb = torch.empty_like(p.B), torch.empty_like(p.F)
        lam = torch.zeros_like(T)
        rep = p.ctx.backward(T.data_ptr(), 0.0 if gS is None else float(gS), 0.0 if gT is None else float(gT),
                             Bb.data_ptr(), Fb.data_ptr(), lam.data_ptr())
        if rep["status"] != "OK":
            raise RuntimeError(f"lambda equations not solved: {rep['status']}")
        p.last_lambda = rep
        return Bb, Fb, None
