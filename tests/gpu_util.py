"""Helpers for the GPU tests: torch device buffers and a libdcsd context."""
import numpy as np
import torch

from paper_2401_11935_amd import libdcsd as L


def dev():
    return torch.device("cuda:0")


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev())


def stream() -> int:
    return torch.cuda.current_stream(dev()).cuda_stream


class GpuProblem:
    def __init__(self, B, F, nc, method="dcsd", **kw):
        nv = B.shape[1] - nc - 2
        self.B = to_dev(B)
        self.F = to_dev(F)
        self.cfg = L.default_config(nc=nc, nv=nv, naux=B.shape[0], method=method, **kw)
        self.ctx = L.Context(self.cfg, self.B.data_ptr(), self.F.data_ptr(), stream())
        self.size = self.ctx.size

    def residual(self, T: np.ndarray):
        Td = to_dev(T)
        Rd = torch.empty_like(Td)
        W = self.ctx.residual(Td.data_ptr(), Rd.data_ptr())
        return Rd.cpu().numpy(), W

    def energy(self, T: np.ndarray) -> dict:
        Td = to_dev(T)
        return self.ctx.energy(Td.data_ptr())

    def solve(self, T0=None, callback=None):
        Td = to_dev(np.zeros(self.size) if T0 is None else T0)
        rep = self.ctx.solve(Td.data_ptr(), callback)
        return rep, Td.cpu().numpy()

    def close(self):
        self.ctx.close()
