"""Design-field front end on the GPU (Sec. 2.1): chi -> chi_phys = P(H chi),
the density filter and threshold projection in front of the objective, as a
torch.autograd.Function over pt_filter_projection / _backward.

    flt = DesignFilter(nx, ny, r_fil=0.03, beta=32.0, eta=0.5)
    rho = flt(chi)                 # differentiable
    theta = OneShotParareal(prob)(rho)
    theta.backward()               # chi.grad = H^T (P'(chi_fil) o dTheta/drho)
"""
from __future__ import annotations

import torch

from . import _pt


class FilterProjection(torch.autograd.Function):
    @staticmethod
    def forward(ctx, chi: torch.Tensor, flt: "DesignFilter") -> torch.Tensor:
        c = chi.detach().contiguous()
        fil = torch.empty_like(c)
        phys = torch.empty_like(c)
        _pt.pt_filter_projection(flt.desc, c, fil, phys)
        ctx.flt = flt
        ctx.save_for_backward(fil)
        return phys

    @staticmethod
    def backward(ctx, grad_phys: torch.Tensor):
        (fil,) = ctx.saved_tensors
        g = grad_phys.detach().contiguous()
        work = torch.empty_like(fil)
        grad_chi = torch.empty_like(fil)
        _pt.pt_filter_projection_backward(ctx.flt.desc, fil, g, work, grad_chi)
        return grad_chi, None


class DesignFilter:
    """Filter radius r_fil (unit-square coordinates), projection sharpness beta
    (<= 0: no projection) and threshold eta; the paper's values are 0.03, 32
    and 0.5 (Sec. 6.1)."""

    def __init__(self, nx: int, ny: int, r_fil: float, beta: float, eta: float = 0.5):
        self.desc = _pt.make_filter(nx, ny, r_fil, beta, eta)
        if _pt.pt_filter_validate(self.desc) != _pt.PT_OK:
            raise _pt.PtError(_pt.PT_EINVAL, "DesignFilter")
        self.n_elem = nx * ny

    def __call__(self, chi: torch.Tensor) -> torch.Tensor:
        if chi.dtype != torch.float64 or chi.numel() != self.n_elem or not chi.is_cuda:
            raise ValueError("chi must be a float64 CUDA tensor of nx*ny elements")
        return FilterProjection.apply(chi, self)
