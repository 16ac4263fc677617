"""One optimisation cycle on the GPU: the three C-ABI calls with torch-owned
device memory (Sec. 4.4, steps 1-4; Alg. 3 lines 9-12 with a warm restart).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import torch

from . import _pt
from ._pt import Problem


@dataclass
class CycleResult:
    Theta: torch.Tensor       # 0-dim device tensor
    grad: torch.Tensor        # [N_e]
    S: torch.Tensor           # [N_t, N_n], or [2 N_tau, N_n] with checkpoints
    uT: torch.Tensor          # [N_tau+1, N_n]  next primal guess
    utheta: torch.Tensor      # [N_tau+1]
    lam: torch.Tensor         # [N_tau+1, N_n]  next adjoint guess


class Cycle:
    """Owns the workspace and outputs of one problem size and runs cycles."""

    def __init__(self, prob: Problem, device="cuda"):
        self.prob = prob
        self.device = torch.device(device)
        if _pt.pt_validate(prob) != _pt.PT_OK:
            raise _pt.PtError(_pt.PT_EINVAL, "Problem")
        nbytes = _pt.pt_workspace_bytes(prob)
        d = self.device
        f64 = torch.float64
        Nn, Nt1 = prob.n_nodes, prob.n_slices + 1
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=d)
        # every fine state, or the checkpoints of PT_CHECKPOINT (T_{Mn}, T_{Mn+1})
        rows = _pt.pt_state_bytes(prob) // (8 * Nn)
        self.S = torch.empty((rows, Nn), dtype=f64, device=d)
        self.uT = torch.empty((Nt1, Nn), dtype=f64, device=d)
        self.utheta = torch.empty(Nt1, dtype=f64, device=d)
        self.lam = torch.empty((Nt1, Nn), dtype=f64, device=d)
        self.Theta = torch.empty((), dtype=f64, device=d)
        self.grad = torch.empty(prob.n_elem, dtype=f64, device=d)

    def forward(self, rho, guess_T=None, guess_theta=None, stream=None):
        _pt.pt_parareal_forward(self.prob, rho, guess_T, guess_theta, self.S, self.uT,
                                self.utheta, self.Theta, self.ws, stream)

    def adjoint(self, rho, guess_lambda=None, stream=None):
        _pt.pt_parareal_adjoint(self.prob, rho, self.S, self.Theta, guess_lambda, self.lam,
                                self.ws, stream)

    def sensitivities(self, rho, stream=None):
        _pt.pt_sensitivities(self.prob, rho, self.ws, self.grad, stream)

    def run(self, rho, guess_T=None, guess_theta=None, guess_lambda=None,
            stream=None) -> CycleResult:
        self.forward(rho, guess_T, guess_theta, stream)
        self.adjoint(rho, guess_lambda, stream)
        self.sensitivities(rho, stream)
        return CycleResult(self.Theta, self.grad, self.S, self.uT, self.utheta, self.lam)

    def status(self, stream=None) -> dict:
        return _pt.pt_query_status(self.ws, stream)
