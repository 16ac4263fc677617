"""Differentiable one-shot Parareal objective: a torch.autograd.Function whose
forward is pt_parareal_forward and whose backward is the hand-written adjoint
pass (pt_parareal_adjoint) plus pt_sensitivities (Sec. 4.1, Eq. 4.7; Sec. 4.4).

`OneShotParareal` keeps the warm-restart state of Alg. 3: every call uses the
previous call's corrected coarse states u_n and adjoint states v_n as the
Parareal guess (the first call starts cold from the coarse sweeps).
"""
from __future__ import annotations

from typing import Optional

import torch

from ._pt import Problem
from .cycle import Cycle


class PararealTO(torch.autograd.Function):
    """Theta(rho) with d Theta / d rho from the reversed Parareal adjoint pass."""

    @staticmethod
    def forward(ctx, rho: torch.Tensor, state: "OneShotParareal") -> torch.Tensor:
        cyc = state.cycle
        r = rho.detach().contiguous()
        if state.warm and state.guess_T is not None:
            cyc.forward(r, state.guess_T, state.guess_theta)
        else:
            cyc.forward(r)
        ctx.state = state
        ctx.save_for_backward(r)
        state._fresh_forward = True
        return cyc.Theta.clone()

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        (r,) = ctx.saved_tensors
        state = ctx.state
        cyc = state.cycle
        if not state._fresh_forward:
            raise RuntimeError("backward needs the S of the matching forward; run forward again")
        if state.warm and state.guess_lambda is not None:
            cyc.adjoint(r, state.guess_lambda)
        else:
            cyc.adjoint(r)
        cyc.sensitivities(r)
        state._fresh_forward = False
        state._store_guesses()
        return grad_out * cyc.grad.clone(), None


class OneShotParareal:
    """Callable objective for a fixed problem size: theta = obj(rho).

    With warm=True each call restarts Parareal from the previous cycle's
    solution (the one-shot method); with warm=False every call is a cold
    one-iteration pass (or, with prob.iterations = N_tau or n_slices = 1, the
    exact sequential result).
    """

    def __init__(self, prob: Problem, device="cuda", warm: bool = True):
        self.prob = prob
        self.cycle = Cycle(prob, device)
        self.warm = warm
        self.guess_T: Optional[torch.Tensor] = None
        self.guess_theta: Optional[torch.Tensor] = None
        self.guess_lambda: Optional[torch.Tensor] = None
        self._fresh_forward = False

    def _store_guesses(self):
        if not self.warm:
            return
        c = self.cycle
        self.guess_T = c.uT.clone()
        self.guess_theta = c.utheta.clone()
        self.guess_lambda = c.lam.clone()

    def reset(self):
        self.guess_T = self.guess_theta = self.guess_lambda = None

    def __call__(self, rho: torch.Tensor) -> torch.Tensor:
        return PararealTO.apply(rho, self)

    def objective(self, rho: torch.Tensor) -> float:
        """Theta only (no warm-state update), e.g. for finite differences."""
        with torch.no_grad():
            if self.warm and self.guess_T is not None:
                self.cycle.forward(rho.contiguous(), self.guess_T, self.guess_theta)
            else:
                self.cycle.forward(rho.contiguous())
            self._fresh_forward = False
            return float(self.cycle.Theta)
