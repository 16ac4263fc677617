"""Many designs in one optimisation cycle: every design's primal pass in one
persistent engine launch, every adjoint pass in a second one, then the
sensitivities (Sec. 4.4 steps 1-4 for each design), with warm restarts kept in
the workspace (Alg. 3). `BatchedOneShot` puts the batch behind a
torch.autograd.Function.
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import _pt
from ._pt import Problem


class BatchedCycle:
    """Owns the workspace and outputs of a fixed list of problems."""

    def __init__(self, probs: Sequence[Problem], device="cuda"):
        self.probs = list(probs)
        self.device = torch.device(device)
        nbytes = _pt.pt_batched_workspace_bytes(self.probs)
        if nbytes == 0:
            raise _pt.PtError(_pt.PT_EINVAL, "BatchedCycle")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.Theta = torch.empty(len(self.probs), dtype=torch.float64, device=self.device)
        self.grads = [torch.empty(p.n_elem, dtype=torch.float64, device=self.device)
                      for p in self.probs]
        self.tuning: Optional[dict] = None
        self.has_state = False

    def run(self, rhos: Sequence[torch.Tensor], warm: Optional[bool] = None, stream=None,
            forward_only: bool = False):
        """One cycle of every design; warm defaults to 'a previous cycle ran'.
        forward_only: the primal passes only (Theta; grads are left as they
        were), e.g. for objective evaluations without gradients."""
        if warm is None:
            warm = self.has_state
        if warm and not self.has_state:
            raise RuntimeError("warm cycle requested before any cycle ran")
        _pt.pt_parareal_batched(self.probs, [r.contiguous() for r in rhos], warm, self.tuning,
                                self.Theta, None if forward_only else self.grads, self.ws,
                                stream)
        self.has_state = True
        return self.Theta, self.grads

    def autotune(self, rhos: Sequence[torch.Tensor], stream=None, progress=None) -> tuple:
        """Picks the launch shape by timing warm cycles of this batch
        (synchronous); returns (shape, its ms, the built-in shape's ms). The
        workspace then holds the tuner's cold-cycle state for a warm cycle.
        progress(shape, ms) is called after each shape is timed."""
        best, ms, ms0 = _pt.pt_autotune_batched(self.probs, [r.contiguous() for r in rhos],
                                                self.Theta, self.grads, self.ws, stream,
                                                progress)
        self.tuning = best
        self.has_state = True
        return best, ms, ms0

    def status(self, stream=None) -> list:
        return _pt.pt_batched_status(self.probs, self.ws, stream)


class _BatchedTO(torch.autograd.Function):
    """Theta of every design; the backward returns grad_out[k] * dTheta_k/drho_k
    from the adjoint pass that ran with the forward (one launch per pass)."""

    @staticmethod
    def forward(ctx, state: "BatchedOneShot", *rhos):
        cyc = state.cycle
        cyc.run([r.detach() for r in rhos], warm=state.warm and cyc.has_state)
        ctx.grads = [g.clone() for g in cyc.grads]
        return cyc.Theta.clone()

    @staticmethod
    def backward(ctx, grad_out):
        return (None, *[grad_out[k] * g for k, g in enumerate(ctx.grads)])


class BatchedOneShot:
    """thetas = obj(rhos): one-shot Parareal objective of many designs at once."""

    def __init__(self, probs: Sequence[Problem], device="cuda", warm: bool = True):
        self.cycle = BatchedCycle(probs, device)
        self.warm = warm

    def __call__(self, rhos: Sequence[torch.Tensor]) -> torch.Tensor:
        """Theta of every design. Without a gradient to compute (torch.no_grad,
        or no density requires grad) only the primal passes run."""
        if not (torch.is_grad_enabled() and any(r.requires_grad for r in rhos)):
            cyc = self.cycle
            cyc.run([r.detach() for r in rhos], warm=self.warm and cyc.has_state,
                    forward_only=True)
            return cyc.Theta.clone()
        return _BatchedTO.apply(self, *rhos)
