"""torch.autograd wrapper of the JTFS transform (forward and exact backward in HIP).

Two memory modes:
* ``"store"``: the forward keeps its intermediates (first-layer scalogram, its DFT,
  second-order stacks) in a backward-sized workspace held by the autograd graph; the
  backward reuses them (``JTFS_REUSE_FORWARD``).
* ``"recompute"``: only x is saved; the backward recomputes the time-axis
  intermediates from x before the adjoint stages. Both passes run the signals of a batch
  one after another in one shared workspace sized for the largest signal
  (``JTFS_SHARED_WORKSPACE``), so nothing is held between forward and backward and the
  backward's peak is one signal's workspace instead of the whole batch's. Results are
  bitwise identical to ``"store"`` (every kernel is deterministic).

The transform is positively homogeneous of degree 1, so gradients are defined almost
everywhere; where a modulus argument is exactly 0 the subgradient 0 is used.
"""
from __future__ import annotations

import torch

from .jtfs import Plan


class _JTFSFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, plan: Plan, mode: str):
        x = x.contiguous()
        if mode == "store":
            ws = plan.workspace(x.device, backward=True)
        elif mode == "recompute":
            ws = plan.workspace(x.device, backward=False, shared=True)
        else:
            raise ValueError("mode must be 'store' or 'recompute'")
        S = plan.forward(x, ws=ws, shared=(mode == "recompute"))
        ctx.plan = plan
        ctx.mode = mode
        ctx.ws = ws if mode == "store" else None
        ctx.save_for_backward(x)
        return S

    @staticmethod
    def backward(ctx, dS: torch.Tensor):
        (x,) = ctx.saved_tensors
        plan = ctx.plan
        dS = dS.contiguous().to(torch.float32)
        if ctx.mode == "store":
            dx = plan.backward(x, dS, ws=ctx.ws, reuse_forward=True)
            ctx.ws = None
        else:
            dx = plan.backward(x, dS, ws=plan.workspace(x.device, backward=True, shared=True), shared=True)
        return dx, None, None


def jtfs(x: torch.Tensor, plan: Plan, mode: str = "store") -> torch.Tensor:
    """S(x) as a differentiable function of x (float32 CUDA/HIP tensor of plan.n_samples)."""
    return _JTFSFunction.apply(x, plan, mode)


class JTFS(torch.nn.Module):
    """Module form: ``JTFS(Params(...))(x)`` returns the coefficient vector."""

    def __init__(self, params, mode: str = "store"):
        super().__init__()
        self.plan = Plan(params)
        self.mode = mode

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        return jtfs(x, self.plan, self.mode)
