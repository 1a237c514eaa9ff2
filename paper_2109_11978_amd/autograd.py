"""torch.autograd wrapper over the hand-written backward of the PPO loss.

PPOLoss.apply(theta, ...) returns the scalar PPO loss of one mini-batch
(clipped surrogate + c_v value loss - c_e entropy) for the flat parameter
vector `theta`; its backward is the library's own gradient (output-layer
gradients, MFMA input-gradient chain and split-sample weight gradients),
computed in the same launch sequence as the loss by ppo_loss_grad when theta
requires a gradient, and skipped otherwise (the loss terms alone).  torch
never traces the network: it only sees one opaque op of theta.
"""
from __future__ import annotations

from typing import Dict, Optional

import torch

from . import _abi
from .api import Context, UpdateHParams, _ptr, _stream, batch_abi, ppo_pack_weights
from ._abi import check


class _ParamsView:
    """theta (and its bf16 shadow) in the ABI's parameter struct."""

    def __init__(self, ctx: Context, theta: torch.Tensor):
        self.theta = theta.detach().contiguous()
        self.shadow = torch.empty(theta.numel(), dtype=torch.int16, device=theta.device)
        if ctx.precision == "bf16":
            ppo_pack_weights(ctx, self.theta, self.shadow)

    def abi(self) -> _abi.Params:
        return _abi.Params(_ptr(self.theta, torch.float32, "theta"), None, None, None,
                           _ptr(self.shadow, torch.int16, "shadow"), None, None)


class PPOLoss(torch.autograd.Function):
    @staticmethod
    def forward(fctx, theta: torch.Tensor, ctx: Context, batch: Dict[str, torch.Tensor], idx: torch.Tensor,
                hp: UpdateHParams, ws: torch.Tensor):
        if theta.dtype != torch.float32 or theta.dim() != 1:
            raise TypeError("theta must be a 1-D float32 tensor")
        view = _ParamsView(ctx, theta)
        stats = torch.zeros(_abi.PPO_STATS_WIDTH, dtype=torch.float32, device=theta.device)
        # the hand-written backward runs only when a gradient wrt theta will be
        # asked for; otherwise the library computes the loss terms alone
        want_grad = fctx.needs_input_grad[0]
        grad = torch.empty_like(view.theta) if want_grad else None
        b = batch_abi(batch)
        p = view.abi()
        h = hp.abi()
        import ctypes
        check(_abi.load().ppo_loss_grad(ctx.handle, _stream(None), ctypes.byref(p), ctypes.byref(b),
                                        _ptr(idx, torch.int32, "idx"), idx.numel(), ctypes.byref(h),
                                        _ptr(stats, torch.float32, "stats"),
                                        _ptr(grad, torch.float32, "grad", allow_none=True),
                                        None, None, _ptr(ws, torch.uint8, "ws"), ws.numel()))
        if want_grad:
            fctx.save_for_backward(grad)
        fctx.stats = stats
        return stats[0].clone()

    @staticmethod
    def backward(fctx, grad_output):
        (grad,) = fctx.saved_tensors
        return grad_output * grad, None, None, None, None, None


def ppo_loss(ctx: Context, theta: torch.Tensor, batch: Dict[str, torch.Tensor], idx: torch.Tensor,
             hp: Optional[UpdateHParams] = None, ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Differentiable PPO loss of the mini-batch rows `idx` at parameters `theta`."""
    hp = hp or UpdateHParams()
    if ws is None:
        ws = ctx.new_workspace(M=idx.numel(), device=theta.device)
    return PPOLoss.apply(theta, ctx, batch, idx, hp, ws)
