"""torch.autograd.Function wrappers around the library's action and adjoint.

``PamdAction`` returns S[X] (Eq. 4 without normalisation) as a 0-dim tensor;
its backward is the hand-written adjoint (pamd_action_grad).  With
``retain=True`` the forward already runs the fused action+gradient pass and
keeps dS/dX (one path-sized buffer); with ``retain=False`` the forward only
evaluates the action and the backward recomputes forces inside the adjoint
pass - the choice for paths whose extra copy would not fit in device memory.
``retain=None`` picks by size: keep the gradient when it needs at most a
quarter of the free device memory.

``PamdPerStepAction`` returns the per-step terms s_n; its backward passes the
incoming gradient as per-step weights, so the adjoint kernel itself forms
sum_n (dL/ds_n) ds_n/dX.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import api


def _retain_choice(x: torch.Tensor, retain: Optional[bool]) -> bool:
    if retain is not None:
        return bool(retain)
    free, _ = torch.cuda.mem_get_info(x.device)
    return x.numel() * x.element_size() <= free // 4


class PamdAction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, path, pot, retain=None, tuning=None):
        x = x.contiguous()
        action = torch.empty((), dtype=torch.float64, device=x.device)
        keep = _retain_choice(x, retain)
        ctx.path, ctx.pot, ctx.tuning = path, pot, tuning
        if keep:
            grad = torch.empty_like(x)
            api.pamd_action_grad(path, pot, x, grad, action=action.view(1), tuning=tuning)
            ctx.save_for_backward(grad)
            ctx.kept = True
        else:
            api.pamd_action(path, pot, x, action.view(1), tuning=tuning)
            ctx.save_for_backward(x)
            ctx.kept = False
        return action

    @staticmethod
    def backward(ctx, g_out):
        (saved,) = ctx.saved_tensors
        if ctx.kept:
            grad = saved
        else:
            grad = torch.empty_like(saved)
            api.pamd_action_grad(ctx.path, ctx.pot, saved, grad, tuning=ctx.tuning)
        return grad * g_out, None, None, None, None


class PamdPerStepAction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, path, pot, tuning=None):
        x = x.contiguous()
        per_step = torch.empty(path.n_steps, dtype=torch.float64, device=x.device)
        action = torch.empty(1, dtype=torch.float64, device=x.device)
        api.pamd_action(path, pot, x, action, per_step=per_step, tuning=tuning)
        ctx.save_for_backward(x)
        ctx.path, ctx.pot, ctx.tuning = path, pot, tuning
        return per_step

    @staticmethod
    def backward(ctx, g_out):
        (x,) = ctx.saved_tensors
        grad = torch.empty_like(x)
        api.pamd_action_grad(ctx.path, ctx.pot, x, grad, step_weights=g_out.contiguous(),
                             tuning=ctx.tuning)
        return grad, None, None, None


def path_action(x, path, pot, retain=None, tuning=None) -> torch.Tensor:
    return PamdAction.apply(x, path, pot, retain, tuning)


def per_step_action(x, path, pot, tuning=None) -> torch.Tensor:
    return PamdPerStepAction.apply(x, path, pot, tuning)
