"""Constant tuning by gradient steps on top of the adjoint (beagle_eval_grad).

EvalGrad is a torch.autograd.Function whose input is the flat constant
tensor of a population and whose output is every program's fitness (MSE or
the correlation fitness 1 - r^2);
its forward runs the adjoint kernel once and keeps dF_p/dconsts, its backward
scales that saved gradient by the incoming gradient of the owning program
(no second kernel launch).  tune_constants runs Adam on the constants with
loss = sum of the finite fitness values (each program's constants only
influence its own fitness, so this is per-program gradient descent).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import torch

from . import api


def const_owner(progs: api.DevicePrograms) -> torch.Tensor:
    """int64 [n_consts]: the program whose constant table holds each slot (-1: none)."""
    n_consts = progs.consts.numel()
    owner = torch.full((n_consts,), -1, dtype=torch.int64, device=progs.device)
    cc = progs.const_count.to(torch.int64)
    total = int(cc.sum().item())
    if total == 0:
        return owner
    prog = torch.repeat_interleave(torch.arange(progs.n, device=progs.device), cc)
    first = torch.repeat_interleave(torch.cumsum(cc, 0) - cc, cc)
    slot = torch.arange(total, device=progs.device) - first
    owner[progs.const_offset[prog] + slot] = prog
    return owner


class EvalGrad(torch.autograd.Function):
    """fitness[N] of every program (kind "mse" or "corr") as a function of the flat constants."""

    @staticmethod
    def forward(fctx, consts: torch.Tensor, progs: api.DevicePrograms, X: torch.Tensor, y: torch.Tensor,
                owner: torch.Tensor, kind: str = "mse"):
        p = dataclasses.replace(progs, consts=consts.detach().contiguous())
        fit, grad = api.evaluate_grad(p, X, y, kind)
        fctx.save_for_backward(grad, owner)
        return fit

    @staticmethod
    def backward(fctx, grad_out: torch.Tensor):
        grad, owner = fctx.saved_tensors
        scale = torch.where(owner >= 0, grad_out[owner.clamp(min=0)], torch.zeros((), dtype=grad_out.dtype,
                                                                                   device=grad_out.device))
        return (scale * grad.to(grad_out.dtype)).to(grad.dtype), None, None, None, None, None


@dataclasses.dataclass
class TuneResult:
    consts: torch.Tensor
    fitness_before: torch.Tensor
    fitness_after: torch.Tensor
    history: list


def tune_constants(progs: api.DevicePrograms, X: torch.Tensor, y: torch.Tensor, steps: int = 20,
                   lr: float = 0.05, betas=(0.9, 0.999), eps: float = 1e-8,
                   record: bool = False, kind: str = "mse") -> TuneResult:
    """Adam on the constants of every program (fitness kind "mse" or
    "corr"); returns the tuned constants."""
    owner = const_owner(progs)
    consts = progs.consts.detach().clone().requires_grad_(True)
    opt = torch.optim.Adam([consts], lr=lr, betas=betas, eps=eps)
    history = []
    before = None
    for _ in range(steps):
        opt.zero_grad(set_to_none=False)
        fit = EvalGrad.apply(consts, progs, X, y, owner, kind)
        if before is None:
            before = fit.detach().clone()
        ok = torch.isfinite(fit)
        loss = torch.where(ok, fit, torch.zeros_like(fit)).sum()
        loss.backward()
        consts.grad = torch.nan_to_num(consts.grad, nan=0.0, posinf=0.0, neginf=0.0)
        opt.step()
        if record:
            history.append(float(loss.detach()))
    final = api.evaluate(dataclasses.replace(progs, consts=consts.detach().contiguous()), X, y, kind)
    return TuneResult(consts.detach(), before, final, history)
