"""Autograd operators (the paper's PyTorch operator wrappers, section 2.8):
A as a linear differentiable operator whose backward is the matched A^T
kernel, and A^T whose backward is A.  Zero-copy: device tensors go straight
to the kernels, batched over a leading dimension.
"""
from __future__ import annotations

import torch

from .ops import Plan


def _batched(t: torch.Tensor, inner):
    lead = t.shape[: t.dim() - len(inner)]
    if tuple(t.shape[t.dim() - len(inner):]) != tuple(inner):
        raise ValueError(f"expected trailing shape {tuple(inner)}, got {tuple(t.shape)}")
    return lead, t.reshape((-1,) + tuple(inner)).contiguous()


class _Project(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, plan: Plan, kind: str):
        ctx.plan, ctx.kind = plan, kind
        lead, xb = _batched(x, plan.vol_shape)
        out = torch.empty((xb.shape[0],) + plan.proj_shape(), dtype=torch.float32, device=x.device)
        for i in range(xb.shape[0]):
            plan.forward(xb[i], out=out[i], kind=kind)
        return out.reshape(lead + plan.proj_shape())

    @staticmethod
    def backward(ctx, g):
        return _BackProject.apply(g, ctx.plan, ctx.kind), None, None


class _BackProject(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, plan: Plan, kind: str):
        ctx.plan, ctx.kind = plan, kind
        lead, yb = _batched(y, plan.proj_shape())
        out = torch.empty((yb.shape[0],) + plan.vol_shape, dtype=torch.float32, device=y.device)
        for i in range(yb.shape[0]):
            plan.backproject(yb[i], out=out[i], kind=kind)
        return out.reshape(lead + plan.vol_shape)

    @staticmethod
    def backward(ctx, g):
        return _Project.apply(g, ctx.plan, ctx.kind), None, None


class Projector:
    """A = Projector(geo, angles, kind="siddon"|"interp"); A(x) projects a
    volume [..., nz, ny, nx]; A.T(y) backprojects [..., nviews, nv, nu] with
    the exact transpose.  Both are differentiable."""

    def __init__(self, geo, angles, kind: str = "siddon", device=None):
        if kind not in ("siddon", "interp"):
            raise ValueError("kind must be 'siddon' or 'interp'")
        self.plan = Plan(geo, angles, device)
        self.kind = kind

    def __call__(self, x: torch.Tensor) -> torch.Tensor:
        return _Project.apply(x, self.plan, self.kind)

    def T(self, y: torch.Tensor) -> torch.Tensor:
        return _BackProject.apply(y, self.plan, self.kind)


def create_pytorch_operator(geo, angles, kind: str = "siddon", device=None):
    """(ax, atb) pair of differentiable operators."""
    A = Projector(geo, angles, kind, device)
    return A, A.T
