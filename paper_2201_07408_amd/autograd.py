"""Differentiable forward projection: forward = ct_project_A, backward = the
hand-written matched transpose ct_backproject_AT (the exact adjoint, which
CGLS requires and the unmatched back-projectors are not)."""

import torch

from .api import ct_project_A, ct_backproject_AT


class ProjectA(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, geom):
        ctx.geom = geom
        return ct_project_A(geom, x.contiguous())

    @staticmethod
    def backward(ctx, grad_y: torch.Tensor):
        return ct_backproject_AT(ctx.geom, grad_y.contiguous()), None


def project(x: torch.Tensor, geom) -> torch.Tensor:
    return ProjectA.apply(x, geom)
