"""torch.autograd wrappers around the library's projector and prior.

``project(x)`` is y = P M x with backward g -> M P^T g (the exact transpose:
both walk the same segments); ``prior_energy(x)`` is lambda_r ||D x||^2 +
lambda_t ||D_t x||^2 = x . (lambda_r D^T D + lambda_t D_t^T D_t) x with
gradient 2 (lambda_r D^T D + lambda_t D_t^T D_t) x; with ``height`` = (cx, cy,
cz, offset) the spatial term is lambda_r ||D R x||^2 (Eq. srt_inversion, R the
voxel heights).  The geometry's gains are part of P.  The operators run in
the HIP library; only the final dot product of the prior is a torch
reduction.
"""
from __future__ import annotations

import torch

from . import tomo as _t


class SiddonProject(torch.autograd.Function):
    """y = P M x; dL/dx = M P^T dL/dy."""

    @staticmethod
    def forward(ctx, cube: torch.Tensor, geom: _t.DeviceGeometry, strategy: int = _t.BP_AUTO):
        ctx.geom = geom
        ctx.strategy = strategy
        ctx.shape = cube.shape
        return _t.project(geom, cube.contiguous())

    @staticmethod
    def backward(ctx, grad_images: torch.Tensor):
        g = _t.backproject(ctx.geom, grad_images.contiguous(), strategy=ctx.strategy)
        return g.reshape(ctx.shape), None, None


class PriorEnergy(torch.autograd.Function):
    """lambda_r ||D R x||^2 + lambda_t ||D_t x||^2 (R = I without a height)
    and its gradient."""

    @staticmethod
    def forward(ctx, cube: torch.Tensor, geom: _t.DeviceGeometry, lam_r: float, lam_t: float = 0.0,
                height=None):
        x = cube.contiguous()
        lx = _t.apply_prior(geom, x, lam_r, lam_t, height=height)
        ctx.save_for_backward(lx)
        return torch.dot(x.reshape(-1).double(), lx.reshape(-1).double())

    @staticmethod
    def backward(ctx, grad):
        (lx,) = ctx.saved_tensors
        return (2.0 * grad.to(lx.dtype)) * lx, None, None, None, None


def project(cube: torch.Tensor, geom: _t.DeviceGeometry, strategy: int = _t.BP_AUTO):
    return SiddonProject.apply(cube, geom, strategy)


def prior_energy(cube: torch.Tensor, geom: _t.DeviceGeometry, lam_r: float, lam_t: float = 0.0, height=None):
    return PriorEnergy.apply(cube, geom, lam_r, lam_t, height)


def data_loss(cube: torch.Tensor, geom: _t.DeviceGeometry, y: torch.Tensor, lam_r: float,
              lam_t: float = 0.0, height=None):
    """0.5 ||P M x - y||^2 + lambda_r ||D R x||^2 (+ temporal term), in FP64
    reductions over FP32 operators; gradient P^T (P x - y) + 2 lambda R D^T D R x
    (R = I without a height)."""
    r = project(cube, geom) - y
    return 0.5 * torch.dot(r.double(), r.double()) + prior_energy(cube, geom, lam_r, lam_t, height)
