"""Differentiable screened-Poisson solve.

u = A(kappa)^{-1} M f with A(kappa) the kappa-weighted SIPDG operator
(lambda M - div kappa grad).  The backward pass solves the adjoint system
A w = dL/du (A is symmetric, so this is the same operator and the same PCG)
and returns dL/df = M w and dL/dkappa_e = -w^T (dA/dkappa_e) u, the latter
from one per-element kernel (ipdg_kappa_grad).  The mass form is provided as
its own differentiable op so that M-weighted losses stay on the device.
"""
from __future__ import annotations

import torch

from . import ipdg as _ipdg


class MassApply(torch.autograd.Function):
    """y = M x (block-diagonal mass); M is symmetric, so dx = M dy."""

    @staticmethod
    def forward(ctx, x, mesh):
        ctx.mesh = mesh
        return mesh.mass(x.contiguous())

    @staticmethod
    def backward(ctx, gy):
        return ctx.mesh.mass(gy.contiguous()), None


class HelmholtzSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, kappa, mesh, lam, tau, tol, opts):
        mesh.set_kappa(kappa.detach().double().cpu().numpy())
        b = mesh.mass(f.detach().contiguous())
        u, info, st = mesh.pcg(b, lam=lam, tau=tau, tol=tol, opts=opts)
        if st != 0:
            raise _ipdg.IpdgError(st, "forward solve did not converge")
        ctx.mesh, ctx.lam, ctx.tau, ctx.tol, ctx.opts = mesh, lam, tau, tol, opts
        ctx.kappa_host = kappa.detach().double().cpu().numpy()
        ctx.forward_info = info
        ctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(ctx, gu):
        (u,) = ctx.saved_tensors
        mesh = ctx.mesh
        mesh.set_kappa(ctx.kappa_host)
        w, info, st = mesh.pcg(gu.contiguous().double(), lam=ctx.lam, tau=ctx.tau, tol=ctx.tol,
                               opts=ctx.opts)
        if st != 0:
            raise _ipdg.IpdgError(st, "adjoint solve did not converge")
        gf = mesh.mass(w) if ctx.needs_input_grad[0] else None
        gk = mesh.kappa_grad(u, w, tau=ctx.tau) if ctx.needs_input_grad[1] else None
        return gf, gk, None, None, None, None, None


def helmholtz_solve(f, kappa, mesh, lam=1.0, tau=0.0, tol=1e-10, opts=None):
    """Differentiable u = (lam M - div kappa grad)^{-1} M f on `mesh`."""
    return HelmholtzSolve.apply(f, kappa, mesh, lam, tau, tol, opts)


def mass(x, mesh):
    return MassApply.apply(x, mesh)
