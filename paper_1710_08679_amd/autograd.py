"""``torch.autograd.Function`` for a surface-displacement misfit of the
multi-case elastic solve, differentiated with respect to the per-element
Young's modulus by the adjoint method.

forward:  K(E) u_c = f_c (one multi-case solve), L = 1/2 sum_c ||S u_c - d_c||^2
backward: K(E) lambda_c = S^T (S u_c - d_c) (one more solve; K is symmetric),
          dL/dE_e = - sum_c lambda_{c,e}^T (K_e/E_e) u_{c,e}  (ebe_adjoint_grad).

The solves and the element gradient run in the HIP library; torch only
gathers the surface DOFs and sums the squared misfit.
"""
from __future__ import annotations

import torch

from . import ebe


class SurfaceMisfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, young, mesh: "ebe.Mesh", poisson, f, surf_dofs, target, opts, grad_dtype=torch.float64):
        mesh.set_material(young.detach().contiguous(), poisson.contiguous())
        u, st = mesh.solve(f, opts=opts, raise_on_nonconv=True)
        n = f.shape[2]
        res = u.view(-1, n)[surf_dofs] - target
        ctx.mesh, ctx.opts, ctx.grad_dtype = mesh, opts, grad_dtype
        ctx.save_for_backward(u, res, surf_dofs)
        ctx.forward_stats = st
        return 0.5 * (res * res).sum()

    @staticmethod
    def backward(ctx, g_out):
        u, res, surf_dofs = ctx.saved_tensors
        n = u.shape[2]
        rhs = torch.zeros_like(u)
        rhs.view(-1, n)[surf_dofs] = res
        lam, _ = ctx.mesh.solve(rhs, opts=ctx.opts, raise_on_nonconv=True)
        dt = ctx.grad_dtype
        g = ctx.mesh.adjoint_grad(u.to(dt).contiguous(), lam.to(dt).contiguous()).to(torch.float64)
        return g_out * g, None, None, None, None, None, None, None


def surface_misfit(young, mesh, poisson, f, surf_dofs, target, opts=None, grad_dtype=torch.float64):
    """L(E) with an adjoint gradient; see the module docstring."""
    if opts is None:
        opts = ebe.default_opts(precond=ebe.PREC_MG3, mode=ebe.MODE_MIXED, tol=1e-10)
    return SurfaceMisfit.apply(young, mesh, poisson, f, surf_dofs, target, opts, grad_dtype)
