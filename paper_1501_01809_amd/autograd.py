"""torch.autograd binding of the nonlinear residual and its adjoint assembly.

F(u, kappa; f)_i = integral of kappa grad(u).grad(v_i) + u^3 v_i - f v_i on a
P1 space (``FEM_NL_RESIDUAL``).  The forward pass assembles F with
``fem_par_loop_assemble_vec``; the backward pass, given lambda = dL/dF,
assembles lambda^T dF/du and lambda^T dF/dkappa with
``fem_par_loop_assemble_adjoint``.  f is data, not differentiated.  Argument
marshalling only: every value is computed by the HIP library.
"""
from __future__ import annotations

import torch

from . import fem as F


class ResidualOp:
    """Mesh, plan and forms of one residual: build once, call many times.

    cell_vertex, coords, cell_node: int32 / float64 device tensors of a P1
    mesh (cell_node numbers the P1 nodes); nnodes: node count; prec:
    F.FEM_FP64 or F.FEM_FP32.
    """

    def __init__(self, ctx: F.Context, cell_vertex, coords, cell_node, nnodes: int, prec: int = F.FEM_FP64):
        dim = coords.shape[1]
        self.ctx = ctx
        self.form = F.form("nl_residual", dim, 1, prec=prec)
        self.mesh = (cell_vertex, coords, cell_node, nnodes)
        self.plan = F.fem_plan_create(ctx, self.form, F.Args(cell_vertex, coords, cell_node, nnodes), None)

    def _args(self, *fields):
        cv, X, cn, n = self.mesh
        return F.Args(cv, X, cn, n, [t.contiguous() for t in fields], nodal=True)

    def residual(self, u, kappa, f, out):
        F.fem_par_loop_assemble_vec(self.ctx, self.plan, self.form, self._args(u, kappa, f), out)

    def adjoint(self, u, kappa, lam, g_u, g_kappa):
        F.fem_par_loop_assemble_adjoint(self.ctx, self.plan, self.form, self._args(u, kappa), lam, g_u, g_kappa)


class NonlinearResidual(torch.autograd.Function):
    """F = NonlinearResidual.apply(u, kappa, f, op) with op a ResidualOp;
    differentiable in u and kappa."""

    @staticmethod
    def forward(ctx, u, kappa, f, op):
        out = torch.empty_like(u)
        op.residual(u, kappa, f, out)
        ctx.save_for_backward(u, kappa)
        ctx.op = op
        return out

    @staticmethod
    def backward(ctx, grad_out):
        u, kappa = ctx.saved_tensors
        lam = grad_out.contiguous()
        g_u = torch.empty_like(u) if ctx.needs_input_grad[0] else None
        g_k = torch.empty_like(kappa) if ctx.needs_input_grad[1] else None
        if ctx.needs_input_grad[2]:
            raise NotImplementedError("the residual is not differentiated with respect to f")
        if g_u is not None or g_k is not None:
            ctx.op.adjoint(u, kappa, lam, g_u, g_k)
        return g_u, g_k, None, None
