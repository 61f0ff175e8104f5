"""torch.autograd.Function over field_eval / field_eval_backward.

    E = field(ctx, mesh, sigma, xs, q, xt, soft, precision, tgt_is_src)

Differentiable in sigma (cell charge densities), xt (targets) and xs
(sources).  The forward keeps only its inputs; the backward calls the
library's adjoint, which recomputes every source and cell tile.  With
tgt_is_src the same tensor is the sources and the targets and its gradient
carries both roles (returned once, through xt).
"""
from __future__ import annotations

import torch

from . import binding as B


class FieldEval(torch.autograd.Function):
    @staticmethod
    def forward(fctx, obem_ctx, mesh, sigma, xs, q, xt, soft, precision, tgt_is_src):
        E = B.field_eval(obem_ctx, mesh, sigma, xs, q, xt, soft, precision, tgt_is_src=tgt_is_src)
        fctx.obem = (obem_ctx, mesh, soft, precision, tgt_is_src)
        fctx.save_for_backward(sigma if sigma is not None else torch.empty(0), xs if xs is not None else torch.empty(0),
                               q if q is not None else torch.empty(0), xt)
        return E

    @staticmethod
    def backward(fctx, gE):
        obem_ctx, mesh, soft, precision, tis = fctx.obem
        sigma, xs, q, xt = fctx.saved_tensors
        has_src = xs.numel() > 0
        need_sigma = mesh is not None and fctx.needs_input_grad[2]
        need_t = fctx.needs_input_grad[5] or (tis and fctx.needs_input_grad[3])
        need_s = has_src and not tis and fctx.needs_input_grad[3]
        gs, gt, gsrc = B.field_eval_backward(obem_ctx, mesh, sigma if mesh is not None else None,
                                             xs if has_src else None, q if has_src else None, xt, soft,
                                             gE.contiguous(), precision, tgt_is_src=tis, want_sigma=need_sigma,
                                             want_t=need_t, want_s=need_s)
        return (None, None, gs if need_sigma else None, gsrc if need_s else None, None, gt if need_t else None,
                None, None, None)


def field(obem_ctx, mesh, sigma, xs, q, xt, soft, precision=B.OBEM_MIXED, tgt_is_src=False):
    """Differentiable field at xt (n_t, 3) from the cells of `mesh` with
    densities sigma and the point charges q at xs (either may be None)."""
    return FieldEval.apply(obem_ctx, mesh, sigma, xs, q, xt, soft, precision, tgt_is_src)


class SolveCharges(torch.autograd.Function):
    """sigma = A^{-1} rhs (eq. (matrixBEM)); backward g_rhs = A^{-T} g_sigma."""

    @staticmethod
    def forward(fctx, obem_ctx, mesh, rhs):
        sigma, _ = B.bem_solve_charges(obem_ctx, mesh, rhs.contiguous(), want_info=False)
        fctx.obem = (obem_ctx, mesh)
        return sigma

    @staticmethod
    def backward(fctx, g_sigma):
        obem_ctx, mesh = fctx.obem
        g_rhs, _ = B.bem_solve_charges_adjoint(obem_ctx, mesh, g_sigma.contiguous(), want_info=False)
        return None, None, g_rhs


def solve_charges(obem_ctx, mesh, rhs):
    """Differentiable collocation solve: cell charge densities from the
    left-hand side [V_i (ed) ; sigma_F,i (dd)]."""
    return SolveCharges.apply(obem_ctx, mesh, rhs)
