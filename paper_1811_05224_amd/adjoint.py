"""Differentiable flux solve: w = V_h^{-1} [(1/2 M_h + K_h) g - M_h^0 u0].

Backward (hand-written adjoint, every product in the HIP library):
    V_h^T lam = dJ/dw                       (stbem_solve, trans: GMRES with Mt^-1 D_h^T Mt^-1)
    dJ/dg     = (1/2 M_h + K_h)^T lam       (stbem_rhs_adjoint)
    dJ/dalpha = lam^T (dK_h/dalpha g - dM_h^0/dalpha u0 - dV_h/dalpha w)   (stbem_grad_alpha)
The alpha-derivative matrices are assembled analytically (closed forms of the
derivatives of the time integrals), see include/stbem.h.
"""
from __future__ import annotations

import torch



class HeatFluxSolve(torch.autograd.Function):
    """w = HeatFluxSolve.apply(g, alpha, ctx, u0, opts).

    g: (N,) float64 Dirichlet data; alpha: 0-d float64 tensor equal to the
    context's alpha (the operators are assembled for that value); ctx: a
    Context with V, K, D (+ M0 if u0 is given) assembled, and DV, DK (+ DM0)
    when alpha needs a gradient; u0: (M_Omega,) tensor or None; opts: dict of
    Context.solve keyword arguments for both solves."""

    @staticmethod
    def forward(fctx, g, alpha, ctx, u0=None, opts=None):
        opts = dict(opts or {})
        if abs(float(alpha) - ctx.alpha_value) > 0.0:
            raise ValueError("alpha must equal the alpha the context was assembled for")
        f = ctx.rhs(g, u0)
        w, info = ctx.solve(f, **opts)
        if info.status:
            raise RuntimeError(f"forward solve did not converge: {info}")
        fctx.ctx, fctx.opts = ctx, opts
        fctx.save_for_backward(g, w, u0 if u0 is not None else torch.empty(0, dtype=g.dtype, device=g.device))
        fctx.has_u0 = u0 is not None
        return w

    @staticmethod
    def backward(fctx, gw):
        ctx, opts = fctx.ctx, dict(fctx.opts)
        g, w, u0 = fctx.saved_tensors
        u0 = u0 if fctx.has_u0 else None
        opts["trans"] = True
        lam, info = ctx.solve(gw.contiguous(), **opts)
        if info.status:
            raise RuntimeError(f"adjoint solve did not converge: {info}")
        grad_g = grad_alpha = None
        if fctx.needs_input_grad[0]:
            grad_g = ctx.rhs_adjoint(lam)
        if fctx.needs_input_grad[1]:
            grad_alpha = ctx.grad_alpha(lam, w, g, u0).reshape(())
        return grad_g, grad_alpha, None, None, None
