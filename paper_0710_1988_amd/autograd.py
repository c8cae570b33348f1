"""Differentiable deflated solve: x = A^{-1} b with A = A(U, kappa, mu).

Forward: D-BiCGStab(k) with left vectors gamma5 V.  Backward: for an incoming gradient g of x,
lambda = A^{-H} g comes from a second D-BiCGStab call on the adjoint system that reuses the same
deflation space with the roles of V and gamma5 V swapped (gamma5-hermiticity); then
grad_b = lambda and grad_links = G from the link-gradient kernel, with dL = Re sum conj(G) dU.
With schur the two solves run on the even-odd reduced system (V then holds even-site vectors, as
gmresdr_first_rhs(..., schur=True) returns them); both still return the full vectors x and
lambda of A x = b and A^H lambda = g, so the link gradient is the one of the full operator.
"""
from __future__ import annotations

import torch


class DeflatedSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, links, b, L, kappa, mu, V, tol, prec, max_mv, schur=False):
        from . import dbicgstab_solve
        X, stats, st = dbicgstab_solve(
            [dict(L=L, links=links, kappa=kappa, mu=mu, B=b, V=V, schur=schur)], tol=tol,
            max_mv=max_mv, prec=prec)
        if st != 0:
            raise RuntimeError(f"forward solve did not converge: {stats}")
        x = X[0]
        ctx.save_for_backward(links, x)
        ctx.cfg = (L, kappa, mu, V, tol, prec, max_mv, schur)
        return x

    @staticmethod
    def backward(ctx, g):
        from . import dbicgstab_solve, link_force
        links, x = ctx.saved_tensors
        L, kappa, mu, V, tol, prec, max_mv, schur = ctx.cfg
        g = g.contiguous()
        Lam, stats, st = dbicgstab_solve(
            [dict(L=L, links=links, kappa=kappa, mu=mu, B=g, V=V, schur=schur)], tol=tol,
            max_mv=max_mv, prec=prec, dagger=True)
        if st != 0:
            raise RuntimeError(f"adjoint solve did not converge: {stats}")
        lam = Lam[0]
        grad_links = None
        if ctx.needs_input_grad[0]:
            grad_links = link_force(L, links, kappa, lam, x, kind="complex")
        grad_b = lam if ctx.needs_input_grad[1] else None
        return grad_links, grad_b, None, None, None, None, None, None, None, None
