"""Differentiable normal-equation solve: chi = (D^+ D)^{-1} phi.

Backward, for the upstream gradient g = dL/dchi (PyTorch's complex
convention, grad = dL/dRe + i dL/dIm):
    lambda   = (D^+ D)^{-1} g        one adjoint CG solve (D^+ D is Hermitian)
    grad_phi = lambda
    grad_U   = G(D chi, lambda) + G(D lambda, chi)
with G the gauge-link force kernel (wilson_force). Derivation: dchi =
-M^{-1} dM chi with M = D^+ D, dM = dD^+ D + D^+ dD, dD = -1/2 dH.
Every step runs in the HIP library: two solves, two operator applications
and two force kernels.
"""
from __future__ import annotations

import torch

from . import ops


class WilsonSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, phi, mass, tol=1e-12, max_iter=100000, inner="f64"):
        chi, info = ops.cg_solve(U, phi, mass, tol=tol, max_iter=max_iter, rhs="normal", inner=inner)
        ctx.save_for_backward(U, chi)
        ctx.mass = float(mass)
        ctx.tol = float(tol)
        ctx.max_iter = int(max_iter)
        ctx.inner = inner
        ctx.info = info
        return chi

    @staticmethod
    def backward(ctx, g):
        U, chi = ctx.saved_tensors
        g = g.contiguous()
        lam, _ = ops.cg_solve(U, g, ctx.mass, tol=ctx.tol, max_iter=ctx.max_iter, rhs="normal", inner=ctx.inner)
        grad_U = None
        if ctx.needs_input_grad[0]:
            eta_chi = ops.wilson_apply(U, chi, ctx.mass)
            eta_lam = ops.wilson_apply(U, lam, ctx.mass)
            grad_U = ops.wilson_force(eta_chi, lam, 1.0)
            ops.wilson_force(eta_lam, chi, 1.0, out=grad_U, accumulate=True)
        grad_phi = lam if ctx.needs_input_grad[1] else None
        return grad_U, grad_phi, None, None, None, None


def wilson_solve(U, phi, mass, tol=1e-12, max_iter=100000, inner="f64"):
    """chi = (D^+ D)^{-1} phi, differentiable in U and phi. inner selects the
    solves' inner storage as for cg_solve (both solves reach tol in FP64)."""
    return WilsonSolve.apply(U, phi, mass, tol, max_iter, inner)
