"""Derivative of the normal-equation solve with respect to the gauge links.

TEST INFRASTRUCTURE ONLY (see the package header).

For chi = M^{-1} phi with M = D^dagger D and a real loss L(chi, phi), an
upstream gradient g = dL/dchi gives (PyTorch's convention for complex
tensors: grad = dL/dRe + i dL/dIm):

    lambda = M^{-1} g                  (adjoint solve; M is Hermitian)
    grad_phi = lambda
    grad_U   = G(D chi, lambda) + G(D lambda, chi)

Derivation: dchi = -M^{-1} dM chi and dM = dD^dagger D + D^dagger dD with
dD = -1/2 dH, so dL = 1/2 Re<D chi, dH lambda> + 1/2 Re<D lambda, dH chi>.
G(a, b) is the gradient of 1/2 Re<a, H b> with respect to the links:

    G(a, b)_mu(x) = 1/2 sum_spin [ ((1 - gamma_mu) a(x)) (x) b(x + mu)^*
                                 + b(x) (x) ((1 + gamma_mu) a(x + mu))^* ]

where (x) is the colour outer product (i, j) -> u_i conj(v_j), summed over
the four spin components.
"""
from __future__ import annotations

import numpy as np

from .dirac import GAMMA, _axis, _ID4, wilson_D
from .solver import cgnr


def _outer(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """sum_s a_{s,i} conj(b_{s,j}) at every site -> (..., 3, 3)."""
    return np.matmul(np.swapaxes(a, -1, -2), b.conj())


def force_G(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """G(a, b), shape (4, Lt, Lz, Ly, Lx, 3, 3)."""
    out = np.empty((4,) + a.shape[:4] + (3, 3), dtype=np.complex128)
    for mu in range(4):
        ax = _axis(mu)
        pm_a = np.matmul(_ID4 - GAMMA[mu], a)                      # (1 - gamma) a(x)
        b_f = np.roll(b, -1, axis=ax)                              # b(x + mu)
        pp_a_f = np.roll(np.matmul(_ID4 + GAMMA[mu], a), -1, axis=ax)  # (1 + gamma) a(x + mu)
        out[mu] = 0.5 * (_outer(pm_a, b_f) + _outer(b, pp_a_f))
    return out


def solve_gradients(U, phi, g, mass, tol=1e-13, max_iter=100000):
    """Forward solve chi = M^{-1} phi and the backward pass for upstream g.

    Returns (chi, grad_U, grad_phi).
    """
    chi, _ = cgnr(U, phi, mass, tol=tol, max_iter=max_iter, rhs="normal")
    lam, _ = cgnr(U, g, mass, tol=tol, max_iter=max_iter, rhs="normal")
    grad_U = force_G(wilson_D(U, chi, mass), lam) + force_G(wilson_D(U, lam, mass), chi)
    return chi, grad_U, lam
