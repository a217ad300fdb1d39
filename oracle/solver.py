"""Conjugate gradient on the normal equations, FP64.

TEST INFRASTRUCTURE ONLY (see the package header).

The paper's solver is the conjugate-gradient method for large sparse linear
systems (Sec. 1), driven by a host loop that owns the solution, residual and
helper vectors and evaluates the stopping test (Sec. 3.1.1), with one
operator application by the accelerator per step (Sec. 3.1). The Wilson-Dirac
matrix D is not Hermitian, so CG runs on the Hermitian positive-definite
normal system D^dagger D x = D^dagger b (CGNR). The steps below are the
Hestenes-Stiefel CG recurrences on M = D^dagger D, with M p evaluated as
D^dagger (D p) so that <p, M p> = ||D p||^2.

Stopping test: relative residual of the normal system,
||b' - M x|| / ||b'|| <= tol, with b' = D^dagger b (or b' = b when the
caller asks for M x = b directly).
"""
from __future__ import annotations

import numpy as np

from .dirac import dense_D, normal_op, wilson_D, wilson_Ddag


def _dot(a: np.ndarray, b: np.ndarray) -> complex:
    return complex(np.vdot(a, b))


def _norm2(a: np.ndarray) -> float:
    return float(np.vdot(a, a).real)


def cgnr(U, b, mass, tol=1e-10, max_iter=10000, rhs="source", x0=None, history=False, progress=None):
    """Solve D^dagger D x = D^dagger b (rhs="source") or D^dagger D x = b (rhs="normal").

    Returns (x, info) where info holds the iteration count, the iterated and
    the recomputed ("true") relative residuals and, if asked, the iterated
    relative residual after every step. ``progress(k, rel)``, if given, is
    called after every step (for long timed runs; it does not touch the
    arithmetic).
    """
    if rhs == "source":
        bp = wilson_Ddag(U, b, mass)
    elif rhs == "normal":
        bp = b.copy()
    else:
        raise ValueError(rhs)
    bnorm = np.sqrt(_norm2(bp))
    x = np.zeros_like(bp) if x0 is None else x0.astype(np.complex128).copy()
    r = bp - normal_op(U, x, mass)
    p = r.copy()
    rho = _norm2(r)
    hist = []
    k = 0
    if bnorm == 0.0:
        return x, dict(iterations=0, iter_rel_res=0.0, true_rel_res=0.0, history=hist)
    rel = np.sqrt(rho) / bnorm
    while rel > tol and k < max_iter:
        t = wilson_D(U, p, mass)
        alpha = rho / _norm2(t)
        x = x + alpha * p
        q = wilson_Ddag(U, t, mass)
        r = r - alpha * q
        rho_new = _norm2(r)
        k += 1
        rel = np.sqrt(rho_new) / bnorm
        if history:
            hist.append(rel)
        if progress is not None:
            progress(k, rel)
        beta = rho_new / rho
        p = r + beta * p
        rho = rho_new
    true = np.sqrt(_norm2(bp - normal_op(U, x, mass))) / bnorm
    return x, dict(iterations=k, iter_rel_res=rel, true_rel_res=true, history=hist)


def true_relative_residual(U, x, b, mass, rhs="source") -> float:
    """||b' - D^dagger D x|| / ||b'|| with b' = D^dagger b (or b)."""
    bp = wilson_Ddag(U, b, mass) if rhs == "source" else b
    return float(np.sqrt(_norm2(bp - normal_op(U, x, mass))) / np.sqrt(_norm2(bp)))


def dense_solve_normal(U, b, mass, dims, rhs="source"):
    """Direct solve of the same system with the dense matrix (tiny lattices)."""
    D = dense_D(U, mass, dims)
    bv = b.reshape(-1)
    if rhs == "source":
        x = np.linalg.solve(D, bv)          # D x = b  <=>  D^+ D x = D^+ b
    else:
        x = np.linalg.solve(D.conj().T @ D, bv)
    return x.reshape(b.shape)
