"""Gauge-covariant lattice Laplacian and plain CG, FP64 -- TEST INFRASTRUCTURE ONLY.

A second linear operator for the same conjugate-gradient machinery: the paper
presents its accelerator design as a backbone on which other linear operators
can be solved with unchanged data transport (abstract; Sec. 3.2; Sec. 7). This
one acts on colour vectors (3 complex numbers per site) with the same 3x3
link matrices and the same nearest-neighbour stencil shape as the Wilson
operator, without spin:

    (L psi)(x) = (m2 + 8) psi(x) - sum_{mu=0..3} [ U_mu(x) psi(x + mu)
                                                 + U_mu(x - mu)^dagger psi(x - mu) ]

For unitary links the hopping sum H has operator norm <= 8, so L is Hermitian
and positive definite for m2 > 0 (spectrum in [m2, m2 + 16]) and plain CG
applies directly, with no normal equations. For U = 1 it is the free
lattice Laplacian -sum_mu (psi(x+mu) + psi(x-mu) - 2 psi(x)) plus m2.

Array layout: U (4, Lt, Lz, Ly, Lx, 3, 3) as for the Wilson operator;
psi (Lt, Lz, Ly, Lx, 3). Direction mu lives on numpy axis 3 - mu.
"""
from __future__ import annotations

import numpy as np


def laplace(U: np.ndarray, psi: np.ndarray, m2: float) -> np.ndarray:
    """L psi by the definition above (periodic wrap by roll)."""
    out = (m2 + 8.0) * psi
    for mu in range(4):
        ax = 3 - mu
        fwd = np.einsum("...ij,...j->...i", U[mu], np.roll(psi, -1, axis=ax))      # U_mu(x) psi(x+mu)
        bwd = np.roll(np.einsum("...ji,...j->...i", U[mu].conj(), psi), 1, axis=ax)  # U_mu(x-mu)^+ psi(x-mu)
        out = out - fwd - bwd
    return out


def laplace_sites(U: np.ndarray, psi: np.ndarray, m2: float, sites) -> np.ndarray:
    """(L psi)(x) at the listed sites (x, y, z, t) only, from the definition
    with explicit periodic neighbour indices; returns (len(sites), 3)."""
    lt, lz, ly, lx = psi.shape[:4]
    dims = (lx, ly, lz, lt)
    out = np.zeros((len(sites), 3), dtype=np.complex128)
    for k, site in enumerate(sites):
        c = list(site)
        x, y, z, t = c
        acc = (m2 + 8.0) * psi[t, z, y, x]
        for mu in range(4):
            f = list(c)
            f[mu] = (f[mu] + 1) % dims[mu]
            b = list(c)
            b[mu] = (b[mu] - 1) % dims[mu]
            acc = acc - U[mu, t, z, y, x] @ psi[f[3], f[2], f[1], f[0]]
            acc = acc - U[mu, b[3], b[2], b[1], b[0]].conj().T @ psi[b[3], b[2], b[1], b[0]]
        out[k] = acc
    return out


def dense_laplace(U: np.ndarray, m2: float, dims) -> np.ndarray:
    """The (3V x 3V) matrix of L, assembled block by block from the formula.

    Row/column index = 3 * site + colour with site = x + Lx (y + Ly (z + Lz t)),
    the order of psi.reshape(-1).
    """
    lx, ly, lz, lt = dims
    V = lx * ly * lz * lt
    A = np.zeros((3 * V, 3 * V), dtype=np.complex128)

    def idx(x, y, z, t):
        return ((t * lz + z) * ly + y) * lx + x

    for t in range(lt):
        for z in range(lz):
            for y in range(ly):
                for x in range(lx):
                    s = idx(x, y, z, t)
                    A[3 * s:3 * s + 3, 3 * s:3 * s + 3] += (m2 + 8.0) * np.eye(3)
                    c = [x, y, z, t]
                    for mu in range(4):
                        L = dims[mu]
                        f = list(c)
                        f[mu] = (f[mu] + 1) % L
                        b = list(c)
                        b[mu] = (b[mu] - 1) % L
                        sf, sb = idx(*f), idx(*b)
                        A[3 * s:3 * s + 3, 3 * sf:3 * sf + 3] -= U[mu, t, z, y, x]
                        ub = U[mu, b[3], b[2], b[1], b[0]]
                        A[3 * s:3 * s + 3, 3 * sb:3 * sb + 3] -= ub.conj().T
    return A


def _dot(a, b) -> complex:
    return complex(np.vdot(a.reshape(-1), b.reshape(-1)))


def cg(U: np.ndarray, b: np.ndarray, m2: float, tol: float = 1e-10, max_iter: int = 10000, history: bool = False):
    """Conjugate gradient on L x = b from x = 0, the textbook recurrences:
    alpha = rho / <p, L p>, x += alpha p, r -= alpha L p, beta = rho' / rho,
    p = r + beta p; stop when ||r|| <= tol ||b||, then report the true
    residual ||b - L x|| / ||b||."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    bn = np.sqrt(_dot(b, b).real)
    rho = _dot(r, r).real
    hist = []
    it = 0
    while it < max_iter and np.sqrt(rho) > tol * bn:
        t = laplace(U, p, m2)
        alpha = rho / _dot(p, t).real
        x = x + alpha * p
        r = r - alpha * t
        rho_new = _dot(r, r).real
        it += 1
        hist.append(np.sqrt(rho_new) / bn)
        p = r + (rho_new / rho) * p
        rho = rho_new
    res = laplace(U, x, m2) - b
    info = {"iterations": it, "iter_rel_res": np.sqrt(rho) / bn,
            "true_rel_res": np.sqrt(_dot(res, res).real) / bn}
    if history:
        info["history"] = hist
    return x, info


def true_relative_residual(U, x, b, m2) -> float:
    r = b - laplace(U, x, m2)
    return float(np.sqrt(_dot(r, r).real / _dot(b, b).real))
