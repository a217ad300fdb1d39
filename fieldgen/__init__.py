"""Seeded synthetic inputs for the Wilson-Dirac solver: gauge links and sources.

This module is shared by the tests, the benchmark and the CPU oracle's tests.
It holds no arithmetic of the method itself (no Dirac operator, no solver):
only random SU(3) link fields, spinor sources and gauge rotations, drawn
from numpy's PCG64 generator with a fixed seed so that every consumer sees
bit-identical inputs.

Array conventions (shared with the library boundary):

* gauge field ``U``: complex128, shape ``(4, Lt, Lz, Ly, Lx, 3, 3)``;
  ``U[mu, t, z, y, x]`` is the colour matrix on the link from site x to
  x + mu_hat, with mu = 0, 1, 2, 3 the x, y, z, t directions.
* spinor field ``psi``: complex128, shape ``(Lt, Lz, Ly, Lx, 4, 3)``
  (spin, colour).
* lattice dims are passed as ``(Lx, Ly, Lz, Lt)`` (x fastest in memory).

The paper's operator is read from a file of real gauge configurations
(Sec. 3.2); none exist here, so these seeded ensembles stand in for them.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "lattice_shape",
    "haar_su3",
    "near_identity_su3",
    "gauge_field",
    "gaussian_spinor",
    "point_sources",
    "gell_mann",
]

# Gell-Mann matrices lambda_1..lambda_8 (the standard basis of traceless
# Hermitian 3x3 matrices, tr(lambda_a lambda_b) = 2 delta_ab).
_GM = np.zeros((8, 3, 3), dtype=np.complex128)
_GM[0][0, 1] = _GM[0][1, 0] = 1
_GM[1][0, 1] = -1j
_GM[1][1, 0] = 1j
_GM[2][0, 0] = 1
_GM[2][1, 1] = -1
_GM[3][0, 2] = _GM[3][2, 0] = 1
_GM[4][0, 2] = -1j
_GM[4][2, 0] = 1j
_GM[5][1, 2] = _GM[5][2, 1] = 1
_GM[6][1, 2] = -1j
_GM[6][2, 1] = 1j
_GM[7][0, 0] = _GM[7][1, 1] = 1 / np.sqrt(3)
_GM[7][2, 2] = -2 / np.sqrt(3)


def gell_mann() -> np.ndarray:
    """Return a copy of the 8 Gell-Mann matrices, shape (8, 3, 3)."""
    return _GM.copy()


def lattice_shape(dims) -> tuple:
    """(Lx, Ly, Lz, Lt) -> numpy site shape (Lt, Lz, Ly, Lx)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    return (lt, lz, ly, lx)


def _chunks(n: int, size: int):
    for s in range(0, n, size):
        yield s, min(n, s + size)


def haar_su3(n: int, rng: np.random.Generator, chunk: int = 1 << 20) -> np.ndarray:
    """n Haar-distributed SU(3) matrices, shape (n, 3, 3), complex128.

    Mezzadri's construction: complex Ginibre matrix -> QR -> fix the phases
    of R's diagonal so that Q is Haar on U(3) -> divide by a cube root of the
    determinant (a centre element does not change the Haar measure).
    """
    out = np.empty((n, 3, 3), dtype=np.complex128)
    for s, e in _chunks(n, chunk):
        m = e - s
        z = (rng.standard_normal((m, 3, 3)) + 1j * rng.standard_normal((m, 3, 3))) / np.sqrt(2.0)
        q, r = np.linalg.qr(z)
        d = np.diagonal(r, axis1=1, axis2=2)
        ph = d / np.abs(d)
        q = q * ph[:, None, :]
        det = np.linalg.det(q)
        q = q * (det ** (-1.0 / 3.0))[:, None, None]
        out[s:e] = q
    return out


def near_identity_su3(n: int, eps: float, rng: np.random.Generator, chunk: int = 1 << 20) -> np.ndarray:
    """n matrices exp(i eps H), H = sum_a omega_a lambda_a / 2 with omega_a ~ N(0,1).

    The exponential is taken through the eigendecomposition of the Hermitian H,
    so the result is unitary with unit determinant to rounding.
    """
    out = np.empty((n, 3, 3), dtype=np.complex128)
    for s, e in _chunks(n, chunk):
        m = e - s
        w = rng.standard_normal((m, 8))
        h = np.einsum("na,aij->nij", w, _GM) * 0.5
        lam, vec = np.linalg.eigh(h)
        ph = np.exp(1j * eps * lam)
        out[s:e] = np.einsum("nij,nj,nkj->nik", vec, ph, vec.conj())
    return out


def gauge_field(dims, kind: str, seed: int, eps: float = 0.3) -> np.ndarray:
    """Seeded gauge field of shape (4, Lt, Lz, Ly, Lx, 3, 3).

    kind: "haar" (Haar-random SU(3) per link), "near_identity" (exp(i eps H)),
    or "unit" (all links the identity: the free field).
    """
    shp = lattice_shape(dims)
    n = 4 * int(np.prod(shp))
    if kind == "unit":
        u = np.zeros((n, 3, 3), dtype=np.complex128)
        u[:, 0, 0] = u[:, 1, 1] = u[:, 2, 2] = 1.0
    elif kind == "haar":
        u = haar_su3(n, np.random.default_rng(seed))
    elif kind == "near_identity":
        u = near_identity_su3(n, eps, np.random.default_rng(seed))
    else:
        raise ValueError(f"unknown gauge field kind {kind!r}")
    return u.reshape((4,) + shp + (3, 3))


def gaussian_spinor(dims, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Gaussian source: every complex component (N(0,1) + i N(0,1)) / sqrt(2).

    Shape (Lt, Lz, Ly, Lx, 4, 3), or (nrhs, Lt, Lz, Ly, Lx, 4, 3) if nrhs is
    given.
    """
    shp = lattice_shape(dims) + (4, 3)
    if nrhs is not None:
        shp = (int(nrhs),) + shp
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(shp)
    im = rng.standard_normal(shp)
    return (re + 1j * im) / np.sqrt(2.0)


def gaussian_colour(dims, seed: int) -> np.ndarray:
    """Gaussian colour vector field, shape (Lt, Lz, Ly, Lx, 3), every complex
    component (N(0,1) + i N(0,1)) / sqrt(2)."""
    shp = lattice_shape(dims) + (3,)
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(shp)
    im = rng.standard_normal(shp)
    return (re + 1j * im) / np.sqrt(2.0)


def point_sources(dims, site=(0, 0, 0, 0)) -> np.ndarray:
    """The 12 point sources delta_{x,site} delta_{spin,s} delta_{colour,c}.

    Shape (12, Lt, Lz, Ly, Lx, 4, 3); source k = 3*s + c. ``site`` is given
    as (x, y, z, t).
    """
    shp = lattice_shape(dims)
    b = np.zeros((12,) + shp + (4, 3), dtype=np.complex128)
    x, y, z, t = site
    for s in range(4):
        for c in range(3):
            b[3 * s + c, t, z, y, x, s, c] = 1.0
    return b


def random_gauge_rotation(dims, seed: int) -> np.ndarray:
    """Haar-random SU(3) matrix per site, shape (Lt, Lz, Ly, Lx, 3, 3)."""
    shp = lattice_shape(dims)
    g = haar_su3(int(np.prod(shp)), np.random.default_rng(seed))
    return g.reshape(shp + (3, 3))


__all__.append("random_gauge_rotation")
