"""Wilson-Dirac operator, FP64, written out from its definition.

TEST INFRASTRUCTURE ONLY (see the package header).

The paper (Sec. 1; Fig. 1 caption) names the operator: a stencil on a 4D
grid whose entries are 3x3 complex colour matrices U acting on 12-component
complex spinors psi, and refers to the lattice-QCD textbook of Gattringer and
Lang for its definition. That definition, with lattice spacing a = 1 and
periodic boundaries in all four directions, is

    (D psi)(x) = (m + 4) psi(x)
                 - 1/2 sum_{mu=0..3} [ (1 - gamma_mu) U_mu(x) psi(x + mu)
                                     + (1 + gamma_mu) U_mu(x - mu)^dagger psi(x - mu) ]

equivalently D = (1 / 2 kappa)(1 - kappa H) with kappa = 1 / (2 m + 8).
Gamma matrices: the Euclidean chiral basis of the same textbook,
gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] (k = 1, 2, 3 -> mu = 0, 1, 2) and
gamma_4 = [[0, 1], [1, 0]] (mu = 3, time), gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4.

Array layout: U (4, Lt, Lz, Ly, Lx, 3, 3); psi (Lt, Lz, Ly, Lx, 4, 3).
Direction mu = 0, 1, 2, 3 (x, y, z, t) lives on numpy axis 3 - mu of a site
array. On a direction of extent 2, x + mu and x - mu are the same site and
both hops add there.
"""
from __future__ import annotations

import numpy as np

_I2 = np.eye(2, dtype=np.complex128)
_Z2 = np.zeros((2, 2), dtype=np.complex128)
_SIGMA = [
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
]


def _chiral_gammas():
    g = []
    for k in range(3):
        g.append(np.block([[_Z2, -1j * _SIGMA[k]], [1j * _SIGMA[k], _Z2]]))
    g.append(np.block([[_Z2, _I2], [_I2, _Z2]]))
    return np.array(g)


#: gamma_mu for mu = 0..3 (x, y, z, t), shape (4, 4, 4).
GAMMA = _chiral_gammas()
#: gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4.
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]

_ID4 = np.eye(4, dtype=np.complex128)


def _axis(mu: int) -> int:
    return 3 - mu


def _colour(Umu: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """Colour matrix times spinor at every site: (U psi)_{s,i} = sum_j U_ij psi_{s,j}."""
    return np.matmul(psi, np.swapaxes(Umu, -1, -2))


def _colour_dag(Umu: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(U^dagger psi)_{s,i} = sum_j conj(U_ji) psi_{s,j}."""
    return np.matmul(psi, Umu.conj())


def _spin(G: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """4x4 spin matrix applied at every site."""
    return np.matmul(G, psi)


def _apply(U, psi, mass, gsign):
    out = (mass + 4.0) * psi
    for mu in range(4):
        ax = _axis(mu)
        fwd = _colour(U[mu], np.roll(psi, -1, axis=ax))          # U_mu(x) psi(x+mu)
        bwd = np.roll(_colour_dag(U[mu], psi), 1, axis=ax)       # U_mu(x-mu)^+ psi(x-mu)
        pm = _ID4 - gsign * GAMMA[mu]
        pp = _ID4 + gsign * GAMMA[mu]
        out = out - 0.5 * (_spin(pm, fwd) + _spin(pp, bwd))
    return out


def wilson_D(U: np.ndarray, psi: np.ndarray, mass: float) -> np.ndarray:
    """D psi by the definition above (all sites at once, periodic wrap by roll)."""
    return _apply(U, psi, mass, 1.0)


def wilson_Ddag(U: np.ndarray, psi: np.ndarray, mass: float) -> np.ndarray:
    """D^dagger psi: the same stencil with every gamma_mu replaced by -gamma_mu.

    Follows from transposing the hop blocks of D: the block of D from x to
    x + mu is -1/2 (1 - gamma_mu) U_mu(x); its conjugate transpose sits at
    (x + mu, x) and equals -1/2 (1 - gamma_mu) U_mu(x)^dagger.
    """
    return _apply(U, psi, mass, -1.0)


def normal_op(U: np.ndarray, psi: np.ndarray, mass: float) -> np.ndarray:
    """D^dagger D psi."""
    return wilson_Ddag(U, wilson_D(U, psi, mass), mass)


# ---------------------------------------------------------------------------
# Dense assembly (tiny lattices only) -- blockwise, straight from the formula.
# ---------------------------------------------------------------------------

def site_index(coords, dims) -> int:
    """Linear site index of (x, y, z, t) in a lattice (Lx, Ly, Lz, Lt), x fastest."""
    x, y, z, t = coords
    lx, ly, lz, lt = dims
    return ((t * lz + z) * ly + y) * lx + x


def _all_sites(dims):
    lx, ly, lz, lt = dims
    for t in range(lt):
        for z in range(lz):
            for y in range(ly):
                for x in range(lx):
                    yield (x, y, z, t)


def _shift(coords, mu, step, dims):
    c = list(coords)
    c[mu] = (c[mu] + step) % dims[mu]
    return tuple(c)


def _link(U, coords, mu):
    x, y, z, t = coords
    return U[mu, t, z, y, x]


def dense_D(U: np.ndarray, mass: float, dims) -> np.ndarray:
    """The (12V x 12V) matrix of D, assembled block by block.

    Row/column index = 12 * site + 3 * spin + colour, the same order as
    ``psi.reshape(-1)``. Each block of a hop is the Kronecker product of the
    4x4 spin projector and the 3x3 link; blocks that land on the same entry
    (directions of extent 2) are summed.
    """
    dims = tuple(int(d) for d in dims)
    V = int(np.prod(dims))
    M = np.zeros((12 * V, 12 * V), dtype=np.complex128)
    for c in _all_sites(dims):
        i = site_index(c, dims)
        M[12 * i:12 * i + 12, 12 * i:12 * i + 12] += (mass + 4.0) * np.eye(12)
        for mu in range(4):
            fwd = _shift(c, mu, +1, dims)
            bwd = _shift(c, mu, -1, dims)
            jf = site_index(fwd, dims)
            jb = site_index(bwd, dims)
            M[12 * i:12 * i + 12, 12 * jf:12 * jf + 12] += -0.5 * np.kron(_ID4 - GAMMA[mu], _link(U, c, mu))
            M[12 * i:12 * i + 12, 12 * jb:12 * jb + 12] += -0.5 * np.kron(
                _ID4 + GAMMA[mu], _link(U, bwd, mu).conj().T)
    return M


# ---------------------------------------------------------------------------
# Site-local evaluation, for sampled checks of full-size results.
# ---------------------------------------------------------------------------

def _psi_at(psi, c):
    x, y, z, t = c
    return psi[t, z, y, x]


def _D_one_site(U, psi, mass, c, dims, gsign):
    out = (mass + 4.0) * _psi_at(psi, c)
    for mu in range(4):
        fwd = _shift(c, mu, +1, dims)
        bwd = _shift(c, mu, -1, dims)
        a = _psi_at(psi, fwd) @ _link(U, c, mu).T
        b = _psi_at(psi, bwd) @ _link(U, bwd, mu).conj()
        out = out - 0.5 * ((_ID4 - gsign * GAMMA[mu]) @ a + (_ID4 + gsign * GAMMA[mu]) @ b)
    return out


def wilson_D_sites(U, psi, mass, sites, dagger: bool = False) -> np.ndarray:
    """(D psi)(x) (or D^dagger) at the listed sites (x, y, z, t); shape (n, 4, 3)."""
    dims = (psi.shape[3], psi.shape[2], psi.shape[1], psi.shape[0])
    g = -1.0 if dagger else 1.0
    return np.array([_D_one_site(U, psi, mass, tuple(c), dims, g) for c in sites])


def normal_op_sites(U, psi, mass, sites) -> np.ndarray:
    """(D^dagger D psi)(x) at the listed sites, from D psi on their neighbourhoods."""
    dims = (psi.shape[3], psi.shape[2], psi.shape[1], psi.shape[0])
    out = []
    for c in sites:
        c = tuple(c)
        need = {c}
        for mu in range(4):
            need.add(_shift(c, mu, +1, dims))
            need.add(_shift(c, mu, -1, dims))
        dpsi = {}
        for n in need:
            dpsi[n] = _D_one_site(U, psi, mass, n, dims, 1.0)
        acc = (mass + 4.0) * dpsi[c]
        for mu in range(4):
            fwd = _shift(c, mu, +1, dims)
            bwd = _shift(c, mu, -1, dims)
            a = dpsi[fwd] @ _link(U, c, mu).T
            b = dpsi[bwd] @ _link(U, bwd, mu).conj()
            acc = acc - 0.5 * ((_ID4 + GAMMA[mu]) @ a + (_ID4 - GAMMA[mu]) @ b)
        out.append(acc)
    return np.array(out)
