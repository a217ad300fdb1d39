"""Pin checks for the CPU oracle: each returns an error measure that is at
rounding level for a correct oracle.

They compare the oracle with facts that do not come from the oracle's own
formula: the Euclidean chiral gamma basis typed out as a table, the
free-field operator in momentum space, gauge and translation covariance,
the adjoint identity against an explicit dense transpose, norm bounds,
direct dense solves and central finite differences. The same checks are run
against deliberately broken copies of the oracle (``test_oracle_mutations``)
to show that each plausible mistake trips at least one of them.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

import fieldgen
import oracle
from oracle import dirac

# The Euclidean chiral basis (Gattringer & Lang, App. A), typed as a table.
# Rows are spin indices 0..3; entries are complex.
I = 1j
CHIRAL_TABLE = np.array([
    [[0, 0, 0, -I], [0, 0, -I, 0], [0, I, 0, 0], [I, 0, 0, 0]],     # gamma_1 (x)
    [[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]],     # gamma_2 (y)
    [[0, 0, -I, 0], [0, 0, 0, I], [I, 0, 0, 0], [0, -I, 0, 0]],     # gamma_3 (z)
    [[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]],       # gamma_4 (t)
], dtype=np.complex128)


def rel(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    den = max(np.linalg.norm(b.ravel()), 1e-300)
    return float(np.linalg.norm((a - b).ravel()) / den)


def dims_shape(dims):
    return fieldgen.lattice_shape(dims)


# ----------------------------------------------------------------- gammas

def clifford_error() -> float:
    g = dirac.GAMMA
    err = 0.0
    for a in range(4):
        for b in range(4):
            ac = g[a] @ g[b] + g[b] @ g[a]
            err = max(err, np.abs(ac - 2.0 * (a == b) * np.eye(4)).max())
    return float(err)


def basis_table_error() -> float:
    return float(np.abs(dirac.GAMMA - CHIRAL_TABLE).max())


# ------------------------------------------------------- momentum space

def free_D_momentum(p, mass, sign=1.0):
    """4x4 spin matrix of the free Wilson operator at momentum p (tested form):
    m + sum_mu (1 - cos p_mu) + i sign sum_mu gamma_mu sin p_mu, with the gammas
    taken from the typed table."""
    m = (mass + sum(1.0 - math.cos(q) for q in p)) * np.eye(4, dtype=np.complex128)
    for mu in range(4):
        m = m + 1j * sign * CHIRAL_TABLE[mu] * math.sin(p[mu])
    return m


def plane_wave(dims, n, u):
    """psi(x) = exp(i p.x) u with p_mu = 2 pi n_mu / L_mu; u is (4, 3)."""
    lx, ly, lz, lt = dims
    p = [2 * math.pi * n[mu] / dims[mu] for mu in range(4)]
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    return phase[..., None, None] * u[None, None, None, None], p, phase


def plane_wave_error(dims, n, mass, seed=5, dagger=False) -> float:
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    psi, p, phase = plane_wave(dims, n, u)
    U = fieldgen.gauge_field(dims, "unit", 0)
    out = oracle.wilson_Ddag(U, psi, mass) if dagger else oracle.wilson_D(U, psi, mass)
    exp = phase[..., None, None] * (free_D_momentum(p, mass, -1.0 if dagger else 1.0) @ u)[None, None, None, None]
    return rel(out, exp)


def free_spectrum_closed_form(dims, mass):
    vals = []
    for n in itertools.product(*[range(L) for L in dims]):
        p = [2 * math.pi * n[mu] / dims[mu] for mu in range(4)]
        a = mass + sum(1 - math.cos(q) for q in p)
        b = sum(math.sin(q) ** 2 for q in p)
        vals.extend([a * a + b] * 12)
    return np.sort(np.array(vals))


def free_spectrum_error(dims, mass) -> float:
    U = fieldgen.gauge_field(dims, "unit", 0)
    D = oracle.dense_D(U, mass, dims)
    ev = np.sort(np.linalg.eigvalsh(D.conj().T @ D))
    return float(np.abs(ev - free_spectrum_closed_form(dims, mass)).max())


# ------------------------------------------------------------ structure

def dense_vs_apply_error(dims, mass, seed=1, kind="haar") -> float:
    U = fieldgen.gauge_field(dims, kind, seed)
    psi = fieldgen.gaussian_spinor(dims, seed + 1)
    D = oracle.dense_D(U, mass, dims)
    return rel(oracle.wilson_D(U, psi, mass).reshape(-1), D @ psi.reshape(-1))


def adjoint_dense_error(dims, mass, seed=1) -> float:
    """D^dagger applied by the oracle vs the explicit conjugate transpose of dense D."""
    U = fieldgen.gauge_field(dims, "haar", seed)
    psi = fieldgen.gaussian_spinor(dims, seed + 1)
    D = oracle.dense_D(U, mass, dims)
    return rel(oracle.wilson_Ddag(U, psi, mass).reshape(-1), D.conj().T @ psi.reshape(-1))


def adjoint_identity_error(dims, mass, seed=1) -> float:
    U = fieldgen.gauge_field(dims, "haar", seed)
    a = fieldgen.gaussian_spinor(dims, seed + 1)
    b = fieldgen.gaussian_spinor(dims, seed + 2)
    lhs = np.vdot(a, oracle.wilson_D(U, b, mass))
    rhs = np.vdot(oracle.wilson_Ddag(U, a, mass), b)
    return float(abs(lhs - rhs) / abs(lhs))


def gamma5_hermiticity_error(dims, mass, seed=1) -> float:
    U = fieldgen.gauge_field(dims, "haar", seed)
    psi = fieldgen.gaussian_spinor(dims, seed + 1)
    g5 = np.diag([1, 1, -1, -1]).astype(np.complex128)       # chiral gamma_5
    lhs = np.matmul(g5, oracle.wilson_D(U, np.matmul(g5, psi), mass))
    return rel(lhs, oracle.wilson_Ddag(U, psi, mass))


def gauge_transform(U, G):
    """U^G_mu(x) = G(x) U_mu(x) G(x + mu)^dagger."""
    out = np.empty_like(U)
    for mu in range(4):
        Gf = np.roll(G, -1, axis=3 - mu)
        out[mu] = G @ U[mu] @ np.swapaxes(Gf.conj(), -1, -2)
    return out


def rotate_spinor(G, psi):
    return np.matmul(psi, np.swapaxes(G, -1, -2))


def gauge_covariance_error(dims, mass, seed=1, dagger=False) -> float:
    U = fieldgen.gauge_field(dims, "haar", seed)
    psi = fieldgen.gaussian_spinor(dims, seed + 1)
    G = fieldgen.random_gauge_rotation(dims, seed + 2)
    op = oracle.wilson_Ddag if dagger else oracle.wilson_D
    lhs = op(gauge_transform(U, G), rotate_spinor(G, psi), mass)
    rhs = rotate_spinor(G, op(U, psi, mass))
    return rel(lhs, rhs)


def pure_gauge_plane_wave_error(dims, n, mass, seed=3) -> float:
    """Links G(x) G(x+mu)^dagger: D[U](G psi_pw) must equal G (D_free psi_pw)."""
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    psi, p, phase = plane_wave(dims, n, u)
    G = fieldgen.random_gauge_rotation(dims, seed + 1)
    U = gauge_transform(fieldgen.gauge_field(dims, "unit", 0), G)
    out = oracle.wilson_D(U, rotate_spinor(G, psi), mass)
    exp = rotate_spinor(G, phase[..., None, None] * (free_D_momentum(p, mass) @ u)[None, None, None, None])
    return rel(out, exp)


def translation_error(dims, mass, shift, seed=1) -> float:
    U = fieldgen.gauge_field(dims, "haar", seed)
    psi = fieldgen.gaussian_spinor(dims, seed + 1)
    axes = (3, 2, 1, 0)
    Us = U
    ps = psi
    for mu in range(4):
        Us = np.roll(Us, shift[mu], axis=axes[mu] + 1)
        ps = np.roll(ps, shift[mu], axis=axes[mu])
    out = oracle.wilson_D(U, psi, mass)
    for mu in range(4):
        out = np.roll(out, shift[mu], axis=axes[mu])
    return rel(oracle.wilson_D(Us, ps, mass), out)


def bounds_margins(dims, mass, seed=1):
    """(Re<psi,D psi> - m||psi||^2, (m+8)||psi|| - ||D psi||) normalised; both >= 0."""
    U = fieldgen.gauge_field(dims, "haar", seed)
    psi = fieldgen.gaussian_spinor(dims, seed + 1)
    n2 = float(np.vdot(psi, psi).real)
    dpsi = oracle.wilson_D(U, psi, mass)
    low = (float(np.vdot(psi, dpsi).real) - mass * n2) / n2
    high = ((mass + 8.0) * math.sqrt(n2) - float(np.linalg.norm(dpsi))) / math.sqrt(n2)
    return low, high


# -------------------------------------------------------------- solver

def dense_solve_error(dims, mass, seed=1, kind="haar", tol=1e-12) -> float:
    U = fieldgen.gauge_field(dims, kind, seed)
    b = fieldgen.gaussian_spinor(dims, seed + 1)
    D = oracle.dense_D(U, mass, dims)
    xd = np.linalg.solve(D, b.reshape(-1)).reshape(b.shape)
    x, info = oracle.cgnr(U, b, mass, tol=tol, max_iter=5000)
    return rel(x, xd)


def plane_wave_solve_error(dims, n, mass, seed=4, tol=1e-12) -> float:
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    b, p, phase = plane_wave(dims, n, u)
    U = fieldgen.gauge_field(dims, "unit", 0)
    x, info = oracle.cgnr(U, b, mass, tol=tol)
    exp = phase[..., None, None] * np.linalg.solve(free_D_momentum(p, mass), u)[None, None, None, None]
    return rel(x, exp)


def finite_termination_residual(mass=0.1, seed=3) -> float:
    """Free field on 2^4: D^+D has 5 distinct eigenvalues, so CG is exact after
    5 steps. Returns the true relative residual after exactly 5 steps."""
    dims = (2, 2, 2, 2)
    U = fieldgen.gauge_field(dims, "unit", 0)
    b = fieldgen.gaussian_spinor(dims, seed)
    x, info = oracle.cgnr(U, b, mass, tol=1e-300, max_iter=5)
    return oracle.true_relative_residual(U, x, b, mass)


def residual_checker_errors(dims, mass, rhs="source", seed=21, c=0.5, eps=1e-3) -> dict:
    """Errors of ``oracle.true_relative_residual`` against what linearity fixes.

    With x_d the dense direct solution of the normal system (D^+ D x_d = b',
    b' = D^+ b or b) the residual of c x_d is (1 - c) b', so the relative
    residual is exactly |1 - c|; x = 0 gives exactly 1; and x_d + eps v
    leaves the residual -eps D^+ D v, whose norm comes from the dense matrix
    (not from the stencil the checker uses).
    """
    U = fieldgen.gauge_field(dims, "haar", seed)
    b = fieldgen.gaussian_spinor(dims, seed + 1)
    v = fieldgen.gaussian_spinor(dims, seed + 2)
    D = oracle.dense_D(U, mass, dims)
    M = D.conj().T @ D
    bv = b.reshape(-1)
    bp = D.conj().T @ bv if rhs == "source" else bv
    xd = np.linalg.solve(M, bp).reshape(b.shape)
    f = oracle.true_relative_residual
    scaled = f(U, c * xd, b, mass, rhs=rhs)
    zero = f(U, np.zeros_like(b), b, mass, rhs=rhs)
    expect = eps * np.linalg.norm(M @ v.reshape(-1)) / np.linalg.norm(bp)
    pert = f(U, xd + eps * v, b, mass, rhs=rhs)
    return {
        "scaled": abs(scaled - abs(1.0 - c)),
        "zero": abs(zero - 1.0),
        "perturbed": abs(pert - expect) / expect,
    }


# --------------------------------------------------------------- force

def loss_dense(D, phi):
    """L = Re phi^dagger (D^dagger D)^{-1} phi = ||D^{-dagger} phi||^2, via two dense solves."""
    y = np.linalg.solve(D.conj().T, phi)
    return float(math.fsum((y.conj() * y).real))


def force_fd_errors(dims, mass, seed=7, h=1e-6, nentries=24):
    """Central finite differences of L = Re phi^+ M^{-1} phi against the oracle's grad_U.

    Returns the largest absolute and relative deviation over the sampled
    (link, entry, real/imag) directions."""
    U = fieldgen.gauge_field(dims, "haar", seed)
    phi = fieldgen.gaussian_spinor(dims, seed + 1)
    # upstream g = phi: grad_U = G(D chi, chi) + G(D chi, chi) is the full gradient of L
    chi, grad, gphi = oracle.solve_gradients(U, phi, phi, mass)
    rng = np.random.default_rng(seed + 2)
    worst_abs = 0.0
    scale = np.abs(grad).max()
    for _ in range(nentries):
        idx = tuple(int(rng.integers(0, s)) for s in U.shape)
        for unit in (1.0, 1j):
            Up = U.copy()
            Um = U.copy()
            Up[idx] += h * unit
            Um[idx] -= h * unit
            fd = (loss_dense(oracle.dense_D(Up, mass, dims), phi.reshape(-1))
                  - loss_dense(oracle.dense_D(Um, mass, dims), phi.reshape(-1))) / (2 * h)
            an = grad[idx].real if unit == 1.0 else grad[idx].imag
            worst_abs = max(worst_abs, abs(fd - an))
    return worst_abs, worst_abs / scale


def force_direction_error(dims, mass, seed=8, h=1e-6):
    """d/dt L(U + t V) at t = 0 by central differences vs Re<grad, V>, for a random
    complex direction V and a general upstream gradient (L = Re <w, chi> + Re phi^+ chi)."""
    U = fieldgen.gauge_field(dims, "haar", seed)
    phi = fieldgen.gaussian_spinor(dims, seed + 1)
    w = fieldgen.gaussian_spinor(dims, seed + 2)
    V = (np.random.default_rng(seed + 3).standard_normal(U.shape)
         + 1j * np.random.default_rng(seed + 4).standard_normal(U.shape))
    g = w + phi
    chi, gU, gphi = oracle.solve_gradients(U, phi, g, mass)

    def L(Ut):
        D = oracle.dense_D(Ut, mass, dims)
        M = D.conj().T @ D
        c = np.linalg.solve(M, phi.reshape(-1))
        return float(np.vdot(g.reshape(-1), c).real)

    fd = (L(U + h * V) - L(U - h * V)) / (2 * h)
    an = float(np.vdot(gU, V).real)
    return abs(fd - an) / abs(an)


def force_gauge_covariance_error(dims, mass, seed=9):
    """grad_U transforms like a link: grad[U^G, G phi]_mu(x) = G(x) grad[U, phi]_mu(x) G(x+mu)^+."""
    U = fieldgen.gauge_field(dims, "haar", seed)
    phi = fieldgen.gaussian_spinor(dims, seed + 1)
    G = fieldgen.random_gauge_rotation(dims, seed + 2)
    _, g0, _ = oracle.solve_gradients(U, phi, phi, mass)
    phiG = rotate_spinor(G, phi)
    _, g1, _ = oracle.solve_gradients(gauge_transform(U, G), phiG, phiG, mass)
    return rel(g1, gauge_transform(g0, G))
