"""Pins of the gauge-covariant Laplacian oracle (CPU only), and planted mistakes.

The Laplacian L = (m2 + 8) - sum_mu [U_mu(x) T_mu + T_mu^+ U_mu(x)^+] is
pinned against facts that do not come from retyping its formula: the free
field's plane waves and its closed-form spectrum, Hermiticity through inner
products, the spectrum bounds that unitary links imply, gauge covariance, a
library dense solve, and finite termination of CG on a spectrum with five
distinct eigenvalues. Each planted mistake must trip at least one pin.
"""
import itertools

import numpy as np
import pytest

import fieldgen
from oracle import laplace as lap

THRESH = 1e-8


def _unit_links(dims):
    U = np.zeros((4,) + fieldgen.lattice_shape(dims) + (3, 3), dtype=np.complex128)
    U[...] = np.eye(3)
    return U


def _colour_field(dims, seed):
    rng = np.random.default_rng(seed)
    shape = fieldgen.lattice_shape(dims) + (3,)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


def _coords(dims):
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    return x, y, z, t


# ---------------------------------------------------------------- pin checks

def plane_wave_error(dims, n, m2, apply=None):
    """Free field: psi = exp(i p.x) v is an eigenvector with eigenvalue
    m2 + sum_mu 4 sin^2(p_mu / 2), p_mu = 2 pi n_mu / L_mu."""
    apply = apply or lap.laplace
    x, y, z, t = _coords(dims)
    p = [2 * np.pi * n[mu] / dims[mu] for mu in range(4)]
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    v = np.array([1.0, -0.5j, 0.25 + 0.75j])
    psi = phase[..., None] * v
    lam = m2 + sum(4 * np.sin(pm / 2) ** 2 for pm in p)
    out = apply(_unit_links(dims), psi, m2)
    return float(np.linalg.norm(out - lam * psi) / np.linalg.norm(lam * psi))


def free_dense_spectrum_error(dims, m2, dense=None):
    """Eigenvalues of the free dense matrix = the closed-form multiset (x3 colours)."""
    dense = dense or lap.dense_laplace
    A = dense(_unit_links(dims), m2, dims)
    ev = np.sort(np.linalg.eigvalsh(A))
    ref = []
    for n in itertools.product(*[range(L) for L in dims]):
        ref += [m2 + sum(4 * np.sin(np.pi * n[mu] / dims[mu]) ** 2 for mu in range(4))] * 3
    return float(np.abs(ev - np.sort(ref)).max())


def hermiticity_error(dims, m2, apply=None):
    """<a, L b> = <L a, b> for random a, b on Haar links."""
    apply = apply or lap.laplace
    U = fieldgen.gauge_field(dims, "haar", 11)
    a, b = _colour_field(dims, 12), _colour_field(dims, 13)
    lhs = np.vdot(a, apply(U, b, m2))
    rhs = np.vdot(apply(U, a, m2), b)
    return float(abs(lhs - rhs) / abs(lhs))


def spectrum_bound_error(dims, m2, dense=None):
    """Unitary links: ||H|| <= 8, so the spectrum lies in [m2, m2 + 16]; also
    L = L^+ exactly. Returns how far outside (or how non-Hermitian) it is."""
    dense = dense or lap.dense_laplace
    A = dense(fieldgen.gauge_field(dims, "haar", 21), m2, dims)
    herm = float(np.abs(A - A.conj().T).max())
    ev = np.linalg.eigvalsh(A)
    outside = max(0.0, m2 - ev.min(), ev.max() - (m2 + 16.0))
    return max(herm, outside)


def gauge_covariance_error(dims, m2, apply=None):
    """U'_mu(x) = g(x) U_mu(x) g(x + mu)^+, psi' = g psi  =>  L[U'] psi' = g L[U] psi."""
    apply = apply or lap.laplace
    U = fieldgen.gauge_field(dims, "haar", 31)
    g = fieldgen.random_gauge_rotation(dims, 32)
    psi = _colour_field(dims, 33)
    Ug = np.empty_like(U)
    for mu in range(4):
        gf = np.roll(g, -1, axis=3 - mu)
        Ug[mu] = g @ U[mu] @ np.swapaxes(gf.conj(), -1, -2)
    lhs = apply(Ug, np.einsum("...ij,...j->...i", g, psi), m2)
    rhs = np.einsum("...ij,...j->...i", g, apply(U, psi, m2))
    return float(np.linalg.norm(lhs - rhs) / np.linalg.norm(rhs))


def dense_vs_apply_error(dims, m2, apply=None, dense=None):
    apply = apply or lap.laplace
    dense = dense or lap.dense_laplace
    U = fieldgen.gauge_field(dims, "haar", 41)
    psi = _colour_field(dims, 42)
    out = apply(U, psi, m2).reshape(-1)
    ref = dense(U, m2, dims) @ psi.reshape(-1)
    return float(np.linalg.norm(out - ref) / np.linalg.norm(ref))


def cg_vs_dense_solve_error(dims, m2, solver=None):
    """CG from the oracle against numpy's dense solve of the assembled matrix."""
    solver = solver or lap.cg
    U = fieldgen.gauge_field(dims, "haar", 51)
    b = _colour_field(dims, 52)
    x, info = solver(U, b, m2, tol=1e-13, max_iter=2000)
    xd = np.linalg.solve(lap.dense_laplace(U, m2, dims), b.reshape(-1)).reshape(b.shape)
    return float(np.linalg.norm(x - xd) / np.linalg.norm(xd))


def finite_termination_residual(m2, solver=None):
    """Free 2^4 lattice: the spectrum has 5 distinct values (m2 + 4k, k = 0..4),
    so exact CG ends after at most 5 steps."""
    solver = solver or lap.cg
    dims = (2, 2, 2, 2)
    b = _colour_field(dims, 61)
    x, info = solver(_unit_links(dims), b, m2, tol=1e-30, max_iter=5, history=True)
    return float(info["history"][4]) if len(info["history"]) >= 5 else 0.0


# ----------------------------------------------------------------- the pins

def test_plane_waves():
    for n in [(0, 0, 0, 0), (1, 2, 3, 5), (2, 0, 7, 1), (3, 5, 4, 9)]:
        assert plane_wave_error((4, 6, 8, 10), n, 0.3) < 1e-13


def test_free_dense_spectrum():
    assert free_dense_spectrum_error((2, 2, 2, 4), 0.3) < 1e-12
    assert free_dense_spectrum_error((3, 2, 2, 3), 0.05) < 1e-12


def test_hermitian_and_bounded():
    assert hermiticity_error((4, 4, 2, 4), 0.2) < 1e-13
    assert spectrum_bound_error((2, 2, 3, 2), 0.2) < 1e-12


def test_gauge_covariance():
    assert gauge_covariance_error((4, 4, 2, 4), 0.2) < 1e-13


def test_dense_matches_apply():
    assert dense_vs_apply_error((3, 2, 4, 2), 0.2) < 1e-14


def test_sites_match_dense_rows():
    # the site-by-site form against the dense matrix (assembled block by block
    # and pinned by the spectrum tests above), every site of a small lattice
    dims = (3, 2, 4, 2)
    U = fieldgen.gauge_field(dims, "haar", 91)
    psi = _colour_field(dims, 92)
    ref = (lap.dense_laplace(U, 0.7, dims) @ psi.reshape(-1)).reshape(psi.shape)
    sites = list(itertools.product(range(3), range(2), range(4), range(2)))
    loc = lap.laplace_sites(U, psi, 0.7, sites)
    for k, (x, y, z, t) in enumerate(sites):
        assert np.abs(loc[k] - ref[t, z, y, x]).max() < 1e-13


def test_sites_free_plane_wave():
    # free field: at any site L psi = lambda psi for a plane wave
    dims = (4, 6, 8, 10)
    x, y, z, t = _coords(dims)
    n = (1, 2, 3, 5)
    p = [2 * np.pi * n[mu] / dims[mu] for mu in range(4)]
    psi = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))[..., None] * np.array([1.0, 2j, -0.5])
    lam = 0.3 + sum(4 * np.sin(pm / 2) ** 2 for pm in p)
    sites = [(0, 0, 0, 0), (3, 5, 7, 9), (2, 1, 4, 6)]
    loc = lap.laplace_sites(_unit_links(dims), psi, 0.3, sites)
    for k, (a, b_, c, d) in enumerate(sites):
        assert np.abs(loc[k] - lam * psi[d, c, b_, a]).max() < 1e-13


def test_cg_matches_dense_solve():
    assert cg_vs_dense_solve_error((2, 2, 3, 2), 0.05) < 1e-10
    assert cg_vs_dense_solve_error((4, 2, 2, 2), 0.5) < 1e-11


def test_cg_finite_termination():
    assert finite_termination_residual(0.3) < 1e-10


def test_cg_reports_true_residual():
    dims = (4, 4, 2, 4)
    U = fieldgen.gauge_field(dims, "haar", 71)
    b = _colour_field(dims, 72)
    x, info = lap.cg(U, b, 0.1, tol=1e-10)
    assert info["true_rel_res"] <= 1e-10 * (1 + 1e-3)
    assert abs(info["true_rel_res"] - lap.true_relative_residual(U, x, b, 0.1)) < 1e-15


def residual_checker_errors(dims, m2, seed=81, c=0.5, eps=1e-3, checker=None) -> dict:
    """``lap.true_relative_residual`` against linearity: with x_d the dense
    solution of L x = b, c x_d leaves (1 - c) b (relative residual |1 - c|),
    x = 0 leaves b (exactly 1), and x_d + eps v leaves -eps L v, whose norm
    comes from the dense matrix."""
    f = checker or lap.true_relative_residual
    U = fieldgen.gauge_field(dims, "haar", seed)
    b = _colour_field(dims, seed + 1)
    v = _colour_field(dims, seed + 2)
    A = lap.dense_laplace(U, m2, dims)
    xd = np.linalg.solve(A, b.reshape(-1)).reshape(b.shape)
    expect = eps * np.linalg.norm(A @ v.reshape(-1)) / np.linalg.norm(b)
    return {
        "scaled": abs(f(U, c * xd, b, m2) - abs(1.0 - c)),
        "zero": abs(f(U, np.zeros_like(b), b, m2) - 1.0),
        "perturbed": abs(f(U, xd + eps * v, b, m2) - expect) / expect,
    }


@pytest.mark.parametrize("dims,m2", [((2, 2, 2, 2), 0.1), ((3, 2, 4, 2), 0.5)])
def test_true_residual_checker(dims, m2):
    errs = residual_checker_errors(dims, m2)
    assert errs["scaled"] < 1e-13, errs
    assert errs["zero"] < 1e-14, errs
    assert errs["perturbed"] < 1e-6, errs


# ------------------------------------------------------- planted mistakes

def _mutated_laplace(kind):
    def apply(U, psi, m2):
        diag = {"diag_4": m2 + 4.0, "diag_no_m2": 8.0}.get(kind, m2 + 8.0)
        out = diag * psi
        for mu in range(4):
            ax = mu if kind == "axis_mu" else 3 - mu
            Uf = np.swapaxes(U[mu], -1, -2) if kind == "fwd_transposed" else U[mu]
            step = +1 if kind == "fwd_roll_swapped" else -1
            fwd = np.einsum("...ij,...j->...i", Uf, np.roll(psi, step, axis=ax))
            if kind == "bwd_no_dagger":
                bwd = np.roll(np.einsum("...ij,...j->...i", U[mu], psi), 1, axis=ax)
            elif kind == "bwd_conj_only":
                bwd = np.roll(np.einsum("...ij,...j->...i", U[mu].conj(), psi), 1, axis=ax)
            elif kind == "bwd_link_unshifted":
                bwd = np.einsum("...ji,...j->...i", U[mu].conj(), np.roll(psi, 1, axis=ax))
            else:
                bwd = np.roll(np.einsum("...ji,...j->...i", U[mu].conj(), psi), 1, axis=ax)
            sb = -1.0 if kind == "bwd_sign" else 1.0
            out = out - fwd - sb * bwd
        return out
    return apply


def _mutated_dense(kind):
    def dense(U, m2, dims):
        A = lap.dense_laplace(U, m2, dims)
        if kind == "dense_diag":
            A = A + 0.5 * np.eye(A.shape[0])
        elif kind == "dense_transposed":
            A = A.T.copy()
        return A
    return dense


def _mutated_cg(kind):
    def solver(U, b, m2, tol=1e-10, max_iter=10000, history=False):
        x = np.zeros_like(b)
        r = b.copy()
        p = r.copy()
        bn = np.linalg.norm(b)
        rho = np.vdot(r, r).real
        hist = []
        it = 0
        while it < max_iter and np.sqrt(rho) > tol * bn:
            t = lap.laplace(U, p, m2)
            den = np.vdot(p, p).real if kind == "alpha_pp" else np.vdot(p, t).real
            alpha = rho / den
            x = x + alpha * (r if kind == "x_with_r" else p)
            r = r - alpha * t if kind != "r_sign" else r + alpha * t
            rho_new = np.vdot(r, r).real
            it += 1
            hist.append(np.sqrt(rho_new) / bn)
            beta = rho / rho_new if kind == "beta_inverted" else rho_new / rho
            p = r + beta * p
            rho = rho_new
        info = {"iterations": it, "history": hist}
        return x, info
    return solver


def _operator_errors(apply):
    return {
        "plane": plane_wave_error((4, 6, 8, 10), (1, 2, 3, 5), 0.3, apply=apply),
        "herm": hermiticity_error((4, 4, 2, 4), 0.2, apply=apply),
        "gauge": gauge_covariance_error((4, 4, 2, 4), 0.2, apply=apply),
        "dense": dense_vs_apply_error((3, 2, 4, 2), 0.2, apply=apply),
    }


@pytest.mark.parametrize("kind", ["diag_4", "diag_no_m2", "axis_mu", "fwd_transposed", "fwd_roll_swapped",
                                  "bwd_no_dagger", "bwd_conj_only", "bwd_link_unshifted", "bwd_sign"])
def test_operator_mutation_detected(kind):
    errs = _operator_errors(_mutated_laplace(kind))
    assert any(not (e <= THRESH) for e in errs.values()), errs


@pytest.mark.parametrize("kind", ["dense_diag", "dense_transposed"])
def test_dense_mutation_detected(kind):
    d = _mutated_dense(kind)
    errs = {"spectrum": free_dense_spectrum_error((2, 2, 2, 4), 0.3, dense=d),
            "bounds": spectrum_bound_error((2, 2, 3, 2), 0.2, dense=d),
            "dense": dense_vs_apply_error((3, 2, 4, 2), 0.2, dense=d)}
    assert any(not (e <= THRESH) for e in errs.values()), errs


@pytest.mark.parametrize("kind", ["alpha_pp", "x_with_r", "r_sign", "beta_inverted"])
def test_cg_mutation_detected(kind):
    s = _mutated_cg(kind)
    with np.errstate(all="ignore"):
        try:
            e1 = cg_vs_dense_solve_error((2, 2, 3, 2), 0.05, solver=s)
        except (ZeroDivisionError, FloatingPointError):
            e1 = np.inf
        try:
            e2 = finite_termination_residual(0.3, solver=s)
        except (ZeroDivisionError, FloatingPointError):
            e2 = np.inf
    assert not (e1 <= THRESH) or not (e2 <= 1e-10), (e1, e2)


def _mutated_checker(kind):
    def true_relative_residual(U, x, b, m2):
        Lx = lap.laplace(U, x, 0.0 if kind == "m2_dropped" else m2)
        r = b + Lx if kind == "sign" else b - Lx
        r2 = np.vdot(r, r).real
        den2 = np.vdot(x, x).real if kind == "normalised_by_x" else np.vdot(b, b).real
        return float(r2 / den2) if kind == "no_sqrt" else float(np.sqrt(r2 / den2))
    return true_relative_residual


@pytest.mark.parametrize("kind", ["no_sqrt", "sign", "normalised_by_x", "m2_dropped"])
def test_true_residual_mutation_detected(kind):
    with np.errstate(all="ignore"):
        errs = residual_checker_errors((2, 2, 2, 2), 0.1, checker=_mutated_checker(kind))
    assert any(not (e <= 1e-6) for e in errs.values()), errs
