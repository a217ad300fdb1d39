"""Pins of the CPU oracle against facts that do not come from its own formula.

All CPU-only; the whole file runs in well under a minute.
"""
import math

import numpy as np
import pytest

import fieldgen
import oracle
import pins

ODD = (3, 2, 4, 2)           # non-cubic, includes extent-2 directions
SMALL = (4, 2, 2, 6)
C0 = (4, 4, 4, 4)


# ------------------------------------------------------------- gammas

def test_gamma_basis_is_the_chiral_table():
    assert pins.basis_table_error() == 0.0


def test_clifford_algebra_and_hermiticity():
    assert pins.clifford_error() < 1e-15
    for g in oracle.GAMMA:
        assert np.abs(g - g.conj().T).max() == 0.0


def test_gamma5_is_product_and_diagonal():
    assert np.abs(oracle.GAMMA5 - np.diag([1, 1, -1, -1])).max() < 1e-15


# ------------------------------------------------------ free field

def test_free_spectrum_2x2x2x2_hand_values():
    # On 2^4 every momentum component is 0 or pi, so sin p = 0 and the
    # eigenvalues of D^+D are (m + 2k)^2, k = number of pi components, each
    # with multiplicity 12 * C(4, k). With m = 0.1: 0.01, 4.41, 16.81, 37.21, 65.61.
    dims = (2, 2, 2, 2)
    U = fieldgen.gauge_field(dims, "unit", 0)
    D = oracle.dense_D(U, 0.1, dims)
    ev = np.sort(np.linalg.eigvalsh(D.conj().T @ D))
    expect = []
    for k, val in enumerate([0.01, 4.41, 16.81, 37.21, 65.61]):
        expect += [val] * (12 * math.comb(4, k))
    assert np.abs(ev - np.array(expect)).max() < 1e-12


@pytest.mark.parametrize("dims", [(2, 2, 2, 4), (2, 4, 2, 2), (3, 2, 2, 3)])
def test_free_spectrum_closed_form(dims):
    assert pins.free_spectrum_error(dims, 0.1) < 1e-12


@pytest.mark.parametrize("dagger", [False, True])
@pytest.mark.parametrize("n", [(1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1), (1, 2, 3, 5), (2, 1, 0, 3)])
def test_plane_wave_eigen(n, dagger):
    # distinct extents so that a direction/axis mix-up changes the momenta
    dims = (4, 6, 8, 10)
    assert pins.plane_wave_error(dims, n, 0.1, dagger=dagger) < 1e-13


def test_pure_gauge_plane_wave():
    assert pins.pure_gauge_plane_wave_error((4, 6, 2, 8), (1, 2, 1, 3), 0.05) < 1e-13


# -------------------------------------------------------- structure

@pytest.mark.parametrize("dims", [(2, 2, 2, 2), ODD])
def test_dense_matches_stencil(dims):
    assert pins.dense_vs_apply_error(dims, 0.1) < 1e-14


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), ODD])
def test_adjoint_against_dense_transpose(dims):
    assert pins.adjoint_dense_error(dims, 0.1) < 1e-14


@pytest.mark.parametrize("dims", [C0, SMALL])
def test_adjoint_identity(dims):
    assert pins.adjoint_identity_error(dims, 0.05) < 1e-13


@pytest.mark.parametrize("dims", [C0, ODD])
def test_gamma5_hermiticity(dims):
    assert pins.gamma5_hermiticity_error(dims, 0.1) < 1e-15


@pytest.mark.parametrize("dagger", [False, True])
@pytest.mark.parametrize("dims", [C0, ODD])
def test_gauge_covariance(dims, dagger):
    assert pins.gauge_covariance_error(dims, 0.1, dagger=dagger) < 1e-13


def test_translation_covariance():
    assert pins.translation_error((4, 6, 2, 4), 0.1, (1, 2, 1, 3)) < 1e-15


@pytest.mark.parametrize("dims", [C0, ODD])
def test_norm_bounds(dims):
    low, high = pins.bounds_margins(dims, 0.1)
    assert low >= 0.0 and high >= 0.0


def test_singular_values_within_bounds():
    dims = (2, 2, 2, 2)
    U = fieldgen.gauge_field(dims, "haar", 11)
    s = np.linalg.svd(oracle.dense_D(U, 0.1, dims), compute_uv=False)
    assert s.min() >= 0.1 - 1e-12 and s.max() <= 8.1 + 1e-12


def test_site_local_matches_full():
    dims = (4, 6, 2, 4)
    U = fieldgen.gauge_field(dims, "haar", 3)
    psi = fieldgen.gaussian_spinor(dims, 4)
    sites = [(0, 0, 0, 0), (3, 5, 1, 3), (2, 1, 0, 2), (1, 3, 1, 0)]
    full = oracle.wilson_D(U, psi, 0.1)
    fulld = oracle.wilson_Ddag(U, psi, 0.1)
    fulln = oracle.normal_op(U, psi, 0.1)
    loc = oracle.wilson_D_sites(U, psi, 0.1, sites)
    locd = oracle.wilson_D_sites(U, psi, 0.1, sites, dagger=True)
    locn = oracle.normal_op_sites(U, psi, 0.1, sites)
    for k, (x, y, z, t) in enumerate(sites):
        assert np.abs(loc[k] - full[t, z, y, x]).max() < 1e-13
        assert np.abs(locd[k] - fulld[t, z, y, x]).max() < 1e-13
        assert np.abs(locn[k] - fulln[t, z, y, x]).max() < 1e-12


# ------------------------------------------------------------ solver

def test_cgnr_matches_dense_solve_2x2x2x2():
    assert pins.dense_solve_error((2, 2, 2, 2), 0.1) < 1e-10


def test_cgnr_matches_dense_solve_odd():
    assert pins.dense_solve_error(ODD, 0.05, kind="near_identity") < 1e-10


@pytest.mark.slow
def test_cgnr_config0_matches_dense_solve():
    # 4^4 Haar links, m = 0.1, Gaussian source, stop at 1e-10 (3072 unknowns)
    dims = C0
    U = fieldgen.gauge_field(dims, "haar", 200105218)
    b = fieldgen.gaussian_spinor(dims, 200105219)
    x, info = oracle.cgnr(U, b, 0.1, tol=1e-10)
    assert info["true_rel_res"] <= 1e-10
    xd = np.linalg.solve(oracle.dense_D(U, 0.1, dims), b.reshape(-1)).reshape(b.shape)
    # error bounded by cond(D) * residual of the normal system
    assert pins.rel(x, xd) < 1e-8


@pytest.mark.parametrize("n", [(1, 0, 2, 3), (0, 0, 0, 0), (2, 1, 1, 5)])
def test_plane_wave_solution(n):
    assert pins.plane_wave_solve_error((4, 2, 4, 6), n, 0.1) < 1e-10


def test_free_field_cg_terminates_in_distinct_eigenvalues():
    # On 2^4 free field, D^+D has 5 distinct eigenvalues: CG is exact after 5 steps.
    dims = (2, 2, 2, 2)
    U = fieldgen.gauge_field(dims, "unit", 0)
    b = fieldgen.gaussian_spinor(dims, 3)
    x, info = oracle.cgnr(U, b, 0.1, tol=1e-14, max_iter=5, history=True)
    # exact after 5 steps up to rounding (cond(D^+D) = 65.61 / 0.01)
    assert info["history"][4] < 1e-10
    assert info["true_rel_res"] < 1e-10
    assert info["history"][3] > 1e-6      # ... and not after 4


def test_finite_termination_pin():
    assert pins.finite_termination_residual() < 1e-10


def test_cgnr_normal_rhs_mode():
    dims = ODD
    U = fieldgen.gauge_field(dims, "haar", 5)
    b = fieldgen.gaussian_spinor(dims, 6)
    x, info = oracle.cgnr(U, b, 0.1, tol=1e-12, rhs="normal")
    xd = oracle.dense_solve_normal(U, b, 0.1, dims, rhs="normal")
    assert pins.rel(x, xd) < 1e-9


@pytest.mark.parametrize("rhs", ["source", "normal"])
@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (3, 2, 4, 2)])
def test_true_residual_checker(dims, rhs):
    # the checker every CG parity test relies on: |1 - c| for c x_d, 1 for
    # x = 0, eps ||D^+D v|| / ||b'|| (dense) for x_d + eps v
    errs = pins.residual_checker_errors(dims, 0.1, rhs=rhs)
    assert errs["scaled"] < 1e-12, errs
    assert errs["zero"] < 1e-14, errs
    assert errs["perturbed"] < 1e-6, errs


def test_true_residual_checker_other_scale():
    # a second scale factor, above 1 (residual -(c - 1) b')
    errs = pins.residual_checker_errors((2, 2, 2, 2), 0.3, c=1.75, seed=31)
    assert errs["scaled"] < 1e-12, errs


# ------------------------------------------------------------- force

def test_force_matches_central_fd_2x2x2x2():
    worst_abs, worst_rel = pins.force_fd_errors((2, 2, 2, 2), 0.1)
    assert worst_rel < 1e-6


def test_force_matches_central_fd_odd():
    worst_abs, worst_rel = pins.force_fd_errors((2, 3, 2, 2), 0.2, seed=12, nentries=12)
    assert worst_rel < 1e-6


def test_force_directional_general_upstream():
    assert pins.force_direction_error((2, 2, 2, 2), 0.1) < 1e-6


def test_force_gauge_covariance():
    assert pins.force_gauge_covariance_error((2, 2, 2, 4), 0.1) < 1e-10
