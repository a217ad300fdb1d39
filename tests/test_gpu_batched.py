"""Batched multi-RHS persistent CG against single-RHS solves, the dense
inverse and the oracle's operator."""
import numpy as np
import pytest
import torch

import fieldgen
import oracle
from gpu_util import log, rel, to_dev, to_np
from paper_2001_05218_amd import _lib

pytestmark = pytest.mark.gpu

wd = pytest.importorskip("paper_2001_05218_amd")

TOL = 1e-10


def _sources(dims, n_gauss, seed):
    pts = fieldgen.point_sources(dims)
    gs = fieldgen.gaussian_spinor(dims, seed, nrhs=n_gauss) if n_gauss else np.zeros((0,) + pts.shape[1:])
    return np.concatenate([pts, gs], axis=0)


def test_point_sources_2x2x2x2_dense_inverse():
    dims, mass = (2, 2, 2, 2), 0.1
    U = fieldgen.gauge_field(dims, "haar", 301)
    B = fieldgen.point_sources(dims)
    X, infos = wd.cg_solve_batched(to_dev(U), to_dev(B), mass, tol=1e-12)
    Dinv = np.linalg.inv(oracle.dense_D(U, mass, dims))
    Xn = to_np(X)
    for k in range(12):
        # D^+D x = D^+ e_k  =>  x = D^{-1} e_k, column k of the inverse (site 0: index k)
        assert rel(Xn[k].reshape(-1), Dinv[:, k]) <= 1e-9
        assert infos[k]["true_rel_res"] <= 1e-12


@pytest.mark.parametrize("nrhs", [1, 5, 16])
def test_each_rhs_matches_single_solve(nrhs):
    dims, mass = (4, 4, 4, 4), 0.1
    log(f"batched 4^4 nrhs={nrhs}")
    U = fieldgen.gauge_field(dims, "haar", 311)
    B = _sources(dims, max(0, nrhs - 12), 312)[:nrhs] if nrhs >= 12 else fieldgen.gaussian_spinor(dims, 313, nrhs=nrhs)
    Ut = to_dev(U)
    X, infos = wd.cg_solve_batched(Ut, to_dev(B), mass, tol=TOL)
    Xn = to_np(X)
    for k in range(nrhs):
        res = oracle.true_relative_residual(U, Xn[k], B[k], mass)
        assert res <= TOL * (1 + 1e-3), (k, res)
        assert abs(res - infos[k]["true_rel_res"]) <= 1e-13
        xs, _ = wd.cg_solve(Ut, to_dev(B[k]), mass, tol=TOL)
        assert rel(Xn[k], to_np(xs)) <= ((mass + 8) / mass) ** 2 * 2 * TOL


def test_normal_mode_and_odd_lattice():
    dims, mass = (5, 3, 7, 4), 0.05
    U = fieldgen.gauge_field(dims, "near_identity", 321)
    B = fieldgen.gaussian_spinor(dims, 322, nrhs=6)
    X, infos = wd.cg_solve_batched(to_dev(U), to_dev(B), mass, tol=TOL, rhs="normal")
    Xn = to_np(X)
    for k in range(6):
        assert oracle.true_relative_residual(U, Xn[k], B[k], mass, rhs="normal") <= TOL * (1 + 1e-3)


def test_complex64_io_and_masks():
    # point sources converge at different iterations than Gaussian ones: masks
    dims, mass = (4, 4, 4, 8), 0.05
    U = fieldgen.gauge_field(dims, "haar", 331)
    B = _sources(dims, 4, 332).astype(np.complex64)
    X, infos = wd.cg_solve_batched(to_dev(U), to_dev(B), mass, tol=TOL)
    assert X.dtype == torch.complex64
    Xn = to_np(X).astype(np.complex128)
    its = [i["iterations"] for i in infos]
    log(f"  iterations per rhs {its}")
    for k in range(16):
        assert infos[k]["true_rel_res"] <= TOL
        # the complex64 output is the FP64 solution rounded: compare with an FP64 solve
        xr, _ = oracle.cgnr(U, B[k].astype(np.complex128), mass, tol=1e-12)
        assert rel(Xn[k], xr) <= 2e-6


def test_not_converged_reports_partial():
    dims, mass = (4, 4, 4, 4), 0.1
    U = fieldgen.gauge_field(dims, "haar", 341)
    B = fieldgen.gaussian_spinor(dims, 342, nrhs=3)
    X, infos = wd.cg_solve_batched(to_dev(U), to_dev(B), mass, tol=TOL, max_iter=5, raise_on_nonconvergence=False)
    Xn = to_np(X)
    for k in range(3):
        assert infos[k]["status"] == 1 and infos[k]["iterations"] == 5
        res = oracle.true_relative_residual(U, Xn[k], B[k], mass)
        assert abs(res - infos[k]["true_rel_res"]) <= 1e-12


@pytest.mark.parametrize("inner,schedule", [("f32", "persistent"), ("f16", "persistent"), ("bf16", "persistent"),
                                            ("i8", "persistent"), ("f16", "lockstep"), ("bf16", "lockstep"),
                                            ("i8", "lockstep")])
def test_config3_24x24x24x48_sixteen_sources(inner, schedule):
    """Full-size batched workload: 12 point sources at the origin + 4 Gaussian,
    Haar links, m = 0.05; every system's FP64 true residual <= 1e-10, and the
    oracle's residual at sampled sites of two systems. Far from a point source
    the inner vectors fall below FP32's normal range, which the scaled
    storages (FP16, int8) must survive."""
    dims, mass = (24, 24, 24, 48), 0.05
    log(f"batched 24^3x48 x16 {inner} {schedule}")
    U = fieldgen.gauge_field(dims, "haar", 200105248)
    B = _sources(dims, 4, 200105249)
    X, infos = wd.cg_solve_batched(to_dev(U), to_dev(B), mass, tol=TOL, inner=inner, schedule=schedule)
    its = [i["iterations"] for i in infos]
    log(f"  iterations {its} seconds {infos[0]['seconds']:.3f}")
    assert all(i["true_rel_res"] <= TOL for i in infos)
    Xn = to_np(X)
    rng = np.random.default_rng(5)
    # the origin, its eight neighbours (where D^+ b of a point source lives)
    # and 23 random sites; the residual there relative to the right-hand side
    # at the same sites (3e-10 allows for the sample's spread around 1e-10)
    near = [(0, 0, 0, 0), (1, 0, 0, 0), (23, 0, 0, 0), (0, 1, 0, 0), (0, 23, 0, 0), (0, 0, 1, 0),
            (0, 0, 23, 0), (0, 0, 0, 1), (0, 0, 0, 47)]
    sites = near + [tuple(int(rng.integers(0, L)) for L in dims) for _ in range(23)]
    for k in (0, 5, 11, 12, 13, 15):
        lhs = oracle.normal_op_sites(U, Xn[k], mass, sites)
        rhs = oracle.wilson_D_sites(U, B[k], mass, sites, dagger=True)
        assert np.linalg.norm(lhs - rhs) <= 3 * TOL * np.linalg.norm(rhs), k


@pytest.mark.parametrize("inner", ["bf16", "f16", "i8"])
@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (5, 3, 7, 4)])
def test_low_precision_storage(inner, dims):
    # p, r, t stored in 16 or 8 bits (tiled and linear site orders): every
    # system still reaches the FP64 tolerance by the oracle's operator
    mass = 0.05
    log(f"batched {inner} {dims}")
    U = fieldgen.gauge_field(dims, "near_identity", 341)
    B = fieldgen.gaussian_spinor(dims, 342, nrhs=6)
    X, infos = wd.cg_solve_batched(to_dev(U), to_dev(B), mass, tol=TOL, inner=inner)
    Xn = to_np(X)
    for k in range(6):
        res = oracle.true_relative_residual(U, Xn[k], B[k], mass)
        assert res <= TOL * (1 + 1e-3), (inner, k, res)
        assert abs(res - infos[k]["true_rel_res"]) <= 1e-13
        assert infos[k]["reliable_updates"] >= 1


# ---- lockstep schedule: the single-system mixed kernels over all systems at once

@pytest.mark.parametrize("inner,nrhs", [("bf16", 5), ("f16", 5), ("i8", 5), ("i8", 1)])
def test_lockstep_each_system_matches_single_solve(inner, nrhs):
    # near-identity links (two-row links in the inner loop), Gaussian sources
    dims, mass = (8, 8, 8, 8), 0.05
    log(f"lockstep {inner} 8^4 x{nrhs}")
    U = fieldgen.gauge_field(dims, "near_identity", 351)
    B = fieldgen.gaussian_spinor(dims, 352, nrhs=nrhs)
    Ut = to_dev(U)
    X, infos = wd.cg_solve_batched(Ut, to_dev(B), mass, tol=TOL, inner=inner, schedule="lockstep")
    Xn = to_np(X)
    for k in range(nrhs):
        res = oracle.true_relative_residual(U, Xn[k], B[k], mass)
        assert res <= TOL * (1 + 1e-3), (k, res)
        assert abs(res - infos[k]["true_rel_res"]) <= 1e-13
        assert infos[k]["two_row_links"] == 1 and infos[k]["reliable_updates"] >= 1
        xs, si = wd.cg_solve(Ut, to_dev(B[k]), mass, tol=TOL, inner=inner)
        # the same kernels, arithmetic and reduction order as a single solve of system k
        assert infos[k]["iterations"] == si["iterations"]
        assert np.array_equal(Xn[k], to_np(xs))


def test_lockstep_point_sources_masks_and_c64():
    # point and Gaussian sources stop at different iterations: the converged
    # systems' gates close while the rest continue
    dims, mass = (4, 4, 4, 8), 0.05
    U = fieldgen.gauge_field(dims, "haar", 361)
    B = _sources(dims, 4, 362).astype(np.complex64)
    X, infos = wd.cg_solve_batched(to_dev(U), to_dev(B), mass, tol=TOL, inner="f16", schedule="lockstep")
    assert X.dtype == torch.complex64
    its = [i["iterations"] for i in infos]
    log(f"  lockstep iterations per rhs {its}")
    Xn = to_np(X).astype(np.complex128)
    for k in range(16):
        assert infos[k]["true_rel_res"] <= TOL
        xr, _ = oracle.cgnr(U, B[k].astype(np.complex128), mass, tol=1e-12)
        assert rel(Xn[k], xr) <= 2e-6


def test_lockstep_normal_mode_initial_guess_and_partial():
    dims, mass = (4, 8, 4, 8), 0.1
    U = fieldgen.gauge_field(dims, "near_identity", 371)
    B = fieldgen.gaussian_spinor(dims, 372, nrhs=3)
    X0 = 0.1 * fieldgen.gaussian_spinor(dims, 373, nrhs=3)
    X, infos = wd.cg_solve_batched(to_dev(U), to_dev(B), mass, tol=TOL, inner="i8", rhs="normal",
                                   X0=to_dev(X0), schedule="lockstep")
    Xn = to_np(X)
    for k in range(3):
        assert oracle.true_relative_residual(U, Xn[k], B[k], mass, rhs="normal") <= TOL * (1 + 1e-3)
    # max_iter reached: every system reports its last iterate and its true residual
    X, infos = wd.cg_solve_batched(to_dev(U), to_dev(B), mass, tol=TOL, inner="bf16", max_iter=7,
                                   raise_on_nonconvergence=False, schedule="lockstep")
    Xn = to_np(X)
    for k in range(3):
        assert infos[k]["status"] == 1 and infos[k]["iterations"] == 7
        res = oracle.true_relative_residual(U, Xn[k], B[k], mass)
        assert abs(res - infos[k]["true_rel_res"]) <= 1e-12


def test_lockstep_zero_and_nan_systems():
    # a zero source converges at once (x = 0) while the others iterate; a NaN
    # in one source ends the call with WD_ERR_NAN
    dims, mass = (4, 4, 4, 8), 0.1
    U = fieldgen.gauge_field(dims, "haar", 391)
    B = fieldgen.gaussian_spinor(dims, 392, nrhs=4)
    B[1] = 0.0
    X, infos = wd.cg_solve_batched(to_dev(U), to_dev(B), mass, tol=TOL, inner="f16", schedule="lockstep")
    Xn = to_np(X)
    assert infos[1]["iterations"] == 0 and np.abs(Xn[1]).max() == 0.0
    for k in (0, 2, 3):
        assert oracle.true_relative_residual(U, Xn[k], B[k], mass) <= TOL * (1 + 1e-3)
    B[2, 0, 1, 2, 3, 1, 2] = np.nan
    with pytest.raises(_lib.WilsonError) as e:
        wd.cg_solve_batched(to_dev(U), to_dev(B), mass, tol=TOL, inner="f16", schedule="lockstep")
    assert e.value.code == _lib.WD_ERR_NAN
