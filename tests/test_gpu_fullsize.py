"""The benchmark's workload at full size -- Wilson-Dirac and Laplacian solves
on 32x32x32x64 with links exp(i 0.3 H), in the launch configuration bench.py
times -- checked against the oracle on sampled sites (the oracle evaluates
the operators site by site; the whole lattice would take minutes).

A solve is accepted when the residual of the returned x, recomputed by the
oracle at 128 sampled sites and divided by the right-hand side's norm at the
same sites, is below 3e-10: the solver's own FP64 recomputation reaches
1e-10 over the whole lattice, and a sample of 128 sites estimates that ratio
to within a small factor, while any error in the operator or the solution
gives an O(1) value.
"""
import numpy as np
import pytest

import fieldgen
import oracle
from oracle import laplace as lap
from gpu_util import log, to_dev, to_np

pytestmark = pytest.mark.gpu

wd = pytest.importorskip("paper_2001_05218_amd")

DIMS = (32, 32, 32, 64)
MASS = 0.02
LAP_M2 = 0.05
TOL = 1e-10
SAMPLED_BOUND = 3e-10


def _sites(n, seed):
    rng = np.random.default_rng(seed)
    fixed = [(0, 0, 0, 0), (31, 31, 31, 63), (31, 0, 15, 32), (0, 31, 0, 63)]
    return fixed + [tuple(int(rng.integers(0, L)) for L in DIMS) for _ in range(n - len(fixed))]


@pytest.fixture(scope="module")
def links():
    log("generating 32^3x64 links (the benchmark's seed)")
    return fieldgen.gauge_field(DIMS, "near_identity", 200105238, eps=0.3)


@pytest.mark.parametrize("inner", ["i8", "f64"])
def test_wilson_solve_sampled_residual(links, inner):
    log(f"wilson cg 32^3x64 inner={inner}")
    b = fieldgen.gaussian_spinor(DIMS, 200105239)
    x, info = wd.cg_solve(to_dev(links), to_dev(b), MASS, tol=TOL, max_iter=20000, inner=inner,
                          reliable_interval=50)
    log(f"  iterations={info['iterations']} true_res={info['true_rel_res']:.3e}")
    assert info["true_rel_res"] <= TOL
    sites = _sites(128, 11)
    lhs = oracle.normal_op_sites(links, to_np(x), MASS, sites)
    rhs = oracle.wilson_D_sites(links, b, MASS, sites, dagger=True)
    sampled = float(np.linalg.norm(lhs - rhs) / np.linalg.norm(rhs))
    log(f"  sampled oracle residual {sampled:.3e}")
    assert sampled <= SAMPLED_BOUND


def test_laplace_apply_sampled_sites(links):
    log("laplace apply 32^3x64 sampled")
    psi = fieldgen.gaussian_colour(DIMS, 200105269)
    out = to_np(wd.laplace_apply(to_dev(links), to_dev(psi), LAP_M2))
    sites = _sites(64, 12)
    ref = lap.laplace_sites(links, psi, LAP_M2, sites)
    for k, (x, y, z, t) in enumerate(sites):
        assert np.abs(out[t, z, y, x] - ref[k]).max() <= 1e-13 * np.abs(ref[k]).max()


def test_laplace_solve_sampled_residual(links):
    log("laplace cg 32^3x64")
    b = fieldgen.gaussian_colour(DIMS, 200105268)
    x, info = wd.laplace_cg_solve(to_dev(links), to_dev(b), LAP_M2, tol=TOL, max_iter=20000)
    log(f"  iterations={info['iterations']} true_res={info['true_rel_res']:.3e}")
    assert info["true_rel_res"] <= TOL
    sites = _sites(128, 13)
    lhs = lap.laplace_sites(links, to_np(x), LAP_M2, sites)
    rhs = np.array([b[t, z, y, xx] for (xx, y, z, t) in sites])
    sampled = float(np.linalg.norm(lhs - rhs) / np.linalg.norm(rhs))
    log(f"  sampled oracle residual {sampled:.3e}")
    assert sampled <= SAMPLED_BOUND
