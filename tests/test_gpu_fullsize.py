"""The benchmark's workloads at full size, checked by the oracle on the whole
lattice.

* 32x32x32x64, links exp(i 0.3 H), m = 0.02, one Gaussian source: every
  solve the benchmark times or reports (plain FP64 CG; reliable-update mixed
  CG with FP32, BF16, FP16 and int8 storage; iterative refinement with int8
  storage), called with the benchmark's parameters. Accepted when the
  oracle's residual ||D^+b - D^+D x|| / ||D^+b||, recomputed in FP64 numpy
  over all 2^21 sites, is <= 1e-10 and agrees with the library's own FP64
  recomputation.
* 24x24x24x48, Haar links, m = 0.05, 12 point sources at the origin and 4
  Gaussian sources in complex64, as the benchmark's batched row solves them:
  all 16 systems checked by the oracle over the whole lattice. The returned
  X is rounded to complex64, so its residual is bounded by the solver's 1e-10
  plus what that rounding can add: ||D^+D (x - X)|| <= (m + 8)^2 2^-24 ||x||
  (each real component is rounded to nearest, |D| <= m + 8 for unitary links).
* The Laplacian at 32x32x32x64 (m2 = 0.05): the operator at sampled sites and
  the CG solution over the whole lattice.
* The gauge force G(a, b) at 32x32x32x64 (the grid and block order the
  benchmark times), every link of every site against the oracle, written and
  then accumulated.
* The packed D^+ of the benchmark's Dslash loop in every storage (and the
  solver's two-row link formats) at 64 sampled sites of 32x32x32x64.
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
# the library's FP64 recomputation and the oracle's differ only by rounding
AGREE = 1e-12


def _sites(n, seed):
    rng = np.random.default_rng(seed)
    fixed = [(0, 0, 0, 0), (31, 31, 31, 63), (31, 0, 15, 32), (0, 31, 0, 63)]
    return fixed + [tuple(int(rng.integers(0, L)) for L in DIMS) for _ in range(n - len(fixed))]


@pytest.fixture(scope="module")
def links():
    log("generating 32^3x64 links (the benchmark's seed)")
    return fieldgen.gauge_field(DIMS, "near_identity", 200105238, eps=0.3)


@pytest.fixture(scope="module")
def source(links):
    log("source and b' = D^+ b by the oracle")
    b = fieldgen.gaussian_spinor(DIMS, 200105239)
    bp = oracle.wilson_Ddag(links, b, MASS)
    return b, bp, float(np.linalg.norm(bp))


def _oracle_residual(U, x, bp, bpn, mass):
    r = bp - oracle.normal_op(U, x, mass)
    return float(np.linalg.norm(r) / bpn)


# (inner storage, scheme, inner_tol) as the benchmark calls them
SOLVES = [("f64", "reliable", 0.0), ("f32", "reliable", 0.0), ("bf16", "reliable", 0.0),
          ("f16", "reliable", 0.0), ("i8", "reliable", 0.0), ("i8", "refinement", 0.1)]


@pytest.mark.parametrize("inner,scheme,inner_tol", SOLVES,
                         ids=[f"{i}-{s}" for i, s, _ in SOLVES])
def test_wilson_solve_whole_lattice_residual(links, source, inner, scheme, inner_tol):
    b, bp, bpn = source
    log(f"wilson cg 32^3x64 inner={inner} scheme={scheme}")
    x, info = wd.cg_solve(to_dev(links), to_dev(b), MASS, tol=TOL, max_iter=20000, inner=inner,
                          reliable_interval=50, scheme=scheme, inner_tol=inner_tol)
    log(f"  iterations={info['iterations']} updates={info['reliable_updates']} "
        f"true_res={info['true_rel_res']:.3e} seconds={info['seconds']:.3f}")
    assert info["true_rel_res"] <= TOL
    res = _oracle_residual(links, to_np(x), bp, bpn, MASS)
    log(f"  oracle whole-lattice residual {res:.4e} (library {info['true_rel_res']:.4e})")
    assert res <= TOL
    assert abs(res - info["true_rel_res"]) <= AGREE


def test_wilson_apply_sampled_sites(links):
    # D and D^+ at 64 sites of the full lattice, <= 1e-12 relative per site
    psi = fieldgen.gaussian_spinor(DIMS, 200105240)
    Ut, pt = to_dev(links), to_dev(psi)
    sites = _sites(64, 14)
    for dag in (False, True):
        out = to_np(wd.wilson_apply(Ut, pt, MASS, dagger=dag))
        ref = oracle.wilson_D_sites(links, psi, MASS, sites, dagger=dag)
        got = np.array([out[t, z, y, x] for (x, y, z, t) in sites])
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_force_whole_lattice():
    log("force 32^3x64 whole lattice")
    a = fieldgen.gaussian_spinor(DIMS, 200105241)
    b = fieldgen.gaussian_spinor(DIMS, 200105242)
    at, bt = to_dev(a), to_dev(b)
    F = wd.wilson_force(at, bt, 1.0)
    ref = oracle.force_G(a, b)
    scale = np.abs(ref).max()
    assert np.abs(to_np(F) - ref).max() <= 1e-13 * scale
    wd.wilson_force(bt, at, -0.5, out=F, accumulate=True)
    ref -= 0.5 * oracle.force_G(b, a)
    assert np.abs(to_np(F) - ref).max() <= 1e-13 * scale


# the benchmark's D^+ loop: each storage as bench.py packs and launches it;
# bounds as for the same kernels on small lattices (relative over the sample)
@pytest.mark.parametrize("prec,bound", [("f64", 1e-12), ("f32", 2e-6), ("bf16", 1.5e-2), ("f16", 3e-3),
                                        ("i8", 2e-2), ("f16_rows2", 3e-3), ("i8_rows2", 2e-2)])
def test_packed_dagger_sampled_sites(links, source, prec, bound):
    log(f"packed D^+ 32^3x64 {prec}")
    b = source[0]
    Ut, bt = to_dev(links), to_dev(b)
    Up = wd.pack_gauge(Ut, prec)
    pin = wd.pack_spinor(bt, prec)
    pout = wd.empty_packed_spinor(DIMS, prec, bt.device)
    wd.wilson_apply_packed(Up, pin, pout, DIMS, MASS, prec, True)
    out = to_np(wd.unpack_spinor(pout, DIMS, prec))
    sites = _sites(64, 15)
    ref = oracle.wilson_D_sites(links, b, MASS, sites, dagger=True)
    got = np.array([out[t, z, y, x] for (x, y, z, t) in sites])
    assert np.linalg.norm(got - ref) <= bound * np.linalg.norm(ref)
    if prec == "f64":
        for k in range(len(sites)):
            assert np.abs(got[k] - ref[k]).max() <= 1e-12 * np.abs(ref[k]).max()


# ---------------------------------------------------------------- batched (c3)

C3_DIMS = (24, 24, 24, 48)
C3_MASS = 0.05


@pytest.fixture(scope="module")
def c3_solution():
    log("batched 24^3x48 x16, complex64 I/O, the benchmark's default schedule")
    U = fieldgen.gauge_field(C3_DIMS, "haar", 200105248)
    pts = fieldgen.point_sources(C3_DIMS)[:12]
    gs = fieldgen.gaussian_spinor(C3_DIMS, 200105249, nrhs=4)
    B = np.concatenate([pts, gs]).astype(np.complex64)
    X, infos = wd.cg_solve_batched(to_dev(U), to_dev(B), C3_MASS, tol=TOL, inner="f16")
    log(f"  iterations {[i['iterations'] for i in infos]} seconds {infos[0]['seconds']:.3f}")
    return U, B, to_np(X), infos


@pytest.mark.parametrize("group", range(4))
def test_config3_complex64_whole_lattice(c3_solution, group):
    U, B, X, infos = c3_solution
    assert X.dtype == np.complex64
    for k in range(4 * group, 4 * group + 4):
        assert infos[k]["true_rel_res"] <= TOL
        b = B[k].astype(np.complex128)
        x = X[k].astype(np.complex128)
        bp = oracle.wilson_Ddag(U, b, C3_MASS)
        bpn = float(np.linalg.norm(bp))
        res = _oracle_residual(U, x, bp, bpn, C3_MASS)
        rounding = (C3_MASS + 8.0) ** 2 * 2.0 ** -24 * float(np.linalg.norm(x)) / bpn
        log(f"  system {k}: residual of the complex64 X {res:.3e} (bound {TOL + rounding:.3e}, "
            f"library FP64 x {infos[k]['true_rel_res']:.3e})")
        assert res <= TOL + rounding


# ------------------------------------------------------------------ Laplacian

def test_laplace_apply_sampled_sites(links):
    log("laplace apply 32^3x64 sampled")
    psi = fieldgen.gaussian_colour(DIMS, 200105269)
    out = to_np(wd.laplace_apply(to_dev(links), to_dev(psi), LAP_M2))
    sites = _sites(64, 12)
    ref = lap.laplace_sites(links, psi, LAP_M2, sites)
    for k, (x, y, z, t) in enumerate(sites):
        assert np.abs(out[t, z, y, x] - ref[k]).max() <= 1e-13 * np.abs(ref[k]).max()


def test_laplace_solve_whole_lattice_residual(links):
    log("laplace cg 32^3x64")
    b = fieldgen.gaussian_colour(DIMS, 200105268)
    x, info = wd.laplace_cg_solve(to_dev(links), to_dev(b), LAP_M2, tol=TOL, max_iter=20000)
    log(f"  iterations={info['iterations']} true_res={info['true_rel_res']:.3e}")
    assert info["true_rel_res"] <= TOL
    res = lap.true_relative_residual(links, to_np(x), b, LAP_M2)
    log(f"  oracle whole-lattice residual {res:.4e}")
    assert res <= TOL
    assert abs(res - info["true_rel_res"]) <= AGREE
