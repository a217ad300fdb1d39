"""Planted mistakes in the oracle (CPU only): each must trip at least one pin.

Every mutation replaces one piece of the oracle with a plausible wrong
version (dropped term, wrong sign, transposed operand, wrong index or
direction) for the duration of one test, then runs the pin checks of
``pins.py``. A mutation that no pin detects would mean the pins leave that
part of the oracle unconstrained.
"""
import numpy as np
import pytest

import oracle
import pins
from oracle import dirac, force, solver

THRESH = 1e-8


def _detected(errs, thresh=THRESH):
    # NaN counts as detected: a broken oracle may blow up
    return any(not (e <= thresh) for e in errs.values())


def _pin_errors_operator():
    errs = {
        "basis": pins.basis_table_error(),
        "clifford": pins.clifford_error(),
        "spectrum": pins.free_spectrum_error((2, 2, 2, 4), 0.1),
        "plane_wave": pins.plane_wave_error((4, 6, 8, 10), (1, 2, 3, 5), 0.1),
        "plane_wave_dag": pins.plane_wave_error((4, 6, 8, 10), (1, 2, 3, 5), 0.1, dagger=True),
        "dense": pins.dense_vs_apply_error((3, 2, 4, 2), 0.1),
        "adjoint": pins.adjoint_dense_error((3, 2, 4, 2), 0.1),
        "gamma5": pins.gamma5_hermiticity_error((3, 2, 4, 2), 0.1),
        "gauge": pins.gauge_covariance_error((4, 4, 2, 4), 0.1),
        "gauge_dag": pins.gauge_covariance_error((4, 4, 2, 4), 0.1, dagger=True),
    }
    return errs


def _mutated_apply(kind):
    G = dirac.GAMMA
    ID4 = np.eye(4, dtype=np.complex128)

    def apply(U, psi, mass, gsign):
        diag = {"mass_plus8": mass + 8.0, "mass_only": mass}.get(kind, mass + 4.0)
        out = diag * psi
        for mu in range(4):
            ax = {"axis_mu": mu}.get(kind, 3 - mu)
            Uf = U[mu]
            if kind == "link_transposed":
                Uf = np.swapaxes(Uf, -1, -2)
            step = +1 if kind == "fwd_roll_swapped" else -1
            fwd = dirac._colour(Uf, np.roll(psi, step, axis=ax))
            if kind == "bwd_no_dagger":
                bwd = np.roll(dirac._colour(U[mu], psi), 1, axis=ax)
            elif kind == "bwd_transpose_only":
                bwd = np.roll(dirac._colour(np.swapaxes(U[mu], -1, -2), psi), 1, axis=ax)
            elif kind == "bwd_link_unshifted":
                bwd = dirac._colour_dag(U[mu], np.roll(psi, 1, axis=ax))
            else:
                bwd = np.roll(dirac._colour_dag(U[mu], psi), 1, axis=ax)
            s = gsign
            if kind == "dagger_not_flipped":
                s = 1.0
            pm = ID4 - s * G[mu]
            pp = ID4 + s * G[mu]
            if kind == "projectors_swapped":
                pm, pp = pp, pm
            if kind == "projector_dropped_fwd":
                pm = ID4
            half = 1.0 if kind == "no_half" else 0.5
            out = out - half * (dirac._spin(pm, fwd) + dirac._spin(pp, bwd))
        return out

    return apply


OPERATOR_MUTATIONS = [
    "mass_plus8", "mass_only", "axis_mu", "link_transposed", "fwd_roll_swapped",
    "bwd_no_dagger", "bwd_transpose_only", "bwd_link_unshifted", "dagger_not_flipped",
    "projectors_swapped", "projector_dropped_fwd", "no_half",
]


@pytest.mark.parametrize("kind", OPERATOR_MUTATIONS)
def test_operator_mutation_is_detected(kind, monkeypatch):
    monkeypatch.setattr(dirac, "_apply", _mutated_apply(kind))
    errs = _pin_errors_operator()
    assert _detected(errs), errs


@pytest.mark.parametrize("which,entry", [(0, (0, 3)), (1, (3, 0)), (2, (1, 3)), (3, (2, 0))])
def test_gamma_entry_sign_flip_is_detected(which, entry, monkeypatch):
    g = dirac.GAMMA.copy()
    g[which][entry] *= -1
    monkeypatch.setattr(dirac, "GAMMA", g)
    errs = _pin_errors_operator()
    assert _detected(errs), errs


def test_gamma_overall_sign_flip_is_detected(monkeypatch):
    # flipping one whole gamma keeps the Clifford algebra: the typed basis
    # table and the plane-wave eigenvalue (i gamma_mu sin p_mu) still catch it
    g = dirac.GAMMA.copy()
    g[2] = -g[2]
    monkeypatch.setattr(dirac, "GAMMA", g)
    errs = _pin_errors_operator()
    assert errs["plane_wave"] > THRESH and errs["basis"] > THRESH


def _cg_pin_errors():
    return {
        "dense": pins.dense_solve_error((2, 2, 2, 2), 0.1),
        "plane": pins.plane_wave_solve_error((4, 2, 4, 6), (1, 0, 2, 3), 0.1),
        "finite_termination": pins.finite_termination_residual(),
    }


def _mutated_cgnr(kind):
    def cgnr(U, b, mass, tol=1e-10, max_iter=10000, rhs="source", x0=None, history=False):
        bp = dirac.wilson_Ddag(U, b, mass) if rhs == "source" else b.copy()
        bnorm = np.linalg.norm(bp)
        x = np.zeros_like(bp)
        r = bp.copy()
        p = r.copy()
        rho = float(np.vdot(r, r).real)
        k = 0
        while np.sqrt(rho) / bnorm > tol and k < max_iter:
            t = dirac.wilson_D(U, p, mass)
            tt = float(np.vdot(t, t).real)
            if not np.isfinite(tt) or tt == 0.0:
                break
            alpha = rho / tt
            x = x + alpha * p
            q = dirac.wilson_D(U, t, mass) if kind == "q_without_dagger" else dirac.wilson_Ddag(U, t, mass)
            r = r - alpha * q
            rho_new = float(np.vdot(r, r).real)
            if not np.isfinite(rho_new) or rho_new == 0.0:
                break
            beta = rho / rho_new if kind == "beta_inverted" else rho_new / rho
            p = (r + beta * r) if kind == "p_from_r" else (r + beta * p)
            rho = rho_new
            k += 1
        return x, dict(iterations=k, iter_rel_res=np.sqrt(rho) / bnorm, true_rel_res=0.0, history=[])
    return cgnr


@pytest.mark.parametrize("kind", ["beta_inverted", "q_without_dagger", "p_from_r"])
def test_cg_mutation_is_detected(kind, monkeypatch):
    m = _mutated_cgnr(kind)
    monkeypatch.setattr(oracle, "cgnr", lambda *a, **k: m(*a, **{**k, "max_iter": 400}))
    errs = _cg_pin_errors()
    assert _detected(errs), errs


def _mutated_force(kind):
    G = dirac.GAMMA
    ID4 = np.eye(4, dtype=np.complex128)

    def force_G(a, b):
        out = np.empty((4,) + a.shape[:4] + (3, 3), dtype=np.complex128)
        for mu in range(4):
            ax = 3 - mu
            pm = ID4 - G[mu]
            pp = ID4 + G[mu]
            if kind == "projector_sign":
                pm, pp = pp, pm
            pm_a = np.matmul(pm, a)
            b_f = np.roll(b, -1, axis=ax)
            pp_a_f = np.roll(np.matmul(pp, a), -1, axis=ax)
            t1 = force._outer(pm_a, b_f)
            t2 = force._outer(b, pp_a_f)
            if kind == "drop_second":
                t2 = 0 * t2
            if kind == "no_conj":
                t1 = np.matmul(np.swapaxes(pm_a, -1, -2), b_f)
            if kind == "transposed":
                t1 = np.swapaxes(t1, -1, -2)
            if kind == "wrong_shift":
                b_f = np.roll(b, 1, axis=ax)
                t1 = force._outer(pm_a, b_f)
            out[mu] = 0.5 * (t1 + t2)
        return out
    return force_G


@pytest.mark.parametrize("kind", ["projector_sign", "drop_second", "no_conj", "transposed", "wrong_shift"])
def test_force_mutation_is_detected(kind, monkeypatch):
    monkeypatch.setattr(force, "force_G", _mutated_force(kind))
    _, worst_rel = pins.force_fd_errors((2, 2, 2, 2), 0.1, nentries=8)
    cov = pins.force_gauge_covariance_error((2, 2, 2, 4), 0.1)
    assert _detected({"fd": worst_rel, "cov": cov}, 1e-6)


def _mutated_true_residual(kind):
    def true_relative_residual(U, x, b, mass, rhs="source"):
        if rhs == "source":
            bp = dirac.wilson_D(U, b, mass) if kind == "bprime_without_dagger" else dirac.wilson_Ddag(U, b, mass)
            if kind == "b_instead_of_bprime":
                bp = b
        else:
            bp = b
        Ax = dirac.wilson_D(U, x, mass) if kind == "D_instead_of_normal" else dirac.normal_op(U, x, mass)
        r2 = float(np.vdot(bp - Ax, bp - Ax).real)
        den2 = float(np.vdot(b, b).real) if kind == "normalised_by_b" else float(np.vdot(bp, bp).real)
        if kind == "no_sqrt":
            return r2 / den2
        return float(np.sqrt(r2) / np.sqrt(den2))
    return true_relative_residual


@pytest.mark.parametrize("kind", ["no_sqrt", "normalised_by_b", "b_instead_of_bprime", "bprime_without_dagger",
                                  "D_instead_of_normal"])
def test_true_residual_mutation_is_detected(kind, monkeypatch):
    monkeypatch.setattr(oracle, "true_relative_residual", _mutated_true_residual(kind))
    errs = {}
    for rhs in ("source", "normal"):
        e = pins.residual_checker_errors((2, 2, 2, 2), 0.1, rhs=rhs)
        errs.update({f"{rhs}_{k}": v for k, v in e.items()})
    assert _detected(errs, 1e-6), errs
