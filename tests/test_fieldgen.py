"""Pins of the seeded input generators (CPU only).

The gauge links stand in for the paper's gauge-configuration files
(Sec. 3.2), and several bounds the operator tests rely on (sigma_min(D) >= m,
||D|| <= m + 8) hold only for unitary links. These tests check the
generators against what their definitions fix: unitarity and unit
determinant to rounding, moments of the Haar measure on SU(3) that
distinguish it from U(3) and from a biased sampler, and the scaling of the
near-identity ensemble exp(i eps H) with eps.
"""
import numpy as np
import pytest

import fieldgen


def _unitarity_errors(u):
    eye = np.eye(3)
    uu = np.einsum("nji,njk->nik", u.conj(), u)   # U^+ U
    return np.abs(uu - eye).max(), np.abs(np.linalg.det(u) - 1.0).max()


@pytest.mark.parametrize("which", ["haar", "near_identity"])
def test_special_unitary(which):
    rng = np.random.default_rng(11)
    u = fieldgen.haar_su3(4096, rng) if which == "haar" else fieldgen.near_identity_su3(4096, 0.3, rng)
    unit, det = _unitarity_errors(u)
    assert unit < 1e-14 and det < 1e-14, (unit, det)


def test_gauge_field_kinds_are_su3():
    for kind in ("haar", "near_identity", "unit"):
        U = fieldgen.gauge_field((4, 2, 2, 4), kind, 5).reshape(-1, 3, 3)
        unit, det = _unitarity_errors(U)
        assert unit < 1e-14 and det < 1e-14, (kind, unit, det)


def test_haar_character_moments():
    # For Haar measure on a compact group the character of an irreducible
    # representation has E[chi] = 0 and E[|chi|^2] = 1. For SU(3),
    # 3 x 3 = 6 + 3bar gives E[|tr U|^4] = 2, and 3 x 3 x 3 contains the
    # singlet once, so E[(tr U)^3] = 1 (it is 0 on U(3), whose determinant
    # phase is free).
    n = 400_000
    u = fieldgen.haar_su3(n, np.random.default_rng(12))
    tr = np.trace(u, axis1=1, axis2=2)
    a2 = np.abs(tr) ** 2
    checks = {
        "E tr": (np.mean(tr), 0.0, np.sqrt(1.0 / n)),
        "E |tr|^2": (np.mean(a2), 1.0, np.std(a2) / np.sqrt(n)),
        "E |tr|^4": (np.mean(a2 ** 2), 2.0, np.std(a2 ** 2) / np.sqrt(n)),
        "E tr^3": (np.mean(tr ** 3), 1.0, np.std(tr ** 3) / np.sqrt(n)),
    }
    for name, (got, want, sem) in checks.items():
        assert abs(got - want) < 6 * sem, (name, got, want, sem)


def test_haar_invariance_of_a_matrix_element():
    # Left invariance: the entries of U are identically distributed; |U_ij|^2
    # has mean 1/3 and E|U_ij|^4 = 2 / (N (N + 1)) = 1/6 for every i, j.
    n = 200_000
    u = fieldgen.haar_su3(n, np.random.default_rng(13))
    a2 = np.abs(u) ** 2
    m2 = a2.mean(axis=0)
    m4 = (a2 ** 2).mean(axis=0)
    assert np.abs(m2 - 1 / 3).max() < 6 * np.sqrt(1 / 18 / n) * 1.5
    assert np.abs(m4 - 1 / 6).max() < 0.01


def _phases(u):
    # eigenphases of unitary matrices, sorted per matrix
    return np.sort(np.angle(np.linalg.eigvals(u)), axis=1)


def test_near_identity_scales_with_eps():
    # exp(i eps H) has eigenphases eps * eig(H) while |eps eig(H)| < pi. The
    # same seed draws the same H, so the phases divided by eps must agree
    # between two eps, and their mean square sum is E tr H^2 = sum_a
    # E[w_a^2] tr(lambda_a^2) / 4 = 8 / 2 = 4 (Gell-Mann normalisation
    # tr(lambda_a lambda_b) = 2 delta_ab).
    n = 40_000
    e1, e2 = 0.05, 0.3
    p1 = _phases(fieldgen.near_identity_su3(n, e1, np.random.default_rng(14))) / e1
    p2 = _phases(fieldgen.near_identity_su3(n, e2, np.random.default_rng(14))) / e2
    ok = np.abs(p2).max(axis=1) * e2 < 3.0    # away from the branch cut
    assert ok.mean() > 0.999
    assert np.abs(p1[ok] - p2[ok]).max() < 1e-10
    # -i log U = eps H: traceless, and ||eps H||_F^2 has mean 4 eps^2
    assert np.abs(p1.sum(axis=1)).max() < 1e-10
    s = (p1 ** 2).sum(axis=1)
    assert abs(s.mean() - 4.0) < 6 * s.std() / np.sqrt(n)


def test_near_identity_distance_from_identity():
    # ||U - 1||_F ~ eps ||H||_F for small eps: the mean square is 4 eps^2 to
    # leading order (the next term is O(eps^4))
    n = 40_000
    eps = 0.01
    u = fieldgen.near_identity_su3(n, eps, np.random.default_rng(15))
    d2 = (np.abs(u - np.eye(3)) ** 2).sum(axis=(1, 2))
    assert abs(d2.mean() / eps ** 2 - 4.0) < 0.05


def test_gaussian_source_moments():
    b = fieldgen.gaussian_spinor((8, 8, 8, 8), 16)
    assert b.shape == (8, 8, 8, 8, 4, 3) and b.dtype == np.complex128
    n = b.size
    assert abs(np.mean(np.abs(b) ** 2) - 1.0) < 6 * np.sqrt(1.0 / n)   # unit complex variance
    assert abs(np.mean(b.real ** 2) - 0.5) < 6 * np.sqrt(0.5 / n)
    assert abs(np.mean(b)) < 6 * np.sqrt(1.0 / n)


def test_point_sources():
    b = fieldgen.point_sources((4, 4, 4, 8), site=(1, 2, 3, 5))
    assert b.shape == (12, 8, 4, 4, 4, 4, 3)
    for k in range(12):
        nz = np.argwhere(b[k] != 0)
        assert nz.tolist() == [[5, 3, 2, 1, k // 3, k % 3]]
        assert b[k][5, 3, 2, 1, k // 3, k % 3] == 1.0


def test_seeded_reproducibility():
    a = fieldgen.gauge_field((4, 4, 2, 2), "haar", 99)
    b = fieldgen.gauge_field((4, 4, 2, 2), "haar", 99)
    c = fieldgen.gauge_field((4, 4, 2, 2), "haar", 100)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
