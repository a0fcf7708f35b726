"""Pins of the comparison metrics at non-zero values (no GPU).

The parity tests judge the GPU library through these functions, so a metric
that under-reports (a stray factor, a wrong normalisation, a transposed
operand) would hide real failures. Each test builds inputs whose answer is
known in closed form -- subspaces at chosen principal angles (Bjorck and
Golub, Math. Comp. 27, 1973: the sines of the principal angles are the
singular values of (I - P_ref) Q_test), low-rank differences of chosen
Frobenius norm -- and checks the metric against it, and against brute force
(forming the m x n products) on small inputs.
"""

import math

import numpy as np
import pytest

from oracle import metrics


def _rot(m, seed):
    """A seeded m x m orthogonal matrix (Householder Q of a Gaussian, diag R > 0)."""
    g = np.random.default_rng(seed).standard_normal((m, m))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))[None, :]


def _pair_at_angles(m, thetas, seed):
    """Orthonormal Phi_ref (m x k) and a basis of a subspace whose principal
    angles to range(Phi_ref) are exactly `thetas`: column i of the second is
    cos(t_i) e_i + sin(t_i) e_{k+i} before a common rotation of R^m."""
    k = len(thetas)
    E = np.zeros((m, k))
    F = np.zeros((m, k))
    for i, t in enumerate(thetas):
        E[i, i] = 1.0
        F[i, i] = math.cos(t)
        F[k + i, i] = math.sin(t)
    Q = _rot(m, seed)
    return Q @ E, Q @ F


@pytest.mark.parametrize("thetas", [[0.3, 0.1, 0.0], [1e-6, 2e-7], [math.pi / 2, 0.2], [0.7]])
def test_sin_theta_at_known_angles(thetas):
    m = 40
    Pr, Pt = _pair_at_angles(m, thetas, 7)
    want = max(math.sin(t) for t in thetas)
    # the test basis may be any (non-orthonormal) basis of its subspace
    mix = np.random.default_rng(3).standard_normal((len(thetas), len(thetas))) + 3 * np.eye(len(thetas))
    got = metrics.sin_theta_max(Pt @ mix, Pr)
    assert got == pytest.approx(want, rel=1e-9, abs=1e-15)


def test_sin_theta_small_angle_relative_accuracy():
    # the sine form keeps relative accuracy where sqrt(1 - cos^2) would cancel to 0
    Pr, Pt = _pair_at_angles(30, [3e-9, 1e-10], 11)
    assert metrics.sin_theta_max(Pt, Pr) == pytest.approx(math.sin(3e-9), rel=1e-5)


def test_sin_theta_brute_force_projectors():
    # largest principal-angle sine = ||P_t - P_r||_2 for equal dimensions (Golub and Van Loan, Thm 2.5.1)
    rng = np.random.default_rng(5)
    Pr, _ = np.linalg.qr(rng.standard_normal((25, 4)))
    Pt = Pr + 0.05 * rng.standard_normal((25, 4))
    Qt, _ = np.linalg.qr(Pt)
    brute = np.linalg.norm(Qt @ Qt.T - Pr @ Pr.T, 2)
    assert metrics.sin_theta_max(Pt, Pr) == pytest.approx(brute, rel=1e-10)
    assert 1e-3 < brute < 0.5


def test_sin_theta_planted_mistakes_are_caught():
    Pr, Pt = _pair_at_angles(40, [0.3, 0.1], 9)
    good = metrics.sin_theta_max(Pt, Pr)
    # a stray 1/sqrt(k) or a cosine in place of a sine would move the value far from the closed form
    assert abs(good / math.sqrt(2) - math.sin(0.3)) > 0.05
    assert abs(math.cos(0.3) - math.sin(0.3)) > 0.5
    assert good == pytest.approx(math.sin(0.3), rel=1e-12)


def _ref_factors(m, n, r, seed):
    rng = np.random.default_rng(seed)
    Pr, _ = np.linalg.qr(rng.standard_normal((m, r)))
    Ar = rng.standard_normal((r, n)) * np.exp(-0.5 * np.arange(r))[:, None]
    return Pr, Ar, rng


def test_lowrank_diff_zero_under_sign_and_rotation():
    Pr, Ar, rng = _ref_factors(60, 35, 5, 1)
    W = _rot(5, 2)
    assert metrics.lowrank_rel_diff(Pr @ W, W.T @ Ar, Pr, Ar) < 1e-14


def test_lowrank_diff_known_rank_one_offset():
    # Phi_t = [Phi_r W, u], A_t = [W^T A_r; eps v^T] with u orthogonal to range(Phi_r):
    # Phi_t A_t - Phi_r A_r = eps u v^T, Frobenius norm eps ||v||
    m, n, r = 60, 35, 5
    Pr, Ar, rng = _ref_factors(m, n, r, 3)
    W = _rot(r, 4)
    u = rng.standard_normal(m)
    u -= Pr @ (Pr.T @ u)
    u /= np.linalg.norm(u)
    v = rng.standard_normal(n)
    eps = 2.5e-3
    Pt = np.hstack([Pr @ W, u[:, None]])
    At = np.vstack([W.T @ Ar, eps * v[None, :]])
    want = eps * np.linalg.norm(v) / np.linalg.norm(Ar)
    assert metrics.lowrank_rel_diff(Pt, At, Pr, Ar) == pytest.approx(want, rel=1e-10)


def test_lowrank_diff_same_span_known_offset():
    # same modes, coefficients off by D: the difference is Phi_r D, norm ||D||_F
    Pr, Ar, rng = _ref_factors(50, 40, 6, 5)
    D = 1e-4 * rng.standard_normal(Ar.shape)
    W = _rot(6, 6)
    want = np.linalg.norm(D) / np.linalg.norm(Ar)
    assert metrics.lowrank_rel_diff(Pr @ W, W.T @ (Ar + D), Pr, Ar) == pytest.approx(want, rel=1e-9)


def test_lowrank_diff_brute_force():
    rng = np.random.default_rng(8)
    m, n = 30, 20
    Pr, _ = np.linalg.qr(rng.standard_normal((m, 4)))
    Ar = rng.standard_normal((4, n))
    Pt = rng.standard_normal((m, 5))   # not orthonormal, other rank
    At = rng.standard_normal((5, n))
    brute = np.linalg.norm(Pt @ At - Pr @ Ar) / np.linalg.norm(Ar)
    assert metrics.lowrank_rel_diff(Pt, At, Pr, Ar) == pytest.approx(brute, rel=1e-12)
    assert brute > 0.5


def test_sigma_rel_err_and_orth_err_values():
    assert metrics.sigma_rel_err([1.1, 2.0, 2.97], [1.0, 2.0, 3.0]) == pytest.approx(0.1, rel=1e-12)
    c = math.cos(1.2)
    Phi = np.array([[1.0, c], [0.0, math.sqrt(1 - c * c)], [0.0, 0.0]])
    assert metrics.orth_err(Phi) == pytest.approx(c, rel=1e-12)
    Phi2 = np.eye(3)[:, :2] * np.array([1.0, 1.001])   # orthogonal columns, one of norm 1.001
    assert metrics.orth_err(Phi2) == pytest.approx(1.001 ** 2 - 1.0, rel=1e-9)


def test_per_mode_sin_values():
    Pr, Pt = _pair_at_angles(20, [0.4, 0.05, 0.0], 12)
    got = metrics.per_mode_sin(-2.0 * Pt, Pr)
    np.testing.assert_allclose(got, [math.sin(0.4), math.sin(0.05), 0.0], rtol=1e-10, atol=1e-14)
