"""Pins of the adaptive-rank oracle (blocked fixed-accuracy range finder,
then steps 6-7 of Alg. 1 and the energy rule of Sec. 4.1), no GPU.

Each pin comes from outside the oracle's own formulas: the reduction to the
non-adaptive O2 at q = 0, the Frobenius identity behind the error indicator
checked against the formed residual, exact low-rank matrices whose rank and
singular values are known, the deflated power iteration written out with
explicit projectors, interlacing, and the monotonicity of the stopping rule.
"""

import numpy as np
import pytest

import synth
from oracle import metrics, philox
from oracle import adaptive as oa
from oracle import rpod as orpod


def _noisy(m=600, n=150, decay=0.05, noise=1e-3, seed=3):
    return synth.lowrank_exp(m, n, decay=decay, noise_std=noise, seed=seed)["St"].T


def test_q0_equals_nonadaptive_rpod_with_the_same_columns():
    S = _noisy()
    om = philox.gaussian_sketch(11, S.shape[1], 64)
    Phi, s, A, info = oa.rpod_adaptive(S, om, 16, 0, 0.9, 64)   # captured: 0.57, 0.85, 0.95, ...
    l = info["l"]
    assert 16 < l < 64            # the threshold stops it after a few blocks
    P2, s2, A2, ex = orpod.rpod_stable(S, l, om[:, :l], 0)
    np.testing.assert_allclose(s, s2, rtol=1e-10)
    k = 20                        # well-separated leading modes
    assert metrics.sin_theta_max(Phi[:, :k], P2[:, :k]) < 1e-8
    assert metrics.lowrank_rel_diff(Phi[:, :k], A[:k], P2[:, :k], A2[:k]) < 1e-8


@pytest.mark.parametrize("q", [0, 1, 2])
def test_indicator_equals_the_formed_residual(q):
    S = _noisy(seed=4)
    om = philox.gaussian_sketch(12, S.shape[1], 96)
    Q, B, info = oa.rand_qb_ei(S, om, 32, q, 0.9999, 96)
    brute = float(np.sum((S - Q @ B) ** 2))
    assert info["E"][-1] == pytest.approx(brute, rel=1e-8, abs=1e-12 * info["fro2"])
    assert np.all(np.diff(info["E"]) < 0)
    assert np.linalg.norm(Q.T @ Q - np.eye(Q.shape[1])) < 1e-12
    np.testing.assert_allclose(B, Q.T @ S, rtol=0, atol=1e-12 * np.sqrt(info["fro2"]))


@pytest.mark.parametrize("k,b", [(10, 16), (37, 16), (48, 16), (20, 32)])
def test_exact_low_rank_stops_at_the_rank(k, b):
    m, n = 400, 120
    U = synth._orthonormal(m, k, 5, 1)
    V = synth._orthonormal(n, k, 5, 2)
    sig = 10.0 * np.exp(-0.1 * np.arange(k))
    S = (U * sig) @ V.T
    om = philox.gaussian_sketch(13, n, 96)
    Phi, s, A, info = oa.rpod_adaptive(S, om, b, 0, 1.0 - 1e-12, 96)
    assert info["l"] == -(-k // b) * b       # the first block count that reaches k columns
    np.testing.assert_allclose(s[:k], sig, rtol=1e-11)
    assert np.all(s[k:] < 1e-12 * sig[0])
    assert info["r"] == k
    assert metrics.sin_theta_max(Phi[:, :k], U) < 1e-10


@pytest.mark.parametrize("q", [1, 2])
def test_power_iterations_are_deflated(q):
    """Block 2's basis spans ((I - P) S S^T (I - P))^q (I - P) S Omega_2,
    P = Q_1 Q_1^T: the deflated power iteration with explicit projectors."""
    S = _noisy(m=200, n=80, decay=0.08, noise=1e-2, seed=6)
    om = philox.gaussian_sketch(14, 80, 32)
    Q, B, info = oa.rand_qb_ei(S, om, 16, q, 1.0, 32)
    assert info["blocks"] == 2
    Q1, Q2 = Q[:, :16], Q[:, 16:]
    M = S - Q1 @ (Q1.T @ S)
    Y = M @ om[:, 16:32]
    for _ in range(q):
        Y = M @ (M.T @ Y)
    assert metrics.sin_theta_max(Q2, np.linalg.qr(Y)[0]) < 1e-9
    # the first block is the undeflated subspace iteration of Alg. 1 step 3
    Y1 = S @ om[:, :16]
    for _ in range(q):
        Y1 = S @ (S.T @ Y1)
    assert metrics.sin_theta_max(Q1, np.linalg.qr(Y1)[0]) < 1e-9


def test_interlacing_and_energy_rank_against_the_exact_svd():
    S = _noisy(seed=8, decay=0.12, noise=1e-4)
    om = philox.gaussian_sketch(15, S.shape[1], 96)
    Phi, s, A, info = oa.rpod_adaptive(S, om, 16, 2, 0.99, 96)
    s_all = np.linalg.svd(S, compute_uv=False)
    assert np.all(s <= s_all[:len(s)] * (1 + 1e-12))
    e_exact = np.cumsum(s_all ** 2) / np.sum(s_all ** 2)
    r_exact = int(np.nonzero(e_exact >= 0.99)[0][0]) + 1
    assert info["r"] == r_exact
    assert info["energy"][info["r"] - 1] >= 0.99 > (info["energy"][info["r"] - 2] if info["r"] > 1 else 0)
    assert metrics.orth_err(Phi) < 1e-12


def test_stopping_is_monotone_in_delta():
    S = _noisy(seed=9)
    om = philox.gaussian_sketch(16, S.shape[1], 128)
    blocks = [oa.rand_qb_ei(S, om, 16, 1, d, 128)[2]["blocks"] for d in (0.5, 0.9, 0.99, 0.999, 0.9999)]
    assert blocks == sorted(blocks) and blocks[0] < blocks[-1]


def test_unreachable_threshold_uses_every_block_and_reports_no_rank():
    S = _noisy(seed=10, noise=1e-1)      # noise floor: full rank
    om = philox.gaussian_sketch(17, S.shape[1], 48)
    Phi, s, A, info = oa.rpod_adaptive(S, om, 16, 0, 1.0, 48)
    assert info["blocks"] == 3 and info["l"] == 48 and info["r"] == -1
    with pytest.raises(ValueError):
        oa.rand_qb_ei(S, om, 16, 0, 0.5, 40)


def test_a_dropped_projection_is_caught_by_the_formed_residual():
    """Planted mistake (a local copy of the loop without the "- Q (B Omega)"
    term): the indicator then disagrees with the formed residual, which is
    what the identity pin above would report."""
    S = _noisy(seed=11)
    om = philox.gaussian_sketch(18, S.shape[1], 48)
    fro2 = float(np.sum(S * S))
    E, Q, B = fro2, np.zeros((S.shape[0], 0)), np.zeros((0, S.shape[1]))
    for i in range(3):
        Qi = np.linalg.qr(S @ om[:, 16 * i:16 * (i + 1)])[0]     # projection dropped
        Bi = Qi.T @ S
        Q, B = np.hstack([Q, Qi]), np.vstack([B, Bi])
        E -= float(np.sum(Bi * Bi))
    assert abs(E - float(np.sum((S - Q @ B) ** 2))) > 1e-3 * fro2
