"""Pins of the warm-start oracle (CPU only): every function is checked
against something other than itself (finite differences, brute-force
matrices, closed forms, the exact SVD)."""

import numpy as np
import pytest

import synth
from oracle import metrics, philox, pod
from oracle import warm as ow


def _params(K=8, seed=0, scale=0.3):
    g = np.random.default_rng(seed)
    return {k: scale * g.standard_normal(sh) for k, sh in ow.param_shapes(K).items()}


def _bank(m=60, r=5, K=8, seed=1):
    g = np.random.default_rng(seed)
    return [np.linalg.qr(g.standard_normal((m, r)))[0] for _ in range(K)]


def test_loss_equals_projector_distance():
    """L(c) = ||Phi_i Phi_i^T - sum_k c_k Phi_k Phi_k^T||_F^2, written out with m x m matrices."""
    bases = _bank()
    r = bases[0].shape[1]
    G8 = ow.block_gram(ow.bank_gram(bases), 8, r)
    g = np.random.default_rng(2)
    Phi_i = np.linalg.qr(g.standard_normal((60, r)))[0]
    b = ow.targets(bases, Phi_i)
    for _ in range(5):
        c = ow.softmax(g.standard_normal(8))
        Pc = sum(ck * B @ B.T for ck, B in zip(c, bases))
        brute = np.sum((Phi_i @ Phi_i.T - Pc) ** 2)
        formula = r - 2 * b @ c + c @ G8 @ c
        assert abs(brute - formula) < 1e-12 * max(1.0, brute)


def test_backward_matches_central_differences():
    P = _params(seed=3)
    bases = _bank(seed=4)
    G8 = ow.block_gram(ow.bank_gram(bases), 8, 5)
    g = np.random.default_rng(5)
    X = g.uniform(-1, 1, (6, 4))
    B = np.stack([ow.targets(bases, np.linalg.qr(g.standard_normal((60, 5)))[0]) for _ in range(6)])
    grads = ow.backward(P, X, B, G8)
    h = 1e-6
    for name in ow.PARAM_ORDER:
        flat = P[name].reshape(-1)
        idx = g.choice(flat.size, size=min(12, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp, _ = ow.loss(P, X, B, G8, 5)
            flat[i] = old - h
            lm, _ = ow.loss(P, X, B, G8, 5)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = grads[name].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1e-3, abs(fd)), (name, i, fd, an)


def test_adam_first_step_is_a_sign_step():
    """At t = 1 the bias-corrected Adam update is lr * g / (|g| + eps) (no weight decay)."""
    P = _params(seed=6)
    g = {k: np.random.default_rng(7).standard_normal(v.shape) for k, v in P.items()}
    P0 = {k: v.copy() for k, v in P.items()}
    ow.adam_step(P, g, {}, lr=1e-2, eps=1e-8, weight_decay=0.0)
    for k in P:
        want = P0[k] - 1e-2 * g[k] / (np.abs(g[k]) + 1e-8)
        assert np.allclose(P[k], want, rtol=0, atol=1e-15)


def test_adam_weight_decay_enters_the_gradient():
    P = {k: np.ones(s) for k, s in ow.param_shapes().items()}
    g = {k: np.zeros(s) for k, s in ow.param_shapes().items()}
    ow.adam_step(P, g, {}, lr=1e-3, weight_decay=0.5)
    # gradient 0.5 * theta = 0.5 > 0: one sign step down
    for k in P:
        assert np.allclose(P[k], 1.0 - 1e-3 * 0.5 / (0.5 + 1e-8))


def test_assemble_one_hot_returns_the_bank_basis():
    bases = _bank(seed=8)
    GW = ow.bank_gram(bases)
    Phi_b = np.hstack(bases)
    for k in (0, 5, 7):
        c = np.zeros(8)
        c[k] = 1.0
        for j in (1, 2, 3):
            W = Phi_b @ ow.assemble(GW, c, k, 5, j)
            assert np.allclose(W, bases[k], atol=1e-13)


def test_assemble_is_power_iteration_on_the_weighted_projector():
    bases = _bank(seed=9)
    GW = ow.bank_gram(bases)
    c = ow.softmax(np.random.default_rng(10).standard_normal(8))
    k = ow.argmax_first(c)
    Pc = sum(ck * B @ B.T for ck, B in zip(c, bases))
    for j in (1, 2):
        W = np.hstack(bases) @ ow.assemble(GW, c, k, 5, j)
        brute = np.linalg.matrix_power(Pc, j) @ bases[k]
        assert np.allclose(W, brute, atol=1e-13)


def test_argmax_takes_lowest_index_on_ties():
    assert ow.argmax_first([0.1, 0.4, 0.4, 0.1]) == 1


def test_warm_start_with_the_exact_basis_equals_exact_pod():
    """W = the exact leading basis (one-hot c on it): q = 0 already gives O1."""
    fam = synth.ParamFamily(32, 64, K=100)
    mu, _ = synth.draw_params(3, seed=12)
    d = fam.matrix(mu[0], 300, noise_std=0.0, seed=13)
    S = d["St"].T
    r = 20
    bases = _bank(m=S.shape[0], r=r, seed=14)
    bases[2] = d["U"][:, :r]
    c = np.full(8, 1e-30)
    c[2] = 1.0
    om = np.random.default_rng(15).standard_normal((300, 10))
    Phi, s, A, ex = ow.warm_rpod(S, bases, c / c.sum(), 2, r, om, q=0)
    P1, s1, A1, _ = pod.pod_svd(S, r)
    assert metrics.sigma_rel_err(s, s1) < 1e-12
    assert metrics.sin_theta_max(Phi, P1) < 1e-10
    # the returned triplets are exact singular triplets: every residual vanishes
    # although the range basis misses most of S (rank ~100 > l = 30)
    assert ex["rho"] < 1e-10


def test_parameter_family_is_smooth_and_orthonormal():
    fam = synth.ParamFamily(32, 64)
    U0 = fam.U(np.zeros(4))
    assert np.abs(U0.T @ U0 - np.eye(fam.K)).max() < 1e-12
    # nearby parameters give nearby leading subspaces, opposite corners about 30 degrees
    d = np.array([1e-3, 0, 0, 0])
    small = metrics.sin_theta_max(fam.U(d)[:, :50], U0[:, :50])
    corner = metrics.sin_theta_max(fam.U(np.ones(4))[:, :50], fam.U(-np.ones(4))[:, :50])
    assert small < 1e-3
    assert 0.4 < corner < 0.6


# --------------------------------------------------------------------------
# per-mode residual and the continued fallback
# --------------------------------------------------------------------------

def _svd_matrix(m, n, s, seed):
    U = synth._orthonormal(m, len(s), seed, 1)
    V = synth._orthonormal(n, len(s), seed, 2)
    return U, np.asarray(s, dtype=np.float64), V, (U * s) @ V.T


def test_mode_residual_zero_for_exact_svd():
    U, s, V, S = _svd_matrix(300, 80, np.exp(-0.2 * np.arange(40)), 3)
    A = (s[:10, None] * V[:, :10].T)
    rho, per = ow.mode_residual(S, U[:, :10], s[:10], A)
    assert rho < 1e-13 and per.shape == (10,)


def test_mode_residual_of_a_shifted_sigma():
    # sigma_k replaced by sigma_k + d: r_k = S v_k - (sigma_k + d) u_k = -d u_k, residual d / (sigma_k + d)
    U, s, V, S = _svd_matrix(200, 60, 1.0 / (1.0 + np.arange(30)), 5)
    st = s[:5].copy()
    st[3] += 1e-3
    A = st[:, None] * V[:, :5].T           # the coefficients follow sigma (A = Sigma V^T)
    rho, per = ow.mode_residual(S, U[:, :5], st, A)
    assert per[3] == pytest.approx(1e-3 / st[3], rel=1e-9)
    assert np.max(np.delete(per, 3)) < 1e-13 and rho == per[3]


def test_mode_residual_of_a_tilted_one_dimensional_basis():
    # Rayleigh-Ritz on q = cos(t) u_1 + sin(t) u_2: sigma~^2 = c^2 s1^2 + s^2 s2^2, v = S^T q / sigma~ and
    # r = S v - sigma~ q = [c (s1^2 - sigma~^2) u_1 + s (s2^2 - sigma~^2) u_2] / sigma~ (closed form)
    U, s, V, S = _svd_matrix(150, 40, [3.0, 1.5, 0.5, 0.1], 7)
    t = 0.05
    c, sn = np.cos(t), np.sin(t)
    q = c * U[:, 0] + sn * U[:, 1]
    st = np.sqrt(c * c * s[0] ** 2 + sn * sn * s[1] ** 2)
    A = (S.T @ q)[None, :]                  # A = phi^T S
    rho, _ = ow.mode_residual(S, q[:, None], np.array([st]), A)
    want = np.hypot(c * (s[0] ** 2 - st * st), sn * (s[1] ** 2 - st * st)) / st / st
    assert rho == pytest.approx(want, rel=1e-10)
    assert rho > 1e-3


def _family_case(seed=0, r=8, n=120):
    fam = synth.ParamFamily(16, 32, n_cand=60, K=40, family_seed=seed)
    mu, mu_hat = synth.draw_params(6, seed=seed)
    mats = [fam.matrix(mu[i], n, noise_std=0.0, seed=10 + i)["St"] for i in range(6)]
    bases = [pod.pod_svd(M.T, r)[0] for M in mats[:4]]
    return fam, mu, mats, bases


def test_continued_fallback_equals_plain_iterations_from_the_warm_basis():
    fam, mu, mats, bases = _family_case()
    S = mats[5].T
    r, p = 8, 4
    om = philox.gaussian_sketch(11, S.shape[1], p)
    c = np.full(4, 0.25)
    # tol 0: always continue; the result equals warm rPOD with q + q_fb iterations
    P1, s1, A1, ex1 = ow.warm_rpod_continued(S, bases, c, 0, r, om, q=0, tol=0.0, q_fb=2)
    P2, s2, A2, ex2 = ow.warm_rpod(S, bases, c, 0, r, om, q=2)
    assert ex1["fell_back"] and ex1["rho"] > 0
    assert metrics.sigma_rel_err(s1, s2) < 1e-13
    assert metrics.sin_theta_max(P1, P2) < 1e-10
    # tol 1: never continues; the result is the warm one
    P3, s3, _, ex3 = ow.warm_rpod_continued(S, bases, c, 0, r, om, q=0, tol=1.0, q_fb=2)
    P4, s4, _, _ = ow.warm_rpod(S, bases, c, 0, r, om, q=0)
    assert not ex3["fell_back"] and np.array_equal(s3, s4)


def test_residual_rule_bounds_the_sigma_error():
    # whenever rho <= tol, every returned sigma lies within (about) tol of a singular value of S
    fam, mu, mats, bases = _family_case(seed=1)
    for i in (4, 5):
        S = mats[i].T
        s_true = np.linalg.svd(S, compute_uv=False)
        for q in (0, 1):
            om = philox.gaussian_sketch(20 + i, S.shape[1], 4)
            P, s, A, ex = ow.warm_rpod(S, bases, np.full(4, 0.25), 0, 8, om, q=q)
            rho, per = ow.mode_residual(S, P, s, A)
            d = np.min(np.abs(s_true[None, :] - s[:, None]), axis=1) / s
            assert np.all(d <= per * (1 + 1e-9) + 1e-12)
