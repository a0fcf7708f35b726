"""Pins for the CPU oracle (no GPU).

Each test ties the oracle to something other than itself: published
known-answer vectors, closed forms of the synthetic generators, brute force
on tiny inputs, special cases where randomized POD reduces to the exact SVD,
and the expected-error bounds of Halko, Martinsson and Tropp (SIAM Review
53(2), 2011, Thm 10.5 and Cor. 10.10).
"""

import math
import os

import numpy as np
import pytest
from scipy import stats

from oracle import metrics, philox, pod, rpod
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Philox4x32-10 and the Gaussian sketch (Sec. 4.2, Alg. 1 step 1)
# --------------------------------------------------------------------------

def _kat_rows():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,want", _kat_rows())
def test_philox_known_answers(ctr, key, want):
    got = philox.philox4x32_10(ctr, key)
    assert [int(x) for x in got] == want


def test_philox_vectorised_matches_scalar():
    bits = philox.sketch_bits(seed=0x123456789ABCDEF, n=7, l=5)
    for j in range(7):
        for t in range(3):
            one = philox.philox4x32_10([j, 0, t, 0], [0x89ABCDEF, 0x01234567])
            assert [int(x) for x in one] == [int(x) for x in bits[j, t]]


def test_sketch_is_standard_normal():
    g = philox.gaussian_sketch(seed=7, n=50000, l=6).ravel()
    assert abs(g.mean()) < 5 * 1 / math.sqrt(g.size)
    assert abs(g.var() - 1.0) < 5 * math.sqrt(2.0 / g.size)
    assert stats.kstest(g, "norm").pvalue > 1e-3
    # the cos and sin halves of one Box-Muller pair are uncorrelated
    G = philox.gaussian_sketch(seed=8, n=100000, l=2)
    assert abs(np.corrcoef(G[:, 0], G[:, 1])[0, 1]) < 5 / math.sqrt(100000)


def test_sketch_extreme_bits_are_finite():
    lo = np.zeros((1, 1, 4), dtype=np.uint32)
    hi = np.full((1, 1, 4), 0xFFFFFFFF, dtype=np.uint32)
    g_lo = philox.bits_to_gaussian(lo, 2)
    g_hi = philox.bits_to_gaussian(hi, 2)
    assert np.all(np.isfinite(g_lo)) and np.all(np.isfinite(g_hi))
    # u1 -> smallest value gives the largest radius sqrt(-2 ln(2^-54))
    assert abs(g_lo[0, 0] - math.sqrt(-2 * math.log(0.5 * 2.0 ** -53))) < 1e-12
    assert np.all(np.abs(g_hi) < 1e-7)          # u1 -> 1 gives radius ~ 0


def test_sketch_column_prefix_and_seed():
    a = philox.gaussian_sketch(seed=3, n=40, l=7)
    b = philox.gaussian_sketch(seed=3, n=40, l=12)
    assert np.array_equal(a, b[:, :7])              # columns do not depend on l
    c = philox.gaussian_sketch(seed=4, n=40, l=7)
    assert not np.allclose(a, c)


# --------------------------------------------------------------------------
# Generators: closed forms
# --------------------------------------------------------------------------

def test_lowrank_generator_closed_form():
    g = synth.lowrank_exp(300, 60, decay=0.1, noise_std=0.0, seed=1)
    s = np.linalg.svd(g["St"].T, compute_uv=False)
    assert np.max(np.abs(s - g["sigma"]) / g["sigma"]) < 1e-12
    assert np.max(np.abs(g["U"].T @ g["U"] - np.eye(60))) < 1e-13


def test_fourier_basis_orthogonal():
    nx, ny = 32, 24
    modes, _ = synth.fourier_modes(nx, ny, 60)
    F = synth.fourier_basis(nx, ny, modes)
    G = F.T @ F
    assert np.max(np.abs(G - np.eye(60) * nx * ny / 4.0)) < 1e-10


def test_fourier_modes_order():
    modes, kmag = synth.fourier_modes(64, 64, 200)
    assert np.all(np.diff(kmag) >= -1e-12)
    assert tuple(modes[0]) == (1, 1) and tuple(modes[1]) == (1, 2)
    assert len({tuple(x) for x in modes}) == 200


def _fourier_exact_sigma(gen):
    # S0 = F diag(amp) T^T and F = (sqrt(nx ny)/2) F_hat with F_hat orthonormal
    return pod.pod_sigma_sine_field(gen["amp"], gen["T"], gen["nx"], gen["ny"])


def test_fourier_field_pins_pod_sigma():
    g = synth.fourier_field(24, 32, 150, n_modes=60, noise_std=0.0, seed=5)
    exact = _fourier_exact_sigma(g)
    _, s, _, s_all = pod.pod_svd(g["St"].T, 30)
    assert np.max(np.abs(s_all[:60] - exact) / exact) < 1e-11
    assert np.max(s_all[60:]) < 1e-12 * s_all[0]        # rank is exactly 60


def test_generator_chunking_invariant():
    a = synth.fourier_field(16, 16, 70, n_modes=20, seed=9, col_block=512)["St"]
    b = synth.fourier_field(16, 16, 70, n_modes=20, seed=9, col_block=16)["St"]
    assert np.array_equal(a, b)


# --------------------------------------------------------------------------
# O1: exact POD (Sec. 4.1, thin SVD; coefficients of Sec. 4.3)
# --------------------------------------------------------------------------

def _jacobi_eigvals(M, sweeps=60):
    """Textbook cyclic two-sided Jacobi eigenvalue iteration, pure Python."""
    A = [list(map(float, row)) for row in M]
    n = len(A)
    for _ in range(sweeps):
        off = sum(A[i][j] ** 2 for i in range(n) for j in range(n) if i != j)
        if off < 1e-300:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                if A[p][q] == 0.0:
                    continue
                theta = (A[q][q] - A[p][p]) / (2 * A[p][q])
                t = (1.0 if theta >= 0 else -1.0) / (abs(theta) + math.sqrt(theta * theta + 1))
                c = 1 / math.sqrt(t * t + 1)
                s = t * c
                for k in range(n):
                    akp, akq = A[k][p], A[k][q]
                    A[k][p], A[k][q] = c * akp - s * akq, s * akp + c * akq
                for k in range(n):
                    apk, aqk = A[p][k], A[q][k]
                    A[p][k], A[q][k] = c * apk - s * aqk, s * apk + c * aqk
    return sorted((A[i][i] for i in range(n)), reverse=True)


def test_pod_brute_force_tiny():
    S = np.random.default_rng(11).standard_normal((8, 6))
    lam = _jacobi_eigvals((S.T @ S).tolist())
    _, s, _, s_all = pod.pod_svd(S, 6)
    assert np.max(np.abs(np.sqrt(lam) - s_all) / s_all) < 1e-13


def test_pod_closed_form_modes():
    g = synth.lowrank_exp(500, 80, decay=0.1, noise_std=0.0, seed=2)
    S = g["St"].T
    Phi, s, A, _ = pod.pod_svd(S, 20)
    assert metrics.sigma_rel_err(s, g["sigma"][:20]) < 1e-13
    assert metrics.sin_theta_max(Phi, g["U"][:, :20]) < 1e-12
    assert metrics.orth_err(Phi) < 1e-12
    # per mode: Phi_k = +-U_k, and A = Sigma_r V_r^T up to the same signs
    sgn = np.sign(np.sum(Phi * g["U"][:, :20], axis=0))
    assert np.max(np.abs(Phi - g["U"][:, :20] * sgn)) < 1e-11
    assert np.max(np.abs(A - (g["V"][:, :20] * g["sigma"][:20] * sgn).T)) < 1e-12


def test_pod_routes_agree_and_invariants():
    g = synth.lowrank_exp(4096, 200, decay=0.1, noise_std=1e-4, seed=1)
    S = g["St"].T
    r = 20
    P1, s1, A1, sall = pod.pod_svd(S, r)
    P2, s2, A2, _ = pod.pod_snapshots(S, r)
    P3, s3, A3, _ = pod.pod_tsqr(S, r, block_rows=1000)
    for P, s, A in ((P2, s2, A2), (P3, s3, A3)):
        assert metrics.sigma_rel_err(s, s1) < 1e-11
        assert metrics.sin_theta_max(P, P1) < 1e-9
        assert metrics.lowrank_rel_diff(P, A, P1, A1) < 1e-9
    assert metrics.orth_err(P1) < 1e-12
    assert np.all(np.diff(sall) <= 0)
    assert np.max(np.abs(A1 @ A1.T - np.diag(s1 ** 2))) < 1e-12 * s1[0] ** 2
    assert np.sum(sall ** 2) <= np.sum(S ** 2) * (1 + 1e-12)
    # sign convention: largest-magnitude entry of every mode is positive
    idx = np.argmax(np.abs(P1), axis=0)
    assert np.all(P1[idx, np.arange(r)] > 0)


def test_pod_wide_matrix_snapshots():
    S = np.random.default_rng(3).standard_normal((40, 90)) * np.exp(-0.2 * np.arange(40))[:, None]
    P1, s1, A1, _ = pod.pod_svd(S, 10)
    P2, s2, A2, _ = pod.pod_snapshots(S, 10)
    assert metrics.sigma_rel_err(s2, s1) < 1e-10
    assert metrics.sin_theta_max(P2, P1) < 1e-8


# --------------------------------------------------------------------------
# O2: randomized POD, Alg. 1 of Sec. 4.2
# --------------------------------------------------------------------------

def test_rpod_equals_pod_when_sketch_covers_rank():
    # exact rank 12 matrix; l = 15 >= rank, so the range finder is exact
    g = synth.lowrank_exp(300, 12, decay=0.3, noise_std=0.0, seed=4)
    U, V, sig = g["U"], g["V"], g["sigma"]
    W = synth._orthonormal(70, 12, 4, 9)        # 70 snapshots, rank 12
    S = U @ np.diag(sig) @ W.T
    om = philox.gaussian_sketch(5, 70, 15)
    P2, s2, A2, _ = rpod.rpod_stable(S, 8, om, q=0)
    P1, s1, A1, _ = pod.pod_svd(S, 8)
    assert metrics.sigma_rel_err(s2, s1) < 1e-12
    assert metrics.sin_theta_max(P2, P1) < 1e-10
    assert metrics.lowrank_rel_diff(P2, A2, P1, A1) < 1e-10


def test_rpod_full_sketch_equals_svd():
    S = np.random.default_rng(6).standard_normal((120, 40))
    om = philox.gaussian_sketch(1, 40, 40)
    P2, s2, A2, _ = rpod.rpod_stable(S, 10, om, q=1)
    P1, s1, A1, _ = pod.pod_svd(S, 10)
    assert metrics.sigma_rel_err(s2, s1) < 1e-12
    assert metrics.sin_theta_max(P2, P1) < 1e-9


def test_rpod_interlacing_and_coefficients():
    g = synth.lowrank_exp(1000, 200, decay=0.05, noise_std=1e-4, seed=7)
    S = g["St"].T
    om = philox.gaussian_sketch(2, 200, 30)
    P, s, A, ex = rpod.rpod_stable(S, 20, om, q=1)
    _, _, _, s_true = pod.pod_svd(S, 20)
    assert np.all(ex["ritz"] <= s_true[:30] * (1 + 1e-12))      # sigma_k(Q^T S) <= sigma_k(S)
    # A = Phi^T S (literal) equals Sigma_r V_r^T of the small SVD
    assert np.max(np.abs(A - s[:, None] * ex["Vt_r"])) < 1e-12 * s[0]
    assert np.max(np.abs(A @ A.T - np.diag(s ** 2))) < 1e-12 * s[0] ** 2
    assert metrics.orth_err(P) < 1e-13
    # the shortcut for very large S (no literal pass) returns the same coefficients, signs included
    P2, s2, A2, _ = rpod.rpod_stable(S, 20, om, q=1, literal_A=False)
    assert np.array_equal(P2, P) and np.array_equal(s2, s)
    assert np.max(np.abs(A2 - A)) < 1e-12 * s[0]


def test_rpod_literal_equals_stable():
    g = synth.lowrank_exp(4096, 200, decay=0.1, noise_std=1e-4, seed=1)
    S = g["St"].T
    om = philox.gaussian_sketch(1, 200, 30)
    Pa, sa, Aa, _ = rpod.rpod_stable(S, 20, om, q=1)
    Pb, sb, Ab, _ = rpod.rpod_literal(S, 20, om, q=1)
    assert metrics.sigma_rel_err(sa, sb) < 1e-12
    assert metrics.sin_theta_max(Pa, Pb) < 1e-10
    assert metrics.lowrank_rel_diff(Pa, Aa, Pb, Ab) < 1e-10


def _proj_err(S, Q, ord_):
    E = S - Q @ (Q.T @ S)
    return np.linalg.norm(E, ord_)


def test_hmt_frobenius_bound_q0():
    # HMT 2011 Thm 10.5: E||(I-P_Y)S||_F <= (1 + k/(p-1))^1/2 (sum_{j>k} s_j^2)^1/2
    g = synth.lowrank_exp(400, 120, decay=0.1, noise_std=0.0, seed=3)
    S = g["St"].T
    s = g["sigma"]
    k, p = 10, 5
    errs = []
    for seed in range(200):
        om = philox.gaussian_sketch(seed, 120, k + p)
        _, _, _, ex = rpod.rpod_stable(S, k, om, q=0)
        errs.append(_proj_err(S, ex["Q"], "fro"))
    bound = math.sqrt(1 + k / (p - 1)) * math.sqrt(np.sum(s[k:] ** 2))
    tail = math.sqrt(np.sum(s[k + p:] ** 2))      # no l-column basis beats this
    assert np.mean(errs) <= bound
    assert min(errs) >= tail * (1 - 1e-12)


@pytest.mark.parametrize("q", [1, 2])
def test_hmt_power_scheme_spectral_bound(q):
    # HMT 2011 Cor. 10.10, spectral error of the power scheme (S S^T)^q S Omega
    g = synth.lowrank_exp(400, 120, decay=0.1, noise_std=0.0, seed=3)
    S = g["St"].T
    s = g["sigma"]
    k, p = 10, 5
    errs = []
    for seed in range(100):
        om = philox.gaussian_sketch(seed, 120, k + p)
        _, _, _, ex = rpod.rpod_stable(S, k, om, q=q)
        errs.append(_proj_err(S, ex["Q"], 2))
    e = 2 * q + 1
    bound = ((1 + math.sqrt(k / (p - 1))) * s[k] ** e
             + math.e * math.sqrt(k + p) / p * math.sqrt(np.sum(s[k:] ** (2 * e)))) ** (1 / e)
    assert np.mean(errs) <= bound
    assert min(errs) >= s[k + p] * (1 - 1e-12)      # Eckart-Young floor


def test_rpod_error_falls_with_q_and_p():
    # Sec. 5 (p-study) and Sec. 4.2 (subspace iterations): accuracy improves with p and q
    g = synth.fourier_field(32, 32, 400, n_modes=200, noise_std=1e-4, seed=12)
    S = g["St"].T
    _, s_true, _, _ = pod.pod_svd(S, 10)

    def err(p, q):
        e = []
        for seed in range(5):
            om = philox.gaussian_sketch(seed, S.shape[1], 10 + p)
            _, s, _, _ = rpod.rpod_stable(S, 10, om, q=q)
            e.append(metrics.sigma_rel_err(s, s_true))
        return np.mean(e)

    e_p0, e_p20, e_p75 = err(0, 0), err(20, 0), err(75, 0)
    assert e_p0 > e_p20 > e_p75
    assert err(5, 0) > err(5, 1) > err(5, 2)


def test_snapshot_major_view_gives_identical_oracle_results():
    # the oracle on S held snapshot-major (transposed row-block views) equals the oracle on S itself
    # (to rounding: BLAS takes the transposed operands in another summation order)
    St = np.random.default_rng(4).standard_normal((120, 3000))
    om = philox.gaussian_sketch(5, 120, 25)
    a = rpod.rpod_stable(St.T.copy(), 15, om, 2, block_rows=700)
    b = rpod.rpod_stable(pod.SnapshotMajor(St), 15, om, 2, block_rows=700)
    assert metrics.sigma_rel_err(b[1], a[1]) < 1e-13
    assert metrics.sin_theta_max(b[0], a[0]) < 1e-12
    assert metrics.lowrank_rel_diff(b[0], b[2], a[0], a[2]) < 1e-12
