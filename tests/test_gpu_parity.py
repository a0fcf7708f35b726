"""GPU parity: the HIP path through the C ABI against the CPU FP64 oracle.

Every case draws S from the seeded generators, runs rpod_compute on the GPU,
and compares with O2 (the oracle's randomized POD on the *same* sketch, the
sketch rounded to the path's precision exactly as the device rounds it) by
sign- and rotation-invariant metrics. Tolerances:
  FP64 path: sigma rel 1e-12, sin(theta) 1e-10, orthogonality 1e-13, A 1e-11
  FP32 path: sigma rel 1e-5,  sin(theta) 1e-4,  orthogonality 1e-5,  A 1e-4
"""

import math
import sys

import numpy as np
import pytest
import torch

import paper_2504_15350_amd as rp
import synth
from oracle import metrics, philox, pod
from oracle import rpod as orpod

pytestmark = pytest.mark.gpu
DEV = "cuda"

TOL = {
    torch.float64: dict(sigma=1e-12, sin=1e-10, orth=1e-13, A=1e-11),
    torch.float32: dict(sigma=1e-5, sin=1e-4, orth=1e-5, A=1e-4),
    torch.bfloat16: dict(sigma=1e-3, sin=1e-3, orth=1e-5, A=1e-3),
    torch.float16: dict(sigma=1e-3, sin=1e-3, orth=1e-5, A=1e-3),
}
NPDT = {torch.float64: np.float64, torch.float32: np.float32}
HALF = (torch.bfloat16, torch.float16)


def round_to(x, dtype):
    """Round an FP64 array to dtype as the device does (16-bit types through FP32)."""
    if dtype in HALF:
        return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dtype)
    return torch.from_numpy(np.ascontiguousarray(x.astype(NPDT[dtype])))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def upload(St, dtype, ld=None):
    """Round St (n, m) to dtype on the host, upload with leading dimension ld."""
    n, m = St.shape
    ld = m if ld is None else ld
    Sr = round_to(St, dtype)
    buf = torch.zeros((n, ld), dtype=dtype)
    buf[:, :m] = Sr
    return buf.to(DEV), Sr.double().numpy().T          # device (n, ld), oracle S (m, n)


def sketch_for(seed, n, l, dtype):
    om = philox.gaussian_sketch(seed, n, l)
    return round_to(om, dtype).double().numpy()


def run_gpu(Sd, m, n, r, p, q, seed, dtype):
    plan = rp.Plan(m, n, r, p, q, dtype=dtype, ld=Sd.stride(0), device=DEV)
    Phi_t, sig, A_t = plan.compute(Sd, seed)
    torch.cuda.synchronize()
    out = (Phi_t.double().cpu().numpy().T, sig.cpu().numpy(), A_t.double().cpu().numpy().T)
    say(f"[gpu] flags={plan.last_flags}")
    plan.close()
    return out


def compare(gpu, ref, dtype, r, ritz):
    Phi, sig, A = gpu
    Pr, sr, Ar = ref
    tol = TOL[dtype]
    res = dict(sigma=metrics.sigma_rel_err(sig, sr), orth=metrics.orth_err(Phi))
    assert np.all(np.diff(sig) <= 0), "sigma must be descending"
    assert res["sigma"] <= tol["sigma"], res
    assert res["orth"] <= tol["orth"], res
    if metrics.gap_ok(ritz, r):
        res["sin"] = metrics.sin_theta_max(Phi, Pr)
        res["A"] = metrics.lowrank_rel_diff(Phi, A, Pr, Ar)
        assert res["sin"] <= tol["sin"], res
        assert res["A"] <= tol["A"], res
    # the device applies the sign convention to its own modes
    idx = np.argmax(np.abs(Phi), axis=0)
    assert np.all(Phi[idx, np.arange(r)] > 0)
    return res


def case(St, r, p, q, seed, dtype, ld=None, name=""):
    n, m = St.shape
    say(f"[case] {name} m={m} n={n} r={r} p={p} q={q} seed={seed} dtype={dtype} ld={ld}")
    Sd, S64 = upload(St, dtype, ld)
    gpu = run_gpu(Sd, m, n, r, p, q, seed, dtype)
    om = sketch_for(seed, n, r + p, dtype)
    P2, s2, A2, ex = orpod.rpod_stable(S64, r, om, q)
    res = compare(gpu, (P2, s2, A2), dtype, r, ex["ritz"])
    say(f"[case] {name} ok {res}")
    return res, gpu, (P2, s2, A2, ex), S64


# ---------------------------------------------------------------------------
# sketch
# ---------------------------------------------------------------------------

def test_sketch_bits_bit_exact():
    seed = 0xDEADBEEF12345678
    got = rp.sketch_bits(seed, 1000, 37).cpu().numpy().view(np.uint32)
    want = philox.sketch_bits(seed, 1000, 37)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16, torch.float16])
def test_sketch_values(dtype):
    seed, n, l = 12345, 3001, 23
    g = rp.generate_omega(seed, n, l, dtype=dtype).double().cpu().numpy().T
    want = philox.gaussian_sketch(seed, n, l)
    if dtype == torch.float64:
        assert np.max(np.abs(g - want) / np.maximum(1.0, np.abs(want))) < 1e-14
    else:
        # the device rounds its FP64 Gaussian exactly as round_to(); the two
        # FP64 values may differ in the last bit, so allow one unit of the
        # narrow type where they straddle a rounding boundary
        wr = round_to(want, dtype).double().numpy()
        eps = {torch.float32: 2.0 ** -23, torch.bfloat16: 2.0 ** -7, torch.float16: 2.0 ** -10}[dtype]
        assert np.all(np.abs(g - wr) <= eps * np.maximum(np.abs(wr), 2.0 ** -14))
        assert np.mean(g == wr) > 0.9999


# ---------------------------------------------------------------------------
# plain rPOD parity
# ---------------------------------------------------------------------------

def test_c1_fp64_full_size():
    """4096 x 200, U diag(exp(-0.1k)) V^T + noise (std 1e-4), r=20, p=10, q=1, FP64."""
    g = synth.lowrank_exp(4096, 200, decay=0.1, noise_std=1e-4, seed=1)
    res, gpu, ref, S64 = case(g["St"], 20, 10, 1, 1, torch.float64, name="c1")
    _, s1, _, _ = pod.pod_svd(S64, 20)
    say("[c1] O2 vs O1 sigma rel err", metrics.sigma_rel_err(ref[1], s1))


def test_fp32_fourier_field():
    g = synth.fourier_field(128, 128, 1000, n_modes=200, noise_std=1e-4, seed=2, dtype=np.float64)
    case(g["St"], 50, 10, 2, 2, torch.float32, name="fourier-fp32")


def test_fp64_fourier_field_l128():
    g = synth.fourier_field(64, 64, 700, n_modes=200, noise_std=1e-4, seed=3)
    case(g["St"], 100, 28, 1, 5, torch.float64, name="fourier-fp64-l128")


@pytest.mark.parametrize("m,n,r,p,q,dtype,ldpad", [
    (1000, 77, 5, 3, 0, torch.float64, 0),
    (1000, 77, 5, 3, 2, torch.float32, 0),
    (4099, 301, 17, 9, 1, torch.float64, 3),     # odd leading dimension: scalar loads
    (4099, 301, 17, 9, 1, torch.float32, 5),
    (257, 513, 30, 20, 1, torch.float32, 0),     # wide matrix
    (40, 30, 20, 10, 0, torch.float64, 0),       # l == n == min(m, n)
    (300, 40, 1, 0, 3, torch.float64, 0),        # r = 1, p = 0
    (70000, 150, 33, 15, 2, torch.float32, 0),   # several row tiles and K splits
    (20011, 600, 100, 28, 1, torch.float32, 0),  # l = 128: eight column tiles on every FP32 kernel
])
def test_ragged_shapes(m, n, r, p, q, dtype, ldpad):
    g = synth.lowrank_exp(m, n, decay=0.08, noise_std=1e-5, seed=m + n)
    case(g["St"], r, p, q, 7, dtype, ld=m + ldpad if ldpad else None, name="ragged")


def test_sketch_covers_rank_matches_exact_pod():
    # exact rank 30 with l = 30: the range finder is exact, O2 == O1
    m, n = 500, 30
    S = np.random.default_rng(3).standard_normal((n, m)) * np.exp(-0.1 * np.arange(1, n + 1))[:, None]
    res, gpu, ref, S64 = case(S, 20, 10, 0, 9, torch.float64, name="l=n")
    P1, s1, A1, _ = pod.pod_svd(S64, 20)
    assert metrics.sigma_rel_err(gpu[1], s1) < 1e-12
    assert metrics.sin_theta_max(gpu[0], P1) < 1e-10


def _graded(m, n, decades_over_r, r, seed):
    """Noise-free S = U diag(sigma) V^T with sigma_k = 10^(-d (k - 1) / (r - 1)), k = 1..n: sigma_1 / sigma_r
    = 10^d exactly (U, V the seeded orthonormal factors of the 4096 x 200 generator). Returns St (n, m)."""
    s = 10.0 ** (-decades_over_r * np.arange(n) / (r - 1))
    U = synth._orthonormal(m, n, seed, 1)
    V = synth._orthonormal(n, n, seed, 2)
    return np.ascontiguousarray(((U * s) @ V.T).T)


def test_fp64_graded_spectrum_kappa_1e3():
    """sigma_1 / sigma_r = 1e3 at the flat FP64 tolerances. Through the Gram matrix T T^T the small SVD
    would lose about u (sigma_1 / sigma_k)^2 ~ 1e-10 on sigma_20; the FP64 path factors T^T itself."""
    St = _graded(4096, 200, 3.0, 20, 31)
    res, *_ = case(St, 20, 10, 1, 7, torch.float64, name="graded 1e3")
    assert res["sigma"] <= 1e-12


def test_fp64_graded_spectrum_kappa_1e6():
    """sigma_1 / sigma_r = 1e6 (sigma_l / sigma_1 ~ 6e-10: every orthonormalisation takes the shifted
    retry). Both the device and the oracle resolve sigma_k to about u sigma_1 absolute (backward-stable
    factorisations), so the bound is 1e-12 sigma_k + 1e3 u sigma_1, and the subspace bound is that
    absolute error over the gap after mode r; the squared route would leave ~u (sigma_1/sigma_k)^2 = 1e-4."""
    m, n, r, p, q, seed = 4096, 200, 20, 10, 1, 8
    St = _graded(m, n, 6.0, r, 32)
    say(f"[case] graded 1e6 m={m} n={n} r={r} p={p} q={q} seed={seed} float64")
    Sd, S64 = upload(St, torch.float64)
    Phi, sig, A = run_gpu(Sd, m, n, r, p, q, seed, torch.float64)
    om = sketch_for(seed, n, r + p, torch.float64)
    P2, s2, A2, ex = orpod.rpod_stable(S64, r, om, q)
    u = 2.0 ** -53
    bound = 1e-12 * s2 + 1e3 * u * s2[0]
    err = np.abs(sig - s2)
    say(f"[case] graded 1e6 sigma abs err / bound max {np.max(err / bound):.3f}, rel err sigma_r {err[-1] / s2[-1]:.2e}")
    assert np.all(err <= bound)
    gap = s2[r - 1] - ex["ritz"][r]
    sin = metrics.sin_theta_max(Phi, P2)
    assert sin <= 1e-10 + 1e3 * u * s2[0] / gap, sin
    assert metrics.orth_err(Phi) <= 1e-13
    assert metrics.lowrank_rel_diff(Phi, A, P2, A2) <= 1e-11


def test_fp32_rank_cut_flag():
    """FP32 path, sigma_l / sigma_1 ~ 1e-14: the pivoted Cholesky of the FP64 Gram matrix stops early, the
    informational RANK_CUT flag is raised, and the leading modes still meet the FP32 tolerances."""
    m, n, r, p, q, seed = 4096, 200, 3, 27, 1, 9
    St = _graded(m, n, 1.0, 3, 33)   # sigma_k = 10^(-(k-1)/2)
    Sd, S64 = upload(St, torch.float32)
    plan = rp.Plan(m, n, r, p, q, dtype=torch.float32, device=DEV)
    Phi_t, sig, A_t = plan.compute(Sd, seed)
    flags = plan.status()
    plan.close()
    say(f"[case] rank cut flags={flags}")
    assert flags & rp.FLAG_RANK_CUT and not flags & rp.FLAG_BREAKDOWN
    om = sketch_for(seed, n, r + p, torch.float32)
    P2, s2, A2, ex = orpod.rpod_stable(S64, r, om, q)
    assert metrics.sigma_rel_err(sig.cpu().numpy(), s2) <= 1e-5
    assert metrics.sin_theta_max(Phi_t.double().cpu().numpy().T, P2) <= 1e-4


def test_rank_deficient_fp32():
    # exact rank 5 with l = 12 > rank: trailing sketch directions are noise
    m, n = 3000, 200
    U = synth._orthonormal(m, 5, 1, 1)
    V = synth._orthonormal(n, 5, 1, 2)
    S = (V * np.array([5.0, 4.0, 3.0, 2.0, 1.0])) @ U.T
    Sd, S64 = upload(S, torch.float32)
    Phi, sig, A = run_gpu(Sd, m, n, 4, 8, 1, 3, torch.float32)
    P1, s1, A1, _ = pod.pod_svd(S64, 4)
    assert metrics.sigma_rel_err(sig, s1) < 1e-5
    assert metrics.sin_theta_max(Phi, P1) < 1e-4


def test_deterministic():
    g = synth.fourier_field(64, 64, 500, n_modes=100, noise_std=1e-4, seed=4)
    Sd, _ = upload(g["St"], torch.float32)
    a = run_gpu(Sd, 4096, 500, 20, 10, 2, 11, torch.float32)
    b = run_gpu(Sd, 4096, 500, 20, 10, 2, 11, torch.float32)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


# ---------------------------------------------------------------------------
# mixed precision: 16-bit S, FP32 accumulation, FP64 small ops, refinement pass
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16])
def test_mixed_fourier_r100(dtype):
    g = synth.fourier_field(128, 128, 2000, n_modes=200, noise_std=1e-4, seed=3)
    res, gpu, ref, S64 = case(g["St"], 100, 20, 2, 3, dtype, name="mixed-fourier")


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16])
def test_mixed_lowrank(dtype):
    g = synth.lowrank_exp(4096, 200, decay=0.1, noise_std=1e-4, seed=1)
    case(g["St"], 20, 10, 1, 1, dtype, name="mixed-c1")


@pytest.mark.parametrize("m,n,r,p,q,dtype,ldpad", [
    (1000, 77, 5, 3, 0, torch.bfloat16, 0),
    (4099, 301, 17, 9, 2, torch.bfloat16, 3),    # odd leading dimension: scalar loads
    (4099, 301, 17, 9, 1, torch.float16, 8),
    (70000, 150, 33, 15, 2, torch.bfloat16, 0),
    (257, 513, 30, 20, 1, torch.float16, 0),
    # widths whose 16-column tiles do not divide the S^T Q wave grid (guarded tiles), or do with
    # three wave columns, and widths not a multiple of 32 (separate hi/lo split pass)
    (20000, 400, 60, 15, 1, torch.bfloat16, 0),  # lp 80
    (9000, 700, 70, 20, 1, torch.float16, 8),    # lp 96
    (20001, 500, 90, 15, 2, torch.float16, 0),   # lp 112
    (12000, 600, 50, 55, 1, torch.bfloat16, 5),  # lp 112, odd leading dimension
])
def test_mixed_ragged(m, n, r, p, q, dtype, ldpad):
    g = synth.lowrank_exp(m, n, decay=0.08, noise_std=1e-5, seed=m + n)
    case(g["St"], r, p, q, 7, dtype, ld=m + ldpad if ldpad else None, name="mixed-ragged")


@pytest.mark.parametrize("m,n,r,p,q,dtype,ldpad", [
    (3000, 20000, 20, 10, 1, torch.float64, 0),     # 12 row tiles: the columns split 19 ways
    (3001, 20000, 20, 10, 2, torch.float32, 3),     # odd leading dimension, ragged rows
    (8192, 33333, 10, 75, 1, torch.float32, 0),     # the paper's rows, ragged last split
    (2048, 9000, 30, 20, 1, torch.bfloat16, 0),
    (2049, 9000, 30, 20, 1, torch.float16, 7),
])
def test_short_wide_split_columns(m, n, r, p, q, dtype, ldpad):
    """Short, wide S: S X splits its columns into slabs summed afterwards."""
    g = synth.lowrank_exp(m, n, decay=0.08, noise_std=1e-5, seed=m + n)
    case(g["St"], r, p, q, 7, dtype, ld=m + ldpad if ldpad else None, name="short-wide")


# ---------------------------------------------------------------------------
# degenerate inputs and errors
# ---------------------------------------------------------------------------

def test_zero_matrix_reports_breakdown():
    Sd = torch.zeros((100, 500), dtype=torch.float64, device=DEV)
    plan = rp.Plan(500, 100, 5, 5, 1, dtype=torch.float64, device=DEV)
    with pytest.raises(rp.RpodError) as e:
        plan.compute(Sd, 1)
    assert e.value.status == 6
    assert plan.last_flags & rp.FLAG_BREAKDOWN


@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_nonfinite_input_reported(bad):
    g = synth.lowrank_exp(800, 60, seed=5)
    St = g["St"].copy()
    St[17, 123] = bad
    Sd, _ = upload(St, torch.float32)
    plan = rp.Plan(800, 60, 5, 5, 1, dtype=torch.float32, device=DEV)
    with pytest.raises(rp.RpodError) as e:
        plan.compute(Sd, 1)
    assert e.value.status == 2


def test_plan_reuse_and_compute_errors():
    g = synth.lowrank_exp(600, 80, seed=6)
    Sd, S64 = upload(g["St"], torch.float32)
    plan = rp.Plan(600, 80, 8, 4, 1, dtype=torch.float32, device=DEV)
    a = plan.compute(Sd, 3)
    b = plan.compute(Sd, 4)   # another sketch through the same plan
    om = sketch_for(4, 80, 12, torch.float32)
    P2, s2, _, _ = orpod.rpod_stable(S64, 8, om, 1)
    assert metrics.sigma_rel_err(b[1].cpu().numpy(), s2) < 1e-5
    assert rp.lib().rpod_compute(plan._h, None, 1, None, None, None) == 1
