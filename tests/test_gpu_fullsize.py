"""GPU parity at the benchmark's full sizes, in the launch configuration the
benchmark times (default plans, the same generators and seeds).

* Plain FP32, S 262144 x 5000 (512 x 512 grid, 200-mode Fourier field), r = 50,
  p = 10, q = 2: compared with the oracle's O2 on the whole matrix (FP64 on
  the host, a few seconds), FP32 tolerances.
* Mixed BF16, S 1048576 x 10000 (1024 x 1024 grid), r = 100, p = 20, q = 2:
  compared with the oracle's O2 on the same BF16 matrix, upcast exactly to
  FP64 on the host (about 84 GB, streamed by row blocks; a minute or so of
  FP64 BLAS), mixed-path tolerances.
"""

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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_fp32_headline_full_size():
    nx, ny, n, r, p, q, seed = 512, 512, 5000, 50, 10, 2, 2
    g = synth.fourier_field(nx, ny, n, n_modes=200, beta=1.5, phi=0.95, noise_std=1e-4, seed=2,
                            dtype=np.float32)
    St = g["St"]
    m = nx * ny
    say(f"[full fp32] m={m} n={n} r={r} p={p} q={q} seed={seed}")
    Sd = torch.from_numpy(St).to(DEV)
    plan = rp.Plan(m, n, r, p, q, dtype=torch.float32, device=DEV)
    Phi_t, sig, A_t = plan.compute(Sd, seed)
    torch.cuda.synchronize()
    flags = plan.last_flags
    plan.close()
    Phi = Phi_t.double().cpu().numpy().T
    A = A_t.double().cpu().numpy().T
    s = sig.cpu().numpy()
    del Sd, Phi_t, A_t
    S64 = np.ascontiguousarray(St.T, dtype=np.float64)
    del St, g
    om = philox.gaussian_sketch(seed, n, r + p).astype(np.float32).astype(np.float64)
    P2, s2, A2, ex = orpod.rpod_stable(S64, r, om, q)
    res = dict(sigma=metrics.sigma_rel_err(s, s2), orth=metrics.orth_err(Phi))
    if metrics.gap_ok(ex["ritz"], r):
        res["sin"] = metrics.sin_theta_max(Phi, P2)
        res["A"] = metrics.lowrank_rel_diff(Phi, A, P2, A2)
    say(f"[full fp32] flags={flags} {res}")
    assert flags == 0
    assert np.all(np.diff(s) <= 0)
    assert res["sigma"] <= 1e-5 and res["orth"] <= 1e-5
    assert res.get("sin", 0.0) <= 1e-4 and res.get("A", 0.0) <= 1e-4


def host_fp64(St_dev, chunk=500):
    """FP64 host copy (n x m) of a device snapshot matrix, exact for 16-bit and FP32 entries."""
    n, m = St_dev.shape
    out = np.empty((n, m), dtype=np.float64)
    o = torch.from_numpy(out)
    for t0 in range(0, n, chunk):
        o[t0:t0 + chunk].copy_(St_dev[t0:t0 + chunk].to(torch.float64))
    return out


def test_bf16_mixed_full_size_against_oracle():
    """The mixed-precision workload at full size against O2 on the same BF16 S
    (upcast exactly to FP64 on the host, about 84 GB) and the same BF16-rounded
    sketch, with the mixed-path tolerances; the coefficients through
    Sigma_r V_r^T of the oracle's small SVD (exact given its T = Q^T S)."""
    nx, ny, n, r, p, q, seed = 1024, 1024, 10000, 100, 20, 2, 3
    m = nx * ny
    say(f"[full bf16] m={m} n={n} r={r} p={p} q={q} seed={seed}")
    St = synth.fourier_field_device(nx, ny, n, seed=3, dtype=torch.bfloat16, device=DEV)["St"]
    plan = rp.Plan(m, n, r, p, q, dtype=torch.bfloat16, device=DEV)
    Phi_t, sig, A_t = plan.compute(St, seed)
    torch.cuda.synchronize()
    flags = plan.last_flags
    plan.close()
    s = sig.cpu().numpy()
    Phi = Phi_t.double().cpu().numpy().T        # (m, r)
    A = A_t.double().cpu().numpy().T            # (r, n)
    del Phi_t, A_t
    S64 = host_fp64(St)
    del St
    torch.cuda.empty_cache()
    om = philox.gaussian_sketch(seed, n, r + p).astype(np.float32)
    om = torch.from_numpy(om).to(torch.bfloat16).double().numpy()
    P2, s2, A2, ex = orpod.rpod_stable(pod.SnapshotMajor(S64), r, om, q, block_rows=32768, literal_A=False)
    res = dict(sigma=metrics.sigma_rel_err(s, s2), orth=metrics.orth_err(Phi))
    if metrics.gap_ok(ex["ritz"], r):
        res["sin"] = metrics.sin_theta_max(Phi, P2)
        res["A"] = metrics.lowrank_rel_diff(Phi, A, P2, A2)
    say(f"[full bf16] flags={flags} {res}")
    assert flags == 0
    assert np.all(np.diff(s) <= 0)
    assert res["sigma"] <= 1e-3 and res["orth"] <= 1e-5
    assert res.get("sin", 0.0) <= 1e-3 and res.get("A", 0.0) <= 1e-3


@pytest.mark.parametrize("dtype,p", [(torch.float32, 20), (torch.bfloat16, 75)])
def test_paper_shape_wide(dtype, p):
    """The paper's own shape, wide: S 8192 x 90225 (64 x 128 cells, 225
    parameter blocks x 401 steps), r = 10, q = 1, psi-like field (beta 2):
    against O2 on the same stored values with the same rounded sketch."""
    nx, ny, n, r, q, seed = 64, 128, 90225, 10, 1, 17
    m = nx * ny
    say(f"[paper wide] m={m} n={n} r={r} p={p} q={q} dtype={dtype} seed={seed}")
    g = synth.fourier_field_device(nx, ny, n, beta=2.0, seed=seed, dtype=dtype, device=DEV)
    Sd = g["St"]
    plan = rp.Plan(m, n, r, p, q, dtype=dtype, device=DEV)
    Phi_t, sig, A_t = plan.compute(Sd, seed)
    torch.cuda.synchronize()
    flags = plan.last_flags
    plan.close()
    Phi = Phi_t.double().cpu().numpy().T
    A = A_t.double().cpu().numpy().T
    s = sig.cpu().numpy()
    S64 = Sd.double().cpu().numpy().T          # the stored values, exactly
    del Sd, g
    om = philox.gaussian_sketch(seed, n, r + p)
    om = torch.from_numpy(om.astype(np.float32)).to(dtype).double().numpy()
    P2, s2, A2, ex = orpod.rpod_stable(S64, r, om, q)
    res = dict(sigma=metrics.sigma_rel_err(s, s2), orth=metrics.orth_err(Phi))
    gap = metrics.gap_ok(ex["ritz"], r)
    if gap:
        res["sin"] = metrics.sin_theta_max(Phi, P2)
        res["A"] = metrics.lowrank_rel_diff(Phi, A, P2, A2)
    say(f"[paper wide] flags={flags} gap={gap} {res}")
    tol = dict(sigma=1e-5, sin=1e-4, A=1e-4) if dtype == torch.float32 else dict(sigma=1e-3, sin=1e-3, A=1e-3)
    assert flags == 0
    assert np.all(np.diff(s) <= 0)
    assert res["sigma"] <= tol["sigma"] and res["orth"] <= 1e-5, res
    assert gap and res["sin"] <= tol["sin"] and res["A"] <= tol["A"], res
