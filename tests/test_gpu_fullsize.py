"""GPU parity at the benchmark's full sizes, in the launch configuration the
benchmark times (default plans, the same generators and seeds).

* Plain FP32, S 262144 x 5000 (512 x 512 grid, 200-mode Fourier field), r = 50,
  p = 10, q = 2: compared with the oracle's O2 on the whole matrix (FP64 on
  the host, a few seconds), FP32 tolerances.
* Mixed BF16, S 1048576 x 10000 (1024 x 1024 grid), r = 100, p = 20, q = 2:
  too large for the oracle as a whole, so checked on what holds at any size
  and on sampled outputs the oracle computes one by one: Phi orthonormal,
  sigma descending and equal to the row norms of A (A = U_r^T T = Sigma V^T),
  and A[:, j] = Phi^T S[:, j] for sampled snapshots j in FP64.
"""

import sys

import numpy as np
import pytest
import torch

import paper_2504_15350_amd as rp
import synth
from oracle import metrics, philox
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


def test_bf16_mixed_full_size_sampled():
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
    orth = metrics.orth_err(Phi)
    rownorm = np.linalg.norm(A, axis=1)
    cons = float(np.max(np.abs(rownorm - s) / s))
    cols = np.random.default_rng(11).choice(n, size=8, replace=False)
    worst = 0.0
    for j in cols:
        sj = St[int(j)].double().cpu().numpy()  # snapshot j, exact in FP64
        ref = Phi.T @ sj
        worst = max(worst, float(np.max(np.abs(A[:, j] - ref)) / np.linalg.norm(sj)))
    say(f"[full bf16] flags={flags} orth={orth:.2e} |A_k|-sigma_k={cons:.2e} A[:, j] vs Phi^T S[:, j]={worst:.2e}")
    assert flags == 0
    assert np.all(s > 0) and np.all(np.diff(s) <= 0)
    assert orth <= 1e-5
    assert cons <= 1e-5
    assert worst <= 1e-4
