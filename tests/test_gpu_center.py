"""GPU parity of fluctuation centring (Sec. 4.1) through the C ABI.

A plan with block_cols = N^t decomposes S' = S minus the time average of each
block of N^t snapshot columns, without forming S'. The oracle forms S'
explicitly in FP64 (oracle.center.fluctuations) and runs its randomized POD on
the same sketch; the comparison and tolerances are those of the plain parity
tests. Inputs: synthetic fields plus a smooth time average per block of the
size of the fluctuations (so the centring changes the modes).
"""

import sys

import numpy as np
import pytest
import torch

import paper_2504_15350_amd as rp
import synth
from oracle import metrics, philox
from oracle import rpod as orpod
from oracle.center import fluctuations

from test_gpu_parity import TOL, compare, round_to, sketch_for, upload

pytestmark = pytest.mark.gpu
DEV = "cuda"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def field(nx, ny, n, N, seed, mean_rms=1.0, noise_std=1e-4, n_modes=100):
    g = synth.fourier_field(nx, ny, n, n_modes=n_modes, noise_std=noise_std, seed=seed)
    St = g["St"]
    rms = float(np.sqrt(np.mean(St * St)))
    synth.add_block_means(St, nx, ny, N, mean_rms * rms, seed)
    return St


def run_centred(Sd, m, n, r, p, q, seed, dtype, N):
    plan = rp.Plan(m, n, r, p, q, dtype=dtype, ld=Sd.stride(0), device=DEV, block_cols=N)
    Phi_t, sig, A_t = plan.compute(Sd, seed)
    torch.cuda.synchronize()
    say(f"[gpu] flags={plan.last_flags}")
    out = (Phi_t.double().cpu().numpy().T, sig.cpu().numpy(), A_t.double().cpu().numpy().T)
    plan.close()
    return out


def centred_case(St, r, p, q, seed, dtype, N, ld=None, name=""):
    n, m = St.shape
    say(f"[center] {name} m={m} n={n} N={N} r={r} p={p} q={q} seed={seed} dtype={dtype} ld={ld}")
    Sd, S64 = upload(St, dtype, ld)
    gpu = run_centred(Sd, m, n, r, p, q, seed, dtype, N)
    om = sketch_for(seed, n, r + p, dtype)
    Sc = fluctuations(S64, N)
    P2, s2, A2, ex = orpod.rpod_stable(Sc, r, om, q)
    res = compare(gpu, (P2, s2, A2), dtype, r, ex["ritz"])
    say(f"[center] {name} ok {res}")
    return res, gpu, Sc


@pytest.mark.parametrize("nx,ny,n,N,r,p,q,dtype,ldpad", [
    (32, 32, 120, 12, 10, 6, 1, torch.float64, 0),      # ten blocks
    (64, 64, 500, 50, 20, 10, 2, torch.float32, 0),     # ten blocks, q = 2
    (64, 64, 300, 300, 17, 9, 1, torch.float32, 3),     # one block (the global time average), odd ld
    (40, 25, 640, 10, 50, 14, 1, torch.float32, 0),     # 64 blocks with l = 64: widest first pass
    (64, 64, 400, 40, 20, 10, 2, torch.bfloat16, 0),
    (64, 64, 400, 100, 20, 10, 1, torch.float16, 8),
    (32, 64, 8000, 400, 20, 10, 1, torch.float32, 0),  # short, wide: the first pass splits its columns
    (32, 64, 8000, 500, 20, 10, 1, torch.bfloat16, 0),
])
def test_centred_matches_oracle(nx, ny, n, N, r, p, q, dtype, ldpad):
    St = field(nx, ny, n, N, seed=nx + n + N)
    m = nx * ny
    res, gpu, Sc = centred_case(St, r, p, q, 5, dtype, N, ld=m + ldpad if ldpad else None, name="centred")
    # the coefficients are those of the fluctuations: every block of A sums to ~0
    A = gpu[2]
    blk = A.reshape(r, n // N, N).sum(axis=2)
    scale = np.abs(A).sum(axis=1, keepdims=True) + 1e-300
    assert np.max(np.abs(blk) / scale) < (1e-10 if dtype == torch.float64 else 1e-3)


def test_centring_changes_the_result():
    # the same matrix without centring gives other modes (the means dominate mode 1)
    nx, ny, n, N = 64, 64, 300, 30
    St = field(nx, ny, n, N, seed=3, mean_rms=3.0)
    Sd, S64 = upload(St, torch.float32)
    plain = rp.Plan(nx * ny, n, 10, 5, 1, dtype=torch.float32, device=DEV)
    Pp, sp, _ = plain.compute(Sd, 4)
    plain.close()
    Pc, sc, _ = run_centred(Sd, nx * ny, n, 10, 5, 1, 4, torch.float32, N)
    assert sp.cpu().numpy()[0] > 1.5 * sc[0]
    assert metrics.sin_theta_max(Pp.double().cpu().numpy().T, Pc) > 0.5


def test_batch_mixes_centred_and_plain_matrices():
    specs = [(4096, 300, 10, 6, 30), (4096, 300, 10, 6, 0), (2500, 200, 12, 4, 50), (4096, 240, 20, 12, 24)]
    Sts, shapes = [], []
    for i, (m, n, r, p, N) in enumerate(specs):
        nx = 64 if m == 4096 else 50
        St = field(nx, m // nx, n, N if N else n, seed=20 + i)
        Sts.append(St)
        shapes.append((m, n, r, p, m, N))
    q, seed = 1, 13
    bp = rp.BatchPlan(shapes, q, dtype=torch.float32, device=DEV)
    devs = [upload(St, torch.float32)[0] for St in Sts]
    outs = bp.compute(devs, [seed + i for i in range(len(specs))])
    torch.cuda.synchronize()
    for i, ((m, n, r, p, N), St) in enumerate(zip(specs, Sts)):
        Phi_t, sig, A_t = outs[i]
        gpu = (Phi_t.double().cpu().numpy().T, sig.cpu().numpy(), A_t.double().cpu().numpy().T)
        S64 = round_to(St, torch.float32).double().numpy().T
        Sx = fluctuations(S64, N) if N else S64
        om = sketch_for(seed + i, n, r + p, torch.float32)
        P2, s2, A2, ex = orpod.rpod_stable(Sx, r, om, q)
        res = compare(gpu, (P2, s2, A2), torch.float32, r, ex["ritz"])
        say(f"[center batch] item {i} N={N} ok {res}")
    bp.close()


def test_fp32_full_size_ten_blocks():
    # the benchmark's FP32 workload with ten parameter blocks of 500 snapshots
    nx, ny, n, N, r, p, q, seed = 512, 512, 5000, 500, 50, 10, 2, 2
    g = synth.fourier_field(nx, ny, n, n_modes=200, beta=1.5, phi=0.95, noise_std=1e-4, seed=2,
                            dtype=np.float32)
    St = g["St"]
    del g
    rms = float(np.sqrt(np.mean(St[:64].astype(np.float64) ** 2)))
    synth.add_block_means(St, nx, ny, N, rms, seed)
    m = nx * ny
    say(f"[center full] m={m} n={n} N={N} r={r} p={p} q={q} seed={seed}")
    Sd = torch.from_numpy(St).to(DEV)
    gpu = run_centred(Sd, m, n, r, p, q, seed, torch.float32, N)
    del Sd
    S64 = np.ascontiguousarray(St.T, dtype=np.float64)
    del St
    Sc = fluctuations(S64, N)
    del S64
    om = philox.gaussian_sketch(seed, n, r + p).astype(np.float32).astype(np.float64)
    P2, s2, A2, ex = orpod.rpod_stable(Sc, r, om, q)
    res = compare(gpu, (P2, s2, A2), torch.float32, r, ex["ritz"])
    say(f"[center full] ok {res}")
