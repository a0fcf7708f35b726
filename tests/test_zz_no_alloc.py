"""GPU test of the entry point that allocates nothing (rpod_reconstruct_noalloc),
through the C ABI, against the workspace entry point rpod_reconstruct on the
same inputs: two calls in a row on the same GPU (so the second runs on the
static scratch the first left behind), the second with a smaller input; the
error must be bit-identical (the same kernels and order of sums), the fields
bit-identical where rpod_reconstruct also uses fused multiply-adds (FP64) and
within FP32 rounding where it uses the matrix cores (FP32, aligned). Sizes
beyond the static scratch are rejected before anything is enqueued."""

import ctypes

import numpy as np
import pytest
import torch

import paper_2504_15350_amd as rp

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _inputs(m, r, T, dtype, seed):
    rng = np.random.default_rng(seed)
    npd = np.float64 if dtype == torch.float64 else np.float32
    Phi = np.linalg.qr(rng.standard_normal((m, r)))[0].astype(npd)
    alpha = (10.0 * rng.standard_normal((r, T))).astype(npd)
    mean = rng.standard_normal(m).astype(npd)
    ref = (Phi.astype(np.float64) @ alpha + mean[:, None] + 1e-2 * rng.standard_normal((m, T))).astype(npd)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
    return t(Phi.T), t(alpha.T), t(mean), t(ref.T)


def _noalloc(dt, m, r, T, Phi_t, alpha_t, mean, ref_t, out_t):
    eps = ctypes.c_double(-1.0)
    sptr, _ = rp._stream_ptr(None, Phi_t.device)
    st = rp.lib().rpod_reconstruct_noalloc(dt, m, r, T, rp._dev_ptr(Phi_t), rp._dev_ptr(mean), rp._dev_ptr(alpha_t),
                                           rp._dev_ptr(out_t), rp._dev_ptr(ref_t), m, sptr, ctypes.byref(eps))
    return st, eps.value


@pytest.mark.parametrize("first,second", [
    ((70001, 50, 300, torch.float32), (4099, 17, 33, torch.float32)),
    ((70000, 128, 257, torch.float64), (1000, 7, 3, torch.float64)),
    ((65536, 40, 129, torch.float32), (513, 3, 1, torch.float64)),
])
def test_noalloc_matches_workspace_entry_point(first, second):
    for k, (m, r, T, dtype) in enumerate((first, second)):
        print(f"[noalloc] call {k}: m={m} r={r} T={T} dtype={dtype}", flush=True)
        Phi_t, alpha_t, mean, ref_t = _inputs(m, r, T, dtype, 100 * k + m)
        F_ws, eps_ws = rp.reconstruct(Phi_t, alpha_t, mean, ref_t)
        out_t = torch.full((T, m), float("nan"), dtype=dtype, device=DEV)
        dt = rp._DTYPES[dtype]
        st, eps = _noalloc(dt, m, r, T, Phi_t, alpha_t, mean, ref_t, out_t)
        torch.cuda.synchronize()
        assert st == 0, rp.lib().rpod_last_error()
        print(f"[noalloc] call {k}: eps {eps!r} vs {eps_ws!r}", flush=True)
        assert eps == eps_ws
        if dtype == torch.float64:
            assert torch.equal(out_t, F_ws)
        else:
            scale = float(F_ws.abs().max())
            assert float((out_t - F_ws).abs().max()) <= 2e-6 * scale


def test_noalloc_rejects_sizes_beyond_its_scratch():
    big = (1 << 24) + 1
    # rejected on the host: no pointer is touched, nothing is enqueued
    st = rp.lib().rpod_reconstruct_noalloc(1, big, 10, 5, 1, None, 1, None, None, big, None, None)
    assert st != 0 and b"static scratch" in rp.lib().rpod_last_error()
    st = rp.lib().rpod_reconstruct_noalloc(1, 1000, 129, 5, 1, None, 1, None, None, 1000, None, None)
    assert st != 0
