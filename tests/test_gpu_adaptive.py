"""GPU parity of the adaptive-rank plan (rpod_plan_create_adaptive /
rpod_compute_adaptive) against the CPU FP64 oracle of the blocked range
finder with the energy stopping rule.

The stopping block and the energy rank are integers decided in FP64 on
both sides from sums that differ by the path's rounding, so each case takes
delta halfway between the oracle's captured energies of two consecutive
blocks, and compares the rank only when no computed energy lies within
1e-4 of delta. Values: the sigma of the modes within three decades of
sigma_1 (FP64 1e-10, FP32 1e-5, 16-bit 1e-3 relative), the subspace of the
leading modes up to a cut with a relative gap of 1e-3 (FP64 1e-9, FP32
1e-4, 16-bit 1e-2), the coefficients of those modes, and the residual
indicator.
"""

import numpy as np
import pytest
import torch

import paper_2504_15350_amd as rp
import synth
from oracle import adaptive as oa
from oracle import metrics

from test_gpu_parity import DEV, say, sketch_for, upload

pytestmark = pytest.mark.gpu

TOL = {
    torch.float64: dict(sigma=1e-10, sin=1e-9, A=1e-9, res=1e-9),
    torch.float32: dict(sigma=1e-5, sin=1e-4, A=1e-4, res=1e-5),
    torch.bfloat16: dict(sigma=1e-3, sin=1e-2, A=1e-2, res=1e-3),
    torch.float16: dict(sigma=1e-3, sin=1e-2, A=1e-2, res=1e-3),
}


def _delta_between(S64, om, b, q, lmax, stop_block):
    """delta halfway between the captured energies of blocks stop_block - 1 and stop_block."""
    _, _, info = oa.rand_qb_ei(S64, om, b, q, 1.0, lmax)
    cap = [1.0 - e / info["fro2"] for e in info["E"]]
    lo = cap[stop_block - 2] if stop_block > 1 else 0.0
    return 0.5 * (lo + cap[stop_block - 1]), cap


def _leading_cut(s, kmax):
    """The largest k <= kmax with a relative gap of 1e-3 after mode k."""
    for k in range(kmax, 0, -1):
        if metrics.gap_ok(s, k):
            return k
    return 0


def run_case(St, dtype, b, q, lmax, stop_block, seed, ld=None, name=""):
    n, m = St.shape
    Sd, S64 = upload(St, dtype, ld)
    om = sketch_for(seed, n, lmax, dtype)
    delta, cap = _delta_between(S64, om, b, q, lmax, stop_block)
    say(f"[adaptive] {name} m={m} n={n} b={b} q={q} l_max={lmax} seed={seed} dtype={dtype} "
        f"delta={delta:.6f} captured={np.round(cap, 5).tolist()}")
    Pr, sr, Ar, info = oa.rpod_adaptive(S64, om, b, q, delta, lmax)
    plan = rp.AdaptivePlan(m, n, lmax, b, q, delta, dtype=dtype, ld=Sd.stride(0), device=DEV)
    Phi_t, sig, A_t, l, rank, resid = plan.compute(Sd, seed)
    torch.cuda.synchronize()
    Phi = Phi_t.double().cpu().numpy().T
    s = sig.cpu().numpy()
    A = A_t.double().cpu().numpy().T
    plan.close()
    tol = TOL[dtype]
    assert l == info["l"] == stop_block * b, (l, info["l"])
    e = info["energy"]
    if np.min(np.abs(e - delta)) > 1e-4:
        assert rank == info["r"], (rank, info["r"])
    keep = sr >= 1e-3 * sr[0]
    res = dict(l=l, rank=rank, oracle_rank=info["r"],
               sigma=metrics.sigma_rel_err(s[keep], sr[keep]), orth=metrics.orth_err(Phi),
               resid=abs(resid - info["E"][-1] / info["fro2"]))
    k = _leading_cut(sr, int(np.sum(keep)))
    if k > 0:
        res["k"] = k
        res["sin"] = metrics.sin_theta_max(Phi[:, :k], Pr[:, :k])
        res["A"] = metrics.lowrank_rel_diff(Phi[:, :k], A[:k], Pr[:, :k], Ar[:k])
    say(f"[adaptive] {name} {res}")
    assert np.all(np.diff(s) <= 0)
    assert res["sigma"] <= tol["sigma"], res
    assert res["orth"] <= (1e-12 if dtype == torch.float64 else 1e-5), res
    assert res["resid"] <= tol["res"], res
    if k > 0:
        assert res["sin"] <= tol["sin"] and res["A"] <= tol["A"], res
    return res


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16, torch.float16])
@pytest.mark.parametrize("q", [0, 1])
def test_adaptive_matches_oracle(dtype, q):
    g = synth.lowrank_exp(5000, 700, decay=0.06, noise_std=1e-3, seed=31)
    run_case(g["St"], dtype, 16, q, 96, 3, seed=41, name="ragged 5000 x 700")


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_adaptive_tall_with_wide_blocks_and_ld(dtype):
    g = synth.lowrank_exp(70001, 400, decay=0.04, noise_std=1e-3, seed=32)
    run_case(g["St"], dtype, 32, 1, 128, 2, seed=42, ld=70008, name="70001 x 400, ld 70008")


def test_adaptive_first_block_stop():
    g = synth.lowrank_exp(3000, 500, decay=0.5, noise_std=1e-6, seed=33)
    run_case(g["St"], torch.float32, 16, 1, 64, 1, seed=43, name="fast decay, one block")


@pytest.mark.parametrize("k,b", [(13, 16), (40, 16), (48, 32)])
def test_exact_low_rank_stops_at_its_rank(k, b):
    m, n = 4000, 300
    U = synth._orthonormal(m, k, 7, 1)
    V = synth._orthonormal(n, k, 7, 2)
    sig = 10.0 * np.exp(-0.1 * np.arange(k))
    St = np.ascontiguousarray(((U * sig) @ V.T).T)
    Sd, _ = upload(St, torch.float64)
    plan = rp.AdaptivePlan(m, n, 96, b, 0, 1.0 - 1e-12, dtype=torch.float64, device=DEV)
    Phi_t, s, A_t, l, rank, resid = plan.compute(Sd, 5)
    plan.close()
    s = s.cpu().numpy()
    say(f"[adaptive] exact rank {k}: l={l} rank={rank} resid={resid:.2e}")
    assert l == -(-k // b) * b and rank == k
    np.testing.assert_allclose(s[:k], sig, rtol=1e-11)
    assert abs(resid) < 1e-12 and np.all(s[k:] < 1e-11 * sig[0])
    assert metrics.sin_theta_max(Phi_t.cpu().numpy().T[:, :k], U) < 1e-10


def test_q0_equals_plain_plan_with_the_same_width():
    g = synth.lowrank_exp(6000, 800, decay=0.05, noise_std=1e-3, seed=34)
    Sd, S64 = upload(g["St"], torch.float64)
    m, n = S64.shape
    # captured energies of the six blocks: 0.261, 0.400, 0.478, 0.528, 0.570, 0.597
    plan = rp.AdaptivePlan(m, n, 96, 16, 0, 0.5, dtype=torch.float64, device=DEV)
    Phi_t, s, A_t, l, rank, resid = plan.compute(Sd, 77)
    plan.close()
    assert l == 64
    plain = rp.Plan(m, n, l, 0, 0, dtype=torch.float64, device=DEV)
    P2, s2, A2 = plain.compute(Sd, 77)
    plain.close()
    s, s2 = s.cpu().numpy(), s2.cpu().numpy()
    say(f"[adaptive] q=0 l={l}: sigma vs plain {metrics.sigma_rel_err(s, s2):.2e}")
    assert metrics.sigma_rel_err(s, s2) < 1e-10
    k = _leading_cut(s2, 20)
    assert metrics.sin_theta_max(Phi_t.cpu().numpy().T[:, :k], P2.cpu().numpy().T[:, :k]) < 1e-9


def test_unreachable_threshold_runs_every_block():
    g = synth.lowrank_exp(3000, 400, decay=0.01, noise_std=1e-1, seed=35)
    Sd, S64 = upload(g["St"], torch.float32)
    m, n = S64.shape
    plan = rp.AdaptivePlan(m, n, 48, 16, 1, 1.0, dtype=torch.float32, device=DEV)
    _, s, _, l, rank, resid = plan.compute(Sd, 3)
    assert l == 48 and rank == -1 and 0.0 < resid < 1.0
    # the same plan again: the status words start from zero on every call
    _, s2, _, l2, rank2, _ = plan.compute(Sd, 3)
    assert l2 == 48 and rank2 == -1 and torch.equal(s, s2)
    plan.close()


def test_asynchronous_call_and_errors():
    g = synth.lowrank_exp(2000, 300, decay=0.08, noise_std=1e-3, seed=36)
    Sd, S64 = upload(g["St"], torch.float32)
    m, n = S64.shape
    plan = rp.AdaptivePlan(m, n, 64, 16, 1, 0.95, dtype=torch.float32, device=DEV)
    Phi_t, s, A_t, l, rank, _ = plan.compute(Sd, 9)
    a = (Phi_t.clone(), s.clone(), A_t.clone())
    P, sg, A, l2, r2, e2 = plan.compute(Sd, 9, info=False)
    torch.cuda.synchronize()
    assert l2 is None and r2 is None and e2 is None
    assert torch.equal(P[:l], a[0]) and torch.equal(sg[:l], a[1])
    assert torch.equal(A.view(-1)[:n * l].view(n, l), a[2])
    # the plain entry point refuses an adaptive plan
    assert rp.lib().rpod_compute(plan._h, rp._dev_ptr(Sd), 9, rp._dev_ptr(P), rp._dev_ptr(sg), rp._dev_ptr(A)) != 0
    plan.close()
    for lmax, b, delta in ((64, 24, 0.9), (60, 16, 0.9), (144, 16, 0.9), (64, 16, 0.0), (64, 16, 1.5)):
        with pytest.raises(rp.RpodError):
            rp.AdaptivePlan(m, n, lmax, b, 1, delta, dtype=torch.float32, device=DEV)
