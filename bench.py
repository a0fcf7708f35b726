#!/usr/bin/env python3
"""Benchmark: randomized POD time-to-r-modes on one MI355X.

One step = one full rPOD call (Alg. 1 of Sec. 4.2: sketch, q subspace
iterations with CholeskyQR2, T = Q^T S, small SVD, lift, coefficients and
sign fix) on a synthetic snapshot matrix already resident in HBM.

Main workload (the JSON line's value): mixed precision, S = 1048576 x 10000
stored in BF16 (a 1024 x 1024 cell-centred grid on [0,1] x [0,2], 10000
snapshots of a 200-mode Fourier field with |k|^-1.5 amplitudes and AR(1) time
series, phi = 0.95, plus 1e-4 white noise), r = 100, p = 20, q = 2, with FP32
accumulation, FP64 Gram / Cholesky / small SVD and the hi + lo refinement
pass. Beside it on the same matrix (under "mixed_vs_plain"): plain FP32 rPOD
(the in-GPU baseline the speedup is quoted against) and the FP16-stored path,
each with its sigma error and largest principal-angle sine against the
oracle's FP64 rPOD (O2) of the unrounded matrix on the same BF16 sketch (so
storage rounding counts), and sigma against the closed-form POD of the
noise-free field (sketch-independent; the noise moves sigma by at most its
spectral norm, reported).

Also measured (unless --no-extra): plain FP32 rPOD on S = 262144 x 5000
(512 x 512 grid, same field), r = 50, p = 10, q = 2, under "plain_fp32_262144x5000".

Also measured (unless --no-batch): the uneven batch of 64 snapshot matrices
(m in {2^16, 2^17, 2^18}, n in [500, 4000], r in {10, 25, 50, 100}, p = 10,
q = 2, spectral decay in [0.05, 0.2], all drawn per matrix from the seed):
one batched plan in BF16 and in FP32 against 64 single plain FP32 plans run
one after another, reported under "batched_vs_plain".

Also measured (unless --no-warm): the learned warm start on the parametric
sweep S(mu) = U(mu) diag(exp(-alpha k)) V^T + noise (1e-9), m = 131072 (a
256 x 512 grid), n = 2000, r = 50, 128 parameter vectors (96 train, 32
test), reported under "warm_vs_plain".

Also measured (unless --no-center): fluctuation centring (Sec. 4.1) and the
energy report on the 262144 x 5000 workload, under "centred_vs_plain" and
"energy_report"; and (unless --no-adaptive) the adaptive-rank plan on the same
matrix (blocks of 16 columns up to 128, q = 2, the threshold set to the energy
of the fixed plan's 40 leading modes) beside fixed plans with the width it
stopped at and with 128 columns, under "adaptive_vs_fixed".

Per-kernel times of the passes over S come from HIP events that the library
records on its stream around every pass during the timed steps.
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
# Matrix-core peaks of the pass kernels, in TFLOP/s of the algorithmic 2 m n l.
# FP32 passes run on the BF16 matrix cores (2.5 PFLOP/s dense) with every
# operand split into three BF16 parts and six products per multiply-add:
# an FP32-accurate peak of 2500 / 6.
PEAK_TFLOPS = {"f64": 78.6, "f32": 2500.0 / 6, "bf16": 2500.0, "f16": 2500.0}

WORKLOADS = {
    "fp32_262144x5000": dict(
        label="plain rPOD FP32, S 262144x5000 (512x512 grid), Fourier field, r=50 p=10 q=2",
        nx=512, ny=512, n=5000, r=50, p=10, q=2, dtype="f32", gen="host", gen_seed=2, seed=2,
        sample_rows=65536),
    "fp64_4096x200": dict(
        label="plain rPOD FP64, S 4096x200, U diag(exp(-0.1k)) V^T + noise, r=20 p=10 q=1",
        m=4096, n=200, r=20, p=10, q=1, dtype="f64", gen="host", gen_seed=1, seed=1, sample_rows=4096),
    "bf16_1048576x10000": dict(
        label="mixed rPOD, S 1048576x10000 (1024x1024 grid) in BF16, Fourier field, r=100 p=20 q=2",
        nx=1024, ny=1024, n=10000, r=100, p=20, q=2, dtype="bf16", gen="device", gen_seed=3, seed=3,
        sample_rows=65536),
    "f16_1048576x10000": dict(
        label="mixed rPOD, S 1048576x10000 (1024x1024 grid) in FP16, Fourier field, r=100 p=20 q=2",
        nx=1024, ny=1024, n=10000, r=100, p=20, q=2, dtype="f16", gen="device", gen_seed=3, seed=3,
        sample_rows=65536),
    "fp32_1048576x10000": dict(
        label="plain rPOD FP32, S 1048576x10000 (1024x1024 grid), Fourier field, r=100 p=20 q=2",
        nx=1024, ny=1024, n=10000, r=100, p=20, q=2, dtype="f32", gen="device", gen_seed=3, seed=3,
        sample_rows=65536),
}
DEFAULT = "bf16_1048576x10000"
PLAIN_SMALL = "fp32_262144x5000"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def torch_dtype(name):
    import torch
    return {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[name]


def make_input(w, dev):
    """Synthetic S as a device tensor St (n, m)."""
    import torch
    import synth
    if w["gen"] == "device":
        return synth.fourier_field_device(w["nx"], w["ny"], w["n"], seed=w["gen_seed"],
                                          dtype=torch_dtype(w["dtype"]), device=dev)["St"]
    npdt = np.float64 if w["dtype"] == "f64" else np.float32
    if "nx" in w:
        g = synth.fourier_field(w["nx"], w["ny"], w["n"], n_modes=200, beta=1.5, phi=0.95, noise_std=1e-4,
                                seed=w["gen_seed"], dtype=npdt)
    else:
        g = synth.lowrank_exp(w["m"], w["n"], decay=0.1, noise_std=1e-4, seed=w["gen_seed"], dtype=npdt)
    return torch.from_numpy(g["St"]).to(dev)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("stream_kernels.hip", "stream16_kernels.hip", "stream_e6_kernels.hip", "device_common.hpp"):
        with open(os.path.join(ROOT, "paper_2504_15350_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload, kernel):
    """HBM bytes per launch from committed rocprofv3 counter runs, if still current."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))[workload][kernel]
    except (KeyError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


PASS_KINDS = ((0, "S_X"), (1, "St_Q"), (2, "St_Q_refine"))
# library kernel behind each pass kind, per storage type (the names rocprofv3 lists)
KERNEL_OF = {
    "bf16": {"S_X": "k_sx16<bf16>", "St_Q": "k_stq16<bf16, hi>", "St_Q_refine": "k_stq16<bf16, hi + lo>"},
    "f16": {"S_X": "k_sx16<f16>", "St_Q": "k_stq16<f16, hi>", "St_Q_refine": "k_stq16<f16, hi + lo>"},
    "f32": {"S_X": "k_sx_e6", "St_Q": "k_stq_e6"},
    "f64": {"S_X": "k_sx<double>", "St_Q": "k_stq<double>"},
}


def measure(name, St, steps, warmup, block_cols=0, energy=False, keep_out=False):
    """Time `steps` rPOD calls; per-pass kernel times from the library's HIP events."""
    import torch
    import paper_2504_15350_amd as rp
    w = WORKLOADS[name]
    n, m = St.shape
    dev = St.device
    plan = rp.Plan(m, n, w["r"], w["p"], w["q"], dtype=St.dtype, device=dev, block_cols=block_cols, energy=energy)
    out = (torch.empty((w["r"], m), dtype=plan.out_dtype, device=dev),
           torch.empty((w["r"],), dtype=torch.float64, device=dev),
           torch.empty((n, w["r"]), dtype=plan.out_dtype, device=dev))
    for _ in range(warmup):
        plan.compute(St, w["seed"], out=out, check=False)
    plan.status()
    # graph replays, no per-pass events
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.compute(St, w["seed"], out=out, check=False)
    torch.cuda.synchronize()
    ms_graph = (time.perf_counter() - t0) * 1e3 / steps
    plan.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.compute(St, w["seed"], out=out, check=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    flags = plan.status()
    ms = wall * 1e3 / steps
    log(f"[bench] {name}: graph replay {ms_graph:.3f} ms per rPOD")
    kern = {}
    for kind, kname in PASS_KINDS:
        nl, tot, bpl, fpl = plan.timing(kind)
        if nl:
            kern[kname] = dict(launches=nl, avg_ms=tot / max(nl, 1), bytes=bpl, flops=fpl, total_ms=tot)
    plan.set_timing(False)
    sigma = out[1].cpu().numpy()
    en = plan.energy(0.9) if energy else None
    plan.close()
    log(f"[bench] {name}: {ms:.3f} ms per rPOD over {steps} steps (flags {flags}); "
        + ", ".join(f"{k} {v['avg_ms']:.3f} ms x{v['launches'] // steps}" for k, v in kern.items()))

    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    kd = kern[dom]
    fl = kd["flops"] / (kd["avg_ms"] * 1e-3) / 1e12
    gbs = kd["bytes"] / (kd["avg_ms"] * 1e-3) / 1e9
    peak = PEAK_TFLOPS[w["dtype"]]
    if kd["flops"] / kd["bytes"] > peak * 1e3 / HBM_PEAK_GBS:
        roof = dict(bound="mfma", achieved=round(fl, 2), peak=peak, unit="TFLOP/s", frac=round(fl / peak, 4))
    else:
        roof = dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(gbs / HBM_PEAK_GBS, 4))
    roof.update(traffic=load_traffic(name, dom), kernel=KERNEL_OF[w["dtype"]].get(dom, dom), pass_kind=dom,
                avg_launch_ms=round(kd["avg_ms"], 4), algorithmic_bytes_per_launch=kd["bytes"],
                algorithmic_flops_per_launch=kd["flops"], hbm_gbs_algorithmic=round(gbs, 1))
    passes = sum(v["launches"] for v in kern.values()) / steps
    s_bytes = passes * m * n * St.element_size()
    res = dict(ms=ms, ms_graph=ms_graph, roofline=roof, sigma=sigma, flags=flags, energy=en,
               hbm_gbs_s_passes=round(s_bytes / (ms * 1e-3) / 1e9, 1),
               kernels={k: {"launches_per_step": v["launches"] // steps, "avg_ms": round(v["avg_ms"], 4),
                            "hbm_gbs_algorithmic": round(v["bytes"] / (v["avg_ms"] * 1e-3) / 1e9, 1)}
                        for k, v in kern.items()})
    if keep_out:
        res["out"] = out
    else:
        del out
    return res


BATCH = dict(count=64, shape_seed=4, p=10, q=2, seed0=1000)
# (stq_workgroups, gram_workgroups) per storage type, 0 = the library's default
BATCH_TUNING = {"fp32": (128, 64), "bf16": (0, 64)}


def make_batch(dev):
    """The 64 uneven matrices as FP32 device tensors (St (n, m) each) and their shapes."""
    import synth
    shapes = synth.batch_shapes(BATCH["count"], seed=BATCH["shape_seed"])
    mats = [synth.lowrank_exp_device(m, n, a, noise_std=1e-4, seed=BATCH["seed0"] + i, device=dev)
            for i, (m, n, r, a) in enumerate(shapes)]
    return shapes, mats


def measure_batch(mats, shapes, steps, warmup, batched=True, tuning=None):
    """Time one batched plan over all matrices (or one plan per matrix in
    sequence); per-pass kernel times from the library's HIP events."""
    import torch
    import paper_2504_15350_amd as rp
    p, q = BATCH["p"], BATCH["q"]
    seeds = [BATCH["seed0"] + 7 * i for i in range(len(mats))]
    dt = mats[0].dtype
    if batched:
        plans = [rp.BatchPlan([(m, n, r, p) for (m, n, r, _a) in shapes], q, dtype=dt, device=mats[0].device,
                              tuning=tuning)]
        outs = [plans[0].alloc_outputs()]
        run = lambda: plans[0].compute(mats, seeds, outs=outs[0], check=False)
    else:
        plans = [rp.Plan(m, n, r, p, q, dtype=dt, device=mats[0].device) for (m, n, r, _a) in shapes]
        outs = [(torch.empty((r, m), dtype=pl.out_dtype, device=mats[0].device),
                 torch.empty((r,), dtype=torch.float64, device=mats[0].device),
                 torch.empty((n, r), dtype=pl.out_dtype, device=mats[0].device))
                for pl, (m, n, r, _a) in zip(plans, shapes)]

        def run():
            for pl, St, sd, o in zip(plans, mats, seeds, outs):
                pl.compute(St, sd, out=o, check=False)
    for _ in range(warmup):
        run()
    for pl in plans:
        pl.status()
    # graph replays (classes of a batch run as concurrent graph branches)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    # the same steps again, kernels launched one by one with per-pass events
    for pl in plans:
        pl.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    ms_timed = (time.perf_counter() - t0) * 1e3 / steps
    flags = [pl.status() for pl in plans]
    tot = {0: [0, 0.0, 0.0], 1: [0, 0.0, 0.0], 2: [0, 0.0, 0.0]}
    for pl in plans:
        for kind in (0, 1, 2):
            nl, t, bpl, _fpl = pl.timing(kind)
            tot[kind][0] += nl
            tot[kind][1] += t
            tot[kind][2] += bpl * nl
        pl.set_timing(False)
    if batched:
        sig = [o[1].cpu().numpy() for o in outs[0]]
    else:
        sig = [o[1].cpu().numpy() for o in outs]
    for pl in plans:
        pl.close()
    kern = {}
    for kind, kname in PASS_KINDS:
        nl, t, b = tot[kind]
        if nl == 0:
            continue
        kern[kname] = dict(launches_per_step=nl // steps, avg_ms=round(t / max(nl, 1), 4),
                           hbm_gbs_algorithmic=round(b / (t * 1e-3) / 1e9, 1) if t > 0 else None)
    s_bytes = sum(m * n for (m, n, _r, _a) in shapes) * mats[0].element_size() * (2 * q + 2)
    log(f"[bench] batch {'batched' if batched else 'sequential'} {dt}: {ms:.2f} ms per batch "
        f"(kernel by kernel with events: {ms_timed:.2f} ms) "
        f"({len(mats)} matrices), flags {sorted(set(sum(([f] if isinstance(f, int) else f for f in flags), [])))}, " + ", ".join(f"{k} {v}" for k, v in kern.items()))
    return dict(ms=ms, ms_timed=ms_timed, sigma=sig, kernels=kern, hbm_gbs_s_passes=round(s_bytes / (ms * 1e-3) / 1e9, 1),
                flags=flags)


def batch_block(dev, steps, warmup):
    import torch
    t0 = time.perf_counter()
    shapes, mats = make_batch(dev)
    torch.cuda.synchronize()
    elems = sum(m * n for (m, n, _r, _a) in shapes)
    log(f"[bench] generated the 64-matrix batch ({elems / 1e9:.2f} G elements) in {time.perf_counter() - t0:.1f} s")
    import paper_2504_15350_amd as rp
    plain = measure_batch(mats, shapes, steps, warmup, batched=False)
    # Launch shapes: the values rpod_autotune chose for this batch when it last ran here. The
    # autotuner itself is not called: one of its runs aborted without a message and the cause
    # has not been found.
    tune32, tune16 = rp.Tuning(*BATCH_TUNING["fp32"]), rp.Tuning(*BATCH_TUNING["bf16"])
    b32 = measure_batch(mats, shapes, steps, warmup, batched=True, tuning=tune32)
    mats16 = [St.to(torch.bfloat16) for St in mats]
    del mats
    torch.cuda.empty_cache()
    b16d = measure_batch(mats16, shapes, steps, warmup, batched=True)
    b16 = measure_batch(mats16, shapes, steps, warmup, batched=True, tuning=tune16)
    del mats16
    torch.cuda.empty_cache()

    def err(a, b):
        return float(max(np.max(np.abs(x - y) / y) for x, y in zip(a["sigma"], b["sigma"])))
    return {
        "config": {"count": len(shapes), "elements": elems, "p": BATCH["p"], "q": BATCH["q"],
                   "m_values": sorted({s[0] for s in shapes}), "n_range": [min(s[1] for s in shapes),
                                                                           max(s[1] for s in shapes)],
                   "r_values": sorted({s[2] for s in shapes}), "steps": steps},
        "plain_fp32_sequential_ms": round(plain["ms"], 3),
        "batched_fp32_ms": round(b32["ms"], 3),
        "batched_bf16_ms": round(b16["ms"], 3),
        "batched_bf16_default_tuning_ms": round(b16d["ms"], 3),
        "tuning": {"fp32": {"stq_workgroups": tune32.stq_workgroups, "gram_workgroups": tune32.gram_workgroups},
                   "bf16": {"stq_workgroups": tune16.stq_workgroups, "gram_workgroups": tune16.gram_workgroups},
                   "source": "fixed: the autotuner's earlier choice for this batch"},
        "kernel_by_kernel_ms": {"plain_fp32": round(plain["ms_timed"], 3), "batched_fp32": round(b32["ms_timed"], 3),
                                "batched_bf16": round(b16["ms_timed"], 3)},
        "speedup_batched_fp32": round(plain["ms"] / b32["ms"], 2),
        "speedup_batched_bf16": round(plain["ms"] / b16["ms"], 2),
        "sigma_rel_diff_batched_fp32_vs_plain": err(b32, plain),
        "sigma_rel_diff_batched_bf16_vs_plain": err(b16, plain),
        "hbm_gbs_s_passes": {"plain_fp32": plain["hbm_gbs_s_passes"], "batched_fp32": b32["hbm_gbs_s_passes"],
                             "batched_bf16": b16["hbm_gbs_s_passes"]},
        "kernels": {"plain_fp32": plain["kernels"], "batched_fp32": b32["kernels"], "batched_bf16": b16["kernels"]},
    }


WARM = dict(nx=256, ny=512, n=2000, r=50, p=10, count=128, n_train=96, seed=5, noise=1e-9, epochs=2000)


def warm_block(dev, reps):
    """Train the warm-start network on the sweep and time plain vs warm rPOD on the test matrices."""
    import torch
    import synth
    import paper_2504_15350_amd as rp
    W = WARM
    t0 = time.perf_counter()
    fam = synth.ParamFamily(W["nx"], W["ny"])
    F_dev = torch.from_numpy(fam.F.astype(np.float32)).to(dev)
    mu, mu_hat = synth.draw_params(W["count"], seed=W["seed"])
    train, test = synth.train_test_split(W["count"], W["n_train"], seed=W["seed"])
    m, n, r, p = fam.m, W["n"], W["r"], W["p"]
    plain = rp.Plan(m, n, r, p, 2, dtype=torch.float32, device=dev)
    bases = {}
    for i in train:
        St = fam.matrix_device(mu[i], n, noise_std=W["noise"], seed=2000 + int(i), device=dev, F_dev=F_dev)
        bases[int(i)] = plain.compute(St, 3000 + int(i))[0].clone()
        del St
    bank_idx = [int(train[j]) for j in synth.farthest_points(mu_hat[train], 8)]
    model = rp.WarmModel(m, r, max_train=len(train), seed=W["seed"], device=dev)
    model.set_bank([bases[i] for i in bank_idx])
    mu_t = torch.tensor(mu_hat[train], dtype=torch.float32, device=dev).contiguous()
    b_t = torch.stack([model.targets(bases[int(i)]) for i in train]).contiguous()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    losses = model.train(mu_t, b_t, W["epochs"], lr=1e-3, weight_decay=1e-5)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    losses = losses.cpu().numpy()
    log(f"[bench] warm start: bank and targets in {t1 - t0:.1f} s, {W['epochs']} epochs in {t_train:.2f} s, "
        f"loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    tests = [fam.matrix_device(mu[i], n, noise_std=W["noise"], seed=2000 + int(i), device=dev, F_dev=F_dev)
             for i in test]
    exact = [fam.spectrum(mu[i][3], fam.K)[:r] for i in test]
    del F_dev

    ok = [e >= 1e-3 * e[0] for e in exact]   # modes within three decades of sigma_1

    def run(kind, mats, q=2, tol=1e9, q_fb=0):
        if kind == "plain":
            pl = rp.Plan(m, n, r, p, q, dtype=mats[0].dtype, device=dev)
            first = lambda j: (pl.compute(mats[j], 4000 + j, check=False)[1], None, None)
            call = lambda j: pl.compute(mats[j], 4000 + j, check=False)
        else:
            pl = rp.WarmPlan(model, n, p, q, q_fallback=q_fb, tol=tol, dtype=mats[0].dtype, device=dev)

            def first(j):
                o = pl.compute(mats[j], mu_hat[test[j]], 4000 + j, check=False)
                return o[1], o[3], o[4]
            call = lambda j: pl.compute(mats[j], mu_hat[test[j]], 4000 + j, check=False, decision=False)
        res = [first(j) for j in range(len(mats))]   # warm-up pass, also the results and decisions
        torch.cuda.synchronize()
        rel = [np.abs(r_[0].cpu().numpy() - e) / e for r_, e in zip(res, exact)]
        errs = [float(np.max(x)) for x in rel]
        errs_ok = [float(np.max(x[k])) for x, k in zip(rel, ok)]
        t = time.perf_counter()
        for _ in range(reps):
            for j in range(len(mats)):
                call(j)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / (reps * len(mats))
        pl.status()
        pl.close()
        d = dict(ms_per_matrix=round(ms, 4), sigma_err_median=float(np.median(errs)),
                 sigma_err_max=float(np.max(errs)), frac_within_1e3=float(np.mean(np.array(errs) <= 1e-3)),
                 sigma_err_max_leading=float(np.max(errs_ok)),
                 frac_within_1e3_leading=float(np.mean(np.array(errs_ok) <= 1e-3)))
        if kind != "plain":
            rho = np.array([r_[2] for r_ in res])
            d.update(continued=int(sum(bool(r_[1]) for r_ in res)), tol=tol if np.isfinite(tol) else "unchecked",
                     q_fallback=q_fb)
            if np.all(np.isfinite(rho)):
                d.update(rho_median=float(np.median(rho)), rho_max=float(np.max(rho)))
        return d

    inf = float("inf")
    out = {"plain_fp32_q2": run("plain", tests), "plain_fp32_q1": run("plain", tests, 1),
           "warm_fp32_q0_unchecked": run("warm", tests, 0, inf),
           "warm_fp32_q1_unchecked": run("warm", tests, 1, inf),
           "warm_fp32_q1_checked_accept_all": run("warm", tests, 1),
           "warm_fp32_q1_tol1e-2_cont1": run("warm", tests, 1, 1e-2, 1),
           "warm_fp32_q0_tol1e-2_cont1": run("warm", tests, 0, 1e-2, 1),
           "warm_fp32_q0_tol1e-3_cont2": run("warm", tests, 0, 1e-3, 2)}
    tests16 = [St.to(torch.bfloat16) for St in tests]
    del tests
    torch.cuda.empty_cache()
    out["plain_bf16_q2"] = run("plain", tests16)
    out["plain_bf16_q1"] = run("plain", tests16, 1)
    out["warm_bf16_q1_unchecked"] = run("warm", tests16, 1, inf)
    out["warm_bf16_q1_tol1e-2_cont1"] = run("warm", tests16, 1, 1e-2, 1)
    del tests16
    model.close()
    plain.close()
    torch.cuda.empty_cache()
    base = out["plain_fp32_q2"]["ms_per_matrix"]
    for k, v in out.items():
        v["speedup_vs_plain_fp32"] = round(base / v["ms_per_matrix"], 2)
        log(f"[bench] warm sweep {k}: {v}")
    return {"config": {"m": m, "n": n, "r": r, "p": p, "matrices": W["count"], "train": W["n_train"],
                       "test": len(test), "bank": 8, "epochs": W["epochs"], "noise_std": W["noise"], "reps": reps,
                       "rule": "accept the warm result if max_k ||S v_k - sigma_k phi_k|| / sigma_k <= tol, "
                               "else continue q_fallback iterations from the warm range basis",
                       "leading": "modes with exact sigma_k >= 1e-3 sigma_1"},
            "train_seconds": round(t_train, 3), "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
            "results": out}


# The paper's own shape: N_C = 8192 cells (64 x 128) and 225 parameter blocks
# x 401 steps = 90225 snapshots per field; 10 modes, p swept, q = 1. beta
# calibrates the field so that 10 modes hold the share of the singular-value
# sum the paper tabulates for its variables (q-like about 27 %, psi-like
# about 41 %; computed from all 8192 singular values of the generated field).
PAPER = dict(nx=64, ny=128, n=90225, r=10, q=1, ps=(0, 5, 10, 20, 50, 75), seed=17,
             fields=(("q_like", 1.5), ("psi_like", 2.0)))
PAPER_NAME = "paper_8192x90225"


def paper_block(dev, steps, warmup, cpu=True, accuracy=True):
    """Row P: GPU FP32 and BF16 rPOD for every p on both calibrated fields,
    their accuracy against O1 (deterministic POD), and O1 / O2 timed on the host."""
    import torch
    import synth
    import paper_2504_15350_amd as rp
    from oracle import metrics, philox, pod
    from oracle import rpod as orpod
    W = PAPER
    out = {"config": {"workload": PAPER_NAME, "m": W["nx"] * W["ny"], "n": W["n"], "r": W["r"], "q": W["q"],
                      "p": list(W["ps"]), "grid": "64 x 128 cells", "snapshots": "225 parameter blocks x 401 steps"},
           "paper": {"pod_seconds": "> 4000", "rpod_seconds_p75": "about 6", "speedup": "about 700",
                     "hardware": "CPU, not stated",
                     "where": "Sec. 5, the figure of POD and rPOD CPU time as p varies; Sec. 5.4, Tab. cpu_time"},
           "fields": {}}
    for fname, beta in W["fields"]:
        t0 = time.perf_counter()
        gen = synth.fourier_field_device(W["nx"], W["ny"], W["n"], beta=beta, seed=W["seed"], device=dev)
        St = gen.pop("St")
        n, m = St.shape
        torch.cuda.synchronize()
        log(f"[bench] paper shape {fname} (beta {beta}): generated S {m}x{n} in {time.perf_counter() - t0:.1f} s")
        St16 = St.to(torch.bfloat16)
        gpu = {}
        for tname, Sd in (("fp32", St), ("bf16", St16)):
            for p in W["ps"]:
                plan = rp.Plan(m, n, W["r"], p, W["q"], dtype=Sd.dtype, device=dev)
                for _ in range(warmup):
                    res = plan.compute(Sd, W["seed"], check=False)
                plan.status()
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                for _ in range(steps):
                    res = plan.compute(Sd, W["seed"], check=False)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t1) * 1e3 / steps
                plan.status()
                plan.close()
                l = W["r"] + p
                passes = 2 * W["q"] + 2
                gbs = passes * m * n * Sd.element_size() / (ms * 1e-3) / 1e9
                gpu[f"{tname}_p{p}"] = dict(ms=round(ms, 4), s_pass_gbs=round(gbs, 1), l=l,
                                            out=(res[0].double().cpu().numpy().T, res[1].cpu().numpy()))
                log(f"[bench] paper {fname} {tname} p={p}: {ms:.3f} ms per rPOD ({gbs:.0f} GB/s over S)")
        del St16
        if not accuracy:   # timing only (profiling runs): no host copy, O1 or O2
            for v in gpu.values():
                v.pop("out")
            out["fields"][fname] = {"beta": beta, "gpu": gpu}
            del St
            torch.cuda.empty_cache()
            continue
        S64 = host_fp64(St)
        del St
        torch.cuda.empty_cache()
        S = S64.T                                   # m x n view
        t1 = time.perf_counter()
        log(f"[bench] paper {fname}: O1 (method of snapshots, eigh of S S^T) on the host ...")
        P1, s1, _A1, s_all = pod.pod_snapshots(S, W["r"])
        t_o1 = time.perf_counter() - t1
        e_sum = float(np.sum(s_all[:W["r"]]) / np.sum(s_all))
        log(f"[bench] paper {fname}: O1 in {t_o1:.1f} s; 10 modes hold {100 * e_sum:.1f} % of the singular-value sum")
        fld = {"beta": beta, "energy_share_10_modes_sigma_sum": round(e_sum, 4),
               "energy_share_10_modes_sigma_squared": round(float(np.sum(s_all[:W['r']] ** 2) / np.sum(s_all ** 2)), 4),
               "o1_seconds": round(t_o1, 1), "by_p": {}}
        for p in W["ps"]:
            row = {}
            if cpu:
                om = philox.gaussian_sketch(W["seed"], n, W["r"] + p)
                t1 = time.perf_counter()
                P2, s2, _A2, _ex = orpod.rpod_stable(S, W["r"], om, W["q"])
                row["o2_seconds"] = round(time.perf_counter() - t1, 2)
                row["o2_sigma_err_vs_o1"] = metrics.sigma_rel_err(s2, s1)
                row["o2_sin_theta_vs_o1"] = metrics.sin_theta_max(P2, P1)
            for tname in ("fp32", "bf16"):
                g = gpu[f"{tname}_p{p}"]
                Phi, sg = g.pop("out")
                g["sigma_err_vs_o1"] = metrics.sigma_rel_err(sg, s1)
                g["sin_theta_vs_o1"] = metrics.sin_theta_max(Phi, P1)
                row[tname] = g
            if cpu:
                row["o1_over_gpu_bf16"] = round(t_o1 * 1e3 / row["bf16"]["ms"], 0)
                row["o2_over_gpu_bf16"] = round(row["o2_seconds"] * 1e3 / row["bf16"]["ms"], 1)
            fld["by_p"][str(p)] = row
            log(f"[bench] paper {fname} p={p}: {row}")
        out["fields"][fname] = fld
        del S64, S
    out["host"] = host_info()
    return out


CENTER = dict(block_cols=500, mean_rms=1.0, seed=2)


def center_block(St, steps, warmup):
    """Fluctuation centring on the main workload: ten parameter blocks of 500
    snapshots, each given a smooth time average of the fluctuations' RMS (added
    to St in place); the plain and the centred plan timed on that matrix."""
    import torch
    import synth
    w = WORKLOADS[PLAIN_SMALL]
    n, m = St.shape
    N = CENTER["block_cols"]
    K = n // N
    rms = float(St[:64].double().pow(2).mean().sqrt())
    means = synth.add_block_means(np.zeros((K, m), np.float32), w["nx"], w["ny"], 1, CENTER["mean_rms"] * rms,
                                  CENTER["seed"])
    St.view(K, N, m).add_(torch.from_numpy(means.T.astype(np.float32)).to(St.device)[:, None, :])
    torch.cuda.synchronize()
    plain = measure(PLAIN_SMALL, St, steps, warmup)
    cen = measure(PLAIN_SMALL, St, steps, warmup, block_cols=N)
    recon = reconstruct_block(St, N)
    return {
        "reconstruct_block0": recon,
        "config": {"workload": PLAIN_SMALL, "block_cols": N, "blocks": K, "mean_rms_over_field_rms": CENTER["mean_rms"],
                   "steps": steps},
        "plain_ms": round(plain["ms"], 4), "centred_ms": round(cen["ms"], 4),
        "overhead": round(cen["ms"] / plain["ms"] - 1.0, 4),
        "sigma1_plain": float(plain["sigma"][0]), "sigma1_centred": float(cen["sigma"][0]),
        "centred_kernels": cen["kernels"], "centred_roofline": cen["roofline"],
    }


def adaptive_block(St, energies, steps, warmup, block=16, l_max=128, q=2, modes=40):
    """The adaptive-rank plan on the FP32 262144 x 5000 field: the sketch grows by
    `block` columns up to l_max until it captures the energy that the leading
    `modes` modes of the fixed plan hold; timed beside fixed plans with the
    width it stopped at and with l_max."""
    import torch
    import paper_2504_15350_amd as rp
    w = WORKLOADS[PLAIN_SMALL]
    n, m = St.shape
    delta = float(energies[modes - 1])
    ap = rp.AdaptivePlan(m, n, l_max, block, q, delta, dtype=St.dtype, device=St.device)
    _, sig_a, _, l, rank, resid = ap.compute(St, w["seed"])
    sig_a = sig_a.cpu().numpy()

    def timed(run):
        for _ in range(warmup):
            run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            run()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    ms_a = timed(lambda: ap.compute(St, w["seed"], check=False, info=False))
    flags = ap.status()
    ap.close()
    out = {"config": {"workload": PLAIN_SMALL, "block": block, "l_max": l_max, "q": q,
                      "delta": round(delta, 6), "delta_rule": f"energy of the fixed plan's {modes} leading modes"},
           "l": l, "rank": rank, "residual": resid, "adaptive_ms": round(ms_a, 4), "flags": flags}
    for tag, lw in (("fixed_same_l", l), ("fixed_l_max", l_max)):
        plan = rp.Plan(m, n, lw - 10, 10, q, dtype=St.dtype, device=St.device)
        o = (torch.empty((lw - 10, m), dtype=plan.out_dtype, device=St.device),
             torch.empty((lw - 10,), dtype=torch.float64, device=St.device),
             torch.empty((n, lw - 10), dtype=plan.out_dtype, device=St.device))
        out[tag + "_ms"] = round(timed(lambda: plan.compute(St, w["seed"], out=o, check=False)), 4)
        plan.status()
        if tag == "fixed_same_l":
            s_f = o[1].cpu().numpy()
            k = min(20, len(s_f))
            out["sigma_leading20_rel_diff_vs_fixed_same_l"] = float(np.max(np.abs(sig_a[:k] - s_f[:k]) / s_f[:k]))
        plan.close()
    log(f"[bench] adaptive: {out}")
    return out


def reconstruct_block(St, N, reps=5):
    """The reduced-order fields of the first parameter block (its time average
    plus the 50 modes of the fluctuations weighted by their coefficients) and the
    relative L2 error of their time average against the block's snapshots."""
    import torch
    import paper_2504_15350_amd as rp
    w = WORKLOADS[PLAIN_SMALL]
    n, m = St.shape
    plan = rp.Plan(m, n, w["r"], w["p"], w["q"], dtype=St.dtype, device=St.device, block_cols=N)
    Phi_t, _, A_t = plan.compute(St, w["seed"])
    plan.close()
    q0 = St[:N].double().mean(0).float().contiguous()
    alpha_t = A_t[:N].contiguous()
    ref_t = St[:N]
    F, eps = rp.reconstruct(Phi_t, alpha_t, q0, ref_t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        rp.reconstruct(Phi_t, alpha_t, q0, ref_t, want_fields=True)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    gb = (N * m * 4 * 2 + m * w["r"] * 4) / 1e9  # fields written, reference read, modes read
    return {"time_steps": N, "ms": round(ms, 4), "gbs": round(gb / (ms * 1e-3), 1), "eps_time_average": eps}


def host_fp64(St_dev, chunk=500):
    """FP64 host copy (n x m) of a device snapshot matrix (exact for FP32 and 16-bit entries)."""
    import torch
    n, m = St_dev.shape
    out = np.empty((n, m), dtype=np.float64)
    o = torch.from_numpy(out)
    for t0 in range(0, n, chunk):
        o[t0:t0 + chunk].copy_(St_dev[t0:t0 + chunk].to(torch.float64))
    return out


def host_info():
    """Host cores seen and their model name (the oracle runs on them)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        blas = sorted({f"{i.get('internal_api')} {i.get('version')}" for i in threadpool_info()})
    except Exception:
        threads, blas = os.cpu_count(), []
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return dict(cpu_count=os.cpu_count(), affinity=affinity, blas_threads=int(threads), model=model, blas=blas)


def cpu_baseline(S64, w, seed, sample_rows, reps=3, m_total=None):
    """The oracle's FP64 rPOD (O2, as it stands) on the first sample_rows rows of
    S (host FP64, snapshot-major n x m), median of reps runs, scaled to the
    whole matrix (m_total rows, default m) by rows (every step of O2 is linear
    in m)."""
    from oracle import philox, pod
    from oracle import rpod as orpod
    import torch
    n, m = S64.shape
    rows = min(m, sample_rows)
    view = pod.SnapshotMajor(S64[:, :rows])
    om = philox.gaussian_sketch(seed, n, w["r"] + w["p"])
    if w["dtype"] != "f64":
        om = torch.from_numpy(om.astype(np.float32)).to(torch_dtype(w["dtype"])).double().numpy()
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        orpod.rpod_stable(view, w["r"], om, w["q"])
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    info = host_info()
    m_all = m if m_total is None else m_total
    scale = m_all / rows
    return dict(value=round(dt * scale * 1e3, 1), unit="ms", cores=info["blas_threads"], kind="oracle",
                sample=f"O2 (the oracle's FP64 rPOD with numpy/LAPACK, same algorithm, sketch and q) on the first "
                       f"{rows} of {m_all} rows of the same matrix, median of {reps} runs {dt:.2f} s "
                       f"(runs {', '.join(f'{x:.2f}' for x in times)} s), scaled x{scale:g} to the whole matrix",
                host=info)


def accuracy_block(S64, gen, w, results):
    """sigma and subspace errors of each GPU result against (a) O2 in FP64 on the
    unrounded FP32 matrix with the same sketch as that path (the Gaussian draws
    rounded to its storage type), so that the comparison isolates the effect of
    the storage precision, and (b) the closed-form POD of the noise-free field."""
    from oracle import metrics, philox, pod
    from oracle import rpod as orpod
    import torch
    n, m = S64.shape
    r, l, q = w["r"], w["r"] + w["p"], w["q"]
    om64 = philox.gaussian_sketch(w["seed"], n, l)
    tdt = {"bf16": torch.bfloat16, "f16": torch.float16, "fp32": torch.float32}
    s0 = pod.pod_sigma_sine_field(gen["amp"], gen["T"], w["nx"], w["ny"])[:r]
    noise = 1e-4 * (np.sqrt(m) + np.sqrt(n))   # spectral norm of the white noise (Bai-Yin limit)
    out = {"oracle": "O2 (FP64 rPOD, Householder QR after every product) on the FP32 matrix as generated, "
                     "with each path's own sketch (the Gaussian draws rounded to its storage type), q = 2; "
                     "and the closed-form POD of the noise-free field",
           "noise_bound_rel_sigma_r": float(noise / s0[-1]), "oracle_seconds": {}}
    for name, res in results.items():
        om = torch.from_numpy(om64).to(tdt[name]).double().numpy()
        t0 = time.perf_counter()
        log(f"[bench] oracle for the {name} sketch: FP64 rPOD of the whole matrix on the host cores ...")
        P2, s2, A2, ex = orpod.rpod_stable(pod.SnapshotMajor(S64), r, om, q, block_rows=32768, literal_A=False)
        out["oracle_seconds"][name] = round(time.perf_counter() - t0, 1)
        gap = bool(metrics.gap_ok(ex["ritz"], r))
        Phi_t, sig, _A = res["out"]
        Phi = Phi_t.double().cpu().numpy().T
        sg = sig.cpu().numpy()
        d = dict(sigma_rel_err_vs_oracle=metrics.sigma_rel_err(sg, s2),
                 sigma_rel_err_vs_noise_free_pod=metrics.sigma_rel_err(sg, s0),
                 oracle_sigma_rel_err_vs_noise_free_pod=metrics.sigma_rel_err(s2, s0),
                 orth=metrics.orth_err(Phi), cut_gapped=gap)
        if gap:
            d["sin_theta_vs_oracle"] = metrics.sin_theta_max(Phi, P2)
        d["within_1e-3"] = bool(d["sigma_rel_err_vs_oracle"] <= 1e-3 and d.get("sin_theta_vs_oracle", 0.0) <= 1e-3)
        out[name] = d
        log(f"[bench] accuracy {name}: {d}")
    return out


def vendor_gemm_reference(S16, lp, reps=5):
    """For context: torch.matmul (hipBLASLt) BF16 GEMMs of the pass shapes on the same matrix,
    S X (X: n x lp), S^T Q (Q: m x lp) and S^T [Q_hi Q_lo] (2 lp columns, the refinement pass's
    work). Random operands; BF16 outputs (FP32 accumulation inside)."""
    import torch
    n, m = S16.shape
    dev = S16.device
    g = torch.Generator(device=dev)
    g.manual_seed(11)
    X = torch.randn((n, lp), generator=g, device=dev).to(torch.bfloat16)
    Q = torch.randn((m, lp), generator=g, device=dev).to(torch.bfloat16)
    Q2 = torch.randn((m, 2 * lp), generator=g, device=dev).to(torch.bfloat16)
    S = S16.t()  # the m x n matrix, column-major
    out = {}
    for name, f in (("S_X", lambda: torch.matmul(S, X)), ("St_Q", lambda: torch.matmul(S16, Q)),
                    ("St_Q_2lp", lambda: torch.matmul(S16, Q2))):
        for _ in range(2):
            f()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            f()
        e1.record()
        torch.cuda.synchronize()
        out[name] = round(e0.elapsed_time(e1) / reps, 4)
    del X, Q, Q2
    torch.cuda.empty_cache()
    log(f"[bench] torch.matmul (hipBLASLt) BF16 at the pass shapes: {out} ms")
    return out


def mixed_block(dev, steps, warmup, accuracy=True, cpu=True, others=True):
    """The headline workload in BF16 (the value) and, on the same matrix, plain
    FP32 (the in-GPU baseline) and FP16."""
    import torch
    import synth
    w = WORKLOADS[DEFAULT]
    t0 = time.perf_counter()
    gen = synth.fourier_field_device(w["nx"], w["ny"], w["n"], seed=w["gen_seed"], dtype=torch.float32, device=dev)
    S32 = gen.pop("St")
    torch.cuda.synchronize()
    log(f"[bench] generated S {S32.shape[1]}x{S32.shape[0]} FP32 in {time.perf_counter() - t0:.1f} s")
    keep = accuracy
    S16 = S32.to(torch.bfloat16)
    res = {"bf16": measure(DEFAULT, S16, steps, warmup, keep_out=keep)}
    vendor = vendor_gemm_reference(S16, 128) if others else None
    del S16
    torch.cuda.empty_cache()
    if others:
        ext_steps, ext_warm = max(3, steps // 2), max(1, warmup // 2)
        Sh = S32.to(torch.float16)
        res["f16"] = measure("f16_1048576x10000", Sh, ext_steps, ext_warm, keep_out=keep)
        del Sh
        torch.cuda.empty_cache()
        res["fp32"] = measure("fp32_1048576x10000", S32, ext_steps, ext_warm, keep_out=keep)
    acc = cpu_res = None
    if accuracy or cpu:
        t0 = time.perf_counter()
        S64 = host_fp64(S32)
        log(f"[bench] FP64 host copy of S ({S64.nbytes / 1e9:.0f} GB) in {time.perf_counter() - t0:.1f} s")
        del S32
        torch.cuda.empty_cache()
        if accuracy:
            acc = accuracy_block(S64, gen, w, res)
        if cpu:
            log("[bench] timing the CPU oracle on a row sample ...")
            cpu_res = cpu_baseline(S64, w, w["seed"], w["sample_rows"])
            log(f"[bench] cpu baseline {cpu_res['value']:.0f} ms ({cpu_res['sample']})")
        del S64
    else:
        del S32
    for v in res.values():
        v.pop("out", None)
    torch.cuda.empty_cache()
    if vendor is not None:
        res["vendor_gemm_ms"] = vendor
    return res, acc, cpu_res


def simple_block(name, dev, steps, warmup, cpu=True):
    """One workload alone (profiling runs): time it, CPU baseline on a row sample."""
    import torch
    w = WORKLOADS[name]
    t0 = time.perf_counter()
    St = make_input(w, dev)
    torch.cuda.synchronize()
    log(f"[bench] generated S {St.shape[1]}x{St.shape[0]} {St.dtype} in {time.perf_counter() - t0:.1f} s")
    r = measure(name, St, steps, warmup)
    cpu_res = None
    if cpu:
        rows = min(St.shape[1], w["sample_rows"])
        S64 = host_fp64(St[:, :rows])
        cpu_res = cpu_baseline(S64, w, w["seed"], rows, m_total=St.shape[1])
    return r, cpu_res, St


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS) + [PAPER_NAME])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the oracle comparison of the mixed workload")
    ap.add_argument("--no-extra", action="store_true", help="skip the 262144 x 5000 FP32 measurement")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-matrix batch measurement")
    ap.add_argument("--no-warm", action="store_true", help="skip the warm-start sweep")
    ap.add_argument("--no-center", action="store_true", help="skip the fluctuation-centring measurement")
    ap.add_argument("--no-adaptive", action="store_true", help="skip the adaptive-rank measurement")
    ap.add_argument("--headline-only", action="store_true",
                    help="on the headline workload, time BF16 alone (no FP16 / FP32 runs on the same matrix)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run 5 device-to-device copies of BYTES bytes (the reference kernel for scaling "
                         "HBM byte counters) and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n * 4, "copies": 5}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the row-sharded multi-GPU "
              f"design is not built in this version", file=sys.stderr)
        sys.exit(2)
    if args.workload == PAPER_NAME:
        import torch
        res = paper_block(torch.device("cuda", 0), args.steps, args.warmup, cpu=not args.no_cpu_baseline,
                          accuracy=not args.no_accuracy)
        f = res["fields"]["psi_like"]
        b = f["by_p"]["75"]["bf16"] if "by_p" in f else f["gpu"]["bf16_p75"]
        line = {"metric": "rPOD time-to-r-modes", "value": b["ms"], "unit": "ms", "n_gpus": 1, "steps": args.steps,
                "warmup": args.warmup, "ms_per_step": b["ms"], "higher_is_better": False, "scaling": "weak",
                "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
                "config": {"workload": PAPER_NAME, "field": "psi_like", "r": 10, "p": 75, "q": 1,
                           "parallelism": "single GPU"},
                "paper_shape": res}
        print(json.dumps(line), flush=True)
        return

    import torch
    dev = torch.device("cuda", 0)
    w = WORKLOADS[args.workload]
    mixed = None
    if args.workload == DEFAULT:
        res, acc, cpu = mixed_block(dev, args.steps, args.warmup, accuracy=not args.no_accuracy,
                                    cpu=not args.no_cpu_baseline, others=not args.headline_only)
        main_res = res["bf16"]
        mixed = {"config": {"m": 1048576, "n": 10000, "r": 100, "p": 20, "q": 2},
                 "mixed_bf16_ms": round(res["bf16"]["ms"], 3), "accuracy": acc}
        if "fp32" in res:
            mixed.update({
                "mixed_f16_ms": round(res["f16"]["ms"], 3), "plain_fp32_ms": round(res["fp32"]["ms"], 3),
                "speedup_bf16_vs_plain_fp32": round(res["fp32"]["ms"] / res["bf16"]["ms"], 2),
                "speedup_f16_vs_plain_fp32": round(res["fp32"]["ms"] / res["f16"]["ms"], 2),
                "f16_roofline": res["f16"]["roofline"], "f16_kernels": res["f16"]["kernels"],
                "plain_roofline": res["fp32"]["roofline"], "plain_kernels": res["fp32"]["kernels"],
                "plain_hbm_gbs_s_passes": res["fp32"]["hbm_gbs_s_passes"]})
        if "vendor_gemm_ms" in res:
            k = res["bf16"]["kernels"]
            mixed["vendor_gemm_reference"] = {
                "what": "torch.matmul (hipBLASLt) BF16 GEMMs with the shapes of the passes over this matrix, random "
                        "operands, l = 128 (S_X: S X; St_Q: S^T Q; St_Q_2lp: S^T Q with 2 l columns, the refinement "
                        "pass's matrix-core work), beside this library's average pass times",
                "hipblaslt_ms": res["vendor_gemm_ms"],
                "library_ms": {kk: k[kk]["avg_ms"] for kk in ("S_X", "St_Q", "St_Q_refine") if kk in k}}
        St_small = None
    else:
        main_res, cpu, St_small = simple_block(args.workload, dev, args.steps, args.warmup,
                                               cpu=not args.no_cpu_baseline)

    extra = energy = center = adaptive = None
    if args.workload == DEFAULT and not (args.no_extra and args.no_center):
        t0 = time.perf_counter()
        St_small = make_input(WORKLOADS[PLAIN_SMALL], dev)
        torch.cuda.synchronize()
        log(f"[bench] generated {PLAIN_SMALL} in {time.perf_counter() - t0:.1f} s")
    if args.workload == DEFAULT and not args.no_extra:
        e = measure(PLAIN_SMALL, St_small, args.steps, args.warmup)
        extra = {"ms": round(e["ms"], 4), "ms_graph_replay": round(e["ms_graph"], 4), "roofline": e["roofline"],
                 "kernels": e["kernels"], "hbm_gbs_s_passes": e["hbm_gbs_s_passes"],
                 "config": {"m": 262144, "n": 5000, "r": 50, "p": 10, "q": 2}}
    if St_small is not None and args.workload in (DEFAULT, PLAIN_SMALL) and not args.no_center:
        base = measure(PLAIN_SMALL, St_small, max(3, args.steps // 2), max(1, args.warmup // 2))
        e_res = measure(PLAIN_SMALL, St_small, max(3, args.steps // 2), max(1, args.warmup // 2), energy=True)
        e, rk = e_res["energy"]
        energy = {"with_energy_ms": round(e_res["ms"], 4), "plain_ms": round(base["ms"], 4),
                  "overhead": round(e_res["ms"] / base["ms"] - 1.0, 4),
                  "energy_first_10": [round(float(x), 6) for x in e[:10]], "energy_at_l": round(float(e[-1]), 6),
                  "rank_for_0.9": rk}
        log(f"[bench] energy: {energy}")
        if not args.no_adaptive:
            adaptive = adaptive_block(St_small, e, max(3, args.steps // 2), max(1, args.warmup // 2))
        center = center_block(St_small, max(3, args.steps // 2), max(1, args.warmup // 2))
        log(f"[bench] centring: plain {center['plain_ms']:.3f} ms, centred {center['centred_ms']:.3f} ms")
    del St_small
    torch.cuda.empty_cache()

    batch = None
    if not args.no_batch:
        batch = batch_block(dev, max(3, args.steps // 4), max(1, args.warmup // 2))

    warm = None
    if not args.no_warm:
        warm = warm_block(dev, 3)

    res = {
        "metric": "rPOD time-to-r-modes",
        "value": round(main_res["ms"], 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms"], 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": w["dtype"],
        "data": "synthetic",
        "config": {"workload": args.workload, "description": w["label"],
                   "m": w.get("m", w.get("nx", 0) * w.get("ny", 0)), "n": w["n"],
                   "r": w["r"], "p": w["p"], "q": w["q"], "parallelism": "single GPU"},
        "hbm_gbs_s_passes": main_res["hbm_gbs_s_passes"],
        "ms_graph_replay": round(main_res["ms_graph"], 4),
        "kernels": main_res["kernels"],
        "roofline": main_res["roofline"],
        "cpu_baseline": cpu,
        "mixed_vs_plain": mixed,
        "plain_fp32_262144x5000": extra,
        "batched_vs_plain": batch,
        "warm_vs_plain": warm,
        "centred_vs_plain": center,
        "energy_report": energy,
        "adaptive_vs_fixed": adaptive,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
