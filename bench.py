#!/usr/bin/env python3
"""Benchmark of the MR-STAT hot path on one MI355X.

Workload: 224x224 brain-like phantom (B1 in [0.8, 1.2]), 1120 TRs
(224 phase-encode lines x 5 sweeps, sine-squared flip train 0-70 degrees),
448 readout samples per TR (2x oversampled), K = 32 EPG states, one coil.

Step: one inexact Gauss-Newton iteration through the C ABI (mrstat_gn_step):
EPG linearisation with tangents, residual and objective, gradient
g = Re(J^H r), n_cg = 20 CG iterations (each one J v + one J^H w pair with
FP64 reductions) and one line-search trial (value-only EPG + residual).
Metric: J v + J^H w pairs per second, GN-amortised (n_cg pairs per step).

The JSON line also reports, for the dominant kernel, its roofline from HIP
events taken live over the timed region, and the FP64 CPU oracle timed on a
bounded sample of the same workload on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Jv+Jᴴw pairs/s at 224², 1120 TRs: surrogate+split-BF16 vs plain FP32"
HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK_TFLOPS = 157.3     # published vector peak (packed); see the design doc

# Algorithmic work per launch (the design doc derives each figure).
EPG_FLOP_PER_STATE_TR = 67        # value 13 + ln T1 15 + ln T2 17 + B1 22 (real form)


def algorithmic(kind, prob):
    """(unit, amount per launch, bound) for a kernel kind."""
    T, nv, nx, C = prob.n_tr, prob.nv, prob.nx, prob.n_coils
    if kind == "ystage_fwd_jv":   # 4 trains + per-voxel weights in, U out
        return "bytes", 16 * T * nv + 28 * nv + 8 * C * T * nx, "hbm"
    if kind == "ystage_fwd_signal":   # m train + rho in, U out
        return "bytes", 4 * T * nv + 8 * nv + 8 * C * T * nx, "hbm"
    if kind == "ystage_adj":      # 4 trains + W in
        return "bytes", 16 * T * nv + 8 * C * T * nx, "hbm"
    if kind == "epg":
        return "flop", EPG_FLOP_PER_STATE_TR * prob.n_states * T * nv, "alu"
    return None


def measured_traffic(kind):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, or None when the kernel source changed since it was taken."""
    import hashlib
    src = os.path.join(ROOT, "paper_1904_13244_amd", "csrc", "encode.hip")
    summary = os.path.join(ROOT, "profiles", "hbm_traffic_224x224_1120tr.txt")
    if not os.path.exists(summary):
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for line in open(summary):
        f = line.split()
        if len(f) == 4 and f[0] == "TRAFFIC" and f[1] == kind and f[2] == sha:
            return float(f[3])
    return None


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n-cg", type=int, default=20)
    ap.add_argument("--epg-lanes", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    return ap.parse_args()


def cpu_baseline(work, n_cg):
    """The oracle as it stands, on this host: EPG with tangents on a voxel
    sample (scaled to all voxels) plus one full-size J v + J^H w pair."""
    import oracle
    from paper_1904_13244_amd import inputs as I

    oracle.build(force=False)
    prob = work.problem
    S = 2048
    sel = np.linspace(0, prob.nv - 1, S).astype(np.int64)
    sub = I.make_problem(S, 1, prob.n_tr, prob.n_read, prob.n_states, flip_deg=prob.flip_deg)
    t0 = time.perf_counter()
    oracle.epg(sub, work.theta[:, sel])
    t_lin = (time.perf_counter() - t0) * prob.nv / S
    trains = np.full((4, prob.n_tr, prob.nv), 1e-3 + 1e-3j, dtype=np.complex128)
    v, w = I.probe_vectors(prob)
    t0 = time.perf_counter()
    y = oracle.jv(prob, work.theta, trains, v)
    oracle.jhw(prob, work.theta, trains, y)
    t_pair = time.perf_counter() - t0
    del trains
    t_step = t_lin + (n_cg + 1) * t_pair   # residual + gradient cost about one pair
    return {"value": n_cg / t_step, "unit": "pairs/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": (f"FP64 oracle: EPG with tangents on {S} of {prob.nv} voxels "
                       f"({t_lin * S / prob.nv:.2f} s, scaled x{prob.nv / S:.1f}) + one "
                       f"full-size Jv + J^H w pair ({t_pair:.2f} s); GN-amortised with "
                       f"n_cg = {n_cg}: t_step = t_lin + (n_cg + 1) t_pair = {t_step:.1f} s")}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1904_13244_amd import inputs as I
    from paper_1904_13244_amd.binding import Context

    torch.cuda.set_device(0)
    work = I.config(3)
    prob = work.problem
    dev = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt)  # noqa: E731

    ctx = Context(prob)
    if args.epg_lanes:
        ctx.set_epg_lanes(args.epg_lanes)
    th_true = dev(work.theta, torch.float32)
    zeros = torch.zeros(prob.data_shape, dtype=torch.complex64, device="cuda")
    _, r = ctx.residual(th_true, zeros)
    data = (-r).contiguous()                   # d = s(theta_true), noiseless
    rng = np.random.default_rng(I.SEED_PROBE)
    th0 = work.theta.copy()
    th0[0] += 0.05 * rng.standard_normal(prob.nv)
    th0[1] += 0.05 * rng.standard_normal(prob.nv)
    th0[2] += 0.02 * rng.standard_normal(prob.nv)
    theta = dev(th0, torch.float32)

    def step():
        return ctx.gn_step(theta, data, args.n_cg, work.param_mask, I.GN_LO, I.GN_HI, n_ls_max=1)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rep = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile(False)
    ms_step = 1e3 * elapsed / args.steps
    value = args.n_cg * args.steps / elapsed

    # Per-kernel averages over the timed region and the dominant kernel.
    kernels = {k: {"launches": n, "avg_ms": (ms / n if n else 0.0), "ms_per_step": ms / args.steps}
               for k, (n, ms) in prof.items() if n}
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    roof = None
    cand = [k for k in kernels if algorithmic(k, prob)]
    if cand:
        rk = max(cand, key=lambda k: kernels[k]["ms_per_step"])
        unit, amount, bound = algorithmic(rk, prob)
        t = kernels[rk]["avg_ms"] * 1e-3
        if unit == "bytes":
            ach = amount / t / 1e9
            roof = {"kernel": rk, "bound": bound, "achieved": ach, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": measured_traffic(rk),
                    "algorithmic_bytes_per_launch": amount}
        else:
            ach = amount / t / 1e12
            roof = {"kernel": rk, "bound": bound, "achieved": ach, "peak": FP32_VALU_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": ach / FP32_VALU_PEAK_TFLOPS, "traffic": None,
                    "algorithmic_flop_per_launch": amount}

    # Cached pair time (reuse = 1) and linearisation time, outside the timed loop.
    ctx.linearise(theta)
    vv, ww = I.probe_vectors(prob, work.param_mask)
    vd, wd = dev(vv, torch.float32), dev(ww, torch.complex64)
    jv_out = torch.empty(prob.data_shape, dtype=torch.complex64, device="cuda")
    g_out = torch.empty((5, prob.nv), dtype=torch.float32, device="cuda")
    for _ in range(3):
        ctx.jv(theta, vd, reuse=True, out=jv_out)
        ctx.jhw(theta, wd, reuse=True, out=g_out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        ctx.jv(theta, vd, reuse=True, out=jv_out)
        ctx.jhw(theta, wd, reuse=True, out=g_out)
    e1.record()
    torch.cuda.synchronize()
    pair_ms = e0.elapsed_time(e1) / 20
    e0.record()
    for _ in range(5):
        ctx.linearise(theta)
    e1.record()
    torch.cuda.synchronize()
    lin_ms = e0.elapsed_time(e1) / 5

    if args.calib_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    out = {
        "metric": METRIC, "value": value, "unit": "pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": ("224x224 brain-like phantom, 1120 TRs (224 lines x 5 sweeps), "
                                "448 readout samples, K=32 EPG states, 1 coil; one GN step = "
                                "linearise + r + g + 20 CG pairs + 1 line-search trial"),
                   "form": "plain FP32 EPG + FP32 MFMA encoding contraction",
                   "n_cg": args.n_cg, "parallelism": "single GPU"},
        "roofline": roof,
        "dominant_kernel": dom,
        "kernels": kernels,
        "pair_cached_ms": pair_ms,
        "pairs_per_s_cached": 1e3 / pair_ms,
        "linearise_ms": lin_ms,
        "gn_report_last": rep.as_dict(),
    }
    ctx.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(work, args.n_cg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
