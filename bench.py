#!/usr/bin/env python3
"""Benchmark of the MR-STAT hot path on one MI355X.

Workload: 224x224 brain-like phantom (B1 in [0.8, 1.2]), 1120 TRs
(224 phase-encode lines x 5 sweeps, sine-squared flip train 0-70 degrees),
448 readout samples per TR (2x oversampled), K = 32 EPG states, one coil.

Step: one inexact Gauss-Newton iteration through the C ABI (mrstat_gn_step):
linearisation (trains and their derivatives), residual and objective,
gradient g = Re(J^H r), n_cg = 20 CG iterations (each one J v + one J^H w
pair with FP64 reductions) and one line-search trial (value-only trains +
residual). Metric: J v + J^H w pairs per second, GN-amortised (n_cg pairs per
step), for two forms on the same workload and starting point:
  - surrogate + split-BF16 (the reported value): the learned network gives
    the trains (BF16 MFMA, EPG fallback outside its box, iterates projected
    onto that box), stored in FP16; the encoding contraction runs in
    split-BF16 on MFMA;
  - plain FP32: EPG trains, FP32 MFMA encoding contraction.
The network is trained first, untimed, on 2M EPG samples the library
simulates itself.

The JSON line also reports, for the dominant kernel, its roofline from HIP
events taken live over the timed region, the surrogate inference kernel's
roofline, and the FP64 CPU oracle timed on a bounded sample of the same
workload on this host.
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
BF16_MFMA_PEAK_TFLOPS = 2500.0    # dense
FP32_VALU_PEAK_TFLOPS = 157.3     # published vector peak (packed FP32; 78.6 unpacked)

# Algorithmic work per launch, counted from the method's arithmetic.
EPG_FLOP_PER_STATE_TR = {4: 67,   # value 13 + ln T1 15 + ln T2 17 + B1 22 (real form)
                         3: 45}   # B1 held fixed: no B1 tangent
# Kernel kinds traced in the timed region (the roofline candidates).
TRACED_KINDS = ["epg", "epg_value", "ystage_fwd_signal", "ystage_fwd_jv", "ystage_adj",
                "surrogate", "surrogate_value"]


def algorithmic(kind, prob, tb=4, ntr=4):
    """(unit, amount per launch, bound) for a kernel kind; tb = bytes per
    stored train value, ntr = trains of the linearisation (4, or 3 when B1 is
    held fixed: no dm/dB1 train)."""
    T, nv, nx, C = prob.n_tr, prob.nv, prob.nx, prob.n_coils
    if kind == "ystage_fwd_jv":   # ntr trains + rho and ntr + 1 direction rows in, U out
        return "bytes", ntr * tb * T * nv + (8 + 4 * (ntr + 1)) * nv + 8 * C * T * nx, "hbm"
    if kind == "ystage_fwd_signal":   # m train + rho in, U out
        return "bytes", tb * T * nv + 8 * nv + 8 * C * T * nx, "hbm"
    if kind == "ystage_adj":      # ntr trains + W in
        return "bytes", ntr * tb * T * nv + 8 * C * T * nx, "hbm"
    if kind == "epg":
        return "flop", EPG_FLOP_PER_STATE_TR[ntr] * prob.n_states * T * nv, "alu"
    return None


def surrogate_work(prob, width=256, depth=4, bytes_per_value=2, ntr=4):
    """Per linearisation through the network with ntr trains (hidden-layer
    kernel + output-layer kernel): (flop, bytes written). Multiply-adds of the
    first layer, the hidden layers and the ntr n_tr imaginary outputs; the
    trains written once (FP16 by default)."""
    macs = 3 * width + (depth - 1) * width * width + ntr * prob.n_tr * width
    return 2 * macs * prob.nv, ntr * bytes_per_value * prob.n_tr * prob.nv


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
    ap.add_argument("--train-epochs", type=int, default=40)
    ap.add_argument("--train-samples", type=int, default=2_000_000)
    ap.add_argument("--form", choices=["both", "surrogate", "plain"], default="both")
    return ap.parse_args()


def cpu_baseline(work, n_cg, n_vox=16384, n_pairs=8):
    """The oracle as it stands, on this host: EPG with tangents on a voxel
    sample (scaled to all voxels) plus n_pairs full-size J v + J^H w pairs
    (about 7 s of CPU work at 224 x 224, 1120 TRs on 16 threads)."""
    import oracle
    from paper_1904_13244_amd import inputs as I

    oracle.build(force=False)
    prob = work.problem
    S = min(n_vox, prob.nv)
    sel = np.linspace(0, prob.nv - 1, S).astype(np.int64)
    sub = I.make_problem(S, 1, prob.n_tr, prob.n_read, prob.n_states, flip_deg=prob.flip_deg)
    t0 = time.perf_counter()
    oracle.epg(sub, work.theta[:, sel])
    t_sample = time.perf_counter() - t0
    t_lin = t_sample * prob.nv / S
    trains = np.full((4, prob.n_tr, prob.nv), 1e-3 + 1e-3j, dtype=np.complex128)
    v, w = I.probe_vectors(prob)
    t0 = time.perf_counter()
    for _ in range(n_pairs):
        y = oracle.jv(prob, work.theta, trains, v)
        oracle.jhw(prob, work.theta, trains, y)
    t_pairs = time.perf_counter() - t0
    t_pair = t_pairs / n_pairs
    del trains
    t_step = t_lin + (n_cg + 1) * t_pair   # residual + gradient cost about one pair
    return {"value": n_cg / t_step, "unit": "pairs/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": (f"FP64 oracle: EPG with tangents on {S} of {prob.nv} voxels "
                       f"({t_sample:.2f} s, scaled x{prob.nv / S:.2f}) + {n_pairs} full-size "
                       f"Jv + J^H w pairs ({t_pairs:.2f} s); GN-amortised with n_cg = {n_cg}: "
                       f"t_step = t_lin + (n_cg + 1) t_pair = {t_step:.1f} s")}


def roofline_for(kernels, prob, tb, ntr):
    cand = [k for k in kernels if algorithmic(k, prob, tb, ntr)]
    if not cand:
        return None
    rk = max(cand, key=lambda k: kernels[k]["ms_per_step"])
    unit, amount, bound = algorithmic(rk, prob, tb, ntr)
    t = kernels[rk]["avg_ms"] * 1e-3
    if unit == "bytes":
        ach = amount / t / 1e9
        return {"kernel": rk, "bound": bound, "achieved": ach, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "traffic": measured_traffic(rk + ("_f16" if tb == 2 else "_f32")),
                "algorithmic_bytes_per_launch": amount}
    ach = amount / t / 1e12
    return {"kernel": rk, "bound": bound, "achieved": ach, "peak": FP32_VALU_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": ach / FP32_VALU_PEAK_TFLOPS, "traffic": None,
            "algorithmic_flop_per_launch": amount}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1904_13244_amd import binding as B
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
    vv, ww = I.probe_vectors(prob, work.param_mask)
    vd, wd = dev(vv, torch.float32), dev(ww, torch.complex64)
    # B1 held fixed: the GN step's linearisation has no dm/dB1 train.
    ntr = 4 if (work.param_mask >> 2) & 1 else 3

    def run_form(net, enc, lo, hi, trains):
        ctx.set_surrogate(net)
        ctx.set_encoding(enc)
        ctx.set_train_precision(trains)
        theta = dev(th0, torch.float32)

        def step():
            return ctx.gn_step(theta, data, args.n_cg, work.param_mask, lo, hi, n_ls_max=1)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        # Timed region: only the kernels the roofline is taken on are traced
        # (two events per traced launch), live on the library's stream.
        ctx.profile_select(TRACED_KINDS)
        ctx.profile(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            rep = step()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        prof = ctx.profile_read()
        ctx.profile(False)
        kernels = {k: {"launches": n, "avg_ms": (ms / n if n else 0.0), "ms_per_step": ms / args.steps}
                   for k, (n, ms) in prof.items() if n}
        # Every kind, from one more (untimed) step with full tracing.
        ctx.profile_select(None)
        ctx.profile(True)
        step()
        full = ctx.profile_read()
        ctx.profile(False)
        breakdown = {k: {"launches": n, "ms": ms} for k, (n, ms) in full.items() if n}
        # Cached pair (reuse = 1) and linearisation, outside the timed loop.
        ctx.linearise(theta)
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
        return {"value": args.n_cg * args.steps / elapsed, "ms_per_step": 1e3 * elapsed / args.steps,
                "kernels": kernels, "step_breakdown_untimed": breakdown,
                "dominant_kernel": max(breakdown, key=lambda k: breakdown[k]["ms"]),
                "roofline": roofline_for(kernels, prob, 2 if trains == B.TRAINS_FP16 else 4, ntr),
                "pair_cached_ms": pair_ms,
                "pairs_per_s_cached": 1e3 / pair_ms, "linearise_ms": lin_ms,
                "gn_report_last": rep.as_dict()}

    forms = {}
    if args.form in ("both", "plain"):
        forms["plain_fp32"] = run_form(None, B.ENC_FP32, I.GN_LO, I.GN_HI, B.TRAINS_FP32)
    surr_info = None
    if args.form in ("both", "surrogate"):
        from paper_1904_13244_amd.surrogate import train_surrogate
        net, trep = train_surrogate(torch, prob, n_samples=args.train_samples, epochs=args.train_epochs)
        lo = tuple(max(a, b) for a, b in zip(I.GN_LO, I.SURR_LO))
        hi = tuple(min(a, b) for a, b in zip(I.GN_HI, I.SURR_HI))
        f = run_form(net, B.ENC_SPLIT_BF16, lo, hi, B.TRAINS_FP16)
        forms["surrogate_split_bf16"] = f
        flop, wbytes = surrogate_work(prob, ntr=ntr)
        k = f["kernels"].get("surrogate")
        t = k["avg_ms"] * 1e-3 if k else None
        surr_info = {
            "training": {"samples": trep.n_samples, "steps": trep.steps, "batch": net.batch,
                         "seconds_data": trep.seconds_data, "seconds_train": trep.seconds_train,
                         "loss_first": trep.loss_first, "loss_last": trep.loss_last,
                         "heldout_rel_err": dict(zip(["m", "dm_dlnT1", "dm_dlnT2", "dm_dB1"],
                                                     trep.val_rel_err))},
            "inference_roofline": None if t is None else {
                "kernel": (f"surrogate (hidden-layer + output-layer kernels, {ntr} trains, "
                           "FP16 out)"),
                "bound": "hbm", "achieved": wbytes / t / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": wbytes / t / 1e9 / HBM_PEAK_GBS,
                "mfma_tflops": flop / t / 1e12, "mfma_frac": flop / t / 1e12 / BF16_MFMA_PEAK_TFLOPS,
                "algorithmic_bytes_per_launch": wbytes, "algorithmic_flop_per_launch": flop},
        }

    if args.calib_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    chosen = "surrogate_split_bf16" if "surrogate_split_bf16" in forms else "plain_fp32"
    c = forms[chosen]
    out = {
        "metric": METRIC, "value": c["value"], "unit": "pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": c["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp32+bf16" if chosen.startswith("surrogate") else "fp32",
        "data": "synthetic",
        "config": {"workload": ("224x224 brain-like phantom, 1120 TRs (224 lines x 5 sweeps), "
                                "448 readout samples, K=32 EPG states, 1 coil; T1, T2, rho fitted "
                                "with B1 known (no dm/dB1 train); one GN step = "
                                "linearise + r + g + 20 CG pairs + 1 line-search trial"),
                   "form": {"surrogate_split_bf16": "surrogate trains (BF16 MFMA network, EPG "
                                                    "fallback, FP16 storage) + split-BF16 MFMA "
                                                    "encoding contraction",
                            "plain_fp32": "plain FP32 EPG + FP32 MFMA encoding contraction"}[chosen],
                   "n_cg": args.n_cg, "parallelism": "single GPU"},
        "roofline": c["roofline"],
        "dominant_kernel": c["dominant_kernel"],
        "kernels": c["kernels"],
        "step_breakdown_untimed": c["step_breakdown_untimed"],
        "pair_cached_ms": c["pair_cached_ms"],
        "pairs_per_s_cached": c["pairs_per_s_cached"],
        "linearise_ms": c["linearise_ms"],
        "gn_report_last": c["gn_report_last"],
    }
    if "plain_fp32" in forms and chosen != "plain_fp32":
        p = forms["plain_fp32"]
        out["plain_fp32"] = {k: p[k] for k in ("value", "ms_per_step", "pair_cached_ms",
                                               "pairs_per_s_cached", "linearise_ms", "roofline",
                                               "kernels", "step_breakdown_untimed")}
        out["speedup_vs_plain_fp32"] = c["value"] / p["value"]
    if surr_info:
        out["surrogate"] = surr_info
    ctx.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(work, args.n_cg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
