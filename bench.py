#!/usr/bin/env python3
"""Benchmark of the MR-STAT hot path on one MI355X.

Workload: 224x224 brain-like phantom (B1 in [0.8, 1.2]), 1120 TRs
(224 phase-encode lines x 5 sweeps, sine-squared flip train 0-70 degrees),
448 readout samples per TR (2x oversampled), K = 32 EPG states, one coil.

Step: one inexact Gauss-Newton iteration through the C ABI (mrstat_gn_step)
fitting all five parameters (ln T1, ln T2, B1, Re rho, Im rho): linearisation
(m and its derivatives in ln T1, ln T2 and B1: four trains), residual and
objective, gradient g = Re(J^H r), n_cg = 20 CG iterations (each one J v + one
J^H w pair with FP64 reductions) and one line-search trial (value-only trains
+ residual). Metric: J v + J^H w pairs per second, GN-amortised (n_cg pairs
per step), for two forms on the same workload and starting point:
  - surrogate + split-BF16 (the reported value): the learned network gives
    the trains (BF16 MFMA, EPG fallback outside its box, iterates projected
    onto that box), stored in FP16; the encoding contraction runs in
    split-BF16 on MFMA;
  - plain FP32: EPG trains, FP32 MFMA encoding contraction.
The same two forms are also timed with B1 held known (three trains, no
dm/dB1), reported as a labelled variant. The network is trained first,
untimed, on 2M EPG samples the library simulates itself.

The JSON line also reports, for the dominant kernel, its roofline from HIP
events taken live over the timed region, the surrogate inference kernel's
roofline, fresh-pair times (every product re-linearises), the surrogate's
linearisation with a share of voxels outside its box, and the FP64 CPU oracle
timed on a bounded sample of the same workload on this host.
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
    ap.add_argument("--no-b1-known", action="store_true",
                    help="skip the B1-known (three-train) variant")
    ap.add_argument("--no-noncartesian", action="store_true",
                    help="skip the golden-angle radial contraction measurement")
    ap.add_argument("--no-isochromats", action="store_true",
                    help="skip the balanced isochromat model's linearisation measurement")
    ap.add_argument("--no-readout-dynamics", action="store_true",
                    help="skip the readout-dynamics (T2 decay and off-resonance per sample) measurement")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--train-epochs", type=int, default=None,
                    help="epochs of surrogate training (default: the library's recipe)")
    ap.add_argument("--train-samples", type=int, default=2_000_000)
    ap.add_argument("--form", choices=["both", "surrogate", "plain"], default="both")
    return ap.parse_args()


def _host_cpu():
    """Host CPU description from lscpu (model, sockets, cores per socket)."""
    import subprocess
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            info[k.strip()] = v.strip()
    except Exception:
        pass
    return {"model": info.get("Model name"), "sockets": info.get("Socket(s)"),
            "cores_per_socket": info.get("Core(s) per socket"), "cpus": info.get("CPU(s)"),
            "nproc": os.cpu_count()}


_ONE_THREAD = r"""
import sys, time, json
import numpy as np
sys.path.insert(0, {root!r})
import oracle
from paper_1904_13244_amd import inputs as I
w = I.config(3)
prob = w.problem
S = {nvox}
sel = np.linspace(0, prob.nv - 1, S).astype(np.int64)
sub = I.make_problem(S, 1, prob.n_tr, prob.n_read, prob.n_states, flip_deg=prob.flip_deg)
t0 = time.perf_counter(); oracle.epg(sub, w.theta[:, sel]); t_lin = (time.perf_counter() - t0) * prob.nv / S
t0 = time.perf_counter(); oracle.epg(sub, w.theta[:, sel], tangents=False)
t_val = (time.perf_counter() - t0) * prob.nv / S
trains = np.full((4, prob.n_tr, prob.nv), 1e-3 + 1e-3j, dtype=np.complex128)
v, ww = I.probe_vectors(prob)
t0 = time.perf_counter(); y = oracle.jv(prob, w.theta, trains, v); oracle.jhw(prob, w.theta, trains, y)
t_pair = time.perf_counter() - t0
print(json.dumps(dict(threads=oracle.num_threads(), t_lin=t_lin, t_val=t_val, t_pair=t_pair)))
"""


def cpu_baseline(work, n_cg, n_vox=16384, n_pairs=6, n_vox_1t=1024):
    """The oracle as it stands, on this host: EPG with tangents (and the
    value-only EPG of the line-search trial) on a voxel sample scaled to all
    voxels, plus full-size J v + J^H w pairs, on all host threads; the same
    with one thread (a smaller voxel sample and one pair, in a child process).
    GN-amortised like the GPU step: t_step = t_lin + (n_cg + 1) t_pair +
    t_trial, the gradient costing about one pair and the trial a value-only
    EPG plus a residual (about half a pair)."""
    import subprocess

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
    t0 = time.perf_counter()
    oracle.epg(sub, work.theta[:, sel], tangents=False)
    t_val = (time.perf_counter() - t0) * prob.nv / S
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
    t_step = t_lin + (n_cg + 1) * t_pair + t_val + 0.5 * t_pair
    one = None
    try:
        env = dict(os.environ, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, "-c", _ONE_THREAD.format(root=ROOT, nvox=n_vox_1t)],
                           capture_output=True, text=True, env=env, timeout=300)
        o = json.loads(r.stdout.strip().splitlines()[-1])
        t1 = o["t_lin"] + (n_cg + 1.5) * o["t_pair"] + o["t_val"]
        one = {"value": n_cg / t1, "cores": o["threads"],
               "sample": (f"EPG on {n_vox_1t} voxels scaled to {prob.nv} "
                          f"({o['t_lin']:.1f} s with tangents, {o['t_val']:.1f} s value-only), "
                          f"one full-size pair ({o['t_pair']:.1f} s)")}
    except Exception as e:   # the one-thread leg is context, never fatal
        one = {"error": str(e)[:200]}
    return {"value": n_cg / t_step, "unit": "pairs/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": (f"FP64 oracle, all five parameters (four trains): EPG with tangents on {S} "
                       f"of {prob.nv} voxels ({t_sample:.2f} s, scaled x{prob.nv / S:.2f}), the "
                       f"value-only EPG on the same sample (scaled: {t_val:.2f} s), {n_pairs} "
                       f"full-size Jv + J^H w pairs ({t_pairs:.2f} s); GN-amortised with n_cg = "
                       f"{n_cg}: t_step = t_lin + (n_cg + 1.5) t_pair + t_value = {t_step:.1f} s"),
            "one_thread": one, "host": _host_cpu()}


def oracle_pair_scaled(prob_small, theta_small, nv_full):
    """The oracle's J v + J^H w pair on a smaller image with the same sequence,
    readout and encoding kind, scaled to the full image by voxel count (its
    direct sums cost T x nk x Nv per product); trains are constants (the cost
    does not depend on their values). Returns (seconds per pair, sample text)."""
    import oracle
    from paper_1904_13244_amd import inputs as I

    oracle.build(force=False)
    npar = I.n_params(prob_small)
    trains = np.full((4, prob_small.n_tr, prob_small.nv), 1e-3 + 1e-3j, dtype=np.complex128)
    v, w = I.probe_vectors(prob_small)
    t0 = time.perf_counter()
    y = oracle.jv(prob_small, theta_small[:npar], trains, v)
    oracle.jhw(prob_small, theta_small[:npar], trains, y)
    t = time.perf_counter() - t0
    scale = nv_full / prob_small.nv
    return t * scale, (f"FP64 oracle, one Jv + J^H w pair on a {prob_small.nx}x{prob_small.ny} image with the "
                       f"same sequence and readout ({t:.2f} s on {oracle.num_threads()} threads), scaled "
                       f"x{scale:.0f} by voxel count")


FP32_MFMA_PEAK_TFLOPS = 157.3    # dense FP32 matrix


def noncartesian(torch, work, reps=5, with_oracle=True):
    """Golden-angle radial sampling of the same workload (one spoke of 448
    samples per TR, 1120 spokes): the voxel x sample contraction on the
    matrix cores (FP32 and split-BF16) for a cached J v + J^H w pair, timed
    per kernel with the library's HIP-event tracing. Algorithmic work per
    product: 8 T nk nx ny flop (complex multiply-adds); split-BF16 issues three
    BF16 products per algorithmic one."""
    import dataclasses

    from paper_1904_13244_amd import binding as B
    from paper_1904_13244_amd import inputs as I
    from paper_1904_13244_amd.binding import Context

    prob = dataclasses.replace(work.problem, traj=I.radial_golden(work.problem.n_tr, work.problem.n_read,
                                                                  work.problem.nx, work.problem.ny))
    dev = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt)  # noqa: E731
    ctx = Context(prob)
    th = dev(work.theta, torch.float32)
    v, w = I.probe_vectors(prob)
    vd, wd = dev(v, torch.float32), dev(w, torch.complex64)
    flop = 8.0 * prob.n_tr * prob.n_read * prob.nx * prob.ny
    out = {"workload": (f"{prob.nx}x{prob.ny}, {prob.n_tr} golden-angle radial spokes of {prob.n_read} "
                        "samples, K=32, FP32 trains"),
           "algorithmic_flop_per_product": flop}
    for name, enc, passes, peak in (("fp32", B.ENC_FP32, 1, FP32_MFMA_PEAK_TFLOPS),
                                    ("split_bf16", B.ENC_SPLIT_BF16, 3, BF16_MFMA_PEAK_TFLOPS)):
        ctx.set_encoding(enc)
        ctx.linearise(th)
        jv = ctx.jv(th, vd, reuse=True)
        g = ctx.jhw(th, wd, reuse=True)
        torch.cuda.synchronize()
        ctx.profile_select(["nc_fwd", "nc_adj", "jhw_finish"])
        ctx.profile(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.jv(th, vd, reuse=True, out=jv)
            ctx.jhw(th, wd, reuse=True, out=g)
        torch.cuda.synchronize()
        pair_ms = 1e3 * (time.perf_counter() - t0) / reps
        prof = ctx.profile_read()
        ctx.profile(False)
        ctx.profile_select(None)
        res = {"pair_ms": pair_ms, "pairs_per_s": 1e3 / pair_ms}
        for k in ("nc_fwd", "nc_adj"):
            n, ms = prof[k]
            t = ms / n * 1e-3
            ach = flop / t / 1e12
            res[k] = {"avg_ms": ms / n, "algorithmic_tflops": ach,
                      "mfma_tflops_issued": passes * ach, "peak_tflops": peak,
                      "frac": passes * ach / peak}
        out[name] = res
    ctx.close()
    if with_oracle:
        small = I.make_problem(32, 32, prob.n_tr, prob.n_read, prob.n_states, flip_deg=prob.flip_deg)
        small = dataclasses.replace(small, traj=I.radial_golden(prob.n_tr, prob.n_read, 32, 32))
        t, sample = oracle_pair_scaled(small, I.iid_maps(small.nv), prob.nv)
        out["cpu_baseline"] = {"value": 1.0 / t, "unit": "pairs/s", "kind": "oracle", "sample": sample}
    return out


def readout_dynamics(torch, work, n_cg, steps=3, with_oracle=True):
    """The benchmark workload with T2 decay and off-resonance during every
    readout (448 samples at 85.6 kHz: 24 power-series and 16 Chebyshev terms
    for T2 >= 5 ms and |Delta B0| <= 200 Hz) and a smooth +-150 Hz
    off-resonance field: GN steps (five parameters with the field as a map;
    six with Delta B0 fitted) and the cached J v + J^H w pair with per-kernel
    times; plain EPG, FP32 trains, split-BF16 contraction. The x-GEMMs carry
    the Chebyshev terms as rows: 8 NC T nx nk algorithmic flop per product."""
    import dataclasses

    from paper_1904_13244_amd import binding as B
    from paper_1904_13244_amd import inputs as I
    from paper_1904_13244_amd.binding import Context

    p0 = work.problem
    yy, xx = np.meshgrid(np.linspace(-1, 1, p0.ny), np.linspace(-1, 1, p0.nx), indexing="ij")
    db0 = (150.0 * (0.6 * xx + 0.3 * yy * yy - 0.1 * xx * yy)).reshape(-1)
    dev = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt)  # noqa: E731
    out = {"workload": ("224x224 phantom, 1120 TRs, 448 samples at 85.6 kHz with T2 decay and "
                        "off-resonance during each readout, K=32, plain EPG, FP32 trains, split-BF16 "
                        "contraction")}
    unit = 1.0 / (2 * np.pi * p0.te)
    for name, prob, theta in (
            ("db0_map", dataclasses.replace(p0, dwell=1 / 85.6e3, db0=db0), work.theta),
            ("db0_fitted", dataclasses.replace(p0, dwell=1 / 85.6e3, db0_unit=unit),
             np.vstack([work.theta, (db0 / unit)[None, :]]))):
        ctx = Context(prob)
        ctx.set_encoding(B.ENC_SPLIT_BF16)
        th_true = dev(theta, torch.float32)
        zeros = torch.zeros(prob.data_shape, dtype=torch.complex64, device="cuda")
        _, r = ctx.residual(th_true, zeros)
        data = (-r).contiguous()
        th0 = theta.copy()
        rng = np.random.default_rng(I.SEED_PROBE)
        th0[0] += 0.05 * rng.standard_normal(prob.nv)
        th0[1] += 0.05 * rng.standard_normal(prob.nv)
        pm = 0b11111 if name == "db0_map" else 0b111111
        th = dev(th0, torch.float32)
        ctx.gn_step(th, data, n_cg, pm, I.GN_LO, I.GN_HI, n_ls_max=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            rep = ctx.gn_step(th, data, n_cg, pm, I.GN_LO, I.GN_HI, n_ls_max=1)
        torch.cuda.synchronize()
        step_ms = 1e3 * (time.perf_counter() - t0) / steps
        v, w = I.probe_vectors(prob)
        vd, wd = dev(v, torch.float32), dev(w, torch.complex64)
        ctx.linearise(th)
        jv = ctx.jv(th, vd, reuse=True)
        g = ctx.jhw(th, wd, reuse=True)
        torch.cuda.synchronize()

        def pairs(n):
            t0 = time.perf_counter()
            for _ in range(n):
                ctx.jv(th, vd, reuse=True, out=jv)
                ctx.jhw(th, wd, reuse=True, out=g)
            torch.cuda.synchronize()
            return 1e3 * (time.perf_counter() - t0) / n

        pair_ms = pairs(10)
        ctx.profile(True)      # per-kernel times from three more pairs, traced
        pairs(3)
        prof = ctx.profile_read()
        ctx.profile(False)
        nq, ncheb = ctx.readout_terms(), ctx.readout_cheb_terms()
        flop = 8.0 * ncheb * prob.n_tr * prob.nx * prob.n_read
        kern = {k: {"launches": n, "avg_ms": ms / n} for k, (n, ms) in prof.items() if n}
        for k in ("xgemm_fwd", "xgemm_adj"):
            if k in kern:
                ach = flop / (kern[k]["avg_ms"] * 1e-3) / 1e12
                kern[k].update({"algorithmic_tflops": ach, "mfma_tflops_issued": 3 * ach,
                                "peak_tflops": BF16_MFMA_PEAK_TFLOPS, "frac": 3 * ach / BF16_MFMA_PEAK_TFLOPS})
        out[name] = {"terms": nq, "cheb_terms": ncheb, "gn_step_ms": step_ms, "pairs_per_s_gn": n_cg * 1e3 / step_ms,
                     "pair_cached_ms": pair_ms, "kernels_per_pair": kern, "param_mask": pm,
                     "gn_report_last": rep.as_dict()}
        ctx.close()
    if with_oracle:
        small = I.make_problem(32, 32, p0.n_tr, p0.n_read, p0.n_states, flip_deg=p0.flip_deg)
        yy, xx = np.meshgrid(np.linspace(-1, 1, 32), np.linspace(-1, 1, 32), indexing="ij")
        small = dataclasses.replace(small, dwell=1 / 85.6e3,
                                    db0=(150.0 * (0.6 * xx + 0.3 * yy * yy - 0.1 * xx * yy)).reshape(-1))
        t, sample = oracle_pair_scaled(small, I.iid_maps(small.nv), p0.nv)
        out["cpu_baseline"] = {"value": 1.0 / t, "unit": "pairs/s", "kind": "oracle", "sample": sample}
    return out


def isochromats(torch, work, n_iso=16, reps=3, with_oracle=True):
    """The paper's balanced isochromat model (16 isochromats over the slice
    profile, RF phases alternating 0 / pi) on the benchmark workload: the
    linearisation (m and its three derivatives for every voxel and TR) on the
    GPU, and the oracle's on a voxel sample scaled to all voxels. Work unit:
    voxel-isochromat-TR updates."""
    import dataclasses

    from paper_1904_13244_amd import inputs as I
    from paper_1904_13244_amd.binding import Context

    prob = dataclasses.replace(work.problem, rf_phase=I.balanced_phases(work.problem.n_tr),
                               iso=I.slice_profile_gaussian(n_iso))
    ctx = Context(prob)
    th = torch.as_tensor(np.ascontiguousarray(work.theta)).to("cuda", torch.float32)
    ctx.linearise(th)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.linearise(th)
    torch.cuda.synchronize()
    t_gpu = (time.perf_counter() - t0) / reps
    ctx.close()
    units = float(prob.nv) * n_iso * prob.n_tr
    out = {"workload": (f"224x224, 1120 TRs, balanced sequence, {n_iso} isochromats per voxel (Gaussian slice "
                        "profile), four trains"),
           "linearise_ms": 1e3 * t_gpu, "voxel_isochromat_trs_per_s": units / t_gpu}
    if with_oracle:
        import oracle
        oracle.build(force=False)
        S = 4096
        sel = np.linspace(0, prob.nv - 1, S).astype(np.int64)
        sub = dataclasses.replace(I.make_problem(S, 1, prob.n_tr, S, prob.n_states, tr=prob.tr, te=prob.te,
                                                 flip_deg=prob.flip_deg, rf_phase=prob.rf_phase), iso=prob.iso)
        t0 = time.perf_counter()
        oracle.epg(sub, work.theta[:, sel])
        t = (time.perf_counter() - t0) * prob.nv / S
        out["cpu_baseline"] = {"value": units / t, "unit": "voxel-isochromat-TRs/s", "kind": "oracle",
                               "sample": (f"FP64 oracle isochromat linearisation of {S} voxels "
                                          f"({t * S / prob.nv:.2f} s on {oracle.num_threads()} threads), scaled to "
                                          f"{prob.nv} voxels: {t:.1f} s")}
    return out


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
                "traffic": measured_traffic(f"{rk}_{'f16' if tb == 2 else 'f32'}_{ntr}tr"),
                "algorithmic_bytes_per_launch": amount}
    ach = amount / t / 1e12
    return {"kernel": rk, "bound": bound, "achieved": ach, "peak": FP32_VALU_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": ach / FP32_VALU_PEAK_TFLOPS, "traffic": None,
            "algorithmic_flop_per_launch": amount}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
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

    def run_form(net, enc, lo, hi, trains, param_mask):
        ntr = 4 if (param_mask >> 2) & 1 else 3
        ctx.set_surrogate(net)
        ctx.set_encoding(enc)
        ctx.set_train_precision(trains)
        theta = dev(th0, torch.float32)

        def step():
            return ctx.gn_step(theta, data, args.n_cg, param_mask, lo, hi, n_ls_max=1)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        # Timed region. The kernels the roofline is taken on are traced (two
        # HIP events per launch, live on the library's stream) during the last
        # timed step only: each recorded event holds the queue for about 4.5 us,
        # which on every step would add some 7 % to the step time.
        ctx.profile_select(TRACED_KINDS)
        t0 = time.perf_counter()
        for i in range(args.steps):
            if i == args.steps - 1:
                ctx.profile(True)
            rep = step()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        prof = ctx.profile_read()
        ctx.profile(False)
        kernels = {k: {"launches": n, "avg_ms": (ms / n if n else 0.0), "ms_per_step": ms}
                   for k, (n, ms) in prof.items() if n}
        # Every kind, from one more (untimed) step with full tracing.
        ctx.profile_select(None)
        ctx.profile(True)
        step()
        full = ctx.profile_read()
        ctx.profile(False)
        breakdown = {k: {"launches": n, "ms": ms} for k, (n, ms) in full.items() if n}
        out = {"value": args.n_cg * args.steps / elapsed, "ms_per_step": 1e3 * elapsed / args.steps,
               "kernels": kernels, "step_breakdown_untimed": breakdown,
               "dominant_kernel": max(breakdown, key=lambda k: breakdown[k]["ms"]),
               "roofline": roofline_for(kernels, prob, 2 if trains == B.TRAINS_FP16 else 4, ntr),
               "gn_report_last": rep.as_dict()}
        if ntr < 4:
            return out
        # Outside the timed loop, all four trains: the cached pair (reuse = 1),
        # the linearisation, and the fresh pair (reuse = 0: J v and J^H w
        # each simulate the trains again, the strict matrix-free practice).
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

        def timed(fn, reps):
            fn()
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps

        ctx.linearise(theta)
        jv_out = torch.empty(prob.data_shape, dtype=torch.complex64, device="cuda")
        g_out = torch.empty((5, prob.nv), dtype=torch.float32, device="cuda")

        def pair(reuse):
            ctx.jv(theta, vd, reuse=reuse, out=jv_out)
            ctx.jhw(theta, wd, reuse=reuse, out=g_out)

        out["pair_cached_ms"] = timed(lambda: pair(True), 20)
        out["pairs_per_s_cached"] = 1e3 / out["pair_cached_ms"]
        out["linearise_ms"] = timed(lambda: ctx.linearise(theta), 5)
        out["pair_fresh_ms"] = timed(lambda: pair(False), 5)
        out["pairs_per_s_fresh"] = 1e3 / out["pair_fresh_ms"]
        if net is not None:
            # Linearisation with a share of voxels outside the network's box:
            # those take the EPG (index-list kernel) after the network.
            fb = {}
            for share in (0.01, 0.1):
                th_out = theta.clone()
                k = int(share * prob.nv)
                idx = torch.from_numpy(np.random.default_rng(9).choice(prob.nv, k, replace=False)).cuda()
                th_out[0, idx] = float(np.log(6.0))        # T1 = 6 s, above the box
                t_ms = timed(lambda: ctx.linearise(th_out), 5)
                fb[f"{share:.0%}"] = {"voxels": ctx.fallback_count(), "linearise_ms": t_ms}
            out["linearise_with_fallback"] = fb
        return out

    masks = {"b1_fitted": 0b11111}
    if not args.no_b1_known:
        masks["b1_known"] = 0b11011
    forms = {}
    if args.form in ("both", "plain"):
        for mname, pm in masks.items():
            forms[("plain_fp32", mname)] = run_form(None, B.ENC_FP32, I.GN_LO, I.GN_HI, B.TRAINS_FP32, pm)
    surr_info = None
    if args.form in ("both", "surrogate"):
        from paper_1904_13244_amd.surrogate import train_surrogate
        from paper_1904_13244_amd.surrogate import RECIPE_EPOCHS, RECIPE_HEAD_WEIGHT, RECIPE_LR
        epochs = args.train_epochs or RECIPE_EPOCHS
        net, trep = train_surrogate(torch, prob, n_samples=args.train_samples, epochs=epochs,
                                    lr=RECIPE_LR, head_weight=RECIPE_HEAD_WEIGHT)
        lo = tuple(max(a, b) for a, b in zip(I.GN_LO, I.SURR_LO))
        hi = tuple(min(a, b) for a, b in zip(I.GN_HI, I.SURR_HI))
        for mname, pm in masks.items():
            forms[("surrogate_split_bf16", mname)] = run_form(net, B.ENC_SPLIT_BF16, lo, hi,
                                                              B.TRAINS_FP16, pm)
        f = forms[("surrogate_split_bf16", "b1_fitted")]
        flop, wbytes = surrogate_work(prob, ntr=4)
        k = f["kernels"].get("surrogate")
        t = k["avg_ms"] * 1e-3 if k else None
        surr_info = {
            "training": {"samples": trep.n_samples, "steps": trep.steps, "batch": net.batch,
                         "epochs": epochs, "lr": RECIPE_LR, "head_weight": list(RECIPE_HEAD_WEIGHT),
                         "seconds_data": trep.seconds_data, "seconds_train": trep.seconds_train,
                         "loss_first": trep.loss_first, "loss_last": trep.loss_last,
                         "heldout_rel_err": dict(zip(["m", "dm_dlnT1", "dm_dlnT2", "dm_dB1"],
                                                     trep.val_rel_err))},
            "inference_roofline": None if t is None else {
                "kernel": "surrogate (hidden-layer + output-layer kernels, 4 trains, FP16 out)",
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

    chosen = "surrogate_split_bf16" if ("surrogate_split_bf16", "b1_fitted") in forms else "plain_fp32"
    c = forms[(chosen, "b1_fitted")]
    form_desc = {"surrogate_split_bf16": ("surrogate trains (BF16 MFMA network, EPG fallback, FP16 "
                                          "storage) + split-BF16 MFMA encoding contraction"),
                 "plain_fp32": "plain FP32 EPG + FP32 MFMA encoding contraction"}
    keep = ("value", "ms_per_step", "roofline", "kernels", "step_breakdown_untimed", "pair_cached_ms",
            "pairs_per_s_cached", "linearise_ms", "pair_fresh_ms", "pairs_per_s_fresh",
            "linearise_with_fallback", "gn_report_last")
    out = {
        "metric": METRIC, "value": c["value"], "unit": "pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": c["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": ("fp32 (BF16 MFMA network, FP16 train storage, split-BF16 contraction)"
                  if chosen.startswith("surrogate") else "fp32"),
        "data": "synthetic",
        "config": {"workload": ("224x224 brain-like phantom, 1120 TRs (224 lines x 5 sweeps), "
                                "448 readout samples, K=32 EPG states, 1 coil; all five parameters "
                                "fitted (T1, T2, B1, complex rho: four trains); one GN step = "
                                "linearise + r + g + 20 CG pairs + 1 line-search trial"),
                   "form": form_desc[chosen], "n_cg": args.n_cg, "parallelism": "single GPU"},
        "roofline": c["roofline"],
    }
    out.update({k: c[k] for k in keep if k in c and k not in ("value", "ms_per_step", "roofline")})
    if chosen != "plain_fp32" and ("plain_fp32", "b1_fitted") in forms:
        p = forms[("plain_fp32", "b1_fitted")]
        out["plain_fp32"] = {k: p[k] for k in keep if k in p}
        out["speedup_vs_plain_fp32"] = c["value"] / p["value"]
    if "b1_known" in masks:
        bk = {"workload": "the same step with B1 known (T1, T2, rho fitted): three trains, no dm/dB1"}
        for form in ("surrogate_split_bf16", "plain_fp32"):
            if (form, "b1_known") in forms:
                f = forms[(form, "b1_known")]
                bk[form] = {k: f[k] for k in ("value", "ms_per_step", "roofline", "step_breakdown_untimed")}
        if "surrogate_split_bf16" in bk and "plain_fp32" in bk:
            bk["speedup_vs_plain_fp32"] = bk["surrogate_split_bf16"]["value"] / bk["plain_fp32"]["value"]
        out["variant_b1_known"] = bk
    if surr_info:
        out["surrogate"] = surr_info
    ctx.close()
    if not args.no_noncartesian:
        out["noncartesian"] = noncartesian(torch, work, with_oracle=not args.no_cpu_baseline)
    if not args.no_readout_dynamics:
        out["readout_dynamics"] = readout_dynamics(torch, work, args.n_cg, with_oracle=not args.no_cpu_baseline)
    if not args.no_isochromats:
        out["isochromats"] = isochromats(torch, work, with_oracle=not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(work, args.n_cg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
