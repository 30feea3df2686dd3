"""Writes config2_gn_oracle.npz: the FP64 oracle's reconstruction of the
128 x 128, 1024-TR workload (Nk 256, K 32, SNR 50), the reference the GPU's
plain FP32 path is compared against.

Recipe (Methods, Numerical Brain Simulation and Reconstructions; every value
from oracle/ and the seeded input generators, nothing from the HIP path):
  * data d = s(theta_true) + n, s by the oracle's EPG and encoding, n the
    seeded unit noise scaled so that ||s|| / ||n|| = 50;
  * start: T1 = 1 s, T2 = 0.1 s, B1 = the phantom's (known), rho by 20
    iterations of the oracle's CGLS on the head mask, then rounded to FP32 so
    that both sides start from the same representable point;
  * 10 inexact Gauss-Newton iterations of 20 CG steps (T1, T2, rho fitted,
    head mask, the standard box and line search).
Stored: the FP32 start, the final maps (float64), each iteration's report,
and ||d||^2 (the test regenerates d and checks it against this).

    python tests/golden/make_config2_gn.py      (about 5 minutes on 8 cores)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1904_13244_amd import inputs as I  # noqa: E402

OUT = os.path.join(HERE, "config2_gn_oracle.npz")


def data(w):
    prob = w.problem
    s = oracle.signal(prob, w.theta, oracle.epg(prob, w.theta, tangents=False))
    n = I.unit_noise(prob)
    return s + n * (np.linalg.norm(s) / (w.snr * np.linalg.norm(n)))


def main():
    oracle.build(force=False)
    w = I.config(2)
    prob, head = w.problem, w.extra["head"].astype(np.uint8)
    t0 = time.perf_counter()
    d = data(w)
    th = I.initial_theta(prob.nv)
    th[2] = w.theta[2]
    th = oracle.rho_init(prob, th, d, n_iter=20, mask=head)
    th0 = th.astype(np.float32)
    th = th0.astype(np.float64)
    reps = []
    for it in range(w.n_gn):
        th, rep = oracle.gn_step(prob, th, d, n_cg=w.n_cg, param_mask=w.param_mask,
                                 lo=I.GN_LO, hi=I.GN_HI, mask=head)
        reps.append([rep.f0, rep.f1, rep.t, rep.cg_iters, rep.accepted, rep.ls_trials])
        print(f"it {it}: f0 {rep.f0:.6e} f1 {rep.f1:.6e} t {rep.t} cg {rep.cg_iters} "
              f"({time.perf_counter() - t0:.0f} s)", flush=True)
    np.savez_compressed(OUT, theta0=th0, theta=th, reports=np.array(reps),
                        d_norm2=np.vdot(d, d).real, n_gn=w.n_gn, n_cg=w.n_cg,
                        param_mask=w.param_mask)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
