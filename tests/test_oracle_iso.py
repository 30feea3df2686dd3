"""Pins of the oracle's balanced isochromat model (the paper's own signal
model: a balanced transient-state gradient echo, TE = TR/2, RF phase
alternating 0 / 180 degrees, isochromats over the slice profile; Methods,
Pulse Sequence and Reconstructions; Supporting Information S2).

  * Steady state: a constant flip angle with alternating phase drives one
    isochromat to the closed-form bSSFP steady state, |m| = sin a (1 - E1)
    sqrt(E2) / (1 - (E1 - E2) cos a - E1 E2) at TE = TR/2.
  * An independent brute force: rotations as matrix exponentials of the
    axis' cross-product matrix (scipy), decay and regrowth, for general RF
    phases, against the oracle's Rodrigues update.
  * Central finite differences of every tangent.
  * The voxel's trains are the weighted sum over the profile's isochromats.
  * Phases in {0, pi}: the demodulated signal is purely imaginary (the form
    the GPU kernels store).
  * Noiseless GN recovery of the truth under this model on a tiny grid.
"""
import dataclasses

import numpy as np
import pytest
from scipy.linalg import expm

from paper_1904_13244_amd import inputs as I


def _prob(n_tr=48, flips=None, tr=0.008, phases=None, t_inv=0.0, n_iso=None):
    if flips is None:
        flips = I.flips_sin2_sweeps(n_tr, 12)
    if phases is None:
        phases = I.balanced_phases(n_tr)
    p = I.make_problem(4, 3, n_tr, 8, 8, tr=tr, te=tr / 2, t_inv=t_inv, flip_deg=flips, rf_phase=phases)
    if n_iso:
        p = dataclasses.replace(p, iso=I.slice_profile_gaussian(n_iso))
    return p


def test_bssfp_steady_state(oracle_lib):
    T1, T2, tr, a = 0.8, 0.08, 0.005, np.deg2rad(40.0)
    p = _prob(n_tr=4000, flips=np.full(4000, 40.0), tr=tr)
    m = oracle_lib.isochromat(p, np.log(T1), np.log(T2), 1.0)[0]
    E1, E2 = np.exp(-tr / T1), np.exp(-tr / T2)
    ss = np.sin(a) * (1 - E1) * np.sqrt(E2) / (1 - (E1 - E2) * np.cos(a) - E1 * E2)
    assert abs(abs(m[-1]) - ss) <= 1e-12 and abs(abs(m[-2]) - ss) <= 1e-12
    assert np.abs(m.real).max() <= 1e-15


def _brute(p, lnT1, lnT2, B1, scale):
    T1, T2 = np.exp(lnT1), np.exp(lnT2)
    x = np.array([0.0, 0.0, -1.0])

    def relax(x, tau):
        E1, E2 = np.exp(-tau / T1), np.exp(-tau / T2)
        return np.array([E2 * x[0], E2 * x[1], E1 * x[2] + 1 - E1])

    x = relax(x, p.t_inv)
    out = []
    for n in range(p.n_tr):
        k = np.array([np.cos(p.rf_phase[n]), np.sin(p.rf_phase[n]), 0.0])
        K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
        x = expm(K * (B1 * np.deg2rad(p.flip_deg[n]) * scale)) @ x
        x = relax(x, p.te)
        out.append((x[0] + 1j * x[1]) * np.exp(-1j * p.rf_phase[n]))
        x = relax(x, p.tr - p.te)
    return np.array(out)


def test_matches_matrix_exponential_brute_force(oracle_lib):
    rng = np.random.default_rng(5)
    p = _prob(n_tr=40, flips=rng.uniform(5, 80, 40), phases=rng.uniform(0, 2 * np.pi, 40), t_inv=0.02)
    for lnT1, lnT2, B1, sc in ((np.log(0.9), np.log(0.07), 1.1, 0.8), (np.log(2.5), np.log(0.6), 0.85, 1.0)):
        m = oracle_lib.isochromat(p, lnT1, lnT2, B1, sc)[0]
        ref = _brute(p, lnT1, lnT2, B1, sc)
        assert np.abs(m - ref).max() <= 1e-13


def test_tangents_finite_differences(oracle_lib):
    p = _prob(n_tr=60, t_inv=0.01)
    x0 = np.array([np.log(1.1), np.log(0.09), 0.95])
    tr = oracle_lib.isochromat(p, *x0, 0.7)
    for q in range(3):
        h = 1e-6
        xp, xm = x0.copy(), x0.copy()
        xp[q] += h
        xm[q] -= h
        fd = (oracle_lib.isochromat(p, *xp, 0.7)[0] - oracle_lib.isochromat(p, *xm, 0.7)[0]) / (2 * h)
        assert np.linalg.norm(tr[q + 1] - fd) <= 1e-7 * np.linalg.norm(fd), q


def test_voxel_trains_are_the_profile_sum(oracle_lib):
    p = _prob(n_tr=32, n_iso=7)
    th = I.iid_maps(p.nv, seed=3, b1=np.linspace(0.8, 1.2, p.nv))
    tr = oracle_lib.epg(p, th)
    scale, weight = p.iso
    j = 5
    ref = sum(w * oracle_lib.isochromat(p, th[0, j], th[1, j], th[2, j], s) for s, w in zip(scale, weight))
    assert np.abs(tr[:, :, j] - ref).max() <= 1e-14
    assert np.abs(tr.real).max() <= 1e-15                  # phases 0 / pi: imaginary trains


def test_noiseless_recovery_balanced(oracle_lib):
    """From a start 5 % off in ln T1 and ln T2 the GN iteration converges to
    the ground truth under this model (the short balanced sequence is
    ill-conditioned, so CG takes many iterations; from the generic initial
    guess it stops in a local minimum)."""
    p = dataclasses.replace(I.make_problem(4, 4, 96, 8, 8, tr=0.008, te=0.004, rf_phase=I.balanced_phases(96),
                                           flip_deg=I.flips_sin2_sweeps(96, 4)),
                            iso=I.slice_profile_gaussian(6))
    th_true = I.iid_maps(p.nv, seed=11)
    d = oracle_lib.signal(p, th_true, oracle_lib.epg(p, th_true, tangents=False))
    rng = np.random.default_rng(1)
    th = th_true.copy()
    th[:2] += 0.05 * rng.standard_normal((2, p.nv))
    for _ in range(30):
        th, rep = oracle_lib.gn_step(p, th, d, n_cg=100, param_mask=0b11011, lo=I.GN_LO, hi=I.GN_HI)
    err = np.linalg.norm(th - th_true) / np.linalg.norm(th_true)
    assert err <= 1e-6, err
