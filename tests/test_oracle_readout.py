"""Pins of the oracle's readout dynamics (Discussion: the volumetric model
follows T2 decay and Delta B0 phase accumulation during each readout):
sample k of a readout is taken at TE + tau_k, tau_k = (k - n_read/2) dwell,
and voxel j's magnetisation carries exp(-tau_k / T2_j) exp(-2 pi i db0_j
(TE + tau_k)) (the precession in the sense of the encoding phase).

  * Off-resonance in the gradient-spoiled model: an isochromat brute force
    (the Supporting Information S2 update with the rotation vector's z part
    2 pi db0 dt, N_iso spoiler dephasings) gives the EPG echo times
    exp(-2 pi i db0 TE) for any db0: the spoiler's dephasing absorbs the
    precession between pulses, so the readout factor is all off-resonance
    changes.
  * A uniform T2 and off-resonance over the image: every sample of the
    signal is the static signal (pinned by the FFT in
    tests/test_oracle_encoding.py) times exp(lambda tau_k) exp(-2 pi i db0 TE),
    lambda = -1/T2 - 2 pi i db0, independently of the direct sum.
  * dwell = 0 with a zero off-resonance map: the direct sum with the factor
    equals the separable evaluation.
  * Central finite differences of the residual for columns of the explicit
    Jacobian (the ln T2 column carries the readout decay's tau_k term), the
    products J v and Re(J^H w) against the explicit Jacobian, the adjoint
    identity, and noiseless recovery by the GN iteration.
  * Delta B0 as a sixth parameter (theta row 5 times db0_unit Hz): the row in
    place of the map gives the map's signal and first five Jacobian rows; its
    column against finite differences and against the closed form
    -2 pi i db0_unit (TE + tau_k) times the voxel's samples; products against
    the explicit six-parameter Jacobian; the +-rd_max_db0 box in the line
    search; noiseless recovery with Delta B0 fitted.
"""
import dataclasses

import numpy as np
import pytest

from paper_1904_13244_amd import inputs as I

DWELL = 1.0 / 85.6e3   # the paper's in-vivo readout bandwidth (85.6 kHz)


def _case(seed=11, nx=6, ny=5, n_tr=24, n_read=12, coils=1, dwell=DWELL, db0_hz=80.0):
    rng = np.random.default_rng(seed)
    prob = I.make_problem(nx, ny, n_tr, n_read, 8, n_coils=coils, tr=0.008, te=0.004,
                          flip_deg=I.flips_sin2_sweeps(n_tr, ny, seed=seed),
                          ky_line=rng.integers(0, ny, n_tr))
    db0 = rng.uniform(-db0_hz, db0_hz, prob.nv)
    prob = dataclasses.replace(prob, dwell=dwell, db0=db0)
    th = I.iid_maps(prob.nv, seed=seed, b1=rng.uniform(0.8, 1.2, prob.nv))
    th[1] = np.log(rng.uniform(0.01, 0.15, prob.nv))   # short T2: visible decay over a readout
    coil = I.coil_maps(nx, ny, coils) if coils > 1 else None
    return prob, th, coil, rng


def _spoiled_isochromats(prob, T1, T2, B1, f, n_iso):
    """S2 update per isochromat with rotation vector [-a cos phi, a sin phi, 0]
    for the pulse and precession 2 pi f t about z in between; spoiler
    dephasing psi_q = 2 pi q / n_iso after each readout. Mean Mx + i My at TE."""
    psi = 2 * np.pi * np.arange(n_iso) / n_iso
    M = np.zeros((n_iso, 3))
    M[:, 2] = -1.0

    def free(M, t, extra=0.0):
        if t <= 0 and extra == 0.0:
            return M
        E1, E2 = np.exp(-t / T1), np.exp(-t / T2)
        F = (M[:, 0] + 1j * M[:, 1]) * E2 * np.exp(1j * (2 * np.pi * f * t + extra))
        out = M.copy()
        out[:, 0], out[:, 1] = F.real, F.imag
        out[:, 2] = E1 * M[:, 2] + (1 - E1)
        return out

    M = free(M, prob.t_inv)
    res = []
    for n in range(prob.n_tr):
        a = B1 * np.deg2rad(prob.flip_deg[n])
        ph = prob.rf_phase[n]
        av = np.array([-a * np.cos(ph), a * np.sin(ph), 0.0])
        th = np.linalg.norm(av)
        k = av / th
        M = np.cos(th) * M + np.sin(th) * np.cross(k, M) + (1 - np.cos(th)) * (M @ k)[:, None] * k[None, :]
        M = free(M, prob.te)
        res.append(np.mean(M[:, 0] + 1j * M[:, 1]))
        M = free(M, prob.tr - prob.te, extra=psi)
    return np.array(res)


@pytest.mark.parametrize("f", [0.0, 37.0, -140.0])
def test_spoiled_offresonance_is_an_echo_phase(oracle_lib, f):
    n_tr = 30
    ph = np.pi * (np.arange(n_tr) % 2)
    prob = I.make_problem(1, 1, n_tr, 4, n_tr + 2, tr=0.008, te=0.004, t_inv=0.01,
                          flip_deg=np.linspace(10, 70, n_tr), rf_phase=ph)
    T1, T2, B1 = 0.9, 0.08, 1.1
    th = I.pack_theta([T1], [T2], [B1], [1.0 + 0j])
    m0 = oracle_lib.epg(prob, th, tangents=False)[0, :, 0]
    brute = _spoiled_isochromats(prob, T1, T2, B1, f, n_tr + 1)
    # The S2 rotation sense is the mirror image of the EPG operator's: the two
    # agree after conjugation, with the demodulation by the RF phase (as in the
    # EPG pin). The echo with off-resonance is the echo without it times the
    # readout factor at tau = 0.
    got = np.conj(brute) * np.exp(-1j * ph)
    ref = m0 * np.exp(-2j * np.pi * f * prob.te)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_uniform_relaxation_and_offresonance_closed_form(oracle_lib):
    prob, th, coil, rng = _case(seed=12, coils=3)
    T2, f = 0.03, 55.0
    th[1] = np.log(T2)
    uni = dataclasses.replace(prob, db0=np.full(prob.nv, f))
    static = dataclasses.replace(prob, dwell=0.0, db0=None)
    mask = (rng.uniform(size=prob.nv) > 0.2).astype(np.uint8)
    tr = oracle_lib.epg(prob, th, tangents=False)
    s_dyn = oracle_lib.signal(uni, th, tr, coil=coil, mask=mask)
    s_0 = oracle_lib.signal(static, th, tr, coil=coil, mask=mask)
    tau = (np.arange(prob.n_read) - prob.n_read // 2) * prob.dwell
    lam = -1.0 / T2 - 2j * np.pi * f
    ref = s_0 * (np.exp(lam * tau) * np.exp(-2j * np.pi * f * prob.te))[None, None, :]
    assert np.linalg.norm(s_dyn - ref) <= 1e-12 * np.linalg.norm(ref)


def test_zero_dwell_and_offresonance_equal_the_static_model(oracle_lib):
    prob, th, coil, rng = _case(seed=13, coils=2)
    zero = dataclasses.replace(prob, dwell=0.0, db0=np.zeros(prob.nv))
    static = dataclasses.replace(prob, dwell=0.0, db0=None)
    tr = oracle_lib.epg(prob, th)
    v, w = I.probe_vectors(prob)
    for fn, args in ((oracle_lib.signal, ()), (oracle_lib.jv, (v,)), (oracle_lib.jhw, (w,))):
        a = fn(zero, th, tr, *args, coil=coil)
        b = fn(static, th, tr, *args, coil=coil)
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b), fn.__name__


def test_jacobian_finite_differences(oracle_lib):
    prob, th, coil, rng = _case(seed=14, coils=2)
    tr = oracle_lib.epg(prob, th)
    J = oracle_lib.jacobian(prob, th, tr, coil=coil)
    d = np.zeros(prob.data_shape, dtype=np.complex128)
    cols = [prob.nv + j for j in rng.choice(prob.nv, 5, replace=False)]   # ln T2: the readout term
    cols += [int(c) for c in rng.choice(5 * prob.nv, 8, replace=False)]
    for col in cols:
        q, j = divmod(int(col), prob.nv)
        h = 1e-6 * max(1.0, abs(th[q, j]))
        tp, tm = th.copy(), th.copy()
        tp[q, j] += h
        tm[q, j] -= h
        rp = oracle_lib.residual(prob, tp, d, coil=coil)[1]
        rm = oracle_lib.residual(prob, tm, d, coil=coil)[1]
        fd = ((rp - rm) / (2 * h)).reshape(-1)
        assert np.linalg.norm(J[:, col] - fd) <= 1e-7 * max(np.linalg.norm(fd), 1e-12), (q, j)


def test_products_match_explicit_jacobian_and_adjoint(oracle_lib):
    prob, th, coil, rng = _case(seed=15, coils=2)
    mask = (rng.uniform(size=prob.nv) > 0.2).astype(np.uint8)
    tr = oracle_lib.epg(prob, th)
    J = oracle_lib.jacobian(prob, th, tr, coil=coil, mask=mask)
    v, w = I.probe_vectors(prob)
    jv = oracle_lib.jv(prob, th, tr, v, coil=coil, mask=mask).reshape(-1)
    jhw = oracle_lib.jhw(prob, th, tr, w, coil=coil, mask=mask).reshape(-1)
    assert np.linalg.norm(jv - J @ v.reshape(-1)) <= 1e-12 * np.linalg.norm(jv)
    ref = (J.conj().T @ w.reshape(-1)).real
    assert np.linalg.norm(jhw - ref) <= 1e-12 * np.linalg.norm(ref)
    lhs = np.vdot(w.reshape(-1), jv).real
    assert abs(lhs - float(v.reshape(-1) @ jhw)) <= 1e-12 * abs(lhs)


def test_noiseless_recovery_with_readout_dynamics(oracle_lib):
    prob, th_true, _, _ = _case(seed=16, nx=6, ny=6, n_tr=48, n_read=12)
    d = oracle_lib.signal(prob, th_true, oracle_lib.epg(prob, th_true, tangents=False))
    th = th_true.copy()
    rng = np.random.default_rng(17)
    th[:2] += 0.05 * rng.standard_normal((2, prob.nv))
    th = oracle_lib.rho_init(prob, th, d, n_iter=20)
    for _ in range(20):
        th, rep = oracle_lib.gn_step(prob, th, d, n_cg=40, param_mask=0b11011, lo=I.GN_LO, hi=I.GN_HI)
    err = np.linalg.norm(th - th_true) / np.linalg.norm(th_true)
    assert err <= 1e-6, err


# --------------------------------------------------------------------------
# Delta B0 as a reconstructed sixth parameter (db0_unit > 0): theta row 5
# times db0_unit is the voxel's off-resonance in Hz.

def _fitted(seed=21, nx=6, ny=5, n_tr=24, n_read=12, coils=1):
    prob, th, coil, rng = _case(seed=seed, nx=nx, ny=ny, n_tr=n_tr, n_read=n_read, coils=coils)
    unit = 1.0 / (2 * np.pi * prob.te)     # theta_5 = the off-resonance phase at TE in radians
    fit = dataclasses.replace(prob, db0=None, db0_unit=unit, rd_max_db0=200.0)
    th6 = np.vstack([th, (prob.db0 / unit)[None, :]])
    return prob, fit, th, th6, coil, rng


def test_fitted_row_equals_the_map(oracle_lib):
    """The sixth row in place of the map gives the same signal, and the
    first five rows of J v, Re(J^H w) and J are those of the map's model."""
    prob, fit, th, th6, coil, rng = _fitted(coils=2)
    tr = oracle_lib.epg(prob, th)
    a = oracle_lib.signal(prob, th, tr, coil=coil)
    b = oracle_lib.signal(fit, th6, tr, coil=coil)
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(a)
    v, w = I.probe_vectors(fit)
    v[5] = 0.0
    assert np.allclose(oracle_lib.jv(fit, th6, tr, v, coil=coil), oracle_lib.jv(prob, th, tr, v[:5], coil=coil),
                       rtol=0, atol=1e-12 * np.abs(a).max())
    g6 = oracle_lib.jhw(fit, th6, tr, w, coil=coil)
    g5 = oracle_lib.jhw(prob, th, tr, w, coil=coil)
    assert np.linalg.norm(g6[:5] - g5) <= 1e-12 * np.linalg.norm(g5)


def test_offresonance_column_finite_differences(oracle_lib):
    prob, fit, th, th6, coil, rng = _fitted(seed=22, coils=2)
    tr = oracle_lib.epg(fit, th6)
    J = oracle_lib.jacobian(fit, th6, tr, coil=coil)
    assert J.shape[1] == 6 * fit.nv
    d = np.zeros(fit.data_shape, dtype=np.complex128)
    for j in rng.choice(fit.nv, 6, replace=False):
        col = 5 * fit.nv + int(j)
        h = 1e-6
        tp, tm = th6.copy(), th6.copy()
        tp[5, j] += h
        tm[5, j] -= h
        fd = ((oracle_lib.residual(fit, tp, d, coil=coil)[1] - oracle_lib.residual(fit, tm, d, coil=coil)[1])
              / (2 * h)).reshape(-1)
        assert np.linalg.norm(J[:, col] - fd) <= 1e-7 * np.linalg.norm(fd), j


def test_offresonance_column_closed_form(oracle_lib):
    """d/dtheta_5 of voxel j's samples is -2 pi i db0_unit (TE + tau_k) times
    them, and voxel j's samples are -rho_j times its Re rho column."""
    prob, fit, th, th6, coil, rng = _fitted(seed=23)
    tr = oracle_lib.epg(fit, th6)
    J = oracle_lib.jacobian(fit, th6, tr)
    tau = (np.arange(fit.n_read) - fit.n_read // 2) * fit.dwell
    fac = np.tile(-2j * np.pi * fit.db0_unit * (fit.te + tau), fit.n_tr)
    for j in range(0, fit.nv, 7):
        rho = th6[3, j] + 1j * th6[4, j]
        samples = -rho * J[:, 3 * fit.nv + j]
        ref = -fac * samples
        assert np.linalg.norm(J[:, 5 * fit.nv + j] - ref) <= 1e-13 * np.linalg.norm(ref)


def test_six_parameter_products_and_adjoint(oracle_lib):
    prob, fit, th, th6, coil, rng = _fitted(seed=24, coils=2)
    mask = (rng.uniform(size=fit.nv) > 0.2).astype(np.uint8)
    tr = oracle_lib.epg(fit, th6)
    J = oracle_lib.jacobian(fit, th6, tr, coil=coil, mask=mask)
    v, w = I.probe_vectors(fit)
    jv = oracle_lib.jv(fit, th6, tr, v, coil=coil, mask=mask).reshape(-1)
    jhw = oracle_lib.jhw(fit, th6, tr, w, coil=coil, mask=mask).reshape(-1)
    assert np.linalg.norm(jv - J @ v.reshape(-1)) <= 1e-12 * np.linalg.norm(jv)
    ref = (J.conj().T @ w.reshape(-1)).real
    assert np.linalg.norm(jhw - ref) <= 1e-12 * np.linalg.norm(ref)


def test_offresonance_box_in_the_line_search(oracle_lib):
    """A GN step in theta_5 alone whose step leaves +-rd_max_db0 Hz is
    projected onto the box; the other rows do not move."""
    prob, fit, th, th6, coil, rng = _fitted(seed=25)
    tight = dataclasses.replace(fit, rd_max_db0=30.0)
    th_true = th6.copy()
    th_true[5] = np.clip(th_true[5], -50.0 / fit.db0_unit, 50.0 / fit.db0_unit)   # partly beyond the box
    d = oracle_lib.signal(tight, th_true, oracle_lib.epg(tight, th_true, tangents=False))
    start = th_true.copy()
    start[5] = 0.0
    th1, rep = oracle_lib.gn_step(tight, start, d, n_cg=20, param_mask=0b100000, lo=I.GN_LO, hi=I.GN_HI)
    assert rep.accepted
    hz = np.abs(th1[5]) * fit.db0_unit
    assert np.all(hz <= 30.0 + 1e-9) and np.sum(np.abs(hz - 30.0) <= 1e-9) > 0
    assert np.array_equal(th1[:5], start[:5])


def test_noiseless_recovery_with_offresonance_fitted(oracle_lib):
    """With one echo time the off-resonance phase at TE is shared with rho's
    phase: Delta B0 is told apart only by its phase ramp across the readout
    (a shift of db0 / (pixel bandwidth) along x). On this 6-pixel grid that
    needs a long readout (12 samples of 0.2 ms) and CG run to the number of
    unknowns (200 >= 5 x 36); then GN converges quadratically to the truth."""
    prob, fit, th, th6, coil, rng = _fitted(seed=26, nx=6, ny=6, n_tr=48, n_read=12)
    fit = dataclasses.replace(fit, dwell=2e-4)
    d = oracle_lib.signal(fit, th6, oracle_lib.epg(fit, th6, tangents=False))
    x = th6.copy()
    r2 = np.random.default_rng(27)
    x[:2] += 0.05 * r2.standard_normal((2, fit.nv))
    x[5] += 0.3 * r2.standard_normal(fit.nv)     # about 12 Hz at TE = 4 ms
    errs = []
    for _ in range(12):
        x, rep = oracle_lib.gn_step(fit, x, d, n_cg=200, param_mask=0b111011, lo=I.GN_LO, hi=I.GN_HI)
        errs.append(np.linalg.norm(x - th6) / np.linalg.norm(th6))
    assert errs[-1] <= 1e-6, errs
    assert errs[6] <= 1e-3 * errs[1]   # superlinear
