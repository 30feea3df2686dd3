"""Pins of the oracle's EPG simulation against things the paper and the physics fix.

Independent references (none of them calls the oracle's arithmetic):
  * brute-force isochromat averaging: the Supporting Information S2 update
    (Rodrigues rotation by the RF rotation vector, then decay and regrowth)
    applied to N_iso isochromats dephased by the spoiler; with N_iso >= N_TR
    and K >= N_TR + 1 its mean transverse magnetisation equals untruncated EPG
    exactly (orders alias only modulo N_iso);
  * closed forms: Ernst-type transient, spin echo, inversion recovery;
  * structure: purely imaginary m for RF phases in {0, pi};
  * central finite differences for every tangent.
"""
import numpy as np
import pytest

from paper_1904_13244_amd import inputs as I


def isochromat_mean(prob, T1, T2, B1, n_iso):
    """S2 update with the paper's rotation vector |B1| [-Re RF, Im RF, 0] and
    RF = alpha e^{i phi}; returns the raw (not demodulated) mean Mx + i My at TE."""
    psi = 2 * np.pi * np.arange(n_iso) / n_iso
    M = np.zeros((n_iso, 3))
    M[:, 2] = -1.0  # equilibrium, then ideal inversion

    def relax(M, tau):
        if tau <= 0:
            return M
        E1, E2 = np.exp(-tau / T1), np.exp(-tau / T2)
        M = M.copy()
        M[:, :2] *= E2
        M[:, 2] = E1 * M[:, 2] + (1 - E1)
        return M

    M = relax(M, prob.t_inv)
    out = []
    for n in range(prob.n_tr):
        a = B1 * np.deg2rad(prob.flip_deg[n])
        phi = prob.rf_phase[n]
        av = np.array([-a * np.cos(phi), a * np.sin(phi), 0.0])
        th = np.linalg.norm(av)
        if th > 0:
            k = av / th
            M = (np.cos(th) * M + np.sin(th) * np.cross(k, M)
                 + (1 - np.cos(th)) * (M @ k)[:, None] * k[None, :])
        M = relax(M, prob.te)
        out.append(np.mean(M[:, 0] + 1j * M[:, 1]))
        M = relax(M, prob.tr - prob.te)
        F = (M[:, 0] + 1j * M[:, 1]) * np.exp(1j * psi)
        M[:, 0], M[:, 1] = F.real, F.imag
    return np.array(out)


def _one_voxel(prob, T1, T2, B1, oracle):
    th = I.pack_theta([T1], [T2], [B1], [1.0 + 0j])
    return oracle.epg(prob, th)[:, :, 0]


@pytest.mark.parametrize("phase_kind", ["zero_pi", "general"])
def test_epg_equals_isochromat_average(oracle_lib, phase_kind):
    rng = np.random.default_rng(11)
    ntr = 24
    if phase_kind == "zero_pi":
        ph = np.pi * rng.integers(0, 2, ntr)
    else:
        ph = rng.uniform(0, 2 * np.pi, ntr)
    prob = I.make_problem(1, 1, ntr, 1, ntr + 1, flip_deg=rng.uniform(5, 80, ntr),
                          rf_phase=ph, t_inv=0.013, tr=0.0079, te=0.0031)
    for (T1, T2, B1) in [(0.8, 0.07, 0.9), (2.0, 0.5, 1.2), (0.3, 0.03, 1.0)]:
        m = _one_voxel(prob, T1, T2, B1, oracle_lib)[0]
        ref = isochromat_mean(prob, T1, T2, B1, ntr)
        # The paper's rotation sense mirrors the transverse plane of the EPG
        # operator; the two agree after conjugation (m is demodulated by e^{-i phi}).
        got = np.conj(m * np.exp(1j * ph))
        assert np.abs(got - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())


def test_isochromat_negative_control(oracle_lib):
    """Too few isochromats alias orders: the brute force must then differ."""
    rng = np.random.default_rng(12)
    ntr = 24
    prob = I.make_problem(1, 1, ntr, 1, ntr + 1, flip_deg=rng.uniform(5, 80, ntr))
    m = _one_voxel(prob, 0.8, 0.07, 1.0, oracle_lib)[0]
    ref = isochromat_mean(prob, 0.8, 0.07, 1.0, ntr - 3)
    assert np.abs(np.conj(m) - ref).max() > 1e-4


def test_ernst_transient(oracle_lib):
    """TE = 0, T2 -> 0 (spoiled), constant flip a, inverted start:
    m_n = -i sin a [Mss + (-1 - Mss)(E1 cos a)^n], Mss = (1-E1)/(1-E1 cos a)."""
    ntr, a_deg, T1, TR = 40, 35.0, 0.9, 0.008
    prob = I.make_problem(1, 1, ntr, 1, 8, flip_deg=np.full(ntr, a_deg), tr=TR, te=0.0)
    m = _one_voxel(prob, T1, 1e-9, 1.0, oracle_lib)[0]
    a = np.deg2rad(a_deg)
    E1 = np.exp(-TR / T1)
    Mss = (1 - E1) / (1 - E1 * np.cos(a))
    n = np.arange(ntr)
    ref = -1j * np.sin(a) * (Mss + (-1 - Mss) * (E1 * np.cos(a)) ** n)
    assert np.abs(m - ref).max() <= 1e-14


def test_spin_echo(oracle_lib):
    """Flips (a, 180, 0): m_1 = 0 and m_2 = conj(m_0 at TE=0) exp(-(2TR+TE)/T2)."""
    a_deg, T1, T2, TR, TE = 50.0, 1.1, 0.09, 0.008, 0.003
    flips = np.array([a_deg, 180.0, 0.0])
    prob = I.make_problem(1, 1, 3, 1, 8, flip_deg=flips, tr=TR, te=TE, t_inv=60.0)
    m = _one_voxel(prob, T1, T2, 1.0, oracle_lib)[0]
    prob0 = I.make_problem(1, 1, 3, 1, 8, flip_deg=flips, tr=TR, te=0.0, t_inv=60.0)
    m0 = _one_voxel(prob0, T1, T2, 1.0, oracle_lib)[0]
    assert abs(m[1]) <= 1e-15
    assert abs(m[2] - np.conj(m0[0]) * np.exp(-(2 * TR + TE) / T2)) <= 1e-14


def test_inversion_recovery(oracle_lib):
    """Zero flips then one 90 degree pulse: m_N = -i (1 - 2 e^{-t/T1}) e^{-TE/T2},
    t = t_inv + N TR; all earlier samples are zero."""
    N, T1, T2, TR, TE, tinv = 17, 0.7, 0.08, 0.008, 0.002, 0.05
    flips = np.zeros(N + 1)
    flips[-1] = 90.0
    prob = I.make_problem(1, 1, N + 1, 1, 8, flip_deg=flips, tr=TR, te=TE, t_inv=tinv)
    m = _one_voxel(prob, T1, T2, 1.0, oracle_lib)[0]
    assert np.abs(m[:N]).max() == 0.0
    ref = -1j * (1 - 2 * np.exp(-(tinv + N * TR) / T1)) * np.exp(-TE / T2)
    assert abs(m[N] - ref) <= 1e-14


def test_real_imaginary_invariant(oracle_lib):
    """RF phases in {0, pi} keep every recorded train purely imaginary (exactly
    for phase 0; to the rounding of e^{i pi} in FP64 otherwise)."""
    rng = np.random.default_rng(5)
    ntr = 64
    prob = I.make_problem(4, 2, ntr, 4, 16, flip_deg=rng.uniform(0, 90, ntr),
                          rf_phase=np.pi * rng.integers(0, 2, ntr), t_inv=0.01)
    th = I.iid_maps(prob.nv, seed=3, b1=rng.uniform(0.7, 1.3, prob.nv))
    tr = oracle_lib.epg(prob, th)
    assert np.abs(tr.real).max() <= 1e-14 * np.abs(tr.imag).max()
    assert np.abs(tr.imag).max() > 0.1
    prob0 = I.make_problem(4, 2, ntr, 4, 16, flip_deg=prob.flip_deg, t_inv=0.01)
    assert np.abs(oracle_lib.epg(prob0, th).real).max() == 0.0


@pytest.mark.parametrize("q", [0, 1, 2])
def test_tangents_match_central_differences(oracle_lib, q):
    rng = np.random.default_rng(21 + q)
    ntr = 96
    prob = I.make_problem(3, 2, ntr, 3, 16, flip_deg=rng.uniform(0, 70, ntr), t_inv=0.02)
    th = I.iid_maps(prob.nv, seed=9, b1=rng.uniform(0.8, 1.2, prob.nv))
    tr = oracle_lib.epg(prob, th)
    h = 1e-5
    tp, tm = th.copy(), th.copy()
    tp[q] += h
    tm[q] -= h
    fd = (oracle_lib.epg(prob, tp, tangents=False)[0] -
          oracle_lib.epg(prob, tm, tangents=False)[0]) / (2 * h)
    ad = tr[q + 1]
    err = np.linalg.norm(fd - ad) / np.linalg.norm(ad)
    assert err <= 1e-7, err


def test_truncation_converges(oracle_lib):
    """Raising K towards N_TR + 1 converges to the untruncated result."""
    rng = np.random.default_rng(2)
    ntr = 48
    prob_full = I.make_problem(1, 1, ntr, 1, ntr + 1, flip_deg=rng.uniform(10, 70, ntr))
    ref = _one_voxel(prob_full, 1.0, 0.2, 1.0, oracle_lib)[0]
    errs = []
    for K in (4, 8, 16, 32):
        prob = I.make_problem(1, 1, ntr, 1, K, flip_deg=prob_full.flip_deg)
        errs.append(np.abs(_one_voxel(prob, 1.0, 0.2, 1.0, oracle_lib)[0] - ref).max())
    assert errs[-1] < errs[0]
    assert errs[-1] < 1e-3
