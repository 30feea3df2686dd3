"""Pins of the oracle's encoding, signal, J v and J^H w.

Independent references:
  * Ex^H Ex = Nk I and Ey^H Ey = Ny I on the centred Cartesian grid;
  * the direct voxel sum equals a centred 2-D FFT (numpy) of the zero-padded
    per-TR image, read at the TR's phase-encode line;
  * the Jacobian column of parameter (q, j) equals minus the central finite
    difference of the signal (Theory: dr/dalpha_i = -d(rho_j m_j)/dalpha_i),
    computed through oracle_epg + oracle_signal_direct only;
  * the adjoint identity Re<Jv, w> = <v, Re(J^H w)>.
"""
import numpy as np
import pytest

from paper_1904_13244_amd import inputs as I


@pytest.mark.parametrize("nx,ny,os", [(8, 6, 2), (7, 5, 1), (16, 16, 2)])
def test_encoding_orthogonality(oracle_lib, nx, ny, os):
    prob = I.make_problem(nx, ny, ny, os * nx, 4)
    # E at the y-centre row is the x-phase; at the x-centre column and the
    # centre readout sample it is the y-phase of the TR's line (line l at TR l).
    Ex = oracle_lib.phases(prob, 0).reshape(prob.n_read, ny, nx)[:, ny // 2, :]
    Ey = np.stack([oracle_lib.phases(prob, n).reshape(prob.n_read, ny, nx)[prob.n_read // 2, :, nx // 2]
                   for n in range(ny)])
    assert np.abs(Ex.conj().T @ Ex - prob.n_read * np.eye(nx)).max() <= 1e-12
    assert np.abs(Ey.conj().T @ Ey - ny * np.eye(ny)).max() <= 1e-12


@pytest.mark.parametrize("nx,ny,os,coils", [(8, 6, 2, 1), (7, 5, 1, 1), (6, 4, 2, 3)])
def test_direct_signal_equals_centred_fft(oracle_lib, nx, ny, os, coils):
    rng = np.random.default_rng(4)
    n_tr = 2 * ny + 1
    prob = I.make_problem(nx, ny, n_tr, os * nx, 4, n_coils=coils,
                          ky_line=rng.integers(0, ny, n_tr))
    nv = prob.nv
    th = I.iid_maps(nv, seed=1)
    trains = rng.standard_normal((4, n_tr, nv)) + 1j * rng.standard_normal((4, n_tr, nv))
    coil = None if coils == 1 else (rng.standard_normal((coils, nv)) + 1j * rng.standard_normal((coils, nv)))
    mask = rng.integers(0, 2, nv).astype(np.uint8)
    s = oracle_lib.signal_direct(prob, th, trains, coil=coil, mask=mask)
    rho = th[3] + 1j * th[4]
    nk = prob.n_read
    for c in range(coils):
        cw = np.ones(nv) if coil is None else coil[c]
        for n in range(n_tr):
            img = (cw * rho * trains[0, n] * mask).reshape(ny, nx)
            pad = np.zeros((ny, nk), dtype=np.complex128)
            pad[:, nk // 2 - nx // 2: nk // 2 - nx // 2 + nx] = img
            ksp = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(pad)))
            ref = ksp[prob.ky_line[n]]
            assert np.abs(s[c, n] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_separable_equals_direct(oracle_lib):
    rng = np.random.default_rng(8)
    prob = I.make_problem(12, 10, 30, 24, 4, n_coils=2)
    th = I.iid_maps(prob.nv, seed=2)
    trains = rng.standard_normal((4, 30, prob.nv)) + 1j * rng.standard_normal((4, 30, prob.nv))
    coil = rng.standard_normal((2, prob.nv)) + 1j * rng.standard_normal((2, prob.nv))
    a = oracle_lib.signal_direct(prob, th, trains, coil=coil)
    b = oracle_lib.signal(prob, th, trains, coil=coil)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def _tiny_problem(coils=1):
    rng = np.random.default_rng(31)
    prob = I.make_problem(4, 3, 12, 8, 8, n_coils=coils, flip_deg=rng.uniform(10, 60, 12),
                          t_inv=0.01)
    th = I.iid_maps(prob.nv, seed=6, b1=rng.uniform(0.85, 1.15, prob.nv))
    coil = None if coils == 1 else I.coil_maps(4, 3, coils)
    return prob, th, coil


@pytest.mark.parametrize("coils", [1, 2])
def test_explicit_jacobian_equals_finite_differences(oracle_lib, coils):
    prob, th, coil = _tiny_problem(coils)
    mask = np.ones(prob.nv, np.uint8)
    mask[5] = 0
    J = oracle_lib.jacobian(prob, th, oracle_lib.epg(prob, th), coil=coil, mask=mask)

    def sig(t):
        return oracle_lib.signal_direct(prob, t, oracle_lib.epg(prob, t, tangents=False),
                                        coil=coil, mask=mask).reshape(-1)

    h = 1e-6
    err = 0.0
    for col in range(5 * prob.nv):
        q, j = divmod(col, prob.nv)
        tp, tm = th.copy(), th.copy()
        tp[q, j] += h
        tm[q, j] -= h
        fd = -(sig(tp) - sig(tm)) / (2 * h)
        err = max(err, np.abs(fd - J[:, col]).max())
    assert err <= 1e-7 * np.abs(J).max(), err
    assert np.abs(J[:, 5::prob.nv]).max() == 0.0  # masked voxel column


@pytest.mark.parametrize("coils", [1, 2])
def test_jv_jhw_match_explicit_jacobian(oracle_lib, coils):
    prob, th, coil = _tiny_problem(coils)
    trains = oracle_lib.epg(prob, th)
    J = oracle_lib.jacobian(prob, th, trains, coil=coil)
    v, w = I.probe_vectors(prob)
    jv = oracle_lib.jv(prob, th, trains, v, coil=coil).reshape(-1)
    jhw = oracle_lib.jhw(prob, th, trains, w, coil=coil).reshape(-1)
    assert np.abs(jv - J @ v.reshape(-1)).max() <= 1e-12 * np.abs(jv).max()
    ref = (J.conj().T @ w.reshape(-1)).real
    assert np.abs(jhw - ref).max() <= 1e-12 * np.abs(ref).max()


def test_adjoint_identity_and_normal_operator(oracle_lib):
    prob = I.make_problem(16, 12, 48, 32, 16, flip_deg=I.flips_sin2_sweeps(48, 12))
    th = I.iid_maps(prob.nv, seed=4, b1=1.05)
    trains = oracle_lib.epg(prob, th)
    v, w = I.probe_vectors(prob)
    lhs = np.vdot(w.reshape(-1), oracle_lib.jv(prob, th, trains, v).reshape(-1)).real
    rhs = float(np.dot(v.reshape(-1), oracle_lib.jhw(prob, th, trains, w).reshape(-1)))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)
    # Re(J^H J) is symmetric positive semi-definite: <u, H v> = <v, H u>, <v, H v> >= 0.
    u = np.random.default_rng(9).standard_normal(v.shape)
    Hv = oracle_lib.jhw(prob, th, trains, oracle_lib.jv(prob, th, trains, v))
    Hu = oracle_lib.jhw(prob, th, trains, oracle_lib.jv(prob, th, trains, u))
    a, b = float(np.sum(u * Hv)), float(np.sum(v * Hu))
    assert abs(a - b) <= 1e-11 * max(abs(a), 1.0)
    assert float(np.sum(v * Hv)) > 0.0
