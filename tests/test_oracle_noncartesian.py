"""Pins of the oracle's non-Cartesian encoding (any k-space trajectory, sums
taken directly over the voxels; the method's non-Cartesian extensibility,
Introduction and Discussion).

  * A trajectory that lists the Cartesian samples gives the Cartesian results
    (signal, J v, Re(J^H w), explicit J), which are pinned by the centred FFT
    of the image in tests/test_oracle_encoding.py.
  * Shift theorem: shifting every sample by a constant (dx, dy) cycles per
    field of view equals multiplying the image by
    exp(-2 pi i (dx (ix - nx/2) / nx + dy (iy - ny/2) / ny)) on the unshifted
    grid, so off-grid evaluation is pinned by on-grid evaluation.
  * On a golden-angle radial problem: the adjoint identity, central finite
    differences of the signal for Jacobian columns, and noiseless recovery of
    the ground truth by the GN iteration.
"""
import dataclasses

import numpy as np
import pytest

from paper_1904_13244_amd import inputs as I


def _case(seed=3, nx=6, ny=5, n_tr=20, n_read=12, coils=1):
    rng = np.random.default_rng(seed)
    prob = I.make_problem(nx, ny, n_tr, n_read, 8, n_coils=coils,
                          flip_deg=I.flips_sin2_sweeps(n_tr, ny, seed=seed),
                          ky_line=rng.integers(0, ny, n_tr))
    th = I.iid_maps(prob.nv, seed=seed, b1=rng.uniform(0.8, 1.2, prob.nv))
    coil = I.coil_maps(nx, ny, coils) if coils > 1 else None
    return prob, th, coil, rng


def test_cartesian_trajectory_equals_cartesian(oracle_lib):
    prob, th, coil, rng = _case(coils=3)
    cprob = dataclasses.replace(prob, traj=I.cartesian_traj(prob))
    mask = (rng.uniform(size=prob.nv) > 0.2).astype(np.uint8)
    tr = oracle_lib.epg(prob, th)
    v, w = I.probe_vectors(prob)
    for f, args in ((oracle_lib.signal, ()), (oracle_lib.jv, (v,)), (oracle_lib.jhw, (w,))):
        a = f(prob, th, tr, *args, coil=coil, mask=mask)
        b = f(cprob, th, tr, *args, coil=coil, mask=mask)
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(a), f.__name__
    Ja = oracle_lib.jacobian(prob, th, tr, coil=coil, mask=mask)
    Jb = oracle_lib.jacobian(cprob, th, tr, coil=coil, mask=mask)
    assert np.linalg.norm(Ja - Jb) <= 1e-12 * np.linalg.norm(Ja)


@pytest.mark.parametrize("dx,dy", [(0.37, -0.21), (-1.6, 2.45)])
def test_shift_theorem_off_grid(oracle_lib, dx, dy):
    prob, th, _, _ = _case(seed=5)
    kx, ky = I.cartesian_traj(prob)
    grid = dataclasses.replace(prob, traj=(kx, ky))
    shifted = dataclasses.replace(prob, traj=(kx + dx, ky + dy))
    tr = oracle_lib.epg(prob, th, tangents=False)
    j = np.arange(prob.nv)
    x, y = j % prob.nx - prob.nx // 2, j // prob.nx - prob.ny // 2
    mod = np.exp(-2j * np.pi * (dx * x / prob.nx + dy * y / prob.ny))
    rho = (th[3] + 1j * th[4]) * mod
    th_mod = th.copy()
    th_mod[3], th_mod[4] = rho.real, rho.imag
    a = oracle_lib.signal(shifted, th, tr)
    b = oracle_lib.signal(grid, th_mod, tr)
    assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)


def _radial(seed=7, nx=6, ny=6, n_tr=24, n_read=12):
    prob, th, _, rng = _case(seed=seed, nx=nx, ny=ny, n_tr=n_tr, n_read=n_read)
    return dataclasses.replace(prob, traj=I.radial_golden(n_tr, n_read, nx, ny)), th, rng


def test_radial_adjoint_identity(oracle_lib):
    prob, th, rng = _radial()
    tr = oracle_lib.epg(prob, th)
    v, w = I.probe_vectors(prob)
    lhs = np.vdot(w, oracle_lib.jv(prob, th, tr, v)).real
    rhs = float(v.reshape(-1) @ oracle_lib.jhw(prob, th, tr, w).reshape(-1))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_radial_jacobian_finite_differences(oracle_lib):
    prob, th, rng = _radial(seed=8)
    tr = oracle_lib.epg(prob, th)
    J = oracle_lib.jacobian(prob, th, tr)
    d = np.zeros(prob.data_shape, dtype=np.complex128)
    for col in rng.choice(5 * prob.nv, 8, replace=False):
        q, j = divmod(int(col), prob.nv)
        h = 1e-6 * max(1.0, abs(th[q, j]))
        tp, tm = th.copy(), th.copy()
        tp[q, j] += h
        tm[q, j] -= h
        rp = oracle_lib.residual(prob, tp, d)[1]
        rm = oracle_lib.residual(prob, tm, d)[1]
        fd = ((rp - rm) / (2 * h)).reshape(-1)
        assert np.linalg.norm(J[:, col] - fd) <= 1e-7 * max(np.linalg.norm(fd), 1e-12), (q, j)


def test_radial_noiseless_recovery(oracle_lib):
    prob, th_true, _ = _radial(seed=9, nx=6, ny=6, n_tr=64, n_read=12)
    d = oracle_lib.signal(prob, th_true, oracle_lib.epg(prob, th_true, tangents=False))
    th = oracle_lib.rho_init(prob, I.initial_theta(prob.nv), d, n_iter=20)
    th[2] = th_true[2]
    for _ in range(25):
        th, rep = oracle_lib.gn_step(prob, th, d, n_cg=40, param_mask=0b11011, lo=I.GN_LO, hi=I.GN_HI)
    err = np.linalg.norm(th - th_true) / np.linalg.norm(th_true)
    assert err <= 1e-6, err
