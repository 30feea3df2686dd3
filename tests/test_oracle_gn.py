"""Pins of the oracle's Gauss-Newton step and proton-density initialisation.

Independent references:
  * after k CG iterations from zero, the step is the Galerkin solution of
    Re(J^H J) p = -g on the Krylov space span{g, Hg, ..., H^{k-1}g}
    (numpy, from the explicit Jacobian, itself pinned by finite differences);
  * noiseless data: the iteration recovers the ground-truth maps from the
    paper's initial guess (T1 = 1 s, T2 = 0.1 s, B1 = 1, rho by least squares);
  * noisy data: 2f at convergence matches the noise level, ||n||^2 (1 - N/(2 M))
    for N real unknowns and M complex samples (the expected residual of a
    least-squares fit);
  * the rho initialisation equals numpy's least-squares solution.
"""
import numpy as np
import pytest

from paper_1904_13244_amd import inputs as I


def _tiny(seed=3):
    rng = np.random.default_rng(seed)
    prob = I.make_problem(4, 3, 24, 8, 8, flip_deg=I.flips_sin2_sweeps(24, 3, seed=seed),
                          t_inv=0.01)
    th_true = I.iid_maps(prob.nv, seed=seed)
    th0 = th_true.copy()
    th0[:2] += 0.02 * rng.standard_normal((2, prob.nv))
    th0[3:] += 0.02 * rng.standard_normal((2, prob.nv))
    return prob, th_true, th0


@pytest.mark.parametrize("k", [1, 3, 5])
def test_cg_step_is_krylov_galerkin_solution(oracle_lib, k):
    prob, th_true, th0 = _tiny()
    d = oracle_lib.signal(prob, th_true, oracle_lib.epg(prob, th_true, tangents=False))
    pmask = 0b11011
    th1, rep = oracle_lib.gn_step(prob, th0, d, n_cg=k, param_mask=pmask,
                                  lo=I.GN_LO, hi=I.GN_HI)
    assert rep.accepted == 1 and rep.t == 1.0 and rep.cg_iters == k
    step = (th1 - th0).reshape(-1)

    J = oracle_lib.jacobian(prob, th0, oracle_lib.epg(prob, th0))
    act = np.repeat([(pmask >> q) & 1 for q in range(5)], prob.nv).astype(bool)
    Ja = J[:, act]
    _, r = oracle_lib.residual(prob, th0, d)
    H = (Ja.conj().T @ Ja).real
    g = (Ja.conj().T @ r.reshape(-1)).real
    V = [g / np.linalg.norm(g)]
    for _ in range(k - 1):
        u = H @ V[-1]
        for b in V:
            u -= (b @ u) * b
        for b in V:
            u -= (b @ u) * b
        V.append(u / np.linalg.norm(u))
    V = np.stack(V, axis=1)
    p = V @ np.linalg.solve(V.T @ H @ V, -(V.T @ g))
    assert np.abs(step[~act]).max() == 0.0
    assert np.linalg.norm(step[act] - p) <= 1e-8 * np.linalg.norm(p)
    assert abs(rep.gnorm - np.linalg.norm(g)) <= 1e-10 * np.linalg.norm(g)
    assert abs(rep.f0 - 0.5 * np.vdot(r, r).real) <= 1e-12 * rep.f0


def test_noiseless_exact_recovery_config1(oracle_lib):
    w = I.config(1)
    prob, th_true = w.problem, w.theta
    d = oracle_lib.signal(prob, th_true, oracle_lib.epg(prob, th_true, tangents=False))
    th = oracle_lib.rho_init(prob, I.initial_theta(prob.nv), d, n_iter=20)
    for _ in range(30):
        th, rep = oracle_lib.gn_step(prob, th, d, n_cg=40, param_mask=w.param_mask,
                                     lo=I.GN_LO, hi=I.GN_HI)
    err = np.linalg.norm(th - th_true) / np.linalg.norm(th_true)
    assert err <= 1e-6, err


def test_noisy_fit_reaches_noise_level(oracle_lib):
    w = I.config(1)
    prob, th_true = w.problem, w.theta
    s = oracle_lib.signal(prob, th_true, oracle_lib.epg(prob, th_true, tangents=False))
    n = I.unit_noise(prob)
    n *= np.linalg.norm(s) / (50.0 * np.linalg.norm(n))   # SNR = ||s|| / ||n|| = 50
    d = s + n
    th = oracle_lib.rho_init(prob, I.initial_theta(prob.nv), d, n_iter=20)
    for _ in range(25):
        th, rep = oracle_lib.gn_step(prob, th, d, n_cg=40, param_mask=w.param_mask,
                                     lo=I.GN_LO, hi=I.GN_HI)
    f, _ = oracle_lib.residual(prob, th, d)
    n_unknown = 4 * prob.nv
    expected = np.vdot(n, n).real * (1.0 - n_unknown / (2.0 * d.size))
    assert abs(2 * f / expected - 1.0) <= 0.05, 2 * f / expected


def test_rho_init_is_least_squares(oracle_lib):
    rng = np.random.default_rng(17)
    prob = I.make_problem(6, 6, 24, 12, 8, flip_deg=I.flips_sin2_sweeps(24, 6, seed=1))
    th = I.iid_maps(prob.nv, seed=2)
    d = rng.standard_normal(prob.data_shape) + 1j * rng.standard_normal(prob.data_shape)
    out = oracle_lib.rho_init(prob, th, d, n_iter=80)
    m = oracle_lib.epg(prob, th, tangents=False)[0]          # [n_tr][Nv]
    E = np.stack([oracle_lib.phases(prob, n) for n in range(prob.n_tr)])  # [n_tr][k][Nv]
    M = (E * m[:, None, :]).reshape(-1, prob.nv)
    ref = np.linalg.lstsq(M, d.reshape(-1), rcond=None)[0]
    got = out[3] + 1j * out[4]
    assert np.linalg.norm(got - ref) <= 1e-8 * np.linalg.norm(ref)
    assert np.array_equal(out[:3], th[:3])


def _galerkin_step(H, g, k):
    """Minimiser of the quadratic model 0.5 p'Hp + g'p over the Krylov space
    span{g, Hg, ..., H^{k-1} g} (orthonormal basis by twice-repeated
    Gram-Schmidt)."""
    V = [g / np.linalg.norm(g)]
    for _ in range(k - 1):
        u = H @ V[-1]
        for _ in range(2):
            for b in V:
                u -= (b @ u) * b
        V.append(u / np.linalg.norm(u))
    V = np.stack(V, axis=1)
    return V @ np.linalg.solve(V.T @ H @ V, -(V.T @ g))


def test_projected_armijo_backtracking(oracle_lib):
    """The line search of the GN step, reproduced in numpy from its
    definition: trial points alpha_t = P(alpha + t p) for t = 1, 1/2, ...,
    with P clamping only the reconstructed ln T1, ln T2, B1 entries of
    unmasked voxels to the box, and the first alpha_t with
    f(alpha_t) <= f + c1 g'(alpha_t - alpha) accepted (the sufficient-
    decrease test on the projected step). The case is built so that the full
    step is rejected, the half step is accepted with active entries clamped,
    an inactive row (B1) lies outside its box interval and a masked voxel's
    ln T1 lies above the box: an Armijo test on the unprojected step, a clamp
    of inactive rows or of masked voxels, or a wrong step sequence gives a
    different accepted point."""
    rng = np.random.default_rng(4)
    prob = I.make_problem(4, 3, 24, 8, 8, flip_deg=I.flips_sin2_sweeps(24, 3, seed=3),
                          t_inv=0.01)
    nv = prob.nv
    th_true = I.iid_maps(nv, seed=3)
    th0 = th_true.copy()
    th0[:2] += 0.2 * rng.standard_normal((2, nv))
    th0[3:] += 0.2 * rng.standard_normal((2, nv))
    mask = np.ones(nv, dtype=np.uint8)
    mask[5] = 0
    th0[0, 5] = np.log(20.0)                      # masked voxel, above the ln T1 box
    d = oracle_lib.signal(prob, th_true, oracle_lib.epg(prob, th_true, tangents=False), mask=mask)
    pmask, k, c1 = 0b11011, 4, 0.6

    J = oracle_lib.jacobian(prob, th0, oracle_lib.epg(prob, th0), mask=mask)
    act = np.zeros((5, nv), dtype=bool)
    for q in range(5):
        act[q] = bool((pmask >> q) & 1) & (mask == 1)
    act = act.reshape(-1)
    Ja = J[:, act]
    f0, r = oracle_lib.residual(prob, th0, d, mask=mask)
    H = (Ja.conj().T @ Ja).real
    ga = (Ja.conj().T @ r.reshape(-1)).real
    p = np.zeros(5 * nv)
    p[act] = _galerkin_step(H, ga, k)
    g = np.zeros(5 * nv)
    g[act] = ga

    # Box: ln T1 capped below where a third of the half-step trial points
    # land; B1 (not reconstructed) has a box that excludes its value 1.
    half = th0.reshape(-1) + 0.5 * p
    hi_t1 = float(np.quantile(half[:nv][mask == 1], 0.66))
    lo = [I.GN_LO[0], I.GN_LO[1], 1.1]
    hi = [hi_t1, I.GN_HI[1], 1.5]

    def project(x):
        x = x.copy().reshape(5, nv)
        for q in range(3):
            if (pmask >> q) & 1:
                sel = mask == 1
                x[q, sel] = np.clip(x[q, sel], lo[q], hi[q])
        return x.reshape(-1)

    expect, t_acc, trials = None, 0.0, 0
    t = 1.0
    for _ in range(8):
        trial = project(th0.reshape(-1) + t * p)
        ft, _ = oracle_lib.residual(prob, trial.reshape(5, nv), d, mask=mask)
        trials += 1
        if ft <= f0 + c1 * (g @ (trial - th0.reshape(-1))):
            expect, t_acc = trial, t
            break
        t *= 0.5
    # Preconditions of the case: backtracking happened and clamps are active.
    assert t_acc == 0.5 and trials == 2
    unclamped = th0.reshape(-1) + t_acc * p
    assert np.count_nonzero(expect != unclamped) >= 3

    got, rep = oracle_lib.gn_step(prob, th0, d, n_cg=k, param_mask=pmask, lo=lo, hi=hi,
                                  n_ls_max=8, armijo_c1=c1, mask=mask)
    assert rep.accepted == 1 and rep.t == t_acc and rep.ls_trials == trials
    assert np.linalg.norm(got.reshape(-1) - expect) <= 1e-8 * np.linalg.norm(expect)
    assert np.array_equal(got[2], th0[2])          # inactive B1 row untouched (1.0 < lo)
    assert got[0, 5] == th0[0, 5]                  # masked voxel untouched
    assert abs(rep.step_norm - np.linalg.norm(expect - th0.reshape(-1))) <= 1e-8 * rep.step_norm
