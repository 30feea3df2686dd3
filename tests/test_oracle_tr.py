"""Pins of the oracle's trust-region Gauss-Newton step (Methods,
Reconstructions: Steihaug's truncated CG, Nocedal & Wright Algorithm 7.2, and
reflection at the feasible bounds after Coleman & Li).

Independent references, none of which repeats the oracle's recurrences:
  * CG iterates from zero are the Galerkin solutions of the model on the
    growing Krylov spaces, and their norms increase (Steihaug; Nocedal &
    Wright Theorem 7.3). Inside a large region the truncated CG returns the
    k-th Galerkin solution; when the region is crossed between the (k-1)-th
    and the k-th, it returns the point of that segment on the boundary.
  * On a model whose first search direction -g has negative curvature the
    step is the boundary point along -g (the lower of the two boundary
    points); with negative curvature found at the second direction of a
    two-dimensional model, that direction is the B-conjugate of the first.
  * The reflection is the end point of a particle moving with the step's
    velocity for unit time between two walls, stepped in small increments.
  * The ratio test uses the Jacobian built explicitly (itself pinned by finite
    differences) and the oracle's residual; a fit of rho alone has an exactly
    quadratic objective, so the ratio is 1.
"""
import numpy as np
import pytest

from paper_1904_13244_amd import inputs as I


def _galerkin(B, g, k):
    """Minimiser of g'p + 0.5 p'Bp over span{g, Bg, ..., B^{k-1} g}."""
    if k == 0:
        return np.zeros_like(g)
    V = [g / np.linalg.norm(g)]
    for _ in range(k - 1):
        u = B @ V[-1]
        for _ in range(2):
            for b in V:
                u -= (b @ u) * b
        V.append(u / np.linalg.norm(u))
    V = np.stack(V, axis=1)
    return V @ np.linalg.solve(V.T @ B @ V, -(V.T @ g))


def _segment_point(a, b, delta):
    """The point of the segment a -> b with norm delta (|a| < delta <= |b|)."""
    d = b - a
    A, Bq, Cq = d @ d, 2 * a @ d, a @ a - delta * delta
    tau = (-Bq + np.sqrt(Bq * Bq - 4 * A * Cq)) / (2 * A)
    return a + tau * d


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Q * np.geomspace(0.05, 20.0, n)) @ Q.T, rng.standard_normal(n)


@pytest.mark.parametrize("k", [1, 2, 4, 6])
def test_steihaug_inside_region_is_galerkin(oracle_lib, k):
    B, g = _spd(12, 1)
    p, kind, it = oracle_lib.steihaug_dense(B, g, 1e6, k)
    ref = _galerkin(B, g, k)
    assert kind == oracle_lib.TR_ITERS and it == k
    assert np.linalg.norm(p - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_steihaug_boundary_exit(oracle_lib, k):
    B, g = _spd(12, 2)
    G = [_galerkin(B, g, j) for j in range(8)]
    norms = [np.linalg.norm(x) for x in G]
    assert all(a < b for a, b in zip(norms, norms[1:]))       # monotone (the theorem)
    delta = 0.5 * (norms[k - 1] + norms[k])
    p, kind, it = oracle_lib.steihaug_dense(B, g, delta, 8)
    ref = _segment_point(G[k - 1], G[k], delta)
    assert kind == oracle_lib.TR_BOUNDARY and it == k - 1
    assert abs(np.linalg.norm(p) - delta) <= 1e-12 * delta
    assert np.linalg.norm(p - ref) <= 1e-10 * delta


def test_steihaug_negative_curvature_first_direction(oracle_lib):
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    B = (Q * np.array([-3.0, -1.0, 0.5, 1.0, 2.0, 4.0])) @ Q.T
    g = Q[:, 0] + 0.1 * Q[:, 5]                  # g'Bg < 0
    assert g @ B @ g < 0
    delta = 0.7
    p, kind, it = oracle_lib.steihaug_dense(B, g, delta, 5)
    assert kind == oracle_lib.TR_CURVATURE and it == 0
    assert np.linalg.norm(p + delta * g / np.linalg.norm(g)) <= 1e-12


@pytest.mark.parametrize("a,b,g1,g2,delta", [(2.0, 1.0, 3.0, 0.5, 5.0),
                                              (3.6, 10.5, -1.14, -0.085, 8.95)])
def test_steihaug_negative_curvature_second_direction(oracle_lib, a, b, g1, g2, delta):
    """The second case's lower model value lies at the boundary point behind
    the current iterate (the negative root along the search direction)."""
    B = np.diag([a, -b])
    g = np.array([g1, g2])
    assert g @ B @ g > 0
    z1 = -(g @ g) / (g @ B @ g) * g               # Galerkin solution on span{g}
    assert np.linalg.norm(z1) < delta
    Bd0 = B @ (-g)
    d1 = np.array([-Bd0[1], Bd0[0]])              # B-conjugate to d0 = -g
    assert d1 @ B @ d1 < 0
    dd, zd, zz = d1 @ d1, z1 @ d1, z1 @ z1
    roots = [(-zd + s * np.sqrt(zd * zd + dd * (delta * delta - zz))) / dd for s in (1, -1)]
    cand = [z1 + t * d1 for t in roots]
    model = [g @ c + 0.5 * c @ B @ c for c in cand]
    ref = cand[int(np.argmin(model))]
    p, kind, it = oracle_lib.steihaug_dense(B, g, delta, 5)
    assert kind == oracle_lib.TR_CURVATURE and it == 1
    assert np.linalg.norm(p - ref) <= 1e-12 * delta


def test_steihaug_zero_gradient(oracle_lib):
    B, _ = _spd(5, 4)
    p, kind, it = oracle_lib.steihaug_dense(B, np.zeros(5), 1.0, 3)
    assert kind == oracle_lib.TR_ZERO and it == 0 and not p.any()


def _bounce(x0, v, lo, hi, steps=200_000):
    x, dt = x0, 1.0 / steps
    for _ in range(steps):
        x += v * dt
        if x > hi:
            x, v = 2 * hi - x, -v
        elif x < lo:
            x, v = 2 * lo - x, -v
    return x


@pytest.mark.parametrize("x0,v", [(0.3, 0.4), (0.3, 1.1), (0.8, -2.7), (0.05, 4.6), (0.5, -0.2)])
def test_reflect_is_the_bouncing_path(oracle_lib, x0, v):
    lo, hi = 0.0, 1.0
    got = oracle_lib.reflect(x0 + v, lo, hi)
    assert lo <= got <= hi
    assert abs(got - _bounce(x0, v, lo, hi)) <= 1e-4
    assert oracle_lib.reflect(2.0, 1.5, 1.5) == 1.5


def _tiny(seed=3, pert=0.05):
    rng = np.random.default_rng(seed)
    prob = I.make_problem(4, 3, 24, 8, 8, flip_deg=I.flips_sin2_sweeps(24, 3, seed=seed), t_inv=0.01)
    th_true = I.iid_maps(prob.nv, seed=seed)
    th0 = th_true.copy()
    th0[:2] += pert * rng.standard_normal((2, prob.nv))
    th0[3:] += pert * rng.standard_normal((2, prob.nv))
    d = None
    return prob, th_true, th0, d


def _model(oracle_lib, prob, th0, d, pmask):
    J = oracle_lib.jacobian(prob, th0, oracle_lib.epg(prob, th0))
    act = np.repeat([(pmask >> q) & 1 for q in range(5)], prob.nv).astype(bool)
    f0, r = oracle_lib.residual(prob, th0, d)
    Ja = J[:, act]
    H = (Ja.conj().T @ Ja).real
    g = (Ja.conj().T @ r.reshape(-1)).real
    return J, act, f0, H, g


def _ratio(oracle_lib, prob, J, g_full, f0, th0, th1, d):
    s = (th1 - th0).reshape(-1)
    ft, _ = oracle_lib.residual(prob, th1, d)
    Js = J @ s
    pred = -(g_full @ s + 0.5 * np.vdot(Js, Js).real)
    return (f0 - ft) / pred, pred


@pytest.mark.parametrize("box", ["wide", "reflecting"])
def test_tr_step_boundary_step_and_ratio(oracle_lib, box):
    prob, th_true, th0, _ = _tiny()
    nv = prob.nv
    d = oracle_lib.signal(prob, th_true, oracle_lib.epg(prob, th_true, tangents=False))
    pmask = 0b11011
    J, act, f0, H, g = _model(oracle_lib, prob, th0, d, pmask)
    n_cg = 6
    G = [_galerkin(H, g, j) for j in range(n_cg + 1)]
    norms = [np.linalg.norm(x) for x in G]
    delta = 0.5 * (norms[2] + norms[3])           # crossed in the third CG iteration
    p = np.zeros(5 * nv)
    p[act] = _segment_point(G[2], G[3], delta)
    lo, hi = list(I.GN_LO), list(I.GN_HI)
    if box == "reflecting":
        x = th0[0] + p[:nv]
        hi[0] = float(np.quantile(x, 0.6))        # 40 % of the ln T1 entries reflect
    th1, delta1, rep = oracle_lib.tr_step(prob, th0, d, delta, n_cg, pmask, lo, hi, eta=0.1)
    expect = th0.reshape(-1) + p
    for j in range(nv):
        expect[j] = oracle_lib.reflect(expect[j], lo[0], hi[0])
        expect[nv + j] = oracle_lib.reflect(expect[nv + j], lo[1], hi[1])
    assert rep["exit_kind"] == oracle_lib.TR_BOUNDARY and rep["cg_iters"] == 2
    assert rep["accepted"] == 1
    assert np.linalg.norm(th1.reshape(-1) - expect) <= 1e-8 * np.linalg.norm(expect)
    n_ref = int(np.count_nonzero(expect != th0.reshape(-1) + p))
    assert rep["n_reflected"] == n_ref and (n_ref > 0) == (box == "reflecting")
    g_full = np.zeros(5 * nv)
    g_full[act] = g
    rho, pred = _ratio(oracle_lib, prob, J, g_full, f0, th0, th1, d)
    assert abs(rep["rho"] - rho) <= 1e-8 * abs(rho) and abs(rep["pred"] - pred) <= 1e-8 * pred
    want = 0.25 * delta if rho < 0.25 else (min(2 * delta, 1e3) if rho > 0.75 else delta)
    assert delta1 == pytest.approx(want, rel=1e-15)
    assert abs(rep["f0"] - f0) <= 1e-12 * f0


def test_tr_step_exact_model_for_rho_alone(oracle_lib):
    """With only rho fitted the signal is linear in the unknowns, the model is
    the objective, the ratio is 1 and a boundary step doubles the radius."""
    prob, th_true, th0, _ = _tiny(seed=5)
    d = oracle_lib.signal(prob, th_true, oracle_lib.epg(prob, th_true, tangents=False))
    pmask = 0b11000
    _, _, _, H, g = _model(oracle_lib, prob, th0, d, pmask)
    G1 = _galerkin(H, g, 1)
    delta = 0.5 * np.linalg.norm(G1)
    th1, delta1, rep = oracle_lib.tr_step(prob, th0, d, delta, 4, pmask, I.GN_LO, I.GN_HI,
                                          delta_max=10 * delta)
    assert rep["exit_kind"] == oracle_lib.TR_BOUNDARY and rep["accepted"] == 1
    assert abs(rep["rho"] - 1.0) <= 1e-9
    assert delta1 == 2 * delta
    assert np.array_equal(th1[:3], th0[:3])
    # Inside the region (the CG count reached first) the radius stays.
    th2, delta2, rep2 = oracle_lib.tr_step(prob, th0, d, 1e3, 1, pmask, I.GN_LO, I.GN_HI,
                                           delta_max=1e4)
    assert rep2["exit_kind"] == oracle_lib.TR_ITERS and abs(rep2["rho"] - 1.0) <= 1e-9
    assert delta2 == 1e3 and rep2["accepted"] == 1
    assert np.linalg.norm((th2 - th0).reshape(-1)[3 * prob.nv:] - G1) <= 1e-10 * np.linalg.norm(G1)


def test_tr_step_rejects_poor_model(oracle_lib):
    """Far from the data's T2 a long interior step predicts more decrease
    than it gets: with eta = 0.5 the ratio (computed here from the explicit
    Jacobian at the Galerkin step, reflected into the box) rejects it, theta
    stays unchanged and the radius follows the ratio."""
    prob, th_true, th0, _ = _tiny(seed=7)
    th0[1] -= 2.0                               # T2 far too short
    nv = prob.nv
    d = oracle_lib.signal(prob, th_true, oracle_lib.epg(prob, th_true, tangents=False))
    pmask, n_cg, delta = 0b11011, 10, 50.0
    J, act, f0, H, g = _model(oracle_lib, prob, th0, d, pmask)
    p = np.zeros(5 * nv)
    p[act] = _galerkin(H, g, n_cg)
    assert np.linalg.norm(p) < delta
    trial = th0.reshape(-1) + p
    for q in range(2):
        for j in range(nv):
            trial[q * nv + j] = oracle_lib.reflect(trial[q * nv + j], I.GN_LO[q], I.GN_HI[q])
    g_full = np.zeros(5 * nv)
    g_full[act] = g
    rho, _ = _ratio(oracle_lib, prob, J, g_full, f0, th0, trial.reshape(5, nv), d)
    th1, delta1, rep = oracle_lib.tr_step(prob, th0, d, delta, n_cg, pmask, I.GN_LO, I.GN_HI, eta=0.5)
    assert rep["exit_kind"] == oracle_lib.TR_ITERS and rep["cg_iters"] == n_cg
    assert abs(rep["rho"] - rho) <= 1e-6 * abs(rho)
    assert rho < 0.5 and rep["accepted"] == 0 and np.array_equal(th1, th0)
    assert delta1 == (0.25 * delta if rho < 0.25 else delta)
    assert rep["f1"] == rep["f0"]
