"""The trust-region Gauss-Newton step (mrstat_tr_step: Steihaug CG inside the
radius, reflection into the box, ratio test and radius update) on the GPU
against the oracle's (oracle_tr_step, pinned in tests/test_oracle_tr.py).

Both sides start from the same FP32-representable point and radius. Each
iteration's decisions (CG exit kind and count, acceptance, the new radius)
must agree exactly, theta to the plain path's 1e-5 relative, the ratio to
1e-4 absolute (it divides two FP32-rounded decreases).
"""
import numpy as np
import pytest

from paper_1904_13244_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_13244_amd import binding
    binding.lib()
    return torch


def _dev(torch, a, dt):
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt).contiguous()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _start(theta_true, seed=13):
    rng = np.random.default_rng(seed)
    th = theta_true.copy()
    th[0] += 0.1 * rng.standard_normal(th.shape[1])
    th[1] += 0.1 * rng.standard_normal(th.shape[1])
    th[3:] *= 1.0 + 0.05 * rng.standard_normal((2, th.shape[1]))
    return th.astype(np.float32).astype(np.float64)


def _compare(rep_g, dg, rep_o, do, th_g, th_o, tag):
    e = _rel(th_g, th_o)
    print(f"  [{tag}] exit {rep_g.exit_kind}/{rep_o['exit_kind']} cg {rep_g.cg_iters}/{rep_o['cg_iters']} "
          f"acc {rep_g.accepted}/{rep_o['accepted']} rho {rep_g.rho:.6f}/{rep_o['rho']:.6f} "
          f"delta {dg:.4g}/{do:.4g} refl {rep_g.n_reflected}/{rep_o['n_reflected']} theta {e:.2e}",
          flush=True)
    assert rep_g.exit_kind == rep_o["exit_kind"] and rep_g.cg_iters == rep_o["cg_iters"]
    assert rep_g.accepted == rep_o["accepted"] and dg == do
    assert rep_g.n_reflected == rep_o["n_reflected"]
    if np.isinf(rep_o["rho"]):
        assert rep_g.rho == rep_o["rho"]
    else:
        assert abs(rep_g.rho - rep_o["rho"]) <= 1e-4
    assert e <= 1e-5


@pytest.mark.parametrize("param_mask,box", [(0b11011, "wide"), (0b11111, "wide"), (0b11011, "reflecting")])
def test_tr_iterations_match_oracle_config1(torch_gpu, oracle_lib, param_mask, box):
    torch = torch_gpu
    from paper_1904_13244_amd.binding import Context
    w = I.config(1)
    prob = w.problem
    d = oracle_lib.signal(prob, w.theta, oracle_lib.epg(prob, w.theta, tangents=False))
    lo, hi = list(I.GN_LO), list(I.GN_HI)
    if box == "reflecting":
        hi[0] = float(np.float32(np.log(2.0)))   # below the longest T1 of the phantom (FP32 exact)
    th_o = _start(w.theta)
    th_o[0] = np.minimum(th_o[0], hi[0] - 1e-3).astype(np.float32)   # a feasible start
    th_g = _dev(torch, th_o, torch.float32)
    dd = _dev(torch, d, torch.complex64)
    ctx = Context(prob)
    do = dg = 1.0
    kinds, refl = set(), 0
    for it in range(6):
        th_o, do, rep_o = oracle_lib.tr_step(prob, th_o, d, do, w.n_cg, param_mask, lo, hi, eta=0.1,
                                             delta_max=8.0)
        dg, rep_g = ctx.tr_step(th_g, dd, dg, w.n_cg, param_mask, lo, hi, eta=0.1, delta_max=8.0)
        _compare(rep_g, dg, rep_o, do, th_g.cpu().numpy().astype(np.float64), th_o, f"it {it}")
        kinds.add(rep_o["exit_kind"])
        refl += rep_o["n_reflected"]
    ctx.close()
    assert 1 in kinds                      # the radius bound the step at least once
    assert (refl > 0) == (box == "reflecting")


def test_tr_step_failure_paths(torch_gpu, oracle_lib):
    torch = torch_gpu
    from paper_1904_13244_amd import binding as B
    from paper_1904_13244_amd.binding import Context
    w = I.config(1)
    prob = w.problem
    d = oracle_lib.signal(prob, w.theta, oracle_lib.epg(prob, w.theta, tangents=False))
    bad = d.copy()
    bad[0, 7, 2] = np.nan
    ctx = Context(prob)
    th = _dev(torch, _start(w.theta), torch.float32)
    before = th.clone()
    with pytest.raises(B.MrstatError) as e:
        ctx.tr_step(th, _dev(torch, bad, torch.complex64), 1.0, 5, 0b11011, I.GN_LO, I.GN_HI)
    assert e.value.status == B.ERR_NONFINITE and torch.equal(th, before)
    dd = _dev(torch, d, torch.complex64)
    for delta, kw in ((0.0, {}), (2.0, {"delta_max": 1.0}), (1.0, {"eta": 1.0}), (float("nan"), {})):
        with pytest.raises(B.MrstatError) as e:
            ctx.tr_step(th, dd, delta, 5, 0b11011, I.GN_LO, I.GN_HI, **kw)
        assert e.value.status == B.ERR_ARG
    # At the truth: zero gradient, zero step, exit on the zero residual.
    tt = _dev(torch, w.theta.astype(np.float32), torch.float32)
    zeros = torch.zeros(prob.data_shape, dtype=torch.complex64, device="cuda")
    _, r = ctx.residual(tt, zeros)
    dn, rep = ctx.tr_step(tt, (-r).contiguous(), 1.0, 5, 0b11011, I.GN_LO, I.GN_HI)
    assert rep.exit_kind == B.TR_ZERO and rep.cg_iters == 0 and rep.gnorm == 0.0 and rep.step_norm == 0.0
    ctx.close()
