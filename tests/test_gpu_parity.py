"""Parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: the FP32 plain path must match the oracle to 1e-5 relative,
measured normwise: ||x_gpu - x_oracle|| / ||x_oracle|| for trains, J v and
Re(J^H w); ||r_gpu - r_oracle|| / ||d|| for the residual (r = d - s cancels
near convergence, so its error is measured against the data it came from).
Every input is seeded; every expected value comes from the oracle.
"""
import numpy as np
import pytest

from paper_1904_13244_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_13244_amd import binding
    binding.lib()   # fail loudly if the HIP library is missing
    return torch


def _dev(torch, a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype).contiguous()


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _ragged():
    """Sizes that leave partial tiles everywhere: nx not a multiple of 64,
    ny not a multiple of 32, K not a power of two, RF phases 0/pi, inversion
    delay, nonuniform line order."""
    rng = np.random.default_rng(77)
    T = 70
    prob = I.make_problem(37, 29, T, 80, 13, flip_deg=rng.uniform(0, 80, T),
                          rf_phase=np.pi * rng.integers(0, 2, T), t_inv=0.02, tr=0.0075,
                          te=0.003, ky_line=rng.integers(0, 29, T))
    th = I.iid_maps(prob.nv, seed=8, b1=rng.uniform(0.75, 1.25, prob.nv))
    return "ragged", prob, th, None, None


def _config1():
    w = I.config(1)
    return "config1", w.problem, w.theta, None, None


def _coils():
    rng = np.random.default_rng(5)
    prob = I.make_problem(24, 20, 60, 48, 16, n_coils=4, flip_deg=I.flips_sin2_sweeps(60, 20))
    th = I.iid_maps(prob.nv, seed=4, b1=rng.uniform(0.8, 1.2, prob.nv))
    mask = (rng.uniform(size=prob.nv) > 0.2).astype(np.uint8)
    return "coils_mask", prob, th, I.coil_maps(24, 20, 4), mask


def _config2():
    w = I.config(2)
    return "config2", w.problem, w.theta, None, None


CASES = {"config1": _config1, "ragged": _ragged, "coils_mask": _coils, "config2": _config2}


@pytest.fixture(scope="module", params=list(CASES))
def case(request, torch_gpu, oracle_lib):
    torch = torch_gpu
    name, prob, th, coil, mask = CASES[request.param]()
    print(f"\n[case {name}] nx={prob.nx} ny={prob.ny} T={prob.n_tr} nk={prob.n_read} "
          f"K={prob.n_states} C={prob.n_coils}", flush=True)
    from paper_1904_13244_amd.binding import Context
    ctx = Context(prob, coil=None if coil is None else _dev(torch, coil, torch.complex64),
                  mask=None if mask is None else _dev(torch, mask, torch.uint8))
    ora_trains = oracle_lib.epg(prob, th)
    v, w = I.probe_vectors(prob)
    yield dict(name=name, prob=prob, th=th, coil=coil, mask=mask, ctx=ctx, ora=ora_trains,
               v=v, w=w, torch=torch)
    ctx.close()


def test_trains(case):
    torch, ctx, prob = case["torch"], case["ctx"], case["prob"]
    thd = _dev(torch, case["th"], torch.float32)
    got = ctx.simulate(thd).cpu().numpy().astype(np.float64)
    ref = case["ora"]
    assert np.abs(ref.real).max() <= 1e-12 * np.abs(ref.imag).max()
    for p in range(4):
        e = _rel(got[p], ref[p].imag)
        print(f"  train {p}: rel err {e:.2e}")
        assert e <= TOL, (p, e)


def test_trains_lane_splits(case, oracle_lib):
    torch, ctx = case["torch"], case["ctx"]
    thd = _dev(torch, case["th"], torch.float32)
    ref = case["ora"].imag
    outs = []
    for lanes in (1, 2, 4, 8):
        ctx.set_epg_lanes(lanes)
        outs.append(ctx.simulate(thd).cpu().numpy().astype(np.float64))
    ctx.set_epg_lanes(0)
    for o in outs:
        for p in range(4):
            assert _rel(o[p], ref[p]) <= TOL


def test_residual(case, oracle_lib):
    torch, ctx, prob = case["torch"], case["ctx"], case["prob"]
    th = case["th"]
    s = oracle_lib.signal(prob, th, case["ora"], coil=case["coil"], mask=case["mask"])
    n = I.unit_noise(prob)
    d = s + n * (np.linalg.norm(s) / (50.0 * np.linalg.norm(n)))
    th0 = th.copy()
    th0[0] += 0.05   # evaluate away from the truth so r is not just the noise
    f_ref, r_ref = oracle_lib.residual(prob, th0, d, coil=case["coil"], mask=case["mask"])
    f, r = ctx.residual(_dev(torch, th0, torch.float32), _dev(torch, d, torch.complex64))
    r = r.cpu().numpy().astype(np.complex128)
    e = float(np.linalg.norm(r - r_ref) / np.linalg.norm(d))
    print(f"  residual err/||d|| {e:.2e}  f {f:.6e} vs {f_ref:.6e}")
    assert e <= TOL
    assert abs(f - f_ref) <= TOL * 0.5 * np.vdot(d, d).real


def test_jv(case, oracle_lib):
    torch, ctx, prob = case["torch"], case["ctx"], case["prob"]
    th, v = case["th"], case["v"]
    ref = oracle_lib.jv(prob, th, case["ora"], v, coil=case["coil"], mask=case["mask"])
    got = ctx.jv(_dev(torch, th, torch.float32), _dev(torch, v, torch.float32))
    got = got.cpu().numpy().astype(np.complex128)
    e = _rel(got, ref)
    print(f"  jv rel err {e:.2e}")
    assert e <= TOL


def test_jhw(case, oracle_lib):
    torch, ctx, prob = case["torch"], case["ctx"], case["prob"]
    th, w = case["th"], case["w"]
    ref = oracle_lib.jhw(prob, th, case["ora"], w, coil=case["coil"], mask=case["mask"])
    got = ctx.jhw(_dev(torch, th, torch.float32), _dev(torch, w, torch.complex64))
    got = got.cpu().numpy().astype(np.float64)
    for q in range(5):
        e = _rel(got[q], ref[q]) if np.linalg.norm(ref[q]) > 0 else np.abs(got[q]).max()
        print(f"  jhw row {q} rel err {e:.2e}")
        assert e <= TOL, (q, e)


def test_reuse_and_adjoint_identity(case):
    torch, ctx = case["torch"], case["ctx"]
    thd = _dev(torch, case["th"], torch.float32)
    vd = _dev(torch, case["v"], torch.float32)
    wd = _dev(torch, case["w"], torch.complex64)
    ctx.linearise(thd)
    a = ctx.jv(thd, vd, reuse=True).cpu().numpy()
    b = ctx.jhw(thd, wd, reuse=True).cpu().numpy()
    a2 = ctx.jv(thd, vd, reuse=False).cpu().numpy()
    b2 = ctx.jhw(thd, wd, reuse=False).cpu().numpy()
    assert np.array_equal(a, a2) and np.array_equal(b, b2)   # deterministic, same trains
    lhs = np.vdot(case["w"].reshape(-1), a.astype(np.complex128).reshape(-1)).real
    rhs = float(np.dot(case["v"].reshape(-1), b.astype(np.float64).reshape(-1)))
    assert abs(lhs - rhs) <= 1e-5 * max(abs(lhs), abs(rhs))


def test_reuse_without_linearisation_is_an_error(torch_gpu):
    torch = torch_gpu
    from paper_1904_13244_amd.binding import Context, MrstatError, ERR_STATE
    prob = I.make_problem(8, 8, 16, 16, 8)
    ctx = Context(prob)
    th = _dev(torch, I.iid_maps(prob.nv), torch.float32)
    v = torch.zeros((5, prob.nv), dtype=torch.float32, device="cuda")
    with pytest.raises(MrstatError) as ei:
        ctx.jv(th, v, reuse=True)
    assert ei.value.status == ERR_STATE
    ctx.close()
