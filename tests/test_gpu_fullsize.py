"""Full-size parity at the benchmark workload (224x224 phantom, 1120 TRs,
448 samples, K = 32, one coil) in the launch configuration bench.py times,
and at the 256x256, 8-coil, 1280-TR workload: every train element, the
residual, J v and Re(J^H w) against the FP64 oracle evaluated on the whole
problem (the oracle EPG takes seconds on the host)."""
import time

import numpy as np
import pytest

from paper_1904_13244_amd import inputs as I

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module", params=[3, 5])
def setup(request, oracle_lib):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_13244_amd.binding import Context
    w = I.config(request.param)
    prob = w.problem
    print(f"\n[full size] {w.name}", flush=True)
    t0 = time.time()
    ora = oracle_lib.epg(prob, w.theta)
    print(f"  oracle EPG at full size: {time.time() - t0:.1f} s", flush=True)
    dev = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt)  # noqa: E731
    ctx = Context(prob, coil=None if w.coil is None else dev(w.coil, torch.complex64))
    yield dict(torch=torch, w=w, prob=prob, ora=ora, ctx=ctx, dev=dev, coil=w.coil)
    ctx.close()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_fullsize_trains(setup):
    torch, ctx, w = setup["torch"], setup["ctx"], setup["w"]
    got = ctx.simulate(setup["dev"](w.theta, torch.float32)).cpu().numpy()
    for p in range(4):
        e = _rel(got[p].astype(np.float64), setup["ora"][p].imag)
        print(f"  train {p} rel err {e:.2e}")
        assert e <= TOL


def test_fullsize_residual_jv_jhw(setup, oracle_lib):
    torch, ctx, w, prob, ora, dev = (setup[k] for k in ("torch", "ctx", "w", "prob", "ora", "dev"))
    th = w.theta
    thd = dev(th, torch.float32)
    # Residual at a perturbed point against noiseless oracle data.
    coil = setup["coil"]
    d = oracle_lib.signal(prob, th, ora, coil=coil)
    th1 = th.copy()
    th1[0] += 0.05
    th1 = th1.astype(np.float32).astype(np.float64)
    f_ref, r_ref = oracle_lib.residual(prob, th1, d, coil=coil)
    f, r = ctx.residual(dev(th1, torch.float32), dev(d, torch.complex64))
    e = float(np.linalg.norm(r.cpu().numpy() - r_ref) / np.linalg.norm(d))
    print(f"  residual err/||d|| {e:.2e}")
    assert e <= TOL
    # Products at theta (re-linearise there).
    v, wv = I.probe_vectors(prob)
    ctx.linearise(thd)
    jv = ctx.jv(thd, dev(v, torch.float32), reuse=True).cpu().numpy()
    jhw = ctx.jhw(thd, dev(wv, torch.complex64), reuse=True).cpu().numpy()
    jv_ref = oracle_lib.jv(prob, th, ora, v, coil=coil)
    jhw_ref = oracle_lib.jhw(prob, th, ora, wv, coil=coil)
    e_jv = _rel(jv.astype(np.complex128), jv_ref)
    print(f"  jv rel err {e_jv:.2e}")
    assert e_jv <= TOL
    for q in range(5):
        e = _rel(jhw[q].astype(np.float64), jhw_ref[q])
        print(f"  jhw row {q} rel err {e:.2e}")
        assert e <= TOL
    lhs = np.vdot(wv.reshape(-1), jv.astype(np.complex128).reshape(-1)).real
    rhs = float(np.dot(v.reshape(-1), jhw.astype(np.float64).reshape(-1)))
    assert abs(lhs - rhs) <= 1e-5 * max(abs(lhs), abs(rhs))
