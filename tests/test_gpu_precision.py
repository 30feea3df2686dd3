"""Precision study of the x-stage contraction on the matrix cores: plain FP32,
split-BF16 (hi*hi + hi*lo + lo*hi, FP32 accumulation) and FP16 (one product,
FP32 accumulation), against the FP64 oracle, separately for the residual,
J v, Re(J^H w) and the reconstructed maps.

Expected error per product (from the arithmetic): FP32 about 2^-24 per term;
split-BF16 drops lo*lo and rounds lo to 8 bits, about 2^-16 relative per term;
FP16 rounds both operands to 11 bits, about 2^-11. The asserted bounds keep a
margin over those: 1e-5 (FP32, the plain path's target), 1e-4 (split-BF16),
5e-3 (FP16). These variants approximate the plain product, so beyond these
stated errors their parity is unpinned.
"""
import numpy as np
import pytest

from paper_1904_13244_amd import inputs as I

pytestmark = pytest.mark.gpu

BOUND = {0: 1e-5, 1: 1e-4, 2: 5e-3}
NAME = {0: "fp32", 1: "split-bf16", 2: "fp16"}


@pytest.fixture(scope="module")
def setup(oracle_lib):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_13244_amd.binding import Context
    w = I.config(3)
    prob = w.problem
    ora = oracle_lib.epg(prob, w.theta)
    dev = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt)  # noqa: E731
    ctx = Context(prob)
    yield dict(torch=torch, w=w, prob=prob, ora=ora, ctx=ctx, dev=dev)
    ctx.close()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("enc", [0, 1, 2])
def test_products_error_vs_oracle(setup, oracle_lib, enc):
    torch, ctx, w, prob, ora, dev = (setup[k] for k in ("torch", "ctx", "w", "prob", "ora", "dev"))
    th = w.theta
    ctx.set_encoding(enc)
    d = oracle_lib.signal(prob, th, ora)
    th1 = th.copy()
    th1[0] += 0.05
    th1 = th1.astype(np.float32).astype(np.float64)
    _, r_ref = oracle_lib.residual(prob, th1, d)
    _, r = ctx.residual(dev(th1, torch.float32), dev(d, torch.complex64))
    e_r = float(np.linalg.norm(r.cpu().numpy() - r_ref) / np.linalg.norm(d))
    v, wv = I.probe_vectors(prob)
    thd = dev(th, torch.float32)
    ctx.linearise(thd)
    jv = ctx.jv(thd, dev(v, torch.float32), reuse=True).cpu().numpy().astype(np.complex128)
    jhw = ctx.jhw(thd, dev(wv, torch.complex64), reuse=True).cpu().numpy().astype(np.float64)
    e_jv = _rel(jv, oracle_lib.jv(prob, th, ora, v))
    e_jhw = _rel(jhw, oracle_lib.jhw(prob, th, ora, wv))
    ctx.set_encoding(0)
    print(f"\n  [{NAME[enc]}] residual err/||d|| {e_r:.2e}  jv {e_jv:.2e}  jhw {e_jhw:.2e}", flush=True)
    for e in (e_r, e_jv, e_jhw):
        assert e <= BOUND[enc]


def test_maps_error_by_precision(setup, oracle_lib):
    """Three GN iterations (20 CG each) on the 128x128 phantom from the same
    start in each precision: the maps' distance to the FP64 oracle's GN
    iterates and their T1/T2 MAPE against the ground truth."""
    torch, dev = setup["torch"], setup["dev"]
    w = I.config(2)
    prob = w.problem
    ora = oracle_lib.epg(prob, w.theta, tangents=False)
    d = oracle_lib.signal(prob, w.theta, ora)
    rng = np.random.default_rng(21)
    th0 = w.theta.copy()
    th0[0] += 0.05 * rng.standard_normal(prob.nv)
    th0[1] += 0.05 * rng.standard_normal(prob.nv)
    th0 = th0.astype(np.float32).astype(np.float64)
    head = w.extra["head"]
    n_gn, n_cg = 3, 20
    th_o = th0.copy()
    for _ in range(n_gn):
        th_o, _ = oracle_lib.gn_step(prob, th_o, d, n_cg=n_cg, param_mask=w.param_mask,
                                     lo=I.GN_LO, hi=I.GN_HI, mask=head.astype(np.uint8))
    mask_t = dev(head.astype(np.uint8), torch.uint8)
    from paper_1904_13244_amd.binding import Context
    res = {}
    for enc in (0, 1, 2):
        c = Context(prob, mask=mask_t)
        c.set_encoding(enc)
        th = dev(th0, torch.float32)
        dd = dev(d, torch.complex64)
        for _ in range(n_gn):
            c.gn_step(th, dd, n_cg, w.param_mask, I.GN_LO, I.GN_HI)
        t = th.cpu().numpy().astype(np.float64)
        c.close()
        e = _rel(t[:, head], th_o[:, head])
        mape = [100 * np.mean(np.abs(np.exp(t[q, head]) - np.exp(w.theta[q, head])) /
                              np.exp(w.theta[q, head])) for q in (0, 1)]
        res[enc] = (e, mape)
        print(f"  [{NAME[enc]}] maps vs oracle GN rel err {e:.2e}; T1 MAPE {mape[0]:.3f} %, "
              f"T2 MAPE {mape[1]:.3f} %", flush=True)
    assert res[0][0] <= 1e-4
    assert res[1][0] <= 1e-3
    assert res[2][0] <= 5e-2
