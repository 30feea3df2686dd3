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


def _shape_cases():
    rng = np.random.default_rng(83)
    T = 45
    # nx odd (no paired A loads in the forward), nk odd (an odd number of
    # 16-column blocks and a ragged last K block in the adjoint).
    ragged = I.make_problem(37, 19, T, 51, 9, flip_deg=rng.uniform(5, 70, T),
                            ky_line=rng.integers(0, 19, T))
    coils = I.make_problem(24, 20, 30, 48, 8, n_coils=4, flip_deg=rng.uniform(5, 70, 30))
    mask = (rng.uniform(size=coils.nv) > 0.2).astype(np.uint8)
    # 8 coils x 530 TRs = 4240 rows: the large-tile x-GEMM, ragged in rows and columns.
    many = I.make_problem(20, 12, 530, 40, 6, n_coils=8, flip_deg=rng.uniform(5, 70, 530))
    mask8 = (rng.uniform(size=many.nv) > 0.2).astype(np.uint8)
    return {"ragged_odd": (ragged, None, None), "coils_mask": (coils, I.coil_maps(24, 20, 4), mask),
            "coils_many_rows": (many, I.coil_maps(20, 12, 8), mask8)}


@pytest.mark.parametrize("name", ["ragged_odd", "coils_mask", "coils_many_rows"])
@pytest.mark.parametrize("enc", [1, 2])
def test_reduced_precision_shapes(oracle_lib, name, enc):
    """The reduced-precision contractions on partial tiles, coils and a mask,
    and with an operand that is not 16-byte aligned, against the oracle."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_13244_amd.binding import Context
    prob, coil, mask = _shape_cases()[name]
    th = I.iid_maps(prob.nv, seed=14, b1=np.full(prob.nv, 1.05))
    dev = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt)  # noqa: E731
    print(f"\n[{NAME[enc]} {name}] nx={prob.nx} ny={prob.ny} nk={prob.n_read} T={prob.n_tr} "
          f"C={prob.n_coils}", flush=True)
    ctx = Context(prob, coil=None if coil is None else dev(coil, torch.complex64),
                  mask=None if mask is None else dev(mask, torch.uint8))
    ctx.set_encoding(enc)
    ora = oracle_lib.epg(prob, th)
    thd = dev(th, torch.float32)
    v, wv = I.probe_vectors(prob)
    jv = ctx.jv(thd, dev(v, torch.float32)).cpu().numpy().astype(np.complex128)
    jhw = ctx.jhw(thd, dev(wv, torch.complex64), reuse=True).cpu().numpy().astype(np.float64)
    e_jv = _rel(jv, oracle_lib.jv(prob, th, ora, v, coil=coil, mask=mask))
    jhw_ref = oracle_lib.jhw(prob, th, ora, wv, coil=coil, mask=mask)
    e_jhw = _rel(jhw, jhw_ref)
    # w at an 8-byte offset: element loads instead of 16-byte loads.
    buf = torch.zeros(wv.size + 1, dtype=torch.complex64, device="cuda")
    w_off = buf[1:].view(wv.shape)
    w_off.copy_(dev(wv, torch.complex64))
    e_off = _rel(ctx.jhw(thd, w_off, reuse=True).cpu().numpy().astype(np.float64), jhw_ref)
    d = oracle_lib.signal(prob, th, ora, coil=coil, mask=mask)
    th1 = th.copy()
    th1[0] += 0.05
    th1 = th1.astype(np.float32).astype(np.float64)
    _, r_ref = oracle_lib.residual(prob, th1, d, coil=coil, mask=mask)
    f, r = ctx.residual(dev(th1, torch.float32), dev(d, torch.complex64))
    e_r = float(np.linalg.norm(r.cpu().numpy() - r_ref) / np.linalg.norm(d))
    f_ref = 0.5 * float(np.linalg.norm(r_ref) ** 2)
    e_f = abs(f - f_ref) / f_ref
    ctx.close()
    print(f"  jv {e_jv:.2e} jhw {e_jhw:.2e} (offset w {e_off:.2e}) residual {e_r:.2e} f {e_f:.2e}",
          flush=True)
    assert max(e_jv, e_jhw, e_off, e_r) <= BOUND[enc]
    assert e_f <= 2 * BOUND[enc]
