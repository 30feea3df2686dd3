"""Readout dynamics on the GPU (mrstat_create_readout with an off-resonance
map from mrstat_set_db0: T2 decay and off-resonance phase during each
readout, the extension the Discussion names) against the FP64 oracle's
direct sum (pinned in tests/test_oracle_readout.py by an isochromat brute
force, a closed form and finite differences).

The GPU evaluates exp(lambda tau) as a power series in tau / tau_max with the
term count its context chose (remainder at most 1e-7 within the context's T2
and off-resonance bounds) and sums the terms in FP32, so the plain path's
bar holds: 1e-5 relative for the residual (against ||d||), J v and each row
of Re(J^H w) with FP32 trains and the FP32 x-stage; FP16 trains take the
static path's 1e-3, the split-BF16 x-stage its 1e-4. The cases span the term
counts 12, 16, 20 and 32, ragged tiles, a mask and three coils; a full-size case
(224 x 224, 1120 TRs, 448 samples, 24 terms) checks 160 masked-in voxels
against the oracle's direct sum. Every input is seeded; every expected value
comes from the oracle.
"""
import dataclasses

import numpy as np
import pytest

from paper_1904_13244_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-5
BW = 85.6e3    # readout bandwidth of the paper's in-vivo scans [Hz]


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


def _maps(prob, rng, seed):
    """T2 from 10 to 150 ms (decay visible over a readout), T1 and rho from the
    i.i.d. recipe, B1 in [0.8, 1.2]; FP32-representable."""
    th = I.iid_maps(prob.nv, seed=seed, b1=rng.uniform(0.8, 1.2, prob.nv))
    th[1] = np.log(rng.uniform(0.01, 0.15, prob.nv))
    return th.astype(np.float32).astype(np.float64)


def _case(name):
    if name == "small":      # 12 terms
        rng = np.random.default_rng(51)
        prob = I.make_problem(20, 18, 60, 40, 8, tr=0.008, te=0.004, flip_deg=I.flips_sin2_sweeps(60, 18),
                              ky_line=rng.integers(0, 18, 60))
        dwell, seed = 1 / BW, 52
    elif name == "ragged":   # 16 terms
        rng = np.random.default_rng(53)
        T = 70
        prob = I.make_problem(37, 29, T, 150, 13, flip_deg=rng.uniform(0, 80, T),
                              rf_phase=np.pi * rng.integers(0, 2, T), t_inv=0.02, tr=0.0075,
                              te=0.003, ky_line=rng.integers(0, 29, T))
        dwell, seed = 1 / BW, 54
    elif name == "half_bandwidth":   # 20 terms; an odd TR count (a forward block's second TR unused)
        rng = np.random.default_rng(55)
        prob = I.make_problem(24, 20, 51, 150, 8, tr=0.01, te=0.005, flip_deg=I.flips_sin2_sweeps(51, 20),
                              ky_line=rng.integers(0, 20, 51))
        dwell, seed = 2 / BW, 56
    elif name == "quarter_bandwidth":   # 32 terms
        rng = np.random.default_rng(57)
        prob = I.make_problem(24, 20, 50, 150, 8, tr=0.012, te=0.006, flip_deg=I.flips_sin2_sweeps(50, 20),
                              ky_line=rng.integers(0, 20, 50))
        dwell, seed = 4 / BW, 58
    else:
        raise ValueError(name)
    db0 = rng.uniform(-150.0, 150.0, prob.nv)
    prob = dataclasses.replace(prob, dwell=dwell, db0=db0)
    th = _maps(prob, rng, seed)
    mask = (rng.uniform(size=prob.nv) > 0.2).astype(np.uint8)
    return prob, th, mask


TERMS = {"small": 12, "ragged": 16, "half_bandwidth": 20, "quarter_bandwidth": 32}
CHEB_TERMS = {"small": 8, "ragged": 12, "half_bandwidth": 16, "quarter_bandwidth": 20}


@pytest.fixture(scope="module", params=list(TERMS))
def case(request, torch_gpu, oracle_lib):
    torch = torch_gpu
    from paper_1904_13244_amd.binding import Context
    prob, th, mask = _case(request.param)
    print(f"\n[readout case {request.param}] nx={prob.nx} ny={prob.ny} T={prob.n_tr} nk={prob.n_read} "
          f"dwell={prob.dwell:.3e}", flush=True)
    ctx = Context(prob, mask=_dev(torch, mask, torch.uint8))
    assert ctx.readout_terms() == TERMS[request.param]
    assert ctx.readout_cheb_terms() == CHEB_TERMS[request.param]
    ora = oracle_lib.epg(prob, th)
    v, w = I.probe_vectors(prob)
    yield dict(name=request.param, prob=prob, th=th, mask=mask, ctx=ctx, ora=ora, v=v, w=w, torch=torch)
    ctx.close()


def _products(c, oracle_lib, enc=0):
    """Errors of the residual, J v and the rows of Re(J^H w) against the oracle."""
    torch, ctx, prob, th, mask = c["torch"], c["ctx"], c["prob"], c["th"], c["mask"]
    ctx.set_encoding(enc)
    s = oracle_lib.signal(prob, th, c["ora"], mask=mask)
    n = I.unit_noise(prob)
    d = s + n * (np.linalg.norm(s) / (50.0 * np.linalg.norm(n)))
    th1 = th.copy()
    th1[0] += 0.05
    th1 = th1.astype(np.float32).astype(np.float64)
    f_ref, r_ref = oracle_lib.residual(prob, th1, d, mask=mask)
    f, r = ctx.residual(_dev(torch, th1, torch.float32), _dev(torch, d, torch.complex64))
    e_r = float(np.linalg.norm(r.cpu().numpy().astype(np.complex128) - r_ref) / np.linalg.norm(d))
    e_f = abs(f - f_ref) / (0.5 * np.vdot(d, d).real)
    thd = _dev(torch, th, torch.float32)
    ctx.linearise(thd)
    jv = ctx.jv(thd, _dev(torch, c["v"], torch.float32), reuse=True).cpu().numpy().astype(np.complex128)
    jhw = ctx.jhw(thd, _dev(torch, c["w"], torch.complex64), reuse=True).cpu().numpy().astype(np.float64)
    ctx.set_encoding(0)
    e_jv = _rel(jv, oracle_lib.jv(prob, th, c["ora"], c["v"], mask=mask))
    ref = oracle_lib.jhw(prob, th, c["ora"], c["w"], mask=mask)
    e_rows = [_rel(jhw[q], ref[q]) for q in range(5)]
    return e_r, e_f, e_jv, e_rows, jv, jhw


def test_products_match_oracle(case, oracle_lib):
    e_r, e_f, e_jv, e_rows, jv, jhw = _products(case, oracle_lib)
    print(f"  residual {e_r:.2e} f {e_f:.2e} jv {e_jv:.2e} jhw rows {['%.1e' % e for e in e_rows]}", flush=True)
    assert max([e_r, e_f, e_jv] + e_rows) <= TOL
    # the adjoint identity <w, J v> = v . Re(J^H w) on the GPU's own products,
    # to the rounding scale of the inner products (|w| |J v|: the two sides
    # can be small by cancellation)
    lhs = np.vdot(case["w"].reshape(-1), jv.reshape(-1)).real
    rhs = float(np.dot(case["v"].reshape(-1), jhw.reshape(-1)))
    assert abs(lhs - rhs) <= TOL * np.linalg.norm(case["w"]) * np.linalg.norm(jv)


@pytest.mark.parametrize("enc,bar", [(1, 1e-4)])
def test_split_bf16_x_stage(case, oracle_lib, enc, bar):
    if case["name"] not in ("small", "ragged"):
        pytest.skip("two cases suffice for the encoding variant")
    e_r, e_f, e_jv, e_rows, _, _ = _products(case, oracle_lib, enc)
    print(f"  [split-bf16] residual {e_r:.2e} jv {e_jv:.2e} jhw rows {['%.1e' % e for e in e_rows]}",
          flush=True)
    assert max([e_r, e_jv] + e_rows) <= bar


def test_fp16_trains(case, oracle_lib):
    if case["name"] != "ragged":
        pytest.skip("one case suffices for the storage variant")
    ctx = case["ctx"]
    ctx.set_train_precision(1)
    try:
        e_r, e_f, e_jv, e_rows, _, _ = _products(case, oracle_lib)
    finally:
        ctx.set_train_precision(0)
    print(f"  [fp16 trains] residual {e_r:.2e} jv {e_jv:.2e} jhw rows {['%.1e' % e for e in e_rows]}",
          flush=True)
    assert max([e_r, e_jv] + e_rows) <= 1e-3


def test_gn_and_tr_steps_match_oracle(torch_gpu, oracle_lib):
    """GN steps (B1 known and fitted) and a trust-region step from the same
    start: the line-search and CG decisions agree exactly, theta to 1e-5."""
    torch = torch_gpu
    from paper_1904_13244_amd.binding import Context
    prob, th_true, mask = _case("small")
    d = oracle_lib.signal(prob, th_true, oracle_lib.epg(prob, th_true, tangents=False), mask=mask)
    rng = np.random.default_rng(59)
    th0 = th_true.copy()
    th0[:2] += 0.05 * rng.standard_normal((2, prob.nv))
    th0[1] = np.maximum(th0[1], I.GN_LO[1] + 1e-3)
    th0 = th0.astype(np.float32).astype(np.float64)
    ctx = Context(prob, mask=_dev(torch, mask, torch.uint8))
    dd = _dev(torch, d, torch.complex64)
    for pm in (0b11011, 0b11111):
        th_o, rep_o = oracle_lib.gn_step(prob, th0, d, n_cg=10, param_mask=pm, lo=I.GN_LO, hi=I.GN_HI,
                                         mask=mask)
        th_g = _dev(torch, th0, torch.float32)
        rep = ctx.gn_step(th_g, dd, 10, pm, I.GN_LO, I.GN_HI)
        e = _rel(th_g.cpu().numpy().astype(np.float64), th_o)
        print(f"\n  [readout gn, mask {pm:#07b}] t {rep.t}/{rep_o.t} cg {rep.cg_iters}/{rep_o.cg_iters} "
              f"theta {e:.2e}", flush=True)
        assert rep.t == rep_o.t and rep.cg_iters == rep_o.cg_iters and e <= TOL
    th_o, do, rep_o = oracle_lib.tr_step(prob, th0, d, 1.0, 10, 0b11011, I.GN_LO, I.GN_HI, mask=mask)
    th_g = _dev(torch, th0, torch.float32)
    dg, rep = ctx.tr_step(th_g, dd, 1.0, 10, 0b11011, I.GN_LO, I.GN_HI)
    e = _rel(th_g.cpu().numpy().astype(np.float64), th_o)
    print(f"  [readout tr] exit {rep.exit_kind}/{rep_o['exit_kind']} cg {rep.cg_iters}/{rep_o['cg_iters']} "
          f"delta {dg:.4g}/{do:.4g} theta {e:.2e}", flush=True)
    assert rep.exit_kind == rep_o["exit_kind"] and rep.cg_iters == rep_o["cg_iters"] and dg == do
    assert e <= TOL
    ctx.close()


def test_rho_init_matches_oracle(torch_gpu, oracle_lib):
    torch = torch_gpu
    from paper_1904_13244_amd.binding import Context
    prob, th_true, mask = _case("ragged")
    d = oracle_lib.signal(prob, th_true, oracle_lib.epg(prob, th_true, tangents=False), mask=mask)
    th0 = th_true.copy()
    th0[3], th0[4] = 1.0, 0.0
    ref = oracle_lib.rho_init(prob, th0, d, n_iter=5, mask=mask)
    ctx = Context(prob, mask=_dev(torch, mask, torch.uint8))
    got = ctx.rho_init(_dev(torch, th0, torch.float32), _dev(torch, d, torch.complex64), n_iter=5)
    got = got.cpu().numpy().astype(np.float64)
    ctx.close()
    e = _rel(got[3:], ref[3:])
    print(f"\n  [readout rho init, 5 CGLS] rho {e:.2e}", flush=True)
    assert e <= TOL and np.array_equal(got[:3], th0[:3].astype(np.float32))


def test_short_readout_equals_the_static_model(torch_gpu):
    """dwell 1 ns and no off-resonance map: the factor is 1 to FP32 rounding,
    so the readout path's products equal the static path's (two different
    kernel chains) to 1e-6."""
    torch = torch_gpu
    from paper_1904_13244_amd.binding import Context
    prob, th, mask = _case("ragged")
    static = dataclasses.replace(prob, dwell=0.0, db0=None)
    short = dataclasses.replace(prob, dwell=1e-9, db0=None)
    md = _dev(torch, mask, torch.uint8)
    a, b = Context(static, mask=md), Context(short, mask=md)
    assert b.readout_terms() == 8
    thd = _dev(torch, th, torch.float32)
    v, w = I.probe_vectors(prob)
    vd, wd = _dev(torch, v, torch.float32), _dev(torch, w, torch.complex64)
    for ctx in (a, b):
        ctx.linearise(thd)
    outs = [(c.jv(thd, vd, reuse=True).cpu().numpy(), c.jhw(thd, wd, reuse=True).cpu().numpy()) for c in (a, b)]
    a.close()
    b.close()
    e_jv = _rel(outs[1][0].astype(np.complex128), outs[0][0].astype(np.complex128))
    e_jhw = _rel(outs[1][1].astype(np.float64), outs[0][1].astype(np.float64))
    print(f"\n  [1 ns readout vs static] jv {e_jv:.2e} jhw {e_jhw:.2e}", flush=True)
    assert max(e_jv, e_jhw) <= 1e-6


def test_t2_box_below_the_bound_is_refused(torch_gpu):
    torch = torch_gpu
    from paper_1904_13244_amd import binding as B
    from paper_1904_13244_amd.binding import Context
    prob, th, mask = _case("small")
    ctx = Context(prob)
    thd = _dev(torch, th, torch.float32)
    dd = torch.zeros(prob.data_shape, dtype=torch.complex64, device="cuda")
    lo = list(I.GN_LO)
    lo[1] = float(np.log(0.004))    # below rd_min_t2 = 5 ms
    for call in (lambda: ctx.gn_step(thd, dd, 5, 0b11011, lo, I.GN_HI),
                 lambda: ctx.tr_step(thd, dd, 1.0, 5, 0b11011, lo, I.GN_HI)):
        with pytest.raises(B.MrstatError) as e:
            call()
        assert e.value.status == B.ERR_ARG
    ctx.gn_step(thd, dd, 5, 0b11001, lo, I.GN_HI)   # ln T2 held fixed: the box is not used
    ctx.close()


@pytest.mark.parametrize("fit", [False, True])
def test_fullsize_sampled(torch_gpu, oracle_lib, fit):
    """224 x 224 phantom, 1120 TRs, 448 samples at 85.6 kHz (24 terms), a
    smooth off-resonance field of +-150 Hz (a map, or theta row 5 with Delta
    B0 fitted): the GPU runs the whole image's kernels with 160 voxels masked
    in; the oracle's direct sum covers those."""
    torch = torch_gpu
    from paper_1904_13244_amd.binding import Context
    w = I.config(3)
    p0 = w.problem
    yy, xx = np.meshgrid(np.linspace(-1, 1, p0.ny), np.linspace(-1, 1, p0.nx), indexing="ij")
    db0 = (150.0 * (0.6 * xx + 0.3 * yy * yy - 0.1 * xx * yy)).reshape(-1)
    prob = dataclasses.replace(p0, dwell=1 / BW, db0=db0)
    rng = np.random.default_rng(61)
    sel = np.sort(rng.choice(prob.nv, 160, replace=False))
    mask = np.zeros(prob.nv, np.uint8)
    mask[sel] = 1
    th = w.theta.copy()
    th[1, sel] = np.log(rng.uniform(0.01, 0.15, sel.size))
    if fit:
        unit = 1.0 / (2 * np.pi * prob.te)
        prob = dataclasses.replace(prob, db0=None, db0_unit=unit)
        th = np.vstack([th, (db0 / unit)[None, :]])
    th = th.astype(np.float32).astype(np.float64)
    # oracle trains on the masked-in voxels only (the others do not enter)
    sub = I.make_problem(sel.size, 1, prob.n_tr, sel.size, prob.n_states, tr=prob.tr, te=prob.te,
                         t_inv=prob.t_inv, flip_deg=prob.flip_deg, rf_phase=prob.rf_phase)
    ora = np.zeros((4, prob.n_tr, prob.nv), np.complex128)
    ora[:, :, sel] = oracle_lib.epg(sub, th[:5, sel])
    ctx = Context(prob, mask=_dev(torch, mask, torch.uint8))
    assert ctx.readout_terms() == 24 and ctx.readout_cheb_terms() == 16
    thd = _dev(torch, th, torch.float32)
    ctx.linearise(thd)
    got = ctx.simulate(thd).cpu().numpy().astype(np.float64)
    e_tr = max(_rel(got[p][:, sel], ora[p][:, sel].imag) for p in range(4))
    v, wv = I.probe_vectors(prob)
    s = oracle_lib.signal(prob, th, ora, mask=mask)
    zeros = torch.zeros(prob.data_shape, dtype=torch.complex64, device="cuda")
    _, r = ctx.residual(thd, zeros, reuse=True, want_f=False)   # r = 0 - s
    e_s = _rel(-r.cpu().numpy().astype(np.complex128), s)
    jv = ctx.jv(thd, _dev(torch, v, torch.float32), reuse=True).cpu().numpy().astype(np.complex128)
    e_jv = _rel(jv, oracle_lib.jv(prob, th, ora, v, mask=mask))
    jhw = ctx.jhw(thd, _dev(torch, wv, torch.complex64), reuse=True).cpu().numpy().astype(np.float64)
    ref = oracle_lib.jhw(prob, th, ora, wv, mask=mask)
    e_rows = [_rel(jhw[q][sel], ref[q][sel]) for q in range(th.shape[0])]
    zero_out = float(np.abs(jhw[:, mask == 0]).max())
    ctx.close()
    print(f"\n  [readout 224x224x1120, 448 samples, 160 voxels, Delta B0 {'fitted' if fit else 'map'}] "
          f"trains {e_tr:.1e} signal {e_s:.1e} "
          f"jv {e_jv:.1e} jhw rows {['%.1e' % e for e in e_rows]}", flush=True)
    assert max([e_tr, e_s, e_jv] + e_rows) <= TOL and zero_out == 0.0


# --------------------------------------------------------------------------
# Delta B0 fitted as the sixth parameter (mrstat_fit_db0): theta row 5 times
# db0_unit Hz, here db0_unit = 1 / (2 pi TE), so that row 5 is the
# off-resonance phase at the echo in radians.

def _fit_case(name):
    prob, th, mask = _case(name)
    unit = 1.0 / (2 * np.pi * prob.te)
    fit = dataclasses.replace(prob, db0=None, db0_unit=unit)
    th6 = np.vstack([th, (prob.db0 / unit)[None, :]]).astype(np.float32).astype(np.float64)
    return fit, th6, mask


@pytest.mark.parametrize("name", ["small", "ragged", "quarter_bandwidth"])
def test_fitted_offresonance_products(torch_gpu, oracle_lib, name):
    torch = torch_gpu
    from paper_1904_13244_amd.binding import Context
    prob, th, mask = _fit_case(name)
    ctx = Context(prob, mask=_dev(torch, mask, torch.uint8))
    assert ctx.np == 6
    ora = oracle_lib.epg(prob, th)
    s = oracle_lib.signal(prob, th, ora, mask=mask)
    n = I.unit_noise(prob)
    d = s + n * (np.linalg.norm(s) / (50.0 * np.linalg.norm(n)))
    th1 = th.copy()
    th1[5] += 0.2
    th1 = th1.astype(np.float32).astype(np.float64)
    f_ref, r_ref = oracle_lib.residual(prob, th1, d, mask=mask)
    f, r = ctx.residual(_dev(torch, th1, torch.float32), _dev(torch, d, torch.complex64))
    e_r = float(np.linalg.norm(r.cpu().numpy().astype(np.complex128) - r_ref) / np.linalg.norm(d))
    v, w = I.probe_vectors(prob)
    thd = _dev(torch, th, torch.float32)
    ctx.linearise(thd)
    jv = ctx.jv(thd, _dev(torch, v, torch.float32), reuse=True).cpu().numpy().astype(np.complex128)
    jhw = ctx.jhw(thd, _dev(torch, w, torch.complex64), reuse=True).cpu().numpy().astype(np.float64)
    ctx.close()
    e_jv = _rel(jv, oracle_lib.jv(prob, th, ora, v, mask=mask))
    ref = oracle_lib.jhw(prob, th, ora, w, mask=mask)
    e_rows = [_rel(jhw[q], ref[q]) for q in range(6)]
    print(f"\n  [Delta B0 fitted, {name}] residual {e_r:.2e} jv {e_jv:.2e} "
          f"jhw rows {['%.1e' % e for e in e_rows]}", flush=True)
    assert max([e_r, e_jv] + e_rows) <= TOL
    lhs = np.vdot(w.reshape(-1), jv.reshape(-1)).real   # adjoint identity, scale |w| |J v|
    rhs = float(np.dot(v.reshape(-1), jhw.reshape(-1)))
    assert abs(lhs - rhs) <= TOL * np.linalg.norm(w) * np.linalg.norm(jv)


def test_fitted_offresonance_steps_match_oracle(torch_gpu, oracle_lib):
    """GN steps with Delta B0 fitted (B1 known, then fitted), a trust-region
    step and the rho initialisation, from the same start as the oracle."""
    torch = torch_gpu
    from paper_1904_13244_amd.binding import Context
    prob, th_true, mask = _fit_case("small")
    d = oracle_lib.signal(prob, th_true, oracle_lib.epg(prob, th_true, tangents=False), mask=mask)
    rng = np.random.default_rng(63)
    th0 = th_true.copy()
    th0[:2] += 0.05 * rng.standard_normal((2, prob.nv))
    th0[5] += 0.3 * rng.standard_normal(prob.nv)
    th0 = th0.astype(np.float32).astype(np.float64)
    ctx = Context(prob, mask=_dev(torch, mask, torch.uint8))
    dd = _dev(torch, d, torch.complex64)
    for pm in (0b111011, 0b111111, 0b100000):
        th_o, rep_o = oracle_lib.gn_step(prob, th0, d, n_cg=10, param_mask=pm, lo=I.GN_LO, hi=I.GN_HI,
                                         mask=mask)
        th_g = _dev(torch, th0, torch.float32)
        rep = ctx.gn_step(th_g, dd, 10, pm, I.GN_LO, I.GN_HI)
        e = _rel(th_g.cpu().numpy().astype(np.float64), th_o)
        print(f"\n  [Delta B0 fitted gn, mask {pm:#08b}] t {rep.t}/{rep_o.t} cg {rep.cg_iters}/{rep_o.cg_iters} "
              f"theta {e:.2e}", flush=True)
        assert rep.t == rep_o.t and rep.cg_iters == rep_o.cg_iters and e <= TOL
    th_o, do, rep_o = oracle_lib.tr_step(prob, th0, d, 1.0, 10, 0b111011, I.GN_LO, I.GN_HI, mask=mask)
    th_g = _dev(torch, th0, torch.float32)
    dg, rep = ctx.tr_step(th_g, dd, 1.0, 10, 0b111011, I.GN_LO, I.GN_HI)
    e = _rel(th_g.cpu().numpy().astype(np.float64), th_o)
    print(f"  [Delta B0 fitted tr] exit {rep.exit_kind}/{rep_o['exit_kind']} cg {rep.cg_iters}/{rep_o['cg_iters']} "
          f"refl {rep.n_reflected}/{rep_o['n_reflected']} delta {dg:.4g}/{do:.4g} theta {e:.2e}", flush=True)
    assert rep.exit_kind == rep_o["exit_kind"] and rep.cg_iters == rep_o["cg_iters"] and dg == do
    assert rep.n_reflected == rep_o["n_reflected"] and e <= TOL
    ref = oracle_lib.rho_init(prob, th0, d, n_iter=5, mask=mask)
    got = ctx.rho_init(_dev(torch, th0, torch.float32), dd, n_iter=5).cpu().numpy().astype(np.float64)
    e = _rel(got[3:5], ref[3:5])
    print(f"  [Delta B0 fitted rho init] {e:.2e}", flush=True)
    assert e <= TOL and np.array_equal(got[[0, 1, 2, 5]], th0[[0, 1, 2, 5]])
    ctx.close()


def test_fitted_offresonance_box(torch_gpu, oracle_lib):
    """A step that would leave +-rd_max_db0 Hz is projected (line search) or
    reflected (trust region) at the same entries as by the oracle."""
    torch = torch_gpu
    from paper_1904_13244_amd.binding import Context
    prob, th_true, mask = _fit_case("small")
    tight = dataclasses.replace(prob, rd_max_db0=30.0)   # below part of the truth
    lim = 50.0 / prob.db0_unit
    th_true[5] = np.clip(th_true[5], -lim, lim).astype(np.float32)
    d = oracle_lib.signal(tight, th_true, oracle_lib.epg(tight, th_true, tangents=False), mask=mask)
    th0 = th_true.copy()
    th0[5] = 0.0
    ctx = Context(tight, mask=_dev(torch, mask, torch.uint8))
    dd = _dev(torch, d, torch.complex64)
    th_o, rep_o = oracle_lib.gn_step(tight, th0, d, n_cg=20, param_mask=0b100000, lo=I.GN_LO, hi=I.GN_HI,
                                     mask=mask)
    th_g = _dev(torch, th0, torch.float32)
    rep = ctx.gn_step(th_g, dd, 20, 0b100000, I.GN_LO, I.GN_HI)
    g = th_g.cpu().numpy().astype(np.float64)
    at_wall_o = np.abs(np.abs(th_o[5]) * prob.db0_unit - 30.0) <= 1e-3
    at_wall_g = np.abs(np.abs(g[5]) * prob.db0_unit - 30.0) <= 1e-3
    print(f"\n  [Delta B0 box, gn] t {rep.t}/{rep_o.t} at the wall {at_wall_g.sum()}/{at_wall_o.sum()} "
          f"theta {_rel(g, th_o):.2e}", flush=True)
    assert at_wall_o.sum() > 0
    assert rep.t == rep_o.t and np.array_equal(at_wall_g, at_wall_o) and _rel(g, th_o) <= TOL
    assert np.all(np.abs(g[5]) * prob.db0_unit <= 30.0 * (1 + 1e-6))
    th_o, do, rep_o = oracle_lib.tr_step(tight, th0, d, 8.0, 20, 0b100000, I.GN_LO, I.GN_HI, delta_max=8.0,
                                         mask=mask)
    th_g = _dev(torch, th0, torch.float32)
    dg, rep = ctx.tr_step(th_g, dd, 8.0, 20, 0b100000, I.GN_LO, I.GN_HI, delta_max=8.0)
    print(f"  [Delta B0 box, tr] reflected {rep.n_reflected}/{rep_o['n_reflected']} exit "
          f"{rep.exit_kind}/{rep_o['exit_kind']}", flush=True)
    assert rep_o["n_reflected"] > 0
    assert rep.n_reflected == rep_o["n_reflected"] and rep.exit_kind == rep_o["exit_kind"]
    assert _rel(th_g.cpu().numpy().astype(np.float64), th_o) <= TOL
    ctx.close()


def test_bit5_needs_the_fit(torch_gpu):
    torch = torch_gpu
    from paper_1904_13244_amd import binding as B
    from paper_1904_13244_amd.binding import Context
    prob, th, mask = _case("small")
    ctx = Context(prob)
    thd = _dev(torch, th, torch.float32)
    dd = torch.zeros(prob.data_shape, dtype=torch.complex64, device="cuda")
    with pytest.raises(B.MrstatError) as e:
        ctx.gn_step(thd, dd, 5, 0b111011, I.GN_LO, I.GN_HI)
    assert e.value.status == B.ERR_ARG
    ctx.close()


def _coil_case(seed=71):
    """24 x 20 image, 3 coils (Gaussian sensitivities with linear phases), 50
    TRs of 64 samples at 85.6 kHz (12 terms), 80 % mask."""
    rng = np.random.default_rng(seed)
    prob = I.make_problem(24, 20, 50, 64, 8, n_coils=3, tr=0.008, te=0.004, flip_deg=I.flips_sin2_sweeps(50, 20),
                          ky_line=rng.integers(0, 20, 50))
    prob = dataclasses.replace(prob, dwell=1 / BW, db0=rng.uniform(-150.0, 150.0, prob.nv))
    th = _maps(prob, rng, seed + 1)
    mask = (rng.uniform(size=prob.nv) > 0.2).astype(np.uint8)
    return prob, th, mask, I.coil_maps(24, 20, 3)


@pytest.mark.parametrize("fit", [False, True])
def test_coils_products_steps_and_rho_init(torch_gpu, oracle_lib, fit):
    torch = torch_gpu
    from paper_1904_13244_amd.binding import Context
    prob, th, mask, coil = _coil_case()
    if fit:
        unit = 1.0 / (2 * np.pi * prob.te)
        th = np.vstack([th, (prob.db0 / unit)[None, :]]).astype(np.float32).astype(np.float64)
        prob = dataclasses.replace(prob, db0=None, db0_unit=unit)
    ctx = Context(prob, coil=_dev(torch, coil, torch.complex64), mask=_dev(torch, mask, torch.uint8))
    assert ctx.readout_terms() == 12 and ctx.readout_cheb_terms() == 8
    ora = oracle_lib.epg(prob, th)
    s = oracle_lib.signal(prob, th, ora, coil=coil, mask=mask)
    n = I.unit_noise(prob)
    d = s + n * (np.linalg.norm(s) / (50.0 * np.linalg.norm(n)))
    th1 = th.copy()
    th1[0] += 0.05
    th1 = th1.astype(np.float32).astype(np.float64)
    _, r_ref = oracle_lib.residual(prob, th1, d, coil=coil, mask=mask)
    dd = _dev(torch, d, torch.complex64)
    _, r = ctx.residual(_dev(torch, th1, torch.float32), dd)
    e_r = float(np.linalg.norm(r.cpu().numpy().astype(np.complex128) - r_ref) / np.linalg.norm(d))
    v, w = I.probe_vectors(prob)
    thd = _dev(torch, th, torch.float32)
    ctx.linearise(thd)
    jv = ctx.jv(thd, _dev(torch, v, torch.float32), reuse=True).cpu().numpy().astype(np.complex128)
    jhw = ctx.jhw(thd, _dev(torch, w, torch.complex64), reuse=True).cpu().numpy().astype(np.float64)
    e_jv = _rel(jv, oracle_lib.jv(prob, th, ora, v, coil=coil, mask=mask))
    ref = oracle_lib.jhw(prob, th, ora, w, coil=coil, mask=mask)
    e_rows = [_rel(jhw[q], ref[q]) for q in range(th.shape[0])]
    print(f"\n  [readout, 3 coils, Delta B0 {'fitted' if fit else 'map'}] residual {e_r:.2e} jv {e_jv:.2e} "
          f"jhw rows {['%.1e' % e for e in e_rows]}", flush=True)
    assert max([e_r, e_jv] + e_rows) <= TOL
    # one GN step from a perturbed start, and the rho initialisation
    rng = np.random.default_rng(72)
    th0 = th.copy()
    th0[:2] += 0.05 * rng.standard_normal((2, prob.nv))
    th0 = th0.astype(np.float32).astype(np.float64)
    pm = 0b111011 if fit else 0b11011
    th_o, rep_o = oracle_lib.gn_step(prob, th0, d, n_cg=10, param_mask=pm, lo=I.GN_LO, hi=I.GN_HI,
                                     coil=coil, mask=mask)
    th_g = _dev(torch, th0, torch.float32)
    rep = ctx.gn_step(th_g, dd, 10, pm, I.GN_LO, I.GN_HI)
    e = _rel(th_g.cpu().numpy().astype(np.float64), th_o)
    ref = oracle_lib.rho_init(prob, th0, d, n_iter=5, coil=coil, mask=mask)
    got = ctx.rho_init(_dev(torch, th0, torch.float32), dd, n_iter=5).cpu().numpy().astype(np.float64)
    e_rho = _rel(got[3:5], ref[3:5])
    ctx.close()
    print(f"  [gn] t {rep.t}/{rep_o.t} cg {rep.cg_iters}/{rep_o.cg_iters} theta {e:.2e}; rho init {e_rho:.2e}",
          flush=True)
    assert rep.t == rep_o.t and rep.cg_iters == rep_o.cg_iters and e <= TOL and e_rho <= TOL


def test_expansion_at_its_bounds(torch_gpu, oracle_lib):
    """T2 = 5 ms in every voxel and |Delta B0| = 200 Hz (the context's bounds)
    over a 448-sample readout at 85.6 kHz (|lambda| tau_max = 3.8, 24 terms):
    the products still meet the plain path's bar against the oracle."""
    torch = torch_gpu
    from paper_1904_13244_amd.binding import Context
    rng = np.random.default_rng(81)
    prob = I.make_problem(32, 16, 40, 448, 8, tr=0.008, te=0.004, flip_deg=I.flips_sin2_sweeps(40, 16),
                          ky_line=rng.integers(0, 16, 40))
    db0 = np.where(rng.uniform(size=prob.nv) < 0.5, -200.0, 200.0)
    prob = dataclasses.replace(prob, dwell=1 / BW, db0=db0)
    th = I.iid_maps(prob.nv, seed=82, b1=rng.uniform(0.8, 1.2, prob.nv))
    th[1] = np.log(0.005)
    th = th.astype(np.float32).astype(np.float64)
    ctx = Context(prob)
    assert ctx.readout_terms() == 24 and ctx.readout_cheb_terms() == 16
    ora = oracle_lib.epg(prob, th)
    s = oracle_lib.signal(prob, th, ora)
    zeros = torch.zeros(prob.data_shape, dtype=torch.complex64, device="cuda")
    thd = _dev(torch, th, torch.float32)
    _, r = ctx.residual(thd, zeros)
    e_s = _rel(-r.cpu().numpy().astype(np.complex128), s)
    v, w = I.probe_vectors(prob)
    jv = ctx.jv(thd, _dev(torch, v, torch.float32), reuse=True).cpu().numpy().astype(np.complex128)
    jhw = ctx.jhw(thd, _dev(torch, w, torch.complex64), reuse=True).cpu().numpy().astype(np.float64)
    ctx.close()
    e_jv = _rel(jv, oracle_lib.jv(prob, th, ora, v))
    ref = oracle_lib.jhw(prob, th, ora, w)
    e_rows = [_rel(jhw[q], ref[q]) for q in range(5)]
    print(f"\n  [expansion at its bounds] signal {e_s:.2e} jv {e_jv:.2e} jhw rows {['%.1e' % e for e in e_rows]}",
          flush=True)
    assert max([e_s, e_jv] + e_rows) <= TOL


def test_balanced_isochromat_model_with_readout_decay(torch_gpu, oracle_lib):
    """The balanced isochromat model (11 isochromats, RF phases 0 / pi) with T2
    decay during each readout (no off-resonance map: the balanced model takes
    none): products against the oracle's model."""
    torch = torch_gpu
    from paper_1904_13244_amd.binding import Context
    rng = np.random.default_rng(91)
    T, ny = 60, 18
    prob = I.make_problem(20, ny, T, 64, 8, tr=0.008, te=0.004, t_inv=0.01, rf_phase=I.balanced_phases(T),
                          flip_deg=I.flips_sin2_sweeps(T, ny), ky_line=rng.integers(0, ny, T))
    prob = dataclasses.replace(prob, iso=I.slice_profile_gaussian(11), dwell=4 / BW)
    th = _maps(prob, rng, 92)
    ctx = Context(prob)
    ora = oracle_lib.epg(prob, th)
    thd = _dev(torch, th, torch.float32)
    zeros = torch.zeros(prob.data_shape, dtype=torch.complex64, device="cuda")
    _, r = ctx.residual(thd, zeros)
    e_s = _rel(-r.cpu().numpy().astype(np.complex128), oracle_lib.signal(prob, th, ora))
    v, w = I.probe_vectors(prob)
    jv = ctx.jv(thd, _dev(torch, v, torch.float32), reuse=True).cpu().numpy().astype(np.complex128)
    jhw = ctx.jhw(thd, _dev(torch, w, torch.complex64), reuse=True).cpu().numpy().astype(np.float64)
    ctx.close()
    e_jv = _rel(jv, oracle_lib.jv(prob, th, ora, v))
    ref = oracle_lib.jhw(prob, th, ora, w)
    e_rows = [_rel(jhw[q], ref[q]) for q in range(5)]
    print(f"\n  [balanced model + readout decay] signal {e_s:.2e} jv {e_jv:.2e} "
          f"jhw rows {['%.1e' % e for e in e_rows]}", flush=True)
    assert max([e_s, e_jv] + e_rows) <= TOL
