"""Non-Cartesian encoding on the GPU (mrstat_create_traj: the voxel x sample
contraction on the matrix cores with phases generated on the fly) against the
FP64 oracle's direct sums (pinned in tests/test_oracle_noncartesian.py).

Sizes span several tiles and a ragged tail in every tiled dimension: 100
samples (two 64-sample tiles of the forward), 70 image rows (three 32-row LDS
tiles of the forward, two 64-row tiles of the adjoint), 36 columns (two
32-column adjoint tiles; 36 of 48 padded columns in the forward's K), several
TR chunks. Bars: FP32 1e-5 relative (the plain path's target); split-BF16
1e-4 (each operand rounded to about 2^-16); FP16 train storage 1e-3.
"""
import dataclasses

import numpy as np
import pytest

from paper_1904_13244_amd import inputs as I

pytestmark = pytest.mark.gpu

BAR = {0: 1e-5, 1: 1e-4}


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


def _radial_case(coils=1, seed=31, nx=36, ny=70, n_tr=40, n_read=100):
    rng = np.random.default_rng(seed)
    prob = I.make_problem(nx, ny, n_tr, n_read, 8, n_coils=coils, flip_deg=rng.uniform(5, 60, n_tr))
    prob = dataclasses.replace(prob, traj=I.radial_golden(n_tr, n_read, nx, ny))
    th = I.iid_maps(prob.nv, seed=seed, b1=rng.uniform(0.8, 1.2, prob.nv))
    th = th.astype(np.float32).astype(np.float64)
    coil = I.coil_maps(nx, ny, coils) if coils > 1 else None
    mask = (rng.uniform(size=prob.nv) > 0.15).astype(np.uint8)
    return prob, th, coil, mask


@pytest.mark.parametrize("coils", [1, 3])
@pytest.mark.parametrize("enc", [0, 1])
def test_products_match_oracle(torch_gpu, oracle_lib, enc, coils):
    torch = torch_gpu
    from paper_1904_13244_amd.binding import Context
    prob, th, coil, mask = _radial_case(coils)
    ora = oracle_lib.epg(prob, th)
    v, w = I.probe_vectors(prob)
    kw = dict(coil=None if coil is None else _dev(torch, coil, torch.complex64),
              mask=_dev(torch, mask, torch.uint8))
    ctx = Context(prob, **kw)
    ctx.set_encoding(enc)
    thd = _dev(torch, th, torch.float32)
    d = oracle_lib.signal(prob, th, ora, coil=coil, mask=mask)
    th1 = th.copy()
    th1[0] += 0.05
    th1 = th1.astype(np.float32).astype(np.float64)
    f_ref, r_ref = oracle_lib.residual(prob, th1, d, coil=coil, mask=mask)
    f, r = ctx.residual(_dev(torch, th1, torch.float32), _dev(torch, d, torch.complex64))
    e_r = float(np.linalg.norm(r.cpu().numpy() - r_ref) / np.linalg.norm(d))
    ctx.linearise(thd)
    jv = ctx.jv(thd, _dev(torch, v, torch.float32), reuse=True).cpu().numpy().astype(np.complex128)
    jhw = ctx.jhw(thd, _dev(torch, w, torch.complex64), reuse=True).cpu().numpy().astype(np.float64)
    e_jv = _rel(jv, oracle_lib.jv(prob, th, ora, v, coil=coil, mask=mask))
    e_jhw = _rel(jhw, oracle_lib.jhw(prob, th, ora, w, coil=coil, mask=mask))
    e_f = abs(f - f_ref) / (0.5 * np.vdot(d, d).real)   # as the residual: relative to the data
    ctx.close()
    print(f"\n  [radial enc {enc}, {coils} coil(s)] residual/||d|| {e_r:.2e} f {e_f:.2e} jv {e_jv:.2e} "
          f"jhw {e_jhw:.2e}", flush=True)
    for e in (e_r, e_jv, e_jhw, e_f):
        assert e <= BAR[enc]


@pytest.mark.parametrize("enc,coils", [(0, 1), (1, 2)])
def test_wide_image_k_parts(torch_gpu, oracle_lib, enc, coils):
    """An image wider than one K part of the forward (200 columns: parts of
    64, 64, 64 and 8), 9 rows (less than one staged row tile), 11 TRs (not a
    multiple of the 8 TRs dealt per XCD) and 70 samples (a ragged sample
    tile): products and residual against the oracle's direct sums."""
    torch = torch_gpu
    from paper_1904_13244_amd.binding import Context
    prob, th, coil, mask = _radial_case(coils, seed=37, nx=200, ny=9, n_tr=11, n_read=70)
    ora = oracle_lib.epg(prob, th)
    v, w = I.probe_vectors(prob)
    ctx = Context(prob, coil=None if coil is None else _dev(torch, coil, torch.complex64),
                  mask=_dev(torch, mask, torch.uint8))
    ctx.set_encoding(enc)
    thd = _dev(torch, th, torch.float32)
    d = oracle_lib.signal(prob, th, ora, coil=coil, mask=mask)
    f_ref, r_ref = oracle_lib.residual(prob, th, 0.5 * d, coil=coil, mask=mask)
    f, r = ctx.residual(thd, _dev(torch, 0.5 * d, torch.complex64))
    e_r = float(np.linalg.norm(r.cpu().numpy() - r_ref) / np.linalg.norm(d))
    ctx.linearise(thd)
    jv = ctx.jv(thd, _dev(torch, v, torch.float32), reuse=True).cpu().numpy().astype(np.complex128)
    jhw = ctx.jhw(thd, _dev(torch, w, torch.complex64), reuse=True).cpu().numpy().astype(np.float64)
    e_jv = _rel(jv, oracle_lib.jv(prob, th, ora, v, coil=coil, mask=mask))
    e_jhw = _rel(jhw, oracle_lib.jhw(prob, th, ora, w, coil=coil, mask=mask))
    ctx.close()
    print(f"\n  [radial 200x9, enc {enc}, {coils} coil(s)] residual {e_r:.2e} jv {e_jv:.2e} jhw {e_jhw:.2e}",
          flush=True)
    for e in (e_r, e_jv, e_jhw):
        assert e <= BAR[enc]


def test_fp16_trains(torch_gpu, oracle_lib):
    torch = torch_gpu
    from paper_1904_13244_amd import binding as B
    from paper_1904_13244_amd.binding import Context
    prob, th, _, mask = _radial_case(seed=33)
    ora = oracle_lib.epg(prob, th)
    v, w = I.probe_vectors(prob)
    ctx = Context(prob, mask=_dev(torch, mask, torch.uint8))
    ctx.set_train_precision(B.TRAINS_FP16)
    ctx.set_encoding(B.ENC_SPLIT_BF16)
    thd = _dev(torch, th, torch.float32)
    ctx.linearise(thd)
    jv = ctx.jv(thd, _dev(torch, v, torch.float32), reuse=True).cpu().numpy().astype(np.complex128)
    jhw = ctx.jhw(thd, _dev(torch, w, torch.complex64), reuse=True).cpu().numpy().astype(np.float64)
    e_jv = _rel(jv, oracle_lib.jv(prob, th, ora, v, mask=mask))
    e_jhw = _rel(jhw, oracle_lib.jhw(prob, th, ora, w, mask=mask))
    with pytest.raises(B.MrstatError) as e:
        ctx.set_encoding(B.ENC_FP16)
    assert e.value.status == B.ERR_UNSUPPORTED
    ctx.close()
    print(f"\n  [radial FP16 trains, split-BF16] jv {e_jv:.2e} jhw {e_jhw:.2e}", flush=True)
    assert max(e_jv, e_jhw) <= 1e-3


def test_cartesian_trajectory_matches_cartesian_kernels(torch_gpu):
    """The same problem through the Cartesian kernels (y-stage + x-GEMM) and
    through the non-Cartesian contraction on the Cartesian trajectory."""
    torch = torch_gpu
    from paper_1904_13244_amd.binding import Context
    rng = np.random.default_rng(35)
    prob = I.make_problem(24, 40, 48, 48, 8, flip_deg=rng.uniform(5, 60, 48),
                          ky_line=rng.integers(0, 40, 48))
    nprob = dataclasses.replace(prob, traj=I.cartesian_traj(prob))
    th = _dev(torch, I.iid_maps(prob.nv, seed=36), torch.float32)
    v, w = I.probe_vectors(prob)
    vd, wd = _dev(torch, v, torch.float32), _dev(torch, w, torch.complex64)
    out = []
    for pb in (prob, nprob):
        c = Context(pb)
        out.append((c.jv(th, vd).cpu().numpy(), c.jhw(th, wd).cpu().numpy()))
        c.close()
    e1, e2 = _rel(out[1][0], out[0][0]), _rel(out[1][1], out[0][1])
    print(f"\n  [Cartesian trajectory] jv {e1:.2e} jhw {e2:.2e}", flush=True)
    assert max(e1, e2) <= 1e-5


@pytest.mark.parametrize("param_mask", [0b11011, 0b11111])
def test_gn_and_tr_steps_match_oracle(torch_gpu, oracle_lib, param_mask):
    torch = torch_gpu
    from paper_1904_13244_amd.binding import Context
    prob, th_true, _, mask = _radial_case(seed=37, nx=20, ny=18, n_tr=64, n_read=40)
    d = oracle_lib.signal(prob, th_true, oracle_lib.epg(prob, th_true, tangents=False), mask=mask)
    rng = np.random.default_rng(38)
    th0 = th_true.copy()
    th0[:2] += 0.1 * rng.standard_normal((2, prob.nv))
    th0 = th0.astype(np.float32).astype(np.float64)
    ctx = Context(prob, mask=_dev(torch, mask, torch.uint8))
    dd = _dev(torch, d, torch.complex64)
    th_o = th0.copy()
    th_g = _dev(torch, th0, torch.float32)
    for it in range(3):
        th_o, rep_o = oracle_lib.gn_step(prob, th_o, d, n_cg=8, param_mask=param_mask, lo=I.GN_LO, hi=I.GN_HI,
                                         mask=mask)
        rep = ctx.gn_step(th_g, dd, 8, param_mask, I.GN_LO, I.GN_HI)
        e = _rel(th_g.cpu().numpy().astype(np.float64), th_o)
        print(f"  [radial gn it {it}] t {rep.t}/{rep_o.t} cg {rep.cg_iters}/{rep_o.cg_iters} theta {e:.2e}",
              flush=True)
        assert rep.t == rep_o.t and rep.cg_iters == rep_o.cg_iters and e <= 1e-5
    delta = 0.5 * float(np.linalg.norm(th_o - th0))
    th_o2, d_o, rep_o = oracle_lib.tr_step(prob, th0, d, delta, 8, param_mask, I.GN_LO, I.GN_HI, mask=mask)
    th_g2 = _dev(torch, th0, torch.float32)
    d_g, rep = ctx.tr_step(th_g2, dd, delta, 8, param_mask, I.GN_LO, I.GN_HI)
    e = _rel(th_g2.cpu().numpy().astype(np.float64), th_o2)
    print(f"  [radial tr] exit {rep.exit_kind}/{rep_o['exit_kind']} cg {rep.cg_iters}/{rep_o['cg_iters']} "
          f"delta {d_g}/{d_o} theta {e:.2e}", flush=True)
    assert rep.exit_kind == rep_o["exit_kind"] and rep.cg_iters == rep_o["cg_iters"] and d_g == d_o
    assert e <= 1e-5
    # rho initialisation (CGLS) on the same context. The radial rho system is
    # ill-conditioned (cond M about 800: the spokes oversample the k-space
    # centre), and CGLS amplifies the products' FP32 rounding as it
    # iterates: CGLS on the explicit M in complex64 differs from complex128
    # by 5e-7 after 5 iterations and 2.1e-4 after 10 (objective 2e-8 and
    # 6e-6). The 1e-5 bar holds at 5; at 10 the bars are five times the
    # emulation's figures, rounded up (rho 1e-3, objective 5e-5).
    th_init = I.initial_theta(prob.nv)
    for n_it in (5, 10):
        ref = oracle_lib.rho_init(prob, th_init, d, n_iter=n_it, mask=mask)
        got = ctx.rho_init(_dev(torch, th_init, torch.float32), dd, n_it).cpu().numpy().astype(np.float64)
        e_rho = _rel(got[3:], ref[3:])
        f_ref, _ = oracle_lib.residual(prob, ref, d, mask=mask)
        f_got, _ = oracle_lib.residual(prob, got, d, mask=mask)
        e_f = abs(f_got - f_ref) / f_ref
        print(f"  [radial rho init, {n_it} iterations] rho {e_rho:.2e} objective {e_f:.2e}", flush=True)
        bar_rho, bar_f = (1e-5, 1e-5) if n_it == 5 else (1e-3, 5e-5)
        assert e_rho <= bar_rho and e_f <= bar_f
    ctx.close()
