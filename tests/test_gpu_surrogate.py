"""The learned surrogate inside the hot path (through the C ABI).

With a surrogate set, a context's linearisation takes the network's trains
for voxels inside its box and the EPG's for the others. Expected values come
from the oracle: the FP64 network (oracle/mlp.py, same BF16-rounded weights)
for in-box voxels, the FP64 EPG for out-of-box ones, and the oracle's
separable signal and Jacobian products applied to those composed trains.
Tolerances: 1e-5 normwise where the EPG decides (the plain path's bar),
2e-2 where the network does (its BF16 activations; derivation in
tests/test_gpu_mlp.py).
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


def _dev(torch, a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype).contiguous()


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _bf16(x):
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _in_box(th):
    lo, hi = np.array(I.SURR_LO, np.float32), np.array(I.SURR_HI, np.float32)
    t = th[:3].astype(np.float32)
    return np.all((t >= lo[:, None]) & (t <= hi[:, None]), axis=0)


@pytest.fixture(scope="module")
def setup(torch_gpu, oracle_lib):
    torch = torch_gpu
    from oracle import mlp as M
    from paper_1904_13244_amd.binding import Context, Surrogate
    rng = np.random.default_rng(61)
    n_tr, width, depth, batch = 64, 64, 2, 128
    prob = I.make_problem(24, 20, n_tr, 32, 16, flip_deg=I.flips_sin2_sweeps(n_tr, 20))
    nv = prob.nv
    th = I.iid_maps(nv, seed=62, b1=rng.uniform(0.8, 1.2, nv))
    # About one voxel in six leaves the box, in each of the three inputs.
    out = rng.choice(nv, nv // 6, replace=False)
    for k, j in enumerate(out):
        q = k % 3
        th[q, j] = [np.log(6.5), np.log(0.006), 1.45][q]
    mask = (rng.uniform(size=nv) > 0.15).astype(np.uint8)
    th = th.astype(np.float32).astype(np.float64)

    flat = I.mlp_init_params(n_tr, width, depth, seed=63).astype(np.float32)
    scale = np.array([0.2, 0.15, 0.05, 0.3], dtype=np.float32)
    net = Surrogate(n_tr, width, depth, batch)
    net.set_scaling(I.SURR_LO, I.SURR_HI, scale)
    net.set_params(torch.from_numpy(flat).cuda())
    ctx = Context(prob, mask=_dev(torch, mask, torch.uint8))
    ctx.set_surrogate(net)

    # Oracle trains: the FP64 network inside the box (and for masked-out
    # voxels, whose trains nothing reads), the FP64 EPG for the fallbacks.
    parts = M.unpack(flat.astype(np.float64), n_tr, width, depth)
    for l in range(1, depth + 1):
        parts[2 * l] = _bf16(parts[2 * l])
    w_ora = np.concatenate([p.reshape(-1) for p in parts])
    x = M.normalise_inputs(th[:3], I.SURR_LO, I.SURR_HI)
    y, _ = M.forward(w_ora, x, n_tr, width, depth)
    net_tr = y[4 * n_tr:].reshape(4, n_tr, nv) * scale.astype(np.float64)[:, None, None]
    fb = (~_in_box(th)) & (mask != 0)
    epg = oracle_lib.epg(prob, th).imag
    ref = np.where(fb[None, None, :], epg, net_tr)
    yield dict(torch=torch, prob=prob, th=th, mask=mask, ctx=ctx, net=net, ref=ref, fb=fb)
    ctx.close()
    net.close()


def test_trains_route_out_of_box_voxels_to_the_epg(setup):
    torch, ctx, th, ref, fb = (setup[k] for k in ("torch", "ctx", "th", "ref", "fb"))
    got = ctx.simulate(_dev(torch, th, torch.float32)).cpu().numpy().astype(np.float64)
    n = ctx.fallback_count()
    print(f"\n[surrogate] fallback voxels {n} (host count {int(fb.sum())})", flush=True)
    assert n == int(fb.sum()) and n > 0
    for p in range(4):
        e_fb = _rel(got[p][:, fb], ref[p][:, fb])
        e_in = _rel(got[p][:, ~fb], ref[p][:, ~fb])
        print(f"  train {p}: EPG fallback rel {e_fb:.2e}, network rel {e_in:.2e}", flush=True)
        assert e_fb <= 1e-5
        assert e_in <= 2e-2


def test_products_on_surrogate_trains(setup, oracle_lib):
    torch, ctx, prob, th, ref, mask = (setup[k] for k in ("torch", "ctx", "prob", "th", "ref", "mask"))
    v, w = I.probe_vectors(prob)
    trains = ref.astype(np.complex128) * 1j
    thd = _dev(torch, th, torch.float32)
    jv = ctx.jv(thd, _dev(torch, v, torch.float32)).cpu().numpy().astype(np.complex128)
    jv_ref = oracle_lib.jv(prob, th, trains, v, mask=mask)
    jhw = ctx.jhw(thd, _dev(torch, w, torch.complex64), reuse=True).cpu().numpy().astype(np.float64)
    jhw_ref = oracle_lib.jhw(prob, th, trains, w, mask=mask)
    d = oracle_lib.signal(prob, th, oracle_lib.epg(prob, th), mask=mask)
    _, r = ctx.residual(thd, _dev(torch, d, torch.complex64), reuse=True)
    r_ref = d - oracle_lib.signal(prob, th, trains, mask=mask)
    e = (_rel(jv, jv_ref), _rel(jhw, jhw_ref),
         float(np.linalg.norm(r.cpu().numpy() - r_ref) / np.linalg.norm(d)))
    print(f"\n[surrogate products] jv {e[0]:.2e} jhw {e[1]:.2e} residual/||d|| {e[2]:.2e}", flush=True)
    assert max(e) <= 2e-2


def test_gn_step_reports_fallbacks(setup):
    torch, ctx, prob, th, fb = (setup[k] for k in ("torch", "ctx", "prob", "th", "fb"))
    d = np.zeros(prob.data_shape, dtype=np.complex64)
    d[0, :, 3] = 1.0
    thd = _dev(torch, th, torch.float32)
    rep = ctx.gn_step(thd, _dev(torch, d, torch.complex64), 3, 0b11111, I.GN_LO, I.GN_HI)
    assert rep.n_fallback == int(fb.sum())
    assert np.isfinite(rep.f0) and rep.cg_iters >= 1


def test_no_surrogate_means_no_fallback(setup):
    torch, ctx, th = setup["torch"], setup["ctx"], setup["th"]
    ctx.set_surrogate(None)
    try:
        ctx.linearise(_dev(torch, th, torch.float32))
        assert ctx.fallback_count() == 0
    finally:
        ctx.set_surrogate(setup["net"])


def test_surrogate_shape_mismatch_rejected(setup):
    from paper_1904_13244_amd import binding as B
    other = B.Surrogate(8, 64, 1, 64)
    try:
        with pytest.raises(B.MrstatError) as e:
            setup["ctx"].set_surrogate(other)
        assert e.value.status == B.ERR_SHAPE
    finally:
        other.close()


@pytest.mark.parametrize("f16", [False, True])
def test_width256_split_inference(torch_gpu, oracle_lib, f16):
    """Width-256 networks run the hidden layers and the output layer as two
    kernels on the routed path: all four trains (4T = 288 outputs: a full and
    a ragged 256-row slice), the value-only trains of the residual (72 rows),
    480 voxels (a ragged 64-voxel tile), against the FP64 network."""
    torch = torch_gpu
    from oracle import mlp as M
    from paper_1904_13244_amd import binding as B
    from paper_1904_13244_amd.binding import Context, Surrogate
    rng = np.random.default_rng(64)
    n_tr, width, depth = 72, 256, 3
    prob = I.make_problem(24, 20, n_tr, 32, 16, flip_deg=I.flips_sin2_sweeps(n_tr, 20))
    nv = prob.nv
    lo, hi = np.array(I.SURR_LO), np.array(I.SURR_HI)
    th = I.iid_maps(nv, seed=65, b1=rng.uniform(0.8, 1.2, nv))
    th[:3] = np.clip(th[:3], lo[:, None] + 1e-3, hi[:, None] - 1e-3)
    th = th.astype(np.float32).astype(np.float64)
    flat = I.mlp_init_params(n_tr, width, depth, seed=66).astype(np.float32)
    scale = np.array([0.2, 0.15, 0.05, 0.3], dtype=np.float32)
    net = Surrogate(n_tr, width, depth, 128)
    net.set_scaling(I.SURR_LO, I.SURR_HI, scale)
    net.set_params(torch.from_numpy(flat).cuda())
    ctx = Context(prob)
    ctx.set_surrogate(net)
    ctx.set_train_precision(B.TRAINS_FP16 if f16 else B.TRAINS_FP32)
    parts = M.unpack(flat.astype(np.float64), n_tr, width, depth)
    for l in range(1, depth + 1):
        parts[2 * l] = _bf16(parts[2 * l])
    y, _ = M.forward(np.concatenate([p.reshape(-1) for p in parts]),
                     M.normalise_inputs(th[:3], I.SURR_LO, I.SURR_HI), n_tr, width, depth)
    net_tr = y[4 * n_tr:].reshape(4, n_tr, nv) * scale.astype(np.float64)[:, None, None]
    thd = _dev(torch, th, torch.float32)
    got = ctx.simulate(thd).cpu().numpy().astype(np.float64)
    assert ctx.fallback_count() == 0
    errs = [_rel(got[p], net_tr[p]) for p in range(4)]
    # Residual on value-only trains: data = the network's own signal at a
    # shifted point, so r compares the value-only inference at theta.
    s_net = oracle_lib.signal(prob, th, 1j * net_tr)
    th1 = th.copy()
    th1[0] = np.clip(th1[0] + 0.05, lo[0], hi[0] - 1e-3)
    th1 = th1.astype(np.float32).astype(np.float64)
    y1, _ = M.forward(np.concatenate([p.reshape(-1) for p in parts]),
                      M.normalise_inputs(th1[:3], I.SURR_LO, I.SURR_HI), n_tr, width, depth)
    net1 = y1[4 * n_tr:].reshape(4, n_tr, nv) * scale.astype(np.float64)[:, None, None]
    r_ref = s_net - oracle_lib.signal(prob, th1, 1j * net1)
    _, r = ctx.residual(_dev(torch, th1, torch.float32), _dev(torch, s_net, torch.complex64))
    e_r = float(np.linalg.norm(r.cpu().numpy() - r_ref) / np.linalg.norm(s_net))
    ctx.close()
    net.close()
    print(f"\n[width 256 f16={f16}] trains rel {['%.2e' % e for e in errs]}, residual {e_r:.2e}", flush=True)
    assert max(errs) <= 2e-2 and e_r <= 2e-2


def test_width192_chunked_inference_and_fp16_refusal(torch_gpu):
    """Widths other than 64, 128 and 256 infer layer by layer in batch-size
    chunks (hidden layers, then the output-layer GEMM with the inference
    epilogue). Their predictions and routed trains match the FP64 network on
    the same BF16-rounded weights (three chunks of 128 voxels, the last one
    ragged); FP16 train storage with such a network is refused in either
    order of the two calls."""
    torch = torch_gpu
    from oracle import mlp as M
    from paper_1904_13244_amd import binding as B
    from paper_1904_13244_amd.binding import Context, Surrogate
    rng = np.random.default_rng(71)
    n_tr, width, depth, batch = 48, 192, 2, 128
    prob = I.make_problem(20, 15, n_tr, 32, 8, flip_deg=I.flips_sin2_sweeps(n_tr, 15))
    nv = prob.nv
    lo, hi = np.array(I.SURR_LO), np.array(I.SURR_HI)
    th = I.iid_maps(nv, seed=72, b1=rng.uniform(0.8, 1.2, nv))
    th[:3] = np.clip(th[:3], lo[:, None] + 1e-3, hi[:, None] - 1e-3)
    th = th.astype(np.float32).astype(np.float64)
    flat = I.mlp_init_params(n_tr, width, depth, seed=73).astype(np.float32)
    scale = np.array([0.2, 0.15, 0.05, 0.3], dtype=np.float32)
    net = Surrogate(n_tr, width, depth, batch)
    net.set_scaling(I.SURR_LO, I.SURR_HI, scale)
    net.set_params(torch.from_numpy(flat).cuda())
    parts = M.unpack(flat.astype(np.float64), n_tr, width, depth)
    for l in range(1, depth + 1):
        parts[2 * l] = _bf16(parts[2 * l])
    y, _ = M.forward(np.concatenate([p.reshape(-1) for p in parts]),
                     M.normalise_inputs(th[:3], I.SURR_LO, I.SURR_HI), n_tr, width, depth)
    ref = y[4 * n_tr:].reshape(4, n_tr, nv) * scale.astype(np.float64)[:, None, None]
    thd = _dev(torch, th, torch.float32)
    pred = net.predict(thd[:3].contiguous()).cpu().numpy().astype(np.float64)
    ctx = Context(prob)
    ctx.set_surrogate(net)
    routed = ctx.simulate(thd).cpu().numpy().astype(np.float64)
    assert ctx.fallback_count() == 0
    e_pred = max(_rel(pred[p], ref[p]) for p in range(4))
    e_routed = max(_rel(routed[p], ref[p]) for p in range(4))
    print(f"\n[width 192] predict {e_pred:.2e}, routed {e_routed:.2e}", flush=True)
    assert e_pred <= 2e-2 and e_routed <= 2e-2
    with pytest.raises(B.MrstatError) as e1:
        ctx.set_train_precision(B.TRAINS_FP16)
    assert e1.value.status == B.ERR_UNSUPPORTED
    ctx.set_surrogate(None)
    ctx.set_train_precision(B.TRAINS_FP16)
    with pytest.raises(B.MrstatError) as e2:
        ctx.set_surrogate(net)
    assert e2.value.status == B.ERR_UNSUPPORTED
    ctx.close()
    net.close()
