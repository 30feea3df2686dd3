"""Surrogate network kernels (through the C ABI) against the FP64 network
oracle (oracle/mlp.py).

Both sides use the same weights: the GPU multiplies with BF16 copies of the
weights of the layers that run on the matrix cores (hidden layers after the
first and the output layer), so the oracle gets those weights rounded to
BF16, the first layer and all biases in FP32. The GPU also rounds every
activation, pre-activation and back-propagated product to BF16 (unit
roundoff u = 2^-9) between layers; the oracle keeps FP64. A depth-L network
passes about 2L such roundings along any path, each a relative perturbation
of at most u, so its outputs and gradients differ from the oracle by about
2L u normwise in the worst case (about 1.6e-2 for L = 4), far less when the
roundings are independent. The bars: 2e-2 normwise for outputs and loss,
3e-2 normwise and cosine >= 0.999 for each parameter block's gradient.
Targets and inputs are seeded; no expected value comes from the GPU.
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


def _bf16(x):
    """Round-to-nearest-even of float32 values to BF16, returned as float64."""
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _oracle_weights(flat, n_tr, width, depth):
    """The weights the GPU multiplies with, in the packed layout."""
    from oracle import mlp as M
    parts = M.unpack(np.asarray(flat, dtype=np.float32).astype(np.float64), n_tr, width, depth)
    for l in range(1, depth + 1):          # hidden layers 2.. and the output layer
        parts[2 * l] = _bf16(parts[2 * l])
    return np.concatenate([p.reshape(-1) for p in parts])


def _params(n_tr, width, depth, seed):
    flat = I.mlp_init_params(n_tr, width, depth, seed=seed).astype(np.float32)
    from oracle import mlp as M
    # Non-zero biases so every bias path is exercised.
    rng = np.random.default_rng(seed + 1)
    o = 0
    for s in M.shapes(n_tr, width, depth):
        k = int(np.prod(s))
        if len(s) == 1:
            flat[o:o + k] = rng.uniform(-0.2, 0.2, k)
        o += k
    return flat


def _case(n_tr, width, depth, batch, seed):
    rng = np.random.default_rng(seed)
    theta = I.surrogate_samples(batch, seed=seed + 2).astype(np.float32)
    trains = (rng.standard_normal((4, n_tr, batch)) * np.array([0.3, 0.2, 0.1, 0.4])[:, None, None])
    scale = np.array([0.31, 0.17, 0.12, 0.45])
    return theta, trains.astype(np.float32), scale.astype(np.float32)


SIZES = {
    "small": (16, 64, 3, 128),
    "ragged_depth1": (24, 64, 1, 64),
    "full_width": (1120, 256, 4, 512),   # the surrogate's layer shapes at 1120 TRs
}


def _blocks(n_tr, width, depth):
    from oracle import mlp as M
    out, o = [], 0
    for s in M.shapes(n_tr, width, depth):
        k = int(np.prod(s))
        out.append((s, slice(o, o + k)))
        o += k
    return out


@pytest.mark.parametrize("size", list(SIZES))
def test_forward_loss_and_gradients_match_oracle(torch_gpu, size):
    torch = torch_gpu
    from oracle import mlp as M
    from paper_1904_13244_amd.binding import Surrogate
    n_tr, width, depth, batch = SIZES[size]
    print(f"\n[mlp {size}] T={n_tr} width={width} depth={depth} batch={batch}", flush=True)
    flat = _params(n_tr, width, depth, seed=11)
    theta, trains, scale = _case(n_tr, width, depth, batch, seed=21)
    net = Surrogate(n_tr, width, depth, batch)
    assert net.n_params == M.n_params(n_tr, width, depth)
    th_d = torch.from_numpy(theta).cuda()
    tr_d = torch.from_numpy(trains).cuda()
    # The scaling fit shares the loss buffer: the loss must not see its sums.
    fitted = net.fit_scaling(tr_d, I.SURR_LO, I.SURR_HI)
    rms = np.sqrt(np.mean(trains.astype(np.float64) ** 2, axis=(1, 2)))
    assert np.allclose(fitted, rms, rtol=1e-5)
    net.set_scaling(I.SURR_LO, I.SURR_HI, scale)
    net.set_params(torch.from_numpy(flat).cuda())
    loss, g = net.gradients(th_d, tr_d)
    pred = net.predict(th_d).cpu().numpy().astype(np.float64)
    g = g.cpu().numpy().astype(np.float64)

    w_ora = _oracle_weights(flat, n_tr, width, depth)
    x = M.normalise_inputs(theta.astype(np.float64), I.SURR_LO, I.SURR_HI)
    tgt = M.scaled_targets(trains.astype(np.float64), scale.astype(np.float64))
    y, _ = M.forward(w_ora, x, n_tr, width, depth)
    loss_o, g_o = M.loss_and_grad(w_ora, x, tgt, n_tr, width, depth)

    # Prediction: imaginary outputs times the head scales, [4][T][batch].
    pred_o = y[4 * n_tr:].reshape(4, n_tr, batch) * scale.astype(np.float64)[:, None, None]
    e_pred = np.linalg.norm(pred - pred_o) / np.linalg.norm(pred_o)
    e_loss = abs(loss - loss_o) / loss_o
    print(f"  pred {e_pred:.2e}  loss {loss:.6e} vs {loss_o:.6e} ({e_loss:.2e})", flush=True)
    assert e_pred < 2e-2
    assert e_loss < 2e-2
    for s, sl in _blocks(n_tr, width, depth):
        a, b = g[sl], g_o[sl]
        e = np.linalg.norm(a - b) / np.linalg.norm(b)
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))
        print(f"  grad block {s}: rel {e:.2e} cos {cos:.6f}", flush=True)
        assert e < 3e-2 and cos > 0.999, (s, e, cos)
    net.close()


def test_predict_ragged_columns_over_several_chunks(torch_gpu):
    """Inference over n columns that span several batches with a ragged
    tail, against the oracle's forward pass."""
    torch = torch_gpu
    from oracle import mlp as M
    from paper_1904_13244_amd.binding import Surrogate
    n_tr, width, depth, batch = SIZES["ragged_depth1"]
    flat = _params(n_tr, width, depth, seed=13)
    n = 3 * batch - 37
    theta = I.surrogate_samples(n, seed=17).astype(np.float32)
    scale = np.array([0.5, 0.25, 0.125, 2.0], dtype=np.float32)
    net = Surrogate(n_tr, width, depth, batch)
    net.set_scaling(I.SURR_LO, I.SURR_HI, scale)
    net.set_params(torch.from_numpy(flat).cuda())
    th_d = torch.from_numpy(theta).cuda()
    pred = net.predict(th_d).cpu().numpy().astype(np.float64)
    x = M.normalise_inputs(theta.astype(np.float64), I.SURR_LO, I.SURR_HI)
    y, _ = M.forward(_oracle_weights(flat, n_tr, width, depth), x, n_tr, width, depth)
    pred_o = y[4 * n_tr:].reshape(4, n_tr, n) * scale.astype(np.float64)[:, None, None]
    e = np.linalg.norm(pred - pred_o) / np.linalg.norm(pred_o)
    print(f"\n[predict ragged] n={n}: rel {e:.2e}", flush=True)
    assert e < 2e-2
    # Every voxel tile of the fused kernel computes the same values.
    for tile in (32, 64, -64):
        net.set_infer_tile(tile)
        other = net.predict(th_d).cpu().numpy().astype(np.float64)
        assert np.array_equal(other, pred), tile
    net.close()


def test_adam_first_steps_closed_form(torch_gpu):
    """Adam's first step moves every weight by lr * g / (|g| + eps) (bias
    correction makes m-hat = g and v-hat = g^2); the BF16 copy used by the
    next step follows the FP32 master."""
    torch = torch_gpu
    from oracle import mlp as M
    from paper_1904_13244_amd.binding import Surrogate
    n_tr, width, depth, batch = SIZES["small"]
    flat = _params(n_tr, width, depth, seed=31)
    theta, trains, scale = _case(n_tr, width, depth, batch, seed=41)
    net = Surrogate(n_tr, width, depth, batch)
    net.set_scaling(I.SURR_LO, I.SURR_HI, scale)
    net.set_params(torch.from_numpy(flat).cuda())
    th_d = torch.from_numpy(theta).cuda()
    tr_d = torch.from_numpy(trains).cuda()
    lr = 1e-3
    net.train_step(th_d, tr_d, lr)
    p1 = net.get_params().cpu().numpy().astype(np.float64)
    x = M.normalise_inputs(theta.astype(np.float64), I.SURR_LO, I.SURR_HI)
    tgt = M.scaled_targets(trains.astype(np.float64), scale.astype(np.float64))
    _, g_o = M.loss_and_grad(_oracle_weights(flat, n_tr, width, depth), x, tgt, n_tr, width, depth)
    big = np.abs(g_o) > 0.05 * np.sqrt(np.mean(g_o ** 2))
    step = (flat.astype(np.float64) - p1) / lr
    assert big.mean() > 0.5
    err = np.abs(step[big] - np.sign(g_o[big]))
    print(f"\n[adam] entries {big.sum()}, max |step/lr - sign g| {err.max():.2e}", flush=True)
    assert np.quantile(err, 0.999) < 5e-3
    # Small gradients move less than lr, never more.
    assert np.all(np.abs(step) <= 1.0 + 1e-3)
    # Setting parameters resets the optimiser: the same first step again.
    net.set_params(torch.from_numpy(flat).cuda())
    net.train_step(th_d, tr_d, lr)
    p1b = net.get_params().cpu().numpy().astype(np.float64)
    assert np.array_equal(p1, p1b)
    net.close()


def test_training_reduces_loss_on_epg_trains(torch_gpu):
    """A few hundred Adam steps on EPG trains of a short sequence reduce the
    loss by more than an order of magnitude (host-side check on the loss the
    kernels report)."""
    torch = torch_gpu
    from paper_1904_13244_amd.binding import Context, Surrogate
    n_tr, n = 64, 8192
    prob = I.make_problem(128, 64, n_tr, 128, 16, flip_deg=I.flips_sin2_sweeps(n_tr, 16))
    th = np.zeros((5, n), dtype=np.float32)
    th[:3] = I.surrogate_samples(n, seed=51)
    th[3] = 1.0
    ctx = Context(prob)
    th_d = torch.from_numpy(th).cuda()
    trains = ctx.simulate(th_d)
    net = Surrogate(n_tr, 128, 3, 1024)
    scales = net.fit_scaling(trains, I.SURR_LO, I.SURR_HI)
    assert all(s > 0 for s in scales)
    net.set_params(torch.from_numpy(I.mlp_init_params(n_tr, 128, 3).astype(np.float32)).cuda())
    first = net.train_step(th_d, trains, 1e-3, col=0, want_loss=True)
    last = None
    for it in range(400):
        last = net.train_step(th_d, trains, 1e-3, col=1024 * (it % 8), want_loss=(it == 399))
    print(f"\n[train] loss {first:.4e} -> {last:.4e}", flush=True)
    assert np.isfinite(last) and last < first / 10
    net.close()
    ctx.close()


def test_argument_errors(torch_gpu):
    from paper_1904_13244_amd import binding as B
    for args in [(12, 64, 2, 64), (16, 60, 2, 64), (16, 64, 0, 64), (16, 64, 2, 100)]:
        with pytest.raises(B.MrstatError) as e:
            B.mrstat_mlp_create(*args)
        assert e.value.status == B.ERR_SHAPE
    net = B.mrstat_mlp_create(16, 64, 2, 64)
    try:
        assert B.lib().mrstat_mlp_train_step(net, None, 64, None, 64, 1e-3, None, None) == B.ERR_ARG
        # Unbound network: no device work.
        import ctypes as C
        st = B.lib().mrstat_mlp_predict(net, C.c_void_p(256), 64, 64, C.c_void_p(512), None)
        assert st == B.ERR_WORKSPACE
    finally:
        B.mrstat_mlp_destroy(net)
