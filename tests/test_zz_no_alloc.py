"""mrstat_bind_static: a context bound to the library's own static device
workspace computes exactly what a context bound to a caller workspace does.

Two bindings in a row share the one static array of the device: the 32 x 32,
128-TR case, then a smaller 24 x 20, 60-TR case with 4 coils and a voxel
mask. For each, the trains, the residual and f, J v, Re(J^H w) and one
Gauss-Newton step are compared with those of a context on a torch-allocated
workspace (same kernels, fixed-order reductions: equal bit for bit). The
first context loses the array to the second and then reports
MRSTAT_ERR_STATE; a problem whose workspace exceeds the static maximum is
refused with MRSTAT_ERR_WORKSPACE.
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


def _outputs(torch, ctx, prob, th, d, v, w, pmask):
    """Everything the context computes on these inputs, as host arrays."""
    out = {"trains": ctx.simulate(th).cpu().numpy()}
    f, r = ctx.residual(th, d)
    out["f"], out["r"] = np.array([f]), r.cpu().numpy()
    out["jv"] = ctx.jv(th, v, reuse=True).cpu().numpy()
    out["jhw"] = ctx.jhw(th, w, reuse=True).cpu().numpy()
    t = th.clone()
    rep = ctx.gn_step(t, d, 5, pmask, I.GN_LO, I.GN_HI)
    out["gn_theta"] = t.cpu().numpy()
    out["gn_f1"] = np.array([rep.f1, rep.t, rep.cg_iters])
    return out


def _case(big):
    if big:
        w = I.config(1)
        return w.problem, w.theta, None, None
    rng = np.random.default_rng(6)
    prob = I.make_problem(24, 20, 60, 48, 16, n_coils=4, flip_deg=I.flips_sin2_sweeps(60, 20))
    th = I.iid_maps(prob.nv, seed=5, b1=rng.uniform(0.8, 1.2, prob.nv))
    coil = I.coil_maps(24, 20, 4)
    mask = (rng.uniform(size=prob.nv) > 0.2).astype(np.uint8)
    return prob, th, coil, mask


def test_static_workspace_matches_caller_workspace(torch_gpu, oracle_lib):
    torch = torch_gpu
    from paper_1904_13244_amd import binding as B
    from paper_1904_13244_amd.binding import Context
    held = None
    for big in (True, False):
        prob, th_true, coil, mask = _case(big)
        d = oracle_lib.signal(prob, th_true, oracle_lib.epg(prob, th_true, tangents=False),
                              coil=coil, mask=mask)
        rng = np.random.default_rng(8)
        th0 = th_true.copy()
        th0[:2] += 0.1 * rng.standard_normal((2, prob.nv))
        th = _dev(torch, th0, torch.float32)
        v, wv = I.probe_vectors(prob)
        args = (prob, th, _dev(torch, d, torch.complex64), _dev(torch, v, torch.float32),
                _dev(torch, wv, torch.complex64), 0b11011)
        kw = dict(coil=None if coil is None else _dev(torch, coil, torch.complex64),
                  mask=None if mask is None else _dev(torch, mask, torch.uint8))
        ref_ctx = Context(prob, **kw)
        ref = _outputs(torch, ref_ctx, *args)
        ref_ctx.close()
        st_ctx = Context(prob, static=True, **kw)
        assert st_ctx.ws is None
        got = _outputs(torch, st_ctx, *args)
        for k in ref:
            assert np.array_equal(got[k], ref[k]), (prob.nx, k)
        print(f"  {prob.nx}x{prob.ny}, {prob.n_tr} TRs, {prob.n_coils} coil(s): static workspace "
              f"equal to the caller workspace ({len(ref)} outputs)", flush=True)
        if held is not None:
            # The earlier context lost the array to this one.
            with pytest.raises(B.MrstatError) as e:
                held.simulate(held_th)
            assert e.value.status == B.ERR_STATE
            held.close()
        held, held_th = st_ctx, th
    held.close()
    # A workspace beyond the static maximum is refused, before any device work.
    big = I.config(3).problem
    h = B.mrstat_create(big)
    try:
        assert B.mrstat_workspace_bytes(h) > (64 << 20)
        assert B.lib().mrstat_bind_static(h, None, None, None) == B.ERR_WORKSPACE
        assert b"static" in B.lib().mrstat_last_error(h)
    finally:
        B.mrstat_destroy(h)
