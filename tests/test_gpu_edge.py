"""Degenerate and extreme shapes through the C ABI against the FP64 oracle:
one voxel with one TR, one readout sample and one EPG state; the maximum of
64 EPG states; a single image row; a single image column. Trains, residual,
J v and Re(J^H w) to the plain path's 1e-5 (FP32 trains) and 1e-3 (FP16
trains), and, where the problem is well posed, one Gauss-Newton step
against the oracle's."""
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


def _rel(a, b):
    """Normwise relative error; absolute when the reference is exactly zero
    (with one TR the ln T1 derivative vanishes: no relaxation before the
    first readout)."""
    nb = np.linalg.norm(np.asarray(b))
    err = float(np.linalg.norm(np.asarray(a) - np.asarray(b)))
    return err / nb if nb > 0 else err


CASES = {
    # name: (nx, ny, T, n_read, K, compare a GN step); the GN comparison runs
    # where the least-squares problem is well posed (more independent data
    # than unknowns), elsewhere FP32 and FP64 CG may part ways legitimately.
    "single_voxel_T1_K1": (1, 1, 1, 1, 1, False),
    "max_states_K64": (6, 5, 24, 8, 64, True),
    "one_row": (50, 1, 9, 64, 7, True),
    "one_column": (1, 40, 33, 3, 20, False),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("f16", [False, True])
def test_edge_shapes(torch_gpu, oracle_lib, name, f16):
    torch = torch_gpu
    from paper_1904_13244_amd import binding as B
    from paper_1904_13244_amd.binding import Context
    nx, ny, T, nk, K, gn = CASES[name]
    rng = np.random.default_rng(sum(map(ord, name)))
    prob = I.make_problem(nx, ny, T, nk, K, flip_deg=rng.uniform(10, 70, T))
    th = I.iid_maps(prob.nv, seed=3, b1=rng.uniform(0.85, 1.15, prob.nv))
    print(f"\n[edge {name} f16={f16}] nx={nx} ny={ny} T={T} nk={nk} K={K}", flush=True)
    dev = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt)  # noqa: E731
    tol = 1e-3 if f16 else 1e-5
    ctx = Context(prob)
    ctx.set_train_precision(B.TRAINS_FP16 if f16 else B.TRAINS_FP32)
    thd = dev(th, torch.float32)
    ora = oracle_lib.epg(prob, th)
    got = ctx.simulate(thd).cpu().numpy().astype(np.float64)
    for p in range(4):
        assert _rel(got[p], ora[p].imag) <= tol, p
    v, w = I.probe_vectors(prob)
    jv = ctx.jv(thd, dev(v, torch.float32), reuse=True).cpu().numpy().astype(np.complex128)
    jhw = ctx.jhw(thd, dev(w, torch.complex64), reuse=True).cpu().numpy().astype(np.float64)
    e_jv = _rel(jv, oracle_lib.jv(prob, th, ora, v))
    e_jhw = _rel(jhw, oracle_lib.jhw(prob, th, ora, w))
    d = oracle_lib.signal(prob, th, ora)
    th0 = th.copy()
    th0[0] += 0.05
    th0 = th0.astype(np.float32).astype(np.float64)
    _, r_ref = oracle_lib.residual(prob, th0, d)
    _, r = ctx.residual(dev(th0, torch.float32), dev(d, torch.complex64))
    e_r = float(np.linalg.norm(r.cpu().numpy() - r_ref) / np.linalg.norm(d))
    print(f"  jv {e_jv:.2e} jhw {e_jhw:.2e} residual {e_r:.2e}", flush=True)
    assert max(e_jv, e_jhw, e_r) <= tol
    if not gn:
        ctx.close()
        return
    # One GN step (T1, T2, rho) from the perturbed point.
    t_ora, _ = oracle_lib.gn_step(prob, th0, d, n_cg=4, param_mask=0b11011, lo=I.GN_LO, hi=I.GN_HI)
    t_gpu = dev(th0, torch.float32)
    rep = ctx.gn_step(t_gpu, dev(d, torch.complex64), 4, 0b11011, I.GN_LO, I.GN_HI)
    e_gn = _rel(t_gpu.cpu().numpy(), t_ora)
    print(f"  gn theta {e_gn:.2e}, report {rep.as_dict()}", flush=True)
    assert e_gn <= (1e-3 if f16 else 1e-4)
    ctx.close()
