"""Host-side checks of the algorithmic work bench.py divides by (no GPU): the
y-stage bytes and EPG flops per launch at 224 x 224, 1120 TRs, counted from
the method's arithmetic, with four trains and with three (B1 held fixed)."""
import importlib.util
import os

from paper_1904_13244_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_ystage_and_epg_work_per_launch():
    b = _bench()
    prob = I.make_problem(224, 224, 1120, 448, 32)
    T, nv, nx = 1120, 224 * 224, 224
    # Adjoint: ntr trains of b bytes per voxel and TR plus the complex W rows.
    assert b.algorithmic("ystage_adj", prob, 2, 3) == ("bytes", 3 * 2 * T * nv + 8 * T * nx, "hbm")
    assert b.algorithmic("ystage_adj", prob, 4, 4)[1] == 4 * 4 * T * nv + 8 * T * nx
    assert b.algorithmic("ystage_adj", prob, 2, 3)[1] == 339_189_760
    # Forward J v: trains, rho (8 bytes) and ntr + 1 direction rows (4 bytes each), U out.
    assert b.algorithmic("ystage_fwd_jv", prob, 2, 3)[1] == 3 * 2 * T * nv + 24 * nv + 8 * T * nx
    assert b.algorithmic("ystage_fwd_jv", prob, 4, 4)[1] == 4 * 4 * T * nv + 28 * nv + 8 * T * nx
    # EPG: 67 flop per state and TR with the B1 tangent, 45 without it.
    assert b.algorithmic("epg", prob, 4, 4)[1] == 67 * 32 * T * nv
    assert b.algorithmic("epg", prob, 4, 3)[1] == 45 * 32 * T * nv
    # Surrogate: the trains written once, FP16.
    flop, wbytes = b.surrogate_work(prob, ntr=3)
    assert wbytes == 3 * 2 * T * nv
    assert flop == 2 * (3 * 256 + 3 * 256 * 256 + 3 * T * 256) * nv
