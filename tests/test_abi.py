"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function include/mrstat.h declares, and validates problems and
arguments before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1904_13244_amd import binding as B
from paper_1904_13244_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "mrstat.h")).read()
    return sorted(set(re.findall(r"\b(mrstat_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = B.lib()
    names = _declared()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(B.exported_symbols()) == names


def _status(prob):
    try:
        h = B.mrstat_create(prob)
    except B.MrstatError as e:
        return e.status
    B.mrstat_destroy(h)
    return B.OK


def test_create_validates_problem():
    good = I.make_problem(8, 6, 12, 16, 8)
    assert _status(good) == B.OK
    assert _status(I.shrink(good, n_read=7)) == B.ERR_SHAPE          # n_read < nx
    assert _status(I.shrink(good, n_states=65)) == B.ERR_SHAPE
    assert _status(I.shrink(good, n_coils=17)) == B.ERR_SHAPE
    assert _status(I.shrink(good, te=0.009)) == B.ERR_ARG             # te > tr
    bad_ky = good.ky_line.copy()
    bad_ky[3] = 6
    assert _status(I.shrink(good, ky_line=bad_ky)) == B.ERR_ARG
    ph = np.zeros(12)
    ph[2] = np.pi
    assert _status(I.shrink(good, rf_phase=ph)) == B.OK               # 0 / pi supported
    ph[4] = 0.3
    assert _status(I.shrink(good, rf_phase=ph)) == B.ERR_UNSUPPORTED  # general phase
    fl = good.flip_deg.copy()
    fl[0] = np.nan
    assert _status(I.shrink(good, flip_deg=fl)) == B.ERR_ARG


def test_workspace_and_unbound_calls():
    prob = I.config(3).problem
    h = B.mrstat_create(prob)
    try:
        ws = B.mrstat_workspace_bytes(h)
        trains = 16 * prob.n_tr * prob.nv
        assert trains < ws < 1.6 * trains   # trains dominate the workspace
        # Calls before mrstat_bind fail without touching the device.
        st = B.lib().mrstat_jv(h, None, 0, None, None, None)
        assert st == B.ERR_WORKSPACE
        st = B.lib().mrstat_bind(h, None, ws, None, None, None)
        assert st == B.ERR_WORKSPACE
        st = B.lib().mrstat_bind(h, C.c_void_p(4096 + 8), ws, None, None, None)
        assert st == B.ERR_WORKSPACE    # misaligned
        assert B.lib().mrstat_set_epg_lanes(h, 3) == B.ERR_ARG
        assert B.lib().mrstat_set_epg_lanes(h, 2) == B.OK
    finally:
        B.mrstat_destroy(h)


def test_bind_static_refuses_oversized_workspace_on_host():
    """The size check of mrstat_bind_static comes before any HIP call: a
    workspace beyond MRSTAT_STATIC_WORKSPACE_BYTES (64 MiB) is refused with
    MRSTAT_ERR_WORKSPACE and a message naming the bytes needed."""
    h = B.mrstat_create(I.config(3).problem)
    try:
        need = B.mrstat_workspace_bytes(h)
        assert need > (64 << 20)
        assert B.lib().mrstat_bind_static(h, None, None, None) == B.ERR_WORKSPACE
        msg = B.lib().mrstat_last_error(h).decode()
        assert str(need) in msg and str(64 << 20) in msg
    finally:
        B.mrstat_destroy(h)
