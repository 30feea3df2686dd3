"""FP64 CPU oracle for the MR-STAT matrix-free Jacobian products (ctypes wrapper).

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. It never imports
the HIP package and the HIP package never imports it; they share only the
seeded input generators, which hold none of the method's arithmetic.

The arithmetic lives in ``oracle.c`` (plain C99, double / double complex,
OpenMP over independent voxels or rows). This module only marshals numpy
arrays. Problem objects are duck-typed: anything with the attributes nx, ny,
n_tr, n_read, n_states, n_coils, tr, te, t_inv, flip_deg, rf_phase, ky_line,
optionally traj = (kx, ky), each [n_tr][n_read] in cycles per field of view
(non-Cartesian sampling; None or absent = the Cartesian grid), and optionally
iso = (scale, weight) [n_iso] (the balanced isochromat model; None = EPG).

Paper: van der Heide et al., arXiv 1904.13244 (MR-STAT, matrix-free inexact
Gauss-Newton). Conventions: theta is [5][Nv] = (ln T1, ln T2, B1, Re rho,
Im rho), the parameter-major layout of the Theory section; r = d - s,
f = 0.5||r||^2, J = dr/dalpha, g = Re(J^H r).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (FP64, OpenMP, no fast-math)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
               "-fno-fast-math", "-Wall", "-o", _SO + ".tmp",
               os.path.join(_HERE, "oracle.c"), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_SO + ".tmp", _SO)
    return _SO


class _Problem(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("n_tr", C.c_int), ("n_read", C.c_int),
                ("n_states", C.c_int), ("n_coils", C.c_int),
                ("tr", C.c_double), ("te", C.c_double), ("t_inv", C.c_double),
                ("flip_deg", C.POINTER(C.c_double)), ("rf_phase", C.POINTER(C.c_double)),
                ("ky_line", C.POINTER(C.c_int)), ("kx", C.POINTER(C.c_double)),
                ("ky", C.POINTER(C.c_double)), ("n_iso", C.c_int),
                ("iso_scale", C.POINTER(C.c_double)), ("iso_weight", C.POINTER(C.c_double)),
                ("dwell", C.c_double), ("db0", C.POINTER(C.c_double)),
                ("db0_unit", C.c_double), ("db0_box", C.c_double)]


class _GnOpts(C.Structure):
    _fields_ = [("n_cg", C.c_int), ("n_ls_max", C.c_int), ("param_mask", C.c_int),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("armijo_c1", C.c_double)]


class _GnReport(C.Structure):
    _fields_ = [("f0", C.c_double), ("f1", C.c_double), ("gnorm", C.c_double),
                ("step_norm", C.c_double), ("t", C.c_double),
                ("cg_iters", C.c_int), ("ls_trials", C.c_int), ("accepted", C.c_int)]


class _TrOpts(C.Structure):
    _fields_ = [("n_cg", C.c_int), ("param_mask", C.c_int), ("lo", C.c_double * 3),
                ("hi", C.c_double * 3), ("eta", C.c_double), ("delta_max", C.c_double)]


class _TrReport(C.Structure):
    _fields_ = [("f0", C.c_double), ("f1", C.c_double), ("gnorm", C.c_double),
                ("step_norm", C.c_double), ("rho", C.c_double), ("pred", C.c_double),
                ("delta_in", C.c_double), ("delta_out", C.c_double), ("cg_iters", C.c_int),
                ("exit_kind", C.c_int), ("accepted", C.c_int), ("n_reflected", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


TR_ITERS, TR_BOUNDARY, TR_CURVATURE, TR_ZERO = 0, 1, 2, 3


@dataclass
class GnReport:
    f0: float
    f1: float
    gnorm: float
    step_norm: float
    t: float
    cg_iters: int
    ls_trials: int
    accepted: int


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = C.CDLL(_SO)
        P = C.POINTER
        vp = C.c_void_p
        L.oracle_epg.argtypes = [P(_Problem), vp, C.c_int, vp]
        L.oracle_signal_direct.argtypes = [P(_Problem), vp, vp, vp, vp, vp]
        L.oracle_signal_separable.argtypes = [P(_Problem), vp, vp, vp, vp, vp]
        L.oracle_jv.argtypes = [P(_Problem), vp, vp, vp, vp, vp, vp]
        L.oracle_jhw.argtypes = [P(_Problem), vp, vp, vp, vp, vp, vp]
        L.oracle_jacobian.argtypes = [P(_Problem), vp, vp, vp, vp, vp]
        L.oracle_residual.argtypes = [P(_Problem), vp, vp, vp, vp, vp]
        L.oracle_residual.restype = C.c_double
        L.oracle_gn_step.argtypes = [P(_Problem), vp, vp, vp, vp, P(_GnOpts), P(_GnReport)]
        L.oracle_phases.argtypes = [P(_Problem), C.c_int, vp]
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = C.c_int
        L.oracle_rho_init.argtypes = [P(_Problem), vp, vp, vp, vp, C.c_int]
        L.oracle_isochromat.argtypes = [P(_Problem), C.c_double, C.c_double, C.c_double, C.c_double,
                                        vp, vp, vp, vp]
        L.oracle_steihaug_dense.argtypes = [C.c_int, vp, vp, C.c_double, C.c_int, vp, P(C.c_int)]
        L.oracle_steihaug_dense.restype = C.c_int
        L.oracle_reflect.argtypes = [C.c_double, C.c_double, C.c_double]
        L.oracle_reflect.restype = C.c_double
        L.oracle_tr_step.argtypes = [P(_Problem), vp, vp, vp, vp, P(_TrOpts), P(C.c_double),
                                     P(_TrReport)]
        _lib = L
    return _lib


class _Bound:
    """Holds the ctypes problem struct and keeps its arrays alive."""

    def __init__(self, prob):
        self.flip = np.ascontiguousarray(prob.flip_deg, dtype=np.float64)
        self.phase = np.ascontiguousarray(prob.rf_phase, dtype=np.float64)
        self.ky = np.ascontiguousarray(prob.ky_line, dtype=np.int32)
        assert self.flip.shape == (prob.n_tr,) and self.phase.shape == (prob.n_tr,)
        assert self.ky.shape == (prob.n_tr,)
        traj = getattr(prob, "traj", None)
        kxp = kyp = None
        if traj is not None:
            self.kx = np.ascontiguousarray(traj[0], dtype=np.float64)
            self.kyt = np.ascontiguousarray(traj[1], dtype=np.float64)
            assert self.kx.shape == (prob.n_tr, prob.n_read) == self.kyt.shape
            kxp = self.kx.ctypes.data_as(C.POINTER(C.c_double))
            kyp = self.kyt.ctypes.data_as(C.POINTER(C.c_double))
        iso = getattr(prob, "iso", None)
        n_iso, sp, wp = 0, None, None
        if iso is not None:
            self.iso_s = np.ascontiguousarray(iso[0], dtype=np.float64)
            self.iso_w = np.ascontiguousarray(iso[1], dtype=np.float64)
            assert self.iso_s.shape == self.iso_w.shape and self.iso_s.ndim == 1
            n_iso = self.iso_s.size
            sp = self.iso_s.ctypes.data_as(C.POINTER(C.c_double))
            wp = self.iso_w.ctypes.data_as(C.POINTER(C.c_double))
        dwell = float(getattr(prob, "dwell", 0.0) or 0.0)
        db0 = getattr(prob, "db0", None)
        bp = None
        if db0 is not None:
            if n_iso:
                raise ValueError("the balanced isochromat model is not combined with off-resonance")
            self.db0 = np.ascontiguousarray(db0, dtype=np.float64)
            assert self.db0.shape == (prob.nx * prob.ny,)
            bp = self.db0.ctypes.data_as(C.POINTER(C.c_double))
        unit = float(getattr(prob, "db0_unit", 0.0) or 0.0)
        box = 0.0
        if unit > 0.0:
            if bp is not None or n_iso:
                raise ValueError("a fitted Delta B0 takes no map and no isochromat model")
            box = float(getattr(prob, "rd_max_db0", 0.0) or 0.0)
        self.s = _Problem(prob.nx, prob.ny, prob.n_tr, prob.n_read, prob.n_states,
                          prob.n_coils, prob.tr, prob.te, prob.t_inv,
                          self.flip.ctypes.data_as(C.POINTER(C.c_double)),
                          self.phase.ctypes.data_as(C.POINTER(C.c_double)),
                          self.ky.ctypes.data_as(C.POINTER(C.c_int)), kxp, kyp, n_iso, sp, wp,
                          dwell, bp, unit, box)
        self.nv = prob.nx * prob.ny
        self.np = 6 if unit > 0.0 else 5
        self.prob = prob


def _f64(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float64)
    assert a.shape == shape, (a.shape, shape)
    return a


def _c128(a, shape):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    assert a.shape == shape, (a.shape, shape)
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data


def _coil(b, coil):
    if coil is None:
        assert b.prob.n_coils == 1
        return None
    return _c128(coil, (b.prob.n_coils, b.nv))


def _mask(b, mask):
    if mask is None:
        return None
    return np.ascontiguousarray(mask, dtype=np.uint8).reshape(b.nv)


def _dshape(prob):
    return (prob.n_coils, prob.n_tr, prob.n_read)


def num_threads():
    return int(lib().oracle_num_threads())


def phases(prob, n):
    """E[n, k, j] for all k, j: [n_read][Nv] complex."""
    b = _Bound(prob)
    out = np.zeros((prob.n_read, b.nv), dtype=np.complex128)
    lib().oracle_phases(C.byref(b.s), int(n), out.ctypes.data)
    return out


def epg(prob, theta, tangents=True):
    """Trains [4][n_tr][Nv] complex: m, dm/dlnT1, dm/dlnT2, dm/dB1."""
    b = _Bound(prob)
    th = _f64(theta, (b.np, b.nv))
    out = np.zeros((4, prob.n_tr, b.nv), dtype=np.complex128)
    lib().oracle_epg(C.byref(b.s), th.ctypes.data, 1 if tangents else 0, out.ctypes.data)
    return out


def signal_direct(prob, theta, trains, coil=None, mask=None):
    b = _Bound(prob)
    th = _f64(theta, (b.np, b.nv))
    tr = _c128(trains, (4, prob.n_tr, b.nv))
    cl, mk = _coil(b, coil), _mask(b, mask)
    out = np.zeros(_dshape(prob), dtype=np.complex128)
    lib().oracle_signal_direct(C.byref(b.s), th.ctypes.data, _ptr(cl), _ptr(mk),
                               tr.ctypes.data, out.ctypes.data)
    return out


def signal(prob, theta, trains, coil=None, mask=None):
    """Separable evaluation of the same sum as signal_direct."""
    b = _Bound(prob)
    th = _f64(theta, (b.np, b.nv))
    tr = _c128(trains, (4, prob.n_tr, b.nv))
    cl, mk = _coil(b, coil), _mask(b, mask)
    out = np.zeros(_dshape(prob), dtype=np.complex128)
    lib().oracle_signal_separable(C.byref(b.s), th.ctypes.data, _ptr(cl), _ptr(mk),
                                  tr.ctypes.data, out.ctypes.data)
    return out


def jv(prob, theta, trains, v, coil=None, mask=None):
    b = _Bound(prob)
    th = _f64(theta, (b.np, b.nv))
    tr = _c128(trains, (4, prob.n_tr, b.nv))
    vv = _f64(v, (b.np, b.nv))
    cl, mk = _coil(b, coil), _mask(b, mask)
    out = np.zeros(_dshape(prob), dtype=np.complex128)
    lib().oracle_jv(C.byref(b.s), th.ctypes.data, _ptr(cl), _ptr(mk), tr.ctypes.data,
                    vv.ctypes.data, out.ctypes.data)
    return out


def jhw(prob, theta, trains, w, coil=None, mask=None):
    b = _Bound(prob)
    th = _f64(theta, (b.np, b.nv))
    tr = _c128(trains, (4, prob.n_tr, b.nv))
    ww = _c128(w, _dshape(prob))
    cl, mk = _coil(b, coil), _mask(b, mask)
    out = np.zeros((b.np, b.nv), dtype=np.float64)
    lib().oracle_jhw(C.byref(b.s), th.ctypes.data, _ptr(cl), _ptr(mk), tr.ctypes.data,
                     ww.ctypes.data, out.ctypes.data)
    return out


def jacobian(prob, theta, trains, coil=None, mask=None):
    b = _Bound(prob)
    th = _f64(theta, (b.np, b.nv))
    tr = _c128(trains, (4, prob.n_tr, b.nv))
    cl, mk = _coil(b, coil), _mask(b, mask)
    rows = prob.n_coils * prob.n_tr * prob.n_read
    out = np.zeros((rows, b.np * b.nv), dtype=np.complex128)
    lib().oracle_jacobian(C.byref(b.s), th.ctypes.data, _ptr(cl), _ptr(mk),
                          tr.ctypes.data, out.ctypes.data)
    return out


def residual(prob, theta, data, coil=None, mask=None):
    """Returns (f, r) with r = d - s(theta), f = 0.5 ||r||^2."""
    b = _Bound(prob)
    th = _f64(theta, (b.np, b.nv))
    d = _c128(data, _dshape(prob))
    cl, mk = _coil(b, coil), _mask(b, mask)
    r = np.zeros(_dshape(prob), dtype=np.complex128)
    f = lib().oracle_residual(C.byref(b.s), th.ctypes.data, _ptr(cl), _ptr(mk),
                              d.ctypes.data, r.ctypes.data)
    return f, r


def gn_step(prob, theta, data, n_cg, param_mask, lo, hi, n_ls_max=8, armijo_c1=1e-4,
            coil=None, mask=None):
    """One inexact GN iteration; returns (theta_new, GnReport)."""
    b = _Bound(prob)
    th = _f64(theta, (b.np, b.nv)).copy()
    d = _c128(data, _dshape(prob))
    cl, mk = _coil(b, coil), _mask(b, mask)
    o = _GnOpts(n_cg, n_ls_max, param_mask, (C.c_double * 3)(*lo), (C.c_double * 3)(*hi),
                armijo_c1)
    rep = _GnReport()
    lib().oracle_gn_step(C.byref(b.s), th.ctypes.data, _ptr(cl), _ptr(mk), d.ctypes.data,
                         C.byref(o), C.byref(rep))
    return th, GnReport(rep.f0, rep.f1, rep.gnorm, rep.step_norm, rep.t,
                        rep.cg_iters, rep.ls_trials, rep.accepted)


def rho_init(prob, theta, data, n_iter=20, coil=None, mask=None):
    """CGLS least-squares rho for fixed (T1, T2, B1); returns a new theta."""
    b = _Bound(prob)
    th = _f64(theta, (b.np, b.nv)).copy()
    d = _c128(data, _dshape(prob))
    cl, mk = _coil(b, coil), _mask(b, mask)
    lib().oracle_rho_init(C.byref(b.s), th.ctypes.data, _ptr(cl), _ptr(mk), d.ctypes.data,
                          n_iter)
    return th


def steihaug_dense(B, g, delta, n_cg):
    """Steihaug truncated CG on a dense symmetric B; returns (p, exit kind, iters)."""
    B = np.ascontiguousarray(B, dtype=np.float64)
    n = B.shape[0]
    g = _f64(g, (n,))
    p = np.zeros(n)
    it = C.c_int(0)
    kind = lib().oracle_steihaug_dense(n, B.ctypes.data, g.ctypes.data, float(delta), int(n_cg),
                                       p.ctypes.data, C.byref(it))
    return p, int(kind), int(it.value)


def reflect(x, lo, hi):
    return float(lib().oracle_reflect(float(x), float(lo), float(hi)))


def tr_step(prob, theta, data, delta, n_cg, param_mask, lo, hi, eta=0.1, delta_max=1e3,
            coil=None, mask=None):
    """One trust-region inexact GN iteration; returns (theta_new, delta_new, report dict)."""
    b = _Bound(prob)
    th = _f64(theta, (b.np, b.nv)).copy()
    d = _c128(data, _dshape(prob))
    cl, mk = _coil(b, coil), _mask(b, mask)
    o = _TrOpts(n_cg, param_mask, (C.c_double * 3)(*lo), (C.c_double * 3)(*hi), eta, delta_max)
    dl = C.c_double(delta)
    rep = _TrReport()
    lib().oracle_tr_step(C.byref(b.s), th.ctypes.data, _ptr(cl), _ptr(mk), d.ctypes.data,
                         C.byref(o), C.byref(dl), C.byref(rep))
    return th, float(dl.value), rep.as_dict()


def isochromat(prob, lnT1, lnT2, B1, scale=1.0):
    """One isochromat of the balanced model: [4][n_tr] complex (m and its
    derivatives in ln T1, ln T2, B1)."""
    b = _Bound(prob)
    out = np.zeros((4, prob.n_tr), dtype=np.complex128)
    lib().oracle_isochromat(C.byref(b.s), float(lnT1), float(lnT2), float(B1), float(scale),
                            out[0].ctypes.data, out[1].ctypes.data, out[2].ctypes.data, out[3].ctypes.data)
    return out
