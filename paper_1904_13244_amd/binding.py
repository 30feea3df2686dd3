"""Thin ctypes binding of libmrstat (include/mrstat.h).

The functions below carry the C names and only marshal arguments: torch
tensors are checked for device, dtype, shape and contiguity and passed as raw
device pointers together with the current HIP stream. Every step of the
computation runs in the HIP kernels of libmrstat.so; there is no fallback:
if the library is missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmrstat.so")

OK, ERR_ARG, ERR_SHAPE, ERR_HIP, ERR_WORKSPACE, ERR_NONFINITE, ERR_STATE, ERR_UNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6, -7)
ENC_FP32, ENC_SPLIT_BF16, ENC_FP16 = 0, 1, 2
TRAINS_FP32, TRAINS_FP16 = 0, 1
_STATUS = {0: "OK", -1: "ERR_ARG", -2: "ERR_SHAPE", -3: "ERR_HIP", -4: "ERR_WORKSPACE",
           -5: "ERR_NONFINITE", -6: "ERR_STATE", -7: "ERR_UNSUPPORTED"}


class MrstatError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Problem(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("n_tr", C.c_int32), ("n_read", C.c_int32),
                ("n_states", C.c_int32), ("n_coils", C.c_int32),
                ("tr_s", C.c_double), ("te_s", C.c_double), ("t_inv_s", C.c_double),
                ("flip_deg", C.POINTER(C.c_double)), ("rf_phase_rad", C.POINTER(C.c_double)),
                ("ky_line", C.POINTER(C.c_int32))]


class GnOpts(C.Structure):
    _fields_ = [("n_cg", C.c_int32), ("n_ls_max", C.c_int32), ("param_mask", C.c_int32),
                ("lo", C.c_float * 3), ("hi", C.c_float * 3), ("armijo_c1", C.c_double)]


class GnReport(C.Structure):
    _fields_ = [("f0", C.c_double), ("f1", C.c_double), ("gnorm", C.c_double),
                ("step_norm", C.c_double), ("t", C.c_double), ("cg_iters", C.c_int32),
                ("ls_trials", C.c_int32), ("accepted", C.c_int32), ("n_fallback", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TrOpts(C.Structure):
    _fields_ = [("n_cg", C.c_int32), ("param_mask", C.c_int32), ("lo", C.c_float * 3),
                ("hi", C.c_float * 3), ("eta", C.c_double), ("delta_max", C.c_double)]


class TrReport(C.Structure):
    _fields_ = [("f0", C.c_double), ("f1", C.c_double), ("gnorm", C.c_double),
                ("step_norm", C.c_double), ("rho", C.c_double), ("pred", C.c_double),
                ("delta_in", C.c_double), ("delta_out", C.c_double), ("cg_iters", C.c_int32),
                ("exit_kind", C.c_int32), ("accepted", C.c_int32), ("n_reflected", C.c_int32),
                ("n_fallback", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


TR_ITERS, TR_BOUNDARY, TR_CURVATURE, TR_ZERO = 0, 1, 2, 3

_lib = None


def lib():
    """Loads libmrstat.so (built by paper_1904_13244_amd.build); raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_1904_13244_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, P = C.c_void_p, C.c_int32, C.POINTER
        sig = {
            "mrstat_create": ([P(Problem), P(vp)], C.c_int),
            "mrstat_create_traj": ([P(Problem), vp, vp, P(vp)], C.c_int),
            "mrstat_create_readout": ([P(Problem), C.c_double, C.c_double, C.c_double, P(vp)],
                                      C.c_int),
            "mrstat_set_db0": ([vp, vp], C.c_int),
            "mrstat_readout_terms": ([vp, P(i32)], C.c_int),
            "mrstat_readout_cheb_terms": ([vp, P(i32)], C.c_int),
            "mrstat_fit_db0": ([vp, C.c_double], C.c_int),
            "mrstat_destroy": ([vp], None),
            "mrstat_last_error": ([vp], C.c_char_p),
            "mrstat_workspace_bytes": ([vp], C.c_size_t),
            "mrstat_bind": ([vp, vp, C.c_size_t, vp, vp, vp], C.c_int),
            "mrstat_bind_static": ([vp, vp, vp, vp], C.c_int),
            "mrstat_set_encoding": ([vp, C.c_int], C.c_int),
            "mrstat_set_epg_lanes": ([vp, i32], C.c_int),
            "mrstat_set_isochromats": ([vp, i32, P(C.c_double), P(C.c_double)], C.c_int),
            "mrstat_set_train_precision": ([vp, C.c_int], C.c_int),
            "mrstat_simulate": ([vp, vp, vp, vp], C.c_int),
            "mrstat_residual": ([vp, vp, i32, vp, vp, P(C.c_double), vp], C.c_int),
            "mrstat_jv": ([vp, vp, i32, vp, vp, vp], C.c_int),
            "mrstat_jhw": ([vp, vp, i32, vp, vp, vp], C.c_int),
            "mrstat_gn_step": ([vp, vp, vp, P(GnOpts), P(GnReport), vp], C.c_int),
            "mrstat_rho_init": ([vp, vp, vp, i32, vp], C.c_int),
            "mrstat_tr_step": ([vp, vp, vp, P(TrOpts), P(C.c_double), P(TrReport), vp], C.c_int),
            "mrstat_profile_enable": ([vp, i32], C.c_int),
            "mrstat_profile_read": ([vp, P(i32), P(C.c_double)], C.c_int),
            "mrstat_profile_select": ([vp, C.c_uint32], C.c_int),
            "mrstat_set_surrogate": ([vp, vp], C.c_int),
            "mrstat_fallback_count": ([vp, P(i32), vp], C.c_int),
            "mrstat_mlp_create": ([i32, i32, i32, i32, P(vp)], C.c_int),
            "mrstat_mlp_destroy": ([vp], None),
            "mrstat_mlp_last_error": ([vp], C.c_char_p),
            "mrstat_mlp_param_count": ([vp], C.c_size_t),
            "mrstat_mlp_workspace_bytes": ([vp], C.c_size_t),
            "mrstat_mlp_bind": ([vp, vp, C.c_size_t, vp], C.c_int),
            "mrstat_mlp_set_scaling": ([vp, P(C.c_float), P(C.c_float), P(C.c_float), vp], C.c_int),
            "mrstat_mlp_fit_scaling": ([vp, vp, C.c_int64, P(C.c_float), P(C.c_float),
                                        P(C.c_float), vp], C.c_int),
            "mrstat_mlp_set_params": ([vp, vp, vp], C.c_int),
            "mrstat_mlp_get_params": ([vp, vp, vp], C.c_int),
            "mrstat_mlp_gradients": ([vp, vp, C.c_int64, vp, C.c_int64, vp, P(C.c_double), vp],
                                     C.c_int),
            "mrstat_mlp_train_step": ([vp, vp, C.c_int64, vp, C.c_int64, C.c_float,
                                       P(C.c_double), vp], C.c_int),
            "mrstat_mlp_predict": ([vp, vp, C.c_int64, i32, vp, vp], C.c_int),
            "mrstat_mlp_set_infer_tile": ([vp, i32], C.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def exported_symbols():
    return ["mrstat_create", "mrstat_destroy", "mrstat_last_error", "mrstat_workspace_bytes",
            "mrstat_bind", "mrstat_set_encoding", "mrstat_set_epg_lanes", "mrstat_simulate", "mrstat_residual", "mrstat_jv",
            "mrstat_jhw", "mrstat_gn_step", "mrstat_rho_init", "mrstat_profile_enable",
            "mrstat_profile_read", "mrstat_set_surrogate", "mrstat_fallback_count",
            "mrstat_mlp_create", "mrstat_mlp_destroy", "mrstat_mlp_last_error",
            "mrstat_mlp_param_count", "mrstat_mlp_workspace_bytes", "mrstat_mlp_bind",
            "mrstat_mlp_set_scaling", "mrstat_mlp_fit_scaling", "mrstat_mlp_set_params",
            "mrstat_mlp_get_params", "mrstat_mlp_gradients", "mrstat_mlp_train_step",
            "mrstat_mlp_predict", "mrstat_mlp_set_infer_tile", "mrstat_set_train_precision",
            "mrstat_profile_select", "mrstat_bind_static", "mrstat_tr_step", "mrstat_create_traj",
            "mrstat_set_isochromats", "mrstat_create_readout", "mrstat_set_db0",
            "mrstat_readout_terms", "mrstat_readout_cheb_terms", "mrstat_fit_db0"]


def _check(status, ctx=None):
    if status != OK:
        msg = lib().mrstat_last_error(ctx)
        raise MrstatError(status, msg.decode() if msg else "")


def _check_mlp(status, net):
    if status != OK:
        msg = lib().mrstat_mlp_last_error(net) if net else b""
        raise MrstatError(status, msg.decode() if msg else "")


# --------------------------------------------------------------- C-named calls
def mrstat_create(prob):
    """prob: object with nx, ny, n_tr, n_read, n_states, n_coils, tr, te, t_inv,
    flip_deg, rf_phase, ky_line and optionally traj = (kx, ky) [n_tr][n_read]
    cycles per field of view (non-Cartesian: mrstat_create_traj), and
    optionally dwell > 0 with the bounds rd_min_t2, rd_max_db0 (readout
    dynamics: mrstat_create_readout). Returns the context handle."""
    flip = np.ascontiguousarray(prob.flip_deg, dtype=np.float64)
    phase = np.ascontiguousarray(prob.rf_phase, dtype=np.float64)
    ky = np.ascontiguousarray(prob.ky_line, dtype=np.int32)
    s = Problem(prob.nx, prob.ny, prob.n_tr, prob.n_read, prob.n_states, prob.n_coils,
                prob.tr, prob.te, prob.t_inv,
                flip.ctypes.data_as(C.POINTER(C.c_double)),
                phase.ctypes.data_as(C.POINTER(C.c_double)),
                ky.ctypes.data_as(C.POINTER(C.c_int32)))
    h = C.c_void_p()
    traj = getattr(prob, "traj", None)
    dwell = float(getattr(prob, "dwell", 0.0) or 0.0)
    if dwell > 0.0:
        if traj is not None:
            raise ValueError("readout dynamics take a Cartesian encoding")
        _check(lib().mrstat_create_readout(C.byref(s), dwell, float(prob.rd_min_t2),
                                           float(prob.rd_max_db0), C.byref(h)))
    elif traj is None:
        _check(lib().mrstat_create(C.byref(s), C.byref(h)))
    else:
        kx = np.ascontiguousarray(traj[0], dtype=np.float64)
        ky = np.ascontiguousarray(traj[1], dtype=np.float64)
        if kx.shape != (prob.n_tr, prob.n_read) or ky.shape != kx.shape:
            raise ValueError("trajectory arrays must be [n_tr][n_read]")
        _check(lib().mrstat_create_traj(C.byref(s), kx.ctypes.data, ky.ctypes.data, C.byref(h)))
    return h


def mrstat_destroy(ctx):
    lib().mrstat_destroy(ctx)


def mrstat_workspace_bytes(ctx):
    return int(lib().mrstat_workspace_bytes(ctx))


def mrstat_bind(ctx, ws_ptr, ws_bytes, coil_ptr, mask_ptr, stream):
    _check(lib().mrstat_bind(ctx, ws_ptr, ws_bytes, coil_ptr, mask_ptr, stream), ctx)


def mrstat_bind_static(ctx, coil_ptr, mask_ptr, stream):
    _check(lib().mrstat_bind_static(ctx, coil_ptr, mask_ptr, stream), ctx)


def mrstat_set_encoding(ctx, enc):
    _check(lib().mrstat_set_encoding(ctx, enc), ctx)


def mrstat_set_train_precision(ctx, prec):
    _check(lib().mrstat_set_train_precision(ctx, int(prec)), ctx)


def mrstat_set_isochromats(ctx, scale, weight):
    sc = np.ascontiguousarray(scale, dtype=np.float64)
    wt = np.ascontiguousarray(weight, dtype=np.float64)
    if sc.shape != wt.shape or sc.ndim != 1:
        raise ValueError("scale and weight must be 1-d arrays of one length")
    _check(lib().mrstat_set_isochromats(ctx, int(sc.size), sc.ctypes.data_as(C.POINTER(C.c_double)),
                                        wt.ctypes.data_as(C.POINTER(C.c_double))), ctx)


def mrstat_set_db0(ctx, db0_ptr):
    _check(lib().mrstat_set_db0(ctx, db0_ptr), ctx)


def mrstat_fit_db0(ctx, hz_per_unit):
    _check(lib().mrstat_fit_db0(ctx, float(hz_per_unit)), ctx)


def mrstat_readout_terms(ctx):
    n = C.c_int32()
    _check(lib().mrstat_readout_terms(ctx, C.byref(n)), ctx)
    return int(n.value)


def mrstat_readout_cheb_terms(ctx):
    n = C.c_int32()
    _check(lib().mrstat_readout_cheb_terms(ctx, C.byref(n)), ctx)
    return int(n.value)


def mrstat_set_epg_lanes(ctx, lanes):
    _check(lib().mrstat_set_epg_lanes(ctx, int(lanes)), ctx)


def mrstat_simulate(ctx, theta_ptr, trains_ptr, stream):
    _check(lib().mrstat_simulate(ctx, theta_ptr, trains_ptr, stream), ctx)


def mrstat_residual(ctx, theta_ptr, reuse, data_ptr, r_ptr, want_f, stream):
    f = C.c_double(0.0)
    _check(lib().mrstat_residual(ctx, theta_ptr, int(reuse), data_ptr, r_ptr,
                                 C.byref(f) if want_f else None, stream), ctx)
    return f.value if want_f else None


def mrstat_jv(ctx, theta_ptr, reuse, v_ptr, out_ptr, stream):
    _check(lib().mrstat_jv(ctx, theta_ptr, int(reuse), v_ptr, out_ptr, stream), ctx)


def mrstat_jhw(ctx, theta_ptr, reuse, w_ptr, out_ptr, stream):
    _check(lib().mrstat_jhw(ctx, theta_ptr, int(reuse), w_ptr, out_ptr, stream), ctx)


def mrstat_gn_step(ctx, theta_ptr, data_ptr, opts: GnOpts, stream) -> GnReport:
    rep = GnReport()
    _check(lib().mrstat_gn_step(ctx, theta_ptr, data_ptr, C.byref(opts), C.byref(rep), stream), ctx)
    return rep


def mrstat_tr_step(ctx, theta_ptr, data_ptr, opts: TrOpts, delta, stream):
    """Returns (new trust radius, TrReport)."""
    rep = TrReport()
    dl = C.c_double(delta)
    _check(lib().mrstat_tr_step(ctx, theta_ptr, data_ptr, C.byref(opts), C.byref(dl), C.byref(rep),
                                stream), ctx)
    return dl.value, rep


def mrstat_rho_init(ctx, theta_ptr, data_ptr, n_iter, stream):
    _check(lib().mrstat_rho_init(ctx, theta_ptr, data_ptr, int(n_iter), stream), ctx)


def mrstat_set_surrogate(ctx, net):
    _check(lib().mrstat_set_surrogate(ctx, net), ctx)


def mrstat_fallback_count(ctx, stream):
    n = C.c_int32(0)
    _check(lib().mrstat_fallback_count(ctx, C.byref(n), stream), ctx)
    return int(n.value)


def mrstat_mlp_create(n_tr, width, depth, batch):
    h = C.c_void_p()
    _check_mlp(lib().mrstat_mlp_create(int(n_tr), int(width), int(depth), int(batch), C.byref(h)),
               None)
    return h


def mrstat_mlp_destroy(net):
    lib().mrstat_mlp_destroy(net)


def mrstat_mlp_param_count(net):
    return int(lib().mrstat_mlp_param_count(net))


def mrstat_mlp_workspace_bytes(net):
    return int(lib().mrstat_mlp_workspace_bytes(net))


def mrstat_mlp_bind(net, ws_ptr, ws_bytes, stream):
    _check_mlp(lib().mrstat_mlp_bind(net, ws_ptr, ws_bytes, stream), net)


def _f3(x, n):
    return (C.c_float * n)(*[float(v) for v in x])


def mrstat_mlp_set_scaling(net, lo, hi, head_scale, stream):
    _check_mlp(lib().mrstat_mlp_set_scaling(net, _f3(lo, 3), _f3(hi, 3), _f3(head_scale, 4), stream),
               net)


def mrstat_mlp_fit_scaling(net, trains_ptr, n, lo, hi, stream):
    out = (C.c_float * 4)()
    _check_mlp(lib().mrstat_mlp_fit_scaling(net, trains_ptr, int(n), _f3(lo, 3), _f3(hi, 3), out,
                                            stream), net)
    return [float(v) for v in out]


def mrstat_mlp_set_params(net, params_ptr, stream):
    _check_mlp(lib().mrstat_mlp_set_params(net, params_ptr, stream), net)


def mrstat_mlp_get_params(net, params_ptr, stream):
    _check_mlp(lib().mrstat_mlp_get_params(net, params_ptr, stream), net)


def mrstat_mlp_gradients(net, theta_ptr, ld_theta, trains_ptr, ld_trains, grad_ptr, want_loss,
                         stream):
    loss = C.c_double(0.0)
    _check_mlp(lib().mrstat_mlp_gradients(net, theta_ptr, int(ld_theta), trains_ptr, int(ld_trains),
                                          grad_ptr, C.byref(loss) if want_loss else None, stream),
               net)
    return loss.value if want_loss else None


def mrstat_mlp_train_step(net, theta_ptr, ld_theta, trains_ptr, ld_trains, lr, want_loss, stream):
    loss = C.c_double(0.0)
    _check_mlp(lib().mrstat_mlp_train_step(net, theta_ptr, int(ld_theta), trains_ptr, int(ld_trains),
                                           float(lr), C.byref(loss) if want_loss else None, stream),
               net)
    return loss.value if want_loss else None


def mrstat_mlp_set_infer_tile(net, voxels):
    _check_mlp(lib().mrstat_mlp_set_infer_tile(net, int(voxels)), net)


def mrstat_mlp_predict(net, theta_ptr, ld_theta, n, out_ptr, stream):
    _check_mlp(lib().mrstat_mlp_predict(net, theta_ptr, int(ld_theta), int(n), out_ptr, stream), net)


KERNEL_KINDS = ["epg", "epg_value", "ystage_fwd_signal", "ystage_fwd_jv", "xgemm_fwd",
                "xgemm_adj", "ystage_adj", "jhw_finish", "vector", "surrogate",
                "surrogate_value", "nc_fwd", "nc_adj"]


def mrstat_profile_enable(ctx, on):
    _check(lib().mrstat_profile_enable(ctx, 1 if on else 0), ctx)


def mrstat_profile_select(ctx, kinds=None):
    """Trace only the named kernel kinds (None = all)."""
    mask = 0xFFFFFFFF if kinds is None else sum(1 << KERNEL_KINDS.index(k) for k in kinds)
    _check(lib().mrstat_profile_select(ctx, mask), ctx)


def mrstat_profile_read(ctx):
    """{kind: (launches, total ms)} since profiling was enabled."""
    n = len(KERNEL_KINDS)
    counts = (C.c_int32 * n)()
    ms = (C.c_double * n)()
    _check(lib().mrstat_profile_read(ctx, counts, ms), ctx)
    return {k: (int(counts[i]), float(ms[i])) for i, k in enumerate(KERNEL_KINDS)}


# --------------------------------------------------------------- torch helper
@dataclass
class Context:
    """Owns a library context plus its workspace tensor (torch allocates all
    device memory; the library allocates none)."""
    prob: object
    coil: object = None      # torch complex64 [C][Nv] on the GPU, or None
    mask: object = None      # torch uint8 [Nv] on the GPU, or None
    static: bool = False     # True: the library's static workspace (mrstat_bind_static)

    def __post_init__(self):
        import torch
        self.torch = torch
        self.h = mrstat_create(self.prob)
        self.ws_bytes = mrstat_workspace_bytes(self.h)
        self.dev = torch.device("cuda", torch.cuda.current_device())
        nv = self.prob.nx * self.prob.ny
        if self.coil is not None:
            self._expect(self.coil, torch.complex64, (self.prob.n_coils, nv))
        if self.mask is not None:
            self._expect(self.mask, torch.uint8, (nv,))
        coil = self.coil.data_ptr() if self.coil is not None else None
        mask = self.mask.data_ptr() if self.mask is not None else None
        iso = getattr(self.prob, "iso", None)
        if iso is not None:
            mrstat_set_isochromats(self.h, iso[0], iso[1])
        self.np = 5
        unit = float(getattr(self.prob, "db0_unit", 0.0) or 0.0)
        if unit > 0.0:
            mrstat_fit_db0(self.h, unit)
            self.np = 6
        self.db0 = None
        db0 = getattr(self.prob, "db0", None)
        if db0 is not None and float(getattr(self.prob, "dwell", 0.0) or 0.0) > 0.0:
            # the library reads the map in place: the context keeps it alive
            self.db0 = torch.as_tensor(np.asarray(db0, dtype=np.float32)).to(self.dev)
            if tuple(self.db0.shape) != (nv,):
                raise ValueError(f"db0 must have shape ({nv},)")
            mrstat_set_db0(self.h, self.db0.data_ptr())
        if self.static:
            self.ws = None
            mrstat_bind_static(self.h, coil, mask, self.stream)
            return
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.dev)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) // 256 * 256
        mrstat_bind(self.h, self.ws_ptr, self.ws_bytes, coil, mask, self.stream)

    # -- helpers
    @property
    def stream(self):
        return self.torch.cuda.current_stream().cuda_stream

    def _expect(self, t, dtype, shape):
        if not isinstance(t, self.torch.Tensor):
            raise TypeError("expected a torch tensor")
        if t.device.type != "cuda" or t.dtype != dtype or tuple(t.shape) != tuple(shape) \
                or not t.is_contiguous():
            raise ValueError(f"expected contiguous {dtype} {tuple(shape)} on the GPU, got "
                             f"{t.dtype} {tuple(t.shape)} on {t.device}")

    @property
    def nv(self):
        return self.prob.nx * self.prob.ny

    @property
    def data_shape(self):
        return (self.prob.n_coils, self.prob.n_tr, self.prob.n_read)

    def close(self):
        if getattr(self, "h", None):
            self.torch.cuda.synchronize()
            mrstat_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- calls
    def set_encoding(self, enc):
        mrstat_set_encoding(self.h, enc)

    def profile(self, on=True):
        mrstat_profile_enable(self.h, on)

    def profile_read(self):
        return mrstat_profile_read(self.h)

    def profile_select(self, kinds=None):
        mrstat_profile_select(self.h, kinds)

    def set_epg_lanes(self, lanes):
        mrstat_set_epg_lanes(self.h, lanes)

    def readout_terms(self):
        return mrstat_readout_terms(self.h)

    def readout_cheb_terms(self):
        return mrstat_readout_cheb_terms(self.h)

    def set_train_precision(self, prec):
        mrstat_set_train_precision(self.h, prec)

    def simulate(self, theta, trains=None):
        T = self.torch
        self._expect(theta, T.float32, (self.np, self.nv))
        if trains is None:
            trains = T.empty((4, self.prob.n_tr, self.nv), dtype=T.float32, device=self.dev)
        self._expect(trains, T.float32, (4, self.prob.n_tr, self.nv))
        mrstat_simulate(self.h, theta.data_ptr(), trains.data_ptr(), self.stream)
        return trains

    def linearise(self, theta):
        self._expect(theta, self.torch.float32, (self.np, self.nv))
        mrstat_simulate(self.h, theta.data_ptr(), None, self.stream)

    def residual(self, theta, data, reuse=False, out=None, want_f=True):
        T = self.torch
        self._expect(theta, T.float32, (self.np, self.nv))
        self._expect(data, T.complex64, self.data_shape)
        if out is None:
            out = T.empty(self.data_shape, dtype=T.complex64, device=self.dev)
        self._expect(out, T.complex64, self.data_shape)
        f = mrstat_residual(self.h, theta.data_ptr(), reuse, data.data_ptr(), out.data_ptr(),
                            want_f, self.stream)
        return f, out

    def jv(self, theta, v, reuse=False, out=None):
        T = self.torch
        self._expect(theta, T.float32, (self.np, self.nv))
        self._expect(v, T.float32, (self.np, self.nv))
        if out is None:
            out = T.empty(self.data_shape, dtype=T.complex64, device=self.dev)
        self._expect(out, T.complex64, self.data_shape)
        mrstat_jv(self.h, theta.data_ptr(), reuse, v.data_ptr(), out.data_ptr(), self.stream)
        return out

    def jhw(self, theta, w, reuse=False, out=None):
        T = self.torch
        self._expect(theta, T.float32, (self.np, self.nv))
        self._expect(w, T.complex64, self.data_shape)
        if out is None:
            out = T.empty((self.np, self.nv), dtype=T.float32, device=self.dev)
        self._expect(out, T.float32, (self.np, self.nv))
        mrstat_jhw(self.h, theta.data_ptr(), reuse, w.data_ptr(), out.data_ptr(), self.stream)
        return out

    def gn_step(self, theta, data, n_cg, param_mask, lo, hi, n_ls_max=8, armijo_c1=1e-4):
        T = self.torch
        self._expect(theta, T.float32, (self.np, self.nv))
        self._expect(data, T.complex64, self.data_shape)
        o = GnOpts(int(n_cg), int(n_ls_max), int(param_mask), (C.c_float * 3)(*lo),
                   (C.c_float * 3)(*hi), float(armijo_c1))
        return mrstat_gn_step(self.h, theta.data_ptr(), data.data_ptr(), o, self.stream)

    def tr_step(self, theta, data, delta, n_cg, param_mask, lo, hi, eta=0.1, delta_max=1e3):
        """One trust-region step; returns (new radius, TrReport)."""
        T = self.torch
        self._expect(theta, T.float32, (self.np, self.nv))
        self._expect(data, T.complex64, self.data_shape)
        o = TrOpts(int(n_cg), int(param_mask), (C.c_float * 3)(*lo), (C.c_float * 3)(*hi),
                   float(eta), float(delta_max))
        return mrstat_tr_step(self.h, theta.data_ptr(), data.data_ptr(), o, float(delta), self.stream)

    def rho_init(self, theta, data, n_iter=20):
        T = self.torch
        self._expect(theta, T.float32, (self.np, self.nv))
        self._expect(data, T.complex64, self.data_shape)
        mrstat_rho_init(self.h, theta.data_ptr(), data.data_ptr(), n_iter, self.stream)
        return theta

    def set_surrogate(self, net):
        """net: a Surrogate (kept alive here while set) or None for plain EPG."""
        mrstat_set_surrogate(self.h, net.h if net is not None else None)
        self._surrogate = net

    def fallback_count(self):
        return mrstat_fallback_count(self.h, self.stream)


class Surrogate:
    """Owns a surrogate network handle plus its workspace tensor."""

    def __init__(self, n_tr, width=256, depth=4, batch=4096):
        import torch
        self.torch = torch
        self.n_tr, self.width, self.depth, self.batch = n_tr, width, depth, batch
        self.h = mrstat_mlp_create(n_tr, width, depth, batch)
        self.n_params = mrstat_mlp_param_count(self.h)
        self.ws_bytes = mrstat_mlp_workspace_bytes(self.h)
        self.dev = torch.device("cuda", torch.cuda.current_device())
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.dev)
        self.ws_ptr = (self.ws.data_ptr() + 255) // 256 * 256
        mrstat_mlp_bind(self.h, self.ws_ptr, self.ws_bytes, self.stream)

    @property
    def stream(self):
        return self.torch.cuda.current_stream().cuda_stream

    def _expect(self, t, dtype, shape=None):
        T = self.torch
        if not isinstance(t, T.Tensor) or t.device.type != "cuda" or t.dtype != dtype \
                or not t.is_contiguous() or (shape is not None and tuple(t.shape) != tuple(shape)):
            raise ValueError(f"expected contiguous {dtype} {shape} on the GPU")

    def close(self):
        if getattr(self, "h", None):
            self.torch.cuda.synchronize()
            mrstat_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_infer_tile(self, voxels):
        mrstat_mlp_set_infer_tile(self.h, voxels)

    def set_scaling(self, lo, hi, head_scale):
        mrstat_mlp_set_scaling(self.h, lo, hi, head_scale, self.stream)

    def fit_scaling(self, trains, lo, hi):
        """trains: float32 [4][n_tr][n] on the GPU. Returns the head scales."""
        self._expect(trains, self.torch.float32)
        if trains.dim() != 3 or trains.shape[0] != 4 or trains.shape[1] != self.n_tr:
            raise ValueError("trains must be [4][n_tr][n]")
        return mrstat_mlp_fit_scaling(self.h, trains.data_ptr(), trains.shape[2], lo, hi, self.stream)

    def set_params(self, params):
        self._expect(params, self.torch.float32, (self.n_params,))
        mrstat_mlp_set_params(self.h, params.data_ptr(), self.stream)

    def get_params(self):
        out = self.torch.empty(self.n_params, dtype=self.torch.float32, device=self.dev)
        mrstat_mlp_get_params(self.h, out.data_ptr(), self.stream)
        return out

    def _batch_views(self, theta, trains, col):
        T = self.torch
        self._expect(theta, T.float32)
        self._expect(trains, T.float32)
        if theta.dim() != 2 or theta.shape[0] < 3 or trains.dim() != 3 or trains.shape[0] != 4 \
                or trains.shape[1] != self.n_tr:
            raise ValueError("theta must be [>=3][n], trains [4][n_tr][n]")
        n_th, n_tr = theta.shape[1], trains.shape[2]
        if col < 0 or col + self.batch > min(n_th, n_tr):
            raise ValueError("batch columns out of range")
        return (theta.data_ptr() + 4 * col, n_th, trains.data_ptr() + 4 * col, n_tr)

    def gradients(self, theta, trains, col=0, want_loss=True):
        """Loss gradient of the batch at columns [col, col + batch)."""
        th, ldt, tr, ldr = self._batch_views(theta, trains, col)
        g = self.torch.empty(self.n_params, dtype=self.torch.float32, device=self.dev)
        loss = mrstat_mlp_gradients(self.h, th, ldt, tr, ldr, g.data_ptr(), want_loss, self.stream)
        return loss, g

    def train_step(self, theta, trains, lr, col=0, want_loss=False):
        th, ldt, tr, ldr = self._batch_views(theta, trains, col)
        return mrstat_mlp_train_step(self.h, th, ldt, tr, ldr, lr, want_loss, self.stream)

    def predict(self, theta):
        T = self.torch
        self._expect(theta, T.float32)
        if theta.dim() != 2 or theta.shape[0] < 3:
            raise ValueError("theta must be [>=3][n]")
        n = theta.shape[1]
        out = T.empty((4, self.n_tr, n), dtype=T.float32, device=self.dev)
        mrstat_mlp_predict(self.h, theta.data_ptr(), n, n, out.data_ptr(), self.stream)
        return out
