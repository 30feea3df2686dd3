/*
 * mrstat.h - C ABI of the MI355X (gfx950) MR-STAT hot path.
 *
 * The library evaluates the matrix-free products of the inexact Gauss-Newton
 * MR-STAT reconstruction of van der Heide, Sbrizzi, Luijten and van den Berg
 * ("High resolution in-vivo MR-STAT using a matrix-free and parallelized
 * reconstruction algorithm", NMR in Biomedicine 2019, arXiv 1904.13244):
 * the signal and residual (Theory, eq. 1 discretised, and Algorithm 2), the
 * Jacobian products J v and Re(J^H w) (Theory, gradient section, Algorithm 4,
 * and the matrix-free Gauss-Newton products around eq. 4), and one inexact
 * Gauss-Newton step (Algorithm 6).
 *
 * Signal model. A gradient-spoiled transient-state sequence simulated per
 * voxel by the extended phase graph (EPG, K states), with forward-mode
 * derivatives in ln T1, ln T2 and B1 (the algorithmic differentiation of
 * Supporting Information S2, applied to EPG states), weighted by complex
 * proton density rho and per-coil sensitivity, and contracted with the
 * Cartesian encoding phases
 *     E[n,k,j] = exp(-2 pi i [ (k - Nk/2)(ix - nx/2)/Nk
 *                             + (l(n) - ny/2)(iy - ny/2)/ny ])
 * (voxel j = iy*nx + ix, readout sample k, TR n sampling line l(n)).
 *
 * Parameters. theta is float32 [5][Nv], Nv = nx*ny, in the paper's
 * parameter-major layout (voxel j's parameters at j + p*Nv, Theory section):
 *     p = 0: ln T1 [s], 1: ln T2 [s], 2: B1 [a.u.], 3: Re rho, 4: Im rho
 * (log scaling of T1 and T2: Methods, Reconstructions).
 *
 * Sign conventions (Theory): r = d - s, f = 0.5 ||r||^2, J = dr/dalpha
 * (so J = -ds/dalpha), gradient g = Re(J^H r).
 *
 * Memory and ownership. Every array argument named d_* is a DEVICE pointer
 * owned by the caller; h_* arguments are HOST pointers. The library never
 * allocates device memory: all scratch lives in one caller-provided
 * workspace (mrstat_workspace_bytes / mrstat_bind). The library owns only the
 * host-side context. Complex arrays are interleaved complex64 (re, im).
 *
 * Streams. Every call is enqueued on the given stream (a hipStream_t passed as
 * void*, NULL = the default stream) and is asynchronous, except the calls
 * that return host scalars (mrstat_residual with h_f != NULL, mrstat_gn_step,
 * mrstat_rho_init), which synchronise that stream. A context is not
 * thread-safe; calls on one context that overlap on different streams race.
 *
 * Errors. Every call returns a status; no exception crosses the ABI. The text
 * of the last error on a context is returned by mrstat_last_error(ctx)
 * (mrstat_last_error(NULL) for mrstat_create failures). After an error the
 * outputs of that call are undefined; the context stays usable.
 */
#ifndef MRSTAT_H
#define MRSTAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mrstat_ctx_s *mrstat_ctx;
typedef void *mrstat_stream; /* hipStream_t */

typedef enum {
    MRSTAT_OK = 0,
    MRSTAT_ERR_ARG = -1,         /* null pointer or invalid scalar argument */
    MRSTAT_ERR_SHAPE = -2,       /* sizes outside what the kernels support */
    MRSTAT_ERR_HIP = -3,         /* a HIP runtime call failed (text has the HIP error) */
    MRSTAT_ERR_WORKSPACE = -4,   /* workspace missing, too small or misaligned */
    MRSTAT_ERR_NONFINITE = -5,   /* objective evaluated to NaN/Inf */
    MRSTAT_ERR_STATE = -6,       /* reuse requested without a valid linearisation */
    MRSTAT_ERR_UNSUPPORTED = -7  /* valid input the library does not implement */
} mrstat_status;

/* Precision of the x-direction encoding contraction (a dense complex GEMM on
 * the matrix cores): plain FP32, split-BF16 (hi + lo operands, three BF16
 * products hi*hi + hi*lo + lo*hi, FP32 accumulation) or FP16 (one product,
 * FP32 accumulation). All other arithmetic is FP32 with FP64 reductions. */
typedef enum {
    MRSTAT_ENC_FP32 = 0,
    MRSTAT_ENC_SPLIT_BF16 = 1,
    MRSTAT_ENC_FP16 = 2
} mrstat_enc;

/* Sequence and grid. Host arrays are read during mrstat_create only.
 * Requirements: nx, ny >= 1; n_tr >= 1; n_read >= nx; 1 <= n_states <= 64;
 * 1 <= n_coils <= 16; 0 <= te_s <= tr_s; t_inv_s >= 0; every ky_line in
 * [0, ny); every RF phase 0 or pi (modulo 2 pi): these keep the EPG states
 * purely imaginary (F) / real (Z), the form the kernels use; other phases
 * return MRSTAT_ERR_UNSUPPORTED. */
typedef struct {
    int32_t nx, ny;       /* image grid; voxel j = iy*nx + ix */
    int32_t n_tr;         /* TRs = readouts */
    int32_t n_read;       /* samples per readout (oversampled readout: n_read > nx) */
    int32_t n_states;     /* EPG truncation K */
    int32_t n_coils;      /* receive coils C */
    double tr_s, te_s;    /* repetition and echo time [s] */
    double t_inv_s;       /* delay from the ideal inversion to the first RF [s] */
    const double *flip_deg;      /* [n_tr] flip angle per TR [degrees] */
    const double *rf_phase_rad;  /* [n_tr] RF phase per TR, or NULL = all 0 */
    const int32_t *ky_line;      /* [n_tr] phase-encode line per TR, or NULL = n mod ny */
} mrstat_problem;

/* Inexact Gauss-Newton options (Algorithm 6 with a line search). */
typedef struct {
    int32_t n_cg;         /* CG iterations on Re(J^H J) p = -g (eq. 4); exact count,
                             early exit only on breakdown (zero residual or
                             non-positive curvature) */
    int32_t n_ls_max;     /* backtracking trials t = 1, 1/2, ... (>= 1) */
    int32_t param_mask;   /* bit p set = parameter p is reconstructed */
    float lo[3], hi[3];   /* projection box for ln T1, ln T2, B1 */
    double armijo_c1;     /* sufficient decrease: f(a_t) <= f + c1 g^T (a_t - a) */
} mrstat_gn_opts;

typedef struct {
    double f0;            /* f at the incoming theta */
    double f1;            /* f at the returned theta (= f0 if no step accepted) */
    double gnorm;         /* ||g|| over active entries */
    double step_norm;     /* ||theta_out - theta_in|| */
    double t;             /* accepted step length (0 if none) */
    int32_t cg_iters;     /* CG iterations performed */
    int32_t ls_trials;    /* objective evaluations in the line search */
    int32_t accepted;     /* 1 if theta was updated */
    int32_t reserved;
} mrstat_gn_report;

/* Validates the problem and builds the host context (no device work). */
mrstat_status mrstat_create(const mrstat_problem *prob, mrstat_ctx *out);
void mrstat_destroy(mrstat_ctx ctx);
const char *mrstat_last_error(mrstat_ctx ctx);

/* Bytes of device workspace the context needs (256-byte aligned start). */
size_t mrstat_workspace_bytes(mrstat_ctx ctx);

/* Attaches the workspace and optional coil / voxel masks, and uploads the
 * per-problem tables (flip angles, encoding phases) into the workspace.
 *   d_coil: complex64 [n_coils][Nv], or NULL when n_coils == 1 (sensitivity 1).
 *   d_mask: uint8 [Nv] (0 = voxel excluded: it contributes nothing to s and
 *           its Jacobian columns and gradient entries are 0), or NULL = all.
 * The caller keeps d_ws, d_coil and d_mask alive and unchanged until the
 * context is destroyed or re-bound. Synchronises the stream. */
mrstat_status mrstat_bind(mrstat_ctx ctx, void *d_ws, size_t ws_bytes,
                          const void *d_coil, const uint8_t *d_mask, mrstat_stream stream);

mrstat_status mrstat_set_encoding(mrstat_ctx ctx, mrstat_enc enc);

/* Tuning: lanes per voxel of the EPG kernel (the K states of a voxel are split
 * over a group of `lanes` lanes: 1, 2, 4 or 8; 0 = automatic choice). Results
 * do not depend on the choice beyond FP32 rounding order (they are identical
 * in practice: every order is updated by the same arithmetic). */
mrstat_status mrstat_set_epg_lanes(mrstat_ctx ctx, int32_t lanes);

/* Linearise at theta: EPG trains m, dm/dlnT1, dm/dlnT2, dm/dB1 per voxel and
 * TR into the workspace; if d_trains != NULL also copy them out as float32
 * [4][n_tr][Nv] holding the imaginary parts (the real parts are exactly 0
 * under the supported RF phases). The trains are m_j[n] = F+_0 e^{-i phi_n}
 * at TE of TR n (sampled once per readout, no decay during the readout). */
mrstat_status mrstat_simulate(mrstat_ctx ctx, const float *d_theta, float *d_trains,
                              mrstat_stream stream);

/* r = d - s(theta), s_c[n,k] = sum_j C_c[j] rho_j m_j[n] E[n,k,j]
 * (Algorithm 2 matrix-free), complex64 [n_coils][n_tr][n_read] in and out.
 * reuse_linearization = 1 asserts theta is unchanged since the last
 * linearisation on this context (mrstat_simulate, or any call with reuse 0)
 * and skips the EPG; 0 re-linearises. If h_f != NULL, *h_f = 0.5 ||r||^2
 * reduced in FP64 and the stream is synchronised. */
mrstat_status mrstat_residual(mrstat_ctx ctx, const float *d_theta, int32_t reuse_linearization,
                              const void *d_data, void *d_r, double *h_f, mrstat_stream stream);

/* d_out = J v for v float32 [5][Nv]; complex64 [n_coils][n_tr][n_read].
 * All five parameter rows are used. */
mrstat_status mrstat_jv(mrstat_ctx ctx, const float *d_theta, int32_t reuse_linearization,
                        const float *d_v, void *d_out, mrstat_stream stream);

/* d_out = Re(J^H w) for w complex64 [n_coils][n_tr][n_read]; float32 [5][Nv]
 * (Algorithm 4: all N_p partial derivatives of a voxel together). */
mrstat_status mrstat_jhw(mrstat_ctx ctx, const float *d_theta, int32_t reuse_linearization,
                         const void *d_w, float *d_out, mrstat_stream stream);

/* One inexact Gauss-Newton iteration (Algorithm 6): linearise at theta,
 * r, f, g = Re(J^H r); exactly n_cg CG iterations on Re(J^H J) p = -g with
 * FP64 dot products and scalars kept on the device; backtracking line search
 * theta_t = P(theta + t p), P the box projection of (ln T1, ln T2, B1),
 * accepting the first t with f(theta_t) <= f + c1 g^T (theta_t - theta).
 * d_theta is updated in place only when a trial is accepted. Inactive
 * parameters (param_mask) and masked voxels never change. Synchronises. */
mrstat_status mrstat_gn_step(mrstat_ctx ctx, float *d_theta, const void *d_data,
                             const mrstat_gn_opts *opts, mrstat_gn_report *h_rep,
                             mrstat_stream stream);

/* Proton-density initialisation (Methods, Reconstructions): least-squares
 * rho solving M(alpha0) rho = d for the current (T1, T2, B1) rows of theta,
 * by n_iter CGLS iterations from rho = 0 (CGLS equals LSQR in exact
 * arithmetic) with FP64 reductions. Rows 3 and 4 of d_theta are overwritten.
 * Leaves the context linearised at the returned theta. Synchronises. */
mrstat_status mrstat_rho_init(mrstat_ctx ctx, float *d_theta, const void *d_data, int32_t n_iter,
                              mrstat_stream stream);

/* Kernel tracing. While enabled, every kernel the context launches is
 * bracketed by HIP events on its stream. mrstat_profile_read synchronises the
 * recorded events and returns, per kernel kind, the number of launches and
 * their summed device time in milliseconds since profiling was (re-)enabled.
 * Enabling or disabling resets the counters. Host memory only; the events are
 * created on first use and kept by the context. */
typedef enum {
    MRSTAT_K_EPG = 0,        /* EPG with tangents (linearisation) */
    MRSTAT_K_EPG_VALUE = 1,  /* EPG value only (line-search trials) */
    MRSTAT_K_YFWD_SIG = 2,   /* forward y-stage of the signal (m train only) */
    MRSTAT_K_YFWD_JV = 3,    /* forward y-stage of J v (all four trains) */
    MRSTAT_K_XFWD = 4,       /* forward x-stage GEMM (+ residual epilogue) */
    MRSTAT_K_XADJ = 5,       /* adjoint x-stage GEMM */
    MRSTAT_K_YADJ = 6,       /* adjoint y-stage (train streaming) */
    MRSTAT_K_FINISH = 7,     /* gradient assembly from the adjoint partials */
    MRSTAT_K_VECTOR = 8,     /* CG / line-search / CGLS vector kernels and reductions */
    MRSTAT_K_COUNT = 9
} mrstat_kernel_kind;

mrstat_status mrstat_profile_enable(mrstat_ctx ctx, int32_t on);
mrstat_status mrstat_profile_read(mrstat_ctx ctx, int32_t *h_counts, double *h_ms);

#ifdef __cplusplus
}
#endif
#endif /* MRSTAT_H */
