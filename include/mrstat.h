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
 * Parameters. theta is float32 [Np][Nv], Nv = nx*ny, in the paper's
 * parameter-major layout (voxel j's parameters at j + p*Nv, Theory section):
 *     p = 0: ln T1 [s], 1: ln T2 [s], 2: B1 [a.u.], 3: Re rho, 4: Im rho
 * (log scaling of T1 and T2: Methods, Reconstructions), Np = 5; a context
 * that fits Delta B0 (mrstat_fit_db0) has Np = 6 with p = 5: Delta B0 in
 * units of its hz_per_unit. Directions v, gradients and param_mask follow Np.
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
typedef struct mrstat_mlp_s *mrstat_mlp;   /* surrogate network (see below) */
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

/* Storage of the linearisation's trains in the workspace: FP32, or FP16
 * (rounded to nearest from the FP32 simulation; relative rounding 2^-11,
 * halving the bytes the J v and J^H w y-stages stream). All arithmetic on
 * them stays FP32. */
typedef enum {
    MRSTAT_TRAINS_FP32 = 0,
    MRSTAT_TRAINS_FP16 = 1
} mrstat_trains;

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
    int32_t param_mask;   /* bit p set = parameter p is reconstructed (p < Np) */
    float lo[3], hi[3];   /* projection box for ln T1, ln T2, B1 (a fitted Delta B0
                             keeps to +-max_abs_db0_hz of mrstat_create_readout) */
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
    int32_t n_fallback;   /* voxels of the linearisation simulated by the EPG because they
                             lie outside the surrogate's box (0 without a surrogate) */
} mrstat_gn_report;

/* Validates the problem and builds the host context (no device work). */
mrstat_status mrstat_create(const mrstat_problem *prob, mrstat_ctx *out);

/* The same for non-Cartesian sampling (the method is not tied to Cartesian
 * trajectories: Introduction, Discussion): sample k of TR n lies at
 * (kx, ky)[n * n_read + k], host FP64 arrays in cycles per field of view
 * (the Cartesian grid is kx = (k - n_read/2) nx / n_read, ky = l(n) - ny/2),
 * read during the call only. The encoding phase is
 *     E[n,k,j] = exp(-2 pi i (kx (ix - nx/2) / nx + ky (iy - ny/2) / ny))
 * and every call of the context evaluates the voxel x sample contraction
 * directly on the matrix cores (FP32 or split-BF16; FP16 is refused) with
 * the phases generated on the fly; ky_line is ignored and n_read may be below
 * nx. The workspace (mrstat_workspace_bytes) then also holds the forward's
 * voxel values, complex FP32 [n_tr][nx ny]. Requirements as mrstat_create,
 * plus nx <= 256 (MRSTAT_ERR_SHAPE) and finite coordinates (MRSTAT_ERR_ARG). */
mrstat_status mrstat_create_traj(const mrstat_problem *prob, const double *kx, const double *ky,
                                 mrstat_ctx *out);
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

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): mrstat_bind
 * with the library's own static workspace of MRSTAT_STATIC_WORKSPACE_BYTES
 * (64 MiB) on the current device instead of a caller-provided one. The
 * library allocates nothing here or later; every device the library is
 * loaded on holds that array until the process ends. Arguments as for
 * mrstat_bind. Errors: MRSTAT_ERR_WORKSPACE (with the bytes needed) when
 * mrstat_workspace_bytes(ctx) exceeds the maximum; MRSTAT_ERR_HIP if the
 * array's device address cannot be looked up.
 * One array per device is shared by every context bound to it: a call binds
 * ctx to it and takes it from any context bound before on that device, whose
 * later calls then return MRSTAT_ERR_STATE (re-bind to use it again). The
 * array keeps the last call's contents; the binding rewrites the tables and
 * clears the device scalars, and every other part of the workspace is
 * written before it is read. Calls on contexts of one device that overlap in
 * time (other host threads, other streams) race on the array.
 * Synchronises the stream. */
#define MRSTAT_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
mrstat_status mrstat_bind_static(mrstat_ctx ctx, const void *d_coil, const uint8_t *d_mask,
                                 mrstat_stream stream);

mrstat_status mrstat_set_encoding(mrstat_ctx ctx, mrstat_enc enc);
/* Train storage precision (default FP32). Invalidates the linearisation. */
mrstat_status mrstat_set_train_precision(mrstat_ctx ctx, mrstat_trains prec);

/* Tuning: lanes per voxel of the EPG kernel (the K states of a voxel are split
 * over a group of `lanes` lanes: 1, 2, 4 or 8; 0 = automatic choice). Results
 * do not depend on the choice beyond FP32 rounding order (they are identical
 * in practice: every order is updated by the same arithmetic). */
mrstat_status mrstat_set_epg_lanes(mrstat_ctx ctx, int32_t lanes);

/* Readout dynamics (Discussion: the volumetric signal model follows T2 decay
 * and Delta B0 phase accumulation during each readout). Creates a Cartesian,
 * single-coil context like mrstat_create whose sample k of every readout is
 * taken at TE + tau_k, tau_k = (k - n_read/2) dwell_s, and whose voxel j's
 * magnetisation carries exp(-tau_k / T2_j) exp(-2 pi i db0_j (TE + tau_k))
 * (db0 in Hz from mrstat_set_db0, zero until set; the precession has the
 * sense of the encoding phase). The residual, J v, J^H w (whose ln T2 column
 * gains the readout decay's tau_k / T2 term), the GN and trust-region steps
 * and the rho initialisation all use this model; the linearisation (the
 * trains at TE) is unchanged, since for the gradient-spoiled EPG model an
 * off-resonance changes the echo by its phase only. On the GPU the factor
 * exp(lambda tau), lambda = -1/T2 - 2 pi i db0, is expanded in powers of
 * tau / tau_max (tau_max = (n_read/2) dwell_s) for the forward products and
 * in Chebyshev polynomials of tau / tau_max for the adjoint ones, each with as
 * many terms (8 to 32; the power series' count from mrstat_readout_terms, the
 * Chebyshev count at most that) as keep the remainder below 1e-7 for
 * T2 >= min_t2_s and |db0| <= max_abs_db0_hz; every product then streams the
 * trains once per term set and runs its x-GEMMs over all terms. GN and trust-region steps
 * refuse an ln T2 box below ln(min_t2_s) (MRSTAT_ERR_ARG); values of db0 or
 * T2 outside the bounds lose the stated accuracy. With coils (the maps of
 * mrstat_bind) the term sums and x-GEMMs carry n_coils x terms rows.
 * nx <= 256 and n_read >= 2 (else MRSTAT_ERR_SHAPE); a bound that no term
 * count meets gives MRSTAT_ERR_UNSUPPORTED; the encoding is Cartesian and the
 * problem is validated as by mrstat_create. */
mrstat_status mrstat_create_readout(const mrstat_problem *p, double dwell_s, double min_t2_s,
                                    double max_abs_db0_hz, mrstat_ctx *out);

/* Off-resonance map of a readout-dynamics context: device float [Nv] in Hz,
 * read by every product while set (not copied; the caller keeps it alive);
 * NULL = zero. MRSTAT_ERR_STATE for a context without readout dynamics, or
 * for a map on a context set to the balanced isochromat model (whose echo an
 * off-resonance changes beyond a phase; its T2 decay during the readout is
 * modelled). */
mrstat_status mrstat_set_db0(mrstat_ctx ctx, const float *d_db0);

/* Delta B0 as a reconstructed parameter (the Discussion's extension of the
 * parameter set) on a readout-dynamics context: with hz_per_unit > 0 theta,
 * J v directions and Re(J^H w) gain a sixth row, p = 5, and voxel j's
 * off-resonance is theta[5 Nv + j] * hz_per_unit Hz in the readout factor
 * (the map of mrstat_set_db0 is then not read); the signal's derivative is
 * ds/dtheta_5 = -2 pi i hz_per_unit (TE + tau_k) times voxel j's term of s,
 * and GN and trust-region steps keep |Delta B0| within max_abs_db0_hz
 * (param_mask bit 5). hz_per_unit = 0 returns to five rows.
 * With one echo time the off-resonance phase at TE is shared with rho's
 * phase: Delta B0 is determined by the phase ramp across each readout only.
 * MRSTAT_ERR_STATE for other contexts or with the balanced model;
 * MRSTAT_ERR_ARG for a negative or non-finite hz_per_unit. */
mrstat_status mrstat_fit_db0(mrstat_ctx ctx, double hz_per_unit);

/* Terms of the readout-dynamics power series, the forward products' (0 for
 * other contexts). */
mrstat_status mrstat_readout_terms(mrstat_ctx ctx, int32_t *h_terms);

/* Terms of the readout-dynamics Chebyshev expansion: the rows per coil of the
 * x-stages and the adjoint's term sums, at most mrstat_readout_terms (0 for
 * other contexts). */
mrstat_status mrstat_readout_cheb_terms(mrstat_ctx ctx, int32_t *h_terms);

/* Signal model of the linearisation: the gradient-spoiled EPG (n_iso = 0,
 * the default) or the balanced isochromat model of the paper's own sequence
 * (Methods, Pulse Sequence and Reconstructions; Supporting Information S2):
 * a balanced transient-state gradient echo on resonance (no spoiling; RF
 * phases 0 / pi as for every context, alternating for the paper's sequence),
 * whose voxel magnetisation is sum_q weight[q] m_q over n_iso isochromats,
 * isochromat q seeing the flip angle scaled by scale[q] (the slice profile
 * of the RF pulse). Each isochromat follows the S2 update: an instantaneous
 * rotation about the RF axis, decay and regrowth, ideal inversion first;
 * derivatives in ln T1, ln T2 and B1 in forward mode. The trains have the
 * layout of the EPG's, and every call of the context (and the surrogate's
 * fallback) uses the model set here. Host arrays [n_iso] read during the
 * call; 0 <= n_iso <= 32; non-finite entries give MRSTAT_ERR_ARG; n_iso > 0
 * while an off-resonance map is set gives MRSTAT_ERR_STATE.
 * Invalidates the linearisation. */
mrstat_status mrstat_set_isochromats(mrstat_ctx ctx, int32_t n_iso, const double *h_scale,
                                     const double *h_weight);

/* Linearise at theta: EPG trains m, dm/dlnT1, dm/dlnT2, dm/dB1 per voxel and
 * TR into the workspace; if d_trains != NULL also copy them out as float32
 * [4][n_tr][Nv] holding the imaginary parts (the real parts are exactly 0
 * under the supported RF phases; FP16-stored trains are widened to FP32). The trains are m_j[n] = F+_0 e^{-i phi_n}
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

/* d_out = J v for v float32 [Np][Nv]; complex64 [n_coils][n_tr][n_read].
 * All Np parameter rows are used (a reused linearisation without the
 * dm/dB1 train, left by a B1-fixed mrstat_gn_step, is redone first). */
mrstat_status mrstat_jv(mrstat_ctx ctx, const float *d_theta, int32_t reuse_linearization,
                        const float *d_v, void *d_out, mrstat_stream stream);

/* d_out = Re(J^H w) for w complex64 [n_coils][n_tr][n_read]; float32 [Np][Nv]
 * (Algorithm 4: all N_p partial derivatives of a voxel together; a reused
 * three-train linearisation is redone first, as for mrstat_jv). */
mrstat_status mrstat_jhw(mrstat_ctx ctx, const float *d_theta, int32_t reuse_linearization,
                         const void *d_w, float *d_out, mrstat_stream stream);

/* One inexact Gauss-Newton iteration (Algorithm 6): linearise at theta,
 * r, f, g = Re(J^H r); exactly n_cg CG iterations on Re(J^H J) p = -g with
 * FP64 dot products and scalars kept on the device; backtracking line search
 * theta_t = P(theta + t p), P the box projection of (ln T1, ln T2, B1),
 * accepting the first t with f(theta_t) <= f + c1 g^T (theta_t - theta).
 * d_theta is updated in place only when a trial is accepted. Inactive
 * parameters (param_mask) and masked voxels never change. With B1 (bit 2)
 * outside param_mask the Jacobian has no B1 column, and the step's
 * linearisation holds no dm/dB1 train (neither simulated nor streamed); a
 * later mrstat_jv / mrstat_jhw that reuses it simulates the trains again at
 * the same theta. Synchronises. */
mrstat_status mrstat_gn_step(mrstat_ctx ctx, float *d_theta, const void *d_data,
                             const mrstat_gn_opts *opts, mrstat_gn_report *h_rep,
                             mrstat_stream stream);

/* Trust-region form of the Gauss-Newton iteration (Methods, Reconstructions:
 * the paper's trust-region framework after Steihaug and Nocedal & Wright's
 * Algorithm 7.2, with reflection at the feasible bounds after Coleman & Li).
 * One call: linearise at theta; r, f, g = Re(J^H r); Steihaug's truncated CG
 * on the model m(p) = f + g'p + p' Re(J^H J) p / 2 inside ||p|| <= delta
 * (at most n_cg iterations; stops on reaching the boundary, on non-positive
 * curvature or on a zero residual), Euclidean norm over the parameter vector
 * (inactive rows and masked voxels are zero); trial = theta + p with the
 * reconstructed ln T1, ln T2, B1 entries of unmasked voxels reflected into
 * [lo, hi] (the end point of the path bouncing off the box walls);
 * rho = (f(theta) - f(trial)) / pred with pred = -(g's + ||J s||^2 / 2) at
 * s = trial - theta (-infinity when pred <= 0 or rho is not finite);
 * theta = trial when rho > eta. The radius (Nocedal & Wright Algorithm 4.1):
 * *h_delta becomes delta / 4 when rho < 1/4, min(2 delta, delta_max) when
 * rho > 3/4 and the CG stopped at the boundary, else stays. FP64 scalars on
 * the device as in mrstat_gn_step. Errors: MRSTAT_ERR_ARG for options
 * outside their ranges (n_cg >= 0, 0 <= eta < 1, 0 < delta <= delta_max,
 * lo <= hi); MRSTAT_ERR_NONFINITE (theta and *h_delta unchanged) when f or
 * g is not finite. Synchronises. */
typedef struct {
    int32_t n_cg;         /* CG iteration limit of the truncated solve */
    int32_t param_mask;   /* bit p set = parameter p is reconstructed (p < Np) */
    float lo[3], hi[3];   /* box of ln T1, ln T2, B1, kept by reflection (a fitted
                             Delta B0: +-max_abs_db0_hz) */
    double eta;           /* acceptance threshold on rho */
    double delta_max;     /* cap of the trust radius */
} mrstat_tr_opts;

enum {
    MRSTAT_TR_ITERS = 0,      /* n_cg iterations inside the region */
    MRSTAT_TR_BOUNDARY = 1,   /* an iterate would leave the region: step on the boundary */
    MRSTAT_TR_CURVATURE = 2,  /* non-positive curvature: step to the boundary */
    MRSTAT_TR_ZERO = 3        /* zero residual of the model: its minimiser */
};

typedef struct {
    double f0, f1;        /* f at the incoming theta and at the returned one */
    double gnorm;         /* ||g|| */
    double step_norm;     /* ||s||, s = trial - theta (after reflection) */
    double rho;           /* actual / predicted decrease */
    double pred;          /* predicted decrease -(g's + ||J s||^2 / 2) */
    double delta_in, delta_out;   /* trust radius before and after */
    int32_t cg_iters;     /* completed CG updates */
    int32_t exit_kind;    /* MRSTAT_TR_* */
    int32_t accepted;     /* 1 if theta was updated */
    int32_t n_reflected;  /* trial entries that were reflected at a wall */
    int32_t n_fallback;   /* surrogate fallbacks of the linearisation */
} mrstat_tr_report;

mrstat_status mrstat_tr_step(mrstat_ctx ctx, float *d_theta, const void *d_data,
                             const mrstat_tr_opts *opts, double *h_delta, mrstat_tr_report *h_rep,
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
    MRSTAT_K_YFWD_JV = 3,    /* forward y-stage of J v (four trains, or three with B1 fixed) */
    MRSTAT_K_XFWD = 4,       /* forward x-stage GEMM (+ residual epilogue) */
    MRSTAT_K_XADJ = 5,       /* adjoint x-stage GEMM */
    MRSTAT_K_YADJ = 6,       /* adjoint y-stage (train streaming) */
    MRSTAT_K_FINISH = 7,     /* gradient assembly from the adjoint partials */
    MRSTAT_K_VECTOR = 8,     /* CG / line-search / CGLS vector kernels and reductions */
    MRSTAT_K_SURR = 9,       /* surrogate inference of the linearisation's trains (+ box test) */
    MRSTAT_K_SURR_VALUE = 10,/* surrogate inference of the m train (line-search trials) */
    MRSTAT_K_NC_FWD = 11,    /* non-Cartesian forward contraction (signal, residual, J v) */
    MRSTAT_K_NC_ADJ = 12,    /* non-Cartesian adjoint contraction with the trains */
    MRSTAT_K_COUNT = 13
} mrstat_kernel_kind;

mrstat_status mrstat_profile_enable(mrstat_ctx ctx, int32_t on);
mrstat_status mrstat_profile_read(mrstat_ctx ctx, int32_t *h_counts, double *h_ms);
/* Kinds traced while profiling is on: bit k of kind_mask = kind k (default
 * all). Each traced launch adds two event records to its stream (about 1.5 us
 * of device time each), so tracing only the kinds of interest keeps a timed
 * region close to its untraced duration. */
mrstat_status mrstat_profile_select(mrstat_ctx ctx, uint32_t kind_mask);

/* ------------------------------------------------------------------------
 * Learned surrogate of the EPG linearisation.
 *
 * Not part of the paper's method: an extension that replaces the per-voxel
 * simulation of the trains (the cost the paper names as dominant, Discussion)
 * by a small network evaluated on the matrix cores, keeping the EPG for
 * voxels outside the network's training box.
 *
 * Network: inputs (ln T1, ln T2, B1), each mapped affinely from the box onto
 * [-1, 1]; `depth` hidden layers of `width` units with the exact GELU
 * z Phi(z); a linear output layer of 8 n_tr values. Output o = c 4 n_tr +
 * p n_tr + n is part c (0 real, 1 imaginary) of train p (m, dm/dlnT1,
 * dm/dlnT2, dm/dB1) at TR n, in units of the head scale s_p. Parameters are
 * one FP32 vector: W1 [width][3], b1, then (W [width][width], b) for each
 * further hidden layer, Wout [8 n_tr][width], bout (row-major [out][in]).
 * Training: mean squared error over all outputs and samples against the EPG
 * trains divided by s_p (real parts target 0), Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8, bias-corrected) on FP32 master weights. Matrix products use BF16
 * operands (weights and activations rounded to BF16) with FP32
 * accumulation; the first layer and all epilogues run in FP32.
 *
 * Device memory: one caller-provided workspace per network
 * (mrstat_mlp_workspace_bytes / mrstat_mlp_bind), holding the parameters,
 * the Adam moments, gradients and the activations of one batch. Calls
 * are asynchronous on the given stream except those returning host values.
 * A network is not thread-safe, and a context using it as surrogate shares
 * its workspace: do not train and reconstruct with one network at once.
 * Requirements: n_tr a multiple of 8; width a multiple of 64, <= 1024;
 * 1 <= depth <= 16; batch a multiple of 64. Inference of widths 64, 128
 * and 256 (depth <= 16) runs in fused kernels that can store FP16 trains;
 * other widths run layer by layer in batch-size chunks and write FP32 only,
 * so a context with FP16 trains refuses them (MRSTAT_ERR_UNSUPPORTED from
 * mrstat_set_surrogate or mrstat_set_train_precision).
 * ------------------------------------------------------------------------ */
mrstat_status mrstat_mlp_create(int32_t n_tr, int32_t width, int32_t depth, int32_t batch,
                                mrstat_mlp *out);
void mrstat_mlp_destroy(mrstat_mlp net);
const char *mrstat_mlp_last_error(mrstat_mlp net);
size_t mrstat_mlp_param_count(mrstat_mlp net);
size_t mrstat_mlp_workspace_bytes(mrstat_mlp net);
/* Attaches a 256-byte aligned workspace (kept alive by the caller). */
mrstat_status mrstat_mlp_bind(mrstat_mlp net, void *d_ws, size_t ws_bytes, mrstat_stream stream);
/* Box [box_lo, box_hi] of (ln T1, ln T2, B1) (host arrays of 3) and head
 * scales s_p > 0 (host array of 4). Synchronises the stream. */
mrstat_status mrstat_mlp_set_scaling(mrstat_mlp net, const float box_lo[3], const float box_hi[3],
                                     const float head_scale[4], mrstat_stream stream);
/* Sets the box and s_p = RMS of train p over d_trains float32 [4][n_tr][n]
 * (FP64 sums on the device); returns the scales in h_scale_out (may be
 * NULL). Synchronises. */
mrstat_status mrstat_mlp_fit_scaling(mrstat_mlp net, const float *d_trains, int64_t n,
                                     const float box_lo[3], const float box_hi[3],
                                     float h_scale_out[4], mrstat_stream stream);
/* Copies parameters in (device float32 [param_count]), refreshes the BF16
 * copy and resets the Adam state; or copies the FP32 parameters out. */
mrstat_status mrstat_mlp_set_params(mrstat_mlp net, const float *d_params, mrstat_stream stream);
mrstat_status mrstat_mlp_get_params(mrstat_mlp net, float *d_params, mrstat_stream stream);
/* One batch of `batch` samples: columns of d_theta (rows ln T1, ln T2, B1
 * with leading dimension ld_theta, e.g. a theta [5][Nv] slice) and of the
 * EPG trains d_trains float32 [4][n_tr][ld_trains] (imaginary parts, as
 * mrstat_simulate writes them). mrstat_mlp_gradients writes the loss
 * gradient (float32 [param_count]) without updating; mrstat_mlp_train_step
 * applies one Adam step with learning rate lr. The batch loss is returned in
 * *h_loss when h_loss != NULL (then the stream is synchronised). */
mrstat_status mrstat_mlp_gradients(mrstat_mlp net, const float *d_theta, int64_t ld_theta,
                                   const float *d_trains, int64_t ld_trains, float *d_grad,
                                   double *h_loss, mrstat_stream stream);
mrstat_status mrstat_mlp_train_step(mrstat_mlp net, const float *d_theta, int64_t ld_theta,
                                    const float *d_trains, int64_t ld_trains, float lr,
                                    double *h_loss, mrstat_stream stream);
/* Tuning: voxels per workgroup of the fused inference kernel (widths 64, 128
 * and 256 evaluate the whole network per voxel tile in one kernel): 32 or 64
 * with the last activations held in registers, -32 or -64 with them read from
 * LDS (more output-weight loads in flight); 0 = automatic (-64 at width 256,
 * else 64). Results are identical for every choice. */
mrstat_status mrstat_mlp_set_infer_tile(mrstat_mlp net, int32_t voxels);
/* Predicted trains (imaginary parts, s_p applied) for n columns of d_theta
 * into d_out float32 [4][n_tr][n]. */
mrstat_status mrstat_mlp_predict(mrstat_mlp net, const float *d_theta, int64_t ld_theta, int32_t n,
                                 float *d_out, mrstat_stream stream);

/* Uses net (bound, built for this n_tr; NULL = plain EPG) for every
 * linearisation and line-search evaluation of the context: voxels whose
 * (ln T1, ln T2, B1) lie in the network's box take its trains, the others
 * (and non-finite ones) are simulated by the EPG. The fallback runs the full
 * recurrence for those voxels, which takes about the time of a whole EPG
 * pass however few they are: Gauss-Newton callers should keep the projection
 * box (mrstat_gn_opts lo/hi) inside the network's box. The caller keeps net
 * alive while it is set. Invalidates the current linearisation. */
mrstat_status mrstat_set_surrogate(mrstat_ctx ctx, mrstat_mlp net);
/* Number of voxels the last linearisation sent to the EPG fallback (0 without
 * a surrogate or linearisation). Synchronises the stream. */
mrstat_status mrstat_fallback_count(mrstat_ctx ctx, int32_t *h_count, mrstat_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* MRSTAT_H */
