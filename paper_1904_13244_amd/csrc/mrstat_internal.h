// Internal declarations shared by the HIP translation units of libmrstat.
// Not part of the public ABI (include/mrstat.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mrstat {

// Problem sizes as the kernels see them.
struct Dims {
    int nx, ny, nv;   // grid, nv = nx*ny (voxel j = iy*nx + ix)
    int T;            // TRs
    int nk;           // readout samples
    int K;            // EPG states
    int C;            // coils
    int np = 5;       // parameter rows: 5, or 6 with Delta B0 fitted (row 5)
};

// ---------------------------------------------------------------- non-Cartesian
// Encoding by an arbitrary trajectory (noncart.hip): ax, ay [T][nk] FP64 =
// kx / nx and ky / ny (kx, ky in cycles per field of view); nx <= 256.
// Forward: mode_y 0 (signal, m train) or 1 / 3 (J v direction, with or
// without dm/dB1); mode_x as for launch_xgemm_fwd (0 residual with FP64
// partials into red, their count in *nred; 1 -s; 2 s). enc 0 FP32 MFMA, 1
// split-BF16 MFMA. Adjoint: chunk partials of A_p = sum_n mu_p V (ntr 4, 3
// or 1) in the Cartesian adjoint's layout, with `chunks` TR chunks.
int nc_adj_chunks(const Dims& d);
int nc_fwd_blocks(const Dims& d);
// X: workspace [T][nv] complex for the forward's voxel values.
hipError_t launch_nc_fwd(const Dims& d, int enc, int mode_y, int mode_x, const void* trains, bool f16,
                         const float* theta, const float* v, const float2* coil, const uint8_t* mask,
                         const double* ax, const double* ay, float2* X, const float2* data, float2* out,
                         double* red, int* nred, hipStream_t s);
hipError_t launch_nc_adj(const Dims& d, int enc, int ntr, int chunks, const void* trains, bool f16,
                         const float2* coil, const uint8_t* mask, const double* ax, const double* ay,
                         const float2* w, float* apart, hipStream_t s);

// Per-voxel EPG timing constants shared by all voxels.
struct SeqTimes {
    float tr, te, tinv;
};

// ---------------------------------------------------------------- readout dynamics
// Term-wise y-stages and sample weighting of the readout-dynamics expansion
// (readout.hip): nq power-series sums per voxel column and TR, economised to
// nc Chebyshev rows V [nc][T][nx]; Y [nc][T][nk] (x-GEMM of V), w_m
// [nc][T][nk], W [nc][T][nx] (adjoint x-GEMM of w_m); apart as for the static
// adjoint. rd_terms: the power series' term count for a bound on
// |lambda| tau_max; rd_cheb_terms: the Chebyshev count (0 = none fits).
int rd_terms(double bound);
int rd_cheb_terms(double bound);
// With d.np == 6 the off-resonance is theta row 5 times db0_unit Hz (db0 is
// then not read) and J v gains that row's column.
// Coils (coil != null, [C][nv]): V, Y, w_m and W_m hold C x nc rows, coil-major.
hipError_t launch_rd_fwd(const Dims& d, int nq, int nc, int mode, const void* trains, bool f16, const float* theta,
                         const float* v, const float2* coil, const uint8_t* mask, const float* db0, float db0_unit,
                         const float2* eytab, float2* U, float te, float tmax, hipStream_t s);
hipError_t launch_rd_combine(const Dims& d, int nc, int mode, const float2* Y, float dwell_u, const float2* data,
                             float2* out, double* red, int* nred, hipStream_t s);
hipError_t launch_rd_expand(const Dims& d, int nc, float dwell_u, const float2* w, float2* wq, hipStream_t s);
// Chunk partials in the gradient assembly's layout; with d.np == 6 (ntr 3 or
// 4) the Delta B0 pair follows as planes 8 and 9 of each chunk.
hipError_t launch_rd_adj(const Dims& d, int nc, int ntr, int chunks, const void* trains, bool f16,
                         const float* theta, const float2* coil, const uint8_t* mask, const float* db0,
                         float db0_unit, const float2* eytab, const float2* W, float* apart, float te, float tmax,
                         hipStream_t s);

// ---------------------------------------------------------------- balanced isochromat model
// Slice profile of the balanced isochromat model (iso.hip): isochromat q has
// the flip angle scaled by scale[q] and weight weight[q]; n in [1, 32].
constexpr int MAX_ISOCHROMATS = 32;
struct IsoProfile {
    int n;
    float scale[MAX_ISOCHROMATS];
    float weight[MAX_ISOCHROMATS];
};
// Trains of the balanced isochromat model, same outputs and layout as
// launch_epg (ntan 3, 2 or 0); with idx non-null only the voxels
// idx[0 .. *count) (the surrogate's fallback list).
hipError_t launch_iso(const Dims& d, SeqTimes st, const float* theta, const float2* seq, void* out, int ntan,
                      bool f16, const IsoProfile& prof, const int* idx, const int* count, hipStream_t s);


// Tiling of the encoding kernels, chosen per problem on the host.
struct YPlan {
    int r_fwd;        // forward y-stage: row steps per lane (32 r_fwd rows per block)
    int nby;          // forward row blocks (partial sums of U when > 1)
    int fwd_tr;       // TRs per forward block
    int r_adj;        // adjoint y-stage: row steps per lane (8 r_adj rows per block)
    int adj_chunks;   // TR chunks of the adjoint y-stage (partial sums per chunk)
    int adj_per_chunk;
    int ksplit_adj;   // split-K of the adjoint x-GEMM (partial W outputs)
    int g16, r_fwd16, nby16, fwd_tr16;   // forward y-stage, FP16 trains, one row per wave
    int r_fwdc, nbyc, fwd_trc;           // forward y-stage with coils (per-TR reduction)
    int ntw16, ntws16, nbyw, roww;       // forward y-stage, wide layout (FP16 trains): TRs per
                                         // block in mode 1 / mode 0 (0 = off), row slabs, rows
                                         // per slab
    int nww;                             // waves per block of the wide forward y-stage (4 or 8)
};

inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

YPlan make_yplan(const Dims& d);

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `s` and return the launch status.

// EPG linearisation. theta [5][nv]; seq[n] = (flip angle [rad], RF sign +-1);
// out: planes [T][nv] of the imaginary parts of m, dm/dlnT1, dm/dlnT2, dm/dB1
// in a [4][T][nv] buffer, the first 1 + ntan of them written (ntan = 3, 2 or
// 0 tangent trains), float or (f16) _Float16. lanes = lanes per voxel
// (0 = automatic).
hipError_t launch_epg(const Dims& d, SeqTimes st, const float* theta, const float2* seq,
                      void* out, int ntan, int lanes, bool f16, hipStream_t s);

// EPG on the voxels idx[0 .. *count) only (same output layout; other voxels
// untouched). The grid covers nv voxels; blocks past the list exit at once.
hipError_t launch_epg_list(const Dims& d, SeqTimes st, const float* theta, const float2* seq,
                           void* out, int ntan, int lanes, bool f16, const int* idx,
                           const int* count, hipStream_t s);

// n stored train elements (float or _Float16) to float.
hipError_t launch_trains_to_f32(const void* in, bool f16, float* out, size_t n, hipStream_t s);

// Clears *count, then lists the voxels (in the mask) whose ln T1, ln T2, B1
// lie outside [lo, hi] (host arrays of 3) or are not finite.
hipError_t launch_box_compact(const Dims& d, const float* theta, const float* lo, const float* hi,
                              const uint8_t* mask, int* idx, int* count, hipStream_t s);

// Forward y-stage: U[c][n][ix] = sum over rows iy of Ey[n][iy] * coil_c[j] *
// x[n][j], with x = i rho m (mode 0) or x = i (rho sum_q v_q dm_q +
// (v3 + i v4) m) (mode 1, the J v direction; mode 3: the same with v2 taken
// as 0 and the dm/dB1 train not read). upart holds nby row-block partials
// when nby > 1 and is summed into its first block.
hipError_t launch_ystage_fwd(const Dims& d, const YPlan& p, int mode, const void* trains, bool f16,
                             const float* theta, const float* v, const float2* coil,
                             const uint8_t* mask, const float2* eytab, float2* upart, int* nby,
                             hipStream_t s);
// Sums the nby row-block partials of U written by the forward y-stage into
// partial 0 (nothing to do for nby = 1).
hipError_t launch_usum(const Dims& d, float2* upart, int nby, hipStream_t s);

// x-stage forward GEMM: s[c][n][k] = sum_ix Ex[k][ix] U[c][n][ix].
// mode 0: out = data - s and per-block FP64 sums of |out|^2 into red;
// mode 1: out = -s; mode 2: out = s.
// enc 0: the LDS-tiled FP32 kernel (extab); enc 1 / 2: the LDS-free kernel
// on the B-fragment table of this direction and encoding (bfrag; required).
hipError_t launch_xgemm_fwd(const Dims& d, const YPlan& p, int enc, int mode, const float2* U,
                            const float2* extab, const void* bfrag, const float2* data, float2* out,
                            double* red, int* nred, hipStream_t s);

// x-stage adjoint GEMM: W[z][c][n][ix] = partial z of sum_k conj(Ex[k][ix]) w[c][n][k]
// (one partial, complete, on the LDS-free path).
hipError_t launch_xgemm_adj(const Dims& d, const YPlan& p, int enc, const float2* w,
                            const float2* extab, const void* bfrag, float2* W, hipStream_t s);

// B-fragment tables of the LDS-free reduced-precision x-GEMMs: bytes per
// table (dir 0 forward, 1 adjoint; enc 1 split-BF16, 2 FP16), their build
// from the phase table (f1/a1: split-BF16 forward/adjoint, f2/a2: FP16), and
// the number of FP64 partials the forward kernel writes in mode 0.
size_t bfrag_bytes(const Dims& d, int dir, int enc);
hipError_t launch_build_bfrag(const Dims& d, const float2* extab, void* f1, void* a1, void* f2,
                              void* a2, hipStream_t s);
int xgemm_direct_blocks(const Dims& d);

// Adjoint y-stage: partial sums over TR chunks of
// A_p[j] = sum_n mu_p[n][j] conj(Ey[n][iy]) sum_c conj(coil_c[j]) W_c[n][ix]
// (p < ntr_trains: 4 = m and the three tangents, 3 = without dm/dB1, whose
// pair in the four-train chunk layout is then left unwritten, 1 = m only).
hipError_t launch_ystage_adj(const Dims& d, const YPlan& p, const void* trains, bool f16, int ntr_trains,
                             const float2* coil, const uint8_t* mask, const float2* eytab,
                             const float2* W, float* apart, hipStream_t s);

// g[np][nv] = Re(J^H w) from the chunk partials (sums in chunk order; 8
// planes per chunk, 10 with Delta B0 fitted); rows of parameters outside
// param_mask (and masked voxels) are zero, and the dm/dB1 partials are read
// only when B1 is in param_mask.
// With dir non-null, also the CG partials dir . g and dir . dir (FP64, one
// per block of 256 voxels: part[b] and part[nblocks + b]) and either, with
// step non-null, step . dir in part[2 nblocks + b], or, with res non-null,
// res . res, res . g and g . g in planes 2, 3 and 4 (dir with neither is
// hipErrorInvalidValue).
hipError_t launch_jhw_finish(const Dims& d, const YPlan& p, const float* apart, const float* theta,
                             const uint8_t* mask, int param_mask, float* g, const float* dir,
                             double* part, hipStream_t s, const float* step = nullptr,
                             const float* res = nullptr);

// CGLS helper: A^H w = -i A_0 from the one-train partials.
hipError_t launch_rho_adj_finish(const Dims& d, const YPlan& p, const float* apart,
                                 const uint8_t* mask, float2* out, hipStream_t s);

// ---------------------------------------------------------------- reductions
// Deterministic FP64 reductions: per-block partials then one block.
constexpr int RED_BLOCKS = 512;
hipError_t launch_sum_partials(const double* partials, int n, double* out, hipStream_t s);
hipError_t launch_dot(const float* a, const float* b, size_t n, double* partials, double* out,
                      hipStream_t s);
hipError_t launch_dot_c(const float2* a, const float2* b, size_t n, double* partials,
                        double* out, hipStream_t s);

// ---------------------------------------------------------------- CG / line search
// Device-resident scalar block (doubles); slot numbers shared with vec.hip.
constexpr int SCAL_DOUBLES = 64;
enum : int {
    SC_RR = 0, SC_ITERS = 6, SC_F0 = 8, SC_G2 = 9, SC_PRED = 10, SC_SN = 11, SC_ACC = 13, SC_FT = 14,
    SC_STAGE = 30, SC_CDONE = 25,
    // trust-region step: |step|^2, radius^2, exit kind, g . s, |J s|^2,
    // reflected entries, ratio, |s|^2
    SC_ZZ = 32, SC_DELTA2 = 33, SC_EXIT = 35, SC_GS = 36, SC_JS2 = 37, SC_NREF = 38,
    SC_SS = 39, SC_RHO = 40
};

hipError_t launch_cg_init(const Dims& d, const float* g, float* step, float* res, float* dir,
                          double* scal, double* partials, hipStream_t s);
// One CG iteration after q = Re(J^H J) dir, in one launch: the finish
// kernel left dir . q, dir . dir, res . res, res . q and q . q in partials
// ([5][nv / 256 blocks]); iter = iteration index from 0; partials hold at
// least cg_partials(d) doubles.
hipError_t launch_cg_update(const Dims& d, const float* q, float* step, float* res, float* dir,
                            double* scal, double* partials, int iter, hipStream_t s);
int cg_partials(const Dims& d);

// Trust-region CG (Steihaug): after launch_cg_init, launch_tr_init sets
// |step|^2 = 0, the radius^2 and the exit kind (zero gradient or not).
// launch_tr_update is one iteration after q = Re(J^H J) dir with the finish
// kernel's three curvature partials (dir . q, dir . dir, step . dir): an
// iterate that would leave the region, or a direction of non-positive
// curvature, moves the step to the boundary and stops CG (exit kind in
// SC_EXIT: 0 iteration count, 1 boundary, 2 curvature, 3 zero residual).
hipError_t launch_tr_init(double* scal, double delta2, hipStream_t s);
hipError_t launch_tr_update(const Dims& d, const float* q, float* step, float* res, float* dir,
                            double* scal, double* partials, int iter, hipStream_t s);
int tr_partials(const Dims& d);
// Boxes lo[6], hi[6] per parameter row; rows 0-2 (ln T1, ln T2, B1) and,
// with d.np == 6, row 5 (Delta B0) are bounded, the rho rows are not.
// trial = theta + step with the active bounded entries of unmasked voxels
// reflected into [lo, hi] (a fold at the walls); sv = trial - theta; the
// number of reflected entries to SC_NREF and |sv|^2 to SC_SS.
hipError_t launch_tr_trial(const Dims& d, const float* theta, const float* step, const float* lo,
                           const float* hi, int param_mask, const uint8_t* mask, float* trial,
                           float* sv, double* scal, double* partials, hipStream_t s);
// ratio = (f0 - ft) / (-(g . s + |J s|^2 / 2)) from the scalars (SC_F0 and
// SC_FT hold 2 f), -inf when the prediction is not positive or the ratio not
// finite; theta = trial when ratio > eta. SC_RHO and SC_ACC record them.
hipError_t launch_tr_accept(const Dims& d, double* scal, double eta, const float* trial, float* theta,
                            hipStream_t s);
hipError_t launch_ls_trial_masked(const Dims& d, const float* theta, const float* step, float t,
                                  const float* lo, const float* hi, int param_mask,
                                  const uint8_t* mask, float* trial, hipStream_t s);
hipError_t launch_pred_dot(const Dims& d, const float* g, const float* trial, const float* theta,
                           double* partials, double* out, hipStream_t s);
// Armijo test on the device, f(trial) <= f0 + c1 pred with f(trial) finite
// (f = SC_FT / 2, f0 = SC_F0 / 2, pred = SC_PRED); when it holds theta = trial. The outcome
// goes to SC_ACC (1 or 0).
hipError_t launch_ls_accept(const Dims& d, double* scal, double c1, const float* trial, float* theta,
                            hipStream_t s);

// CGLS (complex unknown per voxel).
hipError_t launch_set_rho(const Dims& d, const float* theta_in, const float2* p, float* theta_out,
                          hipStream_t s);
hipError_t launch_cgls_step_x(const Dims& d, float2* x, float2* p, const double* scal,
                              hipStream_t s);
hipError_t launch_cgls_step_r(size_t n, float2* r, const float2* q, const double* scal,
                              hipStream_t s);
hipError_t launch_cgls_dir(const Dims& d, float2* p, const float2* sv, const double* scal,
                           hipStream_t s);
hipError_t launch_cgls_scalars(double* scal, int phase, hipStream_t s);
hipError_t launch_copy_rho_out(const Dims& d, const float2* x, float* theta, hipStream_t s);

}  // namespace mrstat
