// Parameter-space vector kernels of the inexact Gauss-Newton driver:
// deterministic FP64 reductions (fixed grid, fixed order), the CG recurrences
// on Re(J^H J) p = -g (eq. 4) with every scalar kept in device memory, the
// projected line-search trial, and the CGLS recurrences of the proton-density
// initialisation. Vectors are FP32 [np][Nv] (np = 5, or 6 with Delta B0
// fitted); dots, norms, alpha and beta FP64.
#include "mrstat_internal.h"

namespace mrstat {

// Scalar slots (double) in the device scalar block.
enum : int {
    S_RR = 0, S_KAPPA = 1, S_ALPHA = 2, S_RRNEW = 3, S_BETA = 4, S_DONE = 5, S_ITERS = 6,
    S_DD = 7, S_F0 = 8, S_G2 = 9, S_PRED = 10, S_FT = 11, S_UPD = 12,
    S_RR1 = 15, S_DONE1 = 16,
    S_GAMMA = 20, S_QQ = 21, S_CA = 22, S_GNEW = 23, S_CB = 24, S_CDONE = 25, S_STAGE = 30
};

// rr and the stop flag alternate between two slots by CG iteration parity:
// iteration k reads slot k & 1 and its direction kernel writes slot
// (k + 1) & 1, so no block reads a scalar that another block of the same
// launch writes.
__device__ __forceinline__ int rr_slot(int par) { return par ? S_RR1 : S_RR; }
__device__ __forceinline__ int done_slot(int par) { return par ? S_DONE1 : S_DONE; }

namespace {

constexpr int RB = 256;   // threads per reduction block
constexpr int PF = 2;     // vector elements per thread loaded ahead in the CG kernels

__device__ __forceinline__ double block_sum(double v, double* sh)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
    __syncthreads();
    return t;   // valid in thread 0
}

__global__ __launch_bounds__(RB) void sum_partials_kernel(const double* __restrict__ p, int n,
                                                          double* __restrict__ out)
{
    __shared__ double sh[RB / 64];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += RB) v += p[i];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) *out = v;
}

__global__ __launch_bounds__(RB) void dot_kernel(const float* __restrict__ a,
                                                 const float* __restrict__ b, size_t n,
                                                 double* __restrict__ part)
{
    __shared__ double sh[RB / 64];
    double v = 0.0;
    for (size_t i = (size_t)blockIdx.x * RB + threadIdx.x; i < n; i += (size_t)gridDim.x * RB)
        v += (double)a[i] * (double)b[i];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// Re sum conj(a) b over complex vectors (= sum a.x b.x + a.y b.y).
__global__ __launch_bounds__(RB) void dot_c_kernel(const float2* __restrict__ a,
                                                   const float2* __restrict__ b, size_t n,
                                                   double* __restrict__ part)
{
    __shared__ double sh[RB / 64];
    double v = 0.0;
    for (size_t i = (size_t)blockIdx.x * RB + threadIdx.x; i < n; i += (size_t)gridDim.x * RB) {
        const float2 x = a[i], y = b[i];
        v += (double)x.x * (double)y.x + (double)x.y * (double)y.y;
    }
    v = block_sum(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// step = 0, res = -g, dir = res; partial sums of res.res.
__global__ __launch_bounds__(RB) void cg_init_kernel(const float* __restrict__ g,
                                                     float* __restrict__ step,
                                                     float* __restrict__ res,
                                                     float* __restrict__ dir, size_t n,
                                                     double* __restrict__ part)
{
    __shared__ double sh[RB / 64];
    double v = 0.0;
    for (size_t i = (size_t)blockIdx.x * RB + threadIdx.x; i < n; i += (size_t)gridDim.x * RB) {
        const float r = -g[i];
        step[i] = 0.f;
        res[i] = r;
        dir[i] = r;
        v += (double)r * (double)r;
    }
    v = block_sum(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// Finish of the init: rr, |g|^2 (= rr), clear the flags.
__global__ __launch_bounds__(RB) void cg_init_finish(const double* __restrict__ part, int n,
                                                     double* __restrict__ sc)
{
    __shared__ double sh[RB / 64];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += RB) v += part[i];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) {
        sc[S_RR] = v;
        sc[S_G2] = v;
        sc[S_DONE] = (v == 0.0) ? 1.0 : 0.0;
        sc[S_ITERS] = 0.0;
        sc[S_ALPHA] = 0.0;
        sc[S_BETA] = 0.0;
        sc[S_UPD] = 0.0;
    }
}

// K kinds of per-block partials ([K][n]) reduced by every block in one fixed
// order (per thread in index order, then lane 0 of each wave's butterfly,
// then the four waves in order): the sums are identical in all threads and
// blocks.
template <int K>
__device__ __forceinline__ void reduce_kinds(const double* __restrict__ part, int n, double (&sh)[K][RB / 64],
                                             double (&v)[K])
{
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = 0.0;
    for (int i = threadIdx.x; i < n; i += RB)
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] += part[(size_t)k * n + i];
#pragma unroll
    for (int k = 0; k < K; ++k)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) sh[k][wave] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = (sh[k][0] + sh[k][1]) + (sh[k][2] + sh[k][3]);
}

// One CG iteration in one launch. From the finish kernel's partials every
// block forms kappa = dir . q, dir . dir, rr = res . res, res . q and q . q;
// CG stops on non-positive curvature or a zero residual; alpha = rr / kappa,
// and the updated residual's norm is known before any element changes,
// |res - alpha q|^2 = rr - 2 alpha res . q + alpha^2 q . q, so beta = that / rr
// and step += alpha dir, res -= alpha q, dir = res + beta dir take one pass.
// rr itself is always the sum over the stored residual, so the formula's
// rounding does not accumulate over iterations. Block 0 records kappa,
// dir . dir, alpha, UPD (the iteration updated the vectors), the new rr and
// beta, counts the iteration and writes the stop flag for the next one.
__global__ __launch_bounds__(RB) void cg_update_kernel(const float* __restrict__ q,
                                                       float* __restrict__ step,
                                                       float* __restrict__ res,
                                                       float* __restrict__ dir, size_t n,
                                                       const double* __restrict__ curv, int nblk,
                                                       double* __restrict__ sc, int par)
{
    __shared__ double sh[5][RB / 64];
    // This thread's first PF elements and the stop flag are loaded before
    // the reduction of the partials (they do not depend on it).
    const size_t i0 = (size_t)blockIdx.x * RB + threadIdx.x, stride = (size_t)gridDim.x * RB;
    float rp[PF], dp[PF], sp[PF], qp[PF];
#pragma unroll
    for (int e = 0; e < PF; ++e) {
        const size_t i = i0 + e * stride;
        const bool ok = i < n;
        rp[e] = ok ? res[i] : 0.f;
        dp[e] = ok ? dir[i] : 0.f;
        sp[e] = ok ? step[i] : 0.f;
        qp[e] = ok ? q[i] : 0.f;
    }
    const double done = sc[done_slot(par)];
    double v[5];
    reduce_kinds<5>(curv, nblk, sh, v);
    const double kappa = v[0], dd = v[1], rr = v[2], rq = v[3], qq = v[4];
    const bool upd = done == 0.0 && rr != 0.0 && !(kappa <= 1e-30 * dd);
    const double alpha = upd ? rr / kappa : 0.0;
    const float al = (float)alpha;
    const double a = al;   // the step the elements take
    double rn = fma(a * a, qq, fma(-2.0 * a, rq, rr));
    if (rn < 0.0) rn = 0.0;
    const double beta = upd ? rn / rr : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[S_KAPPA] = kappa;
        sc[S_DD] = dd;
        sc[S_UPD] = upd ? 1.0 : 0.0;
        sc[S_ALPHA] = alpha;
        if (upd) {
            sc[S_RRNEW] = rn;
            sc[S_BETA] = beta;
            sc[S_ITERS] += 1.0;
        }
        sc[rr_slot(par ^ 1)] = upd ? rn : rr;
        sc[done_slot(par ^ 1)] = (!upd || rn == 0.0) ? 1.0 : 0.0;
    }
    if (!upd) return;
    const float b = (float)beta;
#pragma unroll
    for (int e = 0; e < PF; ++e) {
        const size_t i = i0 + e * stride;
        if (i >= n) break;
        const float r = fmaf(-al, qp[e], rp[e]);
        step[i] = fmaf(al, dp[e], sp[e]);
        res[i] = r;
        dir[i] = fmaf(b, dp[e], r);
    }
    for (size_t i = i0 + PF * stride; i < n; i += stride) {
        const float dv = dir[i];
        const float r = fmaf(-al, q[i], res[i]);
        step[i] = fmaf(al, dv, step[i]);
        res[i] = r;
        dir[i] = fmaf(b, dv, r);
    }
}

// The trust-region CG's direction: beta = rr_new / rr from the step kernel's
// res . res partials, dir = res + beta dir. Block 0 records rr_new, beta and
// |step|^2 (from the step kernel's partials zzp), counts the iteration,
// writes rr and the stop flag for the next iteration (a zero residual, or a
// stopped iteration, stops CG) and marks a zero residual as the exit kind.
__global__ __launch_bounds__(RB) void tr_dir_kernel(const float* __restrict__ res,
                                                    float* __restrict__ dir, size_t n,
                                                    const double* __restrict__ part, int nblk,
                                                    double* __restrict__ sc, int par,
                                                    const double* __restrict__ zzp)
{
    __shared__ double sh[RB / 64];
    __shared__ double bc[1];
    // First PF elements and the scalars ahead of the reduction.
    const size_t i0 = (size_t)blockIdx.x * RB + threadIdx.x, stride = (size_t)gridDim.x * RB;
    float rp[PF], dp[PF];
#pragma unroll
    for (int e = 0; e < PF; ++e) {
        const size_t i = i0 + e * stride;
        const bool ok = i < n;
        rp[e] = ok ? res[i] : 0.f;
        dp[e] = ok ? dir[i] : 0.f;
    }
    const bool upd = sc[S_UPD] != 0.0;
    const double rr = sc[rr_slot(par)];
    double v = 0.0;
    for (int i = threadIdx.x; i < nblk; i += RB) v += part[i];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) bc[0] = v;
    __syncthreads();
    v = bc[0];
    const double beta = upd ? v / rr : 0.0;
    double zz = 0.0;
    for (int i = threadIdx.x; i < nblk; i += RB) zz += zzp[i];
    zz = block_sum(zz, sh);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (upd) {
            sc[S_RRNEW] = v;
            sc[S_BETA] = beta;
            sc[S_ITERS] += 1.0;
        }
        sc[rr_slot(par ^ 1)] = upd ? v : rr;
        sc[done_slot(par ^ 1)] = (!upd || v == 0.0) ? 1.0 : 0.0;
        sc[SC_ZZ] = zz;
        if (upd && v == 0.0) sc[SC_EXIT] = 3.0;
    }
    if (!upd) return;
    const float b = (float)beta;
#pragma unroll
    for (int e = 0; e < PF; ++e) {
        const size_t i = i0 + e * stride;
        if (i < n) dir[i] = fmaf(b, dp[e], rp[e]);
    }
    for (size_t i = i0 + PF * stride; i < n; i += stride) dir[i] = fmaf(b, dir[i], res[i]);
}

// ------------------------------------------------------------ trust region
// Steihaug's truncated CG (Nocedal & Wright Algorithm 7.2) on the same
// vectors as the CG above: step = z, res = -(g + B z), dir = the search
// direction.

__global__ void tr_init_kernel(double* __restrict__ sc, double delta2)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    sc[SC_ZZ] = 0.0;
    sc[SC_DELTA2] = delta2;
    sc[SC_EXIT] = (sc[S_RR] == 0.0) ? 3.0 : 0.0;
}

// The three curvature partials (dir . q, dir . dir, step . dir) reduced in
// every block in one fixed order; broadcast through LDS.
__device__ __forceinline__ void reduce_triple(const double* __restrict__ part, int n, double* sh,
                                              double* bc, double& a, double& b, double& c)
{
    a = b = c = 0.0;
    for (int i = threadIdx.x; i < n; i += RB) {
        a += part[i];
        b += part[n + i];
        c += part[2 * n + i];
    }
    a = block_sum(a, sh);
    b = block_sum(b, sh);
    c = block_sum(c, sh);
    if (threadIdx.x == 0) {
        bc[0] = a;
        bc[1] = b;
        bc[2] = c;
    }
    __syncthreads();
    a = bc[0];
    b = bc[1];
    c = bc[2];
}

// One Steihaug iteration. kappa = dir . B dir; with kappa <= 0 the step
// moves along dir to the boundary point of lower model value (the model
// changes by -t rr + t^2 kappa / 2 along a CG direction, res . dir = rr);
// otherwise alpha = rr / kappa, and if |step + alpha dir| would reach the
// radius the step stops on the boundary instead (|step|^2, step . dir and
// dir . dir give the root); else the usual CG update of step and res. Every
// block takes the same decision; block 0 records it. Partials of res . res
// and step . step for the direction kernel.
__global__ __launch_bounds__(RB) void tr_step_kernel(const float* __restrict__ dir,
                                                     const float* __restrict__ q,
                                                     float* __restrict__ step,
                                                     float* __restrict__ res, size_t n,
                                                     const double* __restrict__ curv, int nblk,
                                                     double* __restrict__ sc, int par,
                                                     double* __restrict__ part_rr,
                                                     double* __restrict__ part_zz)
{
    __shared__ double sh[RB / 64];
    __shared__ double bc[3];
    const size_t i0 = (size_t)blockIdx.x * RB + threadIdx.x, stride = (size_t)gridDim.x * RB;
    const double done = sc[done_slot(par)], rr = sc[rr_slot(par)];
    const double zz = sc[SC_ZZ], d2 = sc[SC_DELTA2];
    double kappa, dd, zd;
    reduce_triple(curv, nblk, sh, bc, kappa, dd, zd);
    int mode = 0;          // 0 nothing, 1 interior update, 2 move to the boundary
    double coef = 0.0;
    double exitk = 0.0;
    if (done == 0.0) {
        const double disc = sqrt(fmax(zd * zd + dd * (d2 - zz), 0.0));
        const double t_hi = (-zd + disc) / dd, t_lo = (-zd - disc) / dd;
        if (!(kappa > 0.0)) {
            const double m_hi = -t_hi * rr + 0.5 * t_hi * t_hi * kappa;
            const double m_lo = -t_lo * rr + 0.5 * t_lo * t_lo * kappa;
            coef = m_lo < m_hi ? t_lo : t_hi;
            mode = 2;
            exitk = 2.0;
        } else {
            const double alpha = rr / kappa;
            if (zz + 2.0 * alpha * zd + alpha * alpha * dd >= d2) {
                coef = t_hi;
                mode = 2;
                exitk = 1.0;
            } else {
                coef = alpha;
                mode = 1;
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[S_KAPPA] = kappa;
        sc[S_DD] = dd;
        sc[S_UPD] = mode == 1 ? 1.0 : 0.0;
        sc[S_ALPHA] = mode == 1 ? coef : 0.0;
        if (mode == 2) sc[SC_EXIT] = exitk;
    }
    const float c = (float)coef;
    double vr = 0.0, vz = 0.0;
    for (size_t i = i0; i < n; i += stride) {
        float z = step[i], r = res[i];
        if (mode != 0) {
            z = fmaf(c, dir[i], z);
            step[i] = z;
        }
        if (mode == 1) {
            r = fmaf(-c, q[i], r);
            res[i] = r;
        }
        vr += (double)r * (double)r;
        vz += (double)z * (double)z;
    }
    vr = block_sum(vr, sh);
    vz = block_sum(vz, sh);
    if (threadIdx.x == 0) {
        part_rr[blockIdx.x] = vr;
        part_zz[blockIdx.x] = vz;
    }
}

// The parameter box by value: rows 0-2 (ln T1, ln T2, B1) and 5 (Delta B0)
// are bounded, the rho rows 3 and 4 are not.
struct Box6 {
    float lo[6], hi[6];
};

__host__ __device__ __forceinline__ bool bounded_row(int q) { return q < 3 || q == 5; }

Box6 box6(const float* lo, const float* hi)
{
    Box6 b;
    for (int q = 0; q < 6; ++q) {
        b.lo[q] = lo[q];
        b.hi[q] = hi[q];
    }
    return b;
}

// Reflection into [lo, hi]: the end point of the straight path that bounces
// off the walls (a fold with period 2 (hi - lo)); inside values pass as they
// are.
__device__ __forceinline__ float reflect_box(float x, float lo, float hi, bool& moved)
{
    moved = false;
    if (x >= lo && x <= hi) return x;
    moved = true;
    const float w = hi - lo;
    if (!(w > 0.f)) return lo;
    float y = fmodf(x - lo, 2.f * w);
    if (y < 0.f) y += 2.f * w;
    if (y > w) y = 2.f * w - y;
    return lo + y;
}

__global__ __launch_bounds__(RB) void tr_trial_kernel(const float* __restrict__ theta,
                                                      const float* __restrict__ step, Box6 box,
                                                      int param_mask,
                                                      const uint8_t* __restrict__ mask,
                                                      float* __restrict__ trial,
                                                      float* __restrict__ sv, int nv, int np,
                                                      double* __restrict__ part)
{
    __shared__ double sh[RB / 64];
    const size_t n = (size_t)np * nv;
    double cnt = 0.0, ss = 0.0;
    for (size_t i = (size_t)blockIdx.x * RB + threadIdx.x; i < n; i += (size_t)gridDim.x * RB) {
        const int q = (int)(i / nv), j = (int)(i % nv);
        const float th = theta[i];
        float x = th + step[i];
        const bool on = ((param_mask >> q) & 1) && (mask == nullptr || mask[j] != 0);
        if (bounded_row(q) && on) {
            bool moved;
            x = reflect_box(x, box.lo[q], box.hi[q], moved);
            cnt += moved ? 1.0 : 0.0;
        }
        const float t = on ? x : th;
        const float d = t - th;
        trial[i] = t;
        sv[i] = d;
        ss += (double)d * (double)d;
    }
    cnt = block_sum(cnt, sh);
    ss = block_sum(ss, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = cnt;
        part[gridDim.x + blockIdx.x] = ss;
    }
}

// Ratio of actual to predicted decrease and the acceptance (every block
// takes the same decision; block 0 records it).
__global__ void tr_accept_kernel(double* __restrict__ sc, double eta, const float* __restrict__ trial,
                                 float* __restrict__ theta, size_t n)
{
    const double f0 = 0.5 * sc[SC_F0], ft = 0.5 * sc[SC_FT];
    const double pred = -(sc[SC_GS] + 0.5 * sc[SC_JS2]);
    double rho = (f0 - ft) / pred;
    if (!(pred > 0.0) || !isfinite(rho)) rho = -INFINITY;
    const bool acc = rho > eta;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[SC_RHO] = rho;
        sc[SC_PRED] = pred;
        sc[SC_ACC] = acc ? 1.0 : 0.0;
    }
    if (!acc) return;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        theta[i] = trial[i];
}

// trial = P(theta + t step): active bounded entries clamped to the box.
__global__ void ls_trial_kernel(const float* __restrict__ theta, const float* __restrict__ step,
                                float t, Box6 box, int param_mask, const uint8_t* __restrict__ mask,
                                float* __restrict__ trial, int nv, int np)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)np * nv) return;
    const int q = (int)(i / nv), j = (int)(i % nv);
    float x = fmaf(t, step[i], theta[i]);
    const bool on = ((param_mask >> q) & 1) && (mask == nullptr || mask[j] != 0);
    if (bounded_row(q) && on) x = fminf(fmaxf(x, box.lo[q]), box.hi[q]);
    trial[i] = on ? x : theta[i];
}

// Partial sums of g . (trial - theta) and |trial - theta|^2.
__global__ __launch_bounds__(RB) void pred_kernel(const float* __restrict__ g,
                                                  const float* __restrict__ trial,
                                                  const float* __restrict__ theta, size_t n,
                                                  double* __restrict__ part)
{
    __shared__ double sh[RB / 64];
    double a = 0.0, b = 0.0;
    for (size_t i = (size_t)blockIdx.x * RB + threadIdx.x; i < n; i += (size_t)gridDim.x * RB) {
        const double d = (double)trial[i] - (double)theta[i];
        a += (double)g[i] * d;
        b += d * d;
    }
    a = block_sum(a, sh);
    b = block_sum(b, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = a;
        part[gridDim.x + blockIdx.x] = b;
    }
}

// Every block takes the same decision from the same scalars; block 0
// records it.
__global__ void ls_accept_kernel(double* __restrict__ sc, double c1, const float* __restrict__ trial,
                                 float* __restrict__ theta, size_t n)
{
    // SC_FT and SC_F0 hold |r|^2 = 2 f.
    const double ft = 0.5 * sc[SC_FT], f0 = 0.5 * sc[SC_F0], pred = sc[SC_PRED];
    const bool acc = isfinite(ft) && ft <= f0 + c1 * pred;
    if (blockIdx.x == 0 && threadIdx.x == 0) sc[SC_ACC] = acc ? 1.0 : 0.0;
    if (!acc) return;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        theta[i] = trial[i];
}

__global__ __launch_bounds__(RB) void sum2_kernel(const double* __restrict__ part, int n,
                                                  double* __restrict__ out)
{
    __shared__ double sh[RB / 64];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < n; i += RB) {
        a += part[i];
        b += part[n + i];
    }
    a = block_sum(a, sh);
    b = block_sum(b, sh);
    if (threadIdx.x == 0) {
        out[0] = a;
        out[1] = b;
    }
}

// ------------------------------------------------------------------ CGLS
__global__ void set_rho_kernel(const float* __restrict__ th, const float2* __restrict__ p,
                               float* __restrict__ out, int nv, int np)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)np * nv) return;
    const int q = (int)(i / nv), j = (int)(i % nv);
    out[i] = q == 3 ? p[j].x : (q == 4 ? p[j].y : th[i]);
}

// x += a p (complex per voxel), a = gamma / qq; stop when qq == 0.
__global__ void cgls_x_kernel(float2* __restrict__ x, const float2* __restrict__ p, int nv,
                              const double* __restrict__ sc)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nv || sc[S_CDONE] != 0.0) return;
    const float a = (float)sc[S_CA];
    x[j] = make_float2(fmaf(a, p[j].x, x[j].x), fmaf(a, p[j].y, x[j].y));
}

__global__ void cgls_r_kernel(float2* __restrict__ r, const float2* __restrict__ q, size_t n,
                              const double* __restrict__ sc)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || sc[S_CDONE] != 0.0) return;
    const float a = (float)sc[S_CA];
    r[i] = make_float2(fmaf(-a, q[i].x, r[i].x), fmaf(-a, q[i].y, r[i].y));
}

__global__ void cgls_p_kernel(float2* __restrict__ p, const float2* __restrict__ s, int nv,
                              const double* __restrict__ sc)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nv || sc[S_CDONE] != 0.0) return;
    const float b = (float)sc[S_CB];
    p[j] = make_float2(fmaf(b, p[j].x, s[j].x), fmaf(b, p[j].y, s[j].y));
}

// phase 0: gamma = dot (init); 1: qq = dot, a = gamma/qq; 2: gnew = dot, b.
__global__ void cgls_scalar_kernel(double* __restrict__ sc, int phase)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double v = sc[S_STAGE];   // reduction result staged by the host-side sequence
    if (phase == 0) {
        sc[S_GAMMA] = v;
        sc[S_CDONE] = (v == 0.0) ? 1.0 : 0.0;
    } else if (phase == 1) {
        if (sc[S_CDONE] != 0.0) return;
        sc[S_QQ] = v;
        if (v == 0.0) {
            sc[S_CDONE] = 1.0;
            sc[S_CA] = 0.0;
        } else {
            sc[S_CA] = sc[S_GAMMA] / v;
        }
    } else {
        if (sc[S_CDONE] != 0.0) return;
        sc[S_GNEW] = v;
        sc[S_CB] = v / sc[S_GAMMA];
        sc[S_GAMMA] = v;
        if (v == 0.0) sc[S_CDONE] = 1.0;
    }
}

__global__ void copy_rho_out_kernel(const float2* __restrict__ x, float* __restrict__ th, int nv)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nv) return;
    th[3 * (size_t)nv + j] = x[j].x;
    th[4 * (size_t)nv + j] = x[j].y;
}

inline int grid_for(size_t n) { return (int)((n + 255) / 256); }

}  // namespace

hipError_t launch_sum_partials(const double* partials, int n, double* out, hipStream_t s)
{
    sum_partials_kernel<<<1, RB, 0, s>>>(partials, n, out);
    return hipGetLastError();
}

hipError_t launch_dot(const float* a, const float* b, size_t n, double* partials, double* out,
                      hipStream_t s)
{
    dot_kernel<<<RED_BLOCKS, RB, 0, s>>>(a, b, n, partials);
    sum_partials_kernel<<<1, RB, 0, s>>>(partials, RED_BLOCKS, out);
    return hipGetLastError();
}

hipError_t launch_dot_c(const float2* a, const float2* b, size_t n, double* partials,
                        double* out, hipStream_t s)
{
    dot_c_kernel<<<RED_BLOCKS, RB, 0, s>>>(a, b, n, partials);
    sum_partials_kernel<<<1, RB, 0, s>>>(partials, RED_BLOCKS, out);
    return hipGetLastError();
}

hipError_t launch_cg_init(const Dims& d, const float* g, float* step, float* res, float* dir,
                          double* scal, double* partials, hipStream_t s)
{
    const size_t n = (size_t)d.np * d.nv;
    cg_init_kernel<<<RED_BLOCKS, RB, 0, s>>>(g, step, res, dir, n, partials);
    cg_init_finish<<<1, RB, 0, s>>>(partials, RED_BLOCKS, scal);
    return hipGetLastError();
}

int cg_partials(const Dims& d) { return 5 * ((d.nv + 255) / 256); }

hipError_t launch_cg_update(const Dims& d, const float* q, float* step, float* res, float* dir,
                            double* scal, double* partials, int iter, hipStream_t s)
{
    // partials: [5][nb] from the finish kernel.
    const size_t n = (size_t)d.np * d.nv;
    const int nb = (d.nv + 255) / 256;
    cg_update_kernel<<<RED_BLOCKS, RB, 0, s>>>(q, step, res, dir, n, partials, nb, scal, iter & 1);
    return hipGetLastError();
}

int tr_partials(const Dims& d) { return 3 * ((d.nv + 255) / 256) + 2 * RED_BLOCKS; }

hipError_t launch_tr_init(double* scal, double delta2, hipStream_t s)
{
    tr_init_kernel<<<1, 64, 0, s>>>(scal, delta2);
    return hipGetLastError();
}

hipError_t launch_tr_update(const Dims& d, const float* q, float* step, float* res, float* dir,
                            double* scal, double* partials, int iter, hipStream_t s)
{
    // partials: curvature triples [3][nb] from the finish kernel, then
    // res.res and step.step [RED_BLOCKS] each.
    const size_t n = (size_t)d.np * d.nv;
    const int nb = (d.nv + 255) / 256;
    double* rrp = partials + 3 * nb;
    double* zzp = rrp + RED_BLOCKS;
    tr_step_kernel<<<RED_BLOCKS, RB, 0, s>>>(dir, q, step, res, n, partials, nb, scal, iter & 1, rrp, zzp);
    tr_dir_kernel<<<RED_BLOCKS, RB, 0, s>>>(res, dir, n, rrp, RED_BLOCKS, scal, iter & 1, zzp);
    return hipGetLastError();
}

hipError_t launch_tr_trial(const Dims& d, const float* theta, const float* step, const float* lo,
                           const float* hi, int param_mask, const uint8_t* mask, float* trial,
                           float* sv, double* scal, double* partials, hipStream_t s)
{
    tr_trial_kernel<<<RED_BLOCKS, RB, 0, s>>>(theta, step, box6(lo, hi), param_mask, mask, trial, sv, d.nv,
                                              d.np, partials);
    sum2_kernel<<<1, RB, 0, s>>>(partials, RED_BLOCKS, scal + SC_NREF);
    return hipGetLastError();
}

hipError_t launch_tr_accept(const Dims& d, double* scal, double eta, const float* trial, float* theta,
                            hipStream_t s)
{
    tr_accept_kernel<<<RED_BLOCKS, 256, 0, s>>>(scal, eta, trial, theta, (size_t)d.np * d.nv);
    return hipGetLastError();
}

hipError_t launch_ls_trial_masked(const Dims& d, const float* theta, const float* step, float t,
                                  const float* lo, const float* hi, int param_mask,
                                  const uint8_t* mask, float* trial, hipStream_t s)
{
    ls_trial_kernel<<<grid_for((size_t)d.np * d.nv), 256, 0, s>>>(theta, step, t, box6(lo, hi), param_mask,
                                                                  mask, trial, d.nv, d.np);
    return hipGetLastError();
}

hipError_t launch_pred_dot(const Dims& d, const float* g, const float* trial, const float* theta,
                           double* partials, double* out, hipStream_t s)
{
    const size_t n = (size_t)d.np * d.nv;
    pred_kernel<<<RED_BLOCKS, RB, 0, s>>>(g, trial, theta, n, partials);
    sum2_kernel<<<1, RB, 0, s>>>(partials, RED_BLOCKS, out);
    return hipGetLastError();
}

hipError_t launch_ls_accept(const Dims& d, double* scal, double c1, const float* trial, float* theta,
                            hipStream_t s)
{
    ls_accept_kernel<<<RED_BLOCKS, 256, 0, s>>>(scal, c1, trial, theta, (size_t)d.np * d.nv);
    return hipGetLastError();
}

hipError_t launch_set_rho(const Dims& d, const float* theta_in, const float2* p, float* theta_out,
                          hipStream_t s)
{
    set_rho_kernel<<<grid_for((size_t)d.np * d.nv), 256, 0, s>>>(theta_in, p, theta_out, d.nv, d.np);
    return hipGetLastError();
}

hipError_t launch_cgls_step_x(const Dims& d, float2* x, float2* p, const double* scal,
                              hipStream_t s)
{
    cgls_x_kernel<<<grid_for(d.nv), 256, 0, s>>>(x, p, d.nv, scal);
    return hipGetLastError();
}

hipError_t launch_cgls_step_r(size_t n, float2* r, const float2* q, const double* scal,
                              hipStream_t s)
{
    cgls_r_kernel<<<grid_for(n), 256, 0, s>>>(r, q, n, scal);
    return hipGetLastError();
}

hipError_t launch_cgls_dir(const Dims& d, float2* p, const float2* sv, const double* scal,
                           hipStream_t s)
{
    cgls_p_kernel<<<grid_for(d.nv), 256, 0, s>>>(p, sv, d.nv, scal);
    return hipGetLastError();
}

hipError_t launch_cgls_scalars(double* scal, int phase, hipStream_t s)
{
    cgls_scalar_kernel<<<1, 64, 0, s>>>(scal, phase);
    return hipGetLastError();
}

hipError_t launch_copy_rho_out(const Dims& d, const float2* x, float* theta, hipStream_t s)
{
    copy_rho_out_kernel<<<grid_for(d.nv), 256, 0, s>>>(x, theta, d.nv);
    return hipGetLastError();
}

}  // namespace mrstat
