// Readout dynamics (Discussion: the volumetric model follows T2 decay and
// Delta B0 phase accumulation during each readout). Sample k of every readout
// is taken at TE + tau_k, tau_k = (k - nk/2) dwell, and voxel j's transverse
// magnetisation carries
//     F[k, j] = exp(-tau_k / T2_j) exp(-2 pi i db0_j (TE + tau_k))
//             = c_j exp(lambda_j tau_k),   lambda_j = -1/T2_j - 2 pi i db0_j,
// c_j = exp(-2 pi i db0_j TE). F depends on voxel and sample together, so the
// Cartesian encoding no longer factors into a y-stage per TR and one x-stage.
// With u = tau / tau_max in [-1, 1] and L_j = lambda_j tau_max the factor is
// expanded as exp(L_j u) = sum_{q < NQ} L_j^q u^q / q! (NQ chosen at context
// creation so the remainder stays below 1e-7, the FP32 level, over the stated
// T2 and db0 bounds), which restores the factorisation term by term:
//     s[n,k] = sum_q (u_k^q / q!) sum_ix Ex[k,ix] U_q[n,ix],
//     U_q[n,ix] = sum_iy Ey[n,iy] c_j (x[n,j] L_j^q + y[n,j] q L_j^(q-1)),
// where x is the voxel weight of the static model and y the readout decay's
// share of the ln T2 column (d/dlnT2 exp(-tau/T2) = (tau/T2) exp(-tau/T2):
// y = i rho mu (tau_max / T2) v_lnT2, multiplied by u in the sum). With Delta
// B0 fitted (theta row 5, in units of db0_unit Hz) its column's factor
// -2 pi i db0_unit (TE + tau) splits the same way: the TE part joins x, the
// tau part y. With coils each coil's weight joins c_j. The sample weights
// u^q / q! are then re-expanded in Chebyshev polynomials (u^q = 2^(1-q)
// sum_j binom(q, j) T_(q-2j)(u), the T_0 term halved), which turns the U_q
// into NC <= NQ sums
//     V_m = sum_q e_mq U_q,   s[n,k] = sum_(m < NC) T_m(u_k) sum_ix Ex[k,ix] V_m[n,ix],
// dropping the Chebyshev terms from NC on, which stay below the same bound
// (Chebyshev economisation): the x-stage and the per-sample sum carry NC rows
// (16 instead of 24 at |L| = 3.8). The x-stage of each term is the library's
// x-GEMM with coils x terms as rows; this file holds the term-wise y-stages
// and the per-sample weighting.
//   forward:  rd_fwd_kernel (U_q summed, then V_m) -> x-GEMM (Y_m = Ex V_m)
//             -> rd_combine_kernel (s = sum_m T_m(u) Y_m, then r = d - s, -s
//             or s);
//   adjoint:  the same factor in the Chebyshev basis directly, exp(L u) =
//             sum_m a_m(L) T_m(u) and u exp(L u) = sum_m b_m(L) T_m(u), NC
//             terms; rd_expand_kernel (w_m = T_m(u) w) -> adjoint x-GEMM
//             (W_m = Ex^H w_m) -> rd_adj_kernel: per voxel and TR
//             V = sum_m conj(a_m) W_m, V' = sum_m conj(b_m) W_m,
//             A_p += mu_p conj(c Ey) V, A_lnT2 += (tau_max/T2) mu_0 conj(c Ey) V'
//             (V, V' summed over the coils with conj(C_c)). Forward and
//             adjoint each approximate the exact operator to the bound, so
//             they are transposes of each other to that bound, not exactly.
// FP32 arithmetic; the sums of the expansion are in the dimensionless u and L
// so no term over- or underflows.
#include "mrstat_internal.h"

#include <cmath>

namespace mrstat {
namespace {

constexpr float kTwoPi = 6.28318530717958647692f;
// TRs per forward block. Measured at 224 x 224, 1120 TRs, 24 terms (J v):
// the power chain per voxel and TR 0.67 ms; powers shared by the block's TRs
// 0.55 with 2 TRs, 0.57 with 1; the next row's inputs loaded while a row is
// summed 0.75 (221 registers: two waves per SIMD instead of three).
constexpr int RD_NTB = 2;

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

__device__ __forceinline__ void cmac(float2& acc, float2 a, float2 b)   // acc += a * b
{
    acc.x = fmaf(a.x, b.x, fmaf(-a.y, b.y, acc.x));
    acc.y = fmaf(a.x, b.y, fmaf(a.y, b.x, acc.y));
}

__device__ __forceinline__ float2 cfmaconj(float2 a, float2 b, float2 acc)   // acc + conj(a) * b
{
    return make_float2(fmaf(a.x, b.x, fmaf(a.y, b.y, acc.x)), fmaf(a.x, b.y, fmaf(-a.y, b.x, acc.y)));
}

__device__ __forceinline__ float2 cmulconj(float2 a, float2 b)   // conj(a) * b
{
    return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.x, b.y, -a.y * b.x));
}

// Per-voxel quantities of the expansion: L = lambda tau_max, r2t = tau_max / T2
// and c = exp(-2 pi i db0 TE).
struct RdVoxel {
    float2 L, c;
    float r2t;
};

__device__ __forceinline__ RdVoxel rd_voxel(const float* __restrict__ theta, const float* __restrict__ db0,
                                             float db0_unit, int nv, int j, float te, float tmax)
{
    RdVoxel o;
    const float r2 = expf(-theta[(size_t)nv + j]);   // theta row 1 = ln T2
    const float f = db0 ? db0[j] * db0_unit : 0.f;
    o.r2t = r2 * tmax;
    o.L = make_float2(-o.r2t, -kTwoPi * f * tmax);
    float sn, cs;
    sincosf(kTwoPi * f * te, &sn, &cs);
    o.c = make_float2(cs, -sn);
    return o;
}

// e_mq: the share of T_m(u) in u^q / q!, (m == 0 ? 1 : 2) 2^-q binom(q, j)
// / q! for m = q - 2j >= 0, else 0; built at compile time (FP64, rounded
// once), indexed with unrolled constants so every entry is an immediate.
template <int NQ>
struct EconTable {
    float e[NQ][NQ];
    constexpr EconTable() : e{}
    {
        for (int q = 0; q < NQ; ++q) {
            double w = 1.0;   // 2^-q / q!
            for (int i = 1; i <= q; ++i) w *= 0.5 / i;
            double bin = 1.0;   // binom(q, j)
            for (int j = 0; 2 * j <= q; ++j) {
                const int m = q - 2 * j;
                e[m][q] = (float)((m == 0 ? 1.0 : 2.0) * w * bin);
                bin = bin * (q - j) / (j + 1);
            }
        }
    }
};
template <int NQ>
__device__ constexpr EconTable<NQ> kEcon{};

// Forward term sums. Block = 256 lanes, one image column per lane (nx <=
// 256), RD_NTB TRs; the lanes walk all rows, keeping the NQ complex sums of
// each TR in registers; then the NC economised sums V_m = sum_q e_mq U_q
// written once per (term, TR, column), no partials.
// MODE as the static y-stages: 0 signal, 1 J v with four trains, 3 J v with
// three (B1 held fixed). db0 (Hz per db0_unit) is the map or theta row 5;
// with Delta B0 fitted (fit, J v only) the direction's row 5 adds
// -2 pi i db0_unit (TE + tau) rho mu v_5 to the voxel's derivative: its TE
// part joins x, its tau part y.
template <int MODE, int NQ, typename TT>
__global__ __launch_bounds__(256) void rd_fwd_kernel(const TT* __restrict__ trains, const float* __restrict__ theta,
                                                     const float* __restrict__ v, const float2* __restrict__ coil,
                                                     const uint8_t* __restrict__ mask,
                                                     const float* __restrict__ db0, float db0_unit, int fit,
                                                     const float2* __restrict__ eytab, float2* __restrict__ U,
                                                     int nc, int nx, int ny, int nv, int T, float te, float tmax)
{
    constexpr bool JV = MODE != 0, DB1 = MODE == 1;
    const int ix = threadIdx.x;
    const bool colok = ix < nx;
    const int n0 = blockIdx.x * RD_NTB;
    const int c = blockIdx.y;   // coil: its sums are rows c nc .. c nc + nc - 1
    const size_t plane = (size_t)T * nv;
    float2 acc[RD_NTB][NQ];
#pragma unroll
    for (int t = 0; t < RD_NTB; ++t)
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[t][q] = make_float2(0.f, 0.f);
    if (colok) {
        for (int iy = 0; iy < ny; ++iy) {
            const int j = iy * nx + ix;
            if (mask != nullptr && mask[j] == 0) continue;   // no contribution
            RdVoxel vx = rd_voxel(theta, db0, db0_unit, nv, j, te, tmax);
            if (coil != nullptr) vx.c = cmul(vx.c, coil[(size_t)c * nv + j]);   // the coil weight joins c
            const float rr = theta[3 * (size_t)nv + j], ri = theta[4 * (size_t)nv + j];
            float nr = 0.f, ni = 0.f, w0 = 0.f, w1 = 0.f, w2 = 0.f, cte = 0.f, ctau = 0.f;
            if constexpr (JV) {
                nr = v[3 * (size_t)nv + j];
                ni = v[4 * (size_t)nv + j];
                w0 = v[j];
                w1 = v[(size_t)nv + j];
                if constexpr (DB1) w2 = v[2 * (size_t)nv + j];
                if (fit) {   // 2 pi db0_unit v_5 times TE, and times tau_max
                    const float w5 = kTwoPi * db0_unit * v[5 * (size_t)nv + j];
                    cte = w5 * te;
                    ctau = w5 * tmax;
                }
            }
            // Powers L^q of this voxel, shared by the block's TRs.
            float2 P[NQ];
            P[0] = make_float2(1.f, 0.f);
#pragma unroll
            for (int q = 1; q < NQ; ++q) P[q] = cmul(P[q - 1], vx.L);
#pragma unroll
            for (int t = 0; t < RD_NTB; ++t) {
                const int n = min(n0 + t, T - 1);   // TRs past the end are not stored
                const TT* b = trains + (size_t)n * nv + j;
                const float mu = (float)b[0];
                float2 x, y = make_float2(0.f, 0.f);   // i rho mu / i (rho a + nu mu); i rho mu r2t v_lnT2
                if constexpr (!JV) {
                    x = make_float2(-ri * mu, rr * mu);
                } else {
                    const float m1 = (float)b[plane], m2 = (float)b[2 * plane];
                    const float a = DB1 ? fmaf(w0, m1, fmaf(w1, m2, w2 * (float)b[3 * plane])) : fmaf(w0, m1, w1 * m2);
                    // i (rho a + nu mu) + rho mu cte; i rho mu r2t w1 + rho mu ctau
                    const float e = mu * cte, et = mu * ctau, yt = mu * vx.r2t * w1;
                    x = make_float2(fmaf(rr, e, -fmaf(ri, a, ni * mu)), fmaf(ri, e, fmaf(rr, a, nr * mu)));
                    y = make_float2(fmaf(rr, et, -ri * yt), fmaf(ri, et, rr * yt));
                }
                const float2 ec = cmul(eytab[(size_t)n * ny + iy], vx.c);
                const float2 z = cmul(ec, x);
                acc[t][0].x += z.x;
                acc[t][0].y += z.y;
                if constexpr (JV) {
                    // z L^q + q zy L^(q-1) = (z L + q zy) L^(q-1)
                    const float2 zy = cmul(ec, y), zl = cmul(z, vx.L);
#pragma unroll
                    for (int q = 1; q < NQ; ++q)
                        cmac(acc[t][q], make_float2(fmaf((float)q, zy.x, zl.x), fmaf((float)q, zy.y, zl.y)), P[q - 1]);
                } else {
#pragma unroll
                    for (int q = 1; q < NQ; ++q) cmac(acc[t][q], z, P[q]);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < RD_NTB; ++t) {
            const int n = n0 + t;
            if (n >= T) continue;
#pragma unroll
            for (int m = 0; m < NQ; ++m) {
                float2 vm = make_float2(0.f, 0.f);
#pragma unroll
                for (int q = m; q < NQ; q += 2) {
                    vm.x = fmaf(kEcon<NQ>.e[m][q], acc[t][q].x, vm.x);
                    vm.y = fmaf(kEcon<NQ>.e[m][q], acc[t][q].y, vm.y);
                }
                if (m < nc) U[(((size_t)c * nc + m) * T + n) * nx + ix] = vm;
            }
        }
    }
}

// s_c[n,k] = sum_m T_m(u_k) Y_cm[n,k]; MODE 0: out = data - s and FP64
// partials of |out|^2 per block; 1: out = -s; 2: out = s.
template <int MODE>
__global__ __launch_bounds__(256) void rd_combine_kernel(const float2* __restrict__ Y, int nc, float dwell_u,
                                                         const float2* __restrict__ data, float2* __restrict__ out,
                                                         double* __restrict__ red, int C, int T, int nk)
{
    const size_t count = (size_t)T * nk;
    double sq = 0.0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < C * count; i += (size_t)gridDim.x * blockDim.x) {
        const size_t c = i / count, ii = i % count;
        const int k = (int)(ii % nk);
        const float u = (float)(k - nk / 2) * dwell_u;
        const float2* yc = Y + c * nc * count + ii;
        float2 s = yc[0];
        float tm1 = 1.f, tm = u;   // T_(m-1), T_m
        if (nc > 1) {
            s.x = fmaf(u, yc[count].x, s.x);
            s.y = fmaf(u, yc[count].y, s.y);
        }
        for (int m = 2; m < nc; ++m) {
            const float tn = fmaf(2.f * u, tm, -tm1);
            tm1 = tm;
            tm = tn;
            const float2 y = yc[(size_t)m * count];
            s.x = fmaf(tm, y.x, s.x);
            s.y = fmaf(tm, y.y, s.y);
        }
        if constexpr (MODE == 0) {
            const float2 d = data[i];
            const float2 r = make_float2(d.x - s.x, d.y - s.y);
            out[i] = r;
            sq += (double)r.x * (double)r.x + (double)r.y * (double)r.y;
        } else if constexpr (MODE == 1) {
            out[i] = make_float2(-s.x, -s.y);
        } else {
            out[i] = s;
        }
    }
    if constexpr (MODE == 0) {
        __shared__ double sh[4];
        for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = sq;
        __syncthreads();
        if (threadIdx.x == 0) red[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    }
}

// The adjoint's expansion (Chebyshev): w_cm[n,k] = T_m(u_k) w_c[n,k],
// m = 0 .. nc - 1, T_0 = 1, T_1 = u, T_(m+1) = 2 u T_m - T_(m-1).
__global__ __launch_bounds__(256) void rd_expand_kernel(const float2* __restrict__ w, float2* __restrict__ wq, int nc,
                                                        float dwell_u, int C, int T, int nk)
{
    const size_t count = (size_t)T * nk;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < C * count; i += (size_t)gridDim.x * blockDim.x) {
        const size_t c = i / count, ii = i % count;
        const int k = (int)(ii % nk);
        const float u = (float)(k - nk / 2) * dwell_u;
        const float2 x = w[i];
        float2* wc = wq + c * nc * count + ii;
        float tm1 = 1.f, tm = u;   // T_(m-1), T_m
        wc[0] = x;
        if (nc > 1) wc[count] = make_float2(u * x.x, u * x.y);
        for (int m = 2; m < nc; ++m) {
            const float tn = fmaf(2.f * u, tm, -tm1);
            tm1 = tm;
            tm = tn;
            wc[(size_t)m * count] = make_float2(tm * x.x, tm * x.y);
        }
    }
}

// Chebyshev coefficients of exp(L u) on [-1, 1]: a_m = eps_m I_m(L) (eps_0 =
// 1, else 2; I_m the modified Bessel function, as a power series in FP64,
// which for |L| <= 6 converges to 1e-17 within 20 terms); and those of
// u exp(L u): u T_0 = T_1, u T_m = (T_(m+1) + T_(m-1)) / 2, so b_0 = a_1 / 2,
// b_1 = a_0 + a_2 / 2, b_m = (a_(m-1) + a_(m+1)) / 2. Returned conjugated
// (the adjoint's coefficients), NC of each.
template <int NC>
__device__ __forceinline__ void cheb_coeffs(float2 Lf, float2 (&ca)[NC], float2 (&cb)[NC])
{
    const double hx = 0.5 * (double)Lf.x, hy = 0.5 * (double)Lf.y;   // h = L / 2
    const double h2x = hx * hx - hy * hy, h2y = 2.0 * hx * hy;       // h^2
    double a[NC + 1][2];
    double tx = 1.0, ty = 0.0;   // h^m / m!
#pragma unroll
    for (int m = 0; m <= NC; ++m) {
        double sx = tx, sy = ty, ex = tx, ey = ty;
        for (int j = 1; j <= 20; ++j) {
            const double f = 1.0 / ((double)j * (double)(m + j));
            const double nx = (ex * h2x - ey * h2y) * f, ny = (ex * h2y + ey * h2x) * f;
            ex = nx;
            ey = ny;
            sx += ex;
            sy += ey;
        }
        const double eps = m == 0 ? 1.0 : 2.0;
        a[m][0] = eps * sx;
        a[m][1] = eps * sy;
        const double f = 1.0 / (double)(m + 1);
        const double nx = (tx * hx - ty * hy) * f, ny = (tx * hy + ty * hx) * f;
        tx = nx;
        ty = ny;
    }
#pragma unroll
    for (int m = 0; m < NC; ++m) {
        ca[m] = make_float2((float)a[m][0], (float)-a[m][1]);
        double bx, by;
        if (m == 0) {
            bx = 0.5 * a[1][0];
            by = 0.5 * a[1][1];
        } else if (m == 1) {
            bx = a[0][0] + 0.5 * a[2][0];
            by = a[0][1] + 0.5 * a[2][1];
        } else {
            bx = 0.5 * (a[m - 1][0] + a[m + 1][0]);
            by = 0.5 * (a[m - 1][1] + a[m + 1][1]);
        }
        cb[m] = make_float2((float)bx, (float)-by);
    }
}

// Adjoint term sums: one thread per pair of voxels of a column and TR chunk;
// per TR the sums V = sum_m conj(a_m) W_m and V' = sum_m conj(b_m) W_m over
// the Chebyshev terms (each voxel's coefficients held in registers across
// its TRs), then the chunk partials A_p
// in the layout the gradient assembly reads ([chunk][pl planes][nv], pl = 8,
// or 10 with Delta B0 fitted; NTR = 1 writes the m pair only, 2 planes, for
// the proton-density initialisation). With Delta B0 fitted (fit, NTR >= 3)
// its pair is A_5 = 2 pi i db0_unit sum_n mu conj(c Ey) (TE V + tau_max V').
// Measured at 224 x 224, 1120 TRs, 24 terms (per J^H w): the Horner form
// 0.83 ms; the power coefficients in registers with the term loads batched
// (two waves per SIMD) 0.80; with a tile of 64 columns x 4 rows per block
// for cache reuse of W 0.92; double-buffered term loads need 256 registers;
// two voxels of a column per thread, sharing each TR's term loads, 0.59; the
// Chebyshev form, 16 terms for the same bound, 0.52 (and its adjoint x-GEMM
// 0.084 instead of 0.122). TR chunks (HIP events, 16 terms): 9 chunks
// 0.53-0.57, 18 0.55; 8, 16, 24 and 32 chunks with each XCD given its own
// chunks (so its L2 holds only their term values) 0.58, 0.60, 0.58, 0.61.
// V' from the a_m alone (u T_m = (T_(m-1) + T_(m+1)) / 2 moved onto the term
// values: 201 registers instead of 233, still two waves per SIMD) 0.60.
// Voxels per thread of the adjoint (rows iy, iy + hy, ... of one column):
// two while each voxel's coefficients and the loaded terms fit the registers.
template <int NQ>
constexpr int rd_adj_rows() { return NQ <= 16 ? 2 : 1; }

template <int NTR, int NQ, typename TT, bool MC>   // MC: coil maps (C >= 1 weighted coils)
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void rd_adj_kernel(const TT* __restrict__ trains, const float* __restrict__ theta,
                                                     const float2* __restrict__ coil,
                                                     const uint8_t* __restrict__ mask, const float* __restrict__ db0,
                                                     float db0_unit, int fit, const float2* __restrict__ eytab,
                                                     const float2* __restrict__ W, float* __restrict__ apart,
                                                     int nx, int ny, int nv, int T, int C, int n_per_chunk, float te,
                                                     float tmax)
{
    const bool f5 = NTR >= 3 && fit;
    const int pl = NTR == 1 ? 2 : (f5 ? 10 : 8);   // planes per chunk
    // A thread takes rows iy, iy + hy, ... of column ix: they read the same
    // term values W_q[n][ix], loaded once per TR for all of them.
    constexpr int R = rd_adj_rows<NQ>();
    const int hy = (ny + R - 1) / R;
    const int jp = blockIdx.x * blockDim.x + threadIdx.x;
    const int chunk = blockIdx.y;
    if (jp >= hy * nx) return;
    const int ix = jp % nx, iy0 = jp / nx;
    const int n0 = chunk * n_per_chunk, n1 = min(T, n0 + n_per_chunk);
    const size_t plane = (size_t)T * nv, wplane = (size_t)T * nx;
    int jv[R], iyv[R];
    bool on[R];
    RdVoxel vx[R];
    // Each voxel's coefficients, fixed over its TRs: conj(a_m), conj(b_m).
    float2 Ca[R][NQ], Cb[R][NQ];
    float2 A[R][NTR], At[R], Af[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        iyv[r] = iy0 + r * hy;
        jv[r] = iyv[r] < ny ? iyv[r] * nx + ix : -1;
        on[r] = jv[r] >= 0 && (mask == nullptr || mask[jv[r]] != 0);
        vx[r] = rd_voxel(theta, db0, db0_unit, nv, on[r] ? jv[r] : jp % nv, te, tmax);
        cheb_coeffs<NQ>(vx[r].L, Ca[r], Cb[r]);
#pragma unroll
        for (int p = 0; p < NTR; ++p) A[r][p] = make_float2(0.f, 0.f);
        At[r] = Af[r] = make_float2(0.f, 0.f);
    }
    // Per TR and voxel: A_p += mu_p conj(c Ey) V, the ln T2 share with V' and
    // the Delta B0 pair with both (V, V' already summed over the coils).
    auto accumulate = [&](int n, int r, float2 V, float2 Vt) {
        const float2 ec = cmul(eytab[(size_t)n * ny + iyv[r]], vx[r].c);   // c Ey
        V = cmulconj(ec, V);
        const TT* b = trains + (size_t)n * nv + jv[r];
#pragma unroll
        for (int p = 0; p < NTR; ++p) {
            const float m = (float)b[p * plane];
            A[r][p].x = fmaf(m, V.x, A[r][p].x);
            A[r][p].y = fmaf(m, V.y, A[r][p].y);
        }
        if constexpr (NTR >= 3) {
            Vt = cmulconj(ec, Vt);
            const float mu = (float)b[0], m0 = mu * vx[r].r2t;
            At[r].x = fmaf(m0, Vt.x, At[r].x);
            At[r].y = fmaf(m0, Vt.y, At[r].y);
            if (f5) {
                Af[r].x = fmaf(mu, fmaf(te, V.x, tmax * Vt.x), Af[r].x);
                Af[r].y = fmaf(mu, fmaf(te, V.y, tmax * Vt.y), Af[r].y);
            }
        }
    };
    // V = sum_m conj(a_m) W_m and V' = sum_m conj(b_m) W_m of one coil, from
    // its TR's term values loaded together (all in flight at once).
    auto term_sums = [&](const float2 (&wv)[NQ], int r, float2& V, float2& Vt) {
        V = make_float2(0.f, 0.f);
        Vt = make_float2(0.f, 0.f);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            cmac(V, wv[q], Ca[r][q]);
            if constexpr (NTR >= 3) cmac(Vt, wv[q], Cb[r][q]);
        }
    };
    for (int n = n0; n < n1; ++n) {
        float2 wv[NQ];
        if constexpr (!MC) {
            const float2* w = W + (size_t)n * nx + ix;
#pragma unroll
            for (int q = 0; q < NQ; ++q) wv[q] = w[(size_t)q * wplane];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (!on[r]) continue;
                float2 V, Vt;
                term_sums(wv, r, V, Vt);
                accumulate(n, r, V, Vt);
            }
        } else {
            // Coils: V and V' weighted by conj(C_c) and summed over c first.
            float2 V[R], Vt[R];
#pragma unroll
            for (int r = 0; r < R; ++r) V[r] = Vt[r] = make_float2(0.f, 0.f);
            for (int c = 0; c < C; ++c) {
                const float2* w = W + (size_t)c * NQ * wplane + (size_t)n * nx + ix;
#pragma unroll
                for (int q = 0; q < NQ; ++q) wv[q] = w[(size_t)q * wplane];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (!on[r]) continue;
                    float2 Vc, Vtc;
                    term_sums(wv, r, Vc, Vtc);
                    const float2 cw = coil[(size_t)c * nv + jv[r]];
                    V[r] = cfmaconj(cw, Vc, V[r]);
                    Vt[r] = cfmaconj(cw, Vtc, Vt[r]);
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (on[r]) accumulate(n, r, V[r], Vt[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (jv[r] < 0) continue;
        float* dst = apart + (size_t)chunk * pl * nv + jv[r];
        if constexpr (NTR >= 3) {
            A[r][2].x += At[r].x;   // the readout decay's share of the ln T2 column
            A[r][2].y += At[r].y;
        }
#pragma unroll
        for (int p = 0; p < NTR; ++p) {   // zeros for a masked voxel
            dst[(size_t)(2 * p) * nv] = A[r][p].x;
            dst[(size_t)(2 * p + 1) * nv] = A[r][p].y;
        }
        if (f5) {   // times 2 pi i db0_unit
            const float k = kTwoPi * db0_unit;
            dst[(size_t)8 * nv] = -k * Af[r].y;
            dst[(size_t)9 * nv] = k * Af[r].x;
        }
    }
}

template <int NQ, typename TT>
hipError_t fwd_q(const Dims& d, int mode, int nc, const TT* trains, const float* theta, const float* v,
                 const float2* coil, const uint8_t* mask, const float* db0, float db0_unit, const float2* eytab,
                 float2* U, float te, float tmax, hipStream_t s)
{
    if (nc < 1 || nc > NQ) return hipErrorInvalidValue;
    const dim3 grid(ceil_div(d.T, RD_NTB), d.C);
    const int fit = d.np == 6;
#define RD_FWD(M)                                                                                                 \
    rd_fwd_kernel<M, NQ, TT><<<grid, 256, 0, s>>>(trains, theta, v, coil, mask, db0, db0_unit, fit, eytab, U, nc, \
                                                  d.nx, d.ny, d.nv, d.T, te, tmax)
    switch (mode) {
    case 0: RD_FWD(0); break;
    case 1: RD_FWD(1); break;
    case 3: RD_FWD(3); break;
    default: return hipErrorInvalidValue;
    }
#undef RD_FWD
    return hipGetLastError();
}

template <int NQ, typename TT>
hipError_t adj_q(const Dims& d, int ntr, int chunks, const TT* trains, const float* theta, const float2* coil,
                 const uint8_t* mask, const float* db0, float db0_unit, const float2* eytab, const float2* W,
                 float* apart, float te, float tmax, hipStream_t s)
{
    const int per = ceil_div(d.T, chunks);
    if (chunks < 1 || ceil_div(d.T, per) != chunks) return hipErrorInvalidValue;
    constexpr int R = rd_adj_rows<NQ>();
    const dim3 grid(ceil_div((d.ny + R - 1) / R * d.nx, 256), chunks);
    const int fit = d.np == 6;
    // Without coil maps there is one unweighted coil.
    if (coil == nullptr && d.C != 1) return hipErrorInvalidValue;
#define RD_ADJ(NT, MC) rd_adj_kernel<NT, NQ, TT, MC><<<grid, 256, 0, s>>>(trains, theta, coil, mask, db0, db0_unit, fit, \
                                                                         eytab, W, apart, d.nx, d.ny, d.nv, d.T, d.C, \
                                                                         per, te, tmax)
#define RD_ADJ_NT(MC)         \
    if (ntr == 1)             \
        RD_ADJ(1, MC);        \
    else if (ntr == 3)        \
        RD_ADJ(3, MC);        \
    else if (ntr == 4)        \
        RD_ADJ(4, MC);        \
    else                      \
        return hipErrorInvalidValue;
    if (coil != nullptr) {
        RD_ADJ_NT(true)
    } else {
        RD_ADJ_NT(false)
    }
#undef RD_ADJ_NT
#undef RD_ADJ
    return hipGetLastError();
}

}  // namespace

int rd_terms(double bound)
{
    // Smallest term count from {8, 12, 16, 20, 24, 32} whose remainder bound
    // L^(NQ-1) / (NQ-1)! e^L (the ln T2 share's expansion stops one order
    // earlier than the factor's) stays below 1e-7; 0 when none does.
    const int choices[] = {8, 12, 16, 20, 24, 32};
    for (int nq : choices) {
        double t = std::exp(bound);
        for (int q = 1; q <= nq - 1; ++q) t *= bound / q;
        if (t <= 1e-7) return nq;
    }
    return 0;
}

int rd_cheb_terms(double bound)
{
    // Smallest term count NC from {8, 12, 16, 20, 24, 32} for the adjoint's
    // Chebyshev expansion: its remainder (the u exp(L u) share, which drops
    // a_NC, is the larger) is at most 2 sum_(m >= NC - 1) |I_m(L)| with
    // |I_m(L)| <= (b/2)^m / m! e^(b^2 / (4 (m + 1))), b >= |L|, bounded by
    // 2 (b/2)^(NC-1) / (NC-1)! e^(b^2 / (4 NC)) / (1 - b / (2 NC)); kept below
    // 1e-7; 0 when none does.
    const int choices[] = {8, 12, 16, 20, 24, 32};
    for (int nc : choices) {
        const double r = bound / (2.0 * nc);
        if (r >= 1.0) continue;
        double t = 2.0;
        for (int m = 1; m <= nc - 1; ++m) t *= 0.5 * bound / m;
        t *= std::exp(bound * bound / (4.0 * nc)) / (1.0 - r);
        if (t <= 1e-7) return nc;
    }
    return 0;
}

#define RD_NQ_DISPATCH(NQ_VAR, CALL)                                     \
    switch (NQ_VAR) {                                                    \
    case 8: { constexpr int NQ = 8; return CALL; }                       \
    case 12: { constexpr int NQ = 12; return CALL; }                     \
    case 16: { constexpr int NQ = 16; return CALL; }                     \
    case 20: { constexpr int NQ = 20; return CALL; }                     \
    case 24: { constexpr int NQ = 24; return CALL; }                     \
    case 32: { constexpr int NQ = 32; return CALL; }                     \
    default: return hipErrorInvalidValue;                                \
    }

// The off-resonance source: theta row 5 in units of db0_unit Hz when Delta
// B0 is fitted, else the map (Hz, or none).
static void rd_source(const Dims& d, const float* theta, const float*& db0, float& unit)
{
    if (d.np == 6) {
        db0 = theta + (size_t)5 * d.nv;
    } else {
        unit = 1.f;
    }
}

hipError_t launch_rd_fwd(const Dims& d, int nq, int nc, int mode, const void* trains, bool f16, const float* theta,
                         const float* v, const float2* coil, const uint8_t* mask, const float* db0, float db0_unit,
                         const float2* eytab, float2* U, float te, float tmax, hipStream_t s)
{
    if (d.nx > 256) return hipErrorInvalidValue;
    rd_source(d, theta, db0, db0_unit);
    if (f16) {
        const _Float16* tr = static_cast<const _Float16*>(trains);
        RD_NQ_DISPATCH(nq, (fwd_q<NQ>(d, mode, nc, tr, theta, v, coil, mask, db0, db0_unit, eytab, U, te, tmax, s)))
    }
    const float* tr = static_cast<const float*>(trains);
    RD_NQ_DISPATCH(nq, (fwd_q<NQ>(d, mode, nc, tr, theta, v, coil, mask, db0, db0_unit, eytab, U, te, tmax, s)))
}

hipError_t launch_rd_combine(const Dims& d, int nc, int mode, const float2* Y, float dwell_u, const float2* data,
                             float2* out, double* red, int* nred, hipStream_t s)
{
    const int blocks = RED_BLOCKS;
    if (nred) *nred = blocks;
    switch (mode) {
    case 0: rd_combine_kernel<0><<<blocks, 256, 0, s>>>(Y, nc, dwell_u, data, out, red, d.C, d.T, d.nk); break;
    case 1: rd_combine_kernel<1><<<blocks, 256, 0, s>>>(Y, nc, dwell_u, data, out, red, d.C, d.T, d.nk); break;
    case 2: rd_combine_kernel<2><<<blocks, 256, 0, s>>>(Y, nc, dwell_u, data, out, red, d.C, d.T, d.nk); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_rd_expand(const Dims& d, int nc, float dwell_u, const float2* w, float2* wq, hipStream_t s)
{
    rd_expand_kernel<<<RED_BLOCKS, 256, 0, s>>>(w, wq, nc, dwell_u, d.C, d.T, d.nk);
    return hipGetLastError();
}

hipError_t launch_rd_adj(const Dims& d, int nq, int ntr, int chunks, const void* trains, bool f16,
                         const float* theta, const float2* coil, const uint8_t* mask, const float* db0,
                         float db0_unit, const float2* eytab, const float2* W, float* apart, float te, float tmax,
                         hipStream_t s)
{
    rd_source(d, theta, db0, db0_unit);
    if (f16) {
        const _Float16* tr = static_cast<const _Float16*>(trains);
        RD_NQ_DISPATCH(nq, (adj_q<NQ>(d, ntr, chunks, tr, theta, coil, mask, db0, db0_unit, eytab, W, apart, te,
                                      tmax, s)))
    }
    const float* tr = static_cast<const float*>(trains);
    RD_NQ_DISPATCH(nq, (adj_q<NQ>(d, ntr, chunks, tr, theta, coil, mask, db0, db0_unit, eytab, W, apart, te, tmax,
                                  s)))
}

#undef RD_NQ_DISPATCH

}  // namespace mrstat
