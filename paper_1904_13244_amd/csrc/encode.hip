// Encoding contraction kernels: the separable evaluation of
//     s_c[n,k] = sum_j C_c[j] x[n,j] E[n,k,j],
//     E[n,k,j] = Ex[k,ix] Ey[n,iy]
// (voxel j = iy*nx + ix), and of its adjoint. Cartesian sampling makes the
// phase factor over x and y, so the voxel sum splits into
//   y-stage  U_c[n,ix] = sum_iy Ey[n,iy] C_c[j] x[n,j]   (streams the trains;
//            HBM bound, one pass over the per-voxel trains per product)
//   x-stage  s_c[n,k]  = sum_ix Ex[k,ix] U_c[n,ix]        (dense complex GEMM on
//            the matrix cores, phase tiles staged in LDS)
// and the adjoint applies the conjugate phases in the opposite order.
//
// Trains hold Im m (and Im dm/dtheta): m = i mu. The voxel weight x is
//   mode 0 (signal):   x = rho m           = i rho mu
//   mode 1 (J v dir.): x = sum_q D_q v_q   = i (rho a + nu mu),
//                      a = v0 mu1 + v1 mu2 + v2 mu3, nu = v3 + i v4
//   mode 3 (J v dir., B1 held fixed): as mode 1 with v2 = 0, so the dm/dB1
//                      train is neither needed nor read
// (D_q = d(rho m)/d alpha_q, the Jacobian columns of the Theory section).
//
// Lane layout of both y-stages: a wave covers 32 consecutive ix (lanes 0-31
// and 32-63) of two adjacent rows, so nx only needs to be a multiple of 32
// for full lanes; consecutive lanes read consecutive elements of a train row.
// Trains are stored as float or _Float16 (TT); arithmetic is FP32.
#include "mrstat_internal.h"

#include <type_traits>

namespace mrstat {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

__device__ __forceinline__ float2 cfma(float2 a, float2 b, float2 c)   // a*b + c
{
    return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, c.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, c.y)));
}

__device__ __forceinline__ float2 cmulconj(float2 a, float2 b)   // conj(a) * b
{
    return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.x, b.y, -a.y * b.x));
}

__device__ __forceinline__ float2 shfl_xor2(float2 v, int m)
{
    return make_float2(__shfl_xor(v.x, m), __shfl_xor(v.y, m));
}

// TR chunk of a forward y-stage block. The adjoint y-stage visits TR chunks
// in increasing order; the forward kernels visit them in decreasing order, so
// each kernel starts on the trains the previous one read last.
__device__ __forceinline__ int fwd_chunk(unsigned b, unsigned nb)
{
    return (int)(nb - 1 - b);
}

// ------------------------------------------------------------------------
// Forward y-stage. Block = FW = 16 waves; wave w, half h covers row
// iy = rowbase + 32 r + 2 w + h for r < R, and ix = 32 bx + lane % 32. A block
// therefore spans 32 R rows (all rows when ny <= 32 R: U is complete and no
// partial sums are written). Each thread keeps its R voxels' weights (and
// coil sensitivities) in registers for its TR chunk. Per TR every lane first
// issues all of its loads (clamped indices, no branches between them), then
// accumulates; the two rows of a wave are folded with a lane swap and the
// per-wave sums of the whole chunk are kept in LDS and reduced after a
// single barrier.
// ------------------------------------------------------------------------
constexpr int FW = 16;

// Lane layouts (G):
//  G = 0: two rows of 32 columns per wave (lanes 0-31 and 32-63), a block of
//         32 columns; a wave reads one 128-byte line per row of FP32 trains.
//  G >= 1: one row of 64 columns per wave and G column groups per block, so
//         a block spans 64 G columns (all of them when 64 G >= nx) and FW / G
//         row groups. With 2-byte trains a row is not a whole number of
//         lines in general (448 bytes at 224 columns); spanning all columns
//         keeps both halves of every line inside one block.
template <int MODE, int R, int CC, typename TT, int G>
__global__ __launch_bounds__(1024) void ystage_fwd_kernel(
    const TT* __restrict__ trains, const float* __restrict__ theta, const float* __restrict__ v,
    const float2* __restrict__ coil, const uint8_t* __restrict__ mask,
    const float2* __restrict__ eytab, float2* __restrict__ U, int nx, int ny, int nv, int T, int C,
    int n_per_chunk)
{
    constexpr int XW = G == 0 ? 32 : 64 * G;          // columns per block
    constexpr int RS = G == 0 ? 2 * FW : FW / G;      // rows per step of the block
    constexpr int NS = G == 0 ? FW : FW / G;          // partial sums per column
    // LDS: per-wave sums [TRs per chunk][CC][NS][XW], then the block's
    // y-phases [TRs per chunk][RS R].
    extern __shared__ float2 lds[];
    float2* eys = lds + (size_t)n_per_chunk * CC * NS * XW;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int half = G == 0 ? lane >> 5 : 0;
    const int xl = G == 0 ? lane & 31 : (wave % (G == 0 ? 1 : G)) * 64 + lane;
    const int rowoff = G == 0 ? 2 * wave + half : wave / (G == 0 ? 1 : G);
    const int slot = G == 0 ? wave : wave / (G == 0 ? 1 : G);   // partial-sum row
    const int ix = blockIdx.x * XW + xl;
    const int yb = blockIdx.y;
    const int iyb = yb * RS * R + rowoff;
    const int n0 = fwd_chunk(blockIdx.z, gridDim.z) * n_per_chunk;
    const int n1 = min(T, n0 + n_per_chunk);
    const bool colok = ix < nx;
    const size_t plane = (size_t)T * nv;
    for (int e = threadIdx.x; e < (n1 - n0) * RS * R; e += blockDim.x) {
        const int nl = e / (RS * R), rr = e % (RS * R);
        const int iy = yb * RS * R + rr;
        eys[e] = iy < ny ? eytab[(size_t)(n0 + nl) * ny + iy] : make_float2(0.f, 0.f);
    }
    __syncthreads();

    constexpr bool JV = MODE != 0, DB1 = MODE == 1;   // J v direction; with the dm/dB1 train
    float2 P[R], Q[R];
    float v0[R], v1[R], v2[R];
    int jr[R], iyr[R];
    float2 cw[R][CC];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int iy = iyb + RS * r;
        const bool ok = colok && iy < ny;
        const int j = ok ? iy * nx + ix : 0;   // invalid voxels read voxel 0 with zero weight
        jr[r] = j;
        iyr[r] = ok ? iy : 0;
        const bool on = ok && (mask == nullptr || mask[j] != 0);
        const float rr = on ? theta[3 * nv + j] : 0.f, ri = on ? theta[4 * nv + j] : 0.f;
        P[r] = make_float2(-ri, rr);   // i rho
        if constexpr (JV) {
            const float nr = on ? v[3 * nv + j] : 0.f, ni = on ? v[4 * nv + j] : 0.f;
            Q[r] = make_float2(-ni, nr);   // i nu
            v0[r] = on ? v[j] : 0.f;
            v1[r] = on ? v[nv + j] : 0.f;
            if constexpr (DB1) v2[r] = on ? v[2 * nv + j] : 0.f;
        }
        if constexpr (CC > 1) {
#pragma unroll
            for (int c = 0; c < CC; ++c)
                cw[r][c] = (ok && c < C) ? coil[(size_t)c * nv + j] : make_float2(0.f, 0.f);
        }
    }

    for (int n = n0; n < n1; ++n) {
        // Loads of this TR for all R voxels.
        // Uniform row bases (scalar registers) plus 32-bit lane offsets.
        float mu[R], m1[R], m2[R], m3[R];
        float2 ey[R];
        const TT* __restrict__ b0 = trains + (size_t)n * nv;
        const TT* __restrict__ b1 = b0 + plane;
        const TT* __restrict__ b2 = b1 + plane;
        const TT* __restrict__ b3 = b2 + plane;
        const float2* eyrow = eys + (size_t)(n - n0) * RS * R + rowoff;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            mu[r] = (float)b0[jr[r]];
            if constexpr (JV) {
                m1[r] = (float)b1[jr[r]];
                m2[r] = (float)b2[jr[r]];
            }
            if constexpr (DB1) m3[r] = (float)b3[jr[r]];
            ey[r] = eyrow[RS * r];
        }
        float2 acc[CC];
#pragma unroll
        for (int c = 0; c < CC; ++c) acc[c] = make_float2(0.f, 0.f);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            float2 x;
            if constexpr (MODE == 0) {
                x = make_float2(P[r].x * mu[r], P[r].y * mu[r]);
            } else {
                const float a = DB1 ? fmaf(v0[r], m1[r], fmaf(v1[r], m2[r], v2[r] * m3[r]))
                                    : fmaf(v0[r], m1[r], v1[r] * m2[r]);
                x = make_float2(fmaf(P[r].x, a, Q[r].x * mu[r]), fmaf(P[r].y, a, Q[r].y * mu[r]));
            }
            const float2 z = cmul(ey[r], x);
            if constexpr (CC == 1) {
                acc[0].x += z.x;
                acc[0].y += z.y;
            } else {
#pragma unroll
                for (int c = 0; c < CC; ++c) acc[c] = cfma(cw[r][c], z, acc[c]);
            }
        }
#pragma unroll
        for (int c = 0; c < CC; ++c) {
            if constexpr (G == 0) {
                const float2 t = shfl_xor2(acc[c], 32);
                if (half == 0)
                    lds[(((n - n0) * CC + c) * NS + slot) * XW + xl] =
                        make_float2(acc[c].x + t.x, acc[c].y + t.y);
            } else {
                lds[(((n - n0) * CC + c) * NS + slot) * XW + xl] = acc[c];
            }
        }
    }
    __syncthreads();
    const int nout = (n1 - n0) * CC * XW;
    for (int o = threadIdx.x; o < nout; o += blockDim.x) {
        const int l = o % XW, bc = o / XW;   // bc = TR-in-chunk * CC + c
        float2 s = lds[(bc * NS) * XW + l];
#pragma unroll
        for (int w = 1; w < NS; ++w) {
            const float2 t = lds[(bc * NS + w) * XW + l];
            s.x += t.x;
            s.y += t.y;
        }
        const int b = bc / CC, c = bc % CC;
        const int oix = blockIdx.x * XW + l;
        if (oix < nx && c < C) U[(((size_t)yb * C + c) * T + (n0 + b)) * nx + oix] = s;
    }
}

// ------------------------------------------------------------------------
// Forward y-stage, wide layout (FP16 trains, one coil, nx a multiple of 4
// and at most 256, 16-byte aligned operands). Each lane owns 4 consecutive
// columns, so one load moves 4 train elements (8 bytes) and a wave covers a
// whole row. Loop order is the transpose of the kernels above: a
// block takes NT TRs and a slab of rows; its NW waves walk the slab's rows
// (wave w: rows y0 + w, y0 + w + NW, ...), loading each voxel's weights
// (from L2: they are shared by every TR chunk) and its NT TRs of trains, and
// keep the NT per-column sums in registers. One LDS reduction across the
// waves per block; U partial sums per row slab.
// ------------------------------------------------------------------------
template <typename TT> struct Vec4;
template <> struct Vec4<_Float16> { typedef _Float16 T __attribute__((ext_vector_type(4))); };

template <int MODE, int NT, int NW, typename TT>
__global__ __launch_bounds__(NW * 64)
void ystage_fwd_wide_kernel(
    const TT* __restrict__ trains, const float* __restrict__ theta, const float* __restrict__ v,
    const uint8_t* __restrict__ mask, const float2* __restrict__ eytab, float2* __restrict__ U,
    int nx, int ny, int nv, int T, int rows)
{
    typedef typename Vec4<TT>::T V4;
    constexpr bool JV = MODE != 0, DB1 = MODE == 1;   // J v direction; with the dm/dB1 train
    // LDS: per-wave sums [NW][NT][nx], then the slab's y-phases [NT][rows].
    extern __shared__ float2 lds[];
    float2* eys = lds + (size_t)NW * NT * nx;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int x0 = 4 * lane;
    const bool colok = x0 < nx;
    const int yb = blockIdx.x;
    const int y0 = yb * rows, y1 = min(ny, y0 + rows);
    const int n0 = fwd_chunk(blockIdx.y, gridDim.y) * NT;
    const int nt = min(NT, T - n0);
    const size_t plane = (size_t)T * nv;
    for (int e = threadIdx.x; e < NT * rows; e += blockDim.x) {
        const int t = e / rows, iy = y0 + e % rows;
        eys[e] = (t < nt && iy < y1) ? eytab[(size_t)(n0 + t) * ny + iy] : make_float2(0.f, 0.f);
    }
    __syncthreads();

    float2 acc[NT][4];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[t][c] = make_float2(0.f, 0.f);
    // TRs past the end of the sequence read the chunk's first TR; their sums
    // are never stored.
    size_t toff[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) toff[t] = (size_t)(n0 + (t < nt ? t : 0)) * nv;

    if (colok) {
        for (int iy = y0 + wave; iy < y1; iy += NW) {
            const int j = iy * nx + x0;
            f4 pr = *(const f4*)(theta + 3 * (size_t)nv + j);
            f4 pi = *(const f4*)(theta + 4 * (size_t)nv + j);
            f4 qr, qi, w0, w1, w2;
            if constexpr (JV) {
                qr = *(const f4*)(v + 3 * (size_t)nv + j);
                qi = *(const f4*)(v + 4 * (size_t)nv + j);
                w0 = *(const f4*)(v + j);
                w1 = *(const f4*)(v + (size_t)nv + j);
                if constexpr (DB1) w2 = *(const f4*)(v + 2 * (size_t)nv + j);
            }
            V4 m0[NT], m1[NT], m2[NT], m3[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const TT* b = trains + toff[t] + j;
                // Plain loads: with the adjoint's, measured faster than
                // non-temporal ones (each kernel then starts on trains the
                // other left in the caches).
                m0[t] = *(const V4*)b;
                if constexpr (JV) {
                    m1[t] = *(const V4*)(b + plane);
                    m2[t] = *(const V4*)(b + 2 * plane);
                }
                if constexpr (DB1) m3[t] = *(const V4*)(b + 3 * plane);
            }
            if (mask != nullptr) {   // masked voxels: zero weights (selects, not products)
                const uchar4 mk = *(const uchar4*)(mask + j);
                const bool on[4] = {mk.x != 0, mk.y != 0, mk.z != 0, mk.w != 0};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    pr[c] = on[c] ? pr[c] : 0.f;
                    pi[c] = on[c] ? pi[c] : 0.f;
                    if constexpr (JV) {
                        qr[c] = on[c] ? qr[c] : 0.f;
                        qi[c] = on[c] ? qi[c] : 0.f;
                        w0[c] = on[c] ? w0[c] : 0.f;
                        w1[c] = on[c] ? w1[c] : 0.f;
                    }
                    if constexpr (DB1) w2[c] = on[c] ? w2[c] : 0.f;
                }
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const float2 ey = eys[t * rows + (iy - y0)];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const float mu = (float)m0[t][c];
                    float2 x;   // i rho mu (mode 0); i (rho a + nu mu) (modes 1, 3)
                    if constexpr (MODE == 0) {
                        x = make_float2(-pi[c] * mu, pr[c] * mu);
                    } else {
                        const float a =
                            DB1 ? fmaf(w0[c], (float)m1[t][c],
                                       fmaf(w1[c], (float)m2[t][c], w2[c] * (float)m3[t][c]))
                                : fmaf(w0[c], (float)m1[t][c], w1[c] * (float)m2[t][c]);
                        x = make_float2(-fmaf(pi[c], a, qi[c] * mu), fmaf(pr[c], a, qr[c] * mu));
                    }
                    acc[t][c] = cfma(ey, x, acc[t][c]);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            f4* dst = (f4*)(lds + ((size_t)wave * NT + t) * nx + x0);
            dst[0] = f4{acc[t][0].x, acc[t][0].y, acc[t][1].x, acc[t][1].y};
            dst[1] = f4{acc[t][2].x, acc[t][2].y, acc[t][3].x, acc[t][3].y};
        }
    }
    __syncthreads();
    for (int o = threadIdx.x; o < nt * nx; o += blockDim.x) {
        const int t = o / nx, ix = o % nx;
        float2 s = lds[(size_t)t * nx + ix];
#pragma unroll
        for (int w = 1; w < NW; ++w) {
            const float2 u = lds[((size_t)w * NT + t) * nx + ix];
            s.x += u.x;
            s.y += u.y;
        }
        U[((size_t)yb * T + n0 + t) * nx + ix] = s;
    }
}

// ------------------------------------------------------------------------
// Forward y-stage with coils (CC = 8 or 16 coil slots). The per-wave sums of
// CC coils make the chunk-wide LDS staging above hold only 1-2 TRs, so the
// voxel weights and coil maps would be re-read every 2 TRs. Here each TR's
// per-wave sums go to one of two LDS buffers and are reduced across the
// waves right after a single barrier (the next TR uses the other buffer), so
// a block streams a long TR chunk with its voxels' weights and coil maps in
// registers. The next TR's trains are loaded before that barrier. Layout as
// G = 0 above: two rows of 32 columns per wave, R row steps per lane.
// ------------------------------------------------------------------------
template <int MODE, int R, int CC, typename TT, int TB>
__global__ __launch_bounds__(1024) void ystage_fwd_coil_kernel(
    const TT* __restrict__ trains, const float* __restrict__ theta, const float* __restrict__ v,
    const float2* __restrict__ coil, const uint8_t* __restrict__ mask,
    const float2* __restrict__ eytab, float2* __restrict__ U, int nx, int ny, int nv, int T, int C,
    int n_per_chunk)
{
    constexpr int RS = 2 * FW;
    constexpr int NT = MODE == 0 ? 1 : (MODE == 1 ? 4 : 3);   // trains read per voxel and TR
    // LDS: two buffers of per-wave sums [TB][CC][FW][32] (TB TRs per
    // barrier), then the block's y-phases [TRs per chunk][RS R].
    extern __shared__ float2 lds[];
    float2* eys = lds + 2 * TB * CC * FW * 32;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int xl = lane & 31, half = lane >> 5;
    const int ix = blockIdx.x * 32 + xl;
    const int yb = blockIdx.y;
    const int iyb = yb * RS * R + 2 * wave + half;
    const int n0 = fwd_chunk(blockIdx.z, gridDim.z) * n_per_chunk;
    const int n1 = min(T, n0 + n_per_chunk);
    const bool colok = ix < nx;
    const size_t plane = (size_t)T * nv;
    for (int e = threadIdx.x; e < (n1 - n0) * RS * R; e += blockDim.x) {
        const int nl = e / (RS * R), rr = e % (RS * R);
        const int iy = yb * RS * R + rr;
        eys[e] = iy < ny ? eytab[(size_t)(n0 + nl) * ny + iy] : make_float2(0.f, 0.f);
    }

    float2 P[R], Q[R];
    float v0[R], v1[R], v2[R];
    int jr[R];
    float2 cw[R][CC];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int iy = iyb + RS * r;
        const bool ok = colok && iy < ny;
        const int j = ok ? iy * nx + ix : 0;   // invalid voxels read voxel 0 with zero weight
        jr[r] = j;
        const bool on = ok && (mask == nullptr || mask[j] != 0);
        const float rr = on ? theta[3 * nv + j] : 0.f, ri = on ? theta[4 * nv + j] : 0.f;
        P[r] = make_float2(-ri, rr);   // i rho
        if constexpr (NT > 1) {
            const float nr = on ? v[3 * nv + j] : 0.f, ni = on ? v[4 * nv + j] : 0.f;
            Q[r] = make_float2(-ni, nr);   // i nu
            v0[r] = on ? v[j] : 0.f;
            v1[r] = on ? v[nv + j] : 0.f;
            if constexpr (NT == 4) v2[r] = on ? v[2 * nv + j] : 0.f;
        }
#pragma unroll
        for (int c = 0; c < CC; ++c)
            cw[r][c] = (ok && c < C) ? coil[(size_t)c * nv + j] : make_float2(0.f, 0.f);
    }
    __syncthreads();   // y-phases staged

    auto load_tr = [&](float (&buf)[R][NT], int n) {
        const TT* __restrict__ b0 = trains + (size_t)n * nv;
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int q = 0; q < NT; ++q) buf[r][q] = (float)b0[q * plane + jr[r]];
    };
    float nxt[R][NT];
    load_tr(nxt, n0);
    int buf = 0;
    for (int nb = n0; nb < n1; nb += TB) {
#pragma unroll
        for (int tb = 0; tb < TB; ++tb) {
            // TRs past the chunk repeat its last TR; their sums are not stored.
            const int n = min(nb + tb, n1 - 1);
            float cur[R][NT];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int q = 0; q < NT; ++q) cur[r][q] = nxt[r][q];
            load_tr(nxt, min(n + 1, n1 - 1));
            const float2* eyrow = eys + (size_t)(n - n0) * RS * R + 2 * wave + half;
            float2 acc[CC];
#pragma unroll
            for (int c = 0; c < CC; ++c) acc[c] = make_float2(0.f, 0.f);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float2 x;
                if constexpr (MODE == 0) {
                    x = make_float2(P[r].x * cur[r][0], P[r].y * cur[r][0]);
                } else {
                    float a;
                    if constexpr (NT == 4)
                        a = fmaf(v0[r], cur[r][1], fmaf(v1[r], cur[r][2], v2[r] * cur[r][3]));
                    else
                        a = fmaf(v0[r], cur[r][1], v1[r] * cur[r][2]);
                    x = make_float2(fmaf(P[r].x, a, Q[r].x * cur[r][0]), fmaf(P[r].y, a, Q[r].y * cur[r][0]));
                }
                const float2 z = cmul(eyrow[RS * r], x);
#pragma unroll
                for (int c = 0; c < CC; ++c) acc[c] = cfma(cw[r][c], z, acc[c]);
            }
            float2* red = lds + (size_t)(buf * TB + tb) * CC * FW * 32;
#pragma unroll
            for (int c = 0; c < CC; ++c) {
                const float2 t = shfl_xor2(acc[c], 32);
                if (half == 0) red[(c * FW + wave) * 32 + xl] = make_float2(acc[c].x + t.x, acc[c].y + t.y);
            }
        }
        __syncthreads();
        // Reduce these TRs across the waves (the next batch writes the other buffer).
        for (int o = threadIdx.x; o < TB * CC * 32; o += blockDim.x) {
            const int tb = o / (CC * 32), c = (o >> 5) % CC, l = o & 31;
            const float2* red = lds + (size_t)(buf * TB + tb) * CC * FW * 32;
            float2 sum = red[(c * FW) * 32 + l];
#pragma unroll
            for (int w = 1; w < FW; ++w) {
                const float2 t = red[(c * FW + w) * 32 + l];
                sum.x += t.x;
                sum.y += t.y;
            }
            const int oix = blockIdx.x * 32 + l;
            if (oix < nx && c < C && nb + tb < n1) U[(((size_t)yb * C + c) * T + nb + tb) * nx + oix] = sum;
        }
        buf ^= 1;
    }
}

// Sums the row-block partials of the forward y-stage into block 0.
__global__ void usum_kernel(float2* __restrict__ upart, int nby, size_t count)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float2 s = upart[i];
    int b = 1;
    for (; b + 4 <= nby; b += 4) {   // four partials' loads in flight, sums in block order
        float2 t[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) t[k] = upart[(size_t)(b + k) * count + i];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            s.x += t[k].x;
            s.y += t[k].y;
        }
    }
    for (; b < nby; ++b) {
        const float2 t = upart[(size_t)b * count + i];
        s.x += t.x;
        s.y += t.y;
    }
    upart[i] = s;
}

// ------------------------------------------------------------------------
// Adjoint y-stage: A_p[j] = sum_n mu_p[n,j] V[n,j],
// V[n,j] = conj(Ey[n,iy]) sum_c conj(C_c[j]) W_c[n,ix], summed over the TRs of
// one chunk. One thread per voxel in voxel order (each wave reads 256
// contiguous bytes per train), blocks of 256 voxels span at most
// 256 / nx + 2 rows, whose y-phases for the chunk are staged in LDS; W comes
// through the vector cache (a block reuses each W row across its rows).
// TRs go in batches of NBA whose loads are all issued before any use
// (indices clamped to the chunk, contributions of padding TRs zeroed).
// Partials per chunk are combined in chunk order by the finish kernel.
// ------------------------------------------------------------------------

// Complex partials per chunk in apart: NTRAIN = 1 (m only) packs one; 3 (no
// dm/dB1 train) keeps the four-train layout with the B1 pair left unwritten.
__host__ __device__ constexpr int apart_planes(int ntrain) { return ntrain == 1 ? 1 : 4; }

template <int NTRAIN, int CC, int NBA, typename TT, int VX>
__global__ __launch_bounds__(256) void ystage_adj_kernel(
    const TT* __restrict__ trains, const float2* __restrict__ coil,
    const uint8_t* __restrict__ mask, const float2* __restrict__ eytab,
    const float2* __restrict__ W, float* __restrict__ apart, int nx, int ny, int nv, int T,
    int C, int n_per_chunk)
{
    // VX consecutive voxels per thread (VX = 2: FP16 trains read as pairs,
    // nx even, so a pair never straddles a row); a block spans 256 VX voxels.
    constexpr int BV = 256 * VX;
    typedef TT tvx __attribute__((ext_vector_type(VX == 1 ? 2 : VX)));
    extern __shared__ float2 eys[];   // [n_per_chunk][rows]
    const int jb = blockIdx.x * BV;
    const int j0 = jb + VX * threadIdx.x;
    const bool ok = j0 < nv;
    const int j = ok ? j0 : nv - VX;
    const int ix = j % nx, iy = j / nx;
    const int row0 = jb / nx;
    const int rows = (min(jb + BV - 1, nv - 1)) / nx - row0 + 1;
    const int chunk = blockIdx.y;
    const int n0 = chunk * n_per_chunk;
    const int n1 = min(T, n0 + n_per_chunk);
    const size_t plane = (size_t)T * nv;

    for (int e = threadIdx.x; e < (n1 - n0) * rows; e += 256) {
        const int nl = e / rows, rr = e % rows;
        eys[nl * rows + rr] = eytab[(size_t)(n0 + nl) * ny + row0 + rr];
    }
    __syncthreads();
    const int myrow = iy - row0;

    float2 cw[VX][CC];
    if constexpr (CC > 1) {
#pragma unroll
        for (int u = 0; u < VX; ++u)
#pragma unroll
            for (int c = 0; c < CC; ++c)
                cw[u][c] = c < C ? coil[(size_t)c * nv + j + u] : make_float2(0.f, 0.f);
    }
    float2 acc[VX][NTRAIN];
#pragma unroll
    for (int u = 0; u < VX; ++u)
#pragma unroll
        for (int p = 0; p < NTRAIN; ++p) acc[u][p] = make_float2(0.f, 0.f);

    for (int nb0 = n0; nb0 < n1; nb0 += NBA) {
        float2 wv[NBA][VX][CC];
        float mu[NBA][VX][NTRAIN];
#pragma unroll
        for (int b = 0; b < NBA; ++b) {
            const int n = min(nb0 + b, n1 - 1);
#pragma unroll
            for (int c = 0; c < CC; ++c) {
                const int cc = c < C ? c : 0;
                const float2* wrow = W + ((size_t)cc * T + n) * nx + ix;
                if constexpr (VX >= 2) {
#pragma unroll
                    for (int h = 0; h < VX / 2; ++h) {
                        const float4 w2 = reinterpret_cast<const float4*>(wrow)[h];
                        wv[b][2 * h][c] = make_float2(w2.x, w2.y);
                        wv[b][2 * h + 1][c] = make_float2(w2.z, w2.w);
                    }
                } else {
                    wv[b][0][c] = wrow[0];
                }
            }
            const TT* __restrict__ t0 = trains + (size_t)n * nv;
#pragma unroll
            for (int p = 0; p < NTRAIN; ++p) {
                if constexpr (VX >= 2) {
                    const tvx a = *reinterpret_cast<const tvx*>(t0 + p * plane + j);
#pragma unroll
                    for (int u = 0; u < VX; ++u) mu[b][u][p] = (float)a[u];
                } else {
                    mu[b][0][p] = (float)(t0 + p * plane)[j];
                }
            }
        }
#pragma unroll
        for (int b = 0; b < NBA; ++b) {
            const int nl = min(nb0 + b, n1 - 1) - n0;
            const float keep = (nb0 + b < n1) ? 1.f : 0.f;
            const float2 eyc = eys[nl * rows + myrow];
#pragma unroll
            for (int u = 0; u < VX; ++u) {
                float2 wc;
                if constexpr (CC == 1) {
                    wc = wv[b][u][0];
                } else {
                    wc = make_float2(0.f, 0.f);
#pragma unroll
                    for (int c = 0; c < CC; ++c) {
                        const float2 t = cmulconj(cw[u][c], wv[b][u][c]);
                        wc.x += t.x;
                        wc.y += t.y;
                    }
                }
                float2 V = cmulconj(eyc, wc);
                V.x *= keep;
                V.y *= keep;
#pragma unroll
                for (int p = 0; p < NTRAIN; ++p) {
                    acc[u][p].x = fmaf(mu[b][u][p], V.x, acc[u][p].x);
                    acc[u][p].y = fmaf(mu[b][u][p], V.y, acc[u][p].y);
                }
            }
        }
    }
    if (!ok) return;
#pragma unroll
    for (int u = 0; u < VX; ++u) {
        const bool on = mask == nullptr || mask[j + u] != 0;
        float* dst = apart + (size_t)chunk * 2 * apart_planes(NTRAIN) * nv + j + u;
#pragma unroll
        for (int p = 0; p < NTRAIN; ++p) {
            dst[(2 * p) * (size_t)nv] = on ? acc[u][p].x : 0.f;
            dst[(2 * p + 1) * (size_t)nv] = on ? acc[u][p].y : 0.f;
        }
    }
}

// ------------------------------------------------------------------------
// Adjoint y-stage, wide layout (FP16 trains, one coil, nx a multiple of 4
// and at most 256, 8-byte aligned trains). A block covers one image row for
// one TR chunk; each lane owns 4 adjacent columns (one 8-byte load per train
// and TR) and the block's NWA waves take every NWA-th TR of the chunk, so a
// block has NWA times the loads in flight of a one-wave row while the
// partial sums per chunk stay those of the kernel above. The waves' sums meet
// in LDS once at the end. Ey[n, iy] is uniform per wave (scalar loads); W
// rows come through L2.
// ------------------------------------------------------------------------
constexpr int NWA = 8;   // waves per block

template <int NB, int R, int NTR>
__global__ __launch_bounds__(NWA * 64) void ystage_adj_wide_kernel(
    const _Float16* __restrict__ trains, const uint8_t* __restrict__ mask,
    const float2* __restrict__ eytab, const float2* __restrict__ W, float* __restrict__ apart,
    int nx, int ny, int nv, int T, int n_per_chunk)
{
    // R image rows per block share each TR's W (loaded once per wave and TR);
    // NTR trains (4, or 3 without dm/dB1).
    typedef _Float16 h4 __attribute__((ext_vector_type(4)));
    constexpr int NV2 = 2 * NTR;       // real values per voxel and chunk
    extern __shared__ float red_s[];   // [NWA][NV2][nx], one row at a time
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int iy0 = blockIdx.x * R;
    const int chunk = blockIdx.y;
    const int n0 = chunk * n_per_chunk;
    const int n1 = min(T, n0 + n_per_chunk);
    const int x0 = 4 * lane;
    const bool colok = x0 < nx;
    const int xc = colok ? x0 : 0;
    const size_t plane = (size_t)T * nv;
    int jr[R], iyr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        iyr[r] = min(iy0 + r, ny - 1);   // rows past the end repeat the last; not stored
        jr[r] = iyr[r] * nx + xc;
    }

    float acc[R][NTR][4][2];   // [row][train][column][re, im]
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int p = 0; p < NTR; ++p)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][p][c][0] = acc[r][p][c][1] = 0.f;

    // TRs n0 + wave + NWA k, NB at a time (loads first; padding TRs read the
    // chunk's first TR with a zero weight).
    for (int nb = n0 + wave; nb < n1; nb += NWA * NB) {
        h4 mu[NB][R][NTR];
        float4 w01[NB], w23[NB];
        float2 ey[NB][R];
        float keep[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int nr = nb + NWA * b;
            const int n = nr < n1 ? nr : n0;
            keep[b] = nr < n1 ? 1.f : 0.f;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const _Float16* t0 = trains + (size_t)n * nv + jr[r];
#pragma unroll
                for (int p = 0; p < NTR; ++p)
                    mu[b][r][p] = *(const h4*)(t0 + p * plane);
                ey[b][r] = eytab[(size_t)n * ny + iyr[r]];
            }
            const float4* wr = reinterpret_cast<const float4*>(W + (size_t)n * nx + xc);
            w01[b] = wr[0];
            w23[b] = wr[1];
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const float2 wc[4] = {make_float2(w01[b].x * keep[b], w01[b].y * keep[b]),
                                  make_float2(w01[b].z * keep[b], w01[b].w * keep[b]),
                                  make_float2(w23[b].x * keep[b], w23[b].y * keep[b]),
                                  make_float2(w23[b].z * keep[b], w23[b].w * keep[b])};
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const float2 V = cmulconj(ey[b][r], wc[c]);
#pragma unroll
                    for (int p = 0; p < NTR; ++p) {
                        const float m = (float)mu[b][r][p][c];
                        acc[r][p][c][0] = fmaf(m, V.x, acc[r][p][c][0]);
                        acc[r][p][c][1] = fmaf(m, V.y, acc[r][p][c][1]);
                    }
                }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (r > 0) __syncthreads();   // the previous row's sums have been read
        if (colok) {
#pragma unroll
            for (int p = 0; p < NTR; ++p)
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    *reinterpret_cast<float4*>(&red_s[((size_t)wave * NV2 + 2 * p + q) * nx + x0]) =
                        make_float4(acc[r][p][0][q], acc[r][p][1][q], acc[r][p][2][q], acc[r][p][3][q]);
        }
        __syncthreads();
        const int iy = iy0 + r;
        if (iy < ny) {
            float* dst = apart + (size_t)chunk * 8 * nv + (size_t)iy * nx;
            for (int o = threadIdx.x; o < NV2 * nx; o += NWA * 64) {
                const int v = o / nx, x = o % nx;
                float sum = red_s[(size_t)v * nx + x];
#pragma unroll
                for (int w = 1; w < NWA; ++w) sum += red_s[((size_t)w * NV2 + v) * nx + x];
                const bool on = mask == nullptr || mask[(size_t)iy * nx + x] != 0;
                dst[(size_t)v * nv + x] = on ? sum : 0.f;
            }
        }
    }
}

// ------------------------------------------------------------------------
// Adjoint y-stage with coils (CC = 8 or 16 coil slots). A block covers 32
// columns x 16 rows (two rows per thread), so each TR's W rows of all coils
// (CC x 32 complex) are staged once in LDS and used by 16 image rows instead
// of being fetched per voxel; TR batches of NBA are double-buffered (the next
// batch's W is loaded into registers while the current one is used, one
// barrier per batch). Partial sums per TR chunk as in the kernel above.
// ------------------------------------------------------------------------
template <int NTRAIN, int CC, int NBA, typename TT>
__global__ __launch_bounds__(256) void ystage_adj_coil_kernel(
    const TT* __restrict__ trains, const float2* __restrict__ coil,
    const uint8_t* __restrict__ mask, const float2* __restrict__ eytab,
    const float2* __restrict__ W, float* __restrict__ apart, int nx, int ny, int nv, int T,
    int C, int n_per_chunk)
{
    constexpr int RY = 2, BR = 8 * RY;               // rows per thread, rows per block
    constexpr int WT = NBA * CC * 32;                 // float2 per W tile
    constexpr int WPT = (WT + 255) / 256;             // W loads per thread
    extern __shared__ float2 sm[];
    float2* Ws = sm;                                  // [2][NBA][CC][32]
    float2* eys = sm + 2 * WT;                        // [n_per_chunk][BR]
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int ix = blockIdx.x * 32 + tx;
    const int row0 = blockIdx.y * BR;
    const int chunk = blockIdx.z;
    const int n0 = chunk * n_per_chunk;
    const int n1 = min(T, n0 + n_per_chunk);
    const size_t plane = (size_t)T * nv;
    for (int e = threadIdx.x; e < (n1 - n0) * BR; e += 256) {
        const int nl = e / BR, rr = e % BR;
        const int iy = row0 + rr;
        eys[e] = iy < ny ? eytab[(size_t)(n0 + nl) * ny + iy] : make_float2(0.f, 0.f);
    }
    int jr[RY];
    bool ok[RY];
    float2 cw[RY][CC];
#pragma unroll
    for (int u = 0; u < RY; ++u) {
        const int iy = row0 + ty + 8 * u;
        ok[u] = ix < nx && iy < ny;
        jr[u] = ok[u] ? iy * nx + ix : 0;
#pragma unroll
        for (int c = 0; c < CC; ++c)
            cw[u][c] = (ok[u] && c < C) ? coil[(size_t)c * nv + jr[u]] : make_float2(0.f, 0.f);
    }
    // W tile of the batch starting at TR nb: [b][c][column], zero outside.
    auto load_w = [&](float2 (&wr)[WPT], int nb) {
#pragma unroll
        for (int i = 0; i < WPT; ++i) {
            const int e = threadIdx.x + 256 * i;
            const int b = e / (CC * 32), c = (e / 32) % CC, col = e % 32;
            const int n = nb + b, x = blockIdx.x * 32 + col;
            wr[i] = (e < WT && n < n1 && c < C && x < nx) ? W[((size_t)c * T + n) * nx + x]
                                                          : make_float2(0.f, 0.f);
        }
    };
    auto store_w = [&](const float2 (&wr)[WPT], int buf) {
#pragma unroll
        for (int i = 0; i < WPT; ++i) {
            const int e = threadIdx.x + 256 * i;
            if (e < WT) Ws[buf * WT + e] = wr[i];
        }
    };
    float2 wr[WPT];
    load_w(wr, n0);
    store_w(wr, 0);
    __syncthreads();

    float2 acc[RY][NTRAIN];
#pragma unroll
    for (int u = 0; u < RY; ++u)
#pragma unroll
        for (int p = 0; p < NTRAIN; ++p) acc[u][p] = make_float2(0.f, 0.f);
    int buf = 0;
    for (int nb0 = n0; nb0 < n1; nb0 += NBA) {
        const bool more = nb0 + NBA < n1;
        if (more) load_w(wr, nb0 + NBA);
        float mu[NBA][RY][NTRAIN];
#pragma unroll
        for (int b = 0; b < NBA; ++b) {
            const int n = min(nb0 + b, n1 - 1);
            const TT* __restrict__ t0 = trains + (size_t)n * nv;
#pragma unroll
            for (int u = 0; u < RY; ++u)
#pragma unroll
                for (int p = 0; p < NTRAIN; ++p) mu[b][u][p] = (float)(t0 + p * plane)[jr[u]];
        }
        const float2* wt = Ws + buf * WT;
#pragma unroll
        for (int b = 0; b < NBA; ++b) {
            const int nl = min(nb0 + b, n1 - 1) - n0;
            const float keep = (nb0 + b < n1) ? 1.f : 0.f;
#pragma unroll
            for (int u = 0; u < RY; ++u) {
                float2 wc = make_float2(0.f, 0.f);
#pragma unroll
                for (int c = 0; c < CC; ++c) {
                    const float2 t = cmulconj(cw[u][c], wt[(b * CC + c) * 32 + tx]);
                    wc.x += t.x;
                    wc.y += t.y;
                }
                float2 V = cmulconj(eys[nl * BR + ty + 8 * u], wc);
                V.x *= keep;
                V.y *= keep;
#pragma unroll
                for (int p = 0; p < NTRAIN; ++p) {
                    acc[u][p].x = fmaf(mu[b][u][p], V.x, acc[u][p].x);
                    acc[u][p].y = fmaf(mu[b][u][p], V.y, acc[u][p].y);
                }
            }
        }
        if (more) store_w(wr, buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int u = 0; u < RY; ++u) {
        if (!ok[u]) continue;
        const int j = jr[u];
        const bool on = mask == nullptr || mask[j] != 0;
        float* dst = apart + (size_t)chunk * 2 * apart_planes(NTRAIN) * nv + j;
#pragma unroll
        for (int p = 0; p < NTRAIN; ++p) {
            dst[(2 * p) * (size_t)nv] = on ? acc[u][p].x : 0.f;
            dst[(2 * p + 1) * (size_t)nv] = on ? acc[u][p].y : 0.f;
        }
    }
}

// Sums the split-K partials of the adjoint x-GEMM into the first.
__global__ void wsum_kernel(float2* __restrict__ W, int nsplit, size_t count)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float2 s = W[i];
    int b = 1;
    for (; b + 2 <= nsplit; b += 2) {   // two partials' loads in flight, sums in split order
        const float2 t0 = W[(size_t)b * count + i], t1 = W[(size_t)(b + 1) * count + i];
        s.x += t0.x;
        s.y += t0.y;
        s.x += t1.x;
        s.y += t1.y;
    }
    for (; b < nsplit; ++b) {
        const float2 t = W[(size_t)b * count + i];
        s.x += t.x;
        s.y += t.y;
    }
    W[i] = s;
}

// g from A: g_q = -Im(conj(rho) A_{q+1}) for q = lnT1, lnT2, B1;
// g_3 = -Im(A_0) (Re rho), g_4 = Re(A_0) (Im rho); with NP = 6 also
// g_5 = -Im(conj(rho) A_5) (Delta B0, chunks of 10 planes).
// CURV: 0 = gradient only; 2 = also the CG partials dir . g, dir . dir and
// step . dir (the trust-region CG's, with its boundary test); 3 = dir . g,
// dir . dir, res . res, res . g and g . g (what the one-launch CG update
// needs for alpha and beta).
template <int CURV, int NP>
__global__ __launch_bounds__(256) void jhw_finish_kernel(const float* __restrict__ apart, int n_chunk,
                                                         const float* __restrict__ theta,
                                                         const uint8_t* __restrict__ mask, int param_mask,
                                                         float* __restrict__ g, int nv,
                                                         const float* __restrict__ dir,
                                                         const float* __restrict__ step,
                                                         const float* __restrict__ res,
                                                         double* __restrict__ part)
{
    constexpr int PL = NP == 6 ? 10 : 8;   // planes per chunk
    constexpr int NPART = CURV == 3 ? 5 : 3;   // partial kinds
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    double acc[NPART];
#pragma unroll
    for (int k = 0; k < NPART; ++k) acc[k] = 0.0;
    if (j < nv) {
        const bool on = mask == nullptr || mask[j] != 0;
        const float rr = theta[3 * nv + j], ri = theta[4 * nv + j];
        float A[PL];
#pragma unroll
        for (int q = 0; q < PL; ++q) A[q] = 0.f;
        // The dm/dB1 pair (A[6], A[7]) is read only when B1 is reconstructed
        // (without it the adjoint y-stage may leave that pair unwritten), the
        // Delta B0 pair only when Delta B0 is.
        // Chunks go three at a time with all their loads issued first (one
        // wave per 64 voxels is all the kernel has); sums stay in chunk order.
        const bool b1 = (param_mask >> 2) & 1, f5 = (param_mask >> 5) & 1;
        auto load = [&](int ch, float (&t)[PL]) {
#pragma unroll
            for (int q = 0; q < 6; ++q) t[q] = apart[((size_t)ch * PL + q) * nv + j];
            t[6] = b1 ? apart[((size_t)ch * PL + 6) * nv + j] : 0.f;
            t[7] = b1 ? apart[((size_t)ch * PL + 7) * nv + j] : 0.f;
            if constexpr (NP == 6) {
                t[8] = f5 ? apart[((size_t)ch * PL + 8) * nv + j] : 0.f;
                t[9] = f5 ? apart[((size_t)ch * PL + 9) * nv + j] : 0.f;
            }
        };
        int ch = 0;
        for (; ch + 3 <= n_chunk; ch += 3) {
            float t[3][PL];
#pragma unroll
            for (int c = 0; c < 3; ++c) load(ch + c, t[c]);
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int q = 0; q < PL; ++q) A[q] += t[c][q];
        }
        for (; ch < n_chunk; ++ch) {
            float t[PL];
            load(ch, t);
#pragma unroll
            for (int q = 0; q < PL; ++q) A[q] += t[q];
        }
        // Rows of parameters outside param_mask are zero.
        float gq[NP];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const float ar = A[2 * (q + 1)], ai = A[2 * (q + 1) + 1];
            gq[q] = (on && ((param_mask >> q) & 1)) ? -(rr * ai - ri * ar) : 0.f;
        }
        gq[3] = (on && ((param_mask >> 3) & 1)) ? -A[1] : 0.f;
        gq[4] = (on && ((param_mask >> 4) & 1)) ? A[0] : 0.f;
        if constexpr (NP == 6) gq[5] = (on && f5) ? -(rr * A[9] - ri * A[8]) : 0.f;
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            g[(size_t)q * nv + j] = gq[q];
            if constexpr (CURV > 0) {
                const double dv = dir[(size_t)q * nv + j], gv = gq[q];
                acc[0] += dv * gv;
                acc[1] += dv * dv;
                if constexpr (CURV == 2) acc[2] += (double)step[(size_t)q * nv + j] * dv;
                if constexpr (CURV == 3) {
                    const double rv = res[(size_t)q * nv + j];
                    acc[2] += rv * rv;
                    acc[3] += rv * gv;
                    acc[4] += gv * gv;
                }
            }
        }
    }
    if constexpr (CURV > 0) {
        // CG partials of this block's voxels in FP64, one per block and kind
        // ([NPART][gridDim.x]; all threads reach the barrier).
        __shared__ double sh[NPART][4];
#pragma unroll
        for (int k = 0; k < NPART; ++k)
            for (int off = 32; off > 0; off >>= 1) acc[k] += __shfl_xor(acc[k], off);
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        if (lane == 0)
#pragma unroll
            for (int k = 0; k < NPART; ++k) sh[k][wave] = acc[k];
        __syncthreads();
        if (threadIdx.x == 0)
#pragma unroll
            for (int k = 0; k < NPART; ++k)
                part[(size_t)k * gridDim.x + blockIdx.x] = (sh[k][0] + sh[k][1]) + (sh[k][2] + sh[k][3]);
    }
}

// CGLS adjoint of the rho-linear map: (M^H w)_j = sum_n conj(m_j[n]) V = -i A_0.
__global__ void rho_adj_finish_kernel(const float* __restrict__ apart, int n_chunk,
                                      const uint8_t* __restrict__ mask, float2* __restrict__ out,
                                      int nv)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nv) return;
    float ar = 0.f, ai = 0.f;
    for (int ch = 0; ch < n_chunk; ++ch) {
        ar += apart[((size_t)ch * 2) * nv + j];
        ai += apart[((size_t)ch * 2 + 1) * nv + j];
    }
    const bool on = mask == nullptr || mask[j] != 0;
    out[j] = on ? make_float2(ai, -ar) : make_float2(0.f, 0.f);
}

// ------------------------------------------------------------------------
// x-stage GEMMs on the matrix cores (v_mfma_f32_16x16x4_f32).
// Real form of the complex product with interleaved (re, im) operands:
//   forward  C[m][2k+b]  = sum_{ix,a} A[m][2ix+a] Bf[2ix+a][2k+b],
//            Bf = [[Er, Ei], [-Ei, Er]] at (ix, k)
//   adjoint  C[m][2ix+b] = sum_{k,a}  A[m][2k+a]  Ba[2k+a][2ix+b],
//            Ba = [[Er, -Ei], [Ei, Er]] at (k, ix)
// with E = Ex[k][ix] read from the exactly range-reduced phase table.
// Tile 64 x 64 per block, 4 waves in 2 x 2, each 32 x 32 = 2 x 2 MFMA blocks;
// K in chunks of 32, double-buffered in LDS with the next chunk's global loads
// in flight during the current chunk's MFMAs. blockIdx.z splits K (partial
// outputs at out + z * out_stride).
// MFMA 16x16x4 f32 operand layout: A lane l -> (row l%16, k l/16),
// B lane l -> (k l/16, col l%16), D lane l -> (rows 4(l/16)+i, col l%16).
// ------------------------------------------------------------------------
constexpr int GBM = 64, GBN = 64, GBK = 32;
constexpr int XPD = 2;   // K chunks in flight (deeper pipelining measured no faster)

template <int DIR, int MODE>   // DIR 0 forward, 1 adjoint; MODE (forward): 0 residual, 1 -s, 2 +s
__global__ __launch_bounds__(256) void xgemm_f32_kernel(
    const float2* __restrict__ Ain, const float2* __restrict__ extab,
    const float2* __restrict__ data, float2* __restrict__ out, double* __restrict__ red, int M,
    int nx, int nk, int chunks_per_split, size_t out_stride)
{
    __shared__ float As[2][GBM][GBK + 1];
    __shared__ __attribute__((aligned(16))) float Bs[2][GBK][GBN + 4];
    __shared__ double rs[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = blockIdx.y * GBM, c0 = blockIdx.x * GBN;
    const int Kr = DIR == 0 ? 2 * nx : 2 * nk;    // real reduction length
    const int Nr = DIR == 0 ? 2 * nk : 2 * nx;    // real output columns
    const int Ka = DIR == 0 ? nx : nk;            // complex A columns
    const int nchunk = (Kr + GBK - 1) / GBK;
    const int kc0 = blockIdx.z * chunks_per_split;
    const int kc1 = min(nchunk, kc0 + chunks_per_split);

    // Chunks past kc1 (padding of the pipelined loop) load zeros.
    auto gload = [&](int kc, float2 (&ra)[4], float2 (&rb)[2]) {
        const int k0 = kc * GBK;
        const bool live = kc < kc1;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = tid + 256 * i;
            const int r = e >> 4, cc = e & 15;
            const int m = m0 + r, kcol = k0 / 2 + cc;
            ra[i] = (live && m < M && kcol < Ka) ? Ain[(size_t)m * Ka + kcol] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int e = tid + 256 * i;
            // Consecutive threads read consecutive ix of the phase table.
            const int rr = DIR == 0 ? (e & 15) : (e >> 5);
            const int cc = DIR == 0 ? (e >> 4) : (e & 31);
            const int kr = k0 / 2 + rr, kcol = c0 / 2 + cc;
            float2 E = make_float2(0.f, 0.f);
            if (DIR == 0) {
                if (live && kr < nx && kcol < nk) E = extab[(size_t)kcol * nx + kr];
            } else {
                if (live && kr < nk && kcol < nx) E = extab[(size_t)kr * nx + kcol];
            }
            rb[i] = E;
        }
    };
    auto sstore = [&](int buf, const float2 (&ra)[4], const float2 (&rb)[2]) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = tid + 256 * i;
            const int r = e >> 4, cc = e & 15;
            As[buf][r][2 * cc] = ra[i].x;
            As[buf][r][2 * cc + 1] = ra[i].y;
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int e = tid + 256 * i;
            const int rr = DIR == 0 ? (e & 15) : (e >> 5);
            const int cc = DIR == 0 ? (e >> 4) : (e & 31);
            const float2 E = rb[i];
            const float ey = DIR == 0 ? E.y : -E.y;
            *reinterpret_cast<float2*>(&Bs[buf][2 * rr][2 * cc]) = make_float2(E.x, ey);
            *reinterpret_cast<float2*>(&Bs[buf][2 * rr + 1][2 * cc]) = make_float2(-ey, E.x);
        }
    };

    f4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};

    // XPD chunks in flight: chunk kc + XPD - 1 is loaded while chunk kc is
    // multiplied from LDS and chunk kc + 1 stored; the loop runs a multiple of
    // XPD chunks (the padding is zero).
    float2 ra[XPD][4], rb[XPD][2];
#pragma unroll
    for (int u = 0; u < XPD - 1; ++u) gload(kc0 + u, ra[u], rb[u]);
    sstore(0, ra[0], rb[0]);
    __syncthreads();
    for (int kb = kc0; kb < kc1; kb += XPD) {
#pragma unroll
        for (int u = 0; u < XPD; ++u) {
            const int kc = kb + u;
            const int buf = (kc - kc0) & 1;
            gload(kc + XPD - 1, ra[(u + XPD - 1) % XPD], rb[(u + XPD - 1) % XPD]);
#pragma unroll
            for (int kk = 0; kk < GBK; kk += 4) {
                float av[2], bv[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) av[a] = As[buf][wm * 32 + a * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
                for (int b = 0; b < 2; ++b) bv[b] = Bs[buf][kk + (lane >> 4)][wn * 32 + b * 16 + (lane & 15)];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
            }
            sstore(buf ^ 1, ra[(u + 1) % XPD], rb[(u + 1) % XPD]);
            __syncthreads();
        }
    }

    // Epilogue.
    double sq = 0.0;
    float* o = reinterpret_cast<float*>(out) + blockIdx.z * out_stride;
    const float* dd = reinterpret_cast<const float*>(data);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = m0 + wm * 32 + a * 16 + 4 * (lane >> 4) + i;
                const int c = c0 + wn * 32 + b * 16 + (lane & 15);
                if (m < M && c < Nr) {
                    const size_t idx = (size_t)m * Nr + c;
                    const float val = acc[a][b][i];
                    if (DIR == 0 && MODE == 0) {
                        const float rv = dd[idx] - val;
                        o[idx] = rv;
                        sq += (double)rv * (double)rv;
                    } else if (DIR == 0 && MODE == 1) {
                        o[idx] = -val;
                    } else {
                        o[idx] = val;
                    }
                }
            }
    if (DIR == 0 && MODE == 0) {
        for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off);
        if (lane == 0) rs[wave] = sq;
        __syncthreads();
        if (tid == 0) red[blockIdx.y * gridDim.x + blockIdx.x] = (rs[0] + rs[1]) + (rs[2] + rs[3]);
    }
}

// ------------------------------------------------------------------------
// Reduced-precision x-stage GEMMs on v_mfma_f32_16x16x32_{bf16,f16}, same
// real 2x2-block form as the FP32 kernel:
//   ENC 1, split-BF16: each FP32 operand x = hi + lo, hi = bf16(x),
//          lo = bf16(x - hi); C = hi*hi + hi*lo + lo*hi with FP32 accumulation
//          (the lo*lo term, ~2^-16 relative, is dropped).
//   ENC 2, FP16: one product of FP16-rounded operands, FP32 accumulation
//          (operands must stay below 65504 in magnitude: |U|, |w| and the
//          unit-modulus phases do for these problems).
// MFMA 16x16x32 operand layout: A lane l -> (row l%16, k 8(l/16)..+7),
// B lane l -> (k 8(l/16)..+7, col l%16), D as for the FP32 instruction.
// ------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ unsigned short bf16_bits_rne(float x)
{
    const unsigned int u = __float_as_uint(x);
    const unsigned int r = u + 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(r >> 16);
}

__device__ __forceinline__ float bf16_bits_to_float(unsigned short b)
{
    return __uint_as_float((unsigned int)b << 16);
}

template <int ENC>
struct MxOps;
template <>
struct MxOps<1> {
    static constexpr int TERMS = 2;   // hi, lo
    __device__ static void split(float x, unsigned short* h, unsigned short* l)
    {
        const unsigned short hb = bf16_bits_rne(x);
        *h = hb;
        *l = bf16_bits_rne(x - bf16_bits_to_float(hb));
    }
    __device__ static f4 mma(const uint4& a, const uint4& b, f4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    }
};
template <>
struct MxOps<2> {
    static constexpr int TERMS = 1;
    __device__ static void split(float x, unsigned short* h, unsigned short* l)
    {
        *h = __builtin_bit_cast(unsigned short, (_Float16)x);
        *l = 0;
    }
    __device__ static f4 mma(const uint4& a, const uint4& b, f4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                      __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
    }
};

// ------------------------------------------------------------------------
// Reduced-precision x-stage GEMMs without LDS. The real-form phase matrix
// (Bf forward, Ba adjoint, as above) is fixed for a context, so it is split
// once at bind into B-fragment tables in the MFMA operand order:
//   bfrag[((kb NCB + cb) NT + t) 64 + l] = 8 16-bit values of term t of
//   B[32 kb + 8(l/16) + e][16 cb + l%16], e = 0..7 (zero beyond Kr, Nr),
// with kb the 32-row K block, cb the 16-column block, t = hi / lo (ENC 1) or
// the FP16 value (ENC 2). One wave computes a 16 x 32 output tile over all
// of K: its A fragment (row l%16, 8 consecutive real k = 4 complex elements,
// two 16-byte loads) is split in registers and its B fragments are single
// 16-byte loads, so waves share nothing, need no barrier, and a launch has
// M/16 x Nr/32 waves to hide load latency with.
// ------------------------------------------------------------------------
template <int DIR, int ENC>
__global__ void build_bfrag_kernel(const float2* __restrict__ extab, uint4* __restrict__ out,
                                   int nx, int nk)
{
    constexpr int NT = MxOps<ENC>::TERMS;
    const int Kr = DIR == 0 ? 2 * nx : 2 * nk, Nr = DIR == 0 ? 2 * nk : 2 * nx;
    const int KB = (Kr + 31) / 32, NCB = (Nr + 15) / 16;
    const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (size_t)KB * NCB * 64) return;
    const int l = (int)(g % 64), cb = (int)((g / 64) % NCB), kb = (int)(g / (64 * (size_t)NCB));
    const int col = 16 * cb + (l & 15);
    unsigned short h[8], lo[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int kr = 32 * kb + 8 * (l >> 4) + e;
        float v = 0.f;
        if (kr < Kr && col < Nr) {
            const int a = kr & 1, b = col & 1;
            const float2 E = DIR == 0 ? extab[(size_t)(col >> 1) * nx + (kr >> 1)]
                                      : extab[(size_t)(kr >> 1) * nx + (col >> 1)];
            // Bf = [[Er, Ei], [-Ei, Er]], Ba = [[Er, -Ei], [Ei, Er]] (row a, column b).
            v = (a == b) ? E.x : ((DIR == 0) == (a == 0) ? E.y : -E.y);
        }
        MxOps<ENC>::split(v, &h[e], &lo[e]);
    }
    const size_t base = ((size_t)kb * NCB + cb) * NT * 64 + l;
    out[base] = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16),
                           h[6] | (h[7] << 16));
    if constexpr (NT > 1)
        out[base + 64] = make_uint4(lo[0] | (lo[1] << 16), lo[2] | (lo[3] << 16),
                                    lo[4] | (lo[5] << 16), lo[6] | (lo[7] << 16));
}

template <int DIR, int MODE, int ENC, int KS, int RW, int CW>
__global__ __launch_bounds__(64 * KS) void xgemm_direct_kernel(
    const float2* __restrict__ Ain, const uint4* __restrict__ bfrag,
    const float2* __restrict__ data, float2* __restrict__ out, double* __restrict__ red, int M,
    int nx, int nk)
{
    // A wave's tile is 16 RW rows x 16 CW columns. KS waves per block share one
    // tile and take every KS-th K block; their sums meet in LDS.
    using Ops = MxOps<ENC>;
    constexpr int NT = Ops::TERMS;
    __shared__ f4 part[KS > 1 ? KS - 1 : 1][RW][CW][64];
    const int lane = threadIdx.x & 63, kw = threadIdx.x >> 6;
    const int Kr = DIR == 0 ? 2 * nx : 2 * nk;
    const int Nr = DIR == 0 ? 2 * nk : 2 * nx;
    const int Ka = Kr / 2;
    const int KB = (Kr + 31) / 32, NCB = (Nr + 15) / 16;
    const int cb0 = CW * blockIdx.x;
    const int m0 = 16 * RW * blockIdx.y;
    const int kq = 4 * (lane >> 4);
    const bool vec = (Ka & 1) == 0 && (reinterpret_cast<uintptr_t>(Ain) & 15) == 0;   // 16-byte loads
    int rowc[RW];
    bool rowok[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        const int row = m0 + 16 * r + (lane & 15);
        rowok[r] = row < M;
        rowc[r] = rowok[r] ? row : 0;
    }

    auto load_a = [&](int kb, float2 (&a)[RW][4]) {
        const int k0 = 16 * kb + kq;
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const float2* __restrict__ arow = Ain + (size_t)rowc[r] * Ka;
            if (vec && rowok[r] && k0 + 3 < Ka) {
                const float4 u = *reinterpret_cast<const float4*>(arow + k0);
                const float4 w = *reinterpret_cast<const float4*>(arow + k0 + 2);
                a[r][0] = make_float2(u.x, u.y);
                a[r][1] = make_float2(u.z, u.w);
                a[r][2] = make_float2(w.x, w.y);
                a[r][3] = make_float2(w.z, w.w);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    a[r][e] = (rowok[r] && k0 + e < Ka) ? arow[k0 + e] : make_float2(0.f, 0.f);
            }
        }
    };
    auto load_b = [&](int kb, uint4 (&b)[CW][NT]) {
#pragma unroll
        for (int c = 0; c < CW; ++c) {
            const int cb = cb0 + c < NCB ? cb0 + c : NCB - 1;   // clamped; its output is not stored
#pragma unroll
            for (int t = 0; t < NT; ++t) b[c][t] = bfrag[(((size_t)kb * NCB + cb) * NT + t) * 64 + lane];
        }
    };

    f4 acc[RW][CW];
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int c = 0; c < CW; ++c) acc[r][c] = f4{0.f, 0.f, 0.f, 0.f};
    float2 a_cur[RW][4], a_nxt[RW][4];
    uint4 b_cur[CW][NT], b_nxt[CW][NT];
    if (kw < KB) {
        load_a(kw, a_cur);
        load_b(kw, b_cur);
    }
    for (int kb = kw; kb < KB; kb += KS) {
        if (kb + KS < KB) {
            load_a(kb + KS, a_nxt);
            load_b(kb + KS, b_nxt);
        }
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            unsigned short hh[8], ll[8];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                Ops::split(a_cur[r][e].x, &hh[2 * e], &ll[2 * e]);
                Ops::split(a_cur[r][e].y, &hh[2 * e + 1], &ll[2 * e + 1]);
            }
            const uint4 ah = make_uint4(hh[0] | (hh[1] << 16), hh[2] | (hh[3] << 16),
                                        hh[4] | (hh[5] << 16), hh[6] | (hh[7] << 16));
            uint4 al = make_uint4(0u, 0u, 0u, 0u);
            if constexpr (NT > 1)
                al = make_uint4(ll[0] | (ll[1] << 16), ll[2] | (ll[3] << 16), ll[4] | (ll[5] << 16),
                                ll[6] | (ll[7] << 16));
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                if constexpr (NT > 1) {
                    acc[r][c] = Ops::mma(al, b_cur[c][0], acc[r][c]);   // lo * hi
                    acc[r][c] = Ops::mma(ah, b_cur[c][1], acc[r][c]);   // hi * lo
                }
                acc[r][c] = Ops::mma(ah, b_cur[c][0], acc[r][c]);       // hi * hi
            }
        }
        if (kb + KS < KB) {
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
                for (int e = 0; e < 4; ++e) a_cur[r][e] = a_nxt[r][e];
#pragma unroll
            for (int c = 0; c < CW; ++c)
#pragma unroll
                for (int t = 0; t < NT; ++t) b_cur[c][t] = b_nxt[c][t];
        }
    }
    if constexpr (KS > 1) {
        if (kw > 0) {
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
                for (int c = 0; c < CW; ++c) part[kw - 1][r][c][lane] = acc[r][c];
        }
        __syncthreads();
        if (kw > 0) return;
#pragma unroll
        for (int w = 0; w < KS - 1; ++w)
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
                for (int c = 0; c < CW; ++c) acc[r][c] += part[w][r][c][lane];
    }

    double sq = 0.0;
    float* o = reinterpret_cast<float*>(out);
    const float* dd = reinterpret_cast<const float*>(data);
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int c = 0; c < CW; ++c)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = m0 + 16 * r + 4 * (lane >> 4) + i;
                const int col = 16 * (cb0 + c) + (lane & 15);
                if (m < M && col < Nr) {
                    const size_t idx = (size_t)m * Nr + col;
                    const float val = acc[r][c][i];
                    if (DIR == 0 && MODE == 0) {
                        const float rv = dd[idx] - val;
                        o[idx] = rv;
                        sq += (double)rv * (double)rv;
                    } else if (DIR == 0 && MODE == 1) {
                        o[idx] = -val;
                    } else {
                        o[idx] = val;
                    }
                }
            }
    if (DIR == 0 && MODE == 0) {
        for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off);
        if (lane == 0) red[blockIdx.y * gridDim.x + blockIdx.x] = sq;
    }
}

template <int DIR, int MODE>
void xgemm_any(dim3 grid, hipStream_t s, const float2* A, const float2* extab, const float2* data,
               float2* out, double* red, int M, int nx, int nk, int per, size_t stride)
{
    xgemm_f32_kernel<DIR, MODE><<<grid, 256, 0, s>>>(A, extab, data, out, red, M, nx, nk, per, stride);
}

template <int MODE, int CC, typename TT>
hipError_t fwd_R(const Dims& d, const YPlan& p, const TT* trains, const float* theta,
                 const float* v, const float2* coil, const uint8_t* mask, const float2* eytab,
                 float2* U, int* nby_used, hipStream_t s)
{
    // Wide layout (FP16 trains) when the plan allows it and every operand is
    // 16-byte aligned.
    if constexpr (CC == 1 && sizeof(TT) == 2) {
        // NT TRs x NW waves per block (the plan's), fewer TRs when their
        // per-wave sums would not fit in 64 KB of LDS.
        int ntw = MODE == 0 ? p.ntws16 : p.ntw16;
        const int nw = p.nww;
        auto lds_of = [&](int nt, int w) { return (size_t)nt * (w * d.nx + p.roww) * sizeof(float2); };
        while (ntw >= 2 && lds_of(ntw, nw) > 65536) ntw /= 2;
        auto al = [](const void* q, uintptr_t a) { return ((uintptr_t)q & (a - 1)) == 0; };
        if (ntw >= 2 && al(trains, 16) && al(theta, 16) && (MODE == 0 || al(v, 16)) &&
            (mask == nullptr || al(mask, 4))) {
            dim3 grid(p.nbyw, ceil_div(d.T, ntw));
            const size_t lds = lds_of(ntw, nw);
            *nby_used = p.nbyw;
#define FWDW_CASE(NN, WW)                                                                       \
    if (ntw == NN && nw == WW) {                                                                \
        ystage_fwd_wide_kernel<MODE, NN, WW, TT><<<grid, WW * 64, lds, s>>>(                    \
            trains, theta, v, mask, eytab, U, d.nx, d.ny, d.nv, d.T, p.roww);                   \
        return hipGetLastError();                                                               \
    }
            FWDW_CASE(8, 4) FWDW_CASE(4, 4) FWDW_CASE(2, 4) FWDW_CASE(8, 8) FWDW_CASE(4, 8)
            FWDW_CASE(2, 8)
#undef FWDW_CASE
            return hipErrorInvalidValue;
        }
    }
    *nby_used = CC > 1 ? p.nbyc : ((sizeof(TT) == 2 && p.g16 > 0) ? p.nby16 : p.nby);
    // 2-byte trains, one coil: one row per wave, all columns per block.
    if constexpr (sizeof(TT) == 2 && CC == 1) {
        if (p.g16 > 0) {
            dim3 grid(ceil_div(d.nx, 64 * p.g16), p.nby16, ceil_div(d.T, p.fwd_tr16));
            const size_t lds = (size_t)p.fwd_tr16 * (FW * 64 + (FW / p.g16) * p.r_fwd16) * sizeof(float2);
#define FWD16_CASE(GG, RR)                                                                      \
    if (p.g16 == GG && p.r_fwd16 == RR) {                                                       \
        ystage_fwd_kernel<MODE, RR, 1, TT, GG><<<grid, FW * 64, lds, s>>>(                      \
            trains, theta, v, coil, mask, eytab, U, d.nx, d.ny, d.nv, d.T, d.C, p.fwd_tr16);    \
        return hipGetLastError();                                                               \
    }
            FWD16_CASE(1, 1) FWD16_CASE(1, 2) FWD16_CASE(1, 3) FWD16_CASE(1, 4)
            FWD16_CASE(2, 1) FWD16_CASE(2, 2) FWD16_CASE(2, 3) FWD16_CASE(2, 4)
            FWD16_CASE(4, 1) FWD16_CASE(4, 2) FWD16_CASE(4, 3) FWD16_CASE(4, 4)
            FWD16_CASE(8, 1) FWD16_CASE(8, 2) FWD16_CASE(8, 3) FWD16_CASE(8, 4)
            FWD16_CASE(16, 1) FWD16_CASE(16, 2) FWD16_CASE(16, 3) FWD16_CASE(16, 4)
#undef FWD16_CASE
            return hipErrorInvalidValue;
        }
    }
    if constexpr (CC > 1) {
        // Coils: per-TR reduction, long TR chunks.
        dim3 grid(ceil_div(d.nx, 32), p.nbyc, ceil_div(d.T, p.fwd_trc));
        // TRs per barrier (LDS 2 TB CC 16 KB): 2 for up to 8 coils (256 x 256,
        // 8 coils, 1280 TRs: FP16 trains 329 -> 261 us, FP32 395 -> 350 us).
        constexpr int TB = CC <= 8 ? 2 : 1;
        const size_t lds = (size_t)(2 * TB * CC * FW * 32 + p.fwd_trc * 2 * FW * p.r_fwdc) * sizeof(float2);
#define FWDC_CASE(RR)                                                                           \
    if (p.r_fwdc == RR) {                                                                       \
        if (lds > 65536) {                                                                      \
            const hipError_t ea = hipFuncSetAttribute(                                          \
                reinterpret_cast<const void*>(&ystage_fwd_coil_kernel<MODE, RR, CC, TT, TB>),   \
                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                          \
            if (ea != hipSuccess) return ea;                                                    \
        }                                                                                       \
        ystage_fwd_coil_kernel<MODE, RR, CC, TT, TB><<<grid, FW * 64, lds, s>>>(                \
            trains, theta, v, coil, mask, eytab, U, d.nx, d.ny, d.nv, d.T, d.C, p.fwd_trc);     \
        return hipGetLastError();                                                               \
    }
        FWDC_CASE(1)
        if constexpr (CC <= 8) { FWDC_CASE(2) }
#undef FWDC_CASE
        return hipErrorInvalidValue;
    }
    dim3 grid(ceil_div(d.nx, 32), p.nby, ceil_div(d.T, p.fwd_tr));
    const size_t lds = (size_t)p.fwd_tr * (CC * FW * 32 + 32 * p.r_fwd) * sizeof(float2);
#define FWD_CASE(RR)                                                                            \
    case RR:                                                                                    \
        if constexpr (CC == 1 || RR <= 2)                                                       \
            ystage_fwd_kernel<MODE, RR, CC, TT, 0><<<grid, FW * 64, lds, s>>>(                  \
                trains, theta, v, coil, mask, eytab, U, d.nx, d.ny, d.nv, d.T, d.C, p.fwd_tr);  \
        else                                                                                    \
            return hipErrorInvalidValue;                                                        \
        break;
    switch (p.r_fwd) {
        FWD_CASE(1) FWD_CASE(2) FWD_CASE(3) FWD_CASE(4) FWD_CASE(5) FWD_CASE(6) FWD_CASE(7)
        FWD_CASE(8)
        default: return hipErrorInvalidValue;
    }
#undef FWD_CASE
    return hipGetLastError();
}

template <int NTRAIN, int CC, typename TT>
hipError_t adj_launch(const Dims& d, const YPlan& p, const TT* trains, const float2* coil,
                      const uint8_t* mask, const float2* eytab, const float2* W, float* apart,
                      hipStream_t s)
{
    // FP16 pairs (nx even, one coil): 512 voxels per block, twice the TRs
    // per batch, so the bytes in flight match the FP32 kernel.
    if constexpr (std::is_same<TT, _Float16>::value && CC == 1) {
        if (NTRAIN >= 3 && d.nx % 4 == 0 && d.nx <= 256 && ((uintptr_t)trains & 7) == 0 &&
            ((uintptr_t)W & 15) == 0) {
            // 2 rows per block, 1 TR per wave in flight (measured at 224 x 224:
            // rows x TRs 1 x 1: 108 us, 2 x 1: 96, 2 x 2: 110, 3 x 1: 128 with
            // 8 chunks; the pair kernel below 107).
            dim3 grid(ceil_div(d.ny, 2), p.adj_chunks);
            const size_t lds = (size_t)NWA * 2 * NTRAIN * d.nx * sizeof(float);
            ystage_adj_wide_kernel<1, 2, (NTRAIN >= 3 ? NTRAIN : 4)><<<grid, NWA * 64, lds, s>>>(
                trains, mask, eytab, W, apart, d.nx, d.ny, d.nv, d.T, p.adj_per_chunk);
            return hipGetLastError();
        }
        if (d.nx % 2 == 0) {
            dim3 grid(ceil_div(d.nv, 512), p.adj_chunks);
            const int rows = std::min(d.ny, 512 / d.nx + 2);
            const size_t lds = (size_t)p.adj_per_chunk * rows * sizeof(float2);
            ystage_adj_kernel<NTRAIN, CC, 8, TT, 2><<<grid, 256, lds, s>>>(
                trains, coil, mask, eytab, W, apart, d.nx, d.ny, d.nv, d.T, d.C, p.adj_per_chunk);
            return hipGetLastError();
        }
    }
    if constexpr (CC > 1) {
        // Coils: 32 x 16 voxel tiles sharing staged W rows.
        constexpr int NBA = 4;
        dim3 grid(ceil_div(d.nx, 32), ceil_div(d.ny, 16), p.adj_chunks);
        const size_t lds = (size_t)(2 * NBA * CC * 32 + p.adj_per_chunk * 16) * sizeof(float2);
        ystage_adj_coil_kernel<NTRAIN, CC, NBA, TT><<<grid, 256, lds, s>>>(
            trains, coil, mask, eytab, W, apart, d.nx, d.ny, d.nv, d.T, d.C, p.adj_per_chunk);
        return hipGetLastError();
    }
    dim3 grid(ceil_div(d.nv, 256), p.adj_chunks);
    const int rows = std::min(d.ny, 256 / d.nx + 2);
    const size_t lds = (size_t)p.adj_per_chunk * rows * sizeof(float2);
    constexpr int NBA = CC == 1 ? 4 : 2;
    ystage_adj_kernel<NTRAIN, CC, NBA, TT, 1><<<grid, 256, lds, s>>>(trains, coil, mask, eytab, W, apart,
                                                                    d.nx, d.ny, d.nv, d.T, d.C,
                                                                    p.adj_per_chunk);
    return hipGetLastError();
}

}  // namespace

YPlan make_yplan(const Dims& d)
{
    YPlan p{};
    // Forward: rows per block 32 R with R <= 4 (one coil; more rows per lane
    // spill registers in the 1024-thread block) or <= 2 / 1 with coils; the
    // rows are split into nby balanced blocks whose partial sums of U are
    // added by a small kernel.
    const int rmax = d.C == 1 ? 4 : (d.C <= 8 ? 2 : 1);
    p.nby = ceil_div(d.ny, 32 * rmax);
    p.r_fwd = ceil_div(d.ny, 32 * p.nby);
    // TRs per block: the chunk's per-wave sums live in LDS (at most 64 KB).
    p.fwd_tr = d.C == 1 ? 16 : (d.C <= 8 ? 2 : 1);
    // Coils: per-TR reduction kernel, 2 row steps per lane for up to 8 coils
    // (1 for 16), 32 TRs per block.
    p.r_fwdc = d.C <= 8 ? 2 : 1;
    p.nbyc = ceil_div(d.ny, 2 * FW * p.r_fwdc);
    p.r_fwdc = ceil_div(d.ny, 2 * FW * p.nbyc);
    p.fwd_trc = 32;
    // One-row-per-wave layout (FP16 trains, one coil): g16 column groups of
    // 64 (a power of two covering nx, so a block spans every column), FW/g16
    // row groups, up to 2 row steps per lane (two blocks per CU), 8 TRs per
    // block; g16 = 0 (the
    // two-row layout) when nx > 64 FW.
    p.g16 = 1;
    while (p.g16 * 64 < d.nx && p.g16 < FW) p.g16 *= 2;
    if (p.g16 * 64 < d.nx) p.g16 = 0;
    const int rg = p.g16 ? FW / p.g16 : 2 * FW;
    p.nby16 = ceil_div(d.ny, rg * 2);
    p.r_fwd16 = ceil_div(d.ny, rg * p.nby16);
    p.fwd_tr16 = 8;
    // Wide layout (FP16 trains, one coil, nx a multiple of 4, at most 256
    // columns): NT TRs per block, nbyw row slabs.
    const bool wide = d.C == 1 && d.nx % 4 == 0 && d.nx <= 256;
    // FP16 trains only (with FP32 trains the kernel's registers allow just 2
    // TRs per block in mode 1, slower than the layouts above). Measured at
    // 224 x 224, 1120 TRs, four trains, inside GN steps (TRs x waves per
    // block, row slabs: forward time): 4 x 8, 8 slabs 87.5 us; 8 x 4 98.4;
    // 4 x 4 89.8; 2 x 8 95.3; 2 x 4 97.7; 4 x 8 with 4 slabs 91.4, with 16
    // 91.4. Standalone, with the trains not in cache, 8 x 4 led (93 against
    // 116 us): inside the CG loop each y-stage starts on trains the other
    // just read, and that order favours 4 x 8.
    p.ntw16 = wide ? 4 : 0;
    p.ntws16 = wide ? 4 : 0;
    p.nww = 8;
    p.nbyw = std::min(d.ny, std::max(8, ceil_div(d.ny, 256)));   // <= 256 rows per slab
    p.roww = ceil_div(d.ny, p.nbyw);
    p.nbyw = ceil_div(d.ny, p.roww);
    // Adjoint: one row per lane (8 rows per block) and 8 TR chunks: enough
    // blocks in flight to stream the trains near the HBM limit, with partial
    // sums of 8 chunks x 8 floats per voxel.
    p.r_adj = 1;
    // One coil: 9 chunks (measured at 224 x 224, 1120 TRs, per chunk count
    // 4 / 5 / 8 / 9 / 12: FP16 wide kernel 92 / 104 / 96 / 92 / 98 us, FP32
    // 183 / 162 / 171 / 162 / 169 us; inside GN steps, four FP16 trains:
    // 4 / 9 / 18 chunks 88.0 / 82.3 / 83.7 us). Coils: 8 (the 256 x 256, 8-coil GN step
    // took 1.6 ms longer with 9).
    p.adj_chunks = std::min(d.C == 1 ? 9 : 8, d.T);
    // LDS staging of the y-phases: chunk TRs x rows of a block (<= 64 KB;
    // rows of the 512-voxel blocks of the FP16 pair kernel).
    const int rows = std::min(d.ny, 512 / d.nx + 2);
    while (ceil_div(d.T, p.adj_chunks) * rows * 8 > 65536) ++p.adj_chunks;
    p.adj_per_chunk = ceil_div(d.T, p.adj_chunks);
    p.adj_chunks = ceil_div(d.T, p.adj_per_chunk);
    // Adjoint x-GEMM: split K when the output tile grid is small.
    const int tiles = ceil_div(2 * d.nx, GBN) * ceil_div(d.C * d.T, GBM);
    const int kchunks = ceil_div(2 * d.nk, GBK);
    const int ks = tiles >= 256 ? 1 : 256 / std::max(tiles, 1);
    p.ksplit_adj = ks >= 4 ? 4 : (ks >= 2 ? 2 : 1);
    while (p.ksplit_adj > kchunks) p.ksplit_adj /= 2;
    return p;
}

template <typename TT>
hipError_t fwd_typed(const Dims& d, const YPlan& p, int mode, const TT* trains, const float* theta,
                     const float* v, const float2* coil, const uint8_t* mask, const float2* eytab,
                     float2* upart, int* nby, hipStream_t s)
{
#define FWD_MODES(CC_)                                                                           \
    switch (mode) {                                                                              \
        case 0: return fwd_R<0, CC_>(d, p, trains, theta, v, coil, mask, eytab, upart, nby, s); \
        case 1: return fwd_R<1, CC_>(d, p, trains, theta, v, coil, mask, eytab, upart, nby, s); \
        case 3: return fwd_R<3, CC_>(d, p, trains, theta, v, coil, mask, eytab, upart, nby, s); \
        default: return hipErrorInvalidValue;                                                   \
    }
    if (d.C == 1) FWD_MODES(1)
    if (d.C <= 8) FWD_MODES(8)
    FWD_MODES(16)
#undef FWD_MODES
}

template <typename TT>
hipError_t adj_typed(const Dims& d, const YPlan& p, const TT* trains, int ntr_trains,
                     const float2* coil, const uint8_t* mask, const float2* eytab, const float2* W,
                     float* apart, hipStream_t s)
{
    if (ntr_trains == 4) {
        if (d.C == 1) return adj_launch<4, 1>(d, p, trains, coil, mask, eytab, W, apart, s);
        if (d.C <= 8) return adj_launch<4, 8>(d, p, trains, coil, mask, eytab, W, apart, s);
        return adj_launch<4, 16>(d, p, trains, coil, mask, eytab, W, apart, s);
    }
    if (ntr_trains == 3) {
        if (d.C == 1) return adj_launch<3, 1>(d, p, trains, coil, mask, eytab, W, apart, s);
        if (d.C <= 8) return adj_launch<3, 8>(d, p, trains, coil, mask, eytab, W, apart, s);
        return adj_launch<3, 16>(d, p, trains, coil, mask, eytab, W, apart, s);
    }
    if (ntr_trains != 1) return hipErrorInvalidValue;
    if (d.C == 1) return adj_launch<1, 1>(d, p, trains, coil, mask, eytab, W, apart, s);
    if (d.C <= 8) return adj_launch<1, 8>(d, p, trains, coil, mask, eytab, W, apart, s);
    return adj_launch<1, 16>(d, p, trains, coil, mask, eytab, W, apart, s);
}

hipError_t launch_ystage_fwd(const Dims& d, const YPlan& p, int mode, const void* trains, bool f16,
                             const float* theta, const float* v, const float2* coil,
                             const uint8_t* mask, const float2* eytab, float2* upart, int* nby,
                             hipStream_t s)
{
    *nby = 1;
    return f16 ? fwd_typed(d, p, mode, static_cast<const _Float16*>(trains), theta, v, coil, mask, eytab, upart, nby, s)
               : fwd_typed(d, p, mode, static_cast<const float*>(trains), theta, v, coil, mask, eytab, upart, nby, s);
}

hipError_t launch_usum(const Dims& d, float2* upart, int nby, hipStream_t s)
{
    if (nby <= 1) return hipSuccess;
    const size_t count = (size_t)d.C * d.T * d.nx;
    usum_kernel<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(upart, nby, count);
    return hipGetLastError();
}

size_t bfrag_bytes(const Dims& d, int dir, int enc)
{
    const int Kr = dir == 0 ? 2 * d.nx : 2 * d.nk, Nr = dir == 0 ? 2 * d.nk : 2 * d.nx;
    return (size_t)ceil_div(Kr, 32) * ceil_div(Nr, 16) * (enc == 1 ? 2 : 1) * 64 * sizeof(uint4);
}

int xgemm_direct_blocks(const Dims& d) { return ceil_div(2 * d.nk, 16) * ceil_div(d.C * d.T, 16); }   // >= any tile

hipError_t launch_build_bfrag(const Dims& d, const float2* extab, void* f1, void* a1, void* f2,
                              void* a2, hipStream_t s)
{
    auto grid = [&](int dir) {
        const int Kr = dir == 0 ? 2 * d.nx : 2 * d.nk, Nr = dir == 0 ? 2 * d.nk : 2 * d.nx;
        return (unsigned)ceil_div(ceil_div(Kr, 32) * ceil_div(Nr, 16) * 64, 256);
    };
    build_bfrag_kernel<0, 1><<<grid(0), 256, 0, s>>>(extab, (uint4*)f1, d.nx, d.nk);
    build_bfrag_kernel<1, 1><<<grid(1), 256, 0, s>>>(extab, (uint4*)a1, d.nx, d.nk);
    build_bfrag_kernel<0, 2><<<grid(0), 256, 0, s>>>(extab, (uint4*)f2, d.nx, d.nk);
    build_bfrag_kernel<1, 2><<<grid(1), 256, 0, s>>>(extab, (uint4*)a2, d.nx, d.nk);
    return hipGetLastError();
}

// Tiles of 32 rows x 32 columns per wave; 2 waves per tile split K in the
// forward (K = 2 nx), 4 in the adjoint (K = 2 nk). Measured at 224 x 224 with
// 1120 TRs (HIP-event times, forward / adjoint): 16 x 32 tiles with 1 wave
// 16 / 23 us, 16 x 32 with 4 waves 16 / 15, 32 x 32 with 2 waves 15.4 / 17.4,
// with 4 waves 16.4 / 13.1, 64 x 32 with 4 waves 18.9 / 14.7; the LDS-tiled
// kernel 19 / 25 (including its split-K sum).
// 32 x 32 tiles per wave; 32 x 16 measured 21 / 19 us (forward / adjoint),
// 32 x 64 17 / 13 us, against 15 / 13 us.
constexpr int XRW = 2, XCW = 2;

// Many rows (coils x TRs >= 4096): 64 x 64 tiles per wave, which halves the
// operand reads through L2, and fewer waves per tile (there are tiles enough).
constexpr int XBIG_M = 4096, XBRW = 4, XBCW = 4;

template <int DIR, int MODE, int RW, int CW, int KS>
void xgemm_direct_t(int enc, const Dims& d, const float2* A, const void* bfrag, const float2* data,
                    float2* out, double* red, int* nred, hipStream_t s)
{
    const int Nr = DIR == 0 ? 2 * d.nk : 2 * d.nx;
    dim3 grid(ceil_div(Nr, 16 * CW), ceil_div(d.C * d.T, 16 * RW));
    if (nred) *nred = grid.x * grid.y;
    if (enc == 1)
        xgemm_direct_kernel<DIR, MODE, 1, KS, RW, CW><<<grid, 64 * KS, 0, s>>>(
            A, (const uint4*)bfrag, data, out, red, d.C * d.T, d.nx, d.nk);
    else
        xgemm_direct_kernel<DIR, MODE, 2, KS, RW, CW><<<grid, 64 * KS, 0, s>>>(
            A, (const uint4*)bfrag, data, out, red, d.C * d.T, d.nx, d.nk);
}

template <int DIR, int MODE>
void xgemm_direct(int enc, const Dims& d, const float2* A, const void* bfrag, const float2* data,
                  float2* out, double* red, int* nred, hipStream_t s)
{
    if (d.C * d.T >= XBIG_M)
        xgemm_direct_t<DIR, MODE, XBRW, XBCW, DIR == 0 ? 1 : 2>(enc, d, A, bfrag, data, out, red, nred, s);
    else
        xgemm_direct_t<DIR, MODE, XRW, XCW, DIR == 0 ? 2 : 4>(enc, d, A, bfrag, data, out, red, nred, s);
}

hipError_t launch_xgemm_fwd(const Dims& d, const YPlan& p, int enc, int mode, const float2* U,
                            const float2* extab, const void* bfrag, const float2* data, float2* out,
                            double* red, int* nred, hipStream_t s)
{
    (void)p;
    const int M = d.C * d.T;
    if (enc != 0) {
        if (bfrag == nullptr) return hipErrorInvalidValue;
        if (mode == 0)
            xgemm_direct<0, 0>(enc, d, U, bfrag, data, out, red, nred, s);
        else if (mode == 1)
            xgemm_direct<0, 1>(enc, d, U, bfrag, data, out, red, nred, s);
        else
            xgemm_direct<0, 2>(enc, d, U, bfrag, data, out, red, nred, s);
        return hipGetLastError();
    }
    dim3 grid(ceil_div(2 * d.nk, GBN), ceil_div(M, GBM), 1);
    if (nred) *nred = grid.x * grid.y;
    const int chunks = ceil_div(2 * d.nx, GBK);
    if (mode == 0)
        xgemm_any<0, 0>(grid, s, U, extab, data, out, red, M, d.nx, d.nk, chunks, 0);
    else if (mode == 1)
        xgemm_any<0, 1>(grid, s, U, extab, data, out, red, M, d.nx, d.nk, chunks, 0);
    else
        xgemm_any<0, 2>(grid, s, U, extab, data, out, red, M, d.nx, d.nk, chunks, 0);
    return hipGetLastError();
}

hipError_t launch_xgemm_adj(const Dims& d, const YPlan& p, int enc, const float2* w,
                            const float2* extab, const void* bfrag, float2* W, hipStream_t s)
{
    const int M = d.C * d.T;
    if (enc != 0) {   // no K split: W complete in partial 0
        if (bfrag == nullptr) return hipErrorInvalidValue;
        xgemm_direct<1, 0>(enc, d, w, bfrag, nullptr, W, nullptr, nullptr, s);
        return hipGetLastError();
    }
    const int kchunks = ceil_div(2 * d.nk, GBK);
    const int per = ceil_div(kchunks, p.ksplit_adj);
    dim3 grid(ceil_div(2 * d.nx, GBN), ceil_div(M, GBM), p.ksplit_adj);
    const size_t stride = (size_t)M * 2 * d.nx;   // floats per partial
    xgemm_any<1, 0>(grid, s, w, extab, nullptr, W, nullptr, M, d.nx, d.nk, per, stride);
    if (p.ksplit_adj > 1) {
        const size_t count = (size_t)M * d.nx;
        wsum_kernel<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(W, p.ksplit_adj, count);
    }
    return hipGetLastError();
}

hipError_t launch_ystage_adj(const Dims& d, const YPlan& p, const void* trains, bool f16, int ntr_trains,
                             const float2* coil, const uint8_t* mask, const float2* eytab,
                             const float2* W, float* apart, hipStream_t s)
{
    return f16 ? adj_typed(d, p, static_cast<const _Float16*>(trains), ntr_trains, coil, mask, eytab, W, apart, s)
               : adj_typed(d, p, static_cast<const float*>(trains), ntr_trains, coil, mask, eytab, W, apart, s);
}

hipError_t launch_jhw_finish(const Dims& d, const YPlan& p, const float* apart, const float* theta,
                             const uint8_t* mask, int param_mask, float* g, const float* dir,
                             double* part, hipStream_t s, const float* step, const float* res)
{
    const int nb = ceil_div(d.nv, 256);
    if (dir != nullptr && step == nullptr && res == nullptr) return hipErrorInvalidValue;
#define FINISH(NP)                                                                                       \
    if (dir != nullptr && step != nullptr)                                                               \
        jhw_finish_kernel<2, NP><<<nb, 256, 0, s>>>(apart, p.adj_chunks, theta, mask, param_mask, g, d.nv, \
                                                    dir, step, nullptr, part);                           \
    else if (dir != nullptr)                                                                             \
        jhw_finish_kernel<3, NP><<<nb, 256, 0, s>>>(apart, p.adj_chunks, theta, mask, param_mask, g, d.nv, \
                                                    dir, nullptr, res, part);                            \
    else                                                                                                 \
        jhw_finish_kernel<0, NP><<<nb, 256, 0, s>>>(apart, p.adj_chunks, theta, mask, param_mask, g, d.nv, \
                                                    nullptr, nullptr, nullptr, nullptr);
    if (d.np == 6) {
        FINISH(6)
    } else {
        FINISH(5)
    }
#undef FINISH
    return hipGetLastError();
}

hipError_t launch_rho_adj_finish(const Dims& d, const YPlan& p, const float* apart,
                                 const uint8_t* mask, float2* out, hipStream_t s)
{
    rho_adj_finish_kernel<<<ceil_div(d.nv, 256), 256, 0, s>>>(apart, p.adj_chunks, mask, out, d.nv);
    return hipGetLastError();
}

}  // namespace mrstat
