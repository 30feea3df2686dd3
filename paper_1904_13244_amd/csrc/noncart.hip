// Non-Cartesian encoding: the voxel x sample contraction for any k-space
// trajectory (the method's non-Cartesian extensibility: Introduction,
// Discussion). Sample k of TR n sits at (kx, ky) cycles per field of view and
//     E[n,k,j] = exp(-2 pi i (ax[n,k] (ix - nx/2) + ay[n,k] (iy - ny/2))),
// ax = kx / nx, ay = ky / ny (FP64 tables). The phase still factors into an x
// and a y part, so per TR the contraction is a dense complex GEMM:
//   forward  s[k] = sum_iy Ey[k,iy] P[k,iy],  P = Ex X^T (nk x ny, K = nx),
//            X[iy,ix] the voxel values of the TR;
//   adjoint  V[iy,ix] = sum_k G[k,iy] H[k,ix],  G = conj(Ey) w, H = conj(Ex),
//            then A_p[j] += mu_p[n,j] V[j] over the TRs of a chunk.
// Both run on the matrix cores in the real 2 x 2-block form of a complex
// product, with every phase generated on the fly (argument reduced in FP64,
// sin/cos of the reduced fraction in FP32):
//   ENC 0: v_mfma_f32_16x16x4_f32 (FP32 operands);
//   ENC 1: v_mfma_f32_16x16x32_bf16 on split operands, hi*hi + hi*lo + lo*hi.
// MFMA operand layouts (as in encode.hip): 16x16x4 f32: A lane l -> (row
// l%16, k l/16), B lane l -> (k l/16, col l%16); 16x16x32: A lane l -> (row
// l%16, k 8(l/16)..+7), B lane l -> (k 8(l/16)..+7, col l%16); D lane l ->
// (rows 4(l/16)+i, col l%16) for both.
#include "mrstat_internal.h"

#include <algorithm>

namespace mrstat {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// exp(-2 pi i a x) for an FP64 coefficient a and an integer position x: the
// product is reduced to a fraction of a cycle in FP64, then sin and cos of pi
// times twice that fraction in FP32.
__device__ __forceinline__ float2 phase_of(double a, int x)
{
    const double t = a * (double)x;
    const double f = t - rint(t);   // [-0.5, 0.5]
    float sn, cs;
    sincospif((float)(-2.0 * f), &sn, &cs);
    return make_float2(cs, sn);
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

__device__ __forceinline__ unsigned int bf16_rne(float x)
{
    const unsigned int u = __float_as_uint(x);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// (re, im) -> hi word (bf16 re | bf16 im << 16) and lo word of the remainders.
__device__ __forceinline__ uint2 split_pair(float re, float im)
{
    const unsigned int hr = bf16_rne(re), hi = bf16_rne(im);
    const unsigned int lr = bf16_rne(re - __uint_as_float(hr << 16));
    const unsigned int li = bf16_rne(im - __uint_as_float(hi << 16));
    return make_uint2(hr | (hi << 16), lr | (li << 16));
}

__device__ __forceinline__ f4 mma_bf16(const uint4& a, const uint4& b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                   c, 0, 0, 0);
}

// Real-form B words of the forward and adjoint: a word holds (re, im) of one
// complex operand entry; column parity b = 0 needs (re, -im), b = 1 (im, re).
__device__ __forceinline__ uint4 bform(uint4 w, int b)
{
    if (b == 0) return make_uint4(w.x ^ 0x80000000u, w.y ^ 0x80000000u, w.z ^ 0x80000000u, w.w ^ 0x80000000u);
    return make_uint4((w.x >> 16) | (w.x << 16), (w.y >> 16) | (w.y << 16), (w.z >> 16) | (w.z << 16),
                      (w.w >> 16) | (w.w << 16));
}

template <typename TT>
__device__ __forceinline__ float ld_train(const TT* p) { return (float)*p; }

// ------------------------------------------------------------------------
// Voxel values of the forward, once per product: X[n][j] = i rho_j mu0[n,j]
// (NTRV 1, the signal) or i (rho_j sum_p v_p dm_p/dtheta_p + (v3 + i v4) mu0)
// (NTRV 4: all tangents; 3: without dm/dB1, whose direction entry is 0);
// zero for masked voxels. A streaming pass over the trains. SPLIT (the
// split-BF16 forward without coil weights) stores each value already split
// into its (hi, lo) words instead of the FP32 pair, the same 8 bytes.
// ------------------------------------------------------------------------
template <int NTRV, typename TT, bool SPLIT>
__global__ __launch_bounds__(256) void nc_x_kernel(const TT* __restrict__ trains, const float* __restrict__ theta,
                                                   const float* __restrict__ v, const uint8_t* __restrict__ mask,
                                                   float2* __restrict__ X, int nv, int T)
{
    const size_t count = (size_t)T * nv, plane = count;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
        const int j = (int)(i % nv);
        float xr = 0.f, xi = 0.f;
        if (mask == nullptr || mask[j] != 0) {
            const float rr = theta[3 * (size_t)nv + j], ri = theta[4 * (size_t)nv + j];
            const float mu0 = ld_train(trains + i);
            if constexpr (NTRV == 1) {
                xr = -ri * mu0;
                xi = rr * mu0;
            } else {
                float t = 0.f;
#pragma unroll
                for (int q = 0; q < NTRV - 1; ++q) t = fmaf(v[(size_t)q * nv + j], ld_train(trains + (q + 1) * plane + i), t);
                const float v3 = v[3 * (size_t)nv + j], v4 = v[4 * (size_t)nv + j];
                // x = i (rho t + (v3 + i v4) mu0)
                xr = -(ri * t + v4 * mu0);
                xi = rr * t + v3 * mu0;
            }
        }
        if constexpr (SPLIT)
            reinterpret_cast<uint2*>(X)[i] = split_pair(xr, xi);
        else
            X[i] = make_float2(xr, xi);
    }
}

// ------------------------------------------------------------------------
// Forward: a block of 4 waves per (TR n, 64 samples, coil); wave w owns
// samples k0 = 64 kt + 16 w .. +15. Its A fragments (Ex of its 16 samples
// over all nx columns, KS K-steps) are generated once and kept in registers;
// the voxel values X of 32 image rows at a time are staged in LDS (times the
// coil weight; ENC 1: split into bf16 hi/lo words), NC_XB of each thread's
// loads issued together, then each wave multiplies them for 4 column blocks
// of 8 rows, and the epilogue applies Ey and sums over the rows. Blocks are
// dealt so that the sample tiles of one TR share an XCD (its voxel values
// come through one L2). K goes in parts of 64 columns (A fragments of one
// part in registers: four waves per SIMD). Measured at 224 x 224, 1120 spokes
// (FP32 / split-BF16): all of K at once 5.08 / 2.32 ms (two waves per SIMD),
// two parts 4.14 / 2.07 (three), four 3.72 / 2.02; the split-BF16 tile staged
// in both lane-parity forms (no operand re-forming in the K loop) 1.91; without
// coil weights the values split once by the voxel-value pass 1.68.
// MODE 0: out = data - s (and FP64 partials of |out|^2); 1: out = -s; 2: s.
// ------------------------------------------------------------------------
constexpr int NC_KS0 = 128;   // FP32 K-steps of 4 real k: nx <= 256
constexpr int NC_KS1 = 16;    // BF16 K-steps of 32 real k: nx <= 256
constexpr int NC_KP = 4;      // K parts of 64 columns; one part's A fragments in registers at a time
constexpr int NC_PCOLS = 64;  // columns per K part
constexpr int NC_ROWS = 32;   // image rows per LDS tile
constexpr int NC_XB = 4;      // voxel values per thread loaded together
static_assert(NC_ROWS == 32, "forward tile: 4 column blocks of 8 rows per lane group");
static_assert(NC_KP * NC_PCOLS == 256 && NC_KS0 % NC_KP == 0 && NC_KS1 % NC_KP == 0, "forward K parts");

template <int ENC, int MODE, bool PRE>   // PRE: X holds split words (ENC 1, no coil weights)
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void nc_fwd_kernel(
    const float2* __restrict__ X, const float2* __restrict__ coil, const double* __restrict__ ax,
    const double* __restrict__ ay, const float2* __restrict__ data, float2* __restrict__ out,
    double* __restrict__ red, int nx, int ny, int nv, int T, int nk, int KT, int nxp)
{
    constexpr int KS0P = NC_KS0 / NC_KP, KS1P = NC_KS1 / NC_KP;   // K-steps per part
    extern __shared__ __attribute__((aligned(16))) unsigned char nc_smem[];
    __shared__ double rs[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int bid = blockIdx.x;
    const int slot = bid >> 3;
    const int kt = slot % KT;
    const int n = (slot / KT) * 8 + (bid & 7);
    const int c = blockIdx.y;
    const size_t red_at = (size_t)c * gridDim.x + bid;
    if (n >= T) {
        if (MODE == 0 && tid == 0) red[red_at] = 0.0;
        return;
    }
    const int k0 = kt * 64 + wave * 16;
    const int krow = k0 + (lane & 15);
    const bool krow_ok = krow < nk;
    const double axk = krow_ok ? ax[(size_t)n * nk + krow] : 0.0;
    const int h = lane >> 4;   // 0..3
    const int KS = ENC == 0 ? (2 * nx + 3) / 4 : (2 * nx + 31) / 32;

    // The phases along a row of Ex are a geometric sequence: a lane's columns
    // come in groups whose first phase is taken from sin/cos and the others
    // as its products with the phases of the group's offsets.
    float2 off[ENC == 0 ? 8 : 4];
#pragma unroll
    for (int o = 0; o < (ENC == 0 ? 8 : 4); ++o)
        off[o] = o == 0 ? make_float2(1.f, 0.f) : phase_of(axk, ENC == 0 ? 2 * o : o);
    // Epilogue phases Ey[k][iy] of the lane's 4 samples, iy = iy0 + 8 cb + rb:
    // phase(iy0 + rb) from sin/cos per tile, times phase(8) once per column
    // block.
    const int rb = (lane & 15) >> 1;
    double ayv[4];
    float2 e8[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int k = k0 + 4 * h + i;
        ayv[i] = k < nk ? ay[(size_t)n * nk + k] : 0.0;
        e8[i] = phase_of(ayv[i], 8);
    }

    float sacc[4] = {0.f, 0.f, 0.f, 0.f};
    const int b = lane & 1;
    const float2* Xn = X + (size_t)n * nv;
    float2* xs0 = reinterpret_cast<float2*>(nc_smem);               // ENC 0: [ROWS][nxp]
    // ENC 1: [2][ROWS][nxp] (hi, lo) words already in the real-form B order of
    // each lane parity (copy 0: (re, -im), copy 1: (im, re)); the copies are
    // one entry apart in banks so the two parities do not collide.
    uint2* xs1 = reinterpret_cast<uint2*>(nc_smem);
    const int tile_n = NC_ROWS * nxp, copy1 = tile_n + 1;
    // K parts: columns [NC_PCOLS kp, NC_PCOLS (kp + 1)); the sums over the
    // rows are linear in P, so each part's Ey-weighted sums simply add up.
    for (int kp = 0; kp < NC_KP && kp * NC_PCOLS < nx; ++kp) {
        const int cx0 = kp * NC_PCOLS;
        // A fragments of this part: Ex[krow][ix] in the real form
        // A'[k][2 ix + a] = (re, im).
        float a0[ENC == 0 ? KS0P : 1];
        uint4 ahi[ENC == 1 ? KS1P : 1], alo[ENC == 1 ? KS1P : 1];
        if constexpr (ENC == 0) {
            // columns ix = cx0 + 2 sl + h/2, sl = 8 g + o: phase(cx0 + 16 g + h/2) phase(2 o)
#pragma unroll
            for (int g = 0; g < KS0P / 8; ++g) {
                const bool any = KS0P * kp + 8 * g < KS && krow_ok;
                const float2 base = any ? phase_of(axk, cx0 + 16 * g + (h >> 1) - nx / 2) : make_float2(0.f, 0.f);
#pragma unroll
                for (int o = 0; o < 8; ++o) {
                    const int sl = 8 * g + o, ix = cx0 + 2 * sl + (h >> 1);
                    float val = 0.f;
                    if (KS0P * kp + sl < KS && krow_ok && ix < nx) {
                        const float2 e = cmul(base, off[o]);
                        val = (h & 1) ? e.y : e.x;
                    }
                    a0[sl] = val;
                }
            }
        } else {
            // columns ix = cx0 + 16 sl + 4 h + m: phase(cx0 + 16 sl + 4 h) phase(m)
#pragma unroll
            for (int sl = 0; sl < KS1P; ++sl) {
                const bool any = KS1P * kp + sl < KS && krow_ok;
                const float2 base = any ? phase_of(axk, cx0 + 16 * sl + 4 * h - nx / 2) : make_float2(0.f, 0.f);
                unsigned int hw[4], lw[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int ix = cx0 + 16 * sl + 4 * h + m;
                    float2 e = make_float2(0.f, 0.f);
                    if (any && ix < nx) e = cmul(base, off[m]);
                    const uint2 w = split_pair(e.x, e.y);
                    hw[m] = w.x;
                    lw[m] = w.y;
                }
                ahi[sl] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
                alo[sl] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
            }
        }
        for (int iy0 = 0; iy0 < ny; iy0 += NC_ROWS) {
            __syncthreads();   // the previous tile has been read
            if constexpr (PRE) {
                // Split words from the voxel-value pass: only the two
                // operand orders are formed here.
                const uint2* Xw = reinterpret_cast<const uint2*>(Xn);
                for (int e0 = tid; e0 < tile_n; e0 += 256 * NC_XB) {
                    uint2 wv[NC_XB];
#pragma unroll
                    for (int u = 0; u < NC_XB; ++u) {
                        const int e = e0 + 256 * u;
                        const int r = e / nxp, ixl = e % nxp, iy = iy0 + r, ix = cx0 + ixl;
                        const bool ok = e < tile_n && ixl < NC_PCOLS && ix < nx && iy < ny;
                        wv[u] = ok ? Xw[(size_t)iy * nx + ix] : make_uint2(0u, 0u);
                    }
#pragma unroll
                    for (int u = 0; u < NC_XB; ++u) {
                        const int e = e0 + 256 * u;
                        if (e >= tile_n) break;
                        const uint2 w = wv[u];
                        xs1[e] = make_uint2(w.x ^ 0x80000000u, w.y ^ 0x80000000u);
                        xs1[copy1 + e] = make_uint2((w.x >> 16) | (w.x << 16), (w.y >> 16) | (w.y << 16));
                    }
                }
            } else {
                for (int e0 = tid; e0 < tile_n; e0 += 256 * NC_XB) {
                    float2 xv[NC_XB], cv[NC_XB];
#pragma unroll
                    for (int u = 0; u < NC_XB; ++u) {
                        const int e = e0 + 256 * u;
                        const int r = e / nxp, ixl = e % nxp, iy = iy0 + r, ix = cx0 + ixl;
                        const bool ok = e < tile_n && ixl < NC_PCOLS && ix < nx && iy < ny;
                        const size_t j = ok ? (size_t)iy * nx + ix : 0;
                        xv[u] = ok ? Xn[j] : make_float2(0.f, 0.f);
                        cv[u] = coil != nullptr && ok ? coil[(size_t)c * nv + j] : make_float2(1.f, 0.f);
                    }
#pragma unroll
                    for (int u = 0; u < NC_XB; ++u) {
                        const int e = e0 + 256 * u;
                        if (e >= tile_n) break;
                        const float xr = cv[u].x * xv[u].x - cv[u].y * xv[u].y;
                        const float xi = cv[u].x * xv[u].y + cv[u].y * xv[u].x;
                        if constexpr (ENC == 0) {
                            xs0[e] = make_float2(xr, xi);
                        } else {
                            const uint2 w = split_pair(xr, xi);
                            xs1[e] = make_uint2(w.x ^ 0x80000000u, w.y ^ 0x80000000u);
                            xs1[copy1 + e] = make_uint2((w.x >> 16) | (w.x << 16), (w.y >> 16) | (w.y << 16));
                        }
                    }
                }
            }
            __syncthreads();
            float2 ebase[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) ebase[i] = phase_of(ayv[i], iy0 + rb - ny / 2);
#pragma unroll
            for (int cb = 0; cb < NC_ROWS / 8; ++cb) {
                const int rl = 8 * cb + rb;   // tile row of this lane's column
                f4 acc = {0.f, 0.f, 0.f, 0.f};
                if constexpr (ENC == 0) {
#pragma unroll
                    for (int sl = 0; sl < KS0P; ++sl) {
                        if (KS0P * kp + sl < KS) {
                            const float2 x = xs0[rl * nxp + 2 * sl + (h >> 1)];
                            const int a = h & 1;
                            const float bv = a == 0 ? (b == 0 ? x.x : x.y) : (b == 0 ? -x.y : x.x);
                            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[sl], bv, acc, 0, 0, 0);
                        }
                    }
                } else {
#pragma unroll
                    for (int sl = 0; sl < KS1P; ++sl) {
                        if (KS1P * kp + sl < KS) {
                            const uint2* src = xs1 + b * copy1 + rl * nxp + 16 * sl + 4 * h;
                            const uint2 p0 = src[0], p1 = src[1], p2 = src[2], p3 = src[3];
                            const uint4 bh = make_uint4(p0.x, p1.x, p2.x, p3.x);
                            const uint4 bl = make_uint4(p0.y, p1.y, p2.y, p3.y);
                            acc = mma_bf16(ahi[sl], bh, acc);
                            acc = mma_bf16(ahi[sl], bl, acc);
                            acc = mma_bf16(alo[sl], bh, acc);
                        }
                    }
                }
                // Epilogue of this column block: P[k, iy] (re in even lanes, im
                // in odd) times Ey[k, iy], summed into the lane's running row
                // sums.
                const int iy = iy0 + rl;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float own = acc[i];
                    const float oth = __shfl_xor(own, 1);
                    const float pr = b == 0 ? own : oth, pi = b == 0 ? oth : own;
                    const int k = k0 + 4 * h + i;
                    if (k < nk && iy < ny) {
                        const float2 ey = ebase[i];
                        sacc[i] += b == 0 ? pr * ey.x - pi * ey.y : pr * ey.y + pi * ey.x;
                    }
                    ebase[i] = cmul(ebase[i], e8[i]);   // the next column block's rows
                }
            }
        }
    }
    // Sum over the 8 column lanes of each parity: lanes 0 and 1 of each
    // 16-lane group then hold (re, im) of s for rows 4 h + i.
    double sq = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        float vv = sacc[i];
        vv += __shfl_xor(vv, 2);
        vv += __shfl_xor(vv, 4);
        vv += __shfl_xor(vv, 8);
        const int k = k0 + 4 * h + i;
        if ((lane & 14) == 0 && k < nk) {
            const size_t idx = ((size_t)c * T + n) * nk + k;
            float* o = reinterpret_cast<float*>(out) + 2 * idx + b;
            if constexpr (MODE == 0) {
                const float rv = reinterpret_cast<const float*>(data)[2 * idx + b] - vv;
                *o = rv;
                sq += (double)rv * (double)rv;
            } else if constexpr (MODE == 1) {
                *o = -vv;
            } else {
                *o = vv;
            }
        }
    }
    if constexpr (MODE == 0) {
        for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off);
        if (lane == 0) rs[wave] = sq;
        __syncthreads();
        if (tid == 0) red[red_at] = (rs[0] + rs[1]) + (rs[2] + rs[3]);
    }
}

// ------------------------------------------------------------------------
// Adjoint: a block of 4 waves per (tile of 64 image rows x 32 columns, TR
// chunk); wave w owns rows 16 w .. +15 of the tile, 4 column blocks of 8
// columns. For each TR and coil the samples go in chunks of 64: the block
// writes G[k][row] = conj(Ey[k][iy]) w_c[k] and H[k][col] = conj(Ex[k][ix])
// into LDS (as [row][k] and [col][k], so a lane's 4 consecutive samples are
// adjacent), then the waves multiply; each coil's product is weighted by
// conj(C_c[j]) per voxel, and after the TR the epilogue adds mu_p[n,j] V[j]
// to the lane's running sums. Chunk partials: apart[chunk][2 p + (re, im)][j]
// with 8 planes per chunk (2 for the m train alone), the layout of the
// Cartesian adjoint, so the same gradient assembly follows. Measured at 224 x
// 224, 1120 spokes (FP32 / split-BF16): unpadded table rows 14.3 / 5.9 ms,
// with the phases by angle addition 13.3 / 3.3, padded rows 5.0 / 2.9; the
// next chunk's trajectory and data values loaded ahead need 6 more registers:
// 5.0 / 2.9 with 56 bytes per lane spilled at three waves per SIMD, 5.8 / 4.2
// at two; H staged in both lane-parity operand orders (no re-forming in the K
// loop, 68 KB of LDS: two blocks per CU instead of three) 3.6 (split-BF16).
// ------------------------------------------------------------------------
constexpr int NCA_TY = 64, NCA_TX = 32, NCA_KC = 64;
// LDS row stride of the tables: two entries of padding, so the rows (16 per
// wave for G, 8 for H) that one MFMA operand read touches fall in different
// banks (the unpadded stride of 512 bytes puts them all in one); 16-byte
// aligned rows.
constexpr int NCA_KCP = NCA_KC + 2;
// The table build gives each of the 256 threads one sample and every 4th
// row (column) of the tile.
static_assert(256 / NCA_KC == 4 && NCA_TY % 16 == 0 && NCA_TX % 16 == 0, "adjoint table build layout");

template <int ENC, int NTR, typename TT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void nc_adj_kernel(
    const TT* __restrict__ trains, const float2* __restrict__ coil, const uint8_t* __restrict__ mask,
    const double* __restrict__ ax, const double* __restrict__ ay, const float2* __restrict__ w,
    float* __restrict__ apart, int nx, int ny, int nv, int T, int nk, int C, int n_per_chunk, int ntx)
{
    // LDS: G [TY][KC] and H [TX][KC] entries of 8 bytes: ENC 0 (re, im) FP32,
    // ENC 1 (hi word, lo word).
    __shared__ __attribute__((aligned(16))) uint2 gs[NCA_TY * NCA_KCP];
    __shared__ __attribute__((aligned(16))) uint2 hs[NCA_TX * NCA_KCP];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tile = blockIdx.x;
    const int iy_base = (tile / ntx) * NCA_TY, ix_base = (tile % ntx) * NCA_TX;
    const int chunk = blockIdx.y;
    const int n0 = chunk * n_per_chunk, n1 = min(T, n0 + n_per_chunk);
    const int h = lane >> 4, b = lane & 1;
    const size_t plane = (size_t)T * nv;

    // This lane's outputs: rows iy_base + 16 wave + 4 h + i, column
    // ix_base + 8 cb + (lane & 15) / 2, part b (0 re, 1 im).
    float aacc[4][4][NTR];   // [cb][i][train]
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int p = 0; p < NTR; ++p) aacc[cb][i][p] = 0.f;

    for (int n = n0; n < n1; ++n) {
        f4 vacc[4];   // V of this TR (summed over coils with their weights)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) vacc[cb] = f4{0.f, 0.f, 0.f, 0.f};
        for (int c = 0; c < C; ++c) {
            f4 cacc[4];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) cacc[cb] = f4{0.f, 0.f, 0.f, 0.f};
            for (int kc0 = 0; kc0 < nk; kc0 += NCA_KC) {
                __syncthreads();   // the previous chunk's tables have been read
                // G: 64 rows x 64 samples; H: 32 columns x 64 samples. A
                // thread takes one sample and every 4th row (column): the
                // phases along them form a geometric sequence, so per sample
                // three phases come from sin/cos (the first row, 4 and 16
                // rows on) and the others from complex products of those.
                {
                    const int kk = tid % NCA_KC, r0 = tid / NCA_KC;
                    const int k = kc0 + kk;
                    const bool kok = k < nk;
                    const double ayk = kok ? ay[(size_t)n * nk + k] : 0.0;
                    const double axk = kok ? ax[(size_t)n * nk + k] : 0.0;
                    const float2 ww = kok ? w[((size_t)c * T + n) * nk + k] : make_float2(0.f, 0.f);
                    auto store = [&](uint2* dst, float2 val) {
                        if constexpr (ENC == 0)
                            *dst = make_uint2(__float_as_uint(val.x), __float_as_uint(val.y));
                        else
                            *dst = split_pair(val.x, val.y);
                    };
                    {   // G[r][kk] = conj(Ey[k][iy]) w[k], iy = iy_base + r0 + 4 m
                        const float2 s4 = phase_of(ayk, 4), s16 = phase_of(ayk, 16);
                        const float2 s8 = cmul(s4, s4), s12 = cmul(s8, s4);
                        float2 q = phase_of(ayk, iy_base + r0 - ny / 2);
#pragma unroll 1
                        for (int u = 0; u < NCA_TY / 16; ++u) {
                            const float2 qv[4] = {q, cmul(q, s4), cmul(q, s8), cmul(q, s12)};
#pragma unroll
                            for (int v4 = 0; v4 < 4; ++v4) {
                                const int r = r0 + 16 * u + 4 * v4;
                                const float2 ey = qv[v4];
                                float2 val = make_float2(0.f, 0.f);
                                if (kok && iy_base + r < ny)   // conj(ey) * w
                                    val = make_float2(ey.x * ww.x + ey.y * ww.y, ey.x * ww.y - ey.y * ww.x);
                                store(gs + r * NCA_KCP + kk, val);
                            }
                            q = cmul(q, s16);
                        }
                    }
                    {   // H[r][kk] = conj(Ex[k][ix]), ix = ix_base + r0 + 4 m
                        const float2 s4 = phase_of(axk, 4), s16 = phase_of(axk, 16);
                        const float2 s8 = cmul(s4, s4), s12 = cmul(s8, s4);
                        float2 q = phase_of(axk, ix_base + r0 - nx / 2);
#pragma unroll 1
                        for (int u = 0; u < NCA_TX / 16; ++u) {
                            const float2 qv[4] = {q, cmul(q, s4), cmul(q, s8), cmul(q, s12)};
#pragma unroll
                            for (int v4 = 0; v4 < 4; ++v4) {
                                const int r = r0 + 16 * u + 4 * v4;
                                const float2 ex = qv[v4];
                                const float2 val = (kok && ix_base + r < nx) ? make_float2(ex.x, -ex.y)
                                                                             : make_float2(0.f, 0.f);
                                store(hs + r * NCA_KCP + kk, val);
                            }
                            q = cmul(q, s16);
                        }
                    }
                }
                __syncthreads();
                const int grow = 16 * wave + (lane & 15);   // A row (image row in the tile)
                if constexpr (ENC == 0) {
                    // K-steps of 2 samples (4 real k): lane k' = 4 s + h ->
                    // sample 2 s + h / 2, part a = h & 1.
#pragma unroll 4
                    for (int s = 0; s < NCA_KC / 2; ++s) {
                        const int kk = 2 * s + (h >> 1), a = h & 1;
                        const uint2 gv = gs[grow * NCA_KCP + kk];
                        const float av = __uint_as_float(a ? gv.y : gv.x);
#pragma unroll
                        for (int cb = 0; cb < 4; ++cb) {
                            const int col = 8 * cb + ((lane & 15) >> 1);
                            const uint2 hv = hs[col * NCA_KCP + kk];
                            const float hr = __uint_as_float(hv.x), hi = __uint_as_float(hv.y);
                            const float bv = a == 0 ? (b == 0 ? hr : hi) : (b == 0 ? -hi : hr);
                            cacc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, cacc[cb], 0, 0, 0);
                        }
                    }
                } else {
                    // K-steps of 16 samples: lane's samples 16 s + 4 h + m.
#pragma unroll
                    for (int s = 0; s < NCA_KC / 16; ++s) {
                        const uint2* gp = gs + grow * NCA_KCP + 16 * s + 4 * h;
                        const uint2 g0 = gp[0], g1 = gp[1], g2 = gp[2], g3 = gp[3];
                        const uint4 ah = make_uint4(g0.x, g1.x, g2.x, g3.x);
                        const uint4 al = make_uint4(g0.y, g1.y, g2.y, g3.y);
#pragma unroll
                        for (int cb = 0; cb < 4; ++cb) {
                            const int col = 8 * cb + ((lane & 15) >> 1);
                            const uint2* hp = hs + col * NCA_KCP + 16 * s + 4 * h;
                            const uint2 q0 = hp[0], q1 = hp[1], q2 = hp[2], q3 = hp[3];
                            const uint4 bh = bform(make_uint4(q0.x, q1.x, q2.x, q3.x), b);
                            const uint4 bl = bform(make_uint4(q0.y, q1.y, q2.y, q3.y), b);
                            cacc[cb] = mma_bf16(ah, bh, cacc[cb]);
                            cacc[cb] = mma_bf16(ah, bl, cacc[cb]);
                            cacc[cb] = mma_bf16(al, bh, cacc[cb]);
                        }
                    }
                }
            }
            // Coil weight conj(C_c[j]) per voxel (1 without coils).
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float own = cacc[cb][i];
                    const float oth = __shfl_xor(own, 1);
                    if (coil == nullptr) {
                        vacc[cb][i] += own;
                    } else {
                        const float vr = b == 0 ? own : oth, vi = b == 0 ? oth : own;
                        const int iy = iy_base + 16 * wave + 4 * h + i;
                        const int ix = ix_base + 8 * cb + ((lane & 15) >> 1);
                        float2 cc = make_float2(0.f, 0.f);
                        if (iy < ny && ix < nx) cc = coil[(size_t)c * nv + (size_t)iy * nx + ix];
                        // conj(cc) * (vr + i vi)
                        vacc[cb][i] += b == 0 ? cc.x * vr + cc.y * vi : cc.x * vi - cc.y * vr;
                    }
                }
        }
        // A_p += mu_p[n, j] V[j] (the lane's part of V).
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int iy = iy_base + 16 * wave + 4 * h + i;
                const int ix = ix_base + 8 * cb + ((lane & 15) >> 1);
                if (iy < ny && ix < nx) {
                    const size_t j = (size_t)iy * nx + ix;
#pragma unroll
                    for (int p = 0; p < NTR; ++p)
                        aacc[cb][i][p] = fmaf(ld_train(trains + p * plane + (size_t)n * nv + j), vacc[cb][i],
                                              aacc[cb][i][p]);
                }
            }
    }
    const int planes = NTR == 1 ? 2 : 8;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int iy = iy_base + 16 * wave + 4 * h + i;
            const int ix = ix_base + 8 * cb + ((lane & 15) >> 1);
            if (iy < ny && ix < nx) {
                const size_t j = (size_t)iy * nx + ix;
                const bool on = mask == nullptr || mask[j] != 0;
                float* dst = apart + (size_t)chunk * planes * nv + j;
#pragma unroll
                for (int p = 0; p < NTR; ++p) dst[(size_t)(2 * p + b) * nv] = on ? aacc[cb][i][p] : 0.f;
            }
        }
}

template <typename TT, bool SPLIT>
hipError_t x_launch(const Dims& d, int mode_y, const TT* trains, const float* theta, const float* v,
                    const uint8_t* mask, float2* X, hipStream_t s)
{
    const unsigned blocks = (unsigned)std::min<size_t>(((size_t)d.T * d.nv + 255) / 256, 8192);
    switch (mode_y) {
    case 0: nc_x_kernel<1, TT, SPLIT><<<blocks, 256, 0, s>>>(trains, theta, v, mask, X, d.nv, d.T); break;
    case 1: nc_x_kernel<4, TT, SPLIT><<<blocks, 256, 0, s>>>(trains, theta, v, mask, X, d.nv, d.T); break;
    case 3: nc_x_kernel<3, TT, SPLIT><<<blocks, 256, 0, s>>>(trains, theta, v, mask, X, d.nv, d.T); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int ENC, int MODE, bool PRE>
hipError_t fwd_launch(const Dims& d, const float2* X, const float2* coil, const double* ax, const double* ay,
                      const float2* data, float2* out, double* red, int* nred, hipStream_t s)
{
    const int KT = ceil_div(d.nk, 64);
    // LDS row stride: one K part's columns and two entries of padding, which
    // put the 8 rows that one B operand read touches in different banks; rows
    // stay 16-byte aligned.
    const int nxp = std::min(ceil_div(d.nx, 16) * 16, NC_PCOLS) + 2;
    const dim3 grid(8 * KT * ceil_div(d.T, 8), d.C);
    const size_t lds = (ENC == 1 ? 2 * (size_t)NC_ROWS * nxp + 1 : (size_t)NC_ROWS * nxp) * 8;
    nc_fwd_kernel<ENC, MODE, PRE><<<grid, 256, lds, s>>>(X, coil, ax, ay, data, out, red, d.nx, d.ny, d.nv, d.T,
                                                         d.nk, KT, nxp);
    if (nred) *nred = (int)(grid.x * grid.y);
    return hipGetLastError();
}

template <int ENC, bool PRE>
hipError_t fwd_mode(const Dims& d, int mode_x, const float2* X, const float2* coil, const double* ax,
                    const double* ay, const float2* data, float2* out, double* red, int* nred, hipStream_t s)
{
    if (mode_x == 0) return fwd_launch<ENC, 0, PRE>(d, X, coil, ax, ay, data, out, red, nred, s);
    if (mode_x == 1) return fwd_launch<ENC, 1, PRE>(d, X, coil, ax, ay, data, out, red, nred, s);
    return fwd_launch<ENC, 2, PRE>(d, X, coil, ax, ay, data, out, red, nred, s);
}

template <int ENC, typename TT>
hipError_t adj_typed(const Dims& d, int ntr, int chunks, const TT* trains, const float2* coil,
                     const uint8_t* mask, const double* ax, const double* ay, const float2* w, float* apart,
                     hipStream_t s)
{
    // Exactly `chunks` chunks (the count the gradient assembly sums), each
    // holding at least one TR.
    const int per = ceil_div(d.T, chunks);
    const int nch = ceil_div(d.T, per);
    if (chunks < 1 || nch != chunks) return hipErrorInvalidValue;
    const int ntx = ceil_div(d.nx, NCA_TX);
    const dim3 grid(ntx * ceil_div(d.ny, NCA_TY), nch);
#define NC_ADJ(NT) nc_adj_kernel<ENC, NT, TT><<<grid, 256, 0, s>>>(trains, coil, mask, ax, ay, w, apart, d.nx, \
                                                                  d.ny, d.nv, d.T, d.nk, d.C, per, ntx)
    if (ntr == 1)
        NC_ADJ(1);
    else if (ntr == 3)
        NC_ADJ(3);
    else
        NC_ADJ(4);
#undef NC_ADJ
    return hipGetLastError();
}

}  // namespace

int nc_adj_chunks(const Dims& d)
{
    // Enough blocks to fill the chip at least twice with partial sums kept
    // modest (chunks x 8 floats per voxel).
    const int tiles = ceil_div(d.nx, NCA_TX) * ceil_div(d.ny, NCA_TY);
    int ch = std::max(1, ceil_div(512, tiles));
    ch = std::min(ch, 32);
    return std::min(ch, d.T);
}

int nc_fwd_blocks(const Dims& d) { return 8 * ceil_div(d.nk, 64) * ceil_div(d.T, 8) * d.C; }

hipError_t launch_nc_fwd(const Dims& d, int enc, int mode_y, int mode_x, const void* trains, bool f16,
                         const float* theta, const float* v, const float2* coil, const uint8_t* mask,
                         const double* ax, const double* ay, float2* X, const float2* data, float2* out,
                         double* red, int* nred, hipStream_t s)
{
    if (d.nx > 256) return hipErrorInvalidValue;
    // The split-BF16 forward without coil weights takes the values split once.
    const bool pre = enc == 1 && coil == nullptr;
    hipError_t e;
    if (f16) {
        const _Float16* tr = static_cast<const _Float16*>(trains);
        e = pre ? x_launch<_Float16, true>(d, mode_y, tr, theta, v, mask, X, s)
                : x_launch<_Float16, false>(d, mode_y, tr, theta, v, mask, X, s);
    } else {
        const float* tr = static_cast<const float*>(trains);
        e = pre ? x_launch<float, true>(d, mode_y, tr, theta, v, mask, X, s)
                : x_launch<float, false>(d, mode_y, tr, theta, v, mask, X, s);
    }
    if (e != hipSuccess) return e;
    if (enc == 0) return fwd_mode<0, false>(d, mode_x, X, coil, ax, ay, data, out, red, nred, s);
    return pre ? fwd_mode<1, true>(d, mode_x, X, coil, ax, ay, data, out, red, nred, s)
               : fwd_mode<1, false>(d, mode_x, X, coil, ax, ay, data, out, red, nred, s);
}

hipError_t launch_nc_adj(const Dims& d, int enc, int ntr, int chunks, const void* trains, bool f16,
                         const float2* coil, const uint8_t* mask, const double* ax, const double* ay,
                         const float2* w, float* apart, hipStream_t s)
{
    if (enc == 0)
        return f16 ? adj_typed<0>(d, ntr, chunks, static_cast<const _Float16*>(trains), coil, mask, ax, ay, w,
                                  apart, s)
                   : adj_typed<0>(d, ntr, chunks, static_cast<const float*>(trains), coil, mask, ax, ay, w, apart, s);
    return f16 ? adj_typed<1>(d, ntr, chunks, static_cast<const _Float16*>(trains), coil, mask, ax, ay, w, apart, s)
               : adj_typed<1>(d, ntr, chunks, static_cast<const float*>(trains), coil, mask, ax, ay, w, apart, s);
}

}  // namespace mrstat
