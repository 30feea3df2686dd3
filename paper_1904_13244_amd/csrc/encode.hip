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
// (D_q = d(rho m)/d alpha_q, the Jacobian columns of the Theory section).
#include "mrstat_internal.h"

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

// ------------------------------------------------------------------------
// Forward y-stage. Block = 4 waves; lane -> ix, wave -> YROWS rows; grid
// (ix tiles, iy blocks, TR chunks). Each thread keeps its voxels' weights in
// registers for the whole TR chunk; per TR the 4 waves' column sums are
// combined through LDS in batches of NB TRs.
// ------------------------------------------------------------------------
constexpr int NB = 4;
constexpr int CMAX = 16;

template <int MODE, int CC>   // CC = coils known at compile time (1), or 0 = runtime
__global__ __launch_bounds__(256) void ystage_fwd_kernel(
    const float* __restrict__ trains, const float* __restrict__ theta, const float* __restrict__ v,
    const float2* __restrict__ coil, const uint8_t* __restrict__ mask,
    const float2* __restrict__ eytab, float2* __restrict__ upart, int nx, int ny, int nv, int T,
    int C, int n_per_chunk)
{
    extern __shared__ float2 lds[];   // [NB][C][YWAVES][64]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ix = blockIdx.x * YLANES + lane;
    const int yb = blockIdx.y;
    const int iyw = yb * YBLOCK + wave * YROWS;
    const int n0 = blockIdx.z * n_per_chunk;
    const int n1 = min(T, n0 + n_per_chunk);
    const int nc = (CC > 0) ? CC : C;
    const bool colok = ix < nx;
    const size_t plane = (size_t)T * nv;

    float2 P[YROWS], Q[YROWS];
    float v0[YROWS], v1[YROWS], v2[YROWS];
#pragma unroll
    for (int r = 0; r < YROWS; ++r) {
        const int iy = iyw + r;
        const bool ok = colok && iy < ny;
        const int j = ok ? iy * nx + ix : 0;
        const bool on = ok && (mask == nullptr || mask[j] != 0);
        const float rr = on ? theta[3 * nv + j] : 0.f, ri = on ? theta[4 * nv + j] : 0.f;
        P[r] = make_float2(-ri, rr);   // i rho
        if constexpr (MODE == 1) {
            const float nr = on ? v[3 * nv + j] : 0.f, ni = on ? v[4 * nv + j] : 0.f;
            Q[r] = make_float2(-ni, nr);   // i nu
            v0[r] = on ? v[j] : 0.f;
            v1[r] = on ? v[nv + j] : 0.f;
            v2[r] = on ? v[2 * nv + j] : 0.f;
        }
    }

    for (int nb0 = n0; nb0 < n1; nb0 += NB) {
        const int nbn = min(NB, n1 - nb0);
        for (int b = 0; b < nbn; ++b) {
            const int n = nb0 + b;
            float2 acc[(CC > 0) ? CC : CMAX];
#pragma unroll
            for (int c = 0; c < ((CC > 0) ? CC : CMAX); ++c) acc[c] = make_float2(0.f, 0.f);
            const float* t0 = trains + (size_t)n * nv;
#pragma unroll
            for (int r = 0; r < YROWS; ++r) {
                const int iy = iyw + r;
                if (iy >= ny) break;
                const int j = iy * nx + ix;
                const float2 ey = eytab[(size_t)n * ny + iy];
                float2 x;
                const float mu = colok ? t0[j] : 0.f;
                if constexpr (MODE == 0) {
                    x = make_float2(P[r].x * mu, P[r].y * mu);
                } else {
                    const float m1 = colok ? t0[plane + j] : 0.f;
                    const float m2 = colok ? t0[2 * plane + j] : 0.f;
                    const float m3 = colok ? t0[3 * plane + j] : 0.f;
                    const float a = fmaf(v0[r], m1, fmaf(v1[r], m2, v2[r] * m3));
                    x = make_float2(fmaf(P[r].x, a, Q[r].x * mu), fmaf(P[r].y, a, Q[r].y * mu));
                }
                const float2 zz = cmul(ey, x);
                if constexpr (CC == 1) {
                    acc[0].x += zz.x;
                    acc[0].y += zz.y;
                } else {
                    for (int c = 0; c < nc; ++c) {
                        const float2 cw = colok ? coil[(size_t)c * nv + j] : make_float2(0.f, 0.f);
                        acc[c] = cfma(cw, zz, acc[c]);
                    }
                }
            }
            for (int c = 0; c < nc; ++c)
                lds[((b * nc + c) * YWAVES + wave) * YLANES + lane] = acc[c];
        }
        __syncthreads();
        const int nout = nbn * nc * YLANES;
        for (int o = threadIdx.x; o < nout; o += blockDim.x) {
            const int l = o % YLANES;
            const int bc = o / YLANES;   // b * nc + c
            float2 s = lds[(bc * YWAVES + 0) * YLANES + l];
#pragma unroll
            for (int w = 1; w < YWAVES; ++w) {
                const float2 t = lds[(bc * YWAVES + w) * YLANES + l];
                s.x += t.x;
                s.y += t.y;
            }
            const int b = bc / nc, c = bc % nc;
            const int oix = blockIdx.x * YLANES + l;
            if (oix < nx)
                upart[(((size_t)yb * nc + c) * T + (nb0 + b)) * nx + oix] = s;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------
// Adjoint y-stage: A_p[j] = sum_n mu_p[n,j] V[n,j],
// V[n,j] = conj(Ey[n,iy]) sum_c conj(C_c[j]) W_c[n,ix], summed over the TRs of
// one chunk (partials per chunk, combined in chunk order by the finish kernel).
// ------------------------------------------------------------------------
template <int NTRAIN, int CC>
__global__ __launch_bounds__(256) void ystage_adj_kernel(
    const float* __restrict__ trains, const float2* __restrict__ coil,
    const uint8_t* __restrict__ mask, const float2* __restrict__ eytab,
    const float2* __restrict__ W, float* __restrict__ apart, int nx, int ny, int nv, int T, int C,
    int n_per_chunk)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ix = blockIdx.x * YLANES + lane;
    const int iyw = blockIdx.y * YBLOCK + wave * YROWS;
    const int chunk = blockIdx.z;
    const int n0 = chunk * n_per_chunk;
    const int n1 = min(T, n0 + n_per_chunk);
    const bool colok = ix < nx;
    const size_t plane = (size_t)T * nv;
    const int nc = (CC > 0) ? CC : C;

    float2 acc[YROWS][NTRAIN];
#pragma unroll
    for (int r = 0; r < YROWS; ++r)
#pragma unroll
        for (int p = 0; p < NTRAIN; ++p) acc[r][p] = make_float2(0.f, 0.f);

    for (int n = n0; n < n1; ++n) {
        float2 w1 = make_float2(0.f, 0.f);
        if constexpr (CC == 1) w1 = colok ? W[(size_t)n * nx + ix] : make_float2(0.f, 0.f);
        const float* t0 = trains + (size_t)n * nv;
#pragma unroll
        for (int r = 0; r < YROWS; ++r) {
            const int iy = iyw + r;
            if (iy >= ny) break;
            const int j = iy * nx + ix;
            float2 wc;
            if constexpr (CC == 1) {
                wc = w1;
            } else {
                wc = make_float2(0.f, 0.f);
                for (int c = 0; c < nc; ++c) {
                    const float2 cw = colok ? coil[(size_t)c * nv + j] : make_float2(0.f, 0.f);
                    const float2 wv = colok ? W[((size_t)c * T + n) * nx + ix] : make_float2(0.f, 0.f);
                    const float2 t = cmulconj(cw, wv);
                    wc.x += t.x;
                    wc.y += t.y;
                }
            }
            const float2 V = cmulconj(eytab[(size_t)n * ny + iy], wc);
#pragma unroll
            for (int p = 0; p < NTRAIN; ++p) {
                const float mu = colok ? t0[p * plane + j] : 0.f;
                acc[r][p].x = fmaf(mu, V.x, acc[r][p].x);
                acc[r][p].y = fmaf(mu, V.y, acc[r][p].y);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < YROWS; ++r) {
        const int iy = iyw + r;
        if (!colok || iy >= ny) continue;
        const int j = iy * nx + ix;
        const bool on = mask == nullptr || mask[j] != 0;
        float* dst = apart + (size_t)chunk * 2 * NTRAIN * nv + j;
#pragma unroll
        for (int p = 0; p < NTRAIN; ++p) {
            dst[(2 * p) * (size_t)nv] = on ? acc[r][p].x : 0.f;
            dst[(2 * p + 1) * (size_t)nv] = on ? acc[r][p].y : 0.f;
        }
    }
}

// g from A: g_q = -Im(conj(rho) A_{q+1}) for q = lnT1, lnT2, B1;
// g_3 = -Im(A_0) (Re rho), g_4 = Re(A_0) (Im rho).
__global__ void jhw_finish_kernel(const float* __restrict__ apart, int n_chunk,
                                  const float* __restrict__ theta,
                                  const uint8_t* __restrict__ mask, float* __restrict__ g, int nv)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nv) return;
    float A[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) A[q] = 0.f;
    for (int ch = 0; ch < n_chunk; ++ch)
#pragma unroll
        for (int q = 0; q < 8; ++q) A[q] += apart[((size_t)ch * 8 + q) * nv + j];
    const bool on = mask == nullptr || mask[j] != 0;
    const float rr = theta[3 * nv + j], ri = theta[4 * nv + j];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const float ar = A[2 * (q + 1)], ai = A[2 * (q + 1) + 1];
        g[(size_t)q * nv + j] = on ? -(rr * ai - ri * ar) : 0.f;
    }
    g[3 * (size_t)nv + j] = on ? -A[1] : 0.f;
    g[4 * (size_t)nv + j] = on ? A[0] : 0.f;
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
// K in chunks of 32 staged through LDS (A rows, B phase tile).
// MFMA 16x16x4 f32 operand layout: A lane l -> (row l%16, k l/16),
// B lane l -> (k l/16, col l%16), D lane l -> (rows 4(l/16)+i, col l%16).
// ------------------------------------------------------------------------
constexpr int GBM = 64, GBN = 64, GBK = 32;

template <int DIR, int MODE>   // DIR 0 forward, 1 adjoint; MODE (forward): 0 residual, 1 -s, 2 +s
__global__ __launch_bounds__(256) void xgemm_f32_kernel(
    const float2* __restrict__ Ain, int nby, const float2* __restrict__ extab,
    const float2* __restrict__ data, float2* __restrict__ out, double* __restrict__ red, int M,
    int nx, int nk, int upart_stride)
{
    __shared__ float As[GBM][GBK + 1];
    __shared__ float Bs[GBK][GBN + 1];
    __shared__ double rs[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = blockIdx.y * GBM, c0 = blockIdx.x * GBN;
    const int Kr = DIR == 0 ? 2 * nx : 2 * nk;    // real reduction length
    const int Nr = DIR == 0 ? 2 * nk : 2 * nx;    // real output columns
    const int Ka = DIR == 0 ? nx : nk;            // complex A columns

    f4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < Kr; k0 += GBK) {
        // A tile: 64 rows x 16 complex columns (sum of the y-stage partials
        // for the forward direction).
        for (int e = tid; e < GBM * (GBK / 2); e += 256) {
            const int r = e / (GBK / 2), cc = e % (GBK / 2);
            const int m = m0 + r, kc = k0 / 2 + cc;
            float2 a = make_float2(0.f, 0.f);
            if (m < M && kc < Ka) {
                if (DIR == 0) {
                    for (int b = 0; b < nby; ++b) {
                        const float2 t = Ain[(size_t)b * upart_stride + (size_t)m * nx + kc];
                        a.x += t.x;
                        a.y += t.y;
                    }
                } else {
                    a = Ain[(size_t)m * nk + kc];
                }
            }
            As[r][2 * cc] = a.x;
            As[r][2 * cc + 1] = a.y;
        }
        // B tile: 16 complex rows x 32 complex columns of 2x2 phase blocks.
        for (int e = tid; e < (GBK / 2) * (GBN / 2); e += 256) {
            // Consecutive threads read consecutive ix of the phase table.
            const int rr = DIR == 0 ? e % (GBK / 2) : e / (GBN / 2);
            const int cc = DIR == 0 ? e / (GBK / 2) : e % (GBN / 2);
            const int kr = k0 / 2 + rr, kc = c0 / 2 + cc;
            float2 E = make_float2(0.f, 0.f);
            if (DIR == 0) {   // rows ix, columns k
                if (kr < nx && kc < nk) E = extab[(size_t)kc * nx + kr];
                Bs[2 * rr][2 * cc] = E.x;
                Bs[2 * rr][2 * cc + 1] = E.y;
                Bs[2 * rr + 1][2 * cc] = -E.y;
                Bs[2 * rr + 1][2 * cc + 1] = E.x;
            } else {          // rows k, columns ix
                if (kr < nk && kc < nx) E = extab[(size_t)kr * nx + kc];
                Bs[2 * rr][2 * cc] = E.x;
                Bs[2 * rr][2 * cc + 1] = -E.y;
                Bs[2 * rr + 1][2 * cc] = E.y;
                Bs[2 * rr + 1][2 * cc + 1] = E.x;
            }
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GBK; kk += 4) {
            float av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = As[wm * 32 + a * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[b] = Bs[kk + (lane >> 4)][wn * 32 + b * 16 + (lane & 15)];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }

    // Epilogue.
    double sq = 0.0;
    float* o = reinterpret_cast<float*>(out);
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

}  // namespace

hipError_t launch_ystage_fwd(const Dims& d, int mode, const float* trains, const float* theta,
                             const float* v, const float2* coil, const uint8_t* mask,
                             const float2* eytab, float2* upart, int n_chunk, hipStream_t s)
{
    dim3 grid(ceil_div(d.nx, YLANES), ceil_div(d.ny, YBLOCK), ceil_div(d.T, n_chunk));
    const size_t lds = (size_t)NB * d.C * YWAVES * YLANES * sizeof(float2);
    if (d.C > CMAX) return hipErrorInvalidValue;
    if (d.C == 1) {
        if (mode == 0)
            ystage_fwd_kernel<0, 1><<<grid, 256, lds, s>>>(trains, theta, v, coil, mask, eytab, upart,
                                                          d.nx, d.ny, d.nv, d.T, 1, n_chunk);
        else
            ystage_fwd_kernel<1, 1><<<grid, 256, lds, s>>>(trains, theta, v, coil, mask, eytab, upart,
                                                          d.nx, d.ny, d.nv, d.T, 1, n_chunk);
    } else {
        if (mode == 0)
            ystage_fwd_kernel<0, 0><<<grid, 256, lds, s>>>(trains, theta, v, coil, mask, eytab, upart,
                                                          d.nx, d.ny, d.nv, d.T, d.C, n_chunk);
        else
            ystage_fwd_kernel<1, 0><<<grid, 256, lds, s>>>(trains, theta, v, coil, mask, eytab, upart,
                                                          d.nx, d.ny, d.nv, d.T, d.C, n_chunk);
    }
    return hipGetLastError();
}

hipError_t launch_xgemm_fwd(const Dims& d, int enc, int mode, const float2* upart, int nby,
                            const float2* extab, const float2* data, float2* out, double* red,
                            int* nred, hipStream_t s)
{
    (void)enc;
    const int M = d.C * d.T;
    dim3 grid(ceil_div(2 * d.nk, GBN), ceil_div(M, GBM));
    if (nred) *nred = grid.x * grid.y;
    const int stride = M * d.nx;
    if (mode == 0)
        xgemm_f32_kernel<0, 0><<<grid, 256, 0, s>>>(upart, nby, extab, data, out, red, M, d.nx, d.nk,
                                                    stride);
    else if (mode == 1)
        xgemm_f32_kernel<0, 1><<<grid, 256, 0, s>>>(upart, nby, extab, data, out, red, M, d.nx, d.nk,
                                                    stride);
    else
        xgemm_f32_kernel<0, 2><<<grid, 256, 0, s>>>(upart, nby, extab, data, out, red, M, d.nx, d.nk,
                                                    stride);
    return hipGetLastError();
}

hipError_t launch_xgemm_adj(const Dims& d, int enc, const float2* w, const float2* extab,
                            float2* W, hipStream_t s)
{
    (void)enc;
    const int M = d.C * d.T;
    dim3 grid(ceil_div(2 * d.nx, GBN), ceil_div(M, GBM));
    xgemm_f32_kernel<1, 0><<<grid, 256, 0, s>>>(w, 1, extab, nullptr, W, nullptr, M, d.nx, d.nk, 0);
    return hipGetLastError();
}

hipError_t launch_ystage_adj(const Dims& d, const float* trains, int ntr_trains,
                             const float2* coil, const uint8_t* mask, const float2* eytab,
                             const float2* W, float* apart, int n_chunk, hipStream_t s)
{
    dim3 grid(ceil_div(d.nx, YLANES), ceil_div(d.ny, YBLOCK), ceil_div(d.T, n_chunk));
    if (d.C > CMAX) return hipErrorInvalidValue;
    if (ntr_trains == 4) {
        if (d.C == 1)
            ystage_adj_kernel<4, 1><<<grid, 256, 0, s>>>(trains, coil, mask, eytab, W, apart, d.nx, d.ny,
                                                       d.nv, d.T, 1, n_chunk);
        else
            ystage_adj_kernel<4, 0><<<grid, 256, 0, s>>>(trains, coil, mask, eytab, W, apart, d.nx, d.ny,
                                                       d.nv, d.T, d.C, n_chunk);
    } else {
        if (d.C == 1)
            ystage_adj_kernel<1, 1><<<grid, 256, 0, s>>>(trains, coil, mask, eytab, W, apart, d.nx, d.ny,
                                                       d.nv, d.T, 1, n_chunk);
        else
            ystage_adj_kernel<1, 0><<<grid, 256, 0, s>>>(trains, coil, mask, eytab, W, apart, d.nx, d.ny,
                                                       d.nv, d.T, d.C, n_chunk);
    }
    return hipGetLastError();
}

hipError_t launch_jhw_finish(const Dims& d, const float* apart, int n_chunk, const float* theta,
                             const uint8_t* mask, float* g, hipStream_t s)
{
    jhw_finish_kernel<<<ceil_div(d.nv, 256), 256, 0, s>>>(apart, n_chunk, theta, mask, g, d.nv);
    return hipGetLastError();
}

hipError_t launch_rho_adj_finish(const Dims& d, const float* apart, int n_chunk,
                                 const uint8_t* mask, float2* out, hipStream_t s)
{
    rho_adj_finish_kernel<<<ceil_div(d.nv, 256), 256, 0, s>>>(apart, n_chunk, mask, out, d.nv);
    return hipGetLastError();
}

}  // namespace mrstat
