// Surrogate network kernels: a small MLP maps (ln T1, ln T2, B1) to the four
// trains (m, dm/dlnT1, dm/dlnT2, dm/dB1) over all TRs, trained on EPG output
// with BF16 operands on the matrix cores and FP32 accumulation, FP32 master
// weights and Adam.
//
// Layout: activations are feature-major, sample-fastest ([features][samples]),
// so the output layer writes the trains' [train][TR][voxel] layout directly.
// Output o = c 4T + p T + n (c 0 real, 1 imaginary; p the train; n the TR),
// scaled by 1 / s_p. Hidden layers use the exact GELU z Phi(z).
// Parameters (FP32, packed): W1 [width][3], b1, (W [width][width], b) for each
// further hidden layer, Wout [8T][width], bout.
#include "mrstat_internal.h"
#include "mlp_internal.h"

#include <type_traits>

namespace mrstat {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t to_bf16(float x)
{
    const uint32_t u = __float_as_uint(x);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ float gelu(float z)
{
    return 0.5f * z * (1.f + erff(z * 0.70710678118654752f));
}

__device__ __forceinline__ float gelu_grad(float z)
{
    return 0.5f * (1.f + erff(z * 0.70710678118654752f)) +
           z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// ------------------------------------------------------------------------
// BF16 GEMM C[M][N] = A[M][K] B[K][N] on v_mfma_f32_16x16x32_bf16 with FP32
// accumulation. A is row-major [M][K] (TA false) or stored [K][M] (TA true);
// B is row-major [K][N] (TB false) or stored [N][K] (TB true). Tiles of
// 64 x 64, K in chunks of 32 double-buffered in LDS, where A is kept
// [m][k] and B [n][k] so each lane's 8-element fragment is one 128-bit read.
// Requirements (checked on the host): K, M (when TA), N (when !TB) and the
// leading dimensions are multiples of 8; 16-byte aligned bases.
// ------------------------------------------------------------------------
constexpr int TM = 64, TN = 64, TK = 32, KP = 8;

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[2][TM][TK + KP];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][TN][TK + KP];
    __shared__ double rs[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    const int nchunk = (g.K + TK - 1) / TK;

    uint4 ra, rb;
    auto load8 = [&](const uint16_t* base, int64_t idx, bool ok) -> uint4 {
        return ok ? *reinterpret_cast<const uint4*>(base + idx) : make_uint4(0, 0, 0, 0);
    };
    auto gload = [&](int kc) {
        const int k0 = kc * TK;
        if (!TA) {   // row m = tid/4, k group 8(tid%4)
            const int r = tid >> 2, kg = (tid & 3) * 8;
            ra = load8(g.A, (int64_t)(m0 + r) * g.lda + k0 + kg, m0 + r < g.M && k0 + kg < g.K);
        } else {     // k = tid/8, m group 8(tid%8)
            const int k = tid >> 3, mg = (tid & 7) * 8;
            ra = load8(g.A, (int64_t)(k0 + k) * g.lda + m0 + mg, k0 + k < g.K && m0 + mg < g.M);
        }
        if (TB) {    // n = tid/4, k group
            const int r = tid >> 2, kg = (tid & 3) * 8;
            rb = load8(g.B, (int64_t)(n0 + r) * g.ldb + k0 + kg, n0 + r < g.N && k0 + kg < g.K);
        } else {     // k = tid/8, n group
            const int k = tid >> 3, ng = (tid & 7) * 8;
            rb = load8(g.B, (int64_t)(k0 + k) * g.ldb + n0 + ng, k0 + k < g.K && n0 + ng < g.N);
        }
    };
    auto sstore = [&](int buf) {
        if (!TA) {
            const int r = tid >> 2, kg = (tid & 3) * 8;
            *reinterpret_cast<uint4*>(&As[buf][r][kg]) = ra;
        } else {
            const int k = tid >> 3, mg = (tid & 7) * 8;
            const uint16_t* v = reinterpret_cast<const uint16_t*>(&ra);
#pragma unroll
            for (int i = 0; i < 8; ++i) As[buf][mg + i][k] = v[i];
        }
        if (TB) {
            const int r = tid >> 2, kg = (tid & 3) * 8;
            *reinterpret_cast<uint4*>(&Bs[buf][r][kg]) = rb;
        } else {
            const int k = tid >> 3, ng = (tid & 7) * 8;
            const uint16_t* v = reinterpret_cast<const uint16_t*>(&rb);
#pragma unroll
            for (int i = 0; i < 8; ++i) Bs[buf][ng + i][k] = v[i];
        }
    };

    f4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};

    if (nchunk > 0) {
        gload(0);
        sstore(0);
    }
    __syncthreads();
    const int kq = 8 * (lane >> 4);
    for (int kc = 0; kc < nchunk; ++kc) {
        const int buf = kc & 1;
        const bool more = kc + 1 < nchunk;
        if (more) gload(kc + 1);
        uint4 af[2], bf[2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
            af[a] = *reinterpret_cast<const uint4*>(&As[buf][wm * 32 + a * 16 + (lane & 15)][kq]);
#pragma unroll
        for (int b = 0; b < 2; ++b)
            bf[b] = *reinterpret_cast<const uint4*>(&Bs[buf][wn * 32 + b * 16 + (lane & 15)][kq]);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    __builtin_bit_cast(bf16x8, af[a]), __builtin_bit_cast(bf16x8, bf[b]), acc[a][b],
                    0, 0, 0);
        if (more) sstore(buf ^ 1);
        __syncthreads();
    }

    double lsum = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = m0 + wm * 32 + a * 16 + 4 * (lane >> 4) + i;
                const int n = n0 + wn * 32 + b * 16 + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                const float v = acc[a][b][i];
                const int64_t o = (int64_t)m * g.ldo + n;
                if constexpr (EPI == EPI_STORE_F32) {
                    g.Cf[o] = v;
                } else if constexpr (EPI == EPI_BIAS_GELU) {
                    const float z = v + g.bias[m];
                    if (g.Zb) g.Zb[o] = to_bf16(z);
                    g.Hb[o] = to_bf16(gelu(z));
                } else if constexpr (EPI == EPI_OUT_LOSS) {
                    const float y = v + g.bias[m];
                    const int T = g.T, c = m / (4 * T), p = (m % (4 * T)) / T, nt = m % T;
                    const float t = c ? g.target[((int64_t)p * T + nt) * g.ld_t + n] / g.head_scale[p] : 0.f;
                    const float d = y - t;
                    g.Hb[o] = to_bf16(g.grad_scale * d);
                    lsum += (double)d * (double)d;
                } else if constexpr (EPI == EPI_GELU_BWD) {
                    g.Hb[o] = to_bf16(v * gelu_grad(from_bf16(g.Zin[o])));
                } else {   // EPI_INFER: rows are the imaginary outputs of trains p = m / T
                    const float y = v + g.bias[m];
                    const int p = m / g.T, nt = m % g.T;
                    g.Cf[(int64_t)p * g.plane + (int64_t)nt * g.ldo + n] = y * g.head_scale[p];
                }
            }
    if constexpr (EPI == EPI_OUT_LOSS) {
        for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off);
        if (lane == 0) rs[wave] = lsum;
        __syncthreads();
        if (tid == 0) g.loss_part[blockIdx.y * gridDim.x + blockIdx.x] = (rs[0] + rs[1]) + (rs[2] + rs[3]);
    }
}

// First layer (3 inputs): x normalised onto [-1, 1] over the box, z = W1 x + b1.
// x_in rows (ln T1, ln T2, B1) with leading dimension ldx; out [width][ldo].
// blockIdx.y selects a group of 32 units.
__global__ void layer1_fwd_kernel(const float* __restrict__ x_in, int64_t ldx, int n,
                                  const float* __restrict__ W1, const float* __restrict__ b1,
                                  int width, float lo0, float lo1, float lo2, float hi0, float hi1,
                                  float hi2, float* __restrict__ xs, uint16_t* __restrict__ Zb,
                                  uint16_t* __restrict__ Hb, int64_t ldo)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const float x0 = 2.f * (x_in[s] - lo0) / (hi0 - lo0) - 1.f;
    const float x1 = 2.f * (x_in[ldx + s] - lo1) / (hi1 - lo1) - 1.f;
    const float x2 = 2.f * (x_in[2 * ldx + s] - lo2) / (hi2 - lo2) - 1.f;
    if (xs && blockIdx.y == 0) {
        xs[s] = x0;
        xs[ldo + s] = x1;
        xs[2 * ldo + s] = x2;
    }
    const int o_end = min(width, (int)(blockIdx.y + 1) * 32);
    for (int o = blockIdx.y * 32; o < o_end; ++o) {
        const float z = fmaf(W1[3 * o], x0, fmaf(W1[3 * o + 1], x1, fmaf(W1[3 * o + 2], x2, b1[o])));
        if (Zb) Zb[(int64_t)o * ldo + s] = to_bf16(z);
        Hb[(int64_t)o * ldo + s] = to_bf16(gelu(z));
    }
}

// Row sums of a bf16 [rows][n] matrix (bias gradients), one block per row,
// fixed-order reduction.
__global__ __launch_bounds__(256) void rowsum_kernel(const uint16_t* __restrict__ X, int64_t ld, int n,
                                                     float* __restrict__ out)
{
    __shared__ float sh[256];
    const int r = blockIdx.x;
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) s += from_bf16(X[(int64_t)r * ld + i]);
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[r] = sh[0];
}

// dW1[o][i] = sum_s dZ1[o][s] x[i][s]: one block per output row.
__global__ __launch_bounds__(256) void layer1_wgrad_kernel(const uint16_t* __restrict__ dZ,
                                                           const float* __restrict__ xs, int64_t ld,
                                                           int n, float* __restrict__ dW1)
{
    __shared__ float sh[3][256];
    const int o = blockIdx.x;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f;
    for (int s = threadIdx.x; s < n; s += 256) {
        const float d = from_bf16(dZ[(int64_t)o * ld + s]);
        a0 = fmaf(d, xs[s], a0);
        a1 = fmaf(d, xs[ld + s], a1);
        a2 = fmaf(d, xs[2 * ld + s], a2);
    }
    sh[0][threadIdx.x] = a0;
    sh[1][threadIdx.x] = a1;
    sh[2][threadIdx.x] = a2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 3; ++q) dW1[3 * o + q] = sh[q][0];
}

// Adam on FP32 master weights; refreshes the BF16 copy.
__global__ void adam_kernel(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ gr, uint16_t* __restrict__ wb, size_t n,
                            float lr, float b1, float b2, float eps, float c1, float c2)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = gr[i];
    const float mi = fmaf(b1, m[i], (1.f - b1) * gi);
    const float vi = fmaf(b2, v[i], (1.f - b2) * gi * gi);
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    wb[i] = to_bf16(wi);
}

__global__ void to_bf16_kernel(const float* __restrict__ x, uint16_t* __restrict__ y, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = to_bf16(x[i]);
}

__device__ __forceinline__ uint32_t pack2(float a, float b)
{
    return (uint32_t)to_bf16(a) | ((uint32_t)to_bf16(b) << 16);
}

// ------------------------------------------------------------------------
// Fused inference: one workgroup (4 waves) evaluates the whole network for
// NV voxels (32 or 64). The first layer runs in FP32; each hidden layer is a
// 16x16x32 BF16 MFMA product with the weights read from L2 and the
// activations ping-ponged between two LDS buffers laid out [voxel][unit]
// (16-byte pad per row); the output layer keeps the last activations of all
// NV voxels in registers as A fragments and streams its output rows (weights
// from L2), 16 outputs per step, each wave taking every fourth 16-row tile
// (with PF, the next tile's weights are loaded while the current one is
// multiplied). Results (bias added, head scale applied) go straight to the
// train layout out[p][n][voxel] as 16-byte (F16: 8-byte) stores of 4
// consecutive voxels. Same roundings as the training forward pass:
// pre-activations in FP32, activations in BF16; trains stored as FP32 or
// rounded to FP16 (F16).
// ------------------------------------------------------------------------
typedef _Float16 h4v __attribute__((ext_vector_type(4)));

// PF: 0 = weights loaded per tile, activations (A fragments) in registers;
// 1 = two tiles of weights in flight, activations in registers; 2 / 3 = two
// / three tiles of weights in flight, activations read from LDS per tile
// (frees the registers that hold them, so more weight loads are in flight).
template <int WIDTH, int NV, int PF, bool F16>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PF >= 2 ? 2 : 1)))
void mlp_infer_kernel(InferArgs a)
{
    constexpr int HP = WIDTH + 8, KS = WIDTH / 32, MT = WIDTH / 64, VT = NV / 16;
    __shared__ __attribute__((aligned(16))) uint16_t Hs[2][NV][HP];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j0 = blockIdx.x * NV;
    const int lr = lane & 15, lk = 8 * (lane >> 4);

    // Layer 1 (3 inputs): thread -> voxel tid % NV, groups of 8 units.
    {
        constexpr int GS = 256 / NV;   // threads per voxel
        const int v = tid % NV, g0 = tid / NV;
        const int j = min(j0 + v, a.n - 1);
        const float x0 = 2.f * (a.theta[j] - a.lo[0]) / (a.hi[0] - a.lo[0]) - 1.f;
        const float x1 = 2.f * (a.theta[a.ldth + j] - a.lo[1]) / (a.hi[1] - a.lo[1]) - 1.f;
        const float x2 = 2.f * (a.theta[2 * a.ldth + j] - a.lo[2]) / (a.hi[2] - a.lo[2]) - 1.f;
        for (int g = g0; g < WIDTH / 8; g += GS) {
            float h[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int u = 8 * g + q;
                const float z = fmaf(a.W1[3 * u], x0, fmaf(a.W1[3 * u + 1], x1, fmaf(a.W1[3 * u + 2], x2, a.b1[u])));
                h[q] = gelu(z);
            }
            *reinterpret_cast<uint4*>(&Hs[0][v][8 * g]) =
                make_uint4(pack2(h[0], h[1]), pack2(h[2], h[3]), pack2(h[4], h[5]), pack2(h[6], h[7]));
        }
    }
    __syncthreads();

    // Hidden layers: wave w computes units [w WIDTH/4, (w+1) WIDTH/4) of all NV voxels.
    int cur = 0;
    for (int l = 0; l < a.n_hidden; ++l) {
        const uint16_t* __restrict__ W = a.Wh[l];
        const float* __restrict__ bias = a.bh[l];
        f4 acc[MT][VT];
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int t = 0; t < VT; ++t) acc[m][t] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
        for (int ks = 0; ks < KS; ++ks) {
            uint4 af[MT], bf[VT];
#pragma unroll
            for (int m = 0; m < MT; ++m)
                af[m] = *reinterpret_cast<const uint4*>(W + (size_t)(wave * (WIDTH / 4) + m * 16 + lr) * WIDTH +
                                                        ks * 32 + lk);
#pragma unroll
            for (int t = 0; t < VT; ++t)
                bf[t] = *reinterpret_cast<const uint4*>(&Hs[cur][t * 16 + lr][ks * 32 + lk]);
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int t = 0; t < VT; ++t)
                    acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        __builtin_bit_cast(bf16x8, af[m]), __builtin_bit_cast(bf16x8, bf[t]), acc[m][t], 0, 0, 0);
        }
        const int nxt = cur ^ 1;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int u0 = wave * (WIDTH / 4) + m * 16 + 4 * (lane >> 4);
            const float c0 = bias[u0], c1 = bias[u0 + 1], c2 = bias[u0 + 2], c3 = bias[u0 + 3];
#pragma unroll
            for (int t = 0; t < VT; ++t) {
                const f4 z = acc[m][t];
                *reinterpret_cast<uint2*>(&Hs[nxt][t * 16 + lr][u0]) =
                    make_uint2(pack2(gelu(z[0] + c0), gelu(z[1] + c1)), pack2(gelu(z[2] + c2), gelu(z[3] + c3)));
            }
        }
        __syncthreads();
        cur = nxt;
    }

    // Output layer: A = activations^T (voxel rows), in registers (PF < 3)
    // or read from LDS per tile (PF = 3).
    constexpr bool AREG = PF < 2;
    uint4 hf[AREG ? VT : 1][AREG ? KS : 1];
    if constexpr (AREG) {
#pragma unroll
        for (int t = 0; t < VT; ++t)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
                hf[t][ks] = *reinterpret_cast<const uint4*>(&Hs[cur][t * 16 + lr][ks * 32 + lk]);
    }

    const int n_tiles = (a.m_out + 15) / 16;
    const bool vec_ok = (a.ld_out % 4) == 0;
    // Weights of output tile `tile` (clamped: a tile past the end reloads
    // the last one, which is never stored).
    auto load_b = [&](uint4 (&b)[KS], int tile) {
        const int o = min(min(tile, n_tiles - 1) * 16 + lr, a.m_out - 1);
        const uint16_t* src = a.Wout + (size_t)o * WIDTH + lk;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) b[ks] = *reinterpret_cast<const uint4*>(src + ks * 32);
    };
    auto tile_out = [&](const uint4 (&b)[KS], int tile) {
        f4 acc[VT];
#pragma unroll
        for (int t = 0; t < VT; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int t = 0; t < VT; ++t) {
                uint4 af;
                if constexpr (AREG) af = hf[t][ks];
                else af = *reinterpret_cast<const uint4*>(&Hs[cur][t * 16 + lr][ks * 32 + lk]);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    __builtin_bit_cast(bf16x8, af), __builtin_bit_cast(bf16x8, b[ks]), acc[t], 0, 0, 0);
            }
        const int o = tile * 16 + lr;
        if (o < a.m_out) {
            const int p = o / a.T, nt = o - p * a.T;
            const float bias = a.bout[o], sc = a.head_scale[p];
            using OT = typename std::conditional<F16, _Float16, float>::type;
            OT* dst = static_cast<OT*>(a.out) + (size_t)p * a.plane + (size_t)nt * a.ld_out;
#pragma unroll
            for (int t = 0; t < VT; ++t) {
                const int jv = j0 + t * 16 + 4 * (lane >> 4);
                const float y0 = (acc[t][0] + bias) * sc, y1 = (acc[t][1] + bias) * sc;
                const float y2 = (acc[t][2] + bias) * sc, y3 = (acc[t][3] + bias) * sc;
                // FP32: 64-byte row pieces, streamed past the caches so the
                // output weights stay resident in L2. FP16: 32-byte pieces,
                // left to L2 to merge into whole lines (the tile's four
                // stores cover 128 bytes of each row).
                if (vec_ok && jv + 3 < a.n) {
                    if constexpr (F16)
                        *reinterpret_cast<h4v*>(dst + jv) = h4v{(_Float16)y0, (_Float16)y1, (_Float16)y2, (_Float16)y3};
                    else
                        __builtin_nontemporal_store(f4{y0, y1, y2, y3}, reinterpret_cast<f4*>(dst + jv));
                } else {
                    if (jv < a.n) dst[jv] = (OT)y0;
                    if (jv + 1 < a.n) dst[jv + 1] = (OT)y1;
                    if (jv + 2 < a.n) dst[jv + 2] = (OT)y2;
                    if (jv + 3 < a.n) dst[jv + 3] = (OT)y3;
                }
            }
        }
    };
    if constexpr (PF == 3) {
        uint4 b0[KS], b1[KS], b2[KS];
        load_b(b0, wave);
        load_b(b1, wave + 4);
        for (int tile = wave; tile < n_tiles; tile += 12) {
            load_b(b2, tile + 8);
            tile_out(b0, tile);
            if (tile + 4 >= n_tiles) break;
            load_b(b0, tile + 12);
            tile_out(b1, tile + 4);
            if (tile + 8 >= n_tiles) break;
            load_b(b1, tile + 16);
            tile_out(b2, tile + 8);
        }
    } else if constexpr (PF == 1 || PF == 2) {
        uint4 b0[KS], b1[KS];
        load_b(b0, wave);
        for (int tile = wave; tile < n_tiles; tile += 8) {
            load_b(b1, tile + 4);
            tile_out(b0, tile);
            if (tile + 4 >= n_tiles) break;
            load_b(b0, tile + 8);
            tile_out(b1, tile + 4);
        }
    } else {
        uint4 b0[KS];
        for (int tile = wave; tile < n_tiles; tile += 4) {
            load_b(b0, tile);
            tile_out(b0, tile);
        }
    }
}

// ------------------------------------------------------------------------
// Hidden layers as their own kernel (width 256): a workgroup of 8 waves takes
// a tile of NV voxels at a time. Activations of the tile live in LDS in MFMA
// B-fragment order ([16-voxel tile][K block][lane], 16 bytes per lane). For
// each hidden layer, wave w loads the layer's weights of units [32 w, 32 w
// + 32) into registers as A fragments (once per tile and layer: 128 KB per
// workgroup instead of per 32-voxel tile), multiplies them against every
// voxel of the tile with the sums in registers, and after a barrier writes
// GELU(sum + bias) back over the activations (BF16, 8-byte stores of 4 units).
// The first layer runs in FP32 from theta; the last activations go to
// a.hout as BF16 [voxel][256]. Same roundings as the fused kernel.
// ------------------------------------------------------------------------
template <int NV>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
void mlp_hidden_kernel(InferArgs a)
{
    constexpr int WIDTH = 256, KB = WIDTH / 32, VT = NV / 16;
    __shared__ uint4 Hf[VT][KB][64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = 8 * (lane >> 4);
    const int n_tiles = (a.n + NV - 1) / NV;
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int j0 = tile * NV;
        // Layer 1: thread -> (voxel v, 8 units q); one 16-byte fragment piece each.
        for (int e = tid; e < NV * (WIDTH / 8); e += 512) {
            const int v = e % NV, q = e / NV;
            const int j = min(j0 + v, a.n - 1);
            const float x0 = 2.f * (a.theta[j] - a.lo[0]) / (a.hi[0] - a.lo[0]) - 1.f;
            const float x1 = 2.f * (a.theta[a.ldth + j] - a.lo[1]) / (a.hi[1] - a.lo[1]) - 1.f;
            const float x2 = 2.f * (a.theta[2 * a.ldth + j] - a.lo[2]) / (a.hi[2] - a.lo[2]) - 1.f;
            float h[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int u = 8 * q + r;
                h[r] = gelu(fmaf(a.W1[3 * u], x0, fmaf(a.W1[3 * u + 1], x1, fmaf(a.W1[3 * u + 2], x2, a.b1[u]))));
            }
            Hf[v / 16][q / 4][(v % 16) + 16 * (q % 4)] =
                make_uint4(pack2(h[0], h[1]), pack2(h[2], h[3]), pack2(h[4], h[5]), pack2(h[6], h[7]));
        }
        __syncthreads();
        for (int l = 0; l < a.n_hidden; ++l) {
            const uint16_t* __restrict__ W = a.Wh[l];
            uint4 wf[2][KB];
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int kb = 0; kb < KB; ++kb)
                    wf[m][kb] = *reinterpret_cast<const uint4*>(W + (size_t)(32 * wave + 16 * m + lr) * WIDTH +
                                                                32 * kb + lk);
            f4 acc[2][VT];
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int vt = 0; vt < VT; ++vt) acc[m][vt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int vt = 0; vt < VT; ++vt)
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) {
                    const uint4 bf = Hf[vt][kb][lane];
#pragma unroll
                    for (int m = 0; m < 2; ++m)
                        acc[m][vt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            __builtin_bit_cast(bf16x8, wf[m][kb]), __builtin_bit_cast(bf16x8, bf), acc[m][vt], 0, 0, 0);
                }
            __syncthreads();   // every wave has read the layer's inputs
            // D: lane holds units 32 w + 16 m + 4 (lane / 16) + i of voxel lr.
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const int u0 = 32 * wave + 16 * m + 4 * (lane >> 4);
                const float c0 = a.bh[l][u0], c1 = a.bh[l][u0 + 1], c2 = a.bh[l][u0 + 2], c3 = a.bh[l][u0 + 3];
                const int kb = u0 / 32, slot = lr + 16 * ((u0 % 32) / 8), half = (u0 % 8) / 4;
#pragma unroll
                for (int vt = 0; vt < VT; ++vt) {
                    const f4 z = acc[m][vt];
                    uint2* dst = reinterpret_cast<uint2*>(&Hf[vt][kb][slot]) + half;
                    *dst = make_uint2(pack2(gelu(z[0] + c0), gelu(z[1] + c1)), pack2(gelu(z[2] + c2), gelu(z[3] + c3)));
                }
            }
            __syncthreads();
        }
        // Last activations to a.hout, 16 bytes per thread and store.
        for (int e = tid; e < NV * (WIDTH / 8); e += 512) {
            const int v = e / (WIDTH / 8), q = e % (WIDTH / 8);
            if (j0 + v < a.n)
                *reinterpret_cast<uint4*>(a.hout + (size_t)(j0 + v) * WIDTH + 8 * q) =
                    Hf[v / 16][q / 4][(v % 16) + 16 * (q % 4)];
        }
        __syncthreads();   // the next tile overwrites Hf
    }
}

// ------------------------------------------------------------------------
// Output layer as its own kernel (width 256): out = (Wout H + b) * scale for
// a slice of 128 MW output rows per workgroup. Each of the 8 waves keeps its
// 16 MW output rows' weights in registers as MFMA B fragments (32 MW VGPRs)
// for the whole launch; the workgroup streams 64-voxel tiles of the
// activations through double-buffered LDS (the next tile's loads are in
// flight while the current one is multiplied) and writes 4 consecutive
// voxels per store as in the fused kernel. A tile of activations is read
// once per output slice (9 slices for 4 trains of 1120 TRs) instead of each
// voxel tile re-reading all output weights.
// ------------------------------------------------------------------------
template <bool F16, int MW>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
void mlp_out_kernel(InferArgs a, const uint16_t* __restrict__ H)
{
    constexpr int WIDTH = 256, KB = WIDTH / 32, NVT = 64;
    // Activation tiles in MFMA A-fragment order: [buffer][16-voxel tile][K
    // block][lane], 16 bytes per lane, so every fragment read is one
    // contiguous, conflict-free 1 KB wave access.
    __shared__ uint4 Hf[2][NVT / 16][KB][64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = 8 * (lane >> 4);
    // MW 16-row output tiles per wave: a slice of 128 MW rows per workgroup.
    const int o0 = blockIdx.x * 128 * MW + wave * 16 * MW;
    uint4 wf[MW][KB];
    float bias[MW], scl[MW];
    int orow[MW];
#pragma unroll
    for (int m = 0; m < MW; ++m) {
        const int o = o0 + 16 * m + lr;
        orow[m] = o;
        const int oc = min(o, a.m_out - 1);   // rows past the end: clamped, never stored
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
            wf[m][kb] = *reinterpret_cast<const uint4*>(a.Wout + (size_t)oc * WIDTH + 32 * kb + lk);
        bias[m] = a.bout[oc];
        scl[m] = a.head_scale[oc / a.T];
    }
    const int n_tiles = (a.n + NVT - 1) / NVT;
    const bool vec_ok = (a.ld_out % 4) == 0;
    // FP16 output of whole tiles goes through a per-wave LDS transpose so
    // that every store instruction writes 64 contiguous bytes of each of 16
    // rows (instead of 32), in the half of Hf that no wave reads this tile.
    const bool vec8_ok = F16 && (a.ld_out % 8) == 0 && (reinterpret_cast<uintptr_t>(a.out) & 15) == 0;
    constexpr int SROW = NVT + 8;   // staging row pitch (halves), padded against bank conflicts
    // Tile loads: 32 fragments of 64 x 16 bytes; wave w loads fragments
    // w, w + 8, w + 16, w + 24, each lane the piece it will be read from.
    // (Four named registers: an array here was placed in LDS by the compiler.)
    uint4 hr0, hr1, hr2, hr3;
    auto piece = [&](int t, int i) {
        const int f = wave + 8 * i, vt = f / KB, kb = f % KB;
        const int j = min(t * NVT + vt * 16 + lr, a.n - 1);
        return *reinterpret_cast<const uint4*>(H + (size_t)j * WIDTH + 32 * kb + lk);
    };
    auto gload = [&](int t) {
        hr0 = piece(t, 0);
        hr1 = piece(t, 1);
        hr2 = piece(t, 2);
        hr3 = piece(t, 3);
    };
    auto sstore = [&](int buf) {
        Hf[buf][wave / KB][wave % KB][lane] = hr0;
        Hf[buf][(wave + 8) / KB][(wave + 8) % KB][lane] = hr1;
        Hf[buf][(wave + 16) / KB][(wave + 16) % KB][lane] = hr2;
        Hf[buf][(wave + 24) / KB][(wave + 24) % KB][lane] = hr3;
    };
    int t = blockIdx.y;
    if (t < n_tiles) {
        gload(t);
        sstore(0);
    }
    __syncthreads();
    using OT = typename std::conditional<F16, _Float16, float>::type;
    for (int buf = 0; t < n_tiles; t += gridDim.y, buf ^= 1) {
        const bool more = t + (int)gridDim.y < n_tiles;
        const bool stage = vec8_ok && t * NVT + NVT <= a.n;   // uniform per workgroup
        uint2 pk[4][MW];                                      // FP16 results of the tile (staged path)
        if (more) gload(t + gridDim.y);
        // One 16-voxel tile at a time (accumulators for MW output tiles).
#pragma unroll
        for (int vt = 0; vt < 4; ++vt) {
            f4 acc[MW];
#pragma unroll
            for (int m = 0; m < MW; ++m) acc[m] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                const uint4 af = Hf[buf][vt][kb][lane];
#pragma unroll
                for (int m = 0; m < MW; ++m)
                    acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        __builtin_bit_cast(bf16x8, af), __builtin_bit_cast(bf16x8, wf[m][kb]), acc[m], 0, 0, 0);
            }
            // D: lane holds voxels 4 (lane / 16) + i of the tile, output row lr.
            const int jv = t * NVT + vt * 16 + 4 * (lane >> 4);
            if (stage) {
#pragma unroll
                for (int m = 0; m < MW; ++m) {
                    const h4v hv = h4v{(_Float16)((acc[m][0] + bias[m]) * scl[m]),
                                       (_Float16)((acc[m][1] + bias[m]) * scl[m]),
                                       (_Float16)((acc[m][2] + bias[m]) * scl[m]),
                                       (_Float16)((acc[m][3] + bias[m]) * scl[m])};
                    pk[vt][m] = __builtin_bit_cast(uint2, hv);
                }
                continue;
            }
#pragma unroll
            for (int m = 0; m < MW; ++m) {
                const int o = orow[m];
                if (o < a.m_out) {
                    const int p = o / a.T, nt = o - p * a.T;
                    OT* dst = static_cast<OT*>(a.out) + (size_t)p * a.plane + (size_t)nt * a.ld_out;
                    const float y0 = (acc[m][0] + bias[m]) * scl[m], y1 = (acc[m][1] + bias[m]) * scl[m];
                    const float y2 = (acc[m][2] + bias[m]) * scl[m], y3 = (acc[m][3] + bias[m]) * scl[m];
                    if (vec_ok && jv + 3 < a.n) {
                        if constexpr (F16)
                            *reinterpret_cast<h4v*>(dst + jv) = h4v{(_Float16)y0, (_Float16)y1, (_Float16)y2, (_Float16)y3};
                        else
                            *reinterpret_cast<f4*>(dst + jv) = f4{y0, y1, y2, y3};
                    } else {
                        if (jv < a.n) dst[jv] = (OT)y0;
                        if (jv + 1 < a.n) dst[jv + 1] = (OT)y1;
                        if (jv + 2 < a.n) dst[jv + 2] = (OT)y2;
                        if (jv + 3 < a.n) dst[jv + 3] = (OT)y3;
                    }
                }
            }
        }
        if (stage) {
            // Wave-private staging rows [16][SROW] in Hf[buf ^ 1]; LDS operations
            // of one wave complete in order, the fences keep the compiler from
            // moving them.
            _Float16* S = reinterpret_cast<_Float16*>(&Hf[buf ^ 1][0][0][0]) + wave * 16 * SROW;
            const int r = lane >> 2, c = lane & 3;
#pragma unroll
            for (int m = 0; m < MW; ++m) {
#pragma unroll
                for (int vt = 0; vt < 4; ++vt)
                    *reinterpret_cast<uint2*>(S + lr * SROW + vt * 16 + 4 * (lane >> 4)) = pk[vt][m];
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                const uint4 v0 = *reinterpret_cast<const uint4*>(S + r * SROW + 8 * c);
                const uint4 v1 = *reinterpret_cast<const uint4*>(S + r * SROW + 32 + 8 * c);
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                const int o = o0 + 16 * m + r;
                if (o < a.m_out) {
                    const int p = o / a.T, nt = o - p * a.T;
                    _Float16* dst = static_cast<_Float16*>(a.out) + (size_t)p * a.plane + (size_t)nt * a.ld_out +
                                    (size_t)t * NVT;
                    *reinterpret_cast<uint4*>(dst + 8 * c) = v0;
                    *reinterpret_cast<uint4*>(dst + 32 + 8 * c) = v1;
                }
            }
            if (more) __syncthreads();   // every wave is done with Hf[buf ^ 1] before it is refilled
        }
        if (more) sstore(buf ^ 1);
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_gemm_bf16(bool ta, bool tb, int epi, const GemmArgs& g, hipStream_t s)
{
    dim3 grid(ceil_div(g.N, TN), ceil_div(g.M, TM));
#define GEMM_CASE(TA_, TB_, E_)                                                  \
    if (ta == TA_ && tb == TB_ && epi == E_) {                                   \
        gemm_bf16_kernel<TA_, TB_, E_><<<grid, 256, 0, s>>>(g);                  \
        return hipGetLastError();                                                \
    }
    GEMM_CASE(false, false, EPI_BIAS_GELU)
    GEMM_CASE(false, false, EPI_OUT_LOSS)
    GEMM_CASE(false, false, EPI_INFER)
    GEMM_CASE(false, true, EPI_STORE_F32)
    GEMM_CASE(true, false, EPI_GELU_BWD)
#undef GEMM_CASE
    return hipErrorInvalidValue;
}

int gemm_tiles(int M, int N) { return ceil_div(N, TN) * ceil_div(M, TM); }

hipError_t launch_layer1_fwd(const float* x_in, int64_t ldx, int n, const float* W1,
                             const float* b1, int width, const float* lo, const float* hi,
                             float* xs, uint16_t* Zb, uint16_t* Hb, int64_t ldo, hipStream_t s)
{
    layer1_fwd_kernel<<<dim3(ceil_div(n, 256), ceil_div(width, 32)), 256, 0, s>>>(x_in, ldx, n, W1, b1, width, lo[0], lo[1], lo[2],
                                                       hi[0], hi[1], hi[2], xs, Zb, Hb, ldo);
    return hipGetLastError();
}

hipError_t launch_rowsum_bf16(const uint16_t* X, int64_t ld, int rows, int n, float* out,
                              hipStream_t s)
{
    rowsum_kernel<<<rows, 256, 0, s>>>(X, ld, n, out);
    return hipGetLastError();
}

hipError_t launch_layer1_wgrad(const uint16_t* dZ, const float* xs, int64_t ld, int width, int n,
                               float* dW1, hipStream_t s)
{
    layer1_wgrad_kernel<<<width, 256, 0, s>>>(dZ, xs, ld, n, dW1);
    return hipGetLastError();
}

hipError_t launch_adam(float* w, float* m, float* v, const float* g, uint16_t* wb, size_t n,
                       float lr, int step, hipStream_t s)
{
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    adam_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(w, m, v, g, wb, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

bool infer_fused_supported(int width, int depth) { return (width == 64 || width == 128 || width == 256) && depth - 1 <= MAX_HIDDEN; }

hipError_t launch_mlp_infer(int width, int tile, const InferArgs& a, hipStream_t s)
{
    if (tile == 0) tile = width == 256 ? -64 : 64;
    const int grid = ceil_div(a.n, tile < 0 ? -tile : tile);
#define INFER(W_, NV_, T_, PF_)                                              \
    if (width == W_ && tile == T_) {                                         \
        if (a.f16) mlp_infer_kernel<W_, NV_, PF_, true><<<grid, 256, 0, s>>>(a);   \
        else mlp_infer_kernel<W_, NV_, PF_, false><<<grid, 256, 0, s>>>(a);        \
        return hipGetLastError();                                            \
    }
    INFER(64, 64, 64, 1)
    INFER(64, 32, 32, 1)
    INFER(128, 64, 64, 1)
    INFER(128, 32, 32, 1)
    INFER(256, 64, 64, 0)
    INFER(256, 32, 32, 1)
    // Negative tile: the same voxel tile with activations read from LDS and
    // three weight tiles in flight.
    INFER(64, 64, -64, 3)
    INFER(128, 64, -64, 3)
    INFER(256, 64, -64, 2)
    INFER(256, 32, -32, 3)
#undef INFER
    return hipErrorInvalidValue;
}

hipError_t launch_mlp_hidden(const InferArgs& a, hipStream_t s)
{
    // 208-voxel tiles (240 VGPRs): 242 tiles at 224 x 224 fill one round of
    // the 256 CUs. Measured there: 72 us; tiles of 112 / 128 / 224 voxels 85 /
    // 88 / 76 us; the fused kernel's hidden layers on 32-voxel tiles 108 us.
    constexpr int NV = 208;
    const int tiles = ceil_div(a.n, NV);
    mlp_hidden_kernel<NV><<<std::min(tiles, 256), 512, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_mlp_out(const InferArgs& a, const uint16_t* H, hipStream_t s)
{
    // 2, 3 or 4 output tiles per wave (slices of 256, 384 or 512 rows): the
    // fewest rows computed, then the widest slice (fewest activation reads).
    // 4 trains of 1120 TRs: 512-row slices (203 us against 229 us for 256);
    // m only: 384-row slices (1152 rows computed instead of 1536).
    int MW = 4, best = 1 << 30;
    for (int mw = 4; mw >= 2; --mw) {
        const int rows = ceil_div(a.m_out, 128 * mw) * 128 * mw;
        if (rows < best) {
            best = rows;
            MW = mw;
        }
    }
    const int slices = ceil_div(a.m_out, 128 * MW);
    const int tiles = ceil_div(a.n, 64);
    // Voxel-tile groups: one workgroup per CU over all output slices, a
    // single round.
    const int groups = std::max(1, std::min(tiles, 256 / slices));
    dim3 grid(slices, groups);
#define OUT_CASE(M_)                                                            \
    if (MW == M_) {                                                             \
        if (a.f16) mlp_out_kernel<true, M_><<<grid, 512, 0, s>>>(a, H);         \
        else mlp_out_kernel<false, M_><<<grid, 512, 0, s>>>(a, H);              \
        return hipGetLastError();                                               \
    }
    OUT_CASE(4) OUT_CASE(3) OUT_CASE(2)
#undef OUT_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_to_bf16(const float* x, uint16_t* y, size_t n, hipStream_t s)
{
    to_bf16_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, y, n);
    return hipGetLastError();
}

}  // namespace mrstat
