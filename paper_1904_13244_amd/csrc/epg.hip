// EPG linearisation kernel: one voxel per group of L lanes, the K states of
// the voxel split over the group (S = Kcap / L consecutive orders per lane),
// value and NTAN tangent state vectors in registers (NTAN = 3: ln T1, ln T2,
// B1; 2: ln T1, ln T2 only, for fits with B1 held fixed, whose Jacobian has
// no B1 column; 0: value only).
//
// Model: gradient-spoiled transient-state sequence; per TR an instantaneous RF
// pulse of angle B1 * alpha_n about an axis at RF phase phi_n in {0, pi},
// relaxation to TE, readout of F+_0 demodulated by the RF phase, relaxation to
// TR, spoiler shift of all orders by one (truncated at K). Tangents in ln T1,
// ln T2 and B1 follow the forward-mode recursion of Supporting Information S2
// (each update differentiated, zero initial tangents, sin/cos/exp of a TR
// computed once and reused by value and tangents).
//
// Real form: with phi_n in {0, pi} and no off-resonance every F state stays
// purely imaginary and every Z state real, so the kernel carries
// f = Im F+, g = Im F-, z = Z (3 reals per order instead of 6). With
// sg = cos(phi_n) = +-1 and a = B1 alpha_n, the RF operator is
//     f' = c^2 f + s^2 g - sg sin(a) z
//     g' = s^2 f + c^2 g + sg sin(a) z
//     z' = (sg/2) sin(a) (f - g) + cos(a) z          (c, s = cos, sin of a/2)
// and the relaxation over a whole TR (E1, E2, regrowth 1 - E1 of Z_0) is
// folded into its coefficients; the readout uses the unrelaxed RF output at
// order 0 times E2(TE). Recorded value: Im m = sg E2(TE) f_0.
#include "mrstat_internal.h"

namespace mrstat {
namespace {

// Spoiler shift of one state vector: order k of F+ takes order k-1, order k
// of F- takes order k+1, F-_{K-1} = 0, and the new F+_0 = conj(F-_0), which
// is -g_0 in the real form. Orders are spread over the L lanes of a group.
template <int S, int L>
__device__ __forceinline__ void shift_orders(float (&f)[S], float (&g)[S], bool lead, bool last)
{
    float up = 0.f, dn = 0.f;
    if constexpr (L > 1) {
        up = __shfl_up(f[S - 1], 1, L);
        dn = __shfl_down(g[0], 1, L);
    }
#pragma unroll
    for (int i = S - 1; i >= 1; --i) f[i] = f[i - 1];
#pragma unroll
    for (int i = 0; i < S - 1; ++i) g[i] = g[i + 1];
    g[S - 1] = last ? 0.f : dn;
    f[0] = lead ? -g[0] : up;
}

template <int S>
__device__ __forceinline__ void clear_above(float (&f)[S], int base, int K)
{
#pragma unroll
    for (int i = 0; i < S; ++i)
        if (base + i >= K) f[i] = 0.f;
}

// LIST: the group handles voxel idx[vox] for vox < *count (the other voxels'
// outputs are left untouched); whole blocks past the list exit at once.
// TT: element type of the stored trains (float, or _Float16 rounded to
// nearest from the FP32 recursion).
template <int S, int L, int NTAN, bool MASKED, bool LIST, typename TT>
__global__ __launch_bounds__(256) void epg_kernel(const float* __restrict__ theta,
                                                  const float2* __restrict__ seq,
                                                  TT* __restrict__ out, int nv, int T,
                                                  int K, SeqTimes st,
                                                  const int* __restrict__ idx,
                                                  const int* __restrict__ count)
{
    const int gt = blockIdx.x * blockDim.x + threadIdx.x;
    const int vox = gt / L;
    const int l = gt % L;
    int j;
    bool valid;
    if constexpr (LIST) {
        const int cnt = *count;
        if ((int)(blockIdx.x * blockDim.x / L) >= cnt) return;   // uniform per block
        valid = vox < cnt;
        j = idx[valid ? vox : cnt - 1];
    } else {
        valid = vox < nv;
        j = valid ? vox : nv - 1;   // keep every lane active for the shuffles
    }
    const bool lead = (l == 0), last = (l == L - 1);
    const bool store = valid && lead;
    const int base = l * S;

    const float lnT1 = theta[j], lnT2 = theta[nv + j], B1 = theta[2 * nv + j];
    const float rT1 = expf(-lnT1), rT2 = expf(-lnT2);   // 1/T1, 1/T2
    const float tau1 = st.tr * rT1, tau2 = st.tr * rT2, tau2e = st.te * rT2;
    const float E1 = expf(-tau1), E2 = expf(-tau2);
    const float R1 = lead ? -expm1f(-tau1) : 0.f;       // regrowth of Z_0 only
    const float dR1 = lead ? tau1 * E1 : 0.f;           // -d(1-E1)/dlnT1
    const float E2e = expf(-tau2e);
    const float taui = st.tinv * rT1;
    const float E1i = expf(-taui), R1i = -expm1f(-taui);

    constexpr bool TANG = NTAN > 0, TB1 = NTAN == 3;
    float f[S], g[S], z[S];
    float f1[S], g1[S], z1[S];   // d/d ln T1
    float f2[S], g2[S], z2[S];   // d/d ln T2
    float f3[S], g3[S], z3[S];   // d/d B1
#pragma unroll
    for (int i = 0; i < S; ++i) {
        f[i] = g[i] = z[i] = 0.f;
        if constexpr (TANG) {
            f1[i] = g1[i] = z1[i] = 0.f;
            f2[i] = g2[i] = z2[i] = 0.f;
        }
        if constexpr (TB1) f3[i] = g3[i] = z3[i] = 0.f;
    }
    // Ideal inversion of the equilibrium Z_0 = 1, then relaxation over t_inv.
    if (lead) {
        z[0] = R1i - E1i;
        if constexpr (TANG) z1[0] = -2.f * taui * E1i;
    }

    const size_t plane = (size_t)T * nv;
    TT* o0 = out + j;
    for (int n = 0; n < T; ++n) {
        const float2 sq = seq[n];
        const float alpha = sq.x, sg = sq.y;
        float sh, ch;
        sincosf(0.5f * (B1 * alpha), &sh, &ch);
        const float c2 = ch * ch, s2 = sh * sh;
        const float sa = 2.f * sh * ch, ca = (ch - sh) * (ch + sh);
        const float sgsa = sg * sa;
        // Coefficients with the TR relaxation folded in.
        const float A = E2 * c2, B = E2 * s2, Cc = E2 * sgsa;
        const float D = 0.5f * E1 * sgsa, G = E1 * ca;

        // Readout at TE from the unrelaxed RF output of order 0.
        {
            const float rp = fmaf(c2, f[0], fmaf(s2, g[0], -sgsa * z[0]));
            const float ke = sg * E2e;
            if (store) o0[(size_t)n * nv] = (TT)(ke * rp);
            if constexpr (TANG) {
                const float rp1 = fmaf(c2, f1[0], fmaf(s2, g1[0], -sgsa * z1[0]));
                const float rp2 = fmaf(c2, f2[0], fmaf(s2, g2[0], -sgsa * z2[0]));
                if (store) {
                    o0[plane + (size_t)n * nv] = (TT)(ke * rp1);
                    o0[2 * plane + (size_t)n * nv] = (TT)(ke * fmaf(tau2e, rp, rp2));
                }
            }
            if constexpr (TB1) {
                const float drp = fmaf(-0.5f * sa, f[0] - g[0], -sg * ca * z[0]);
                const float rp3 = fmaf(c2, f3[0], fmaf(s2, g3[0], fmaf(alpha, drp, -sgsa * z3[0])));
                if (store) o0[3 * plane + (size_t)n * nv] = (TT)(ke * rp3);
            }
        }

        if constexpr (TANG) {
            // B1 derivatives of the folded coefficients (d a / d B1 = alpha).
            const float dA = -0.5f * E2 * alpha * sa;      // dA/dB1 = -dB/dB1
            const float dC = E2 * alpha * sg * ca;
            const float dD = 0.5f * E1 * alpha * sg * ca;
            const float dG = -E1 * alpha * sa;
#pragma unroll
            for (int i = 0; i < S; ++i) {
                const float w = f[i] - g[i];
                const float Cz = Cc * z[i];
                const float nf = fmaf(A, f[i], fmaf(B, g[i], -Cz));
                const float ng = fmaf(B, f[i], fmaf(A, g[i], Cz));
                const float nz = fmaf(D, w, G * z[i]);
                {   // ln T1: only E1 (Z rows) depends on T1
                    const float w1 = f1[i] - g1[i];
                    const float Cz1 = Cc * z1[i];
                    const float a = fmaf(A, f1[i], fmaf(B, g1[i], -Cz1));
                    const float b = fmaf(B, f1[i], fmaf(A, g1[i], Cz1));
                    const float c = fmaf(D, w1, fmaf(G, z1[i], tau1 * nz));
                    f1[i] = a; g1[i] = b; z1[i] = c;
                }
                {   // ln T2: only E2 (F rows) depends on T2
                    const float w2 = f2[i] - g2[i];
                    const float Cz2 = Cc * z2[i];
                    const float a = fmaf(A, f2[i], fmaf(B, g2[i], fmaf(tau2, nf, -Cz2)));
                    const float b = fmaf(B, f2[i], fmaf(A, g2[i], fmaf(tau2, ng, Cz2)));
                    const float c = fmaf(D, w2, G * z2[i]);
                    f2[i] = a; g2[i] = b; z2[i] = c;
                }
                if constexpr (TB1) {   // B1: the RF coefficients depend on a = B1 alpha
                    const float w3 = f3[i] - g3[i];
                    const float t3 = fmaf(dA, w, -dC * z[i]);
                    const float Cz3 = Cc * z3[i];
                    const float a = fmaf(A, f3[i], fmaf(B, g3[i], t3 - Cz3));
                    const float b = fmaf(B, f3[i], fmaf(A, g3[i], Cz3 - t3));
                    const float c = fmaf(D, w3, fmaf(G, z3[i], fmaf(dD, w, dG * z[i])));
                    f3[i] = a; g3[i] = b; z3[i] = c;
                }
                f[i] = nf; g[i] = ng; z[i] = nz;
            }
            z[0] += R1;
            z1[0] -= dR1;
        } else {
#pragma unroll
            for (int i = 0; i < S; ++i) {
                const float w = f[i] - g[i];
                const float Cz = Cc * z[i];
                const float nf = fmaf(A, f[i], fmaf(B, g[i], -Cz));
                const float ng = fmaf(B, f[i], fmaf(A, g[i], Cz));
                z[i] = fmaf(D, w, G * z[i]);
                f[i] = nf; g[i] = ng;
            }
            z[0] += R1;
        }

        shift_orders<S, L>(f, g, lead, last);
        if constexpr (MASKED) clear_above<S>(f, base, K);
        if constexpr (TANG) {
            shift_orders<S, L>(f1, g1, lead, last);
            shift_orders<S, L>(f2, g2, lead, last);
            if constexpr (MASKED) {
                clear_above<S>(f1, base, K);
                clear_above<S>(f2, base, K);
            }
        }
        if constexpr (TB1) {
            shift_orders<S, L>(f3, g3, lead, last);
            if constexpr (MASKED) clear_above<S>(f3, base, K);
        }
    }
}

template <int S, int L, int NTAN, bool LIST, typename TT>
hipError_t launch_sl(const Dims& d, SeqTimes st, const float* theta, const float2* seq, TT* out,
                     const int* idx, const int* count, hipStream_t s)
{
    const long threads = (long)d.nv * L;
    const int block = 256;
    const int grid = (int)((threads + block - 1) / block);
    if (d.K == S * L)
        epg_kernel<S, L, NTAN, false, LIST, TT><<<grid, block, 0, s>>>(theta, seq, out, d.nv, d.T, d.K,
                                                                       st, idx, count);
    else
        epg_kernel<S, L, NTAN, true, LIST, TT><<<grid, block, 0, s>>>(theta, seq, out, d.nv, d.T, d.K,
                                                                      st, idx, count);
    return hipGetLastError();
}

template <int NTAN, bool LIST, typename TT>
hipError_t launch_any(const Dims& d, SeqTimes st, const float* theta, const float2* seq,
                      TT* out, int lanes, const int* idx, const int* count, hipStream_t s)
{
    const int K = d.K;
#define SL(S_, L_) launch_sl<S_, L_, NTAN, LIST, TT>(d, st, theta, seq, out, idx, count, s)
    if (K <= 8) {
        if (lanes == 2) return SL(4, 2);
        return SL(8, 1);
    }
    if (K <= 16) {
        if (lanes == 1) return SL(16, 1);
        if (lanes == 4) return SL(4, 4);
        return SL(8, 2);
    }
    if (K <= 32) {
        if (lanes == 4) return SL(8, 4);
        if (lanes == 8) return SL(4, 8);
        return SL(16, 2);
    }
    if (K <= 64) {
        if (lanes == 8) return SL(8, 8);
        return SL(16, 4);
    }
#undef SL
    return hipErrorInvalidValue;
}

// Appends to idx every voxel (in the mask) whose (ln T1, ln T2, B1) lies
// outside [lo, hi] or is not finite; *count must be 0 on entry. One atomic per
// wave; the order of the list is unspecified (each voxel is simulated alone).
__global__ __launch_bounds__(256) void box_compact_kernel(const float* __restrict__ theta, int nv,
                                                          float lo0, float lo1, float lo2, float hi0,
                                                          float hi1, float hi2,
                                                          const uint8_t* __restrict__ mask,
                                                          int* __restrict__ idx, int* __restrict__ count)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    bool out = false;
    if (j < nv && (!mask || mask[j])) {
        const float a = theta[j], b = theta[nv + j], c = theta[2 * nv + j];
        const bool in = (a >= lo0 && a <= hi0) && (b >= lo1 && b <= hi1) && (c >= lo2 && c <= hi2);
        out = !in;   // NaN compares false, so it falls back as well
    }
    const uint64_t bal = __ballot(out);
    if (bal == 0) return;
    const int lane = threadIdx.x & 63;
    int base = 0;
    if (lane == __ffsll((unsigned long long)bal) - 1) base = atomicAdd(count, __popcll(bal));
    base = __shfl(base, __ffsll((unsigned long long)bal) - 1);
    if (out) idx[base + __popcll(bal & ((1ull << lane) - 1ull))] = j;
}

__global__ void zero_int_kernel(int* p) { *p = 0; }

__global__ void half_to_float_kernel(const _Float16* __restrict__ in, float* __restrict__ out, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

}  // namespace

template <bool LIST, typename TT>
hipError_t launch_ntan(const Dims& d, SeqTimes st, const float* theta, const float2* seq, TT* out,
                       int ntan, int lanes, const int* idx, const int* count, hipStream_t s)
{
    switch (ntan) {
        case 0: return launch_any<0, LIST>(d, st, theta, seq, out, lanes, idx, count, s);
        case 2: return launch_any<2, LIST>(d, st, theta, seq, out, lanes, idx, count, s);
        case 3: return launch_any<3, LIST>(d, st, theta, seq, out, lanes, idx, count, s);
        default: return hipErrorInvalidValue;
    }
}

template <bool LIST>
hipError_t launch_typed(const Dims& d, SeqTimes st, const float* theta, const float2* seq, void* out,
                        int ntan, int lanes, bool f16, const int* idx, const int* count,
                        hipStream_t s)
{
    if (f16)
        return launch_ntan<LIST>(d, st, theta, seq, static_cast<_Float16*>(out), ntan, lanes, idx, count, s);
    return launch_ntan<LIST>(d, st, theta, seq, static_cast<float*>(out), ntan, lanes, idx, count, s);
}

hipError_t launch_epg(const Dims& d, SeqTimes st, const float* theta, const float2* seq,
                      void* out, int ntan, int lanes, bool f16, hipStream_t s)
{
    return launch_typed<false>(d, st, theta, seq, out, ntan, lanes, f16, nullptr, nullptr, s);
}

hipError_t launch_epg_list(const Dims& d, SeqTimes st, const float* theta, const float2* seq,
                           void* out, int ntan, int lanes, bool f16, const int* idx,
                           const int* count, hipStream_t s)
{
    return launch_typed<true>(d, st, theta, seq, out, ntan, lanes, f16, idx, count, s);
}

hipError_t launch_trains_to_f32(const void* in, bool f16, float* out, size_t n, hipStream_t s)
{
    if (!f16) return hipMemcpyAsync(out, in, n * sizeof(float), hipMemcpyDeviceToDevice, s);
    half_to_float_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(static_cast<const _Float16*>(in),
                                                                   out, n);
    return hipGetLastError();
}

hipError_t launch_box_compact(const Dims& d, const float* theta, const float* lo, const float* hi,
                              const uint8_t* mask, int* idx, int* count, hipStream_t s)
{
    zero_int_kernel<<<1, 1, 0, s>>>(count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    box_compact_kernel<<<ceil_div(d.nv, 256), 256, 0, s>>>(theta, d.nv, lo[0], lo[1], lo[2], hi[0], hi[1],
                                                           hi[2], mask, idx, count);
    return hipGetLastError();
}

}  // namespace mrstat
