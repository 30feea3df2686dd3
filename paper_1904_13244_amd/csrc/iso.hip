// Linearisation by the balanced isochromat model (the paper's own signal
// model: balanced transient-state gradient echo, RF phase alternating 0 /
// 180 degrees, isochromats over the slice profile; Methods, Pulse Sequence
// and Reconstructions; the update of Supporting Information S2).
//
// Per voxel, isochromat q sees the flip angle scaled by scale[q] and enters
// the voxel's magnetisation with weight weight[q]. On resonance with the RF
// axis along +-x (phase 0 or pi) every isochromat stays in the y-z plane, so
// it is carried as (y, z) = (my, mz): the RF rotates it by a = B1 alpha_n
// scale about sg x (sg = cos phi_n = +-1),
//     y' = y cos a - sg z sin a,   z' = sg y sin a + z cos a,
// the readout at TE records Im m = sg E2(TE) y' (demodulated by the RF
// phase), and the relaxation over the whole TR follows (E2 on y, E1 and the
// regrowth 1 - E1 on z; the same as TE then TR - TE). Tangents in ln T1,
// ln T2 and B1 are carried in forward mode through both updates (zero at
// the start; d a / d B1 = alpha_n scale).
//
// Four lanes per voxel, isochromat q on lane q % 4 (slot q / 4); per TR the
// lanes' weighted sums meet by two shuffles and lane p stores train p.
#include "mrstat_internal.h"

namespace mrstat {
namespace {

constexpr int ISO_L = 4;                          // lanes per voxel
constexpr int ISO_SLOTS = MAX_ISOCHROMATS / ISO_L;

template <int NTAN, bool LIST, typename TT>
__global__ __launch_bounds__(256) void iso_kernel(const float* __restrict__ theta, const float2* __restrict__ seq,
                                                  TT* __restrict__ out, int nv, int T, SeqTimes st, IsoProfile prof,
                                                  const int* __restrict__ idx, const int* __restrict__ count)
{
    const int gt = blockIdx.x * blockDim.x + threadIdx.x;
    const int vox = gt / ISO_L;
    const int l = gt % ISO_L;
    int j;
    bool valid;
    if constexpr (LIST) {
        const int cnt = *count;
        if ((int)(blockIdx.x * blockDim.x / ISO_L) >= cnt) return;   // uniform per block
        valid = vox < cnt;
        j = idx[valid ? vox : cnt - 1];
    } else {
        valid = vox < nv;
        j = valid ? vox : nv - 1;   // every lane stays active for the shuffles
    }
    constexpr bool TANG = NTAN > 0, TB1 = NTAN == 3;

    const float lnT1 = theta[j], lnT2 = theta[nv + j], B1 = theta[2 * nv + j];
    const float rT1 = expf(-lnT1), rT2 = expf(-lnT2);
    const float tau1 = st.tr * rT1, tau2 = st.tr * rT2, tau2e = st.te * rT2;
    const float E1 = expf(-tau1), E2 = expf(-tau2), E2e = expf(-tau2e);
    const float R1 = -expm1f(-tau1);
    const float taui = st.tinv * rT1;
    const float E1i = expf(-taui), R1i = -expm1f(-taui);

    float sc[ISO_SLOTS], wt[ISO_SLOTS];
    float y[ISO_SLOTS], z[ISO_SLOTS], y1[ISO_SLOTS], z1[ISO_SLOTS], y2[ISO_SLOTS], z2[ISO_SLOTS];
    float y3[ISO_SLOTS], z3[ISO_SLOTS];
#pragma unroll
    for (int k = 0; k < ISO_SLOTS; ++k) {
        const int q = ISO_L * k + l;
        const bool on = q < prof.n;
        sc[k] = on ? prof.scale[q] : 0.f;
        wt[k] = on ? prof.weight[q] : 0.f;
        // Ideal inversion of the equilibrium, then relaxation over t_inv.
        y[k] = 0.f;
        z[k] = R1i - E1i;
        y1[k] = y2[k] = y3[k] = 0.f;
        z1[k] = -2.f * taui * E1i;
        z2[k] = z3[k] = 0.f;
    }

    const size_t plane = (size_t)T * nv;
    for (int n = 0; n < T; ++n) {
        const float2 sq = seq[n];
        const float alpha = sq.x, sg = sq.y;
        float m0 = 0.f, m1 = 0.f, m2 = 0.f, m3 = 0.f;   // this lane's weighted sums of y' at TE
#pragma unroll
        for (int k = 0; k < ISO_SLOTS; ++k) {
            if (ISO_L * k >= prof.n) break;   // uniform: no isochromat in this slot on any lane
            const float da = alpha * sc[k];   // d a / d B1
            float sa, ca;
            sincosf(B1 * da, &sa, &ca);
            const float ssa = sg * sa;
            const float yr = fmaf(y[k], ca, -ssa * z[k]);
            const float zr = fmaf(ssa, y[k], z[k] * ca);
            m0 = fmaf(wt[k], yr, m0);
            if constexpr (TANG) {
                const float y1r = fmaf(y1[k], ca, -ssa * z1[k]);
                const float z1r = fmaf(ssa, y1[k], z1[k] * ca);
                const float y2r = fmaf(y2[k], ca, -ssa * z2[k]);
                const float z2r = fmaf(ssa, y2[k], z2[k] * ca);
                m1 = fmaf(wt[k], y1r, m1);
                m2 = fmaf(wt[k], fmaf(tau2e, yr, y2r), m2);   // d(E2e y)/dlnT2 = E2e (y2 + tau2e y)
                y1[k] = E2 * y1r;
                z1[k] = fmaf(E1, z1r, tau1 * E1 * (zr - 1.f));
                y2[k] = E2 * fmaf(tau2, yr, y2r);
                z2[k] = E1 * z2r;
                if constexpr (TB1) {
                    // d/da of the rotated vector, times d a / d B1.
                    const float dyr = -fmaf(y[k], sa, sg * z[k] * ca);
                    const float dzr = fmaf(sg * ca, y[k], -z[k] * sa);
                    const float y3r = fmaf(y3[k], ca, fmaf(-ssa, z3[k], da * dyr));
                    const float z3r = fmaf(ssa, y3[k], fmaf(z3[k], ca, da * dzr));
                    m3 = fmaf(wt[k], y3r, m3);
                    y3[k] = E2 * y3r;
                    z3[k] = E1 * z3r;
                }
            }
            y[k] = E2 * yr;
            z[k] = fmaf(E1, zr, R1);
        }
        // Sum over the voxel's four lanes; lane p stores train p.
        m0 += __shfl_xor(m0, 1, ISO_L);
        m0 += __shfl_xor(m0, 2, ISO_L);
        if constexpr (TANG) {
            m1 += __shfl_xor(m1, 1, ISO_L);
            m1 += __shfl_xor(m1, 2, ISO_L);
            m2 += __shfl_xor(m2, 1, ISO_L);
            m2 += __shfl_xor(m2, 2, ISO_L);
        }
        if constexpr (TB1) {
            m3 += __shfl_xor(m3, 1, ISO_L);
            m3 += __shfl_xor(m3, 2, ISO_L);
        }
        const float ke = sg * E2e;
        if (valid && l <= NTAN) {
            const float vv = l == 0 ? m0 : (l == 1 ? m1 : (l == 2 ? m2 : m3));
            out[(size_t)l * plane + (size_t)n * nv + j] = (TT)(ke * vv);
        }
    }
}

template <bool LIST, typename TT>
hipError_t iso_typed(const Dims& d, SeqTimes st, const float* theta, const float2* seq, TT* out, int ntan,
                     const IsoProfile& prof, const int* idx, const int* count, hipStream_t s)
{
    const long threads = (long)d.nv * ISO_L;
    const int grid = (int)((threads + 255) / 256);
    switch (ntan) {
    case 0: iso_kernel<0, LIST, TT><<<grid, 256, 0, s>>>(theta, seq, out, d.nv, d.T, st, prof, idx, count); break;
    case 2: iso_kernel<2, LIST, TT><<<grid, 256, 0, s>>>(theta, seq, out, d.nv, d.T, st, prof, idx, count); break;
    case 3: iso_kernel<3, LIST, TT><<<grid, 256, 0, s>>>(theta, seq, out, d.nv, d.T, st, prof, idx, count); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_iso(const Dims& d, SeqTimes st, const float* theta, const float2* seq, void* out, int ntan,
                      bool f16, const IsoProfile& prof, const int* idx, const int* count, hipStream_t s)
{
    if (prof.n < 1 || prof.n > MAX_ISOCHROMATS) return hipErrorInvalidValue;
    if (idx != nullptr)
        return f16 ? iso_typed<true>(d, st, theta, seq, static_cast<_Float16*>(out), ntan, prof, idx, count, s)
                   : iso_typed<true>(d, st, theta, seq, static_cast<float*>(out), ntan, prof, idx, count, s);
    return f16 ? iso_typed<false>(d, st, theta, seq, static_cast<_Float16*>(out), ntan, prof, nullptr, nullptr, s)
               : iso_typed<false>(d, st, theta, seq, static_cast<float*>(out), ntan, prof, nullptr, nullptr, s);
}

}  // namespace mrstat
