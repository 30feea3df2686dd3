// Internal declarations of the surrogate-network kernels (mlp.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mrstat.h"

namespace mrstat {

enum : int {
    EPI_STORE_F32 = 0,   // Cf[m][n] = acc
    EPI_BIAS_GELU = 1,   // z = acc + bias[m]; Zb = bf16(z) (if set); Hb = bf16(gelu(z))
    EPI_OUT_LOSS = 2,    // y = acc + bias[m]; d = y - scaled target; Hb = bf16(grad_scale d); loss partials
    EPI_GELU_BWD = 3,    // Hb = bf16(acc * gelu'(Zin))
    EPI_INFER = 4        // trains[p][n_tr][col] = (acc + bias[m]) * head_scale[p], p = m / T
};

struct GemmArgs {
    const uint16_t* A;   // bf16 operands
    int64_t lda;
    const uint16_t* B;
    int64_t ldb;
    int M, N, K;
    int64_t ldo;             // leading dimension of the outputs (and of Zin)
    float* Cf;               // FP32 output (STORE) or trains (INFER)
    uint16_t* Zb;            // pre-activation out (BIAS_GELU), optional
    uint16_t* Hb;            // bf16 output
    const uint16_t* Zin;     // pre-activation in (GELU_BWD)
    const float* bias;
    const float* target;     // [4][T][ld_t] imaginary parts (OUT_LOSS)
    int64_t ld_t;
    int T;
    const float* head_scale; // [4]
    float grad_scale;        // dY = grad_scale (y - t)
    double* loss_part;       // one double per tile (OUT_LOSS)
    int64_t plane;           // INFER: floats between trains
};

// Fused inference (one workgroup per 32 or 64 voxels) for widths 64, 128, 256.
constexpr int MAX_HIDDEN = 15;
struct InferArgs {
    const float* theta;            // rows ln T1, ln T2, B1 with leading dimension ldth
    int64_t ldth;
    int n;                         // voxels
    const float* W1;               // FP32 [width][3]
    const float* b1;
    float lo[3], hi[3];            // input box
    const uint16_t* Wh[MAX_HIDDEN];   // BF16 [width][width] of hidden layers 2..depth
    const float* bh[MAX_HIDDEN];
    int n_hidden;                  // depth - 1
    const uint16_t* Wout;          // BF16 rows of the outputs produced (row 0 = output 0)
    const float* bout;
    const float* head_scale;       // [4]
    int T;                         // TRs per train
    int m_out;                     // outputs produced: 4T (all trains) or T (m only)
    void* out;                     // out[p * plane + n * ld_out + voxel], float or _Float16
    int64_t ld_out, plane;
    bool f16;                      // trains stored as FP16
    uint16_t* hout;                // launch_mlp_hidden: the last hidden activations
                                   // (BF16 [voxel][width])
};
bool infer_fused_supported(int width, int depth);
// tile: voxels per workgroup, 32 or 64 (activations in registers), -32 or
// -64 (activations read from LDS); 0 = default.
hipError_t launch_mlp_infer(int width, int tile, const InferArgs& a, hipStream_t s);
// Output layer alone (width 256) from activations H (BF16 [voxel][256], as
// stored by launch_mlp_hidden): same outputs and layout as the fused kernel.
hipError_t launch_mlp_out(const InferArgs& a, const uint16_t* H, hipStream_t s);
// Hidden layers alone (width 256): the last activations to a.hout (BF16
// [voxel][256]), weights of one layer at a time in registers.
hipError_t launch_mlp_hidden(const InferArgs& a, hipStream_t s);

hipError_t launch_gemm_bf16(bool ta, bool tb, int epi, const GemmArgs& g, hipStream_t s);
int gemm_tiles(int M, int N);
hipError_t launch_layer1_fwd(const float* x_in, int64_t ldx, int n, const float* W1,
                             const float* b1, int width, const float* lo, const float* hi,
                             float* xs, uint16_t* Zb, uint16_t* Hb, int64_t ldo, hipStream_t s);
hipError_t launch_rowsum_bf16(const uint16_t* X, int64_t ld, int rows, int n, float* out,
                              hipStream_t s);
hipError_t launch_layer1_wgrad(const uint16_t* dZ, const float* xs, int64_t ld, int width, int n,
                               float* dW1, hipStream_t s);
hipError_t launch_adam(float* w, float* m, float* v, const float* g, uint16_t* wb, size_t n,
                       float lr, int step, hipStream_t s);
hipError_t launch_to_bf16(const float* x, uint16_t* y, size_t n, hipStream_t s);

// Surrogate inference for the context (mlp_api.hip): trains of n voxels whose
// theta rows (ln T1, ln T2, B1) have leading dimension ld_theta, into
// out[p][n_tr][ld_out] (float, or _Float16 when f16) for p < n_trains
// (4: m and the three derivatives; 3: without dm/dB1; 1: m only).
// hbuf (optional, n x 256 BF16): for width 256, the hidden layers and the
// output layer run as two kernels through it.
hipError_t mlp_infer_trains(mrstat_mlp net, const float* theta, int64_t ld_theta, int n, void* out,
                            int64_t ld_out, int n_trains, bool f16, uint16_t* hbuf, hipStream_t s);
const float* mlp_box_lo(mrstat_mlp net);
const float* mlp_box_hi(mrstat_mlp net);
int mlp_n_tr(mrstat_mlp net);
bool mlp_ready(mrstat_mlp net);
// True when the network's inference can store FP16 trains (the fused widths
// 64, 128 and 256; the chunked path of other widths writes FP32 only).
bool mlp_writes_f16(mrstat_mlp net);

}  // namespace mrstat
