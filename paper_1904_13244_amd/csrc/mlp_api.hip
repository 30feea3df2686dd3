// C ABI of the surrogate network (include/mrstat.h, mrstat_mlp_*): workspace
// layout and the host sequencing of forward, backward, Adam and inference.
#include "mrstat.h"
#include "mlp_internal.h"
#include "mrstat_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

using namespace mrstat;

struct mrstat_mlp_s {
    int T = 0, width = 0, depth = 0, B = 0;
    size_t P = 0;                      // parameter count
    std::vector<size_t> off_w, off_b;  // offsets of W_l, b_l in the packed vector (l < depth), then out
    size_t off_wo = 0, off_bo = 0;
    float lo[3]{}, hi[3]{}, scale[4]{1.f, 1.f, 1.f, 1.f};
    int step = 0;
    int infer_tile = 0;    // voxels per workgroup of the fused inference (0 = default)
    // workspace
    char* ws = nullptr;
    size_t ws_bytes = 0;
    size_t o_w32, o_wb, o_m, o_v, o_g, o_z, o_h, o_dy, o_dz, o_xs, o_loss, o_scale, total;
    int n_loss = 0;    // doubles in the loss buffer (also the scaling reduction's partials)
    int n_tiles = 0;   // loss partials written by the output layer (one per tile)
    std::string err;

    float* w32() const { return (float*)(ws + o_w32); }
    uint16_t* wb() const { return (uint16_t*)(ws + o_wb); }
    float* gr() const { return (float*)(ws + o_g); }
    uint16_t* Z(int l) const { return (uint16_t*)(ws + o_z) + (size_t)l * width * B; }
    uint16_t* H(int l) const { return (uint16_t*)(ws + o_h) + (size_t)l * width * B; }
    uint16_t* dY() const { return (uint16_t*)(ws + o_dy); }
    uint16_t* dZ(int i) const { return (uint16_t*)(ws + o_dz) + (size_t)i * width * B; }
    float* xs() const { return (float*)(ws + o_xs); }
    double* loss() const { return (double*)(ws + o_loss); }
    float* dscale() const { return (float*)(ws + o_scale); }
};

namespace {

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

mrstat_status mfail(mrstat_mlp n, mrstat_status st, const std::string& m)
{
    if (n) n->err = m;
    return st;
}

#define MTRY(call)                                                                          \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return mfail(net, MRSTAT_ERR_HIP, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

GemmArgs gargs() { GemmArgs g; std::memset(&g, 0, sizeof(g)); return g; }

// Forward through the hidden layers for ncol samples; h(l) outputs keep their
// pre-activations when keep_z. Input rows (ln T1, ln T2, B1) at theta with ld.
mrstat_status hidden_forward(mrstat_mlp net, const float* theta, int64_t ld, int ncol, bool keep_z,
                             hipStream_t s)
{
    const int W = net->width, B = net->B;
    MTRY(launch_layer1_fwd(theta, ld, ncol, net->w32() + net->off_w[0], net->w32() + net->off_b[0], W,
                           net->lo, net->hi, net->xs(), keep_z ? net->Z(0) : nullptr, net->H(0), B, s));
    for (int l = 1; l < net->depth; ++l) {
        GemmArgs g = gargs();
        g.A = net->wb() + net->off_w[l];
        g.lda = W;
        g.B = net->H(l - 1);
        g.ldb = B;
        g.M = W;
        g.N = ncol;
        g.K = W;
        g.ldo = B;
        g.bias = net->w32() + net->off_b[l];
        g.Zb = keep_z ? net->Z(l) : nullptr;
        g.Hb = net->H(l);
        MTRY(launch_gemm_bf16(false, false, EPI_BIAS_GELU, g, s));
    }
    return MRSTAT_OK;
}

// One batch: forward, loss gradient fused into the output layer, backward into
// gr(). Loss partials in loss()[0..n_loss).
mrstat_status forward_backward(mrstat_mlp net, const float* theta, int64_t ldth,
                               const float* trains, int64_t ldtr, hipStream_t s)
{
    const int W = net->width, B = net->B, T = net->T, L = net->depth;
    mrstat_status st = hidden_forward(net, theta, ldth, B, true, s);
    if (st != MRSTAT_OK) return st;
    // Output layer + loss gradient dY = 2 (y - t) / count.
    {
        GemmArgs g = gargs();
        g.A = net->wb() + net->off_wo;
        g.lda = W;
        g.B = net->H(L - 1);
        g.ldb = B;
        g.M = 8 * T;
        g.N = B;
        g.K = W;
        g.ldo = B;
        g.bias = net->w32() + net->off_bo;
        g.Hb = net->dY();
        g.target = trains;
        g.ld_t = ldtr;
        g.T = T;
        g.head_scale = net->dscale();
        g.grad_scale = (float)(2.0 / ((double)8 * T * B));
        g.loss_part = net->loss();
        MTRY(launch_gemm_bf16(false, false, EPI_OUT_LOSS, g, s));
    }
    // dWout = dY H^T (NT), dbout = row sums of dY.
    {
        GemmArgs g = gargs();
        g.A = net->dY();
        g.lda = B;
        g.B = net->H(L - 1);
        g.ldb = B;
        g.M = 8 * T;
        g.N = W;
        g.K = B;
        g.ldo = W;
        g.Cf = net->gr() + net->off_wo;
        MTRY(launch_gemm_bf16(false, true, EPI_STORE_F32, g, s));
        MTRY(launch_rowsum_bf16(net->dY(), B, 8 * T, B, net->gr() + net->off_bo, s));
    }
    // dZ_{L-1} = (Wout^T dY) * gelu'(Z_{L-1}) (TN).
    int cur = 0;
    {
        GemmArgs g = gargs();
        g.A = net->wb() + net->off_wo;
        g.lda = W;
        g.B = net->dY();
        g.ldb = B;
        g.M = W;
        g.N = B;
        g.K = 8 * T;
        g.ldo = B;
        g.Zin = net->Z(L - 1);
        g.Hb = net->dZ(cur);
        MTRY(launch_gemm_bf16(true, false, EPI_GELU_BWD, g, s));
    }
    for (int l = L - 1; l >= 1; --l) {
        // dW_l = dZ_l H_{l-1}^T, db_l = row sums; dZ_{l-1} = (W_l^T dZ_l) * gelu'(Z_{l-1}).
        GemmArgs g = gargs();
        g.A = net->dZ(cur);
        g.lda = B;
        g.B = net->H(l - 1);
        g.ldb = B;
        g.M = W;
        g.N = W;
        g.K = B;
        g.ldo = W;
        g.Cf = net->gr() + net->off_w[l];
        MTRY(launch_gemm_bf16(false, true, EPI_STORE_F32, g, s));
        MTRY(launch_rowsum_bf16(net->dZ(cur), B, W, B, net->gr() + net->off_b[l], s));
        GemmArgs h = gargs();
        h.A = net->wb() + net->off_w[l];
        h.lda = W;
        h.B = net->dZ(cur);
        h.ldb = B;
        h.M = W;
        h.N = B;
        h.K = W;
        h.ldo = B;
        h.Zin = net->Z(l - 1);
        h.Hb = net->dZ(cur ^ 1);
        MTRY(launch_gemm_bf16(true, false, EPI_GELU_BWD, h, s));
        cur ^= 1;
    }
    MTRY(launch_layer1_wgrad(net->dZ(cur), net->xs(), B, W, B, net->gr() + net->off_w[0], s));
    MTRY(launch_rowsum_bf16(net->dZ(cur), B, W, B, net->gr() + net->off_b[0], s));
    return MRSTAT_OK;
}

mrstat_status read_loss(mrstat_mlp net, double* h_loss, hipStream_t s)
{
    if (!h_loss) return MRSTAT_OK;
    std::vector<double> part(net->n_tiles);
    MTRY(hipMemcpyAsync(part.data(), net->loss(), part.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    MTRY(hipStreamSynchronize(s));
    double t = 0.0;
    for (double v : part) t += v;
    *h_loss = t / ((double)8 * net->T * net->B);
    return MRSTAT_OK;
}

}  // namespace

namespace mrstat {

// Surrogate trains for n columns of theta rows (ln T1, ln T2, B1) with leading
// dimension ld_theta, written as [rows/T][T][ld_out] (all four trains, or the
// m train only) in chunks of the network's batch size.
hipError_t mlp_infer_trains(mrstat_mlp net, const float* theta, int64_t ld_theta, int n,
                            void* out, int64_t ld_out, int n_trains, bool f16, uint16_t* hbuf,
                            hipStream_t s)
{
    if (n_trains < 1 || n_trains > 4) return hipErrorInvalidValue;
    const int W = net->width, B = net->B, T = net->T, L = net->depth;
    if (infer_fused_supported(W, L)) {
        InferArgs a;
        std::memset(&a, 0, sizeof(a));
        a.theta = theta;
        a.ldth = ld_theta;
        a.n = n;
        a.W1 = net->w32() + net->off_w[0];
        a.b1 = net->w32() + net->off_b[0];
        for (int q = 0; q < 3; ++q) {
            a.lo[q] = net->lo[q];
            a.hi[q] = net->hi[q];
        }
        for (int l = 1; l < L; ++l) {
            a.Wh[l - 1] = net->wb() + net->off_w[l];
            a.bh[l - 1] = net->w32() + net->off_b[l];
        }
        a.n_hidden = L - 1;
        a.Wout = net->wb() + net->off_wo + (size_t)4 * T * W;   // imaginary outputs
        a.bout = net->w32() + net->off_bo + (size_t)4 * T;
        a.head_scale = net->dscale();
        a.T = T;
        a.m_out = n_trains * T;
        a.out = out;
        a.ld_out = ld_out;
        a.plane = (int64_t)T * ld_out;
        a.f16 = f16;
        if (hbuf != nullptr && W == 256) {
            a.hout = hbuf;
            const hipError_t e = launch_mlp_hidden(a, s);
            if (e != hipSuccess) return e;
            a.hout = nullptr;
            return launch_mlp_out(a, hbuf, s);
        }
        return launch_mlp_infer(W, net->infer_tile, a, s);
    }
    if (f16) return hipErrorInvalidValue;   // the chunked path writes FP32 only
    for (int c0 = 0; c0 < n; c0 += B) {
        const int nc = std::min(B, n - c0);
        if (hidden_forward(net, theta + c0, ld_theta, nc, false, s) != MRSTAT_OK) return hipErrorUnknown;
        GemmArgs g = gargs();
        g.A = net->wb() + net->off_wo + (size_t)4 * T * W;   // imaginary outputs
        g.lda = W;
        g.B = net->H(L - 1);
        g.ldb = B;
        g.M = n_trains * T;
        g.N = nc;
        g.K = W;
        g.ldo = ld_out;
        g.bias = net->w32() + net->off_bo + (size_t)4 * T;
        g.Cf = static_cast<float*>(out) + c0;
        g.T = T;
        g.plane = (int64_t)T * ld_out;
        g.head_scale = net->dscale();
        hipError_t e = launch_gemm_bf16(false, false, EPI_INFER, g, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

const float* mlp_box_lo(mrstat_mlp net) { return net->lo; }
const float* mlp_box_hi(mrstat_mlp net) { return net->hi; }
int mlp_n_tr(mrstat_mlp net) { return net->T; }
bool mlp_ready(mrstat_mlp net) { return net && net->ws != nullptr; }
bool mlp_writes_f16(mrstat_mlp net) { return infer_fused_supported(net->width, net->depth); }

}  // namespace mrstat

extern "C" {

mrstat_status mrstat_mlp_create(int32_t n_tr, int32_t width, int32_t depth, int32_t batch,
                                mrstat_mlp* out)
{
    if (!out) return MRSTAT_ERR_ARG;
    *out = nullptr;
    if (n_tr < 8 || n_tr % 8 != 0 || width < 8 || width % 64 != 0 || width > 1024 || depth < 1 ||
        depth > 16 || batch < 64 || batch % 64 != 0)
        return MRSTAT_ERR_SHAPE;
    mrstat_mlp net = new (std::nothrow) mrstat_mlp_s();
    if (!net) return MRSTAT_ERR_ARG;
    net->T = n_tr;
    net->width = width;
    net->depth = depth;
    net->B = batch;
    size_t o = 0;
    net->off_w.push_back(o); o += (size_t)width * 3;
    net->off_b.push_back(o); o += width;
    for (int l = 1; l < depth; ++l) {
        net->off_w.push_back(o); o += (size_t)width * width;
        net->off_b.push_back(o); o += width;
    }
    net->off_wo = o; o += (size_t)8 * n_tr * width;
    net->off_bo = o; o += (size_t)8 * n_tr;
    net->P = o;
    const size_t P = net->P, WB = (size_t)width * batch;
    net->n_tiles = gemm_tiles(8 * n_tr, batch);
    net->n_loss = std::max(net->n_tiles, RED_BLOCKS + 8);
    size_t w = 0;
    auto take = [&](size_t b) { size_t at = w; w = a256(w + b); return at; };
    net->o_w32 = take(P * 4);
    net->o_wb = take(P * 2);
    net->o_m = take(P * 4);
    net->o_v = take(P * 4);
    net->o_g = take(P * 4);
    net->o_z = take(depth * WB * 2);
    net->o_h = take(depth * WB * 2);
    net->o_dy = take((size_t)8 * n_tr * batch * 2);
    net->o_dz = take(2 * WB * 2);
    net->o_xs = take((size_t)3 * batch * 4);
    net->o_loss = take((size_t)net->n_loss * 8);
    net->o_scale = take(4 * 4);
    net->total = w;
    *out = net;
    return MRSTAT_OK;
}

void mrstat_mlp_destroy(mrstat_mlp net) { delete net; }

const char* mrstat_mlp_last_error(mrstat_mlp net) { return net ? net->err.c_str() : ""; }

size_t mrstat_mlp_param_count(mrstat_mlp net) { return net ? net->P : 0; }

size_t mrstat_mlp_workspace_bytes(mrstat_mlp net) { return net ? net->total : 0; }

mrstat_status mrstat_mlp_set_infer_tile(mrstat_mlp net, int32_t voxels)
{
    if (!net) return MRSTAT_ERR_ARG;
    if (!(voxels == 0 || voxels == 32 || voxels == 64 || voxels == -32 || voxels == -64))
        return mfail(net, MRSTAT_ERR_ARG, "voxels per workgroup must be 0, +-32 or +-64");
    net->infer_tile = voxels;
    return MRSTAT_OK;
}

mrstat_status mrstat_mlp_bind(mrstat_mlp net, void* d_ws, size_t ws_bytes, mrstat_stream stream)
{
    if (!net) return MRSTAT_ERR_ARG;
    if (!d_ws || ((uintptr_t)d_ws % 256) || ws_bytes < net->total)
        return mfail(net, MRSTAT_ERR_WORKSPACE, "workspace missing, misaligned or too small");
    net->ws = (char*)d_ws;
    net->ws_bytes = ws_bytes;
    hipStream_t s = (hipStream_t)stream;
    MTRY(hipMemcpyAsync(net->dscale(), net->scale, sizeof(net->scale), hipMemcpyHostToDevice, s));
    MTRY(hipStreamSynchronize(s));
    return MRSTAT_OK;
}

mrstat_status mrstat_mlp_set_scaling(mrstat_mlp net, const float box_lo[3], const float box_hi[3],
                                     const float head_scale[4], mrstat_stream stream)
{
    if (!net || !box_lo || !box_hi || !head_scale) return MRSTAT_ERR_ARG;
    for (int q = 0; q < 3; ++q)
        if (!(box_lo[q] < box_hi[q])) return mfail(net, MRSTAT_ERR_ARG, "empty box");
    for (int p = 0; p < 4; ++p)
        if (!(head_scale[p] > 0.f) || !std::isfinite(head_scale[p]))
            return mfail(net, MRSTAT_ERR_ARG, "head scales must be positive");
    std::memcpy(net->lo, box_lo, sizeof(net->lo));
    std::memcpy(net->hi, box_hi, sizeof(net->hi));
    std::memcpy(net->scale, head_scale, sizeof(net->scale));
    if (net->ws) {
        hipStream_t s = (hipStream_t)stream;
        MTRY(hipMemcpyAsync(net->dscale(), net->scale, sizeof(net->scale), hipMemcpyHostToDevice, s));
        MTRY(hipStreamSynchronize(s));
    }
    return MRSTAT_OK;
}

mrstat_status mrstat_mlp_fit_scaling(mrstat_mlp net, const float* d_trains, int64_t n,
                                     const float box_lo[3], const float box_hi[3], float h_scale_out[4],
                                     mrstat_stream stream)
{
    if (!net || !d_trains || !box_lo || !box_hi || n < 1) return MRSTAT_ERR_ARG;
    if (!net->ws) return mfail(net, MRSTAT_ERR_WORKSPACE, "network has no workspace");
    hipStream_t s = (hipStream_t)stream;
    const size_t plane = (size_t)net->T * (size_t)n;
    double ss[4];
    for (int p = 0; p < 4; ++p) {
        const float* a = d_trains + p * plane;
        MTRY(launch_dot(a, a, plane, net->loss(), net->loss() + RED_BLOCKS, s));
        MTRY(hipMemcpyAsync(&ss[p], net->loss() + RED_BLOCKS, sizeof(double), hipMemcpyDeviceToHost, s));
        MTRY(hipStreamSynchronize(s));
    }
    float hs[4];
    for (int p = 0; p < 4; ++p) {
        const double rms = std::sqrt(ss[p] / (double)plane);
        if (!(rms > 0.0) || !std::isfinite(rms))
            return mfail(net, MRSTAT_ERR_NONFINITE, "a train has zero or non-finite RMS over the data");
        hs[p] = (float)rms;
    }
    if (h_scale_out) std::memcpy(h_scale_out, hs, sizeof(hs));
    return mrstat_mlp_set_scaling(net, box_lo, box_hi, hs, stream);
}

mrstat_status mrstat_mlp_set_params(mrstat_mlp net, const float* d_params, mrstat_stream stream)
{
    if (!net || !d_params) return MRSTAT_ERR_ARG;
    if (!net->ws) return mfail(net, MRSTAT_ERR_WORKSPACE, "network has no workspace");
    hipStream_t s = (hipStream_t)stream;
    MTRY(hipMemcpyAsync(net->w32(), d_params, net->P * 4, hipMemcpyDeviceToDevice, s));
    MTRY(launch_to_bf16(net->w32(), net->wb(), net->P, s));
    MTRY(hipMemsetAsync(net->ws + net->o_m, 0, net->P * 4, s));
    MTRY(hipMemsetAsync(net->ws + net->o_v, 0, net->P * 4, s));
    net->step = 0;
    return MRSTAT_OK;
}

mrstat_status mrstat_mlp_get_params(mrstat_mlp net, float* d_params, mrstat_stream stream)
{
    if (!net || !d_params) return MRSTAT_ERR_ARG;
    if (!net->ws) return mfail(net, MRSTAT_ERR_WORKSPACE, "network has no workspace");
    MTRY(hipMemcpyAsync(d_params, net->w32(), net->P * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return MRSTAT_OK;
}

mrstat_status mrstat_mlp_gradients(mrstat_mlp net, const float* d_theta, int64_t ld_theta,
                                   const float* d_trains, int64_t ld_trains, float* d_grad,
                                   double* h_loss, mrstat_stream stream)
{
    if (!net || !d_theta || !d_trains || !d_grad) return MRSTAT_ERR_ARG;
    if (!net->ws) return mfail(net, MRSTAT_ERR_WORKSPACE, "network has no workspace");
    if (ld_theta < net->B || ld_trains < net->B) return mfail(net, MRSTAT_ERR_ARG, "leading dimension below batch");
    hipStream_t s = (hipStream_t)stream;
    mrstat_status st = forward_backward(net, d_theta, ld_theta, d_trains, ld_trains, s);
    if (st != MRSTAT_OK) return st;
    MTRY(hipMemcpyAsync(d_grad, net->gr(), net->P * 4, hipMemcpyDeviceToDevice, s));
    return read_loss(net, h_loss, s);
}

mrstat_status mrstat_mlp_train_step(mrstat_mlp net, const float* d_theta, int64_t ld_theta,
                                    const float* d_trains, int64_t ld_trains, float lr,
                                    double* h_loss, mrstat_stream stream)
{
    if (!net || !d_theta || !d_trains) return MRSTAT_ERR_ARG;
    if (!net->ws) return mfail(net, MRSTAT_ERR_WORKSPACE, "network has no workspace");
    if (ld_theta < net->B || ld_trains < net->B) return mfail(net, MRSTAT_ERR_ARG, "leading dimension below batch");
    if (!(lr > 0.f) || !std::isfinite(lr)) return mfail(net, MRSTAT_ERR_ARG, "learning rate must be positive");
    hipStream_t s = (hipStream_t)stream;
    mrstat_status st = forward_backward(net, d_theta, ld_theta, d_trains, ld_trains, s);
    if (st != MRSTAT_OK) return st;
    net->step += 1;
    MTRY(launch_adam(net->w32(), (float*)(net->ws + net->o_m), (float*)(net->ws + net->o_v), net->gr(),
                     net->wb(), net->P, lr, net->step, s));
    return read_loss(net, h_loss, s);
}

mrstat_status mrstat_mlp_predict(mrstat_mlp net, const float* d_theta, int64_t ld_theta, int32_t n,
                                 float* d_out, mrstat_stream stream)
{
    if (!net || !d_theta || !d_out || n < 1) return MRSTAT_ERR_ARG;
    if (!net->ws) return mfail(net, MRSTAT_ERR_WORKSPACE, "network has no workspace");
    if (ld_theta < n) return mfail(net, MRSTAT_ERR_ARG, "leading dimension below n");
    MTRY(mlp_infer_trains(net, d_theta, ld_theta, n, d_out, n, 4, false, nullptr, (hipStream_t)stream));
    return MRSTAT_OK;
}

}  // extern "C"
