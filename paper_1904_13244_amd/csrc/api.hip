// C ABI of libmrstat (include/mrstat.h): context, validation, workspace
// layout, per-problem tables, and the host sequencing of the kernels for the
// signal/residual, J v, Re(J^H w), the inexact Gauss-Newton step and the
// CGLS proton-density initialisation.
#include "mrstat.h"
#include "mlp_internal.h"
#include "mrstat_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace mrstat;

namespace {

constexpr double kPi = 3.14159265358979323846;

struct Layout {
    size_t trains, trial_m, upart, W, apart, r, y, vec, red, scal, seq, eytab, extab;
    size_t bf[2][2];   // B-fragment tables [direction][split-BF16, FP16]
    size_t hbuf;       // surrogate hidden activations, BF16 [nv][256]
    size_t cx, csv, cp, cth, fb, total;
    size_t ax, ay;     // non-Cartesian trajectory tables, FP64 [T][nk] (0 bytes otherwise)
    size_t ncx;        // non-Cartesian forward voxel values [T][nv] complex (0 bytes otherwise)
    size_t rdU, rdY, rdw, rdW;   // readout-dynamics term buffers (0 bytes otherwise)
    int n_red;
    YPlan yp;
    YPlan rdp;         // plan of the x-GEMMs over the readout-dynamics terms (nc Chebyshev rows)
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

struct mrstat_ctx_s {
    Dims d{};
    SeqTimes st{};
    std::vector<float2> seq;      // (flip [rad], RF sign)
    std::vector<float2> eytab;    // [T][ny]
    std::vector<float2> extab;    // [nk][nx]
    bool nc = false;              // non-Cartesian trajectory (kx, ky per sample)
    std::vector<double> ax, ay;   // [T][nk] kx / nx, ky / ny
    Layout L{};
    mrstat_enc enc = MRSTAT_ENC_FP32;
    int epg_lanes = 0;
    mrstat_mlp surr = nullptr;    // surrogate replacing the EPG inside its box (not owned)
    IsoProfile iso{};             // balanced isochromat model when iso.n > 0 (else the EPG)
    int rd_nq = 0;                // readout dynamics: power-series terms of the forward sums (0 = off)
    int rd_nc = 0;                // Chebyshev terms: rows of the x-stages, the adjoint's sums
    float rd_tmax = 0.f;          // largest |tau| of a sample, seconds
    float rd_dwell_u = 0.f;       // sample spacing in units of rd_tmax
    double rd_min_t2 = 0.0;       // T2 bound of the expansion, seconds
    double rd_max_db0 = 0.0;      // |db0| bound of the expansion, Hz
    const float* rd_db0 = nullptr;   // off-resonance map [nv] in Hz (device, caller's; null = 0)
    float db0_unit = 0.f;         // Delta B0 fitted as theta row 5 in these Hz (d.np == 6), else 0
    bool f16 = false;             // trains stored as FP16
    // bound device state
    char* ws = nullptr;
    const float2* coil = nullptr;
    const uint8_t* mask = nullptr;
    bool bound = false;
    int static_dev = -1;          // device whose static workspace this context uses (-1: none)
    uint64_t static_gen = 0;      // claim number of that binding
    bool lin_valid = false;
    int lin_ntr = 4;              // trains of the linearisation: 4, or 3 without dm/dB1
    std::string err;
    // kernel tracing
    struct Rec { int kind; hipEvent_t a, b; };
    bool prof_on = false;
    uint32_t prof_mask = 0xFFFFFFFFu;   // kernel kinds traced while profiling is on
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<Rec> recs;

    template <class T>
    T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
    void* trains() const { return ws + L.trains; }    // float or _Float16
    void* trial_m() const { return ws + L.trial_m; }
    float2* upart() const { return at<float2>(L.upart); }
    float2* W() const { return at<float2>(L.W); }
    float* apart() const { return at<float>(L.apart); }
    float2* r() const { return at<float2>(L.r); }
    float2* y() const { return at<float2>(L.y); }
    float* vec(int i) const { return at<float>(L.vec) + (size_t)i * d.np * d.nv; }
    double* red() const { return at<double>(L.red); }
    double* scal() const { return at<double>(L.scal); }
    const float2* dseq() const { return at<float2>(L.seq); }
    const float2* deytab() const { return at<float2>(L.eytab); }
    const float2* dextab() const { return at<float2>(L.extab); }
    const double* dax() const { return at<double>(L.ax); }
    float2* ncx() const { return at<float2>(L.ncx); }
    const double* day() const { return at<double>(L.ay); }
    // B-fragment table of the current encoding for direction dir (null for FP32).
    const void* bfrag(int dir) const { return enc == 0 ? nullptr : (const void*)(ws + L.bf[dir][enc - 1]); }
    int* fb_count(int slot) const { return at<int>(L.fb) + slot; }   // 0: linearisation, 1: value
    int* fb_idx() const { return at<int>(L.fb) + 64; }
    float2* rdU() const { return at<float2>(L.rdU); }
    float2* rdY() const { return at<float2>(L.rdY); }
    float2* rdw() const { return at<float2>(L.rdw); }
    float2* rdW() const { return at<float2>(L.rdW); }
    Dims rd_dims() const { Dims q = d; q.C = rd_nc * d.C; return q; }   // coils x terms as rows of the x-GEMMs
};

namespace {

thread_local std::string g_create_err;

mrstat_status fail(mrstat_ctx c, mrstat_status st, const std::string& msg)
{
    if (c)
        c->err = msg;
    else
        g_create_err = msg;
    return st;
}

#define HIP_TRY(call)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(ctx, MRSTAT_ERR_HIP, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

hipError_t next_event(mrstat_ctx ctx, hipEvent_t* e)
{
    if (ctx->ev_used == ctx->ev_pool.size()) {
        hipEvent_t ne;
        // Timing events without the system-scope fences of a default event:
        // device kernels only, so device-scope ordering is all they need.
        hipError_t st = hipEventCreateWithFlags(&ne, hipEventDisableSystemFence);
        if (st != hipSuccess) return st;
        ctx->ev_pool.push_back(ne);
    }
    *e = ctx->ev_pool[ctx->ev_used++];
    return hipSuccess;
}

// Runs one launcher, bracketed by events when tracing is on.
template <class F>
hipError_t traced(mrstat_ctx ctx, int kind, hipStream_t s, F&& launch)
{
    if (!ctx->prof_on || !((ctx->prof_mask >> kind) & 1u)) return launch();
    mrstat_ctx_s::Rec r{kind, nullptr, nullptr};
    hipError_t st = next_event(ctx, &r.a);
    if (st == hipSuccess) st = next_event(ctx, &r.b);
    if (st == hipSuccess) st = hipEventRecord(r.a, s);
    if (st != hipSuccess) return st;
    st = launch();
    if (st != hipSuccess) return st;
    st = hipEventRecord(r.b, s);
    if (st == hipSuccess) ctx->recs.push_back(r);
    return st;
}

#define TRACED(kind, call) traced(ctx, (kind), s, [&]() { return (call); })

Layout make_layout(const Dims& d, bool nc, int rd_rows = 0)
{
    Layout L{};
    L.yp = make_yplan(d);
    Dims dq = d;
    dq.C = rd_rows > 0 ? rd_rows * d.C : 1;
    L.rdp = make_yplan(dq);
    if (nc) {
        // The non-Cartesian adjoint's TR chunks replace the y-stage's in the
        // partial-sum layout the gradient assembly reads.
        const int per = ceil_div(d.T, nc_adj_chunks(d));
        L.yp.adj_chunks = ceil_div(d.T, per);
    }
    // Readout-dynamics contexts may fit Delta B0: room for six parameter rows
    // and ten partial planes per adjoint chunk.
    const size_t npmax = rd_rows > 0 ? 6 : 5, plmax = rd_rows > 0 ? 10 : 8;
    const int M = d.C * d.T;
    const int gemm_blocks = std::max(ceil_div(2 * d.nk, 64) * ceil_div(M, 64), xgemm_direct_blocks(d));
    L.n_red = std::max({3 * RED_BLOCKS, gemm_blocks, cg_partials(d), tr_partials(d), nc ? nc_fwd_blocks(d) : 0});
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
    const size_t nv = d.nv, T = d.T;
    L.trains = take(4 * T * nv * sizeof(float));
    L.trial_m = take(T * nv * sizeof(float));
    L.upart = take((size_t)std::max({L.yp.nby, L.yp.nby16, L.yp.nbyc, L.yp.nbyw}) * d.C * T * d.nx * sizeof(float2));
    L.W = take((size_t)L.yp.ksplit_adj * d.C * T * d.nx * sizeof(float2));
    L.apart = take((size_t)L.yp.adj_chunks * plmax * nv * sizeof(float));
    L.r = take((size_t)d.C * T * d.nk * sizeof(float2));
    L.y = take((size_t)d.C * T * d.nk * sizeof(float2));
    L.vec = take(6 * npmax * nv * sizeof(float));
    L.red = take((size_t)L.n_red * sizeof(double));
    L.scal = take(SCAL_DOUBLES * sizeof(double));
    L.seq = take(T * sizeof(float2));
    L.eytab = take(T * d.ny * sizeof(float2));
    L.extab = take((size_t)d.nk * d.nx * sizeof(float2));
    for (int dir = 0; dir < 2; ++dir)
        for (int e = 0; e < 2; ++e) L.bf[dir][e] = take(bfrag_bytes(d, dir, e + 1));
    L.cx = take(nv * sizeof(float2));
    L.csv = take(nv * sizeof(float2));
    L.cp = take(nv * sizeof(float2));
    L.cth = take(npmax * nv * sizeof(float));
    L.fb = take((64 + nv) * sizeof(int));
    L.hbuf = take(nv * 256 * sizeof(uint16_t));
    L.ax = take(nc ? T * d.nk * sizeof(double) : 0);
    L.ay = take(nc ? T * d.nk * sizeof(double) : 0);
    L.ncx = take(nc ? T * nv * sizeof(float2) : 0);
    const size_t nq = rd_rows > 0 ? (size_t)rd_rows * d.C : 0;   // rows per TR: coils x terms
    L.rdU = take(nq * T * d.nx * sizeof(float2));
    L.rdY = take(nq * T * d.nk * sizeof(float2));
    L.rdw = take(nq * T * d.nk * sizeof(float2));
    L.rdW = take((size_t)(nq ? L.rdp.ksplit_adj : 0) * nq * T * d.nx * sizeof(float2));
    L.total = o;
    return L;
}

// Exact phase tables: the phase index of (k, ix) is the integer
// (k - nk/2)(ix - nx/2) reduced modulo nk, so exp(-2 pi i q / nk) is evaluated
// in FP64 at a reduced argument and rounded once to FP32.
void build_tables(mrstat_ctx c, const mrstat_problem* p)
{
    const Dims& d = c->d;
    c->seq.resize(d.T);
    c->eytab.resize((size_t)d.T * d.ny);
    c->extab.resize((size_t)d.nk * d.nx);
    for (int n = 0; n < d.T; ++n) {
        const double ph = p->rf_phase_rad ? p->rf_phase_rad[n] : 0.0;
        const float sg = std::cos(ph) > 0.0 ? 1.f : -1.f;
        c->seq[n] = make_float2((float)(p->flip_deg[n] * kPi / 180.0), sg);
        const long ky = (p->ky_line ? p->ky_line[n] : n % d.ny) - d.ny / 2;
        for (int iy = 0; iy < d.ny; ++iy) {
            long q = (ky * (long)(iy - d.ny / 2)) % d.ny;
            if (q < 0) q += d.ny;
            const double a = -2.0 * kPi * (double)q / (double)d.ny;
            c->eytab[(size_t)n * d.ny + iy] = make_float2((float)std::cos(a), (float)std::sin(a));
        }
    }
    for (int k = 0; k < d.nk; ++k) {
        const long kx = k - d.nk / 2;
        for (int ix = 0; ix < d.nx; ++ix) {
            long q = (kx * (long)(ix - d.nx / 2)) % d.nk;
            if (q < 0) q += d.nk;
            const double a = -2.0 * kPi * (double)q / (double)d.nk;
            c->extab[(size_t)k * d.nx + ix] = make_float2((float)std::cos(a), (float)std::sin(a));
        }
    }
}

// The library's own workspace for callers that cannot allocate device memory
// (mrstat_bind_static). Each device the library runs on holds one copy of this
// array from the load of the code object until the process ends. In host code
// `scratch` names a host-side stand-in, never the device memory: its device
// address comes from hipGetSymbolAddress once per device (static_ws_ptr), and
// only that address is ever passed to kernels or copies.
constexpr size_t kStaticWsBytes = MRSTAT_STATIC_WORKSPACE_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticWsBytes];

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
char* g_static_ptr[kMaxDevices] = {};        // device address of `scratch` per device
uint64_t g_static_owner[kMaxDevices] = {};   // claim number of the context bound to it
uint64_t g_static_claims = 0;

// Device address of the static workspace on the current device (looked up
// once per device, with that device current). Caller holds g_static_mu.
hipError_t static_ws_ptr(int dev, char** out)
{
    if (!g_static_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_static_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_static_ptr[dev];
    return hipSuccess;
}

mrstat_status check_ready(mrstat_ctx ctx)
{
    if (!ctx) return MRSTAT_ERR_ARG;
    if (!ctx->bound) return fail(ctx, MRSTAT_ERR_WORKSPACE, "context has no workspace (mrstat_bind)");
    if (ctx->static_dev >= 0) {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (g_static_owner[ctx->static_dev] != ctx->static_gen) {
            ctx->bound = false;
            return fail(ctx, MRSTAT_ERR_STATE,
                        "the static workspace of device " + std::to_string(ctx->static_dev) +
                            " was bound to another context since (mrstat_bind_static)");
        }
    }
    return MRSTAT_OK;
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

// ----------------------------------------------------------- kernel sequences
// Trains at theta into out ([ntr][T][nv]: m, then dm/dlnT1, dm/dlnT2 and,
// with ntr = 4, dm/dB1; ntr = 1: the m train only): by the EPG, or by the
// surrogate with the EPG for the voxels outside its box (their count in
// fb_count(slot)).
mrstat_status simulate_into(mrstat_ctx ctx, const float* theta, void* out, int ntr, int slot,
                            hipStream_t s)
{
    const Dims& d = ctx->d;
    const bool tangents = ntr > 1;
    const int ntan = ntr - 1;   // tangent trains: 3, 2 or 0
    const int kind = tangents ? MRSTAT_K_EPG : MRSTAT_K_EPG_VALUE;
    if (!ctx->surr) {
        if (ctx->iso.n > 0)
            HIP_TRY(TRACED(kind, launch_iso(d, ctx->st, theta, ctx->dseq(), out, ntan, ctx->f16, ctx->iso,
                                            nullptr, nullptr, s)));
        else
            HIP_TRY(TRACED(kind, launch_epg(d, ctx->st, theta, ctx->dseq(), out, ntan, ctx->epg_lanes,
                                            ctx->f16, s)));
        return MRSTAT_OK;
    }
    const int skind = tangents ? MRSTAT_K_SURR : MRSTAT_K_SURR_VALUE;
    HIP_TRY(TRACED(skind, mlp_infer_trains(ctx->surr, theta, d.nv, d.nv, out, d.nv, ntr, ctx->f16,
                                                    ctx->at<uint16_t>(ctx->L.hbuf), s)));
    HIP_TRY(TRACED(MRSTAT_K_VECTOR, launch_box_compact(d, theta, mlp_box_lo(ctx->surr),
                                                       mlp_box_hi(ctx->surr), ctx->mask, ctx->fb_idx(),
                                                       ctx->fb_count(slot), s)));
    // A short list of scattered voxels is latency bound: spread each voxel's
    // states over the most lanes unless a split was set explicitly.
    if (ctx->iso.n > 0) {
        HIP_TRY(TRACED(kind, launch_iso(d, ctx->st, theta, ctx->dseq(), out, ntan, ctx->f16, ctx->iso,
                                        ctx->fb_idx(), ctx->fb_count(slot), s)));
        return MRSTAT_OK;
    }
    const int fb_lanes = ctx->epg_lanes ? ctx->epg_lanes : (d.K <= 8 ? 2 : d.K <= 16 ? 4 : 8);
    HIP_TRY(TRACED(kind, launch_epg_list(d, ctx->st, theta, ctx->dseq(), out, ntan, fb_lanes,
                                         ctx->f16, ctx->fb_idx(), ctx->fb_count(slot), s)));
    return MRSTAT_OK;
}

// Linearisation with all four trains (ntr = 4) or, for fits that hold B1
// fixed, without dm/dB1 (ntr = 3): their Jacobian has no B1 column, so
// that train is neither simulated nor streamed.
mrstat_status linearise(mrstat_ctx ctx, const float* theta, hipStream_t s, int ntr = 4)
{
    ctx->lin_valid = false;
    mrstat_status st = simulate_into(ctx, theta, ctx->trains(), ntr, 0, s);
    if (st != MRSTAT_OK) return st;
    ctx->lin_valid = true;
    ctx->lin_ntr = ntr;
    return MRSTAT_OK;
}

// s-type forward product into out: mode 0 r = data - s (+ f partials),
// 1 out = -J-direction signal, 2 out = s.
mrstat_status forward(mrstat_ctx ctx, int mode_y, int mode_x, const void* trains,
                      const float* theta, const float* v, const void* data, void* out,
                      double* f_out, hipStream_t s)
{
    const Dims& d = ctx->d;
    const YPlan& p = ctx->L.yp;
    if (ctx->rd_nq > 0) {
        // Readout dynamics: the term sums, their x-GEMM, the per-sample weighting.
        const int nq = ctx->rd_nq, nc = ctx->rd_nc;
        HIP_TRY(TRACED(mode_y == 0 ? MRSTAT_K_YFWD_SIG : MRSTAT_K_YFWD_JV,
                       launch_rd_fwd(d, nq, nc, mode_y, trains, ctx->f16, theta, v, ctx->coil, ctx->mask, ctx->rd_db0,
                                     ctx->db0_unit, ctx->deytab(), ctx->rdU(), ctx->st.te, ctx->rd_tmax, s)));
        HIP_TRY(TRACED(MRSTAT_K_XFWD, launch_xgemm_fwd(ctx->rd_dims(), ctx->L.rdp, ctx->enc, 2, ctx->rdU(),
                                                       ctx->dextab(), ctx->bfrag(0), nullptr, ctx->rdY(), nullptr,
                                                       nullptr, s)));
        int nred = 0;
        HIP_TRY(TRACED(MRSTAT_K_VECTOR, launch_rd_combine(d, nc, mode_x, ctx->rdY(), ctx->rd_dwell_u,
                                                          (const float2*)data, (float2*)out, ctx->red(), &nred,
                                                          s)));
        if (mode_x == 0 && f_out)
            HIP_TRY(TRACED(MRSTAT_K_VECTOR, launch_sum_partials(ctx->red(), nred, f_out, s)));
        return MRSTAT_OK;
    }
    if (ctx->nc) {
        int nred = 0;
        HIP_TRY(TRACED(MRSTAT_K_NC_FWD, launch_nc_fwd(d, ctx->enc, mode_y, mode_x, trains, ctx->f16, theta, v,
                                                      ctx->coil, ctx->mask, ctx->dax(), ctx->day(), ctx->ncx(),
                                                      (const float2*)data, (float2*)out, ctx->red(), &nred, s)));
        if (mode_x == 0 && f_out)
            HIP_TRY(TRACED(MRSTAT_K_VECTOR, launch_sum_partials(ctx->red(), nred, f_out, s)));
        return MRSTAT_OK;
    }
    int nby = 1;
    HIP_TRY(TRACED(mode_y == 0 ? MRSTAT_K_YFWD_SIG : MRSTAT_K_YFWD_JV,
                   launch_ystage_fwd(d, p, mode_y, trains, ctx->f16, theta, v, ctx->coil, ctx->mask,
                                     ctx->deytab(), ctx->upart(), &nby, s)));
    if (nby > 1) HIP_TRY(TRACED(MRSTAT_K_VECTOR, launch_usum(d, ctx->upart(), nby, s)));
    int nred = 0;
    HIP_TRY(TRACED(MRSTAT_K_XFWD, launch_xgemm_fwd(d, p, ctx->enc, mode_x, ctx->upart(),
                                                   ctx->dextab(), ctx->bfrag(0), (const float2*)data, (float2*)out,
                                                   ctx->red(), &nred, s)));
    if (mode_x == 0 && f_out)
        HIP_TRY(TRACED(MRSTAT_K_VECTOR, launch_sum_partials(ctx->red(), nred, f_out, s)));
    return MRSTAT_OK;
}

// With dir non-null the finish kernel also leaves the CG partials in
// ctx->red(): dir . g and dir . dir, with step . dir (the trust region's) or
// res . res, res . g and g . g (the one-launch CG update's). Without the
// dm/dB1 train (a linearisation with 3 trains) B1 must lie outside param_mask.
mrstat_status adjoint(mrstat_ctx ctx, const float* theta, const void* w, float* g, int param_mask,
                      hipStream_t s, const float* dir = nullptr, const float* step = nullptr,
                      const float* res = nullptr)
{
    const Dims& d = ctx->d;
    const YPlan& p = ctx->L.yp;
    const int ntr = ctx->lin_ntr;
    if (ntr < 4 && ((param_mask >> 2) & 1))
        return fail(ctx, MRSTAT_ERR_STATE, "linearisation holds no dm/dB1 train");
    if (ctx->rd_nq > 0) {
        const int nc = ctx->rd_nc;
        HIP_TRY(TRACED(MRSTAT_K_VECTOR, launch_rd_expand(d, nc, ctx->rd_dwell_u, (const float2*)w, ctx->rdw(), s)));
        HIP_TRY(TRACED(MRSTAT_K_XADJ, launch_xgemm_adj(ctx->rd_dims(), ctx->L.rdp, ctx->enc, ctx->rdw(),
                                                       ctx->dextab(), ctx->bfrag(1), ctx->rdW(), s)));
        HIP_TRY(TRACED(MRSTAT_K_YADJ, launch_rd_adj(d, nc, ntr, p.adj_chunks, ctx->trains(), ctx->f16, theta,
                                                    ctx->coil, ctx->mask, ctx->rd_db0, ctx->db0_unit, ctx->deytab(),
                                                    ctx->rdW(), ctx->apart(), ctx->st.te, ctx->rd_tmax, s)));
        HIP_TRY(TRACED(MRSTAT_K_FINISH, launch_jhw_finish(d, p, ctx->apart(), theta, ctx->mask, param_mask, g,
                                                          dir, dir ? ctx->red() : nullptr, s, step, res)));
        return MRSTAT_OK;
    }
    if (ctx->nc) {
        HIP_TRY(TRACED(MRSTAT_K_NC_ADJ, launch_nc_adj(d, ctx->enc, ntr, p.adj_chunks, ctx->trains(), ctx->f16,
                                                      ctx->coil, ctx->mask, ctx->dax(), ctx->day(),
                                                      (const float2*)w, ctx->apart(), s)));
        HIP_TRY(TRACED(MRSTAT_K_FINISH, launch_jhw_finish(d, p, ctx->apart(), theta, ctx->mask, param_mask, g,
                                                          dir, dir ? ctx->red() : nullptr, s, step, res)));
        return MRSTAT_OK;
    }
    HIP_TRY(TRACED(MRSTAT_K_XADJ, launch_xgemm_adj(d, p, ctx->enc, (const float2*)w, ctx->dextab(),
                                                   ctx->bfrag(1), ctx->W(), s)));
    HIP_TRY(TRACED(MRSTAT_K_YADJ, launch_ystage_adj(d, p, ctx->trains(), ctx->f16, ntr, ctx->coil, ctx->mask,
                                                    ctx->deytab(), ctx->W(), ctx->apart(), s)));
    HIP_TRY(TRACED(MRSTAT_K_FINISH, launch_jhw_finish(d, p, ctx->apart(), theta, ctx->mask, param_mask, g,
                                                      dir, dir ? ctx->red() : nullptr, s, step, res)));
    return MRSTAT_OK;
}

}  // namespace

namespace {

mrstat_status create_impl(const mrstat_problem* p, const double* kx, const double* ky, mrstat_ctx* out,
                          int rd_nq = 0, int rd_nc = 0)
{
    mrstat_ctx ctx = nullptr;
    if (!p || !out) return fail(nullptr, MRSTAT_ERR_ARG, "null problem or output pointer");
    *out = nullptr;
    const bool nc = kx != nullptr || ky != nullptr;
    if (nc) {
        if (!kx || !ky) return fail(nullptr, MRSTAT_ERR_ARG, "kx and ky must both be given");
        if (p->nx > 256) return fail(nullptr, MRSTAT_ERR_SHAPE, "non-Cartesian encoding needs nx <= 256");
        if (p->n_tr >= 1 && p->n_read >= 1)
            for (size_t i = 0; i < (size_t)p->n_tr * p->n_read; ++i)
                if (!std::isfinite(kx[i]) || !std::isfinite(ky[i]))
                    return fail(nullptr, MRSTAT_ERR_ARG, "non-finite trajectory coordinate");
    }
    if (!p->flip_deg) return fail(nullptr, MRSTAT_ERR_ARG, "flip_deg is NULL");
    if (p->nx < 1 || p->ny < 1 || p->n_tr < 1 || p->n_read < 1)
        return fail(nullptr, MRSTAT_ERR_SHAPE, "sizes must be positive");
    if (!nc && p->n_read < p->nx) return fail(nullptr, MRSTAT_ERR_SHAPE, "n_read must be >= nx");
    if (p->n_states < 1 || p->n_states > 64)
        return fail(nullptr, MRSTAT_ERR_SHAPE, "n_states must be in [1, 64]");
    if (p->n_coils < 1 || p->n_coils > 16)
        return fail(nullptr, MRSTAT_ERR_SHAPE, "n_coils must be in [1, 16]");
    if ((long)p->nx * p->ny > (1L << 26) || (long)p->n_tr * p->nx * p->ny > (1L << 34))
        return fail(nullptr, MRSTAT_ERR_SHAPE, "problem too large");
    if (!(std::isfinite(p->tr_s) && std::isfinite(p->te_s) && std::isfinite(p->t_inv_s)) ||
        p->tr_s <= 0.0 || p->te_s < 0.0 || p->te_s > p->tr_s || p->t_inv_s < 0.0)
        return fail(nullptr, MRSTAT_ERR_ARG, "timing must satisfy 0 <= te <= tr, tr > 0, t_inv >= 0");
    for (int n = 0; n < p->n_tr; ++n) {
        if (!std::isfinite(p->flip_deg[n])) return fail(nullptr, MRSTAT_ERR_ARG, "non-finite flip angle");
        if (!nc && p->ky_line && (p->ky_line[n] < 0 || p->ky_line[n] >= p->ny))
            return fail(nullptr, MRSTAT_ERR_ARG, "ky_line out of [0, ny)");
        if (p->rf_phase_rad) {
            const double ph = p->rf_phase_rad[n];
            if (!std::isfinite(ph)) return fail(nullptr, MRSTAT_ERR_ARG, "non-finite RF phase");
            const double sn = std::fabs(std::sin(ph));
            if (sn > 1e-9)
                return fail(nullptr, MRSTAT_ERR_UNSUPPORTED, "RF phases other than 0 or pi are not supported");
        }
    }
    ctx = new (std::nothrow) mrstat_ctx_s();
    if (!ctx) return fail(nullptr, MRSTAT_ERR_ARG, "out of host memory");
    ctx->d = Dims{p->nx, p->ny, p->nx * p->ny, p->n_tr, p->n_read, p->n_states, p->n_coils};
    ctx->st = SeqTimes{(float)p->tr_s, (float)p->te_s, (float)p->t_inv_s};
    if (nc) {
        // The Cartesian tables are built for a ky_line of n mod ny (unused).
        mrstat_problem q = *p;
        q.ky_line = nullptr;
        build_tables(ctx, &q);
        ctx->nc = true;
        const size_t ns = (size_t)p->n_tr * p->n_read;
        ctx->ax.resize(ns);
        ctx->ay.resize(ns);
        for (size_t i = 0; i < ns; ++i) {
            ctx->ax[i] = kx[i] / (double)p->nx;
            ctx->ay[i] = ky[i] / (double)p->ny;
        }
    } else {
        build_tables(ctx, p);
    }
    ctx->rd_nq = rd_nq;
    ctx->rd_nc = rd_nc;
    ctx->L = make_layout(ctx->d, nc, rd_nc);
    *out = ctx;
    return MRSTAT_OK;
}

}  // namespace

extern "C" {

mrstat_status mrstat_create(const mrstat_problem* p, mrstat_ctx* out)
{
    return create_impl(p, nullptr, nullptr, out);
}

mrstat_status mrstat_create_traj(const mrstat_problem* p, const double* kx, const double* ky, mrstat_ctx* out)
{
    if (!kx || !ky) {
        if (out) *out = nullptr;
        return fail(nullptr, MRSTAT_ERR_ARG, "kx or ky is NULL");
    }
    return create_impl(p, kx, ky, out);
}

mrstat_status mrstat_create_readout(const mrstat_problem* p, double dwell_s, double min_t2_s,
                                    double max_abs_db0_hz, mrstat_ctx* out)
{
    if (out) *out = nullptr;
    if (!p || !out) return fail(nullptr, MRSTAT_ERR_ARG, "null problem or output pointer");
    if (!(std::isfinite(dwell_s) && dwell_s > 0.0) || !(std::isfinite(min_t2_s) && min_t2_s > 0.0) ||
        !(std::isfinite(max_abs_db0_hz) && max_abs_db0_hz >= 0.0))
        return fail(nullptr, MRSTAT_ERR_ARG, "dwell and min_t2 must be positive, max_abs_db0 >= 0");
    if (p->nx > 256 || p->n_read < 2) return fail(nullptr, MRSTAT_ERR_SHAPE, "readout dynamics need nx <= 256, n_read >= 2");
    const double tmax = (double)(p->n_read / 2) * dwell_s;
    const double bound = (1.0 / min_t2_s + 2.0 * kPi * max_abs_db0_hz) * tmax;
    const int nq = rd_terms(bound), nc = rd_cheb_terms(bound);
    if (nq == 0 || nc == 0 || nc > nq)
        return fail(nullptr, MRSTAT_ERR_UNSUPPORTED, "readout too long for the expansion (|lambda| tau > bound)");
    mrstat_status st = create_impl(p, nullptr, nullptr, out, nq, nc);
    if (st != MRSTAT_OK) return st;
    mrstat_ctx c = *out;
    c->rd_tmax = (float)tmax;
    c->rd_dwell_u = (float)(dwell_s / tmax);
    c->rd_min_t2 = min_t2_s;
    c->rd_max_db0 = max_abs_db0_hz;
    return MRSTAT_OK;
}

mrstat_status mrstat_set_db0(mrstat_ctx ctx, const float* d_db0)
{
    if (!ctx) return MRSTAT_ERR_ARG;
    if (ctx->rd_nq == 0) return fail(ctx, MRSTAT_ERR_STATE, "the context models no readout dynamics");
    if (d_db0 && ctx->iso.n > 0)
        return fail(ctx, MRSTAT_ERR_STATE, "an off-resonance map needs the gradient-spoiled model");
    ctx->rd_db0 = d_db0;
    return MRSTAT_OK;
}

mrstat_status mrstat_fit_db0(mrstat_ctx ctx, double hz_per_unit)
{
    if (!ctx) return MRSTAT_ERR_ARG;
    if (ctx->rd_nq == 0) return fail(ctx, MRSTAT_ERR_STATE, "the context models no readout dynamics");
    if (!(std::isfinite(hz_per_unit) && hz_per_unit >= 0.0))
        return fail(ctx, MRSTAT_ERR_ARG, "hz_per_unit must be finite and >= 0");
    if (hz_per_unit > 0.0 && ctx->iso.n > 0)
        return fail(ctx, MRSTAT_ERR_STATE, "Delta B0 is not fitted with the balanced model");
    ctx->db0_unit = (float)hz_per_unit;
    ctx->d.np = hz_per_unit > 0.0 ? 6 : 5;
    return MRSTAT_OK;
}

mrstat_status mrstat_readout_terms(mrstat_ctx ctx, int32_t* h_terms)
{
    if (!ctx || !h_terms) return MRSTAT_ERR_ARG;
    *h_terms = ctx->rd_nq;
    return MRSTAT_OK;
}

mrstat_status mrstat_readout_cheb_terms(mrstat_ctx ctx, int32_t* h_terms)
{
    if (!ctx || !h_terms) return MRSTAT_ERR_ARG;
    *h_terms = ctx->rd_nc;
    return MRSTAT_OK;
}

void mrstat_destroy(mrstat_ctx ctx)
{
    if (!ctx) return;
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    delete ctx;
}

mrstat_status mrstat_profile_enable(mrstat_ctx ctx, int32_t on)
{
    if (!ctx) return MRSTAT_ERR_ARG;
    ctx->prof_on = on != 0;
    ctx->recs.clear();
    ctx->ev_used = 0;
    return MRSTAT_OK;
}

mrstat_status mrstat_profile_select(mrstat_ctx ctx, uint32_t kind_mask)
{
    if (!ctx) return MRSTAT_ERR_ARG;
    ctx->prof_mask = kind_mask;
    return MRSTAT_OK;
}

mrstat_status mrstat_profile_read(mrstat_ctx ctx, int32_t* h_counts, double* h_ms)
{
    if (!ctx || !h_counts || !h_ms) return MRSTAT_ERR_ARG;
    for (int k = 0; k < MRSTAT_K_COUNT; ++k) {
        h_counts[k] = 0;
        h_ms[k] = 0.0;
    }
    for (const auto& r : ctx->recs) {
        HIP_TRY(hipEventSynchronize(r.b));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
        h_counts[r.kind] += 1;
        h_ms[r.kind] += ms;
    }
    return MRSTAT_OK;
}

const char* mrstat_last_error(mrstat_ctx ctx)
{
    return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

size_t mrstat_workspace_bytes(mrstat_ctx ctx) { return ctx ? ctx->L.total : 0; }

}  // extern "C"

namespace {

// Attaches ws (at least ctx->L.total bytes, 256-byte aligned), uploads the
// tables, builds the B-fragment tables and clears the device scalars.
mrstat_status bind_impl(mrstat_ctx ctx, char* ws, const void* d_coil, const uint8_t* d_mask,
                        hipStream_t s)
{
    if (ctx->d.C > 1 && !d_coil) return fail(ctx, MRSTAT_ERR_ARG, "coil maps required when n_coils > 1");
    if (d_coil && !aligned(d_coil, 8)) return fail(ctx, MRSTAT_ERR_ARG, "coil maps must be 8-byte aligned");
    ctx->ws = ws;
    ctx->coil = (const float2*)d_coil;
    ctx->mask = d_mask;
    ctx->bound = false;
    ctx->lin_valid = false;
    HIP_TRY(hipMemcpyAsync(ctx->ws + ctx->L.seq, ctx->seq.data(), ctx->seq.size() * sizeof(float2),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(ctx->ws + ctx->L.eytab, ctx->eytab.data(),
                           ctx->eytab.size() * sizeof(float2), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(ctx->ws + ctx->L.extab, ctx->extab.data(),
                           ctx->extab.size() * sizeof(float2), hipMemcpyHostToDevice, s));
    if (ctx->nc) {
        HIP_TRY(hipMemcpyAsync(ctx->ws + ctx->L.ax, ctx->ax.data(), ctx->ax.size() * sizeof(double),
                               hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(ctx->ws + ctx->L.ay, ctx->ay.data(), ctx->ay.size() * sizeof(double),
                               hipMemcpyHostToDevice, s));
    }
    HIP_TRY(launch_build_bfrag(ctx->d, ctx->dextab(), ctx->ws + ctx->L.bf[0][0], ctx->ws + ctx->L.bf[1][0],
                               ctx->ws + ctx->L.bf[0][1], ctx->ws + ctx->L.bf[1][1], s));
    // Device scalars start from zero.
    HIP_TRY(hipMemsetAsync(ctx->ws + ctx->L.scal, 0, SCAL_DOUBLES * sizeof(double), s));
    HIP_TRY(hipStreamSynchronize(s));
    ctx->bound = true;
    return MRSTAT_OK;
}

}  // namespace

extern "C" {

mrstat_status mrstat_bind(mrstat_ctx ctx, void* d_ws, size_t ws_bytes, const void* d_coil,
                          const uint8_t* d_mask, mrstat_stream stream)
{
    if (!ctx) return MRSTAT_ERR_ARG;
    if (!d_ws) return fail(ctx, MRSTAT_ERR_WORKSPACE, "workspace pointer is NULL");
    if (!aligned(d_ws, 256)) return fail(ctx, MRSTAT_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < ctx->L.total) return fail(ctx, MRSTAT_ERR_WORKSPACE, "workspace too small");
    ctx->static_dev = -1;
    return bind_impl(ctx, (char*)d_ws, d_coil, d_mask, (hipStream_t)stream);
}

mrstat_status mrstat_bind_static(mrstat_ctx ctx, const void* d_coil, const uint8_t* d_mask,
                                 mrstat_stream stream)
{
    if (!ctx) return MRSTAT_ERR_ARG;
    if (ctx->L.total > kStaticWsBytes)
        return fail(ctx, MRSTAT_ERR_WORKSPACE,
                    "problem needs " + std::to_string(ctx->L.total) + " bytes of workspace; the static "
                    "workspace holds " + std::to_string(kStaticWsBytes) + " (use mrstat_bind)");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(ctx, MRSTAT_ERR_ARG, "device index out of range");
    char* ws = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        HIP_TRY(static_ws_ptr(dev, &ws));
        g_static_owner[dev] = ++g_static_claims;
        ctx->static_dev = dev;
        ctx->static_gen = g_static_owner[dev];
    }
    return bind_impl(ctx, ws, d_coil, d_mask, (hipStream_t)stream);
}

mrstat_status mrstat_set_encoding(mrstat_ctx ctx, mrstat_enc enc)
{
    if (!ctx) return MRSTAT_ERR_ARG;
    if (enc != MRSTAT_ENC_FP32 && enc != MRSTAT_ENC_SPLIT_BF16 && enc != MRSTAT_ENC_FP16)
        return fail(ctx, MRSTAT_ERR_ARG, "unknown encoding precision");
    if (ctx->nc && enc == MRSTAT_ENC_FP16)
        return fail(ctx, MRSTAT_ERR_UNSUPPORTED, "non-Cartesian encoding runs in FP32 or split-BF16");
    ctx->enc = enc;
    return MRSTAT_OK;
}

mrstat_status mrstat_set_train_precision(mrstat_ctx ctx, mrstat_trains prec)
{
    if (!ctx) return MRSTAT_ERR_ARG;
    if (prec != MRSTAT_TRAINS_FP32 && prec != MRSTAT_TRAINS_FP16)
        return fail(ctx, MRSTAT_ERR_ARG, "unknown train precision");
    if (prec == MRSTAT_TRAINS_FP16 && ctx->surr && !mlp_writes_f16(ctx->surr))
        return fail(ctx, MRSTAT_ERR_UNSUPPORTED,
                    "FP16 trains need a surrogate of width 64, 128 or 256 (the other widths infer in FP32)");
    ctx->f16 = prec == MRSTAT_TRAINS_FP16;
    ctx->lin_valid = false;
    return MRSTAT_OK;
}

mrstat_status mrstat_set_isochromats(mrstat_ctx ctx, int32_t n_iso, const double* h_scale,
                                     const double* h_weight)
{
    if (!ctx) return MRSTAT_ERR_ARG;
    if (n_iso < 0 || n_iso > MAX_ISOCHROMATS)
        return fail(ctx, MRSTAT_ERR_ARG, "n_iso must be in [0, 32]");
    if (n_iso > 0 && (!h_scale || !h_weight)) return fail(ctx, MRSTAT_ERR_ARG, "scale or weight is NULL");
    if (n_iso > 0 && (ctx->rd_db0 || ctx->d.np == 6))
        return fail(ctx, MRSTAT_ERR_STATE, "the balanced model takes no off-resonance map or fit");
    IsoProfile p{};
    p.n = n_iso;
    for (int q = 0; q < n_iso; ++q) {
        if (!std::isfinite(h_scale[q]) || !std::isfinite(h_weight[q]))
            return fail(ctx, MRSTAT_ERR_ARG, "non-finite isochromat scale or weight");
        p.scale[q] = (float)h_scale[q];
        p.weight[q] = (float)h_weight[q];
    }
    ctx->iso = p;
    ctx->lin_valid = false;
    return MRSTAT_OK;
}

mrstat_status mrstat_set_epg_lanes(mrstat_ctx ctx, int32_t lanes)
{
    if (!ctx) return MRSTAT_ERR_ARG;
    if (!(lanes == 0 || lanes == 1 || lanes == 2 || lanes == 4 || lanes == 8))
        return fail(ctx, MRSTAT_ERR_ARG, "lanes must be 0, 1, 2, 4 or 8");
    ctx->epg_lanes = lanes;
    return MRSTAT_OK;
}

mrstat_status mrstat_set_surrogate(mrstat_ctx ctx, mrstat_mlp net)
{
    if (!ctx) return MRSTAT_ERR_ARG;
    if (net) {
        if (!mlp_ready(net)) return fail(ctx, MRSTAT_ERR_WORKSPACE, "surrogate network has no workspace");
        if (mlp_n_tr(net) != ctx->d.T)
            return fail(ctx, MRSTAT_ERR_SHAPE, "surrogate network was built for another number of TRs");
        if (ctx->f16 && !mlp_writes_f16(net))
            return fail(ctx, MRSTAT_ERR_UNSUPPORTED,
                        "FP16 trains need a surrogate of width 64, 128 or 256 (the other widths infer in FP32)");
    }
    ctx->surr = net;
    ctx->lin_valid = false;
    return MRSTAT_OK;
}

mrstat_status mrstat_fallback_count(mrstat_ctx ctx, int32_t* h_count, mrstat_stream stream)
{
    mrstat_status st = check_ready(ctx);
    if (st != MRSTAT_OK) return st;
    if (!h_count) return fail(ctx, MRSTAT_ERR_ARG, "h_count is NULL");
    *h_count = 0;
    if (!ctx->surr || !ctx->lin_valid) return MRSTAT_OK;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(h_count, ctx->fb_count(0), sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MRSTAT_OK;
}

mrstat_status mrstat_simulate(mrstat_ctx ctx, const float* d_theta, float* d_trains,
                              mrstat_stream stream)
{
    mrstat_status st = check_ready(ctx);
    if (st != MRSTAT_OK) return st;
    if (!d_theta) return fail(ctx, MRSTAT_ERR_ARG, "theta is NULL");
    hipStream_t s = (hipStream_t)stream;
    st = linearise(ctx, d_theta, s);
    if (st != MRSTAT_OK) return st;
    if (d_trains)
        HIP_TRY(launch_trains_to_f32(ctx->trains(), ctx->f16, d_trains, (size_t)4 * ctx->d.T * ctx->d.nv, s));
    return MRSTAT_OK;
}

// need_all: the call uses every Jacobian column, so a linearisation without
// the dm/dB1 train (left by a B1-fixed GN step) is redone at the same theta.
static mrstat_status prepare(mrstat_ctx ctx, const float* d_theta, int32_t reuse, hipStream_t s,
                             bool need_all = true)
{
    mrstat_status st = check_ready(ctx);
    if (st != MRSTAT_OK) return st;
    if (!d_theta) return fail(ctx, MRSTAT_ERR_ARG, "theta is NULL");
    if (reuse) {
        if (!ctx->lin_valid) return fail(ctx, MRSTAT_ERR_STATE, "reuse requested without a linearisation");
        if (!need_all || ctx->lin_ntr == 4) return MRSTAT_OK;
    }
    return linearise(ctx, d_theta, s);
}

mrstat_status mrstat_residual(mrstat_ctx ctx, const float* d_theta, int32_t reuse,
                              const void* d_data, void* d_r, double* h_f, mrstat_stream stream)
{
    hipStream_t s = (hipStream_t)stream;
    mrstat_status st = prepare(ctx, d_theta, reuse, s, false);
    if (st != MRSTAT_OK) return st;
    if (!d_data || !d_r) return fail(ctx, MRSTAT_ERR_ARG, "data or r is NULL");
    if (!aligned(d_data, 8) || !aligned(d_r, 8)) return fail(ctx, MRSTAT_ERR_ARG, "complex arrays must be 8-byte aligned");
    double* f_dev = ctx->scal() + SC_F0;
    st = forward(ctx, 0, 0, ctx->trains(), d_theta, nullptr, d_data, d_r, f_dev, s);
    if (st != MRSTAT_OK) return st;
    if (h_f) {
        double f2 = 0.0;
        HIP_TRY(hipMemcpyAsync(&f2, f_dev, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        *h_f = 0.5 * f2;
    }
    return MRSTAT_OK;
}

mrstat_status mrstat_jv(mrstat_ctx ctx, const float* d_theta, int32_t reuse, const float* d_v,
                        void* d_out, mrstat_stream stream)
{
    hipStream_t s = (hipStream_t)stream;
    mrstat_status st = prepare(ctx, d_theta, reuse, s);
    if (st != MRSTAT_OK) return st;
    if (!d_v || !d_out) return fail(ctx, MRSTAT_ERR_ARG, "v or out is NULL");
    if (!aligned(d_out, 8)) return fail(ctx, MRSTAT_ERR_ARG, "complex arrays must be 8-byte aligned");
    return forward(ctx, 1, 1, ctx->trains(), d_theta, d_v, nullptr, d_out, nullptr, s);
}

mrstat_status mrstat_jhw(mrstat_ctx ctx, const float* d_theta, int32_t reuse, const void* d_w,
                         float* d_out, mrstat_stream stream)
{
    hipStream_t s = (hipStream_t)stream;
    mrstat_status st = prepare(ctx, d_theta, reuse, s);
    if (st != MRSTAT_OK) return st;
    if (!d_w || !d_out) return fail(ctx, MRSTAT_ERR_ARG, "w or out is NULL");
    if (!aligned(d_w, 8)) return fail(ctx, MRSTAT_ERR_ARG, "complex arrays must be 8-byte aligned");
    return adjoint(ctx, d_theta, d_w, d_out, (1 << ctx->d.np) - 1, s);
}

}  // extern "C"

namespace {

// The six-row box of the line search and the trust region: the caller's
// ln T1, ln T2, B1 intervals, the rho rows unbounded (not read), and a fitted
// Delta B0 within the readout expansion's +-max_abs_db0 Hz.
void param_box(mrstat_ctx ctx, const float* lo3, const float* hi3, float* lo6, float* hi6)
{
    for (int q = 0; q < 3; ++q) {
        lo6[q] = lo3[q];
        hi6[q] = hi3[q];
    }
    lo6[3] = lo6[4] = -INFINITY;
    hi6[3] = hi6[4] = INFINITY;
    const float b = ctx->d.np == 6 ? (float)(ctx->rd_max_db0 / ctx->db0_unit) : INFINITY;
    lo6[5] = -b;
    hi6[5] = b;
}

}  // namespace

extern "C" {

mrstat_status mrstat_gn_step(mrstat_ctx ctx, float* d_theta, const void* d_data,
                             const mrstat_gn_opts* o, mrstat_gn_report* rep, mrstat_stream stream)
{
    hipStream_t s = (hipStream_t)stream;
    mrstat_status st = check_ready(ctx);
    if (st != MRSTAT_OK) return st;
    if (!d_theta || !d_data || !o || !rep) return fail(ctx, MRSTAT_ERR_ARG, "null argument");
    if (!aligned(d_data, 8)) return fail(ctx, MRSTAT_ERR_ARG, "complex arrays must be 8-byte aligned");
    if (o->n_cg < 0 || o->n_ls_max < 1 || o->param_mask < 0 || o->param_mask >= (1 << ctx->d.np) ||
        !(o->armijo_c1 >= 0.0 && o->armijo_c1 < 1.0))
        return fail(ctx, MRSTAT_ERR_ARG, "invalid GN options");
    for (int q = 0; q < 3; ++q)
        if (!(o->lo[q] <= o->hi[q])) return fail(ctx, MRSTAT_ERR_ARG, "invalid parameter box");
    float lo6[6], hi6[6];
    param_box(ctx, o->lo, o->hi, lo6, hi6);
    if (ctx->rd_nq > 0 && ((o->param_mask >> 1) & 1) && o->lo[1] < std::log(ctx->rd_min_t2) - 1e-6)
        return fail(ctx, MRSTAT_ERR_ARG, "the ln T2 box reaches below the readout expansion's min_t2");
    std::memset(rep, 0, sizeof(*rep));
    const Dims& d = ctx->d;
    float* g = ctx->vec(0);
    float* step = ctx->vec(1);
    float* res = ctx->vec(2);
    float* dir = ctx->vec(3);
    float* q = ctx->vec(4);
    float* trial = ctx->vec(5);
    double* sc = ctx->scal();

    // Linearise at theta; r, f, g = Re(J^H r). With B1 outside param_mask the
    // Jacobian has no B1 column: no dm/dB1 train (J v in y-stage mode 3).
    const int ntr = ((o->param_mask >> 2) & 1) ? 4 : 3;
    st = linearise(ctx, d_theta, s, ntr);
    if (st != MRSTAT_OK) return st;
    st = forward(ctx, 0, 0, ctx->trains(), d_theta, nullptr, d_data, ctx->r(), sc + SC_F0, s);
    if (st != MRSTAT_OK) return st;
    st = adjoint(ctx, d_theta, ctx->r(), g, o->param_mask, s);
    if (st != MRSTAT_OK) return st;

    // CG on Re(J^H J) p = -g with device-resident FP64 scalars.
    HIP_TRY(TRACED(MRSTAT_K_VECTOR, launch_cg_init(d, g, step, res, dir, sc, ctx->red(), s)));
    for (int it = 0; it < o->n_cg; ++it) {
        st = forward(ctx, ntr == 4 ? 1 : 3, 1, ctx->trains(), d_theta, dir, nullptr, ctx->y(), nullptr, s);
        if (st != MRSTAT_OK) return st;
        st = adjoint(ctx, d_theta, ctx->y(), q, o->param_mask, s, dir, nullptr, res);
        if (st != MRSTAT_OK) return st;
        HIP_TRY(TRACED(MRSTAT_K_VECTOR, launch_cg_update(d, q, step, res, dir, sc, ctx->red(), it, s)));
    }
    // The report's scalars are read with the first line-search trial's: one
    // host synchronisation per trial. The Armijo test and the update of theta
    // run on the device.
    double hs[16];
    int32_t nfb = 0;
    HIP_TRY(hipMemcpyAsync(hs, sc, sizeof(hs), hipMemcpyDeviceToHost, s));
    if (ctx->surr) HIP_TRY(hipMemcpyAsync(&nfb, ctx->fb_count(0), sizeof(nfb), hipMemcpyDeviceToHost, s));

    // Backtracking line search on the projected step.
    float t = 1.f;
    for (int k = 0; k < o->n_ls_max; ++k) {
        HIP_TRY(TRACED(MRSTAT_K_VECTOR, launch_ls_trial_masked(d, d_theta, step, t, lo6, hi6,
                                                               o->param_mask, ctx->mask, trial, s)));
        st = simulate_into(ctx, trial, ctx->trial_m(), 1, 1, s);
        if (st != MRSTAT_OK) return st;
        st = forward(ctx, 0, 0, ctx->trial_m(), trial, nullptr, d_data, ctx->y(), sc + SC_FT, s);
        if (st != MRSTAT_OK) return st;
        HIP_TRY(TRACED(MRSTAT_K_VECTOR, launch_pred_dot(d, g, trial, d_theta, ctx->red(), sc + SC_PRED, s)));
        HIP_TRY(TRACED(MRSTAT_K_VECTOR, launch_ls_accept(d, sc, o->armijo_c1, trial, d_theta, s)));
        double h3[16];
        HIP_TRY(hipMemcpyAsync(h3, sc, sizeof(h3), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (k == 0) {
            rep->n_fallback = nfb;
            const double f0 = 0.5 * hs[SC_F0];
            rep->f0 = f0;
            rep->f1 = f0;
            rep->gnorm = std::sqrt(hs[SC_G2]);
            rep->cg_iters = (int32_t)hs[SC_ITERS];
            // A non-finite f0 or gradient fails every Armijo test, so theta
            // is unchanged here.
            if (!std::isfinite(f0) || !std::isfinite(rep->gnorm))
                return fail(ctx, MRSTAT_ERR_NONFINITE, "objective or gradient is not finite");
        }
        rep->ls_trials++;
        if (h3[SC_ACC] != 0.0) {
            rep->accepted = 1;
            rep->f1 = 0.5 * h3[SC_FT];
            rep->t = t;
            rep->step_norm = std::sqrt(h3[SC_SN]);
            ctx->lin_valid = false;
            break;
        }
        t *= 0.5f;
    }
    return MRSTAT_OK;
}

mrstat_status mrstat_tr_step(mrstat_ctx ctx, float* d_theta, const void* d_data, const mrstat_tr_opts* o,
                             double* h_delta, mrstat_tr_report* rep, mrstat_stream stream)
{
    hipStream_t s = (hipStream_t)stream;
    mrstat_status st = check_ready(ctx);
    if (st != MRSTAT_OK) return st;
    if (!d_theta || !d_data || !o || !h_delta || !rep) return fail(ctx, MRSTAT_ERR_ARG, "null argument");
    if (!aligned(d_data, 8)) return fail(ctx, MRSTAT_ERR_ARG, "complex arrays must be 8-byte aligned");
    const double delta = *h_delta;
    if (o->n_cg < 0 || o->param_mask < 0 || o->param_mask >= (1 << ctx->d.np) ||
        !(o->eta >= 0.0 && o->eta < 1.0) || !(o->delta_max > 0.0) || !std::isfinite(o->delta_max) ||
        !(delta > 0.0) || !(delta <= o->delta_max))
        return fail(ctx, MRSTAT_ERR_ARG, "invalid trust-region options or radius");
    for (int q = 0; q < 3; ++q)
        if (!(o->lo[q] <= o->hi[q])) return fail(ctx, MRSTAT_ERR_ARG, "invalid parameter box");
    float lo6[6], hi6[6];
    param_box(ctx, o->lo, o->hi, lo6, hi6);
    if (ctx->rd_nq > 0 && ((o->param_mask >> 1) & 1) && o->lo[1] < std::log(ctx->rd_min_t2) - 1e-6)
        return fail(ctx, MRSTAT_ERR_ARG, "the ln T2 box reaches below the readout expansion's min_t2");
    std::memset(rep, 0, sizeof(*rep));
    rep->delta_in = delta;
    rep->delta_out = delta;
    const Dims& d = ctx->d;
    float* g = ctx->vec(0);
    float* step = ctx->vec(1);
    float* res = ctx->vec(2);
    float* dir = ctx->vec(3);
    float* q = ctx->vec(4);
    float* trial = ctx->vec(5);
    float* sv = q;   // q is free once CG has ended
    double* sc = ctx->scal();

    // Linearise at theta; r, f, g = Re(J^H r) (no dm/dB1 train with B1 fixed).
    const int ntr = ((o->param_mask >> 2) & 1) ? 4 : 3;
    const int mode_jv = ntr == 4 ? 1 : 3;
    st = linearise(ctx, d_theta, s, ntr);
    if (st != MRSTAT_OK) return st;
    st = forward(ctx, 0, 0, ctx->trains(), d_theta, nullptr, d_data, ctx->r(), sc + SC_F0, s);
    if (st != MRSTAT_OK) return st;
    st = adjoint(ctx, d_theta, ctx->r(), g, o->param_mask, s);
    if (st != MRSTAT_OK) return st;

    // Steihaug CG inside ||p|| <= delta.
    HIP_TRY(TRACED(MRSTAT_K_VECTOR, launch_cg_init(d, g, step, res, dir, sc, ctx->red(), s)));
    HIP_TRY(TRACED(MRSTAT_K_VECTOR, launch_tr_init(sc, delta * delta, s)));
    for (int it = 0; it < o->n_cg; ++it) {
        st = forward(ctx, mode_jv, 1, ctx->trains(), d_theta, dir, nullptr, ctx->y(), nullptr, s);
        if (st != MRSTAT_OK) return st;
        st = adjoint(ctx, d_theta, ctx->y(), q, o->param_mask, s, dir, step);
        if (st != MRSTAT_OK) return st;
        HIP_TRY(TRACED(MRSTAT_K_VECTOR, launch_tr_update(d, q, step, res, dir, sc, ctx->red(), it, s)));
    }

    // Trial point reflected into the box, the model's predicted decrease at
    // s = trial - theta (g . s and |J s|^2 at the linearisation), f(trial).
    HIP_TRY(TRACED(MRSTAT_K_VECTOR, launch_tr_trial(d, d_theta, step, lo6, hi6, o->param_mask, ctx->mask,
                                                    trial, sv, sc, ctx->red(), s)));
    HIP_TRY(TRACED(MRSTAT_K_VECTOR, launch_dot(g, sv, (size_t)d.np * d.nv, ctx->red(), sc + SC_GS, s)));
    st = forward(ctx, mode_jv, 1, ctx->trains(), d_theta, sv, nullptr, ctx->y(), nullptr, s);
    if (st != MRSTAT_OK) return st;
    HIP_TRY(TRACED(MRSTAT_K_VECTOR, launch_dot_c(ctx->y(), ctx->y(), (size_t)d.C * d.T * d.nk, ctx->red(),
                                                 sc + SC_JS2, s)));
    st = simulate_into(ctx, trial, ctx->trial_m(), 1, 1, s);
    if (st != MRSTAT_OK) return st;
    st = forward(ctx, 0, 0, ctx->trial_m(), trial, nullptr, d_data, ctx->y(), sc + SC_FT, s);
    if (st != MRSTAT_OK) return st;
    HIP_TRY(TRACED(MRSTAT_K_VECTOR, launch_tr_accept(d, sc, o->eta, trial, d_theta, s)));

    double hs[48];
    int32_t nfb = 0;
    HIP_TRY(hipMemcpyAsync(hs, sc, sizeof(hs), hipMemcpyDeviceToHost, s));
    if (ctx->surr) HIP_TRY(hipMemcpyAsync(&nfb, ctx->fb_count(0), sizeof(nfb), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    rep->f0 = 0.5 * hs[SC_F0];
    rep->gnorm = std::sqrt(hs[SC_G2]);
    rep->cg_iters = (int32_t)hs[SC_ITERS];
    rep->exit_kind = (int32_t)hs[SC_EXIT];
    rep->n_reflected = (int32_t)hs[SC_NREF];
    rep->n_fallback = nfb;
    rep->pred = hs[SC_PRED];
    rep->rho = hs[SC_RHO];
    rep->step_norm = std::sqrt(hs[SC_SS]);
    rep->accepted = hs[SC_ACC] != 0.0;
    rep->f1 = rep->accepted ? 0.5 * hs[SC_FT] : rep->f0;
    // A non-finite f0 or gradient gives a ratio of -inf, so theta is
    // unchanged; the radius is kept.
    if (!std::isfinite(rep->f0) || !std::isfinite(rep->gnorm))
        return fail(ctx, MRSTAT_ERR_NONFINITE, "objective or gradient is not finite");
    const bool at_boundary = rep->exit_kind == MRSTAT_TR_BOUNDARY || rep->exit_kind == MRSTAT_TR_CURVATURE;
    double nd = delta;
    if (rep->rho < 0.25)
        nd = 0.25 * delta;
    else if (rep->rho > 0.75 && at_boundary)
        nd = std::min(2.0 * delta, o->delta_max);
    rep->delta_out = nd;
    *h_delta = nd;
    if (rep->accepted) ctx->lin_valid = false;
    return MRSTAT_OK;
}

mrstat_status mrstat_rho_init(mrstat_ctx ctx, float* d_theta, const void* d_data, int32_t n_iter,
                              mrstat_stream stream)
{
    hipStream_t s = (hipStream_t)stream;
    mrstat_status st = check_ready(ctx);
    if (st != MRSTAT_OK) return st;
    if (!d_theta || !d_data) return fail(ctx, MRSTAT_ERR_ARG, "null argument");
    if (n_iter < 0) return fail(ctx, MRSTAT_ERR_ARG, "n_iter must be >= 0");
    const Dims& d = ctx->d;
    const size_t ndata = (size_t)d.C * d.T * d.nk;
    float2* x = ctx->at<float2>(ctx->L.cx);
    float2* sv = ctx->at<float2>(ctx->L.csv);
    float2* p = ctx->at<float2>(ctx->L.cp);
    float* th = ctx->at<float>(ctx->L.cth);
    float2* res = ctx->r();
    float2* qv = ctx->y();
    double* sc = ctx->scal();

    st = linearise(ctx, d_theta, s);
    if (st != MRSTAT_OK) return st;
    // M^H w for the rho-linear map: adjoint y-stage on the m train only.
    auto adj_rho = [&](const float2* w, float2* out) -> mrstat_status {
        const YPlan& p = ctx->L.yp;
        if (ctx->rd_nq > 0) {
            const int nc = ctx->rd_nc;
            HIP_TRY(TRACED(MRSTAT_K_VECTOR, launch_rd_expand(d, nc, ctx->rd_dwell_u, w, ctx->rdw(), s)));
            HIP_TRY(TRACED(MRSTAT_K_XADJ, launch_xgemm_adj(ctx->rd_dims(), ctx->L.rdp, ctx->enc, ctx->rdw(),
                                                           ctx->dextab(), ctx->bfrag(1), ctx->rdW(), s)));
            HIP_TRY(TRACED(MRSTAT_K_YADJ, launch_rd_adj(d, nc, 1, p.adj_chunks, ctx->trains(), ctx->f16,
                                                        d_theta, ctx->coil, ctx->mask, ctx->rd_db0, ctx->db0_unit,
                                                        ctx->deytab(), ctx->rdW(), ctx->apart(), ctx->st.te,
                                                        ctx->rd_tmax, s)));
        } else if (ctx->nc) {
            HIP_TRY(TRACED(MRSTAT_K_NC_ADJ, launch_nc_adj(d, ctx->enc, 1, p.adj_chunks, ctx->trains(), ctx->f16,
                                                          ctx->coil, ctx->mask, ctx->dax(), ctx->day(), w,
                                                          ctx->apart(), s)));
        } else {
            HIP_TRY(TRACED(MRSTAT_K_XADJ, launch_xgemm_adj(d, p, ctx->enc, w, ctx->dextab(), ctx->bfrag(1),
                                                           ctx->W(), s)));
            HIP_TRY(TRACED(MRSTAT_K_YADJ, launch_ystage_adj(d, p, ctx->trains(), ctx->f16, 1, ctx->coil,
                                                            ctx->mask, ctx->deytab(), ctx->W(), ctx->apart(), s)));
        }
        HIP_TRY(TRACED(MRSTAT_K_FINISH, launch_rho_adj_finish(d, p, ctx->apart(), ctx->mask, out, s)));
        return MRSTAT_OK;
    };
    HIP_TRY(hipMemsetAsync(x, 0, d.nv * sizeof(float2), s));
    HIP_TRY(hipMemcpyAsync(res, d_data, ndata * sizeof(float2), hipMemcpyDeviceToDevice, s));
    if ((st = adj_rho(res, sv)) != MRSTAT_OK) return st;
    HIP_TRY(hipMemcpyAsync(p, sv, d.nv * sizeof(float2), hipMemcpyDeviceToDevice, s));
    HIP_TRY(launch_dot_c(sv, sv, d.nv, ctx->red(), sc + SC_STAGE, s));
    HIP_TRY(launch_cgls_scalars(sc, 0, s));
    for (int it = 0; it < n_iter; ++it) {
        HIP_TRY(launch_set_rho(d, d_theta, p, th, s));
        if ((st = forward(ctx, 0, 2, ctx->trains(), th, nullptr, nullptr, qv, nullptr, s)) != MRSTAT_OK)
            return st;
        HIP_TRY(launch_dot_c(qv, qv, ndata, ctx->red(), sc + SC_STAGE, s));
        HIP_TRY(launch_cgls_scalars(sc, 1, s));
        HIP_TRY(launch_cgls_step_x(d, x, p, sc, s));
        HIP_TRY(launch_cgls_step_r(ndata, res, qv, sc, s));
        if ((st = adj_rho(res, sv)) != MRSTAT_OK) return st;
        HIP_TRY(launch_dot_c(sv, sv, d.nv, ctx->red(), sc + SC_STAGE, s));
        HIP_TRY(launch_cgls_scalars(sc, 2, s));
        HIP_TRY(launch_cgls_dir(d, p, sv, sc, s));
    }
    HIP_TRY(launch_copy_rho_out(d, x, d_theta, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MRSTAT_OK;
}

}  // extern "C"
