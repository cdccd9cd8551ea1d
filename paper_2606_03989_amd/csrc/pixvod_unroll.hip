// Unrolled tracking with a checkpoint tape and the reverse sweep (C-ABI in
// include/pixvod.h, "Differentiation").
//
// Forward: the fused schedule in segments of at most ckpt_every iterations;
// every segment starts from a canonical state, which is copied to the tape
// (per-factor and fused schedules are the same iteration bit for bit, so the
// tape holds exactly the per-factor states).
// Backward, for frames and segments in reverse: recompute the segment's
// states from its checkpoint, one prologue + final pass per state, which also
// keep each state's marginals and new messages; then run the three reverse
// kernels for each state from last to first.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pixvod.h"
#include "gbp_adjoint.h"
#include "gbp_device.hpp"
#include "gbp_kernels.h"
#include "runtime_internal.h"

using namespace pv;

namespace {
constexpr int MSG_PLANES = 116;  // 4 x (eta 6, Lambda 21, normal eta, normal lambda): cotangents (FP64)
constexpr int LAM_PLANES = 88;   // 4 x (Lambda 21, normal lambda): the tape of new messages (FP32)
constexpr int MARG_PLANES = 64;  // pose marginal 21 + 6, depth marginal 2, their belief 28 + 7
constexpr int BEL_PLANES = 35;   // belief of the update: 28 + 7
constexpr int UB_PLANES = 42;
constexpr int EB_PLANES = 36;
constexpr int CB_PLANES = 29;
}  // namespace

struct pixvod_unroll {
    int H = 0, W = 0, pitch = 0;
    long plane = 0;
    pixvod_intrinsics K{};
    pixvod_params P{};
    int max_frames = 0, n_iters = 0, ckpt_every = 0, seg_per_frame = 0;
    hipStream_t own_stream = nullptr, stream = nullptr;
    float *Is = nullptr, *cxt = nullptr, *cyt = nullptr, *sig = nullptr;
    float *It = nullptr, *Gx = nullptr, *Gy = nullptr;
    float *frames = nullptr, *stage = nullptr;
    float *X0 = nullptr, *Xw[2] = {nullptr, nullptr}, *tape = nullptr, *Xend = nullptr, *seg = nullptr;
    float *var_ll = nullptr, *valid = nullptr;
    double *marg = nullptr, *bel = nullptr;
    float *Mb = nullptr, *Ub = nullptr, *Eb = nullptr;   // reverse-sweep cotangents, FP32 storage
    float* M = nullptr;
    // the reverse sweep recomputes the next segment on a side stream while
    // the current one is reversed: a second set of recompute buffers (and of
    // frame-prep planes, for segments of the next frame)
    float *seg2 = nullptr, *tmp2 = nullptr, *sink2 = nullptr, *It2 = nullptr, *Gx2 = nullptr, *Gy2 = nullptr;
    double *marg2 = nullptr, *bel2 = nullptr;
    float* M2 = nullptr;
    hipStream_t side = nullptr;
    std::vector<hipEvent_t> evs;      // two per segment of a reverse sweep

    float* Xb[2] = {nullptr, nullptr};
    float* Cb[2] = {nullptr, nullptr};   // slot-common message cotangents (with Xb)
    double *gsig = nullptr, *gN = nullptr, *gk = nullptr;
    double *partial = nullptr, *stats = nullptr, *h_stats = nullptr;
    int* health = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    int n_fwd = 0;
    double sigma_N = 0.0, huber_k = 0.0;
    bool have_kf = false;
    double fwd_ms = 0.0, bwd_ms = 0.0;
};

static int ufail(int code, const std::string& msg) {
    record_error(msg);
    return code;
}

#define UHIP(expr)                                                                     \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) return ufail(PIXVOD_EHIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

static Geo ugeo(const pixvod_unroll* u) {
    Geo g;
    g.H = u->H;
    g.W = u->W;
    g.pitch = u->pitch;
    g.plane = u->plane;
    g.fx = u->K.fx;
    g.fy = u->K.fy;
    g.cx = u->K.cx;
    g.cy = u->K.cy;
    return g;
}

static Strengths ustrengths(const pixvod_unroll* u) {
    pixvod_params P = u->P;
    Strengths s = strengths_from(P, true);
    s.lamN = 1.0 / (u->sigma_N * u->sigma_N);
    s.huber_k = u->huber_k;
    return s;
}

static Inputs uinputs(const pixvod_unroll* u) {
    Inputs in;
    in.Is = u->Is;
    in.cxt = u->cxt;
    in.cyt = u->cyt;
    in.sigD = u->sig;
    in.It = u->It;
    in.Gx = u->Gx;
    in.Gy = u->Gy;
    in.prior_ell = nullptr;
    return in;
}

static size_t state_floats(const pixvod_unroll* u) { return (size_t)N_PLANES * (size_t)u->plane; }
static float* ckpt(const pixvod_unroll* u, int f, int s) {
    return u->tape + (size_t)(f * u->seg_per_frame + s) * state_floats(u);
}
static int seg_len(const pixvod_unroll* u, int s) {
    const int rest = u->n_iters - s * u->ckpt_every;
    return rest < u->ckpt_every ? rest : u->ckpt_every;
}

template <typename T>
static bool ualloc(T** p, size_t n) {
    if (hipMalloc((void**)p, n * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        return false;
    }
    return true;
}

static void urelease(pixvod_unroll* u) {
    void* bufs[] = {u->Is, u->cxt, u->cyt, u->sig, u->It, u->Gx, u->Gy, u->frames, u->stage, u->X0, u->Xw[0],
                    u->Xw[1], u->tape, u->Xend, u->seg, u->var_ll, u->valid, u->marg, u->M, u->bel, u->Mb, u->Ub, u->Eb,
                    u->Cb[0], u->Cb[1], u->seg2, u->tmp2, u->sink2, u->It2, u->Gx2, u->Gy2, u->marg2, u->M2, u->bel2,
                    u->Xb[0], u->Xb[1], u->gsig, u->gN, u->gk, u->partial, u->stats, u->health};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (u->h_stats) (void)hipHostFree(u->h_stats);
    for (hipEvent_t e : u->ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : u->evs) (void)hipEventDestroy(e);
    if (u->side) (void)hipStreamDestroy(u->side);
    if (u->own_stream) (void)hipStreamDestroy(u->own_stream);
}

// canonical state after n fused iterations from src; returns the buffer that
// holds it (src is left unchanged when n >= 1; a and b are the work buffers)
static int fused_run(pixvod_unroll* u, const Geo& g, const Strengths& s, const Inputs& in, const float* src,
                     float* a, float* b, float* dst, int n) {
    // prologue src -> a, passes alternate a <-> b, the last one writes dst
    UHIP(launch_fu_prologue(g, s, in, src, a, u->health, u->stream));
    float* cur = a;
    for (int it = 0; it < n; ++it) {
        const bool last = (it == n - 1);
        float* nxt = last ? dst : (cur == a ? b : a);
        UHIP(launch_fu_iterate(g, s, in, cur, nxt, last, u->var_ll, u->valid, u->health, u->stream));
        cur = nxt;
    }
    return PIXVOD_OK;
}

static int stage_to(pixvod_unroll* u, const float* src, int where, size_t n, float* dst) {
    UHIP(hipMemcpyAsync(dst, src, n * sizeof(float),
                        where == PIXVOD_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, u->stream));
    return PIXVOD_OK;
}

extern "C" {

int pixvod_unroll_create(int H, int W, const pixvod_intrinsics* K, const pixvod_params* params, int max_frames,
                         int n_iters, int ckpt_every, pixvod_unroll** out) {
    if (!out) return ufail(PIXVOD_EINVAL, "out_unroll is NULL");
    *out = nullptr;
    if (H < 2 || W < 2) return ufail(PIXVOD_EINVAL, "H and W must be >= 2");
    if ((long)H * (long)W > (1L << 26)) return ufail(PIXVOD_EINVAL, "image too large");
    if (max_frames < 1 || n_iters < 1 || ckpt_every < 1)
        return ufail(PIXVOD_EINVAL, "max_frames, n_iters and ckpt_every must be >= 1");
    if (!K || !(K->fx > 0) || !(K->fy > 0) || !std::isfinite(K->cx) || !std::isfinite(K->cy))
        return ufail(PIXVOD_EINVAL, "intrinsics must be finite with fx, fy > 0");
    pixvod_params P;
    if (params) P = *params;
    else pixvod_default_params(&P);
    if (!params_valid(&P)) return ufail(PIXVOD_EINVAL, "invalid parameters");
    if (P.damping != 0.0f) return ufail(PIXVOD_EINVAL, "the unroll does not support message damping");
    if (ckpt_every > n_iters) ckpt_every = n_iters;
    const int spf = (n_iters + ckpt_every - 1) / ckpt_every;
    if ((long)max_frames * spf > 100000) return ufail(PIXVOD_EINVAL, "too many checkpoints");

    int ndev = 0, dev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return ufail(PIXVOD_ENODEV, "no HIP device available");
    if (hipGetDevice(&dev) != hipSuccess) return ufail(PIXVOD_ENODEV, "hipGetDevice failed");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return ufail(PIXVOD_ENODEV, "hipGetDeviceProperties failed");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return ufail(PIXVOD_ENODEV, std::string("device is ") + prop.gcnArchName + ", need gfx950");

    pixvod_unroll* u = new pixvod_unroll();
    u->H = H;
    u->W = W;
    u->pitch = (W + 63) / 64 * 64;
    u->plane = (long)H * u->pitch;
    u->K = *K;
    u->P = P;
    u->max_frames = max_frames;
    u->n_iters = n_iters;
    u->ckpt_every = ckpt_every;
    u->seg_per_frame = spf;
    u->sigma_N = P.sigma_N;
    u->huber_k = P.huber_k;
    const size_t pl = (size_t)u->plane, N = (size_t)H * W, S = state_floats(u);
    const int nb = stats_blocks(ugeo(u)) > sum2_blocks(ugeo(u)) ? stats_blocks(ugeo(u)) : sum2_blocks(ugeo(u));
    bool ok = ualloc(&u->Is, pl) && ualloc(&u->cxt, pl) && ualloc(&u->cyt, pl) && ualloc(&u->sig, pl) &&
              ualloc(&u->It, pl) && ualloc(&u->Gx, pl) && ualloc(&u->Gy, pl) &&
              ualloc(&u->frames, N * (size_t)max_frames) && ualloc(&u->stage, N * 4) && ualloc(&u->X0, S) &&
              ualloc(&u->Xw[0], S) && ualloc(&u->Xw[1], S) && ualloc(&u->tape, S * (size_t)max_frames * spf) &&
              ualloc(&u->Xend, S) && ualloc(&u->seg, S * (size_t)ckpt_every) && ualloc(&u->var_ll, pl) &&
              ualloc(&u->valid, pl) && ualloc(&u->marg, pl * MARG_PLANES * (size_t)ckpt_every) &&
              ualloc(&u->M, pl * LAM_PLANES * (size_t)ckpt_every) &&
              ualloc(&u->bel, pl * BEL_PLANES * (size_t)ckpt_every) &&
              ualloc(&u->Mb, pl * MSG_PLANES) && ualloc(&u->Ub, pl * UB_PLANES) && ualloc(&u->Eb, pl * EB_PLANES) &&
              ualloc(&u->Xb[0], S) && ualloc(&u->Xb[1], S) && ualloc(&u->gsig, pl) && ualloc(&u->gN, pl) &&
              ualloc(&u->gk, pl) && ualloc(&u->partial, (size_t)nb * 8) &&
              ualloc(&u->Cb[0], pl * CB_PLANES) && ualloc(&u->Cb[1], pl * CB_PLANES) &&
              ualloc(&u->seg2, S * (size_t)ckpt_every) && ualloc(&u->tmp2, S) && ualloc(&u->sink2, S) &&
              ualloc(&u->It2, pl) && ualloc(&u->Gx2, pl) && ualloc(&u->Gy2, pl) &&
              ualloc(&u->marg2, pl * MARG_PLANES * (size_t)ckpt_every) &&
              ualloc(&u->M2, pl * LAM_PLANES * (size_t)ckpt_every) &&
              ualloc(&u->bel2, pl * BEL_PLANES * (size_t)ckpt_every) &&
              ualloc(&u->stats, (size_t)max_frames * 8 + 8) && ualloc(&u->health, 1);
    if (ok) ok = hipHostMalloc((void**)&u->h_stats, ((size_t)max_frames * 8 + 8) * sizeof(double)) == hipSuccess;
    for (int k = 0; ok && k < 4; ++k) ok = hipEventCreate(&u->ev[k]) == hipSuccess;
    if (ok) ok = hipStreamCreateWithFlags(&u->own_stream, hipStreamNonBlocking) == hipSuccess;
    if (ok) ok = hipStreamCreateWithFlags(&u->side, hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
        urelease(u);
        delete u;
        return ufail(PIXVOD_ENOMEM, "unroll allocation failed (tape of " + std::to_string(max_frames * spf) +
                                        " checkpoints of " + std::to_string(S * 4) + " bytes)");
    }
    u->stream = u->own_stream;
    const float ell0 = (float)(-std::log((double)P.init_inv_depth));
    if (launch_init_state(ugeo(u), u->X0, ell0, u->stream) != hipSuccess ||
        hipMemsetAsync(u->var_ll, 0, pl * sizeof(float), u->stream) != hipSuccess ||
        hipStreamSynchronize(u->stream) != hipSuccess) {
        urelease(u);
        delete u;
        return ufail(PIXVOD_EHIP, "state initialisation failed");
    }
    *out = u;
    return PIXVOD_OK;
}

int pixvod_unroll_destroy(pixvod_unroll* u) {
    if (!u) return PIXVOD_OK;
    if (u->stream) (void)hipStreamSynchronize(u->stream);
    urelease(u);
    delete u;
    return PIXVOD_OK;
}

int pixvod_unroll_set_stream(pixvod_unroll* u, void* s) {
    if (!u) return ufail(PIXVOD_EINVAL, "unroll is NULL");
    UHIP(hipStreamSynchronize(u->stream));
    u->stream = s ? (hipStream_t)s : u->own_stream;
    return PIXVOD_OK;
}

int pixvod_unroll_set_keyframe(pixvod_unroll* u, const float* img, const float* normals, int where) {
    if (!u) return ufail(PIXVOD_EINVAL, "unroll is NULL");
    if (!img || !normals) return ufail(PIXVOD_EINVAL, "img and normals are required");
    if (where != PIXVOD_HOST && where != PIXVOD_DEVICE) return ufail(PIXVOD_EINVAL, "bad location");
    const size_t N = (size_t)u->H * u->W;
    int rc = stage_to(u, img, where, N, u->stage);
    if (!rc) rc = stage_to(u, normals, where, 3 * N, u->stage + N);
    if (rc) return rc;
    // the initial state: log-depth -log(init_inv_depth), the rest zero
    const Geo g = ugeo(u);
    const float ell0 = (float)(-std::log((double)u->P.init_inv_depth));
    UHIP(launch_init_state(g, u->X0, ell0, u->stream));
    UHIP(launch_keyframe_prep(g, u->stage, u->stage + N, u->Is, u->cxt, u->cyt, u->X0, u->Xw[0], u->stream));
    UHIP(hipStreamSynchronize(u->stream));
    u->have_kf = true;
    u->n_fwd = 0;
    return PIXVOD_OK;
}

int pixvod_unroll_set_state(pixvod_unroll* u, const float* state, int where) {
    if (!u) return ufail(PIXVOD_EINVAL, "unroll is NULL");
    if (!state) return ufail(PIXVOD_EINVAL, "state is NULL");
    if (where != PIXVOD_HOST && where != PIXVOD_DEVICE) return ufail(PIXVOD_EINVAL, "bad location");
    if (!u->have_kf) return ufail(PIXVOD_ESTATE, "pixvod_unroll_set_state before pixvod_unroll_set_keyframe");
    const size_t S = state_floats(u);
    const float* d = state;
    if (where == PIXVOD_HOST) {
        // staged through the first work buffer, which no forward pass needs kept
        UHIP(hipMemcpyAsync(u->Xw[1], state, S * sizeof(float), hipMemcpyHostToDevice, u->stream));
        d = u->Xw[1];
    }
    UHIP(launch_pack_state(ugeo(u), u->X0, const_cast<float*>(d), 0, u->stream));
    UHIP(hipStreamSynchronize(u->stream));
    u->n_fwd = 0;
    return PIXVOD_OK;
}

int pixvod_unroll_forward(pixvod_unroll* u, const float* frames, int n_frames, int where, const float* sigma_map,
                          int sigma_where, double sigma_N, double huber_k, double* xi_out, float* inv_depth_out,
                          int out_where) {
    if (!u) return ufail(PIXVOD_EINVAL, "unroll is NULL");
    if (!frames || !sigma_map) return ufail(PIXVOD_EINVAL, "frames and sigma_map are required");
    if (n_frames < 1 || n_frames > u->max_frames) return ufail(PIXVOD_EINVAL, "n_frames out of range");
    if (where != PIXVOD_HOST && where != PIXVOD_DEVICE) return ufail(PIXVOD_EINVAL, "bad location");
    if (sigma_where != PIXVOD_HOST && sigma_where != PIXVOD_DEVICE) return ufail(PIXVOD_EINVAL, "bad sigma location");
    if (inv_depth_out && out_where != PIXVOD_HOST && out_where != PIXVOD_DEVICE)
        return ufail(PIXVOD_EINVAL, "bad output location");
    if (!(sigma_N > 0.0) || !std::isfinite(sigma_N) || !(huber_k > 0.0) || !std::isfinite(huber_k))
        return ufail(PIXVOD_EINVAL, "sigma_N and huber_k must be finite and > 0");
    if (!u->have_kf) return ufail(PIXVOD_ESTATE, "pixvod_unroll_forward before pixvod_unroll_set_keyframe");
    const Geo g = ugeo(u);
    const size_t N = (size_t)u->H * u->W, S = state_floats(u);
    int rc = stage_to(u, frames, where, N * (size_t)n_frames, u->frames);
    if (!rc) rc = stage_to(u, sigma_map, sigma_where, N, u->stage);
    if (rc) return rc;
    UHIP(launch_copy_plane(g, u->stage, u->sig, u->stream));
    u->sigma_N = sigma_N;
    u->huber_k = huber_k;
    const Strengths s = ustrengths(u);
    const Inputs in = uinputs(u);
    UHIP(hipEventRecord(u->ev[0], u->stream));
    UHIP(hipMemsetAsync(u->health, 0, sizeof(int), u->stream));
    UHIP(hipMemcpyAsync(u->Xw[0], u->X0, S * sizeof(float), hipMemcpyDeviceToDevice, u->stream));
    float* cur = u->Xw[0];
    for (int f = 0; f < n_frames; ++f) {
        UHIP(launch_frame_prep(g, u->frames + N * f, u->W, u->It, u->Gx, u->Gy, u->stream));
        for (int sg = 0; sg < u->seg_per_frame; ++sg) {
            float* ck = ckpt(u, f, sg);
            UHIP(hipMemcpyAsync(ck, cur, S * sizeof(float), hipMemcpyDeviceToDevice, u->stream));
            // the tape copy is the segment's source; the result lands in cur
            rc = fused_run(u, g, s, in, ck, u->Xw[0] == cur ? u->Xw[1] : u->Xw[0], u->seg, cur, seg_len(u, sg));
            if (rc) return rc;
        }
        UHIP(launch_frame_stats(g, cur, u->valid, 0, u->partial, u->stats + 8 * f, u->stream));
        if (inv_depth_out) {
            float* dst = out_where == PIXVOD_DEVICE ? inv_depth_out + N * f : u->stage;
            UHIP(launch_outputs(g, cur, u->var_ll, 0, dst, nullptr, u->stream));
            if (out_where == PIXVOD_HOST)
                UHIP(hipMemcpyAsync(inv_depth_out + N * f, u->stage, N * sizeof(float), hipMemcpyDeviceToHost,
                                    u->stream));
        }
    }
    UHIP(hipMemcpyAsync(u->Xend, cur, S * sizeof(float), hipMemcpyDeviceToDevice, u->stream));
    UHIP(hipEventRecord(u->ev[1], u->stream));
    UHIP(hipMemcpyAsync(u->h_stats, u->stats, (size_t)n_frames * 8 * sizeof(double), hipMemcpyDeviceToHost,
                        u->stream));
    UHIP(hipStreamSynchronize(u->stream));
    float ms = 0.0f;
    UHIP(hipEventElapsedTime(&ms, u->ev[0], u->ev[1]));
    u->fwd_ms = ms;
    if (xi_out)
        for (int f = 0; f < n_frames; ++f)
            for (int k = 0; k < 6; ++k) xi_out[6 * f + k] = u->h_stats[8 * f + k] / (double)N;
    u->n_fwd = n_frames;
    return PIXVOD_OK;
}

int pixvod_unroll_backward(pixvod_unroll* u, const double* xi_bar, const float* inv_depth_bar, int where,
                           float* grad_sigma_map, int grad_where, double* grad_sigma_N, double* grad_huber_k) {
    if (!u) return ufail(PIXVOD_EINVAL, "unroll is NULL");
    if (inv_depth_bar && where != PIXVOD_HOST && where != PIXVOD_DEVICE) return ufail(PIXVOD_EINVAL, "bad location");
    if (grad_sigma_map && grad_where != PIXVOD_HOST && grad_where != PIXVOD_DEVICE)
        return ufail(PIXVOD_EINVAL, "bad gradient location");
    if (u->n_fwd < 1) return ufail(PIXVOD_ESTATE, "pixvod_unroll_backward before pixvod_unroll_forward");
    const Geo g = ugeo(u);
    const size_t N = (size_t)u->H * u->W, S = state_floats(u), pl = (size_t)u->plane;
    const int F = u->n_fwd;
    // host cotangents of the inverse-depth maps are staged one frame at a
    // time into the Mb buffer, which the reverse kernels only overwrite after
    // the frame's injection has read it (stream order)
    float* rho_stage = u->Mb;
    const Strengths s = ustrengths(u);
    const Inputs in = uinputs(u);
    UHIP(hipEventRecord(u->ev[2], u->stream));
    UHIP(hipMemsetAsync(u->Xb[0], 0, S * sizeof(float), u->stream));
    UHIP(hipMemsetAsync(u->Xb[1], 0, S * sizeof(float), u->stream));
    UHIP(hipMemsetAsync(u->Cb[0], 0, pl * CB_PLANES * sizeof(float), u->stream));
    UHIP(hipMemsetAsync(u->Cb[1], 0, pl * CB_PLANES * sizeof(float), u->stream));
    UHIP(hipMemsetAsync(u->gsig, 0, pl * sizeof(double), u->stream));
    UHIP(hipMemsetAsync(u->gN, 0, pl * sizeof(double), u->stream));
    UHIP(hipMemsetAsync(u->gk, 0, pl * sizeof(double), u->stream));

    // Segments in reverse order, item i = (frame f, segment sg). Item i is
    // recomputed on the side stream into buffer set i % 2 (frame-prep planes
    // of set f % 2) while the main stream reverses item i - 1: recompute i
    // waits for the reversal of item i - 2, the previous user of both sets,
    // and reversal i waits for recompute i.
    const int S_ = u->seg_per_frame, T = F * S_;
    struct Set {
        float *seg, *tmp, *sink;
        double* marg;
        float* M;
        double* bel;
    };
    const Set sets[2] = {{u->seg, u->Xw[0], u->Xw[1], u->marg, u->M, u->bel},
                         {u->seg2, u->tmp2, u->sink2, u->marg2, u->M2, u->bel2}};
    Inputs ins[2] = {in, in};
    ins[1].It = u->It2;
    ins[1].Gx = u->Gx2;
    ins[1].Gy = u->Gy2;
    while ((int)u->evs.size() < 2 * T + 1) {
        hipEvent_t e = nullptr;
        UHIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        u->evs.push_back(e);
    }
    hipEvent_t* evC = u->evs.data();          // recompute i done
    hipEvent_t* evR = u->evs.data() + T;      // reversal i done
    hipEvent_t ev_start = u->evs[2 * T];
    // the side stream starts after everything queued on the main stream
    UHIP(hipEventRecord(ev_start, u->stream));
    UHIP(hipStreamWaitEvent(u->side, ev_start, 0));

    auto item_f = [&](int i) { return F - 1 - i / S_; };
    auto item_sg = [&](int i) { return S_ - 1 - i % S_; };
    auto recompute = [&](int i) -> int {
        const int f = item_f(i), sg = item_sg(i);
        const Set& B = sets[i & 1];
        const Inputs& I = ins[f & 1];
        if (i >= 2) UHIP(hipStreamWaitEvent(u->side, evR[i - 2], 0));
        if (sg == S_ - 1)
            UHIP(launch_frame_prep(g, u->frames + N * f, u->W, const_cast<float*>(I.It), const_cast<float*>(I.Gx),
                                   const_cast<float*>(I.Gy), u->side));
        // states of the segment: seg[0] = checkpoint, seg[i] after i
        // iterations; the recompute also keeps, per iteration, the marginals
        // and the new messages of its source state (one prologue, then one
        // rotated pass per iteration; the last state is not needed and goes
        // to a work buffer)
        const int len = seg_len(u, sg);
        UHIP(hipMemcpyAsync(B.seg, ckpt(u, f, sg), S * sizeof(float), hipMemcpyDeviceToDevice, u->side));
        UHIP(launch_fu_segment_tape(g, s, I, B.seg, B.seg, (long)S, len, B.tmp, B.sink, B.marg,
                                    (long)(pl * MARG_PLANES), B.M, (long)(pl * LAM_PLANES), B.bel,
                                    (long)(pl * BEL_PLANES), u->var_ll, u->valid, u->health, u->side));
        UHIP(hipEventRecord(evC[i], u->side));
        return PIXVOD_OK;
    };

    int cur = 0;
    int rc = recompute(0);
    if (rc) return rc;
    for (int i = 0; i < T; ++i) {
        if (i + 1 < T) {
            rc = recompute(i + 1);
            if (rc) return rc;
        }
        const int f = item_f(i), sg = item_sg(i);
        const Set& B = sets[i & 1];
        const Inputs& I = ins[f & 1];
        if (sg == S_ - 1) {
            // the frame's output cotangents enter at its last state
            const float* xend = (f == F - 1) ? u->Xend : ckpt(u, f + 1, 0);
            PoseBar xb;
            for (int k = 0; k < 6; ++k) xb.v[k] = xi_bar ? xi_bar[6 * f + k] / (double)N : 0.0;
            const float* rb = nullptr;
            if (inv_depth_bar && where == PIXVOD_HOST) {
                UHIP(hipMemcpyAsync(rho_stage, inv_depth_bar + N * f, N * sizeof(float), hipMemcpyHostToDevice,
                                    u->stream));
                rb = rho_stage;
            } else if (inv_depth_bar) {
                rb = inv_depth_bar + N * f;
            }
            UHIP(launch_adj_inject(g, xend, u->Xb[cur], xb, rb, u->stream));
        }
        UHIP(hipStreamWaitEvent(u->stream, evC[i], 0));
        for (int k = seg_len(u, sg) - 1; k >= 0; --k) {
            const float* X = B.seg + S * k;
            const double* marg = B.marg + pl * MARG_PLANES * k;
            const float* M = B.M + pl * LAM_PLANES * k;
            const double* bel = B.bel + pl * BEL_PLANES * k;
            UHIP(launch_adj_update(g, s, I, X, M, bel, u->Xb[cur], u->Cb[cur], u->Mb, u->Ub, u->stream));
            UHIP(launch_adj_edges(g, s, I, X, marg, M, u->Mb, u->Xb[cur ^ 1], u->Eb, u->gN, u->stream));
            UHIP(launch_adj_belief(g, s, I, X, marg, u->Ub, u->Eb, u->Xb[cur ^ 1], u->Cb[cur ^ 1], u->gsig, u->gk,
                                   u->stream));
            cur ^= 1;
        }
        UHIP(hipEventRecord(evR[i], u->stream));
    }
    UHIP(launch_sum2(g, u->gN, u->gk, u->partial, u->stats, u->stream));
    if (grad_sigma_map) {
        float* dst = grad_where == PIXVOD_DEVICE ? grad_sigma_map : u->stage;
        UHIP(launch_plane_to_dense(g, u->gsig, dst, u->stream));
        if (grad_where == PIXVOD_HOST)
            UHIP(hipMemcpyAsync(grad_sigma_map, u->stage, N * sizeof(float), hipMemcpyDeviceToHost, u->stream));
    }
    UHIP(hipEventRecord(u->ev[3], u->stream));
    UHIP(hipMemcpyAsync(u->h_stats, u->stats, 2 * sizeof(double), hipMemcpyDeviceToHost, u->stream));
    UHIP(hipStreamSynchronize(u->stream));
    float ms = 0.0f;
    UHIP(hipEventElapsedTime(&ms, u->ev[2], u->ev[3]));
    u->bwd_ms = ms;
    // lamN = sigma_N^-2: d lamN / d sigma_N = -2 sigma_N^-3
    if (grad_sigma_N) *grad_sigma_N = u->h_stats[0] * (-2.0 / (u->sigma_N * u->sigma_N * u->sigma_N));
    if (grad_huber_k) *grad_huber_k = u->h_stats[1];
    return PIXVOD_OK;
}

int pixvod_unroll_last_ms(const pixvod_unroll* u, double* forward_ms, double* backward_ms) {
    if (!u) return ufail(PIXVOD_EINVAL, "unroll is NULL");
    if (forward_ms) *forward_ms = u->fwd_ms;
    if (backward_ms) *backward_ms = u->bwd_ms;
    return PIXVOD_OK;
}

}  // extern "C"
