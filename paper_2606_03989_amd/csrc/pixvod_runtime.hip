// Host runtime and C-ABI of libpixvod (declarations in include/pixvod.h).
//
// A context owns the FP32 state planes (two ping-pong copies of 123 planes,
// row pitch padded to 64 floats), the keyframe/frame input planes and the
// reduction buffers of one image sequence on one device, and drives the
// iteration schedules on a caller-selected HIP stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pixvod.h"
#include "gbp_device.hpp"
#include "gbp_kernels.h"
#include "gbp_transfer.h"
#include "gbp_tree.h"
#include "runtime_internal.h"

using namespace pv;

static thread_local std::string g_last_error;

struct pixvod_ctx {
    int H = 0, W = 0, pitch = 0;
    long plane = 0;
    pixvod_intrinsics K{};
    pixvod_params P{};
    int device = 0;
    hipStream_t own_stream = nullptr, stream = nullptr;
    int schedule = PIXVOD_SCHED_FUSED;
    int topology = PIXVOD_TOPO_GRID;
    float* X[2] = {nullptr, nullptr};
    float* NX[2] = {nullptr, nullptr};   // quadtree node state (ping-pong like X)
    TreeGeo tg{};
    int cur = 0;
    float *Is = nullptr, *cxt = nullptr, *cyt = nullptr, *sig = nullptr;
    float *It = nullptr, *Gx = nullptr, *Gy = nullptr;
    float* prior_ell = nullptr;      // per-pixel log-depth prior means (allocated on first use)
    bool has_prior_map = false, has_prior_pose = false;
    double prior_xi[6] = {0, 0, 0, 0, 0, 0};
    float *var_ll = nullptr, *valid = nullptr;
    float *frame_stage = nullptr, *kf_stage = nullptr, *out_stage = nullptr;
    float* dense_state = nullptr;
    unsigned* zbuf = nullptr;            // depth-transfer z-buffer (allocated on first use)
    double* marg = nullptr;
    double* msg = nullptr;
    double *partial = nullptr, *result = nullptr;
    int* health = nullptr;
    double* h_result = nullptr;
    bool have_kf = false, have_frame = false, has_sigma = false, have_track = false, have_var = false;
    double T_w_kf[16];
    double xi_last[6];
    int frames_since_kf = 0;
    std::string err;
    // kernel timing
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    struct Pending { hipEvent_t a, b; int kind; int launches; };
    std::vector<Pending> pending;
    double prof_ms[PIXVOD_PROF_KINDS] = {0, 0, 0, 0};
    int64_t prof_n[PIXVOD_PROF_KINDS] = {0, 0, 0, 0};
    // captured frame steps of the fused grid schedule, one per starting
    // buffer; `key` holds the bytes of every captured kernel argument
    struct TrackGraph {
        hipGraphExec_t exec = nullptr;
        std::vector<unsigned char> key;
        std::vector<hipEvent_t> ev;      // profiled graphs: an event pair per timed run of launches
        std::vector<int> kind, launches;
    };
    bool use_graph = false;
    std::vector<Pending> graph_pending;  // event pairs owned by a graph, read after its replay
    bool graph_events_ok = true;         // event nodes can be captured for profiling
    TrackGraph tgraph[2];
};

// ---------------------------------------------------------------------------
// helpers

static int fail(pixvod_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    g_last_error = msg;
    return code;
}

#define HIP_TRY(ctx, expr)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail((ctx), PIXVOD_EHIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

static void host_se3_exp(const double xi[6], double T[16]) {
    const double* w = xi;
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double A, B, C;
    if (th2 < 1e-2) {
        const double t4 = th2 * th2, t6 = t4 * th2, t8 = t4 * t4;
        A = 1.0 - th2 / 6.0 + t4 / 120.0 - t6 / 5040.0 + t8 / 362880.0;
        B = 0.5 - th2 / 24.0 + t4 / 720.0 - t6 / 40320.0 + t8 / 3628800.0;
        C = 1.0 / 6.0 - th2 / 120.0 + t4 / 5040.0 - t6 / 362880.0 + t8 / 39916800.0;
    } else {
        const double th = std::sqrt(th2), sh = std::sin(0.5 * th);
        A = std::sin(th) / th;
        B = 2.0 * sh * sh / th2;
        C = (th - std::sin(th)) / (th2 * th);
    }
    const double Wm[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0};
    const double W2[9] = {w[0] * w[0] - th2, w[0] * w[1], w[0] * w[2], w[1] * w[0], w[1] * w[1] - th2,
                          w[1] * w[2], w[2] * w[0], w[2] * w[1], w[2] * w[2] - th2};
    std::memset(T, 0, 16 * sizeof(double));
    for (int r = 0; r < 3; ++r) {
        double tr = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double I = (r == c) ? 1.0 : 0.0;
            T[r * 4 + c] = I + A * Wm[r * 3 + c] + B * W2[r * 3 + c];
            tr += (I + B * Wm[r * 3 + c] + C * W2[r * 3 + c]) * xi[3 + c];
        }
        T[r * 4 + 3] = tr;
    }
    T[15] = 1.0;
}

static void host_se3_inverse(const double T[16], double Ti[16]) {
    std::memset(Ti, 0, 16 * sizeof(double));
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) Ti[r * 4 + c] = T[c * 4 + r];
    for (int r = 0; r < 3; ++r)
        Ti[r * 4 + 3] = -(Ti[r * 4] * T[3] + Ti[r * 4 + 1] * T[7] + Ti[r * 4 + 2] * T[11]);
    Ti[15] = 1.0;
}

static void host_mat4_mul(const double A[16], const double B[16], double C[16]) {
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            double s = 0.0;
            for (int k = 0; k < 4; ++k) s += A[r * 4 + k] * B[k * 4 + c];
            C[r * 4 + c] = s;
        }
}

static Geo geo_of(const pixvod_ctx* c) {
    Geo g;
    g.H = c->H;
    g.W = c->W;
    g.pitch = c->pitch;
    g.plane = c->plane;
    g.fx = c->K.fx;
    g.fy = c->K.fy;
    g.cx = c->K.cx;
    g.cy = c->K.cy;
    return g;
}

static double inv_sq(float s) {
    if (std::isinf(s)) return 0.0;
    return 1.0 / ((double)s * (double)s);
}

static Inputs inputs_of(const pixvod_ctx* c) {
    Inputs in;
    in.Is = c->Is;
    in.cxt = c->cxt;
    in.cyt = c->cyt;
    in.sigD = c->sig;
    in.It = c->It;
    in.Gx = c->Gx;
    in.Gy = c->Gy;
    in.prior_ell = c->prior_ell;
    return in;
}

static bool finite_params(const pixvod_params* p) {
    const float v[] = {p->sigma_D, p->sigma_P, p->huber_k, p->init_inv_depth, p->prior_log_depth,
                       p->kf_min_valid_frac, p->damping};
    for (float x : v)
        if (!std::isfinite(x)) return false;
    for (int k = 0; k < 6; ++k)
        if (!std::isfinite(p->prior_xi[k])) return false;
    return p->sigma_D > 0 && p->sigma_P > 0 && p->sigma_R > 0 && p->sigma_N > 0 && p->huber_k > 0 &&
           p->init_inv_depth > 0 && p->damping >= 0 && p->damping < 1 && p->kf_max_frames >= 1;
}

Strengths pv::strengths_from(const pixvod_params& P, bool has_sigma_map) {
    Strengths s;
    std::memset(&s, 0, sizeof(s));
    s.lamP = inv_sq(P.sigma_P);
    s.lamR = inv_sq(P.sigma_R);
    s.lamN = inv_sq(P.sigma_N);
    s.lamD = inv_sq(P.sigma_D);
    s.inv_sigD = 1.0 / (double)P.sigma_D;
    s.huber_k = P.huber_k;
    s.prior_ell = P.prior_log_depth;
    bool ident = true;
    double xi[6];
    for (int k = 0; k < 6; ++k) {
        xi[k] = P.prior_xi[k];
        ident = ident && (xi[k] == 0.0);
    }
    double T[16], Ti[16];
    host_se3_exp(xi, T);
    host_se3_inverse(T, Ti);
    for (int r = 0; r < 3; ++r) {
        for (int cc = 0; cc < 3; ++cc) s.prior_R[r * 3 + cc] = Ti[r * 4 + cc];
        s.prior_t[r] = Ti[r * 4 + 3];
    }
    s.prior_is_identity = ident ? 1 : 0;
    s.has_sigma_map = has_sigma_map ? 1 : 0;
    return s;
}

static Strengths strengths_of(const pixvod_ctx* c) {
    Strengths s = strengths_from(c->P, c->has_sigma);
    if (c->has_prior_pose) {
        // a prior pose mean set at run time (kept in double)
        double T[16], Ti[16];
        host_se3_exp(c->prior_xi, T);
        host_se3_inverse(T, Ti);
        bool ident = true;
        for (int k = 0; k < 6; ++k) ident = ident && (c->prior_xi[k] == 0.0);
        for (int r = 0; r < 3; ++r) {
            for (int cc = 0; cc < 3; ++cc) s.prior_R[r * 3 + cc] = Ti[r * 4 + cc];
            s.prior_t[r] = Ti[r * 4 + 3];
        }
        s.prior_is_identity = ident ? 1 : 0;
    }
    s.has_prior_map = c->has_prior_map ? 1 : 0;
    return s;
}

void pv::record_error(const std::string& msg) { g_last_error = msg; }

bool pv::params_valid(const pixvod_params* p) { return finite_params(p); }

template <typename T>
static int dev_alloc(pixvod_ctx* c, T** p, size_t n) {
    if (hipMalloc((void**)p, n * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        return fail(c, PIXVOD_ENOMEM, "device allocation of " + std::to_string(n * sizeof(T)) + " bytes failed");
    }
    return PIXVOD_OK;
}

static hipEvent_t take_event(pixvod_ctx* c) {
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// records the start event of a timed launch (nullptr when not profiling)
static hipEvent_t prof_begin(pixvod_ctx* c) {
    if (!c->prof) return nullptr;
    hipEvent_t a = take_event(c);
    if (a) (void)hipEventRecord(a, c->stream);
    return a;
}

// closes a timed run of `launches` consecutive launches of one kind
static void prof_end(pixvod_ctx* c, hipEvent_t a, int kind, int launches = 1) {
    if (!a) return;
    hipEvent_t b = take_event(c);
    if (!b) {
        c->ev_pool.push_back(a);
        return;
    }
    (void)hipEventRecord(b, c->stream);
    c->pending.push_back({a, b, kind, launches});
}

// folds completed event pairs into the per-kind totals (stream must be idle)
static void prof_collect(pixvod_ctx* c) {
    for (auto& p : c->pending) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            c->prof_ms[p.kind] += ms;
            c->prof_n[p.kind] += p.launches;
        }
        c->ev_pool.push_back(p.a);
        c->ev_pool.push_back(p.b);
    }
    c->pending.clear();
    for (auto& p : c->graph_pending) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            c->prof_ms[p.kind] += ms;
            c->prof_n[p.kind] += p.launches;
        }
    }
    c->graph_pending.clear();
}

static void release(pixvod_ctx* c) {
    void* bufs[] = {c->X[0], c->X[1], c->NX[0], c->NX[1], c->Is, c->cxt, c->cyt, c->sig, c->It, c->Gx, c->Gy, c->prior_ell, c->var_ll,
                    c->valid, c->frame_stage, c->kf_stage, c->out_stage, c->dense_state, c->zbuf, c->marg, c->msg,
                    c->partial, c->result, c->health};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (c->h_result) (void)hipHostFree(c->h_result);
    for (auto& t : c->tgraph) {
        if (t.exec) (void)hipGraphExecDestroy(t.exec);
        for (hipEvent_t e : t.ev) (void)hipEventDestroy(e);
    }
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    for (auto& p : c->pending) {
        c->ev_pool.push_back(p.a);
        c->ev_pool.push_back(p.b);
    }
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
}

// ---------------------------------------------------------------------------
// the ABI

extern "C" {

void pixvod_default_params(pixvod_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->sigma_D = 5e-3f;
    p->sigma_P = 1.0f;
    p->sigma_R = 4e-4f;
    p->sigma_N = 1e-3f;
    p->huber_k = 400.0f;
    p->init_inv_depth = 1.0f;
    p->prior_log_depth = 0.0f;
    p->kf_max_frames = 150;
    p->kf_min_valid_frac = 0.5f;
    p->damping = 0.0f;
}

const char* pixvod_version(void) { return "pixvod 0.1.0 (gfx950)"; }

const char* pixvod_last_error(const pixvod_ctx* c) { return c ? c->err.c_str() : g_last_error.c_str(); }

int pixvod_create(int H, int W, const pixvod_intrinsics* K, const pixvod_params* params, pixvod_ctx** out) {
    if (!out) return fail(nullptr, PIXVOD_EINVAL, "out_ctx is NULL");
    *out = nullptr;
    if (H < 2 || W < 2) return fail(nullptr, PIXVOD_EINVAL, "H and W must be >= 2");
    if ((long)H * (long)W > (1L << 28)) return fail(nullptr, PIXVOD_EINVAL, "image too large");
    if (!K || !(K->fx > 0) || !(K->fy > 0) || !std::isfinite(K->cx) || !std::isfinite(K->cy))
        return fail(nullptr, PIXVOD_EINVAL, "intrinsics must be finite with fx, fy > 0");
    pixvod_params P;
    if (params) P = *params;
    else pixvod_default_params(&P);
    if (!finite_params(&P)) return fail(nullptr, PIXVOD_EINVAL, "invalid parameters");

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
        return fail(nullptr, PIXVOD_ENODEV, "no HIP device available");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(nullptr, PIXVOD_ENODEV, "hipGetDevice failed");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return fail(nullptr, PIXVOD_ENODEV, "hipGetDeviceProperties failed");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, PIXVOD_ENODEV, std::string("device is ") + prop.gcnArchName + ", need gfx950");

    pixvod_ctx* c = new pixvod_ctx();
    c->H = H;
    c->W = W;
    c->pitch = (W + 63) / 64 * 64;
    c->plane = (long)H * c->pitch;
    c->K = *K;
    c->P = P;
    c->device = dev;
    if (transfer_scratch_init(dev) != hipSuccess) {
        delete c;
        return fail(nullptr, PIXVOD_EHIP, "hipGetSymbolAddress of the static z-buffer failed");
    }
    c->schedule = (P.damping != 0.0f) ? PIXVOD_SCHED_PER_FACTOR : PIXVOD_SCHED_FUSED;
    std::memset(c->T_w_kf, 0, sizeof(c->T_w_kf));
    for (int k = 0; k < 4; ++k) c->T_w_kf[k * 5] = 1.0;
    std::memset(c->xi_last, 0, sizeof(c->xi_last));
    int rc = PIXVOD_OK;
    const size_t pl = (size_t)c->plane, N = (size_t)H * W;
    const int nb = stats_blocks(geo_of(c));
    if (!rc) rc = dev_alloc(c, &c->X[0], pl * N_PLANES);
    if (!rc) rc = dev_alloc(c, &c->X[1], pl * N_PLANES);
    if (!rc) rc = dev_alloc(c, &c->Is, pl);
    if (!rc) rc = dev_alloc(c, &c->cxt, pl);
    if (!rc) rc = dev_alloc(c, &c->cyt, pl);
    if (!rc) rc = dev_alloc(c, &c->sig, pl);
    if (!rc) rc = dev_alloc(c, &c->It, pl);
    if (!rc) rc = dev_alloc(c, &c->Gx, pl);
    if (!rc) rc = dev_alloc(c, &c->Gy, pl);
    if (!rc) rc = dev_alloc(c, &c->var_ll, pl);
    if (!rc) rc = dev_alloc(c, &c->valid, pl);
    if (!rc) rc = dev_alloc(c, &c->frame_stage, N);
    if (!rc) rc = dev_alloc(c, &c->kf_stage, N * 4);
    if (!rc) rc = dev_alloc(c, &c->out_stage, N * 2);
    if (!rc) rc = dev_alloc(c, &c->partial, (size_t)nb * 8);
    if (!rc) rc = dev_alloc(c, &c->result, 9);
    if (!rc) rc = dev_alloc(c, &c->health, 1);
    if (!rc && hipHostMalloc((void**)&c->h_result, 9 * sizeof(double)) != hipSuccess) rc = PIXVOD_ENOMEM;
    if (!rc && hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking) != hipSuccess) rc = PIXVOD_EHIP;
    if (rc) {
        std::string m = c->err.empty() ? "context allocation failed" : c->err;
        release(c);
        delete c;
        return fail(nullptr, rc, m);
    }
    c->stream = c->own_stream;
    const Geo g = geo_of(c);
    const float ell0 = (float)(-std::log((double)P.init_inv_depth));
    if (launch_init_state(g, c->X[0], ell0, c->stream) != hipSuccess ||
        launch_init_state(g, c->X[1], ell0, c->stream) != hipSuccess ||
        hipMemsetAsync(c->var_ll, 0, pl * sizeof(float), c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        release(c);
        delete c;
        return fail(nullptr, PIXVOD_EHIP, "state initialisation failed");
    }
    *out = c;
    return PIXVOD_OK;
}

int pixvod_destroy(pixvod_ctx* c) {
    if (!c) return PIXVOD_OK;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    release(c);
    delete c;
    return PIXVOD_OK;
}

int pixvod_set_stream(pixvod_ctx* c, void* s) {
    if (!c) return fail(nullptr, PIXVOD_EINVAL, "ctx is NULL");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->stream = s ? (hipStream_t)s : c->own_stream;
    return PIXVOD_OK;
}

int pixvod_set_schedule(pixvod_ctx* c, int schedule) {
    if (!c) return fail(nullptr, PIXVOD_EINVAL, "ctx is NULL");
    if (schedule != PIXVOD_SCHED_FUSED && schedule != PIXVOD_SCHED_PER_FACTOR)
        return fail(c, PIXVOD_EINVAL, "unknown schedule");
    if (schedule == PIXVOD_SCHED_FUSED && c->P.damping != 0.0f)
        return fail(c, PIXVOD_EINVAL, "the fused schedule does not support message damping");
    if (schedule == PIXVOD_SCHED_PER_FACTOR && c->topology == PIXVOD_TOPO_QUADTREE)
        return fail(c, PIXVOD_EINVAL, "the quadtree topology runs the fused schedule only");
    c->schedule = schedule;
    return PIXVOD_OK;
}

int pixvod_set_topology(pixvod_ctx* c, int topology) {
    if (!c) return fail(nullptr, PIXVOD_EINVAL, "ctx is NULL");
    if (topology != PIXVOD_TOPO_GRID && topology != PIXVOD_TOPO_QUADTREE)
        return fail(c, PIXVOD_EINVAL, "unknown topology");
    if (c->have_kf) return fail(c, PIXVOD_ESTATE, "the topology is set before the first keyframe");
    if (topology == PIXVOD_TOPO_QUADTREE) {
        if (c->schedule != PIXVOD_SCHED_FUSED || c->P.damping != 0.0f)
            return fail(c, PIXVOD_EINVAL, "the quadtree topology runs the fused schedule without damping");
        TreeGeo t;
        if (!make_tree_geo(c->H, c->W, (double)c->P.sigma_P, (double)c->P.sigma_R, &t))
            return fail(c, PIXVOD_EINVAL, "image too large for the quadtree");
        if (!c->NX[0]) {
            const size_t n = (size_t)TN_PLANES * (size_t)t.nplane;
            int rc = dev_alloc(c, &c->NX[0], n);
            if (!rc) rc = dev_alloc(c, &c->NX[1], n);
            if (rc) return rc;
        }
        c->tg = t;
        HIP_TRY(c, launch_tree_clear_nodes(t, c->NX[0], c->stream));
        HIP_TRY(c, launch_tree_clear_nodes(t, c->NX[1], c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    c->topology = topology;
    return PIXVOD_OK;
}

int pixvod_tree_levels(const pixvod_ctx* c, int* n_levels, int* hw) {
    if (!c || !n_levels) return fail(const_cast<pixvod_ctx*>(c), PIXVOD_EINVAL, "ctx and n_levels are required");
    const bool tree = c->topology == PIXVOD_TOPO_QUADTREE;
    *n_levels = tree ? c->tg.L + 1 : 1;
    if (hw) {
        if (!tree) {
            hw[0] = c->H;
            hw[1] = c->W;
        } else {
            for (int l = 0; l <= c->tg.L; ++l) {
                hw[2 * l] = c->tg.Hl[l];
                hw[2 * l + 1] = c->tg.Wl[l];
            }
        }
    }
    return PIXVOD_OK;
}

static int stage_in(pixvod_ctx* c, const float* src, int where, size_t n, float* stage, const float** out) {
    if (where == PIXVOD_DEVICE) {
        *out = src;
        return PIXVOD_OK;
    }
    HIP_TRY(c, hipMemcpyAsync(stage, src, n * sizeof(float), hipMemcpyHostToDevice, c->stream));
    *out = stage;
    return PIXVOD_OK;
}

int pixvod_set_keyframe(pixvod_ctx* c, const float* img, const float* normals, int where) {
    if (!c) return fail(nullptr, PIXVOD_EINVAL, "ctx is NULL");
    if (!img || !normals) return fail(c, PIXVOD_EINVAL, "img and normals are required");
    if (where != PIXVOD_HOST && where != PIXVOD_DEVICE) return fail(c, PIXVOD_EINVAL, "bad location");
    const size_t N = (size_t)c->H * c->W;
    const float *di = nullptr, *dn = nullptr;
    int rc = stage_in(c, img, where, N, c->kf_stage, &di);
    if (rc) return rc;
    rc = stage_in(c, normals, where, 3 * N, c->kf_stage + N, &dn);
    if (rc) return rc;
    const Geo g = geo_of(c);
    // the canonical state lives in X[cur]; both copies are reset (log-depth kept)
    float* Xc = c->X[c->cur];
    float* Xo = c->X[1 - c->cur];
    HIP_TRY(c, launch_keyframe_prep(g, di, dn, c->Is, c->cxt, c->cyt, Xc, Xo, c->stream));
    if (c->topology == PIXVOD_TOPO_QUADTREE) {
        HIP_TRY(c, launch_tree_clear_nodes(c->tg, c->NX[0], c->stream));
        HIP_TRY(c, launch_tree_clear_nodes(c->tg, c->NX[1], c->stream));
    }
    if (c->have_track) {
        double E[16], Ei[16], Tw[16];
        host_se3_exp(c->xi_last, E);
        host_se3_inverse(E, Ei);
        host_mat4_mul(c->T_w_kf, Ei, Tw);
        std::memcpy(c->T_w_kf, Tw, sizeof(Tw));
    }
    std::memset(c->xi_last, 0, sizeof(c->xi_last));
    // the pose prior is relative to the keyframe: back to the parameters' mean
    c->has_prior_pose = false;
    c->have_track = false;
    c->have_kf = true;
    c->have_var = false;
    c->frames_since_kf = 0;
    if (where == PIXVOD_HOST) HIP_TRY(c, hipStreamSynchronize(c->stream));
    return PIXVOD_OK;
}

int pixvod_set_keyframe_transfer(pixvod_ctx* c, const float* img, const float* normals, int where) {
    if (!c) return fail(nullptr, PIXVOD_EINVAL, "ctx is NULL");
    if (!img || !normals) return fail(c, PIXVOD_EINVAL, "img and normals are required");
    if (where != PIXVOD_HOST && where != PIXVOD_DEVICE) return fail(c, PIXVOD_EINVAL, "bad location");
    if (!c->have_track) return fail(c, PIXVOD_ESTATE, "no tracked frame since the keyframe");
    if (!c->zbuf) {
        int rc = dev_alloc(c, &c->zbuf, (size_t)c->plane);
        if (rc) return rc;
    }
    double T[16];
    host_se3_exp(c->xi_last, T);
    Pose p;
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) p.R[r * 3 + k] = T[r * 4 + k];
        p.t[r] = T[r * 4 + 3];
    }
    HIP_TRY(c, launch_depth_transfer(geo_of(c), p, c->X[c->cur], c->zbuf, c->stream));
    return pixvod_set_keyframe(c, img, normals, where);
}

int pixvod_set_keyframe_transfer_noalloc(pixvod_ctx* c, const float* img, const float* normals, int where) {
    if (!c) return fail(nullptr, PIXVOD_EINVAL, "ctx is NULL");
    if (!img || !normals) return fail(c, PIXVOD_EINVAL, "img and normals are required");
    if (where != PIXVOD_HOST && where != PIXVOD_DEVICE) return fail(c, PIXVOD_EINVAL, "bad location");
    if (!c->have_track) return fail(c, PIXVOD_ESTATE, "no tracked frame since the keyframe");
    if (c->plane > kTransferScratchMax)
        return fail(c, PIXVOD_EINVAL, "frame too large for the static z-buffer (H * pitch > 2^21)");
    unsigned* zb = transfer_scratch(c->device);
    if (!zb) return fail(c, PIXVOD_ESTATE, "static z-buffer not set up on this device");
    double T[16];
    host_se3_exp(c->xi_last, T);
    Pose p;
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) p.R[r * 3 + k] = T[r * 4 + k];
        p.t[r] = T[r * 4 + 3];
    }
    HIP_TRY(c, launch_depth_transfer(geo_of(c), p, c->X[c->cur], zb, c->stream));
    return pixvod_set_keyframe(c, img, normals, where);
}

int pixvod_set_sigma_map(pixvod_ctx* c, const float* map, int where) {
    if (!c) return fail(nullptr, PIXVOD_EINVAL, "ctx is NULL");
    if (where != PIXVOD_HOST && where != PIXVOD_DEVICE) return fail(c, PIXVOD_EINVAL, "bad location");
    if (!map) {
        c->has_sigma = false;
        return PIXVOD_OK;
    }
    const size_t N = (size_t)c->H * c->W;
    const float* d = nullptr;
    int rc = stage_in(c, map, where, N, c->frame_stage, &d);
    if (rc) return rc;
    HIP_TRY(c, launch_copy_plane(geo_of(c), d, c->sig, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->has_sigma = true;
    return PIXVOD_OK;
}

int pixvod_set_prior(pixvod_ctx* c, const double xi[6], const float* log_depth, int where) {
    if (!c) return fail(nullptr, PIXVOD_EINVAL, "ctx is NULL");
    if (log_depth && where != PIXVOD_HOST && where != PIXVOD_DEVICE) return fail(c, PIXVOD_EINVAL, "bad location");
    if (xi) {
        for (int k = 0; k < 6; ++k)
            if (!std::isfinite(xi[k])) return fail(c, PIXVOD_EINVAL, "prior pose must be finite");
        std::memcpy(c->prior_xi, xi, sizeof(c->prior_xi));
        c->has_prior_pose = true;
    }
    if (log_depth) {
        if (!c->prior_ell) {
            int rc = dev_alloc(c, &c->prior_ell, (size_t)c->plane);
            if (rc) return rc;
        }
        const size_t N = (size_t)c->H * c->W;
        const float* d = nullptr;
        int rc = stage_in(c, log_depth, where, N, c->frame_stage, &d);
        if (rc) return rc;
        HIP_TRY(c, launch_copy_plane(geo_of(c), d, c->prior_ell, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        c->has_prior_map = true;
    }
    return PIXVOD_OK;
}

int pixvod_set_prior_from_state(pixvod_ctx* c) {
    if (!c) return fail(nullptr, PIXVOD_EINVAL, "ctx is NULL");
    if (!c->have_track) return fail(c, PIXVOD_ESTATE, "no tracked frame since the keyframe");
    if (!c->prior_ell) {
        int rc = dev_alloc(c, &c->prior_ell, (size_t)c->plane);
        if (rc) return rc;
    }
    std::memcpy(c->prior_xi, c->xi_last, sizeof(c->prior_xi));
    c->has_prior_pose = true;
    HIP_TRY(c, hipMemcpyAsync(c->prior_ell, c->X[c->cur] + (size_t)P_ELL * c->plane, (size_t)c->plane * sizeof(float),
                              hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->has_prior_map = true;
    return PIXVOD_OK;
}

static int stage_frame(pixvod_ctx* c, const float* frame, int where) {
    const size_t N = (size_t)c->H * c->W;
    const float* d = nullptr;
    int rc = stage_in(c, frame, where, N, c->frame_stage, &d);
    if (rc) return rc;
    HIP_TRY(c, launch_frame_prep(geo_of(c), d, c->W, c->It, c->Gx, c->Gy, c->stream, c->health));
    c->have_frame = true;
    return PIXVOD_OK;
}

static int run_iterations(pixvod_ctx* c, int n) {
    if (n <= 0) return PIXVOD_OK;
    const Geo g = geo_of(c);
    const Strengths s = strengths_of(c);
    const Inputs in = inputs_of(c);
    if (c->topology == PIXVOD_TOPO_QUADTREE) {
        int src = c->cur, dst = 1 - c->cur;
        hipEvent_t a = prof_begin(c);
        HIP_TRY(c, launch_tree_prologue(g, c->tg, s, in, c->X[src], c->NX[src], c->X[dst], c->NX[dst], c->health,
                                        c->stream));
        prof_end(c, a, PIXVOD_PROF_FUSED_PROLOGUE);
        src = dst;
        // one event pair around the n - 1 passes of a kind, one around the last
        a = n > 1 ? prof_begin(c) : nullptr;
        for (int it = 0; it < n; ++it) {
            dst = 1 - src;
            const bool last = (it == n - 1);
            if (last) {
                prof_end(c, a, PIXVOD_PROF_FUSED_ITERATE, n - 1);
                a = prof_begin(c);
            }
            HIP_TRY(c, launch_tree_iterate(g, c->tg, s, in, c->X[src], c->NX[src], c->X[dst], c->NX[dst], last,
                                           c->var_ll, c->valid, c->health, c->stream));
            src = dst;
        }
        prof_end(c, a, PIXVOD_PROF_FUSED_FINAL);
        c->cur = src;
    } else if (c->schedule == PIXVOD_SCHED_PER_FACTOR) {
        const size_t pl = (size_t)c->plane;
        if (!c->marg) {
            int rc = dev_alloc(c, &c->marg, pl * 29);
            if (rc) return rc;
        }
        if (!c->msg) {
            int rc = dev_alloc(c, &c->msg, pl * 116);
            if (rc) return rc;
        }
        hipEvent_t a = prof_begin(c);
        for (int it = 0; it < n; ++it)
            HIP_TRY(c, launch_pf_iteration(g, s, in, c->X[c->cur], c->marg, c->msg, c->var_ll, c->valid,
                                           c->P.damping, c->health, c->stream));
        prof_end(c, a, PIXVOD_PROF_PER_FACTOR, n);
    } else {
        int src = c->cur, dst = 1 - c->cur;
        hipEvent_t a = prof_begin(c);
        HIP_TRY(c, launch_fu_prologue(g, s, in, c->X[src], c->X[dst], c->health, c->stream));
        prof_end(c, a, PIXVOD_PROF_FUSED_PROLOGUE);
        src = dst;
        a = n > 1 ? prof_begin(c) : nullptr;
        for (int it = 0; it < n; ++it) {
            dst = 1 - src;
            const bool last = (it == n - 1);
            if (last) {
                prof_end(c, a, PIXVOD_PROF_FUSED_ITERATE, n - 1);
                a = prof_begin(c);
            }
            HIP_TRY(c, launch_fu_iterate(g, s, in, c->X[src], c->X[dst], last, c->var_ll, c->valid,
                                         c->health, c->stream));
            src = dst;
        }
        prof_end(c, a, PIXVOD_PROF_FUSED_FINAL);
        c->cur = src;
    }
    c->have_var = true;
    return PIXVOD_OK;
}

// ---------------------------------------------------------------------------
// the fused grid schedule's frame step as a replayed HIP graph: health word
// cleared, prologue, n passes, frame reductions (one graph per starting buffer)

static void key_bytes(std::vector<unsigned char>& k, const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    k.insert(k.end(), b, b + n);
}
#define key_put(k, v) key_bytes((k), &(v), sizeof(v))

// the bytes of every argument the captured launches take (field by field, so
// that struct padding plays no part): a graph is replayed only while they are
// unchanged
static std::vector<unsigned char> track_graph_key(const pixvod_ctx* c, int n_iters) {
    std::vector<unsigned char> k;
    const Geo g = geo_of(c);
    key_put(k, g.H);
    key_put(k, g.W);
    key_put(k, g.pitch);
    key_put(k, g.plane);
    key_put(k, g.fx);
    key_put(k, g.fy);
    key_put(k, g.cx);
    key_put(k, g.cy);
    const Strengths s = strengths_of(c);
    key_put(k, s.lamP);
    key_put(k, s.lamR);
    key_put(k, s.lamN);
    key_put(k, s.lamD);
    key_put(k, s.inv_sigD);
    key_put(k, s.huber_k);
    key_put(k, s.prior_ell);
    key_put(k, s.prior_R);
    key_put(k, s.prior_t);
    key_put(k, s.prior_is_identity);
    key_put(k, s.has_sigma_map);
    key_put(k, s.has_prior_map);
    const Inputs in = inputs_of(c);
    const void* ptrs[] = {in.Is,     in.cxt,   in.cyt,      in.sigD,   in.It,     in.Gx,       in.Gy,
                          in.prior_ell, c->X[0], c->X[1], c->var_ll, c->valid, c->health, c->partial,
                          c->result};
    key_put(k, ptrs);
    key_put(k, n_iters);
    key_put(k, c->prof);
    return k;
}
#undef key_put

static int track_graph_capture(pixvod_ctx* c, pixvod_ctx::TrackGraph& t, int src, int n_iters, bool events) {
    const Geo g = geo_of(c);
    const Strengths s = strengths_of(c);
    const Inputs in = inputs_of(c);
    const size_t n_ev = events ? 6 : 0;
    while (t.ev.size() < n_ev) {
        hipEvent_t e = nullptr;
        HIP_TRY(c, hipEventCreate(&e));
        t.ev.push_back(e);
    }
    t.kind.clear();
    t.launches.clear();
    HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    hipError_t le = launch_set_ints(c->health, 1, 0, c->stream);
    size_t e = 0;
    auto mark = [&]() {
        if (events && le == hipSuccess) le = hipEventRecordWithFlags(t.ev[e++], c->stream, hipEventRecordExternal);
    };
    // an event pair around the prologue, the n - 1 passes and the last pass
    mark();
    if (le == hipSuccess) le = launch_fu_prologue(g, s, in, c->X[src], c->X[1 - src], c->health, c->stream);
    mark();
    t.kind.push_back(PIXVOD_PROF_FUSED_PROLOGUE);
    t.launches.push_back(1);
    int cur = 1 - src;
    if (n_iters > 1) mark();
    for (int it = 0; it < n_iters; ++it) {
        const bool last = (it == n_iters - 1);
        if (last && n_iters > 1) {
            mark();
            t.kind.push_back(PIXVOD_PROF_FUSED_ITERATE);
            t.launches.push_back(n_iters - 1);
        }
        if (last) mark();
        if (le == hipSuccess)
            le = launch_fu_iterate(g, s, in, c->X[cur], c->X[1 - cur], last, c->var_ll, c->valid, c->health,
                                   c->stream);
        cur = 1 - cur;
    }
    mark();
    t.kind.push_back(PIXVOD_PROF_FUSED_FINAL);
    t.launches.push_back(1);
    if (le == hipSuccess)
        le = launch_frame_stats(g, c->X[cur], c->valid, 1, c->partial, c->result, c->stream, c->health);
    hipGraph_t gr = nullptr;
    const hipError_t ce = hipStreamEndCapture(c->stream, &gr);
    if (le != hipSuccess || ce != hipSuccess) {
        if (gr) (void)hipGraphDestroy(gr);
        return fail(c, PIXVOD_EHIP, std::string("frame step capture failed: ") +
                                        hipGetErrorString(le != hipSuccess ? le : ce));
    }
    const hipError_t ie = hipGraphInstantiate(&t.exec, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (ie != hipSuccess) {
        t.exec = nullptr;
        return fail(c, PIXVOD_EHIP, std::string("frame step instantiation failed: ") + hipGetErrorString(ie));
    }
    return PIXVOD_OK;
}

// one frame step by graph replay; *used = false when it fell back to
// run_iterations (profiling without capturable event nodes)
static int track_graph_run(pixvod_ctx* c, int n_iters, bool* used) {
    *used = false;
    if (c->prof && !c->graph_events_ok) return PIXVOD_OK;
    pixvod_ctx::TrackGraph& t = c->tgraph[c->cur];
    std::vector<unsigned char> key = track_graph_key(c, n_iters);
    if (!t.exec || t.key != key) {
        if (t.exec) {
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            (void)hipGraphExecDestroy(t.exec);
            t.exec = nullptr;
        }
        t.key.clear();
        int rc = track_graph_capture(c, t, c->cur, n_iters, c->prof);
        if (rc && c->prof) {
            // event nodes not capturable here: profiled frames run unrolled
            c->graph_events_ok = false;
            (void)hipGetLastError();
            return PIXVOD_OK;
        }
        if (rc) return rc;
        t.key.swap(key);
    }
    HIP_TRY(c, hipGraphLaunch(t.exec, c->stream));
    if (c->prof)
        for (size_t i = 0; i < t.kind.size(); ++i)
            c->graph_pending.push_back({t.ev[2 * i], t.ev[2 * i + 1], t.kind[i], t.launches[i]});
    c->cur ^= (n_iters + 1) & 1;
    c->have_var = true;
    *used = true;
    return PIXVOD_OK;
}

int pixvod_iterate(pixvod_ctx* c, int n) {
    if (!c) return fail(nullptr, PIXVOD_EINVAL, "ctx is NULL");
    if (n < 0) return fail(c, PIXVOD_EINVAL, "n_iters must be >= 0");
    if (!c->have_kf || !c->have_frame) return fail(c, PIXVOD_ESTATE, "no keyframe or frame staged");
    return run_iterations(c, n);
}

int pixvod_track(pixvod_ctx* c, const float* frame, int where, int n_iters, pixvod_track_out* out) {
    if (!c) return fail(nullptr, PIXVOD_EINVAL, "ctx is NULL");
    if (!frame || !out) return fail(c, PIXVOD_EINVAL, "frame and out are required");
    if (where != PIXVOD_HOST && where != PIXVOD_DEVICE) return fail(c, PIXVOD_EINVAL, "bad location");
    if (out->out_where != PIXVOD_HOST && out->out_where != PIXVOD_DEVICE)
        return fail(c, PIXVOD_EINVAL, "bad output location");
    if (n_iters < 0) return fail(c, PIXVOD_EINVAL, "n_iters must be >= 0");
    if (!c->have_kf) return fail(c, PIXVOD_ESTATE, "pixvod_track before pixvod_set_keyframe");
    const Geo g = geo_of(c);
    const size_t N = (size_t)c->H * c->W;
    int rc = stage_frame(c, frame, where);
    if (rc) return rc;
    bool graphed = false;
    if (c->use_graph && n_iters > 0 && c->schedule == PIXVOD_SCHED_FUSED && c->topology == PIXVOD_TOPO_GRID) {
        rc = track_graph_run(c, n_iters, &graphed);
        if (rc) return rc;
    }
    if (!graphed) {
        // the health flag was cleared by the frame preparation of stage_frame
        if (n_iters == 0) {
            HIP_TRY(c, launch_valid_only(g, strengths_of(c), inputs_of(c), c->X[c->cur], c->valid, c->stream));
            c->have_var = false;
        } else {
            rc = run_iterations(c, n_iters);
            if (rc) return rc;
        }
        HIP_TRY(c, launch_frame_stats(g, c->X[c->cur], c->valid, 1, c->partial, c->result, c->stream, c->health));
    }
    if (out->inv_depth || out->inv_depth_var) {
        float* d_inv = out->inv_depth;
        float* d_var = out->inv_depth_var;
        if (out->out_where == PIXVOD_HOST) {
            d_inv = out->inv_depth ? c->out_stage : nullptr;
            d_var = out->inv_depth_var ? c->out_stage + N : nullptr;
        }
        HIP_TRY(c, launch_outputs(g, c->X[c->cur], c->var_ll, c->have_var ? 1 : 0, d_inv, d_var, c->stream));
        if (out->out_where == PIXVOD_HOST) {
            if (out->inv_depth)
                HIP_TRY(c, hipMemcpyAsync(out->inv_depth, c->out_stage, N * sizeof(float), hipMemcpyDeviceToHost,
                                          c->stream));
            if (out->inv_depth_var)
                HIP_TRY(c, hipMemcpyAsync(out->inv_depth_var, c->out_stage + N, N * sizeof(float),
                                          hipMemcpyDeviceToHost, c->stream));
        }
    }
    HIP_TRY(c, hipMemcpyAsync(c->h_result, c->result, 9 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (!c->pending.empty() || !c->graph_pending.empty()) prof_collect(c);

    const double inv_n = 1.0 / (double)N;
    for (int k = 0; k < 6; ++k) {
        c->xi_last[k] = c->h_result[k] * inv_n;
        out->xi_rel[k] = c->xi_last[k];
    }
    c->have_track = true;
    c->frames_since_kf += 1;
    double E[16], Ei[16];
    host_se3_exp(c->xi_last, E);
    host_se3_inverse(E, Ei);
    host_mat4_mul(c->T_w_kf, Ei, out->T_world);
    const float vf = (float)(c->h_result[6] * inv_n);
    out->valid_fraction = vf;
    out->frames_since_keyframe = c->frames_since_kf;
    unsigned f = 0;
    if (c->frames_since_kf >= c->P.kf_max_frames || vf < c->P.kf_min_valid_frac) f |= PIXVOD_KEYFRAME_DUE;
    if (vf < c->P.kf_min_valid_frac) f |= PIXVOD_LOW_OVERLAP;
    if (c->h_result[7] > 0.0 || c->h_result[8] != 0.0) f |= PIXVOD_DIVERGED;
    out->flags = f;
    return PIXVOD_OK;
}

int pixvod_profile_enable(pixvod_ctx* c, int enable) {
    if (!c) return fail(nullptr, PIXVOD_EINVAL, "ctx is NULL");
    c->prof = enable != 0;
    return PIXVOD_OK;
}

int pixvod_set_graph(pixvod_ctx* c, int enable) {
    if (!c) return fail(nullptr, PIXVOD_EINVAL, "ctx is NULL");
    c->use_graph = enable != 0;
    return PIXVOD_OK;
}

int pixvod_profile_read(pixvod_ctx* c, int kind, double* total_ms, int64_t* launches) {
    if (!c) return fail(nullptr, PIXVOD_EINVAL, "ctx is NULL");
    if (kind < 0 || kind >= PIXVOD_PROF_KINDS || !total_ms || !launches)
        return fail(c, PIXVOD_EINVAL, "bad profile query");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    prof_collect(c);
    *total_ms = c->prof_ms[kind];
    *launches = c->prof_n[kind];
    c->prof_ms[kind] = 0.0;
    c->prof_n[kind] = 0;
    return PIXVOD_OK;
}

static size_t state_floats(const pixvod_ctx* c) {
    const size_t N = (size_t)c->H * c->W;
    if (c->topology == PIXVOD_TOPO_QUADTREE) return (size_t)TP_PLANES * N + (size_t)TN_PLANES * c->tg.NT;
    return (size_t)N_PLANES * N;
}

int pixvod_state_bytes(const pixvod_ctx* c, size_t* bytes) {
    if (!c || !bytes) return fail(const_cast<pixvod_ctx*>(c), PIXVOD_EINVAL, "ctx and bytes are required");
    *bytes = state_floats(c) * sizeof(float);
    return PIXVOD_OK;
}

// staging of the exchange layout; sized for both topologies
static int ensure_dense(pixvod_ctx* c) {
    if (c->dense_state) return PIXVOD_OK;
    const size_t N = (size_t)c->H * c->W;
    TreeGeo t;
    size_t n = (size_t)N_PLANES * N;
    if (make_tree_geo(c->H, c->W, 1.0, 1.0, &t)) n = std::max(n, (size_t)TP_PLANES * N + (size_t)TN_PLANES * t.NT);
    return dev_alloc(c, &c->dense_state, n);
}

// quadtree exchange: 42 pixel planes of H*W, then 141 node planes of NT
static int tree_exchange(pixvod_ctx* c, float* d, int to_dense) {
    const size_t N = (size_t)c->H * c->W;
    float* X = c->X[c->cur];
    float* NX = c->NX[c->cur];
    HIP_TRY(c, launch_tree_pack_pixels(geo_of(c), X, d, to_dense, c->stream));
    float* dn = d + (size_t)TP_PLANES * N;
    const size_t w = (size_t)c->tg.NT * sizeof(float), sp = (size_t)c->tg.nplane * sizeof(float);
    if (to_dense)
        HIP_TRY(c, hipMemcpy2DAsync(dn, w, NX, sp, w, TN_PLANES, hipMemcpyDeviceToDevice, c->stream));
    else
        HIP_TRY(c, hipMemcpy2DAsync(NX, sp, dn, w, w, TN_PLANES, hipMemcpyDeviceToDevice, c->stream));
    return PIXVOD_OK;
}

int pixvod_get_state(pixvod_ctx* c, void* dst, int where) {
    if (!c) return fail(nullptr, PIXVOD_EINVAL, "ctx is NULL");
    if (!dst) return fail(c, PIXVOD_EINVAL, "dst is NULL");
    if (where != PIXVOD_HOST && where != PIXVOD_DEVICE) return fail(c, PIXVOD_EINVAL, "bad location");
    const size_t n = state_floats(c);
    float* d = (float*)dst;
    if (where == PIXVOD_HOST) {
        int rc = ensure_dense(c);
        if (rc) return rc;
        d = c->dense_state;
    }
    if (c->topology == PIXVOD_TOPO_QUADTREE) {
        int rc = tree_exchange(c, d, 1);
        if (rc) return rc;
    } else {
        HIP_TRY(c, launch_pack_state(geo_of(c), c->X[c->cur], d, 1, c->stream));
    }
    if (where == PIXVOD_HOST)
        HIP_TRY(c, hipMemcpyAsync(dst, d, n * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return PIXVOD_OK;
}

int pixvod_set_state(pixvod_ctx* c, const void* src, int where) {
    if (!c) return fail(nullptr, PIXVOD_EINVAL, "ctx is NULL");
    if (!src) return fail(c, PIXVOD_EINVAL, "src is NULL");
    if (where != PIXVOD_HOST && where != PIXVOD_DEVICE) return fail(c, PIXVOD_EINVAL, "bad location");
    const size_t n = state_floats(c);
    const float* d = (const float*)src;
    if (where == PIXVOD_HOST) {
        int rc = ensure_dense(c);
        if (rc) return rc;
        HIP_TRY(c, hipMemcpyAsync(c->dense_state, src, n * sizeof(float), hipMemcpyHostToDevice, c->stream));
        d = c->dense_state;
    }
    if (c->topology == PIXVOD_TOPO_QUADTREE) {
        int rc = tree_exchange(c, const_cast<float*>(d), 0);
        if (rc) return rc;
    } else {
        HIP_TRY(c, launch_pack_state(geo_of(c), c->X[c->cur], const_cast<float*>(d), 0, c->stream));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return PIXVOD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batches

namespace {

struct BatchSeq {
    int H = 0, W = 0, pitch = 0;
    long plane = 0;
    pixvod_intrinsics K{};
    float* X[2] = {nullptr, nullptr};
    float *Is = nullptr, *cxt = nullptr, *cyt = nullptr, *sig = nullptr;
    float *It = nullptr, *Gx = nullptr, *Gy = nullptr, *var_ll = nullptr, *valid = nullptr;
    float *frame = nullptr, *kf_stage = nullptr, *out_stage = nullptr, *dense = nullptr;
    float* normals_stage = nullptr;      // staged normals of host-input frames (re-anchoring steps)
    bool have_kf = false, have_track = false;
    double T_w_kf[16];
    double xi_last[6];
    int frames_since_kf = 0;
};

}  // namespace

struct pixvod_batch {
    int n = 0;
    pixvod_params P{};
    hipStream_t own_stream = nullptr, stream = nullptr;
    std::vector<BatchSeq> seq;
    SeqDesc* d_seqs = nullptr;
    int2* d_work = nullptr;
    int n_work = 0, tile_x = 64, tile_y = 4;
    int max_stat_tiles = 0;  // 64 x 4 statistics tiles of the largest image
    double *d_partial = nullptr, *d_result = nullptr, *h_result = nullptr;
    int *d_health = nullptr, *h_health = nullptr;
    int parity = 0;
    // captured frame steps per (canonical buffer, re-anchoring on/off) for graph_iters iterations
    hipGraphExec_t exec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    hipGraph_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    int graph_iters = -1;
    std::vector<SeqDesc> descs;          // host copy of the device descriptors
    SeqDesc* h_desc = nullptr;           // pinned staging of the descriptors
    int *d_fsk = nullptr;                // per sequence: frames since the keyframe (device keyframe test)
    unsigned *d_flags = nullptr, *h_flags = nullptr;
    bool persistent = false;             // iteration block as one cooperative launch
    int persistent_grid = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double last_ms = 0.0;
    std::string err;
};

static int bfail(pixvod_batch* b, int code, const std::string& msg) {
    if (b) b->err = msg;
    g_last_error = msg;
    return code;
}

#define HIP_TRY_B(b, expr)                                                                    \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return bfail((b), PIXVOD_EHIP, std::string(#expr ": ") + hipGetErrorString(e_));  \
    } while (0)

static Geo geo_of_seq(const BatchSeq& q) {
    Geo g;
    g.H = q.H;
    g.W = q.W;
    g.pitch = q.pitch;
    g.plane = q.plane;
    g.fx = q.K.fx;
    g.fy = q.K.fy;
    g.cx = q.K.cx;
    g.cy = q.K.cy;
    return g;
}

static Strengths strengths_of_params(const pixvod_params& P) {
    pixvod_ctx tmp;
    tmp.P = P;
    tmp.has_sigma = false;
    return strengths_of(&tmp);
}

static void batch_drop_graphs(pixvod_batch* b) {
    for (int k = 0; k < 2; ++k)
        for (int r = 0; r < 2; ++r) {
            if (b->exec[k][r]) (void)hipGraphExecDestroy(b->exec[k][r]);
            if (b->graph[k][r]) (void)hipGraphDestroy(b->graph[k][r]);
            b->exec[k][r] = nullptr;
            b->graph[k][r] = nullptr;
        }
    b->graph_iters = -1;
}

static void batch_release(pixvod_batch* b) {
    batch_drop_graphs(b);
    for (auto& q : b->seq) {
        void* bufs[] = {q.X[0], q.X[1], q.Is, q.cxt, q.cyt, q.sig, q.It, q.Gx, q.Gy, q.var_ll, q.valid,
                        q.frame, q.kf_stage, q.out_stage, q.dense, q.normals_stage};
        for (void* p : bufs)
            if (p) (void)hipFree(p);
    }
    void* bufs[] = {b->d_seqs, b->d_work, b->d_partial, b->d_result, b->d_health, b->d_fsk, b->d_flags};
    for (void* p : bufs)
        if (p) (void)hipFree(p);
    if (b->h_result) (void)hipHostFree(b->h_result);
    if (b->h_health) (void)hipHostFree(b->h_health);
    if (b->h_flags) (void)hipHostFree(b->h_flags);
    if (b->h_desc) (void)hipHostFree(b->h_desc);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    if (b->own_stream) (void)hipStreamDestroy(b->own_stream);
}

// work list for the current tile shape: natural order is sequence-major,
// row-major tiles; workgroup w runs natural item perm(w) so that the
// workgroups dispatched to one XCD (w mod 8) cover a contiguous range
static int batch_build_work(pixvod_batch* b) {
    std::vector<SeqDesc> descs(b->n);
    int total = 0, n_stat = 0, max_stat = 0;
    for (int i = 0; i < b->n; ++i) {
        BatchSeq& q = b->seq[i];
        SeqDesc& d = descs[i];
        std::memset(&d, 0, sizeof(d));
        d.g = geo_of_seq(q);
        d.in.Is = q.Is;
        d.in.cxt = q.cxt;
        d.in.cyt = q.cyt;
        d.in.sigD = q.sig;
        d.in.It = q.It;
        d.in.Gx = q.Gx;
        d.in.Gy = q.Gy;
        d.X0 = q.X[0];
        d.X1 = q.X[1];
        d.var_ll = q.var_ll;
        d.valid = q.valid;
        d.frame = q.frame;
        d.normals = nullptr;
        d.It = q.It;
        d.Gx = q.Gx;
        d.Gy = q.Gy;
        d.Is = q.Is;
        d.cxt = q.cxt;
        d.cyt = q.cyt;
        d.tiles_x = (q.W + b->tile_x - 1) / b->tile_x;
        const int ty = (q.H + b->tile_y - 1) / b->tile_y;
        d.n_tiles = d.tiles_x * ty;
        d.tile_base = total;
        total += d.n_tiles;
        const int nst = stats_blocks(d.g);
        d.stat_base = n_stat;
        n_stat += nst;
        if (nst > max_stat) max_stat = nst;
    }
    std::vector<int2> natural(total);
    for (int i = 0; i < b->n; ++i)
        for (int t = 0; t < descs[i].n_tiles; ++t) natural[descs[i].tile_base + t] = make_int2(descs[i].tile_base + t, i);
    const int X = 8;
    std::vector<int> start(X + 1, 0);
    for (int x = 0; x < X; ++x) start[x + 1] = start[x] + (total - x + X - 1) / X;
    std::vector<int2> work(total);
    for (int w = 0; w < total; ++w) work[w] = natural[start[w % X] + w / X];
    if (b->d_work) (void)hipFree(b->d_work);
    if (b->d_partial) (void)hipFree(b->d_partial);
    b->d_work = nullptr;
    b->d_partial = nullptr;
    if (hipMalloc((void**)&b->d_work, sizeof(int2) * total) != hipSuccess ||
        hipMalloc((void**)&b->d_partial, sizeof(double) * 8 * n_stat) != hipSuccess)
        return bfail(b, PIXVOD_ENOMEM, "work list allocation failed");
    HIP_TRY_B(b, hipMemcpy(b->d_work, work.data(), sizeof(int2) * total, hipMemcpyHostToDevice));
    HIP_TRY_B(b, hipMemcpy(b->d_seqs, descs.data(), sizeof(SeqDesc) * b->n, hipMemcpyHostToDevice));
    b->descs = descs;
    b->n_work = total;
    b->max_stat_tiles = max_stat;
    b->persistent_grid = 0;
    batch_drop_graphs(b);
    return PIXVOD_OK;
}

static BatchLaunch batch_launch_args(const pixvod_batch* b) {
    BatchLaunch L;
    L.seqs = b->d_seqs;
    L.work = b->d_work;
    L.n_work = b->n_work;
    L.n_seq = b->n;
    L.tile_x = b->tile_x;
    L.tile_y = b->tile_y;
    L.parity = b->parity;
    L.s = strengths_of_params(b->P);
    L.health = b->d_health;
    L.partial = b->d_partial;
    L.max_stat_tiles = b->max_stat_tiles;
    L.result = b->d_result;
    L.fsk = b->d_fsk;
    L.flags = b->d_flags;
    L.kf_max_frames = b->P.kf_max_frames;
    L.kf_min_valid = b->P.kf_min_valid_frac;
    L.reanchor = 0;
    return L;
}

extern "C" {

int pixvod_batch_create(int n, const int* H, const int* W, const pixvod_intrinsics* K, const pixvod_params* params,
                        pixvod_batch** out) {
    if (!out) return bfail(nullptr, PIXVOD_EINVAL, "out_batch is NULL");
    *out = nullptr;
    if (n < 1 || !H || !W || !K) return bfail(nullptr, PIXVOD_EINVAL, "need n >= 1 and H, W, K arrays");
    long total = 0;
    for (int i = 0; i < n; ++i) {
        if (H[i] < 2 || W[i] < 2) return bfail(nullptr, PIXVOD_EINVAL, "H and W must be >= 2");
        if (!(K[i].fx > 0) || !(K[i].fy > 0) || !std::isfinite(K[i].cx) || !std::isfinite(K[i].cy))
            return bfail(nullptr, PIXVOD_EINVAL, "intrinsics must be finite with fx, fy > 0");
        total += (long)H[i] * W[i];
    }
    if (total > (1L << 30)) return bfail(nullptr, PIXVOD_EINVAL, "batch too large");
    pixvod_params P;
    if (params) P = *params;
    else pixvod_default_params(&P);
    if (!finite_params(&P)) return bfail(nullptr, PIXVOD_EINVAL, "invalid parameters");
    if (P.damping != 0.0f) return bfail(nullptr, PIXVOD_EINVAL, "batches use the fused schedule (damping 0)");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
        return bfail(nullptr, PIXVOD_ENODEV, "no HIP device available");
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
        std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return bfail(nullptr, PIXVOD_ENODEV, "need a gfx950 device");

    pixvod_batch* b = new pixvod_batch();
    b->n = n;
    b->P = P;
    b->seq.resize(n);
    int rc = PIXVOD_OK;
    auto alloc = [&](float** p, size_t cnt) {
        if (rc) return;
        if (hipMalloc((void**)p, cnt * sizeof(float)) != hipSuccess) {
            *p = nullptr;
            rc = PIXVOD_ENOMEM;
        }
    };
    for (int i = 0; i < n && !rc; ++i) {
        BatchSeq& q = b->seq[i];
        q.H = H[i];
        q.W = W[i];
        q.pitch = (W[i] + 63) / 64 * 64;
        q.plane = (long)q.H * q.pitch;
        q.K = K[i];
        std::memset(q.T_w_kf, 0, sizeof(q.T_w_kf));
        for (int k = 0; k < 4; ++k) q.T_w_kf[k * 5] = 1.0;
        std::memset(q.xi_last, 0, sizeof(q.xi_last));
        const size_t pl = (size_t)q.plane, N = (size_t)q.H * q.W;
        alloc(&q.X[0], pl * N_PLANES);
        alloc(&q.X[1], pl * N_PLANES);
        float** planes[] = {&q.Is, &q.cxt, &q.cyt, &q.sig, &q.It, &q.Gx, &q.Gy, &q.var_ll, &q.valid};
        for (float** p : planes) alloc(p, pl);
        alloc(&q.frame, N);
        alloc(&q.kf_stage, 4 * N);
        alloc(&q.out_stage, 2 * N);
    }
    if (!rc && hipMalloc((void**)&b->d_seqs, sizeof(SeqDesc) * n) != hipSuccess) rc = PIXVOD_ENOMEM;
    if (!rc && hipMalloc((void**)&b->d_result, sizeof(double) * 8 * n) != hipSuccess) rc = PIXVOD_ENOMEM;
    if (!rc && hipMalloc((void**)&b->d_health, sizeof(int)) != hipSuccess) rc = PIXVOD_ENOMEM;
    if (!rc && hipHostMalloc((void**)&b->h_result, sizeof(double) * 8 * n) != hipSuccess) rc = PIXVOD_ENOMEM;
    if (!rc && hipHostMalloc((void**)&b->h_health, sizeof(int)) != hipSuccess) rc = PIXVOD_ENOMEM;
    if (!rc && hipMalloc((void**)&b->d_fsk, sizeof(int) * n) != hipSuccess) rc = PIXVOD_ENOMEM;
    if (!rc && hipMalloc((void**)&b->d_flags, sizeof(unsigned) * n) != hipSuccess) rc = PIXVOD_ENOMEM;
    if (!rc && hipHostMalloc((void**)&b->h_flags, sizeof(unsigned) * n) != hipSuccess) rc = PIXVOD_ENOMEM;
    if (!rc && hipHostMalloc((void**)&b->h_desc, sizeof(SeqDesc) * n) != hipSuccess) rc = PIXVOD_ENOMEM;
    if (!rc && hipStreamCreateWithFlags(&b->own_stream, hipStreamNonBlocking) != hipSuccess) rc = PIXVOD_EHIP;
    if (!rc && (hipEventCreate(&b->ev0) != hipSuccess || hipEventCreate(&b->ev1) != hipSuccess)) rc = PIXVOD_EHIP;
    if (!rc) rc = batch_build_work(b);
    if (!rc) {
        const float ell0 = (float)(-std::log((double)P.init_inv_depth));
        for (auto& q : b->seq) {
            const Geo g = geo_of_seq(q);
            if (launch_init_state(g, q.X[0], ell0, b->own_stream) != hipSuccess ||
                launch_init_state(g, q.X[1], ell0, b->own_stream) != hipSuccess ||
                hipMemsetAsync(q.var_ll, 0, (size_t)q.plane * sizeof(float), b->own_stream) != hipSuccess) {
                rc = PIXVOD_EHIP;
                break;
            }
        }
        if (!rc && launch_set_ints(b->d_fsk, n, 0, b->own_stream) != hipSuccess) rc = PIXVOD_EHIP;
        if (!rc && hipStreamSynchronize(b->own_stream) != hipSuccess) rc = PIXVOD_EHIP;
    }
    if (rc) {
        std::string m = b->err.empty() ? "batch allocation failed" : b->err;
        batch_release(b);
        delete b;
        return bfail(nullptr, rc, m);
    }
    b->stream = b->own_stream;
    *out = b;
    return PIXVOD_OK;
}

int pixvod_batch_destroy(pixvod_batch* b) {
    if (!b) return PIXVOD_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    batch_release(b);
    delete b;
    return PIXVOD_OK;
}

int pixvod_batch_set_stream(pixvod_batch* b, void* s) {
    if (!b) return bfail(nullptr, PIXVOD_EINVAL, "batch is NULL");
    HIP_TRY_B(b, hipStreamSynchronize(b->stream));
    b->stream = s ? (hipStream_t)s : b->own_stream;
    batch_drop_graphs(b);
    return PIXVOD_OK;
}

int pixvod_batch_set_keyframes(pixvod_batch* b, int m, const int* ids, const float* const* imgs,
                               const float* const* normals, int where) {
    if (!b) return bfail(nullptr, PIXVOD_EINVAL, "batch is NULL");
    if (m < 0 || (m > 0 && (!ids || !imgs || !normals))) return bfail(b, PIXVOD_EINVAL, "bad keyframe list");
    if (where != PIXVOD_HOST && where != PIXVOD_DEVICE) return bfail(b, PIXVOD_EINVAL, "bad location");
    for (int k = 0; k < m; ++k)
        if (ids[k] < 0 || ids[k] >= b->n || !imgs[k] || !normals[k])
            return bfail(b, PIXVOD_EINVAL, "bad keyframe entry");
    for (int k = 0; k < m; ++k) {
        BatchSeq& q = b->seq[ids[k]];
        const size_t N = (size_t)q.H * q.W;
        const float *di = imgs[k], *dn = normals[k];
        if (where == PIXVOD_HOST) {
            HIP_TRY_B(b, hipMemcpyAsync(q.kf_stage, imgs[k], N * sizeof(float), hipMemcpyHostToDevice, b->stream));
            HIP_TRY_B(b, hipMemcpyAsync(q.kf_stage + N, normals[k], 3 * N * sizeof(float), hipMemcpyHostToDevice,
                                        b->stream));
            di = q.kf_stage;
            dn = q.kf_stage + N;
        }
        HIP_TRY_B(b, launch_keyframe_prep(geo_of_seq(q), di, dn, q.Is, q.cxt, q.cyt, q.X[b->parity],
                                          q.X[1 - b->parity], b->stream));
        if (q.have_track) {
            double E[16], Ei[16], Tw[16];
            host_se3_exp(q.xi_last, E);
            host_se3_inverse(E, Ei);
            host_mat4_mul(q.T_w_kf, Ei, Tw);
            std::memcpy(q.T_w_kf, Tw, sizeof(Tw));
        }
        std::memset(q.xi_last, 0, sizeof(q.xi_last));
        q.have_track = false;
        q.have_kf = true;
        q.frames_since_kf = 0;
        HIP_TRY_B(b, launch_set_ints(b->d_fsk + ids[k], 1, 0, b->stream));
    }
    HIP_TRY_B(b, hipStreamSynchronize(b->stream));
    return PIXVOD_OK;
}

int pixvod_batch_set_tile(pixvod_batch* b, int tx, int ty) {
    if (!b) return bfail(nullptr, PIXVOD_EINVAL, "batch is NULL");
    if (tx < 1 || ty < 1 || tx * ty > 256) return bfail(b, PIXVOD_EINVAL, "tile must have 1..256 threads");
    HIP_TRY_B(b, hipStreamSynchronize(b->stream));
    b->tile_x = tx;
    b->tile_y = ty;
    return batch_build_work(b);
}

// graph of one frame step for the current parity
static int batch_graph(pixvod_batch* b, int n_iters, int reanchor, hipGraphExec_t* exec) {
    if (b->graph_iters != n_iters) batch_drop_graphs(b);
    const int k = b->parity;
    if (!b->exec[k][reanchor]) {
        BatchLaunch L = batch_launch_args(b);
        L.reanchor = reanchor;
        HIP_TRY_B(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        hipError_t le = launch_batch_frame_step(L, n_iters, b->stream);
        hipGraph_t g = nullptr;
        hipError_t ce = hipStreamEndCapture(b->stream, &g);
        if (le != hipSuccess || ce != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return bfail(b, PIXVOD_EHIP, std::string("graph capture failed: ") +
                                             hipGetErrorString(le != hipSuccess ? le : ce));
        }
        b->graph[k][reanchor] = g;
        HIP_TRY_B(b, hipGraphInstantiate(&b->exec[k][reanchor], g, nullptr, nullptr, 0));
        b->graph_iters = n_iters;
    }
    *exec = b->exec[k][reanchor];
    return PIXVOD_OK;
}

// one frame step for every sequence; normals != NULL re-anchors, inside the
// step, the sequences whose keyframe test fires on the frame just tracked
static int batch_step(pixvod_batch* b, const float* const* frames, const float* const* normals, int where,
                      int n_iters, pixvod_track_out* outs) {
    if (!frames || !outs) return bfail(b, PIXVOD_EINVAL, "frames and outs are required");
    if (where != PIXVOD_HOST && where != PIXVOD_DEVICE) return bfail(b, PIXVOD_EINVAL, "bad location");
    if (n_iters < 1) return bfail(b, PIXVOD_EINVAL, "n_iters must be >= 1");
    const int reanchor = normals ? 1 : 0;
    for (int i = 0; i < b->n; ++i) {
        if (!frames[i] || (reanchor && !normals[i])) return bfail(b, PIXVOD_EINVAL, "missing frame or normals");
        if (outs[i].out_where != PIXVOD_HOST && outs[i].out_where != PIXVOD_DEVICE)
            return bfail(b, PIXVOD_EINVAL, "bad output location");
        if (!b->seq[i].have_kf) return bfail(b, PIXVOD_ESTATE, "a sequence has no keyframe");
    }
    // the step's frames (and normals): device inputs are read in place through
    // the sequence descriptors, host inputs are staged first
    for (int i = 0; i < b->n; ++i) {
        BatchSeq& q = b->seq[i];
        SeqDesc& d = b->descs[i];
        const size_t N = (size_t)q.H * q.W;
        if (where == PIXVOD_HOST) {
            HIP_TRY_B(b, hipMemcpyAsync(q.frame, frames[i], N * sizeof(float), hipMemcpyHostToDevice, b->stream));
            d.frame = q.frame;
            d.normals = nullptr;
            if (reanchor) {
                if (!q.normals_stage && hipMalloc((void**)&q.normals_stage, 3 * N * sizeof(float)) != hipSuccess)
                    return bfail(b, PIXVOD_ENOMEM, "normal staging allocation failed");
                HIP_TRY_B(b, hipMemcpyAsync(q.normals_stage, normals[i], 3 * N * sizeof(float),
                                            hipMemcpyHostToDevice, b->stream));
                d.normals = q.normals_stage;
            }
        } else {
            d.frame = frames[i];
            d.normals = reanchor ? normals[i] : nullptr;
        }
    }
    std::memcpy(b->h_desc, b->descs.data(), sizeof(SeqDesc) * b->n);
    HIP_TRY_B(b, hipMemcpyAsync(b->d_seqs, b->h_desc, sizeof(SeqDesc) * b->n, hipMemcpyHostToDevice, b->stream));
    if (b->persistent) {
        BatchLaunch L = batch_launch_args(b);
        L.reanchor = reanchor;
        if (!b->persistent_grid) b->persistent_grid = batch_persistent_grid(L);
        if (b->persistent_grid < 1) return bfail(b, PIXVOD_EHIP, "no co-resident grid for the persistent step");
        HIP_TRY_B(b, hipEventRecord(b->ev0, b->stream));
        HIP_TRY_B(b, launch_batch_frame_step_persistent(L, n_iters, b->persistent_grid, b->stream));
        HIP_TRY_B(b, hipEventRecord(b->ev1, b->stream));
    } else {
        hipGraphExec_t exec = nullptr;
        int rc = batch_graph(b, n_iters, reanchor, &exec);
        if (rc) return rc;
        HIP_TRY_B(b, hipEventRecord(b->ev0, b->stream));
        HIP_TRY_B(b, hipGraphLaunch(exec, b->stream));
        HIP_TRY_B(b, hipEventRecord(b->ev1, b->stream));
    }
    b->parity ^= (n_iters + 1) & 1;
    HIP_TRY_B(b, hipMemcpyAsync(b->h_result, b->d_result, sizeof(double) * 8 * b->n, hipMemcpyDeviceToHost,
                                b->stream));
    HIP_TRY_B(b, hipMemcpyAsync(b->h_health, b->d_health, sizeof(int), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY_B(b, hipMemcpyAsync(b->h_flags, b->d_flags, sizeof(unsigned) * b->n, hipMemcpyDeviceToHost, b->stream));
    for (int i = 0; i < b->n; ++i) {
        BatchSeq& q = b->seq[i];
        pixvod_track_out* o = &outs[i];
        if (!o->inv_depth && !o->inv_depth_var) continue;
        const size_t N = (size_t)q.H * q.W;
        float* di = o->inv_depth;
        float* dv = o->inv_depth_var;
        if (o->out_where == PIXVOD_HOST) {
            di = o->inv_depth ? q.out_stage : nullptr;
            dv = o->inv_depth_var ? q.out_stage + N : nullptr;
        }
        // re-anchoring keeps the log-depths and the variance plane: the maps
        // are those of the frame just tracked
        HIP_TRY_B(b, launch_outputs(geo_of_seq(q), q.X[b->parity], q.var_ll, 1, di, dv, b->stream));
        if (o->out_where == PIXVOD_HOST) {
            if (o->inv_depth)
                HIP_TRY_B(b, hipMemcpyAsync(o->inv_depth, q.out_stage, N * sizeof(float), hipMemcpyDeviceToHost,
                                            b->stream));
            if (o->inv_depth_var)
                HIP_TRY_B(b, hipMemcpyAsync(o->inv_depth_var, q.out_stage + N, N * sizeof(float),
                                            hipMemcpyDeviceToHost, b->stream));
        }
    }
    HIP_TRY_B(b, hipStreamSynchronize(b->stream));
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, b->ev0, b->ev1) == hipSuccess) b->last_ms = ms;
    for (int i = 0; i < b->n; ++i) {
        BatchSeq& q = b->seq[i];
        pixvod_track_out* o = &outs[i];
        const double inv_n = 1.0 / ((double)q.H * q.W);
        for (int k = 0; k < 6; ++k) {
            q.xi_last[k] = b->h_result[8 * i + k] * inv_n;
            o->xi_rel[k] = q.xi_last[k];
        }
        q.have_track = true;
        q.frames_since_kf += 1;
        double E[16], Ei[16];
        host_se3_exp(q.xi_last, E);
        host_se3_inverse(E, Ei);
        host_mat4_mul(q.T_w_kf, Ei, o->T_world);
        o->valid_fraction = (float)(b->h_result[8 * i + 6] * inv_n);
        o->frames_since_keyframe = q.frames_since_kf;
        o->flags = b->h_flags[i];
        if (reanchor && (o->flags & PIXVOD_KEYFRAME_DUE)) {
            // re-anchored inside the step on the frame just tracked
            std::memcpy(q.T_w_kf, o->T_world, sizeof(q.T_w_kf));
            std::memset(q.xi_last, 0, sizeof(q.xi_last));
            q.have_track = false;
            q.frames_since_kf = 0;
        }
    }
    return PIXVOD_OK;
}

int pixvod_batch_track(pixvod_batch* b, const float* const* frames, int where, int n_iters, pixvod_track_out* outs) {
    if (!b) return bfail(nullptr, PIXVOD_EINVAL, "batch is NULL");
    return batch_step(b, frames, nullptr, where, n_iters, outs);
}

int pixvod_batch_track_reanchor(pixvod_batch* b, const float* const* frames, const float* const* normals,
                                int where, int n_iters, pixvod_track_out* outs) {
    if (!b) return bfail(nullptr, PIXVOD_EINVAL, "batch is NULL");
    if (!normals) return bfail(b, PIXVOD_EINVAL, "normals are required");
    return batch_step(b, frames, normals, where, n_iters, outs);
}

int pixvod_batch_set_persistent(pixvod_batch* b, int enable) {
    if (!b) return bfail(nullptr, PIXVOD_EINVAL, "batch is NULL");
    b->persistent = enable != 0;
    b->persistent_grid = 0;
    return PIXVOD_OK;
}

int pixvod_batch_last_step_ms(pixvod_batch* b, double* ms) {
    if (!b || !ms) return bfail(b, PIXVOD_EINVAL, "batch and ms are required");
    *ms = b->last_ms;
    return PIXVOD_OK;
}

int pixvod_batch_get_state(pixvod_batch* b, int seq, void* dst, int where) {
    if (!b) return bfail(nullptr, PIXVOD_EINVAL, "batch is NULL");
    if (seq < 0 || seq >= b->n || !dst) return bfail(b, PIXVOD_EINVAL, "bad sequence or destination");
    if (where != PIXVOD_HOST && where != PIXVOD_DEVICE) return bfail(b, PIXVOD_EINVAL, "bad location");
    BatchSeq& q = b->seq[seq];
    const size_t n = (size_t)N_PLANES * q.H * q.W;
    float* d = (float*)dst;
    if (where == PIXVOD_HOST) {
        if (!q.dense && hipMalloc((void**)&q.dense, n * sizeof(float)) != hipSuccess)
            return bfail(b, PIXVOD_ENOMEM, "staging allocation failed");
        d = q.dense;
    }
    HIP_TRY_B(b, launch_pack_state(geo_of_seq(q), q.X[b->parity], d, 1, b->stream));
    if (where == PIXVOD_HOST) HIP_TRY_B(b, hipMemcpyAsync(dst, d, n * sizeof(float), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY_B(b, hipStreamSynchronize(b->stream));
    return PIXVOD_OK;
}

int pixvod_batch_set_state(pixvod_batch* b, int seq, const void* src, int where) {
    if (!b) return bfail(nullptr, PIXVOD_EINVAL, "batch is NULL");
    if (seq < 0 || seq >= b->n || !src) return bfail(b, PIXVOD_EINVAL, "bad sequence or source");
    if (where != PIXVOD_HOST && where != PIXVOD_DEVICE) return bfail(b, PIXVOD_EINVAL, "bad location");
    BatchSeq& q = b->seq[seq];
    const size_t n = (size_t)N_PLANES * q.H * q.W;
    const float* d = (const float*)src;
    if (where == PIXVOD_HOST) {
        if (!q.dense && hipMalloc((void**)&q.dense, n * sizeof(float)) != hipSuccess)
            return bfail(b, PIXVOD_ENOMEM, "staging allocation failed");
        HIP_TRY_B(b, hipMemcpyAsync(q.dense, src, n * sizeof(float), hipMemcpyHostToDevice, b->stream));
        d = q.dense;
    }
    HIP_TRY_B(b, launch_pack_state(geo_of_seq(q), q.X[b->parity], const_cast<float*>(d), 0, b->stream));
    HIP_TRY_B(b, hipStreamSynchronize(b->stream));
    return PIXVOD_OK;
}

int pixvod_batch_autotune(pixvod_batch* b, int n_iters, int* tx_out, int* ty_out) {
    if (!b) return bfail(nullptr, PIXVOD_EINVAL, "batch is NULL");
    if (n_iters < 1 || !tx_out || !ty_out) return bfail(b, PIXVOD_EINVAL, "bad autotune arguments");
    for (auto& q : b->seq)
        if (!q.have_kf) return bfail(b, PIXVOD_ESTATE, "a sequence has no keyframe");
    static const int cand[][2] = {{64, 1}, {64, 2}, {64, 4}, {128, 1}, {128, 2}, {256, 1}, {32, 4}, {32, 8}, {16, 16}};
    // snapshot of both state copies; the passes below run on the live buffers
    std::vector<float*> snap(2 * b->n, nullptr);
    for (int i = 0; i < b->n && true; ++i)
        for (int k = 0; k < 2; ++k) {
            const size_t bytes = (size_t)b->seq[i].plane * N_PLANES * sizeof(float);
            if (hipMalloc((void**)&snap[2 * i + k], bytes) != hipSuccess) {
                for (float* p : snap)
                    if (p) (void)hipFree(p);
                return bfail(b, PIXVOD_ENOMEM, "autotune snapshot allocation failed");
            }
            HIP_TRY_B(b, hipMemcpyAsync(snap[2 * i + k], b->seq[i].X[k], bytes, hipMemcpyDeviceToDevice, b->stream));
        }
    const int tx0 = b->tile_x, ty0 = b->tile_y;
    double best = 1e300;
    int bx = tx0, by = ty0;
    int rc = PIXVOD_OK;
    for (auto& c : cand) {
        b->tile_x = c[0];
        b->tile_y = c[1];
        if ((rc = batch_build_work(b))) break;
        BatchLaunch L = batch_launch_args(b);
        // prologue and one warm-up pass (two buffer swaps), then the timed passes
        if (launch_batch_passes(L, 1, true, false, b->stream) != hipSuccess) { rc = PIXVOD_EHIP; break; }
        (void)hipEventRecord(b->ev0, b->stream);
        if (launch_batch_passes(L, n_iters, false, false, b->stream) != hipSuccess) { rc = PIXVOD_EHIP; break; }
        (void)hipEventRecord(b->ev1, b->stream);
        if (hipStreamSynchronize(b->stream) != hipSuccess) { rc = PIXVOD_EHIP; break; }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, b->ev0, b->ev1);
        if (ms < best) {
            best = ms;
            bx = c[0];
            by = c[1];
        }
        for (int i = 0; i < b->n; ++i)
            for (int k = 0; k < 2; ++k)
                (void)hipMemcpyAsync(b->seq[i].X[k], snap[2 * i + k], (size_t)b->seq[i].plane * N_PLANES * sizeof(float),
                                     hipMemcpyDeviceToDevice, b->stream);
    }
    (void)hipStreamSynchronize(b->stream);
    for (float* p : snap)
        if (p) (void)hipFree(p);
    if (rc) return rc;
    b->tile_x = bx;
    b->tile_y = by;
    rc = batch_build_work(b);
    *tx_out = bx;
    *ty_out = by;
    return rc;
}

}  // extern "C"
