// Centralised direct tracking on the GPU (PixVOD, arXiv 2606.03989, Sec. 3.1,
// Eq. photo; the centralised baseline of Sec. 4.4): one global pose and a
// log-depth per keyframe pixel, solved by IRLS Gauss-Newton with every pixel
// accessible at once.
//
// The energy is Eq. (photo) with the per-pixel model's factors at exact
// consensus (every pixel's pose equal to the global one): photometric factors
// with the Huber covariance weighting frozen at the current residuals, each
// pixel's log-depth prior, the normal-integration factors, and one prior
// factor on the pose. Each IRLS iteration:
//   1. linearises every pixel's photometric factor with the per-pixel model's
//      code at the shared pose (the pose block and gradient summed over pixels
//      by a deterministic two-stage reduction, the pose-depth coupling and
//      depth diagonal kept per pixel), its log-depth prior and the
//      normal-integration terms; the pose prior is added once;
//   2. solves the (6 + N) normal equations
//        [A  B ] [d_xi ]   [g_xi ]
//        [B' D ] [d_ell] = [g_ell],  D = diag + lamN * graph Laplacian,
//      by preconditioned conjugate gradients with a block-Jacobi
//      preconditioner (A^-1 for the pose, 1/D_ii for the depths), FP64
//      vectors, to a relative residual tolerance; a device flag ends the
//      remaining launches once it is met;
//   3. applies xi <- Log(Exp(xi) Exp(d_xi)), ell <- ell + d_ell.
// Each CG iteration is four launches: the stencil product and its reductions,
// the pose-block scalar step, the vector update, the next direction's scalars.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pixvod.h"
#include "gbp_device.hpp"
#include "gbp_kernels.h"
#include "runtime_internal.h"

using namespace pv;

namespace {

constexpr int kThreads = 256;      // 64 x 4 pixel blocks
constexpr int kLinPartials = 30;   // A (21), g_xi (6), r.z, r.r, valid count
constexpr int kMvPartials = 7;     // sum b_i p_i (6), p.q
constexpr int kUpPartials = 2;     // r.z, r.r

// solver state in device memory
struct CgState {
    double xi[6];
    double A[21];        // pose block, packed upper
    double g[6];         // pose right-hand side
    double x[6], r[6], z[6], p[6];
    double rz, alpha, beta, rr0, rr;
    double nvalid;
    int done, iters;     // this solve
    int total;           // CG iterations since the frame started
};

struct Planes {            // per-pixel FP64 planes (pitched)
    double *ell, *diag, *b, *gl, *x, *r, *z, *p0, *p1, *q;
};

// ---------------------------------------------------------------------------
// block reduction of `n` doubles per thread into partial[block * n + k]

template <int NV>
__device__ inline void block_reduce(double v[NV], double* __restrict__ partial) {
    __shared__ double sh[kThreads];
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int nthreads = blockDim.x * blockDim.y;
    const long blk = (long)blockIdx.x + (long)blockIdx.y * gridDim.x;
    for (int k = 0; k < NV; ++k) {
        sh[tid] = v[k];
        __syncthreads();
        for (int s = nthreads / 2; s > 0; s >>= 1) {
            if (tid < s) sh[tid] += sh[tid + s];
            __syncthreads();
        }
        if (tid == 0) partial[blk * NV + k] = sh[0];
        __syncthreads();
    }
}

// single-workgroup sum of nb partial records of NV doubles, fixed order
template <int NV>
__device__ inline void final_sum(const double* __restrict__ partial, int nb, double out[NV]) {
    __shared__ double sh[kThreads];
    const int tid = threadIdx.x;
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
        for (int b = tid; b < nb; b += kThreads) s += partial[(long)b * NV + k];
        sh[tid] = s;
        __syncthreads();
        for (int st = kThreads / 2; st > 0; st >>= 1) {
            if (tid < st) sh[tid] += sh[tid + st];
            __syncthreads();
        }
        out[k] = sh[0];
        __syncthreads();
    }
}

// z = A^-1 r for the packed 6x6 pose block
__device__ inline void pose_precondition(const double A[21], const double r[6], double z[6]) {
    double L[21], idg[6];
    for (int k = 0; k < 21; ++k) L[k] = A[k];
    chol6(L, idg);
    for (int k = 0; k < 6; ++k) z[k] = r[k];
    chol6_solve(L, idg, z);
}

__device__ inline double dot6(const double a[6], const double b[6]) {
    double s = 0.0;
    for (int k = 0; k < 6; ++k) s += a[k] * b[k];
    return s;
}

__device__ inline void sym6_mul(const double A[21], const double x[6], double y[6]) {
    for (int r = 0; r < 6; ++r) {
        double s = 0.0;
        for (int c = 0; c < 6; ++c) s += A[s6(r, c)] * x[c];
        y[r] = s;
    }
}

// pose prior (Eq. prior) at xi with precision lamP added to (A, g):
// r = Log(Exp(xi_hat)^-1 Exp(xi)), J = I + ad(r)/2 + ad(r)^2/12
__device__ inline void add_pose_prior(const Strengths& s, const double xi[6], double A[21], double g[6]) {
    double R[9], t[3], rp[6];
    se3_exp(xi, R, t);
    if (s.prior_is_identity) {
        for (int k = 0; k < 6; ++k) rp[k] = xi[k];
    } else {
        double Rr[9], tr[3];
        se3_compose(s.prior_R, s.prior_t, R, t, Rr, tr);
        se3_log(Rr, tr, rp);
    }
    double ad[36], J[36];
    for (int k = 0; k < 36; ++k) ad[k] = 0.0;
    const double* w = rp;
    const double* p = rp + 3;
    const double Wm[9] = {0.0, -w[2], w[1], w[2], 0.0, -w[0], -w[1], w[0], 0.0};
    const double Pm[9] = {0.0, -p[2], p[1], p[2], 0.0, -p[0], -p[1], p[0], 0.0};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            ad[r * 6 + c] = Wm[r * 3 + c];
            ad[(r + 3) * 6 + c] = Pm[r * 3 + c];
            ad[(r + 3) * 6 + c + 3] = Wm[r * 3 + c];
        }
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) {
            double a2 = 0.0;
            for (int k = 0; k < 6; ++k) a2 += ad[r * 6 + k] * ad[k * 6 + c];
            J[r * 6 + c] = (r == c ? 1.0 : 0.0) + 0.5 * ad[r * 6 + c] + a2 * (1.0 / 12.0);
        }
    for (int a = 0; a < 6; ++a) {
        double e = 0.0;
        for (int k = 0; k < 6; ++k) e += J[k * 6 + a] * rp[k];
        g[a] -= s.lamP * e;
        for (int b = a; b < 6; ++b) {
            double m = 0.0;
            for (int k = 0; k < 6; ++k) m += J[k * 6 + a] * J[k * 6 + b];
            A[s6(a, b)] += s.lamP * m;
        }
    }
}

// ---------------------------------------------------------------------------
// kernels

__global__ void k_c_keyframe(Geo g, const float* __restrict__ img, const float* __restrict__ normals,
                             float* __restrict__ Is, float* __restrict__ cxt, float* __restrict__ cyt) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    if (u >= g.W || v >= g.H) return;
    const long dense = (long)v * g.W + u;
    const long p = pix_of(g, u, v);
    Is[p] = img[dense];
    // normal-integration targets of Eq. (gbpni), inactive at grazing normals
    const double q0 = ((double)u - g.cx) / g.fx, q1 = ((double)v - g.cy) / g.fy;
    const double n0 = normals[3 * dense], n1 = normals[3 * dense + 1], n2 = normals[3 * dense + 2];
    const double nq = n0 * q0 + n1 * q1 + n2;
    const double qn = sqrt(q0 * q0 + q1 * q1 + 1.0);
    const bool ok = isfinite(nq) && fabs(nq) >= 1e-3 * qn;
    cxt[p] = ok ? (float)(n0 / (g.fx * nq)) : __int_as_float(0x7fc00000);
    cyt[p] = ok ? (float)(n1 / (g.fy * nq)) : __int_as_float(0x7fc00000);
}

// linearisation at the shared pose and CG start (x = 0, r = g, z = P^-1 r, p = z)
__global__ __launch_bounds__(kThreads) void k_c_linearise(Geo g, Strengths s, Inputs in,
                                                          const CgState* __restrict__ cs, Planes P,
                                                          double* __restrict__ partial) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    double red[kLinPartials];
    for (int k = 0; k < kLinPartials; ++k) red[k] = 0.0;
    if (u < g.W && v < g.H) {
        const long pi = pix_of(g, u, v);
        double tau[6], R[9], t[3], L[28], eta[7];
        for (int k = 0; k < 6; ++k) tau[k] = cs->xi[k];
        se3_exp(tau, R, t);
        const double ell = P.ell[pi];
        // the photometric factor alone (zero prior weight); the log-depth prior
        // is added here, the pose prior once per solve
        Strengths sp = s;
        sp.lamP = 0.0;
        const bool val = unary_factors(g, sp, in, u, v, tau, R, t, ell, L, eta);
        double diag = L[s7(6, 6)] + s.lamP, gl = eta[6] - s.lamP * (ell - s.prior_ell);
        if (s.lamN > 0.0) {
            for (int d = 0; d < 4; ++d) {
                int nu, nv;
                if (!neighbour(g, u, v, d, nu, nv)) continue;
                const long pj = pix_of(g, nu, nv);
                double rn;
                if (normal_residual(g, in, pi, pj, d, ell, P.ell[pj], rn)) {
                    diag += s.lamN;
                    gl -= s.lamN * rn;
                }
            }
        }
        P.diag[pi] = diag;
        for (int k = 0; k < 6; ++k) P.b[(long)k * g.plane + pi] = L[s7(k, 6)];
        P.gl[pi] = gl;
        const double z = gl / diag;
        P.x[pi] = 0.0;
        P.r[pi] = gl;
        P.z[pi] = z;
        P.p0[pi] = z;
        for (int r = 0, k = 0; r < 6; ++r)
            for (int c = r; c < 6; ++c) red[k++] = L[s7(r, c)];
        for (int k = 0; k < 6; ++k) red[21 + k] = eta[k];
        red[27] = gl * z;
        red[28] = gl * gl;
        red[29] = val ? 1.0 : 0.0;
    }
    block_reduce<kLinPartials>(red, partial);
}

__global__ __launch_bounds__(kThreads) void k_c_lin_final(Strengths s, int nb, const double* __restrict__ partial,
                                                          CgState* __restrict__ cs) {
    double tot[kLinPartials];
    final_sum<kLinPartials>(partial, nb, tot);
    if (threadIdx.x != 0) return;
    double xi[6];
    for (int k = 0; k < 6; ++k) xi[k] = cs->xi[k];
    add_pose_prior(s, xi, tot, tot + 21);
    for (int k = 0; k < 21; ++k) cs->A[k] = tot[k];
    for (int k = 0; k < 6; ++k) {
        cs->g[k] = tot[21 + k];
        cs->x[k] = 0.0;
        cs->r[k] = tot[21 + k];
    }
    pose_precondition(cs->A, cs->r, cs->z);
    for (int k = 0; k < 6; ++k) cs->p[k] = cs->z[k];
    cs->rz = tot[27] + dot6(cs->r, cs->z);
    cs->rr0 = tot[28] + dot6(cs->r, cs->r);
    cs->rr = cs->rr0;
    cs->beta = 0.0;
    cs->alpha = 0.0;
    cs->nvalid = tot[29];
    cs->iters = 0;
    cs->done = (cs->rr0 > 0.0) ? 0 : 1;
}

// q = M p with p = z + beta p_prev formed on the fly (written to p_out)
__global__ __launch_bounds__(kThreads) void k_c_matvec(Geo g, Strengths s, Inputs in, const CgState* __restrict__ cs,
                                                       Planes P, const double* __restrict__ p_in,
                                                       double* __restrict__ p_out, double* __restrict__ partial) {
    if (cs->done) return;
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    const double beta = cs->beta;
    double red[kMvPartials];
    for (int k = 0; k < kMvPartials; ++k) red[k] = 0.0;
    if (u < g.W && v < g.H) {
        const long pi = pix_of(g, u, v);
        const double pv_ = P.z[pi] + beta * p_in[pi];
        double q = P.diag[pi] * pv_;
        if (s.lamN > 0.0) {
            for (int d = 0; d < 4; ++d) {
                int nu, nv;
                if (!neighbour(g, u, v, d, nu, nv)) continue;
                const long pj = pix_of(g, nu, nv);
                if (normal_active(g, in, pi, pj, d)) q -= s.lamN * (P.z[pj] + beta * p_in[pj]);
            }
        }
        for (int k = 0; k < 6; ++k) {
            const double bk = P.b[(long)k * g.plane + pi];
            q += bk * cs->p[k];
            red[k] = bk * pv_;
        }
        p_out[pi] = pv_;
        P.q[pi] = q;
        red[6] = pv_ * q;
    }
    block_reduce<kMvPartials>(red, partial);
}

__global__ __launch_bounds__(kThreads) void k_c_alpha(int nb, const double* __restrict__ partial,
                                                      CgState* __restrict__ cs) {
    if (cs->done) return;
    double tot[kMvPartials];
    final_sum<kMvPartials>(partial, nb, tot);
    if (threadIdx.x != 0) return;
    double qx[6];
    sym6_mul(cs->A, cs->p, qx);
    for (int k = 0; k < 6; ++k) qx[k] += tot[k];
    const double pq = tot[6] + dot6(cs->p, qx);
    const double alpha = cs->rz / pq;
    cs->alpha = alpha;
    for (int k = 0; k < 6; ++k) {
        cs->x[k] += alpha * cs->p[k];
        cs->r[k] -= alpha * qx[k];
    }
    pose_precondition(cs->A, cs->r, cs->z);
}

__global__ __launch_bounds__(kThreads) void k_c_update(Geo g, const CgState* __restrict__ cs, Planes P,
                                                       const double* __restrict__ p_cur, double* __restrict__ partial) {
    if (cs->done) return;
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    double red[kUpPartials] = {0.0, 0.0};
    if (u < g.W && v < g.H) {
        const long pi = pix_of(g, u, v);
        const double alpha = cs->alpha;
        P.x[pi] += alpha * p_cur[pi];
        const double r = P.r[pi] - alpha * P.q[pi];
        P.r[pi] = r;
        const double z = r / P.diag[pi];
        P.z[pi] = z;
        red[0] = r * z;
        red[1] = r * r;
    }
    block_reduce<kUpPartials>(red, partial);
}

__global__ __launch_bounds__(kThreads) void k_c_beta(int nb, const double* __restrict__ partial,
                                                     CgState* __restrict__ cs, double tol2) {
    if (cs->done) return;
    double tot[kUpPartials];
    final_sum<kUpPartials>(partial, nb, tot);
    if (threadIdx.x != 0) return;
    const double rz = tot[0] + dot6(cs->r, cs->z);
    const double rr = tot[1] + dot6(cs->r, cs->r);
    cs->beta = rz / cs->rz;
    cs->rz = rz;
    cs->rr = rr;
    for (int k = 0; k < 6; ++k) cs->p[k] = cs->z[k] + cs->beta * cs->p[k];
    cs->iters += 1;
    cs->total += 1;
    if (rr <= tol2 * cs->rr0) cs->done = 1;
}

__global__ void k_c_apply(Geo g, Planes P) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    if (u >= g.W || v >= g.H) return;
    const long pi = pix_of(g, u, v);
    P.ell[pi] += P.x[pi];
}

// xi <- Log(Exp(xi) Exp(d_xi))
__global__ void k_c_apply_pose(CgState* __restrict__ cs) {
    if (threadIdx.x != 0) return;
    double R0[9], t0[3], Rd[9], td[3], R1[9], t1[3], d[6], xi[6];
    for (int k = 0; k < 6; ++k) {
        xi[k] = cs->xi[k];
        d[k] = cs->x[k];
    }
    se3_exp(xi, R0, t0);
    se3_exp(d, Rd, td);
    se3_compose(R0, t0, Rd, td, R1, t1);
    se3_log(R1, t1, xi);
    for (int k = 0; k < 6; ++k) cs->xi[k] = xi[k];
}

__global__ void k_c_dense_depth(Geo g, double* __restrict__ ell, double* __restrict__ dense, int to_dense,
                                float* __restrict__ inv_depth) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    if (u >= g.W || v >= g.H) return;
    const long pi = pix_of(g, u, v), d = (long)v * g.W + u;
    if (dense) {
        if (to_dense) dense[d] = ell[pi];
        else ell[pi] = dense[d];
    }
    if (inv_depth) inv_depth[d] = (float)exp(-ell[pi]);
}

__global__ void k_c_reset_total(CgState* __restrict__ cs) {
    if (threadIdx.x == 0) cs->total = 0;
}

__global__ void k_c_fill(double* __restrict__ p, long n, double v) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

// ---------------------------------------------------------------------------
// the ABI

struct pixvod_central {
    int H = 0, W = 0, pitch = 0;
    long plane = 0;
    pixvod_intrinsics K{};
    pixvod_params P{};
    int max_cg = 0;
    double tol = 0.0;
    hipStream_t own_stream = nullptr, stream = nullptr;
    float *Is = nullptr, *cxt = nullptr, *cyt = nullptr, *It = nullptr, *Gx = nullptr, *Gy = nullptr;
    float *stage = nullptr, *out_stage = nullptr;
    double* planes = nullptr;       // ell, diag, b (6), gl, x, r, z, p0, p1, q
    double* partial = nullptr;
    double* dense = nullptr;
    CgState* cs = nullptr;
    CgState* h_cs = nullptr;        // pinned host copy
    int nb = 0;
    bool have_kf = false;
    double last_ms = 0.0;
    hipEvent_t ev[2] = {nullptr, nullptr};
    // one IRLS iteration captured as a HIP graph on `graph_stream`
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t graph_stream = nullptr;
    std::string err;
};

namespace {

int cfail(pixvod_central* c, int code, const std::string& m) {
    if (c) c->err = m;
    record_error(m);
    return code;
}

#define C_TRY(c, expr)                                                                        \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return cfail((c), PIXVOD_EHIP, std::string(#expr ": ") + hipGetErrorString(e_));  \
    } while (0)

Geo cgeo(const pixvod_central* c) {
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

Planes cplanes(const pixvod_central* c) {
    const long pl = c->plane;
    double* b = c->planes;
    Planes P;
    P.ell = b;
    P.diag = b + pl;
    P.b = b + 2 * pl;
    P.gl = b + 8 * pl;
    P.x = b + 9 * pl;
    P.r = b + 10 * pl;
    P.z = b + 11 * pl;
    P.p0 = b + 12 * pl;
    P.p1 = b + 13 * pl;
    P.q = b + 14 * pl;
    return P;
}
constexpr int kPlanes = 15;

Inputs cinputs(const pixvod_central* c) {
    Inputs in;
    std::memset(&in, 0, sizeof(in));
    in.Is = c->Is;
    in.cxt = c->cxt;
    in.cyt = c->cyt;
    in.It = c->It;
    in.Gx = c->Gx;
    in.Gy = c->Gy;
    return in;
}

dim3 cgrid(const Geo& g) { return dim3((g.W + 63) / 64, (g.H + 3) / 4); }

void crelease(pixvod_central* c) {
    void* bufs[] = {c->Is, c->cxt, c->cyt, c->It, c->Gx, c->Gy, c->stage, c->out_stage, c->planes, c->partial,
                    c->dense, c->cs};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (c->h_cs) (void)hipHostFree(c->h_cs);
    for (hipEvent_t e : c->ev)
        if (e) (void)hipEventDestroy(e);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
}

template <class T>
int calloc_dev(pixvod_central* c, T** p, size_t n) {
    if (hipMalloc((void**)p, n * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        return cfail(c, PIXVOD_ENOMEM, "device allocation failed");
    }
    return PIXVOD_OK;
}

}  // namespace

extern "C" {

int pixvod_central_create(int H, int W, const pixvod_intrinsics* K, const pixvod_params* params, int max_cg,
                          double cg_tol, pixvod_central** out) {
    if (!out) return cfail(nullptr, PIXVOD_EINVAL, "out is NULL");
    *out = nullptr;
    if (H < 2 || W < 2 || (long)H * W > (1L << 26)) return cfail(nullptr, PIXVOD_EINVAL, "need 2 <= H, W and H*W <= 2^26");
    if (!K || !(K->fx > 0) || !(K->fy > 0) || !std::isfinite(K->cx) || !std::isfinite(K->cy))
        return cfail(nullptr, PIXVOD_EINVAL, "intrinsics must be finite with fx, fy > 0");
    if (max_cg < 1 || !(cg_tol > 0.0) || !(cg_tol < 1.0)) return cfail(nullptr, PIXVOD_EINVAL, "need max_cg >= 1, 0 < cg_tol < 1");
    pixvod_params P;
    if (params) P = *params;
    else pixvod_default_params(&P);
    if (!params_valid(&P)) return cfail(nullptr, PIXVOD_EINVAL, "invalid parameters");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return cfail(nullptr, PIXVOD_ENODEV, "no HIP device");
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
        std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return cfail(nullptr, PIXVOD_ENODEV, "need a gfx950 device");
    pixvod_central* c = new pixvod_central();
    c->H = H;
    c->W = W;
    c->pitch = (W + 63) / 64 * 64;
    c->plane = (long)H * c->pitch;
    c->K = *K;
    c->P = P;
    c->max_cg = max_cg;
    c->tol = cg_tol;
    const Geo g = cgeo(c);
    const dim3 gr = cgrid(g);
    c->nb = (int)(gr.x * gr.y);
    const size_t pl = (size_t)c->plane, N = (size_t)H * W;
    int rc = PIXVOD_OK;
    float** fb[] = {&c->Is, &c->cxt, &c->cyt, &c->It, &c->Gx, &c->Gy};
    for (float** f : fb)
        if (!rc) rc = calloc_dev(c, f, pl);
    if (!rc) rc = calloc_dev(c, &c->stage, 4 * N);
    if (!rc) rc = calloc_dev(c, &c->out_stage, N);
    if (!rc) rc = calloc_dev(c, &c->planes, pl * kPlanes);
    if (!rc) rc = calloc_dev(c, &c->partial, (size_t)c->nb * kLinPartials);
    if (!rc) rc = calloc_dev(c, &c->dense, N);
    if (!rc) rc = calloc_dev(c, &c->cs, 1);
    if (!rc && hipHostMalloc((void**)&c->h_cs, sizeof(CgState)) != hipSuccess) rc = cfail(c, PIXVOD_ENOMEM, "pinned allocation failed");
    if (!rc && hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking) != hipSuccess) rc = PIXVOD_EHIP;
    if (!rc && (hipEventCreate(&c->ev[0]) != hipSuccess || hipEventCreate(&c->ev[1]) != hipSuccess)) rc = PIXVOD_EHIP;
    if (rc) {
        std::string m = c->err.empty() ? "allocation failed" : c->err;
        crelease(c);
        delete c;
        return cfail(nullptr, rc, m);
    }
    c->stream = c->own_stream;
    // initial point: identity pose, log-depth -log(init_inv_depth), zero planes
    const long n = (long)pl * kPlanes;
    hipLaunchKernelGGL(k_c_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, c->planes, n, 0.0);
    hipLaunchKernelGGL(k_c_fill, dim3((unsigned)((pl + 255) / 256)), dim3(256), 0, c->stream, c->planes, (long)pl,
                       -std::log((double)P.init_inv_depth));
    std::memset(c->h_cs, 0, sizeof(CgState));
    if (hipMemcpyAsync(c->cs, c->h_cs, sizeof(CgState), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        crelease(c);
        delete c;
        return cfail(nullptr, PIXVOD_EHIP, "initialisation failed");
    }
    *out = c;
    return PIXVOD_OK;
}

int pixvod_central_destroy(pixvod_central* c) {
    if (!c) return PIXVOD_OK;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    crelease(c);
    delete c;
    return PIXVOD_OK;
}

int pixvod_central_set_stream(pixvod_central* c, void* s) {
    if (!c) return cfail(nullptr, PIXVOD_EINVAL, "solver is NULL");
    C_TRY(c, hipStreamSynchronize(c->stream));
    c->stream = s ? (hipStream_t)s : c->own_stream;
    return PIXVOD_OK;
}

int pixvod_central_set_keyframe(pixvod_central* c, const float* img, const float* normals, int where) {
    if (!c) return cfail(nullptr, PIXVOD_EINVAL, "solver is NULL");
    if (!img || !normals || (where != PIXVOD_HOST && where != PIXVOD_DEVICE))
        return cfail(c, PIXVOD_EINVAL, "img, normals and a valid location are required");
    const size_t N = (size_t)c->H * c->W;
    const float *di = img, *dn = normals;
    if (where == PIXVOD_HOST) {
        C_TRY(c, hipMemcpyAsync(c->stage, img, N * sizeof(float), hipMemcpyHostToDevice, c->stream));
        C_TRY(c, hipMemcpyAsync(c->stage + N, normals, 3 * N * sizeof(float), hipMemcpyHostToDevice, c->stream));
        di = c->stage;
        dn = c->stage + N;
    }
    const Geo g = cgeo(c);
    hipLaunchKernelGGL(k_c_keyframe, cgrid(g), dim3(64, 4), 0, c->stream, g, di, dn, c->Is, c->cxt, c->cyt);
    C_TRY(c, hipGetLastError());
    // the pose restarts at the identity; log-depths are kept
    for (int k = 0; k < 6; ++k) c->h_cs->xi[k] = 0.0;
    C_TRY(c, hipMemcpyAsync(c->cs, c->h_cs->xi, sizeof(double) * 6, hipMemcpyHostToDevice, c->stream));
    C_TRY(c, hipStreamSynchronize(c->stream));
    c->have_kf = true;
    return PIXVOD_OK;
}

int pixvod_central_set_point(pixvod_central* c, const double xi[6], const double* log_depth) {
    if (!c) return cfail(nullptr, PIXVOD_EINVAL, "solver is NULL");
    if (xi) {
        for (int k = 0; k < 6; ++k) {
            if (!std::isfinite(xi[k])) return cfail(c, PIXVOD_EINVAL, "xi must be finite");
            c->h_cs->xi[k] = xi[k];
        }
        C_TRY(c, hipMemcpyAsync(c->cs, c->h_cs->xi, sizeof(double) * 6, hipMemcpyHostToDevice, c->stream));
    }
    if (log_depth) {
        const size_t N = (size_t)c->H * c->W;
        C_TRY(c, hipMemcpyAsync(c->dense, log_depth, N * sizeof(double), hipMemcpyHostToDevice, c->stream));
        const Geo g = cgeo(c);
        hipLaunchKernelGGL(k_c_dense_depth, cgrid(g), dim3(64, 4), 0, c->stream, g, cplanes(c).ell, c->dense, 0,
                           (float*)nullptr);
        C_TRY(c, hipGetLastError());
    }
    C_TRY(c, hipStreamSynchronize(c->stream));
    return PIXVOD_OK;
}

int pixvod_central_get_point(pixvod_central* c, double xi[6], double* log_depth) {
    if (!c) return cfail(nullptr, PIXVOD_EINVAL, "solver is NULL");
    if (log_depth) {
        const size_t N = (size_t)c->H * c->W;
        const Geo g = cgeo(c);
        hipLaunchKernelGGL(k_c_dense_depth, cgrid(g), dim3(64, 4), 0, c->stream, g, cplanes(c).ell, c->dense, 1,
                           (float*)nullptr);
        C_TRY(c, hipGetLastError());
        C_TRY(c, hipMemcpyAsync(log_depth, c->dense, N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    }
    C_TRY(c, hipMemcpyAsync(c->h_cs, c->cs, sizeof(CgState), hipMemcpyDeviceToHost, c->stream));
    C_TRY(c, hipStreamSynchronize(c->stream));
    if (xi)
        for (int k = 0; k < 6; ++k) xi[k] = c->h_cs->xi[k];
    return PIXVOD_OK;
}

int pixvod_central_track(pixvod_central* c, const float* frame, int where, int n_iters, double xi_out[6],
                         float* inv_depth, int out_where, pixvod_central_stats* stats) {
    if (!c) return cfail(nullptr, PIXVOD_EINVAL, "solver is NULL");
    if (!frame || (where != PIXVOD_HOST && where != PIXVOD_DEVICE) ||
        (out_where != PIXVOD_HOST && out_where != PIXVOD_DEVICE) || n_iters < 0)
        return cfail(c, PIXVOD_EINVAL, "frame, valid locations and n_iters >= 0 are required");
    if (!c->have_kf) return cfail(c, PIXVOD_ESTATE, "no keyframe");
    const size_t N = (size_t)c->H * c->W;
    const Geo g = cgeo(c);
    const float* df = frame;
    if (where == PIXVOD_HOST) {
        C_TRY(c, hipMemcpyAsync(c->stage, frame, N * sizeof(float), hipMemcpyHostToDevice, c->stream));
        df = c->stage;
    }
    C_TRY(c, launch_frame_prep(g, df, c->W, c->It, c->Gx, c->Gy, c->stream));
    const Strengths s = strengths_from(c->P, false);
    const Inputs in = cinputs(c);
    const Planes P = cplanes(c);
    const dim3 gr = cgrid(g), blk(64, 4);
    const double tol2 = c->tol * c->tol;
    // one IRLS iteration: linearise, max_cg CG iterations (the launches after
    // convergence return at once), apply the step
    auto irls_iteration = [&](hipStream_t st) {
        hipLaunchKernelGGL(k_c_linearise, gr, blk, 0, st, g, s, in, c->cs, P, c->partial);
        hipLaunchKernelGGL(k_c_lin_final, dim3(1), dim3(kThreads), 0, st, s, c->nb, c->partial, c->cs);
        for (int k = 0; k < c->max_cg; ++k) {
            const double* pin = (k & 1) ? P.p1 : P.p0;
            double* pout = (k & 1) ? P.p0 : P.p1;
            hipLaunchKernelGGL(k_c_matvec, gr, blk, 0, st, g, s, in, c->cs, P, pin, pout, c->partial);
            hipLaunchKernelGGL(k_c_alpha, dim3(1), dim3(kThreads), 0, st, c->nb, c->partial, c->cs);
            hipLaunchKernelGGL(k_c_update, gr, blk, 0, st, g, c->cs, P, pout, c->partial);
            hipLaunchKernelGGL(k_c_beta, dim3(1), dim3(kThreads), 0, st, c->nb, c->partial, c->cs, tol2);
        }
        hipLaunchKernelGGL(k_c_apply, gr, blk, 0, st, g, P);
        hipLaunchKernelGGL(k_c_apply_pose, dim3(1), dim3(64), 0, st, c->cs);
    };
    // captured once per stream as a graph (every argument is fixed for the
    // solver's lifetime); plain launches if capture is unavailable
    if (n_iters > 0 && c->graph_stream != c->stream) {
        if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
        if (c->graph) (void)hipGraphDestroy(c->graph);
        c->graph_exec = nullptr;
        c->graph = nullptr;
        c->graph_stream = nullptr;
        if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            irls_iteration(c->stream);
            hipGraph_t gph = nullptr;
            if (hipStreamEndCapture(c->stream, &gph) == hipSuccess && gph) {
                hipGraphExec_t ex = nullptr;
                if (hipGraphInstantiate(&ex, gph, nullptr, nullptr, 0) == hipSuccess) {
                    c->graph = gph;
                    c->graph_exec = ex;
                    c->graph_stream = c->stream;
                } else {
                    (void)hipGraphDestroy(gph);
                }
            }
        }
        (void)hipGetLastError();
    }
    hipLaunchKernelGGL(k_c_reset_total, dim3(1), dim3(64), 0, c->stream, c->cs);
    C_TRY(c, hipEventRecord(c->ev[0], c->stream));
    for (int it = 0; it < n_iters; ++it) {
        if (c->graph_exec) C_TRY(c, hipGraphLaunch(c->graph_exec, c->stream));
        else irls_iteration(c->stream);
        C_TRY(c, hipGetLastError());
    }
    C_TRY(c, hipEventRecord(c->ev[1], c->stream));
    float* d_inv = inv_depth;
    if (inv_depth && out_where == PIXVOD_HOST) d_inv = c->out_stage;
    if (inv_depth) {
        hipLaunchKernelGGL(k_c_dense_depth, gr, blk, 0, c->stream, g, P.ell, (double*)nullptr, 1, d_inv);
        C_TRY(c, hipGetLastError());
        if (out_where == PIXVOD_HOST)
            C_TRY(c, hipMemcpyAsync(inv_depth, c->out_stage, N * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    }
    C_TRY(c, hipMemcpyAsync(c->h_cs, c->cs, sizeof(CgState), hipMemcpyDeviceToHost, c->stream));
    C_TRY(c, hipStreamSynchronize(c->stream));
    float ms = 0.0f;
    C_TRY(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
    c->last_ms = ms;
    bool finite = true;
    for (int k = 0; k < 6; ++k) {
        if (xi_out) xi_out[k] = c->h_cs->xi[k];
        finite = finite && std::isfinite(c->h_cs->xi[k]);
    }
    if (stats) {
        stats->cg_iters = c->h_cs->total;
        stats->last_cg_iters = n_iters > 0 ? c->h_cs->iters : 0;
        stats->last_rel_residual = (n_iters > 0 && c->h_cs->rr0 > 0.0) ? std::sqrt(c->h_cs->rr / c->h_cs->rr0) : 0.0;
        stats->valid_fraction = n_iters > 0 ? (float)(c->h_cs->nvalid / (double)N) : 0.0f;
        stats->flags = finite ? 0u : (uint32_t)PIXVOD_DIVERGED;
    }
    return PIXVOD_OK;
}

int pixvod_central_last_ms(const pixvod_central* c, double* ms) {
    if (!c || !ms) return cfail(const_cast<pixvod_central*>(c), PIXVOD_EINVAL, "solver and ms are required");
    *ms = c->last_ms;
    return PIXVOD_OK;
}

}  // extern "C"
