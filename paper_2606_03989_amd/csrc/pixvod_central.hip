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
//      vectors, to a relative residual tolerance;
//   3. applies xi <- Log(Exp(xi) Exp(d_xi)), ell <- ell + d_ell.
// The conjugate gradients take the single-reduction form of Chronopoulos and
// Gear (1989): with u = P^-1 r and w = M u carried along, the two inner
// products of an iteration (r.u, w.u) come out of one reduction, so each CG
// iteration is one launch over the pixels. The launch updates p, s = M p, x
// and r, forms the new u and, from the neighbours' new u (recomputed by each
// pixel from the neighbours' stored r, w, s, so that no pixel waits for
// another), the new w, and writes per-workgroup partial sums. Its scalar step
// (alpha and beta from the previous launch's partial sums, the pose block's
// part of every vector, the stop test) is evaluated by every workgroup in
// one fixed order, so all take the same values. The scalars pass between
// launches in two alternating records, the per-pixel vectors read by
// neighbours (r, w, s) in two alternating plane sets, the partial sums in two
// alternating buffers, so no launch reads what it writes. The host launches
// the iterations in chunks and stops after the chunk that follows the first
// one whose end state reports convergence (launches after convergence return
// at once).
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
constexpr int kLinPartials = 29;   // A (21), g_xi (6), r.r, valid count
constexpr int kCgPartials = 9;     // r.u, w.u, r.r, sum b_i u_i (6)
constexpr int kCgThreads = 256;    // work-items per workgroup of the CG launches
constexpr int kCgPx = 2;           // pixels per work-item and round in those launches
constexpr int kCgMaxBlocks = 1024; // most workgroups of those launches (a multiple of 8)
constexpr int kCgChunk = 16;       // CG iterations launched between convergence checks

// solver state in device memory
struct CgState {
    double xi[6];
    double A[21];        // pose block, packed upper
    double Ainv[21];     // its inverse (the pose part of the preconditioner)
    double g[6];         // pose right-hand side
    double x[6];         // the pose step of the last solve
    double rr0, rr;      // |r|^2 at the start and the end of the last solve
    double nvalid;
    int done, iters;     // this solve
    int total;           // CG iterations since the frame started
};

// the CG state between launches: pose parts of the vectors and the scalars
// of the last step
struct CgIter {
    double x[6], r[6], u[6], p[6], s[6];
    double gamma, alpha, rr;
    int done, iters;
};

struct Planes {            // per-pixel FP64 planes (pitched)
    double *ell, *diag, *b, *gl, *x, *p;
    double *r[2], *w[2], *s[2];   // read by neighbours: two alternating sets
};

// ---------------------------------------------------------------------------
// reductions: wavefront butterflies of lane exchanges, then the wavefronts'
// sums in order. Every step adds the same two operands in every lane (in
// either order), so all lanes hold the same sum, and a reduction evaluated
// in several workgroups over the same data gives the same value in each.

template <int NV>
__device__ inline void wave_sum(double v[NV]) {
    for (int m = 32; m > 0; m >>= 1)
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] += __shfl_xor(v[k], m, 64);
}

// workgroup (NT work-items) sum of NV doubles per work-item into
// partial[block * NV + k]
template <int NV, int NT>
__device__ inline void block_reduce(double v[NV], double* __restrict__ partial) {
    __shared__ double sh[NT / 64][NV];
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int lane = tid & 63, w = tid >> 6;
    const long blk = (long)blockIdx.x + (long)blockIdx.y * gridDim.x;
    wave_sum<NV>(v);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[w][k] = v[k];
    __syncthreads();
    if (tid < NV) {
        double t = 0.0;
        for (int j = 0; j < NT / 64; ++j) t += sh[j][tid];
        partial[blk * NV + tid] = t;
    }
}

// sum of nb partial records of NV doubles, in one fixed order, given to
// every work-item of the workgroup (NT work-items, 1-D); once per kernel
template <int NV, int NT>
__device__ inline void final_sum(const double* __restrict__ partial, int nb, double out[NV]) {
    __shared__ double sh[NT / 64][NV];
    __shared__ double tot[NV];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double t[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) t[k] = 0.0;
    for (int b = threadIdx.x; b < nb; b += NT)
#pragma unroll
        for (int k = 0; k < NV; ++k) t[k] += partial[(long)b * NV + k];
    wave_sum<NV>(t);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[w][k] = t[k];
    __syncthreads();
    if (threadIdx.x < NV) {
        double u = 0.0;
        for (int j = 0; j < NT / 64; ++j) u += sh[j][threadIdx.x];
        tot[threadIdx.x] = u;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) out[k] = tot[k];
}

// inverse of the packed 6x6 pose block (through its Cholesky factor)
__device__ inline void pose_inverse(const double A[21], double Ai[21]) {
    double L[21], idg[6];
    for (int k = 0; k < 21; ++k) L[k] = A[k];
    chol6(L, idg);
    chol6_inverse(L, idg, Ai);
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

// per pixel, bit d: the normal edge to neighbour d exists and is active (a
// keyframe property)
__global__ void k_c_edges(Geo g, Inputs in, unsigned char* __restrict__ act) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    if (u >= g.W || v >= g.H) return;
    const long pi = pix_of(g, u, v);
    int a = 0;
    for (int d = 0; d < 4; ++d) {
        int nu, nv;
        if (neighbour(g, u, v, d, nu, nv) && normal_active(g, in, pi, pix_of(g, nu, nv), d)) a |= 1 << d;
    }
    act[pi] = (unsigned char)a;
}

// linearisation at the shared pose and CG start (x = 0, r = g)
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
        P.x[pi] = 0.0;
        P.r[0][pi] = gl;
        for (int r = 0, k = 0; r < 6; ++r)
            for (int c = r; c < 6; ++c) red[k++] = L[s7(r, c)];
        for (int k = 0; k < 6; ++k) red[21 + k] = eta[k];
        red[27] = gl * gl;
        red[28] = val ? 1.0 : 0.0;
    }
    block_reduce<kLinPartials, kThreads>(red, partial);
}

// the pose block, its inverse, the pose part of the CG start (x = 0, r = g,
// u = A^-1 g) and |r_0|^2
__global__ __launch_bounds__(kThreads) void k_c_lin_final(Strengths s, int nb, const double* __restrict__ partial,
                                                          CgState* __restrict__ cs, CgIter* __restrict__ rec0) {
    double tot[kLinPartials];
    final_sum<kLinPartials, kThreads>(partial, nb, tot);
    if (threadIdx.x != 0) return;
    double xi[6];
    for (int k = 0; k < 6; ++k) xi[k] = cs->xi[k];
    add_pose_prior(s, xi, tot, tot + 21);
    for (int k = 0; k < 21; ++k) cs->A[k] = tot[k];
    for (int k = 0; k < 6; ++k) cs->g[k] = tot[21 + k];
    pose_inverse(cs->A, cs->Ainv);
    CgIter st;
    for (int k = 0; k < 6; ++k) {
        st.x[k] = 0.0;
        st.r[k] = cs->g[k];
        st.p[k] = 0.0;
        st.s[k] = 0.0;
    }
    sym6_mul(cs->Ainv, st.r, st.u);
    cs->rr0 = tot[27] + dot6(st.r, st.r);
    cs->rr = cs->rr0;
    cs->nvalid = tot[28];
    cs->iters = 0;
    cs->done = (cs->rr0 > 0.0) ? 0 : 1;
    st.gamma = 0.0;
    st.alpha = 0.0;
    st.rr = cs->rr0;
    st.done = cs->done;
    st.iters = 0;
    *rec0 = st;
}

// The CG launches: kCgThreads work-items per workgroup, kCgPx pixels per
// work-item and round (range base + j * kCgThreads + work-item). Workgroup b
// takes range (b mod 8) * (nbx / 8) + b / 8 (nbx, the grid, a multiple of 8):
// workgroups are dealt to the eight XCDs in turn, so each XCD gets adjacent
// ranges and finds most of their vertical neighbours in its own L2. Rounds
// stride over the image when the grid is smaller than it. The first round's
// own-pixel loads are issued before the scalar step, which does not depend on
// them; the neighbours' (L1 and L2 hits: other work-items load them as their
// own) after it.

__device__ inline int cg_range(int b, int nbx) { return (b & 7) * (nbx >> 3) + (b >> 3); }

struct CgPix {             // what an iteration needs of one pixel's own planes
    int u, v, act;
    double x, p, r, w, s, diag, b[6];
};

__device__ inline void cg_load(const Geo& g, const Planes& P, const unsigned char* __restrict__ act, int cur,
                               bool first, int i, CgPix& a) {
    a.u = i % g.W;
    a.v = i / g.W;
    const long pi = pix_of(g, a.u, a.v);
    a.act = act[pi];
    a.x = P.x[pi];
    a.p = first ? 0.0 : P.p[pi];
    a.r = P.r[cur][pi];
    a.w = P.w[cur][pi];
    a.s = first ? 0.0 : P.s[cur][pi];
    a.diag = P.diag[pi];
#pragma unroll
    for (int k = 0; k < 6; ++k) a.b[k] = P.b[(long)k * g.plane + pi];
}

// one pixel's new residual and preconditioned residual from its stored r, w,
// s (explicit FMAs, so that a pixel and its neighbours evaluate the same
// expression bit for bit)
__device__ inline double cg_new_r(double r, double w, double s_prev, double alpha, double beta, bool first,
                                  double& s_new) {
    s_new = first ? w : fma(beta, s_prev, w);
    return fma(-alpha, s_new, r);
}

// w = M u at one pixel: the diagonal, the active normal edges and the pose
// column, with the partial sums of r.u, w.u, r.r and b_k u
__device__ inline void cg_apply_pixel(double diag, const double b[6], const double un[4], int act, double lamN,
                                      const double upose[6], double r, double u, double& w, double red[kCgPartials]) {
    double q = diag * u;
#pragma unroll
    for (int d = 0; d < 4; ++d)
        if (act & (1 << d)) q -= lamN * un[d];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        q += b[k] * upose[k];
        red[3 + k] += b[k] * u;
    }
    w = q;
    red[0] += r * u;
    red[1] += q * u;
    red[2] += r * r;
}

// CG start: u_0 = P^-1 r_0 and w_0 = M u_0 (planes of set 0), partial sums
__global__ __launch_bounds__(kCgThreads) void k_c_cg_init(Geo g, Strengths s, Planes P,
                                                          const unsigned char* __restrict__ act,
                                                          const CgIter* __restrict__ rec0,
                                                          double* __restrict__ part_out) {
    __shared__ double sh_u[6];
    __shared__ int sh_done;
    if (threadIdx.x == 0) {
        for (int k = 0; k < 6; ++k) sh_u[k] = rec0->u[k];
        sh_done = rec0->done;
    }
    __syncthreads();
    if (sh_done) return;
    double up[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) up[k] = sh_u[k];
    double red[kCgPartials];
#pragma unroll
    for (int k = 0; k < kCgPartials; ++k) red[k] = 0.0;
    const int N = g.H * g.W;
    const int round = kCgThreads * kCgPx;
    for (int rb = cg_range(blockIdx.x, gridDim.x); rb * round < N; rb += gridDim.x) {
#pragma unroll
        for (int j = 0; j < kCgPx; ++j) {
            const int i = rb * round + j * kCgThreads + threadIdx.x;
            if (i >= N) continue;
            const int u = i % g.W, v = i / g.W;
            const long pi = pix_of(g, u, v);
            const double r = P.r[0][pi], diag = P.diag[pi];
            double b[6], un[4];
#pragma unroll
            for (int k = 0; k < 6; ++k) b[k] = P.b[(long)k * g.plane + pi];
            const int ea = s.lamN > 0.0 ? act[pi] : 0;
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                un[d] = 0.0;
                if (ea & (1 << d)) {
                    int nu, nv;
                    neighbour(g, u, v, d, nu, nv);
                    const long pj = pix_of(g, nu, nv);
                    un[d] = P.r[0][pj] / P.diag[pj];
                }
            }
            double w;
            cg_apply_pixel(diag, b, un, ea, s.lamN, up, r, r / diag, w, red);
            P.w[0][pi] = w;
        }
    }
    block_reduce<kCgPartials, kCgThreads>(red, part_out);
}

// CG iteration k (planes of set cur in, set 1 - cur out): the scalar step
//   gamma = r.u, delta = w.u (w's pose part: A u + sum b_i u_i), stop test,
//   beta = gamma / gamma_prev, alpha = gamma / (delta - beta gamma / alpha_prev)
//   (k = 0: beta = 0, alpha = gamma / delta),
// then p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s, u = P^-1 r,
// w = M u and the partial sums for the next step. The scalar step runs on the
// first work-item of each workgroup and reaches the others via LDS.
__global__ __launch_bounds__(kCgThreads, 3) void k_c_cg_iter(Geo g, Strengths s, const CgState* __restrict__ cs,
                                                             Planes P, const unsigned char* __restrict__ act,
                                                             const CgIter* __restrict__ rin,
                                                             CgIter* __restrict__ rout,
                                                             const double* __restrict__ part_in,
                                                             double* __restrict__ part_out, int cur, double tol2,
                                                             int first, int* __restrict__ done_flag) {
    __shared__ double sh_u[6];
    __shared__ double sh_ab[2];
    __shared__ int sh_done;
    if (rin->done) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            *rout = *rin;
            if (done_flag) *done_flag = 1;
        }
        return;
    }
    const int N = g.H * g.W;
    const int round = kCgThreads * kCgPx;
    int rb = cg_range(blockIdx.x, gridDim.x);
    CgPix a[kCgPx];
#pragma unroll
    for (int j = 0; j < kCgPx; ++j) {
        const int i = rb * round + j * kCgThreads + threadIdx.x;
        if (i < N) cg_load(g, P, act, cur, first != 0, i, a[j]);
    }
    double tot[kCgPartials];
    final_sum<kCgPartials, kCgThreads>(part_in, gridDim.x, tot);
    if (threadIdx.x == 0) {
        CgIter st = *rin;
        double w[6];
        sym6_mul(cs->A, st.u, w);
        for (int k = 0; k < 6; ++k) w[k] += tot[3 + k];
        const double gamma = tot[0] + dot6(st.r, st.u);
        const double delta = tot[1] + dot6(w, st.u);
        const double rr = tot[2] + dot6(st.r, st.r);
        if (!first) {
            st.iters += 1;
            if (rr <= tol2 * cs->rr0) st.done = 1;
        }
        st.rr = rr;
        double alpha = 0.0, beta = 0.0;
        if (!st.done) {
            beta = first ? 0.0 : gamma / st.gamma;
            alpha = first ? gamma / delta : gamma / (delta - beta * gamma / st.alpha);
            for (int k = 0; k < 6; ++k) {
                st.p[k] = first ? st.u[k] : fma(beta, st.p[k], st.u[k]);
                st.s[k] = first ? w[k] : fma(beta, st.s[k], w[k]);
                st.x[k] = fma(alpha, st.p[k], st.x[k]);
                st.r[k] = fma(-alpha, st.s[k], st.r[k]);
            }
            sym6_mul(cs->Ainv, st.r, st.u);
            st.gamma = gamma;
            st.alpha = alpha;
        }
        for (int k = 0; k < 6; ++k) sh_u[k] = st.u[k];
        sh_ab[0] = alpha;
        sh_ab[1] = beta;
        sh_done = st.done;
        if (blockIdx.x == 0) {
            *rout = st;
            if (done_flag) *done_flag = st.done;
        }
    }
    __syncthreads();
    if (sh_done) return;
    const double alpha = sh_ab[0], beta = sh_ab[1], lamN = s.lamN;
    const int nxt = 1 - cur;
    double up[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) up[k] = sh_u[k];
    double red[kCgPartials];
#pragma unroll
    for (int k = 0; k < kCgPartials; ++k) red[k] = 0.0;
    while (true) {
#pragma unroll
        for (int j = 0; j < kCgPx; ++j) {
            const int i = rb * round + j * kCgThreads + threadIdx.x;
            if (i >= N) continue;
            const CgPix& c = a[j];
            const long pi = pix_of(g, c.u, c.v);
            double un[4];
            const int ea = lamN > 0.0 ? c.act : 0;
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                un[d] = 0.0;
                if (ea & (1 << d)) {
                    int nu, nv;
                    neighbour(g, c.u, c.v, d, nu, nv);
                    const long pj = pix_of(g, nu, nv);
                    double sj;
                    const double rj = cg_new_r(P.r[cur][pj], P.w[cur][pj], first ? 0.0 : P.s[cur][pj], alpha, beta,
                                               first != 0, sj);
                    un[d] = rj / P.diag[pj];
                }
            }
            const double u_old = c.r / c.diag;
            const double pn = first ? u_old : fma(beta, c.p, u_old);
            double sv;
            const double r = cg_new_r(c.r, c.w, c.s, alpha, beta, first != 0, sv);
            double w;
            cg_apply_pixel(c.diag, c.b, un, ea, lamN, up, r, r / c.diag, w, red);
            P.x[pi] = fma(alpha, pn, c.x);
            P.p[pi] = pn;
            P.s[nxt][pi] = sv;
            P.r[nxt][pi] = r;
            P.w[nxt][pi] = w;
        }
        rb += gridDim.x;
        if (rb * round >= N) break;
#pragma unroll
        for (int j = 0; j < kCgPx; ++j) {
            const int i = rb * round + j * kCgThreads + threadIdx.x;
            if (i < N) cg_load(g, P, act, cur, first != 0, i, a[j]);
        }
    }
    block_reduce<kCgPartials, kCgThreads>(red, part_out);
}

// after the last launched iteration: the stop test of the last update (if the
// solve had not stopped) and the solve's results into the solver state
__global__ __launch_bounds__(kCgThreads) void k_c_cg_end(CgState* __restrict__ cs, const CgIter* __restrict__ rin,
                                                         const double* __restrict__ part_in, int nbx, double tol2) {
    CgIter st = *rin;
    if (!st.done) {
        double tot[kCgPartials];
        final_sum<kCgPartials, kCgThreads>(part_in, nbx, tot);
        st.rr = tot[2] + dot6(st.r, st.r);
        st.iters += 1;
        if (st.rr <= tol2 * cs->rr0) st.done = 1;
    }
    if (threadIdx.x != 0) return;
    for (int k = 0; k < 6; ++k) cs->x[k] = st.x[k];
    cs->rr = st.rr;
    cs->done = st.done;
    cs->iters = st.iters;
    cs->total += st.iters;
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
    double* planes = nullptr;       // ell, diag, b (6), gl, x, p, r (2), w (2), s (2)
    double* partial = nullptr;
    double* dense = nullptr;
    CgState* cs = nullptr;
    CgState* h_cs = nullptr;        // pinned host copy
    int nb = 0;
    bool have_kf = false;
    double last_ms = 0.0;
    hipEvent_t ev[2] = {nullptr, nullptr};
    CgIter* rec = nullptr;          // the CG launches' two scalar records
    double* part_cg = nullptr;      // their per-workgroup partial sums (two alternating buffers)
    unsigned char* act = nullptr;   // active normal edges per pixel (bit per direction)
    int* h_done = nullptr;          // pinned, coherent: the stop flag after each of the last two chunks
    int* d_done = nullptr;          // its device address
    hipEvent_t evc[2] = {nullptr, nullptr};
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
    P.p = b + 10 * pl;
    for (int k = 0; k < 2; ++k) {
        P.r[k] = b + (11 + k) * pl;
        P.w[k] = b + (13 + k) * pl;
        P.s[k] = b + (15 + k) * pl;
    }
    return P;
}
constexpr int kPlanes = 17;

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
    void* bufs[] = {c->Is,     c->cxt,   c->cyt,   c->It,      c->Gx,         c->Gy,    c->stage, c->out_stage,
                    c->planes, c->partial, c->dense, c->cs, c->rec, c->part_cg, c->act};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (c->h_cs) (void)hipHostFree(c->h_cs);
    if (c->h_done) (void)hipHostFree(c->h_done);
    for (hipEvent_t e : c->ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->evc)
        if (e) (void)hipEventDestroy(e);
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
    if (!rc) rc = calloc_dev(c, &c->rec, 2);
    if (!rc) rc = calloc_dev(c, &c->part_cg, (size_t)2 * kCgMaxBlocks * kCgPartials);
    if (!rc && hipHostMalloc((void**)&c->h_cs, sizeof(CgState)) != hipSuccess) rc = cfail(c, PIXVOD_ENOMEM, "pinned allocation failed");
    if (!rc) rc = calloc_dev(c, &c->act, pl);
    if (!rc && (hipHostMalloc((void**)&c->h_done, 2 * sizeof(int), hipHostMallocMapped | hipHostMallocCoherent) !=
                    hipSuccess ||
                hipHostGetDevicePointer((void**)&c->d_done, c->h_done, 0) != hipSuccess))
        rc = cfail(c, PIXVOD_ENOMEM, "pinned allocation failed");
    if (!rc && hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking) != hipSuccess) rc = PIXVOD_EHIP;
    if (!rc && (hipEventCreate(&c->ev[0]) != hipSuccess || hipEventCreate(&c->ev[1]) != hipSuccess)) rc = PIXVOD_EHIP;
    if (!rc && (hipEventCreateWithFlags(&c->evc[0], hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&c->evc[1], hipEventDisableTiming) != hipSuccess))
        rc = PIXVOD_EHIP;
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
    hipLaunchKernelGGL(k_c_edges, cgrid(g), dim3(64, 4), 0, c->stream, g, cinputs(c), c->act);
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
    const long round = (long)kCgThreads * kCgPx;
    const int nbx = (int)std::min<long>(((long)N + 8 * round - 1) / (8 * round) * 8, kCgMaxBlocks);
    double* part[2] = {c->part_cg, c->part_cg + (size_t)kCgMaxBlocks * kCgPartials};
    const hipStream_t st = c->stream;
    hipLaunchKernelGGL(k_c_reset_total, dim3(1), dim3(64), 0, st, c->cs);
    C_TRY(c, hipEventRecord(c->ev[0], st));
    for (int it = 0; it < n_iters; ++it) {
        // linearise, CG start, then CG iterations in chunks: the last launch of
        // chunk j writes the stop flag to host memory; after launching chunk
        // j the host waits for chunk j - 1's (chunk j keeps the device busy
        // meanwhile)
        hipLaunchKernelGGL(k_c_linearise, gr, blk, 0, st, g, s, in, c->cs, P, c->partial);
        hipLaunchKernelGGL(k_c_lin_final, dim3(1), dim3(kThreads), 0, st, s, c->nb, c->partial, c->cs, c->rec);
        hipLaunchKernelGGL(k_c_cg_init, dim3(nbx), dim3(kCgThreads), 0, st, g, s, P, c->act, c->rec, part[0]);
        C_TRY(c, hipGetLastError());
        int launched = 0;
        for (int chunk = 0; launched < c->max_cg; ++chunk) {
            const int n = std::min(kCgChunk, c->max_cg - launched);
            const bool last = launched + n >= c->max_cg;
            for (int k = launched; k < launched + n; ++k) {
                const int cur = k & 1;
                int* flag = (!last && k == launched + n - 1) ? c->d_done + (chunk & 1) : nullptr;
                hipLaunchKernelGGL(k_c_cg_iter, dim3(nbx), dim3(kCgThreads), 0, st, g, s, c->cs, P, c->act,
                                   c->rec + cur, c->rec + (1 - cur), part[cur], part[1 - cur], cur, tol2,
                                   k == 0 ? 1 : 0, flag);
            }
            C_TRY(c, hipGetLastError());
            launched += n;
            if (last) break;
            C_TRY(c, hipEventRecord(c->evc[chunk & 1], st));
            if (chunk > 0) {
                C_TRY(c, hipEventSynchronize(c->evc[(chunk - 1) & 1]));
                if (c->h_done[(chunk - 1) & 1]) break;
            }
        }
        hipLaunchKernelGGL(k_c_cg_end, dim3(1), dim3(kCgThreads), 0, st, c->cs, c->rec + (launched & 1),
                           part[launched & 1], nbx, tol2);
        hipLaunchKernelGGL(k_c_apply, gr, blk, 0, st, g, P);
        hipLaunchKernelGGL(k_c_apply_pose, dim3(1), dim3(64), 0, st, c->cs);
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
