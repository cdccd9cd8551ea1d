// HIP kernels of the per-pixel GBP iteration (PixVOD, arXiv 2606.03989) for
// gfx950. One lane per pixel; FP32 structure-of-arrays state planes with a
// padded row pitch, FP64 per-pixel algebra in registers.
//
// Two schedules of the same synchronous iteration (Sec. 4.1):
//   per-factor: linearise + marginals -> messages -> belief update, one kernel
//               each, intermediates through device memory;
//   fused:      each pixel completes the partial messages its neighbours sent
//               (partials do not depend on the receiver's linearisation point),
//               updates and relinearises its variable, then linearises again
//               and sends the next partials. One pass over the state per
//               iteration; a prologue pass per frame starts the rotation and
//               the last pass writes the canonical messages back.
#include "gbp_kernels.h"
#include "gbp_device.hpp"

#include <hip/hip_cooperative_groups.h>

namespace cg = cooperative_groups;

namespace pv {

// belief mean, relinearisation (Eq. var) and first-order transport of the
// stored messages into the new tangent space (Sec. 4.1)
__device__ inline bool update_and_transport(double L[28], double eta[7], double tau[6], double& ell,
                                            float mid[4][27], float mn[4][2], double& var_ll) {
    double idg[7];
    const bool ok = chol7(L, idg);
    double m[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) m[k] = eta[k];
    chol7_solve(L, idg, m);
    var_ll = chol7_var_last(idg);
    double R0[9], t0[3], Rm[9], tm[3], R1[9], t1[3];
    se3_exp(tau, R0, t0);
    se3_exp(m, Rm, tm);
    se3_compose(R0, t0, Rm, tm, R1, t1);
    se3_log(R1, t1, tau);
    ell += m[6];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
#pragma unroll
        for (int a = 0; a < 6; ++a) {
            double s = (double)mid[d][a];
#pragma unroll
            for (int b = 0; b < 6; ++b) s -= (double)mid[d][6 + s6(a, b)] * m[b];
            mid[d][a] = (float)s;
        }
        mn[d][0] = (float)((double)mn[d][0] - (double)mn[d][1] * m[6]);
    }
    return ok;
}

// sender side: partial messages of pixel i towards each neighbour, from its
// belief (L, eta) and its stored messages; written to the neighbour's slot
__device__ inline void emit_partials(const Geo& g, const Strengths& s, const Inputs& in, int u, int v,
                                     const double L[28], const double eta[7], const float mid[4][27],
                                     const float mn[4][2], float* __restrict__ Y, bool& ok,
                                     double* __restrict__ marg_out = nullptr) {
    double P[21], p[6], D, dv;
    pose_marginal(L, eta, P, p);
    ok = depth_marginal(L, eta, D, dv) && ok;
    const long pi = pix_of(g, u, v);
    if (marg_out) {
        // the marginals in the per-factor layout (k_pf_linearise): P 21, p 6,
        // D, dv; then the belief they come from: L 28, eta 7 (the reverse
        // sweep's tape, written non-temporally)
#pragma unroll
        for (int k = 0; k < 21; ++k) __builtin_nontemporal_store(P[k], &marg_out[(long)k * g.plane + pi]);
#pragma unroll
        for (int k = 0; k < 6; ++k) __builtin_nontemporal_store(p[k], &marg_out[(long)(21 + k) * g.plane + pi]);
        __builtin_nontemporal_store(D, &marg_out[27L * g.plane + pi]);
        __builtin_nontemporal_store(dv, &marg_out[28L * g.plane + pi]);
#pragma unroll
        for (int k = 0; k < 28; ++k) __builtin_nontemporal_store(L[k], &marg_out[(long)(29 + k) * g.plane + pi]);
#pragma unroll
        for (int k = 0; k < 7; ++k) __builtin_nontemporal_store(eta[k], &marg_out[(long)(57 + k) * g.plane + pi]);
    }
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        int nu, nv;
        if (!neighbour(g, u, v, d, nu, nv)) continue;
        const long pj = pix_of(g, nu, nv);
        const int slot = opposite(d);
        double V[21], vv[6], Lp[21], h[6];
#pragma unroll
        for (int k = 0; k < 21; ++k) V[k] = P[k] - (double)mid[d][6 + k];
#pragma unroll
        for (int k = 0; k < 6; ++k) vv[k] = p[k] - (double)mid[d][k];
        ok = identity_partial(s.lamR, V, vv, Lp, h) && ok;
        float* dst = Y + (long)(P_MID + slot * MID_STRIDE) * g.plane + pj;
#pragma unroll
        for (int k = 0; k < 6; ++k) dst[k * g.plane] = (float)h[k];
#pragma unroll
        for (int k = 0; k < 21; ++k) dst[(6 + k) * g.plane] = (float)Lp[k];
        float* dn = Y + (long)(P_MN + 2 * slot) * g.plane + pj;
        if (normal_active(g, in, pi, pj, d) && s.lamN > 0.0) {
            double lp, hn;
            normal_partial(s.lamN, D - (double)mn[d][1], dv - (double)mn[d][0], lp, hn);
            dn[0] = (float)hn;
            dn[g.plane] = (float)lp;
        } else {
            dn[0] = 0.0f;
            dn[g.plane] = 0.0f;
        }
    }
}

// adds one completed message (identity eta/Lambda, normal eta/lambda) of slot
// d to the belief in FP64 and keeps its FP32 storage copy
__device__ inline void accumulate_message(double L[28], double eta[7], const double id_eta[6], const float id_lam[21],
                                          double n_eta, float n_lam, float mid_d[27], float mn_d[2]) {
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        eta[a] += id_eta[a];
        mid_d[a] = (float)id_eta[a];
    }
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = r; c < 6; ++c) L[s7(r, c)] += (double)id_lam[s6(r, c)];
#pragma unroll
    for (int k = 0; k < 21; ++k) mid_d[6 + k] = id_lam[k];
    eta[6] += n_eta;
    L[s7(6, 6)] += (double)n_lam;
    mn_d[0] = (float)n_eta;
    mn_d[1] = n_lam;
}

// receiver side: completes the partial in slot d with the residual at both
// linearisation points, eta = h - Lambda' r, and adds it to the belief.
// Lam_out (reverse-sweep tape) receives each new message's information (the
// identity Lambda and the normal lambda, 22 FP32 planes per slot: they are
// the partials' FP32 values, so the FP32 tape is exact)
__device__ inline void complete_partials(const Geo& g, const Strengths& s, const Inputs& in,
                                         const float* __restrict__ X, int u, int v, const double R[9],
                                         const double t[3], double ell, double L[28], double eta[7],
                                         float mid[4][27], float mn[4][2], float* __restrict__ Lam_out = nullptr) {
    const long pi = pix_of(g, u, v);
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        int nu, nv;
        if (!neighbour(g, u, v, d, nu, nv)) {
#pragma unroll
            for (int k = 0; k < 27; ++k) mid[d][k] = 0.0f;
            mn[d][0] = mn[d][1] = 0.0f;
            if (Lam_out)
#pragma unroll
                for (int k = 0; k < LAM_STRIDE; ++k) __builtin_nontemporal_store(0.0f, &Lam_out[(long)(d * LAM_STRIDE + k) * g.plane + pi]);
            continue;
        }
        const long pj = pix_of(g, nu, nv);
        double tj[6], ellj, Rj[9], trj[3], r[6];
        load_point(X, g, pj, tj, ellj);
        se3_exp(tj, Rj, trj);
        se3_between(Rj, trj, R, t, r);
        const float* src = X + (long)(P_MID + d * MID_STRIDE) * g.plane + pi;
        float part[27];
#pragma unroll
        for (int k = 0; k < 27; ++k) part[k] = src[k * g.plane];
        double e6[6];
#pragma unroll
        for (int a = 0; a < 6; ++a) {
            double e = (double)part[a];
#pragma unroll
            for (int b = 0; b < 6; ++b) e -= (double)part[6 + s6(a, b)] * r[b];
            e6[a] = e;
        }
        double ne = 0.0;
        float nl = 0.0f;
        double rn;
        if (s.lamN > 0.0 && normal_residual(g, in, pi, pj, d, ell, ellj, rn)) {
            const float* sn = X + (long)(P_MN + 2 * d) * g.plane + pi;
            nl = sn[g.plane];
            ne = (double)sn[0] - (double)nl * rn;
        }
        accumulate_message(L, eta, e6, part + 6, ne, nl, mid[d], mn[d]);
        if (Lam_out) {
            // the reverse sweep's tape of the new messages' information, written
            // non-temporally like the FP64 tape
            float* o = Lam_out + (long)(d * LAM_STRIDE) * g.plane + pi;
#pragma unroll
            for (int k = 0; k < 21; ++k) __builtin_nontemporal_store(part[6 + k], &o[k * g.plane]);
            __builtin_nontemporal_store(nl, &o[21 * g.plane]);
        }
    }
}

// one float of state; NT: a non-temporal store (streamed past the caches),
// for passes whose output is not read again while it could stay cached: the
// batch's passes over many sequences and a frame's final pass
template <bool NT = false>
__device__ inline void put(float* __restrict__ a, float v) {
    if constexpr (NT) __builtin_nontemporal_store(v, a);
    else *a = v;
}

template <bool NT = false>
__device__ inline void store_point(float* __restrict__ Y, const Geo& g, long p, const double tau[6], double ell) {
    if constexpr (NT) {
#pragma unroll
        for (int k = 0; k < 6; ++k) put<true>(&Y[(P_TAU + k) * g.plane + p], (float)tau[k]);
        put<true>(&Y[P_ELL * g.plane + p], (float)ell);
    } else {
#pragma unroll
        for (int k = 0; k < 6; ++k) Y[(P_TAU + k) * g.plane + p] = (float)tau[k];
        Y[P_ELL * g.plane + p] = (float)ell;
    }
}

template <bool NT = false>
__device__ inline void store_messages(float* __restrict__ Y, const Geo& g, long p, const float mid[4][27],
                                      const float mn[4][2]) {
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        if constexpr (NT) {
#pragma unroll
            for (int k = 0; k < 27; ++k) put<true>(&Y[(long)(P_MID + d * MID_STRIDE + k) * g.plane + p], mid[d][k]);
            put<true>(&Y[(long)(P_MN + 2 * d) * g.plane + p], mn[d][0]);
            put<true>(&Y[(long)(P_MN + 2 * d + 1) * g.plane + p], mn[d][1]);
        } else {
#pragma unroll
            for (int k = 0; k < 27; ++k) Y[(long)(P_MID + d * MID_STRIDE + k) * g.plane + p] = mid[d][k];
            Y[(long)(P_MN + 2 * d) * g.plane + p] = mn[d][0];
            Y[(long)(P_MN + 2 * d + 1) * g.plane + p] = mn[d][1];
        }
    }
}

// rounds a double point to the stored FP32 precision
__device__ inline void round_point(double tau[6], double& ell) {
#pragma unroll
    for (int k = 0; k < 6; ++k) tau[k] = (double)(float)tau[k];
    ell = (double)(float)ell;
}

// ---------------------------------------------------------------------------
// frame and keyframe preparation

// central differences inside, one-sided at the border
__device__ __attribute__((always_inline)) inline void frame_prep_pixel(const Geo& g, const float* __restrict__ src, long src_pitch,
                                        float* __restrict__ It, float* __restrict__ Gx, float* __restrict__ Gy,
                                        int u, int v) {
    const float* row = src + (long)v * src_pitch;
    const float c = row[u];
    float gx, gy;
    if (u == 0) gx = row[1] - row[0];
    else if (u == g.W - 1) gx = row[u] - row[u - 1];
    else gx = 0.5f * (row[u + 1] - row[u - 1]);
    if (v == 0) gy = src[src_pitch + u] - row[u];
    else if (v == g.H - 1) gy = row[u] - src[(long)(v - 1) * src_pitch + u];
    else gy = 0.5f * (src[(long)(v + 1) * src_pitch + u] - src[(long)(v - 1) * src_pitch + u]);
    const long p = pix_of(g, u, v);
    It[p] = c;
    Gx[p] = gx;
    Gy[p] = gy;
}

__global__ void k_frame_prep(Geo g, const float* __restrict__ src, long src_pitch, float* __restrict__ It,
                             float* __restrict__ Gx, float* __restrict__ Gy, int* __restrict__ clear) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    if (clear && u == 0 && v == 0) *clear = 0;
    if (u >= g.W || v >= g.H) return;
    frame_prep_pixel(g, src, src_pitch, It, Gx, Gy, u, v);
}

// keyframe image, normal-integration targets and the state reset:
// pose linearisation points to identity, messages to zero, log-depth kept
__device__ __attribute__((always_inline)) inline void keyframe_prep_pixel(
    const Geo& g, const float* __restrict__ img, const float* __restrict__ normals, float* __restrict__ Is,
    float* __restrict__ cxt, float* __restrict__ cyt, float* __restrict__ X, float* __restrict__ X2, int u, int v) {
    const long dense = (long)v * g.W + u;
    const long p = pix_of(g, u, v);
    Is[p] = img[dense];
    const double q0 = ((double)u - g.cx) / g.fx, q1 = ((double)v - g.cy) / g.fy;
    const double n0 = normals[3 * dense], n1 = normals[3 * dense + 1], n2 = normals[3 * dense + 2];
    const double nq = n0 * q0 + n1 * q1 + n2;
    const double qn = sqrt(q0 * q0 + q1 * q1 + 1.0);
    const bool ok = isfinite(nq) && fabs(nq) >= 1e-3 * qn;
    cxt[p] = ok ? (float)(n0 / (g.fx * nq)) : __int_as_float(0x7fc00000);
    cyt[p] = ok ? (float)(n1 / (g.fy * nq)) : __int_as_float(0x7fc00000);
    const float ell = X[P_ELL * g.plane + p];
    for (int k = 0; k < N_PLANES; ++k) {
        X[(long)k * g.plane + p] = 0.0f;
        X2[(long)k * g.plane + p] = 0.0f;
    }
    X[P_ELL * g.plane + p] = ell;
    X2[P_ELL * g.plane + p] = ell;
}

__global__ void k_keyframe_prep(Geo g, const float* __restrict__ img, const float* __restrict__ normals,
                                float* __restrict__ Is, float* __restrict__ cxt, float* __restrict__ cyt,
                                float* __restrict__ X, float* __restrict__ X2) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    if (u >= g.W || v >= g.H) return;
    keyframe_prep_pixel(g, img, normals, Is, cxt, cyt, X, X2, u, v);
}

__global__ void k_init_state(Geo g, float* __restrict__ X, float ell0) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    if (u >= g.W || v >= g.H) return;
    const long p = pix_of(g, u, v);
    for (int k = 0; k < N_PLANES; ++k) X[(long)k * g.plane + p] = 0.0f;
    X[P_ELL * g.plane + p] = ell0;
}

// ---------------------------------------------------------------------------
// per-factor schedule

// L + B + V: unary factors, belief, pose and depth marginals (FP64 scratch,
// 29 planes: P packed 21, p 6, D, dv)
__global__ __launch_bounds__(256) void k_pf_linearise(Geo g, Strengths s, Inputs in, const float* __restrict__ X,
                                                      double* __restrict__ marg, float* __restrict__ valid,
                                                      int* __restrict__ health) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    if (u >= g.W || v >= g.H) return;
    const long p = pix_of(g, u, v);
    double tau[6], ell, R[9], t[3], L[28], eta[7];
    load_point(X, g, p, tau, ell);
    se3_exp(tau, R, t);
    const bool val = unary_factors(g, s, in, u, v, tau, R, t, ell, L, eta);
    float mid[4][27], mn[4][2];
    load_messages(X, g, p, mid, mn);
    add_messages(L, eta, mid, mn);
    double P[21], pv_[6], D, dv;
    pose_marginal(L, eta, P, pv_);
    const bool ok = depth_marginal(L, eta, D, dv);
#pragma unroll
    for (int k = 0; k < 21; ++k) marg[(long)k * g.plane + p] = P[k];
#pragma unroll
    for (int k = 0; k < 6; ++k) marg[(long)(21 + k) * g.plane + p] = pv_[k];
    marg[(long)27 * g.plane + p] = D;
    marg[(long)28 * g.plane + p] = dv;
    valid[p] = val ? 1.0f : 0.0f;
    if (!ok) atomicOr(health, 1);
}

// F: every pixel computes its four incoming messages from its neighbours'
// marginals and the messages those neighbours hold from the shared factor.
// Output (FP64 scratch, 29 planes per direction): identity eta(6), identity
// Lambda(21, already at storage precision), normal eta, normal lambda.
__global__ __launch_bounds__(256, 2) void k_pf_messages(Geo g, Strengths s, Inputs in, const float* __restrict__ X,
                                                     const double* __restrict__ marg, double* __restrict__ M,
                                                     float beta, int* __restrict__ health) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    if (u >= g.W || v >= g.H) return;
    const long pi = pix_of(g, u, v);
    double tau[6], ell, R[9], t[3];
    load_point(X, g, pi, tau, ell);
    se3_exp(tau, R, t);
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        double out[29];
#pragma unroll
        for (int k = 0; k < 29; ++k) out[k] = 0.0;
        int nu, nv;
        if (neighbour(g, u, v, d, nu, nv)) {
            const long pj = pix_of(g, nu, nv);
            const int slot = opposite(d);
            double V[21], vv[6], Lp[21], h[6];
#pragma unroll
            for (int k = 0; k < 21; ++k)
                V[k] = marg[(long)k * g.plane + pj] - (double)X[(long)(P_MID + slot * MID_STRIDE + 6 + k) * g.plane + pj];
#pragma unroll
            for (int k = 0; k < 6; ++k)
                vv[k] = marg[(long)(21 + k) * g.plane + pj] - (double)X[(long)(P_MID + slot * MID_STRIDE + k) * g.plane + pj];
            ok = identity_partial(s.lamR, V, vv, Lp, h) && ok;
            // the partial is rounded to storage precision as in the fused schedule
            float part[27];
#pragma unroll
            for (int k = 0; k < 6; ++k) part[k] = (float)h[k];
#pragma unroll
            for (int k = 0; k < 21; ++k) part[6 + k] = (float)Lp[k];
            double tj[6], ellj, Rj[9], trj[3], r[6];
            load_point(X, g, pj, tj, ellj);
            se3_exp(tj, Rj, trj);
            se3_between(Rj, trj, R, t, r);
#pragma unroll
            for (int a = 0; a < 6; ++a) {
                double e = (double)part[a];
#pragma unroll
                for (int b = 0; b < 6; ++b) e -= (double)part[6 + s6(a, b)] * r[b];
                out[a] = e;
            }
#pragma unroll
            for (int k = 0; k < 21; ++k) out[6 + k] = (double)part[6 + k];
            double rn;
            if (s.lamN > 0.0 && normal_residual(g, in, pi, pj, d, ell, ellj, rn)) {
                const double ls = marg[(long)27 * g.plane + pj] - (double)X[(long)(P_MN + 2 * slot + 1) * g.plane + pj];
                const double vs = marg[(long)28 * g.plane + pj] - (double)X[(long)(P_MN + 2 * slot) * g.plane + pj];
                double lp, hn;
                normal_partial(s.lamN, ls, vs, lp, hn);
                const float fl = (float)lp, fh = (float)hn;
                out[27] = (double)fh - (double)fl * rn;
                out[28] = (double)fl;
            }
            if (beta != 0.0f) {
                // damping towards the stored message; the blended Lambda is
                // rounded to storage precision like every stored Lambda
                const double b = beta, a = 1.0 - b;
#pragma unroll
                for (int k = 0; k < 6; ++k)
                    out[k] = a * out[k] + b * X[(long)(P_MID + d * MID_STRIDE + k) * g.plane + pi];
#pragma unroll
                for (int k = 6; k < 27; ++k)
                    out[k] = (double)(float)(a * out[k] + b * X[(long)(P_MID + d * MID_STRIDE + k) * g.plane + pi]);
                out[27] = a * out[27] + b * X[(long)(P_MN + 2 * d) * g.plane + pi];
                out[28] = (double)(float)(a * out[28] + b * X[(long)(P_MN + 2 * d + 1) * g.plane + pi]);
            }
        }
#pragma unroll
        for (int k = 0; k < 29; ++k) M[(long)(d * 29 + k) * g.plane + pi] = out[k];
    }
    if (!ok) atomicOr(health, 1);
}

// U: new belief from the recomputed unary and the new messages, relinearise,
// transport, write the state in place
__global__ __launch_bounds__(256) void k_pf_update(Geo g, Strengths s, Inputs in, float* __restrict__ X,
                                                   const double* __restrict__ M, float* __restrict__ var_ll,
                                                   float* __restrict__ valid, int* __restrict__ health) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    if (u >= g.W || v >= g.H) return;
    const long p = pix_of(g, u, v);
    double tau[6], ell, R[9], t[3], L[28], eta[7];
    load_point(X, g, p, tau, ell);
    se3_exp(tau, R, t);
    const bool val = unary_factors(g, s, in, u, v, tau, R, t, ell, L, eta);
    float mid[4][27], mn[4][2];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        double e6[6];
        float lam[21];
#pragma unroll
        for (int k = 0; k < 6; ++k) e6[k] = M[(long)(d * 29 + k) * g.plane + p];
#pragma unroll
        for (int k = 0; k < 21; ++k) lam[k] = (float)M[(long)(d * 29 + 6 + k) * g.plane + p];
        const double ne = M[(long)(d * 29 + 27) * g.plane + p];
        const float nl = (float)M[(long)(d * 29 + 28) * g.plane + p];
        accumulate_message(L, eta, e6, lam, ne, nl, mid[d], mn[d]);
    }
    double var;
    const bool ok = update_and_transport(L, eta, tau, ell, mid, mn, var);
    round_point(tau, ell);
    store_point(X, g, p, tau, ell);
    store_messages(X, g, p, mid, mn);
    var_ll[p] = (float)var;
    valid[p] = val ? 1.0f : 0.0f;
    if (!ok) atomicOr(health, 1);
}

// ---------------------------------------------------------------------------
// fused schedule

// prologue of one pixel: belief of the canonical state and the first partials
__device__ __attribute__((always_inline)) inline void prologue_pixel(const Geo& g, const Strengths& s, const Inputs& in, const float* __restrict__ X,
                                      float* __restrict__ Y, int* __restrict__ health, int u, int v,
                                      double* __restrict__ marg_out = nullptr) {
    const long p = pix_of(g, u, v);
    double tau[6], ell, R[9], t[3], L[28], eta[7];
    load_point(X, g, p, tau, ell);
    se3_exp(tau, R, t);
    const PixelInputs pin = load_pixel_inputs(g, s, in, u, v);
    unary_factors(g, s, in, u, v, tau, R, t, ell, pin, L, eta);
    float mid[4][27], mn[4][2];
    load_messages(X, g, p, mid, mn);
    add_messages(L, eta, mid, mn);
    bool ok = true;
    emit_partials(g, s, in, u, v, L, eta, mid, mn, Y, ok, marg_out);
    store_point(Y, g, p, tau, ell);
    if (!ok) atomicOr(health, 1);
}

// one iteration of one pixel: complete, update, relinearise, then (not
// FINAL) emit the next partials or (FINAL) write the canonical state and the
// per-pixel outputs. Not FINAL, Yc (when given) also receives the canonical
// state after the update, and marg_next the marginals of the next emission.
template <bool FINAL>
__device__ __attribute__((always_inline)) inline void iterate_pixel(const Geo& g, const Strengths& s, const Inputs& in, const float* __restrict__ X,
                                     float* __restrict__ Y, float* __restrict__ var_ll, float* __restrict__ valid,
                                     int* __restrict__ health, int u, int v, float* __restrict__ Lam_out = nullptr,
                                     double* __restrict__ bel_out = nullptr, float* __restrict__ Yc = nullptr,
                                     double* __restrict__ marg_next = nullptr) {
    const long p = pix_of(g, u, v);
    double tau[6], ell, R[9], t[3], L[28], eta[7];
    load_point(X, g, p, tau, ell);
    se3_exp(tau, R, t);
    const bool val = unary_factors(g, s, in, u, v, tau, R, t, ell, L, eta);
    float mid[4][27], mn[4][2];
    complete_partials(g, s, in, X, u, v, R, t, ell, L, eta, mid, mn, Lam_out);
    if (bel_out) {
        // the belief of the update (unary + new messages): L 28, eta 7; the
        // FP64 tape is written non-temporally (read back only by the reverse
        // sweep, after the segment's recompute)
#pragma unroll
        for (int k = 0; k < 28; ++k) __builtin_nontemporal_store(L[k], &bel_out[(long)k * g.plane + p]);
#pragma unroll
        for (int k = 0; k < 7; ++k) __builtin_nontemporal_store(eta[k], &bel_out[(long)(28 + k) * g.plane + p]);
    }
    double var;
    bool ok = update_and_transport(L, eta, tau, ell, mid, mn, var);
    round_point(tau, ell);
    store_point(Y, g, p, tau, ell);
    if (FINAL) {
        store_messages(Y, g, p, mid, mn);
        var_ll[p] = (float)var;
        valid[p] = val ? 1.0f : 0.0f;
    } else {
        if (Yc) {
            store_point(Yc, g, p, tau, ell);
            store_messages(Yc, g, p, mid, mn);
        }
        se3_exp(tau, R, t);
        unary_factors(g, s, in, u, v, tau, R, t, ell, L, eta);
        add_messages(L, eta, mid, mn);
        emit_partials(g, s, in, u, v, L, eta, mid, mn, Y, ok, marg_next);
    }
    if (!ok) atomicOr(health, 1);
}

// ---------------------------------------------------------------------------
// fused pass with its loads issued together
//
// With one wave per SIMD (the pass keeps ~450 registers live) nothing hides
// memory latency, so the number of dependent round trips to memory sets the
// pass time. Every load whose address does not depend on computed values
// (own point, the four neighbours' points, the four partials and normal
// partials in flight, the normal targets, the keyframe intensity and the
// optional sigma and prior maps) is issued at once at the start; a missing
// neighbour's loads read the pixel itself and are discarded. What remains
// dependent are the bilinear samples at the two warps. The arithmetic and its
// order are those of iterate_pixel.

// preloaded normal targets of the four edges: c of the left/upper pixel a
struct EdgeTargets {
    float c[4];
};

// normal_residual with a preloaded target
__device__ inline bool normal_residual_c(float c, int d, double ell_i, double ell_j, double& r_recv) {
    if (!isfinite(c)) return false;
    const bool recv_is_b = (d == DIR_L || d == DIR_U);
    r_recv = recv_is_b ? (ell_i - ell_j + (double)c) : (ell_i - ell_j - (double)c);
    return true;
}

// Linearisation points of the neighbours: either loaded from the state and
// exponentiated by every pixel that needs them (SH = false), or, in the
// 64 x 4 workgroups of the single-sequence pass (SH = true), exponentiated
// once per point into a shared table of the workgroup's points and its
// one-pixel halo (HALO_W x HALO_H points, FP64 R, t and ell per point,
// structure of arrays): each point's Exp is then computed by one lane instead
// of five, and the neighbours' points are not loaded per pixel.
constexpr int HALO_W = 66, HALO_H = 6, HALO_N = HALO_W * HALO_H;
constexpr int SH_FIELDS = 13;   // R 9, t 3, ell

__device__ inline void sh_put(double* __restrict__ sh, int h, const double R[9], const double t[3], double ell) {
#pragma unroll
    for (int k = 0; k < 9; ++k) sh[k * HALO_N + h] = R[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) sh[(9 + k) * HALO_N + h] = t[k];
    sh[12 * HALO_N + h] = ell;
}

// the halo ring of a 64 x 4 tile at (u0, v0), lane l < 140: its point, or
// false outside the image
__device__ inline bool halo_point(const Geo& g, int u0, int v0, int l, int& u, int& v, int& h) {
    int hx, hy;
    if (l < HALO_W) { hx = l - 1; hy = -1; }
    else if (l < 2 * HALO_W) { hx = l - HALO_W - 1; hy = 4; }
    else if (l < 2 * HALO_W + 4) { hx = -1; hy = l - 2 * HALO_W; }
    else { hx = 64; hy = l - 2 * HALO_W - 4; }
    u = u0 + hx;
    v = v0 + hy;
    h = (hy + 1) * HALO_W + (hx + 1);
    return u >= 0 && u < g.W && v >= 0 && v < g.H;
}

// The stored messages of a pixel (eta 6 and Lambda 21 of the four identity
// slots, eta and lambda of the four normal slots) are the 116 consecutive
// planes from P_MID. The persistent single-sequence pass keeps them for the
// next 64 x 4 tile in LDS, loaded straight from memory into LDS (no
// registers) while the current tile computes: wave w loads tile row w, plane
// k of lane l at buf[k * 256 + w * 64 + l]. Lanes outside the image load any
// valid pixel; their values are not used.
constexpr int MSG_PLANES = 116;
static_assert(P_MN + 8 == P_MID + MSG_PLANES, "messages are contiguous planes");

__device__ inline void prefetch_messages(const Geo& g, const float* __restrict__ X, float* buf, int u0, int v0,
                                         int w, int lane) {
    const int u = u0 + lane, v = v0 + w;
    const long p = (u < g.W && v < g.H) ? pix_of(g, u, v) : 0;
    const float* src = X + (long)P_MID * g.plane + p;
    float* dst = buf + w * 64;
#pragma unroll 4
    for (int k = 0; k < MSG_PLANES; ++k)
        __builtin_amdgcn_global_load_lds((const void*)(src + (long)k * g.plane),
                                         (__attribute__((address_space(3))) void*)(dst + k * 256), 4, 0, 0);
}

// wait for this wave's loads into LDS: the compiler does not track them, so
// the wait is explicit, and the memory clobber keeps the LDS reads after it
__device__ inline void wait_lds_loads() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

template <bool FINAL, bool SH, bool PIPE = false, bool NT = false>
__device__ __attribute__((always_inline)) inline void iterate_pixel_pf(
    const Geo& g, const Strengths& s, const Inputs& in, const float* __restrict__ X, float* __restrict__ Y,
    float* __restrict__ var_ll, float* __restrict__ valid, int* __restrict__ health, int u, int v,
    bool inside = true, double* __restrict__ sh = nullptr, int u0 = 0, int v0 = 0, int tid = 0,
    float* mbuf = nullptr, bool pre = false, int nu0 = 0, int nv0 = 0) {
    const long p = inside ? pix_of(g, u, v) : 0;
    bool has[4];
    long pn[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        int nu, nv;
        has[d] = inside && neighbour(g, u, v, d, nu, nv);
        pn[d] = has[d] ? pix_of(g, nu, nv) : p;
    }
    // --- loads with computable addresses, all issued before any use
    float pt[7], npt[4][7], mid[4][27], mn[4][2];
    EdgeTargets ct;
    PixelInputs pin;
    double tau[6], ell, R[9], t[3];
    if (inside) {
#pragma unroll
        for (int k = 0; k < 7; ++k) pt[k] = X[(long)(P_TAU + k) * g.plane + p];
        if constexpr (!SH) {
#pragma unroll
            for (int d = 0; d < 4; ++d)
#pragma unroll
                for (int k = 0; k < 7; ++k) npt[d][k] = X[(long)(P_TAU + k) * g.plane + pn[d]];
        }
        if constexpr (!PIPE) {
#pragma unroll
            for (int d = 0; d < 4; ++d) {
#pragma unroll
                for (int k = 0; k < 27; ++k) mid[d][k] = X[(long)(P_MID + d * MID_STRIDE + k) * g.plane + p];
                mn[d][0] = X[(long)(P_MN + 2 * d) * g.plane + p];
                mn[d][1] = X[(long)(P_MN + 2 * d + 1) * g.plane + p];
            }
        }
        ct.c[DIR_L] = in.cxt[pn[DIR_L]];
        ct.c[DIR_R] = in.cxt[p];
        ct.c[DIR_U] = in.cyt[pn[DIR_U]];
        ct.c[DIR_D] = in.cyt[p];
        pin = load_pixel_inputs(g, s, in, u, v);
        if constexpr (PIPE) {
            // this tile's messages, prefetched into LDS during the previous tile
            wait_lds_loads();
#pragma unroll
            for (int d = 0; d < 4; ++d) {
#pragma unroll
                for (int k = 0; k < 27; ++k) mid[d][k] = mbuf[(d * MID_STRIDE + k) * 256 + tid];
                mn[d][0] = mbuf[(P_MN - P_MID + 2 * d) * 256 + tid];
                mn[d][1] = mbuf[(P_MN - P_MID + 2 * d + 1) * 256 + tid];
            }
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) tau[k] = (double)pt[k];
        ell = (double)pt[6];
        se3_exp(tau, R, t);
    }
    if constexpr (SH) {
        // the tile's points and its halo into the shared table
        if (inside) sh_put(sh, (v - v0 + 1) * HALO_W + (u - u0 + 1), R, t, ell);
        int hu, hv, hh;
        if (tid < 2 * HALO_W + 8 && halo_point(g, u0, v0, tid, hu, hv, hh)) {
            const long hp = pix_of(g, hu, hv);
            double ht[6], hR[9], htr[3];
#pragma unroll
            for (int k = 0; k < 6; ++k) ht[k] = (double)X[(long)(P_TAU + k) * g.plane + hp];
            const double hell = (double)X[(long)P_ELL * g.plane + hp];
            se3_exp(ht, hR, htr);
            sh_put(sh, hh, hR, htr, hell);
        }
        __syncthreads();
    }
    if (!inside) {
        if constexpr (PIPE) {
            wait_lds_loads();   // this lane's slots of the buffer are read (nothing) before they are refilled
            if (pre) prefetch_messages(g, X, mbuf, nu0, nv0, tid >> 6, tid & 63);
        }
        return;
    }

    // --- linearise at the current point
    double L[28], eta[7];
    const bool val = unary_factors(g, s, in, u, v, tau, R, t, ell, pin, L, eta);
    if constexpr (PIPE && FINAL) {
        if (pre) prefetch_messages(g, X, mbuf, nu0, nv0, tid >> 6, tid & 63);
    }

    // --- complete the partials in flight (complete_partials)
    const int hown = SH ? (v - v0 + 1) * HALO_W + (u - u0 + 1) : 0;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        if (!has[d]) {
#pragma unroll
            for (int k = 0; k < 27; ++k) mid[d][k] = 0.0f;
            mn[d][0] = mn[d][1] = 0.0f;
            continue;
        }
        double Rj[9], trj[3], ellj, r[6];
        if constexpr (SH) {
            const int hj = hown + (d == DIR_L ? -1 : d == DIR_R ? 1 : d == DIR_U ? -HALO_W : HALO_W);
#pragma unroll
            for (int k = 0; k < 9; ++k) Rj[k] = sh[k * HALO_N + hj];
#pragma unroll
            for (int k = 0; k < 3; ++k) trj[k] = sh[(9 + k) * HALO_N + hj];
            ellj = sh[12 * HALO_N + hj];
        } else {
            double tj[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) tj[k] = (double)npt[d][k];
            ellj = (double)npt[d][6];
            se3_exp(tj, Rj, trj);
        }
        se3_between(Rj, trj, R, t, r);
        double e6[6];
#pragma unroll
        for (int a = 0; a < 6; ++a) {
            double e = (double)mid[d][a];
#pragma unroll
            for (int b = 0; b < 6; ++b) e -= (double)mid[d][6 + s6(a, b)] * r[b];
            e6[a] = e;
        }
        double ne = 0.0;
        float nl = 0.0f;
        double rn;
        if (s.lamN > 0.0 && normal_residual_c(ct.c[d], d, ell, ellj, rn)) {
            nl = mn[d][1];
            ne = (double)mn[d][0] - (double)nl * rn;
        }
        float lam[21];
#pragma unroll
        for (int k = 0; k < 21; ++k) lam[k] = mid[d][6 + k];
        accumulate_message(L, eta, e6, lam, ne, nl, mid[d], mn[d]);
    }

    // --- update, relinearise, transport
    double var;
    bool ok = update_and_transport(L, eta, tau, ell, mid, mn, var);
    round_point(tau, ell);
    store_point<NT>(Y, g, p, tau, ell);
    if (FINAL) {
        store_messages<NT>(Y, g, p, mid, mn);
        var_ll[p] = (float)var;
        valid[p] = val ? 1.0f : 0.0f;
    } else {
        // --- linearise at the new point and send the next partials (emit_partials)
        se3_exp(tau, R, t);
        unary_factors(g, s, in, u, v, tau, R, t, ell, pin, L, eta);
        if constexpr (PIPE) {
            // the next tile's messages stream into LDS during the rest of this one
            if (pre) prefetch_messages(g, X, mbuf, nu0, nv0, tid >> 6, tid & 63);
        }
        add_messages(L, eta, mid, mn);
        double P[21], pm[6], D, dv;
        pose_marginal(L, eta, P, pm);
        ok = depth_marginal(L, eta, D, dv) && ok;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            if (!has[d]) continue;
            const long pj = pn[d];
            const int slot = opposite(d);
            double V[21], vv[6], Lp[21], h[6];
#pragma unroll
            for (int k = 0; k < 21; ++k) V[k] = P[k] - (double)mid[d][6 + k];
#pragma unroll
            for (int k = 0; k < 6; ++k) vv[k] = pm[k] - (double)mid[d][k];
            ok = identity_partial(s.lamR, V, vv, Lp, h) && ok;
            float* dst = Y + (long)(P_MID + slot * MID_STRIDE) * g.plane + pj;
            if constexpr (NT) {
#pragma unroll
                for (int k = 0; k < 6; ++k) put<true>(&dst[k * g.plane], (float)h[k]);
#pragma unroll
                for (int k = 0; k < 21; ++k) put<true>(&dst[(6 + k) * g.plane], (float)Lp[k]);
            } else {
#pragma unroll
                for (int k = 0; k < 6; ++k) dst[k * g.plane] = (float)h[k];
#pragma unroll
                for (int k = 0; k < 21; ++k) dst[(6 + k) * g.plane] = (float)Lp[k];
            }
            float* dn = Y + (long)(P_MN + 2 * slot) * g.plane + pj;
            if (isfinite(ct.c[d]) && s.lamN > 0.0) {
                double lp, hn;
                normal_partial(s.lamN, D - (double)mn[d][1], dv - (double)mn[d][0], lp, hn);
                if constexpr (NT) {
                    put<true>(&dn[0], (float)hn);
                    put<true>(&dn[g.plane], (float)lp);
                } else {
                    dn[0] = (float)hn;
                    dn[g.plane] = (float)lp;
                }
            } else if constexpr (NT) {
                put<true>(&dn[0], 0.0f);
                put<true>(&dn[g.plane], 0.0f);
            } else {
                dn[0] = 0.0f;
                dn[g.plane] = 0.0f;
            }
        }
    }
    if (!ok) atomicOr(health, 1);
}

__global__ __launch_bounds__(256) void k_fu_prologue(Geo g, Strengths s, Inputs in, const float* __restrict__ X,
                                                     float* __restrict__ Y, int* __restrict__ health) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    if (u >= g.W || v >= g.H) return;
    prologue_pixel(g, s, in, X, Y, health, u, v);
}

// Persistent: each workgroup (one per CU: the LDS of the shared table and the
// message buffer fill a CU) takes the 64 x 4 tiles blockIdx, blockIdx +
// gridDim, ... in turn, loading the next tile's messages into LDS while it
// computes the current one. Every lane reaches the barriers of every tile;
// lanes outside the image only help fill the shared table.
template <bool FINAL>
__global__ __launch_bounds__(256) void k_fu_iterate(Geo g, Strengths s, Inputs in, const float* __restrict__ X,
                                                    float* __restrict__ Y, float* __restrict__ var_ll,
                                                    float* __restrict__ valid, int* __restrict__ health,
                                                    int tiles_x, int ntiles) {
    __shared__ double sh[SH_FIELDS * HALO_N];
    __shared__ float mbuf[MSG_PLANES * 256];
    const int tid = threadIdx.y * 64 + threadIdx.x;
    int tile = blockIdx.x;
    if (tile >= ntiles) return;
    prefetch_messages(g, X, mbuf, (tile % tiles_x) * 64, (tile / tiles_x) * 4, threadIdx.y, threadIdx.x);
    for (; tile < ntiles; tile += gridDim.x) {
        const int next = tile + gridDim.x;
        const int u0 = (tile % tiles_x) * 64, v0 = (tile / tiles_x) * 4;
        const int u = u0 + threadIdx.x, v = v0 + threadIdx.y;
        // everything the pass derives from the arguments and the lane index is
        // made opaque per tile, so the compiler recomputes it inside the tile
        // instead of hoisting it out of the loop (hundreds of plane and LDS
        // addresses, which would not fit in registers)
        int z = 0;
        asm volatile("" : "+s"(z));
        Geo gt = g;
        gt.H += z;
        gt.W += z;
        gt.pitch += z;
        gt.plane += z;
        Inputs it = in;
        it.Is += z;
        it.cxt += z;
        it.cyt += z;
        it.sigD += z;
        it.It += z;
        it.Gx += z;
        it.Gy += z;
        it.prior_ell += z;
        const int tz = tid + z;
        __syncthreads();   // the previous tile's readers of the shared table are done
        iterate_pixel_pf<FINAL, true, true, FINAL>(gt, s, it, X + z, Y + z, var_ll + z, valid + z, health, u + z, v + z,
                                            u < g.W && v < g.H, sh, u0, v0, tz, mbuf, next < ntiles,
                                            (next % tiles_x) * 64, (next / tiles_x) * 4);
    }
}

// the same passes for the reverse sweep's recompute: the prologue also writes
// the belief of its state and its marginals, the final pass the new messages
// computed from its source state and the belief they form with the unary
// factors (exactly the values of k_pf_linearise, k_pf_messages, k_pf_update)
__global__ __launch_bounds__(256) void k_fu_prologue_tape(Geo g, Strengths s, Inputs in, const float* __restrict__ X,
                                                          float* __restrict__ Y, double* __restrict__ marg,
                                                          int* __restrict__ health) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    if (u >= g.W || v >= g.H) return;
    prologue_pixel(g, s, in, X, Y, health, u, v, marg);
}

// the rotated form of the recompute: the update of iteration k from its
// partial state X (new messages into M, belief into bel, canonical state
// k + 1 into Yc) and the prologue of iteration k + 1 (partials into Y,
// marginals and belief into marg_next) in one pass; the same arithmetic as
// k_fu_final_tape followed by k_fu_prologue_tape on the canonical state
__global__ __launch_bounds__(256) void k_fu_rot_tape(Geo g, Strengths s, Inputs in, const float* __restrict__ X,
                                                     float* __restrict__ Y, float* __restrict__ Yc,
                                                     float* __restrict__ M, double* __restrict__ bel,
                                                     double* __restrict__ marg_next, int* __restrict__ health) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    if (u >= g.W || v >= g.H) return;
    iterate_pixel<false>(g, s, in, X, Y, nullptr, nullptr, health, u, v, M, bel, Yc, marg_next);
}

__global__ __launch_bounds__(256) void k_fu_final_tape(Geo g, Strengths s, Inputs in, const float* __restrict__ X,
                                                       float* __restrict__ Y, float* __restrict__ M,
                                                       double* __restrict__ bel, float* __restrict__ var_ll,
                                                       float* __restrict__ valid, int* __restrict__ health) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    if (u >= g.W || v >= g.H) return;
    iterate_pixel<true>(g, s, in, X, Y, var_ll, valid, health, u, v, M, bel);
}

// ---------------------------------------------------------------------------
// per-frame statistics (pose mean, valid count, health), deterministic two-stage reduction

constexpr int RED_THREADS = 256;

// the eight sums of a workgroup of RED_THREADS work-items: wavefront
// butterflies (every lane adds the same two operands, in either order), then
// the wavefronts' sums in order
__device__ inline void red8_block(double acc[8], double* __restrict__ out) {
    __shared__ double sh[RED_THREADS / 64][8];
    for (int m = 32; m > 0; m >>= 1)
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k] += __shfl_xor(acc[k], m, 64);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < 8; ++k) sh[threadIdx.x >> 6][k] = acc[k];
    __syncthreads();
    if (threadIdx.x < 8) {
        double t = 0.0;
        for (int w = 0; w < RED_THREADS / 64; ++w) t += sh[w][threadIdx.x];
        out[threadIdx.x] = t;
    }
}

// The sums are taken over a fixed decomposition of the image, independent of
// any launch shape: 64 x 4 pixel tiles in row-major tile order, one record per
// tile, then the records of an image in one strided order. A single context and
// a batch therefore reduce a sequence's planes in the same order and agree bit
// for bit.
constexpr int ST_X = 64, ST_Y = RED_THREADS / ST_X;

__host__ __device__ inline int stat_tiles_x(int W) { return (W + ST_X - 1) / ST_X; }
__host__ __device__ inline int stat_tiles(int H, int W) { return stat_tiles_x(W) * ((H + ST_Y - 1) / ST_Y); }

// one 64 x 4 tile: sum of the six pose planes, valid count (when use_valid),
// non-finite count, written as out[0..7]; one workgroup of RED_THREADS
__device__ inline void tile_stats(const Geo& g, const float* __restrict__ X, const float* __restrict__ valid,
                                  int use_valid, int tile, double* __restrict__ out) {
    const int ntx = stat_tiles_x(g.W);
    const int u = (tile % ntx) * ST_X + (int)(threadIdx.x % ST_X);
    const int v = (tile / ntx) * ST_Y + (int)(threadIdx.x / ST_X);
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (u < g.W && v < g.H) {
        const long p = pix_of(g, u, v);
        bool fin = true;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const float x = X[(long)k * g.plane + p];
            acc[k] = (double)x;
            fin = fin && isfinite(x);
        }
        fin = fin && isfinite(X[(long)P_ELL * g.plane + p]);
        acc[6] = use_valid ? (double)valid[p] : 0.0;
        acc[7] = fin ? 0.0 : 1.0;
    }
    red8_block(acc, out);
}

// the n tile records of one image, strided over the workgroup, then reduced
__device__ inline void image_stats(const double* __restrict__ partial, int n, double* __restrict__ out) {
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < n; b += RED_THREADS)
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k] += partial[(long)b * 8 + k];
    red8_block(acc, out);
}

__global__ __launch_bounds__(RED_THREADS) void k_frame_stats(Geo g, const float* __restrict__ X,
                                                            const float* __restrict__ valid, int use_valid,
                                                            double* __restrict__ partial) {
    tile_stats(g, X, valid, use_valid, blockIdx.x, partial + (long)blockIdx.x * 8);
}

// one workgroup: the sum of the nb tile records, in one fixed order;
// result[8] receives the health flag (when given) so that one copy returns both
__global__ __launch_bounds__(RED_THREADS) void k_frame_final(int nblocks, const double* __restrict__ partial,
                                                            double* __restrict__ result,
                                                            const int* __restrict__ health) {
    image_stats(partial, nblocks, result);
    if (health && threadIdx.x == 0) result[8] = (double)*health;
}

// output maps: inverse depth and its delta-method variance (dense H x W)
__global__ void k_outputs(Geo g, const float* __restrict__ X, const float* __restrict__ var_ll, int have_var,
                          float* __restrict__ inv_depth, float* __restrict__ inv_var) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    if (u >= g.W || v >= g.H) return;
    const long p = pix_of(g, u, v);
    const double rho = exp(-(double)X[(long)P_ELL * g.plane + p]);
    const long o = (long)v * g.W + u;
    if (inv_depth) inv_depth[o] = (float)rho;
    if (inv_var) inv_var[o] = have_var ? (float)(rho * rho * (double)var_ll[p]) : __int_as_float(0x7fc00000);
}

// valid-warp flags of the current state without iterating (n_iters == 0)
__global__ __launch_bounds__(256) void k_valid_only(Geo g, Strengths s, Inputs in, const float* __restrict__ X,
                                                    float* __restrict__ valid) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    if (u >= g.W || v >= g.H) return;
    const long p = pix_of(g, u, v);
    double tau[6], ell, R[9], t[3], L[28], eta[7];
    load_point(X, g, p, tau, ell);
    se3_exp(tau, R, t);
    valid[p] = unary_factors(g, s, in, u, v, tau, R, t, ell, L, eta) ? 1.0f : 0.0f;
}

// state exchange: pitched planes <-> dense planes
__global__ void k_pack_state(Geo g, const float* __restrict__ X, float* __restrict__ dense, int to_dense) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    if (u >= g.W || v >= g.H) return;
    const long p = pix_of(g, u, v);
    const long N = (long)g.H * g.W, o = (long)v * g.W + u;
    for (int k = 0; k < N_PLANES; ++k) {
        if (to_dense) dense[(long)k * N + o] = X[(long)k * g.plane + p];
        else ((float*)X)[(long)k * g.plane + p] = dense[(long)k * N + o];
    }
}

__global__ void k_copy_plane(Geo g, const float* __restrict__ dense, float* __restrict__ plane) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    if (u >= g.W || v >= g.H) return;
    plane[pix_of(g, u, v)] = dense[(long)v * g.W + u];
}

// ---------------------------------------------------------------------------
// batched schedule: many sequences of mixed resolution in one launch per pass.
// Each workgroup takes one (sequence, tile) item of the work list; the
// per-pixel arithmetic is the single-sequence code, so results do not depend
// on batching or on the tile shape.

__device__ inline bool batch_pixel(const SeqDesc* __restrict__ seqs, const int2* __restrict__ work,
                                   const SeqDesc*& d, int& u, int& v, int& item) {
    const int2 w = work[blockIdx.x];
    item = w.x;
    d = &seqs[w.y];
    const int tile = w.x - d->tile_base;
    u = (tile % d->tiles_x) * (int)blockDim.x + (int)threadIdx.x;
    v = (tile / d->tiles_x) * (int)blockDim.y + (int)threadIdx.y;
    return u < d->g.W && v < d->g.H;
}

__global__ void k_batch_frame_prep(const SeqDesc* __restrict__ seqs, const int2* __restrict__ work) {
    const SeqDesc* d;
    int u, v, item;
    if (!batch_pixel(seqs, work, d, u, v, item)) return;
    frame_prep_pixel(d->g, d->frame, d->g.W, d->It, d->Gx, d->Gy, u, v);
}

__global__ __launch_bounds__(256) void k_batch_prologue(const SeqDesc* __restrict__ seqs, const int2* __restrict__ work,
                                                        int parity, Strengths s, int* __restrict__ health) {
    const SeqDesc* d;
    int u, v, item;
    if (!batch_pixel(seqs, work, d, u, v, item)) return;
    const float* X = parity ? d->X1 : d->X0;
    float* Y = parity ? d->X0 : d->X1;
    prologue_pixel(d->g, s, d->in, X, Y, health, u, v);
}

template <bool FINAL>
__global__ __launch_bounds__(256) void k_batch_iterate(const SeqDesc* __restrict__ seqs, const int2* __restrict__ work,
                                                       int parity, Strengths s, int* __restrict__ health) {
    const SeqDesc* d;
    int u, v, item;
    if (!batch_pixel(seqs, work, d, u, v, item)) return;
    const float* X = parity ? d->X1 : d->X0;
    float* Y = parity ? d->X0 : d->X1;
    iterate_pixel_pf<FINAL, false, false, true>(d->g, s, d->in, X, Y, d->var_ll, d->valid, health, u, v);
}

// per sequence (blockIdx.y) and 64 x 4 tile of its image (blockIdx.x): the
// tile's sums, at the sequence's record base; the same tiles and order as a
// single context's statistics
__global__ __launch_bounds__(RED_THREADS) void k_batch_stats(const SeqDesc* __restrict__ seqs, int parity,
                                                            double* __restrict__ partial) {
    const SeqDesc* d = &seqs[blockIdx.y];
    if ((int)blockIdx.x >= stat_tiles(d->g.H, d->g.W)) return;
    const float* X = parity ? d->X1 : d->X0;
    tile_stats(d->g, X, d->valid, 1, blockIdx.x, partial + (long)(d->stat_base + (int)blockIdx.x) * 8);
}

// one workgroup per sequence: its tile records in the single-context order
__global__ __launch_bounds__(RED_THREADS) void k_batch_final(const SeqDesc* __restrict__ seqs,
                                                            const double* __restrict__ partial,
                                                            double* __restrict__ result) {
    const SeqDesc* d = &seqs[blockIdx.x];
    image_stats(partial + (long)d->stat_base * 8, stat_tiles(d->g.H, d->g.W), result + (long)blockIdx.x * 8);
}

static void launch_batch_stats(const BatchLaunch& b, int parity, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_stats, dim3(b.max_stat_tiles, b.n_seq), dim3(RED_THREADS), 0, st, b.seqs, parity,
                       b.partial);
    hipLaunchKernelGGL(k_batch_final, dim3(b.n_seq), dim3(RED_THREADS), 0, st, b.seqs, b.partial, b.result);
}

__global__ void k_clear_int(int* __restrict__ p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = 0;
}

// keyframe test of the frame just tracked for every sequence (Sec. 3.5: frame
// count and overlap), on the device: flags and the frame counter
__global__ void k_batch_keyframe_test(const SeqDesc* __restrict__ seqs, int n_seq, const double* __restrict__ result,
                                      const int* __restrict__ health, int* __restrict__ fsk,
                                      unsigned* __restrict__ flags, int max_frames, float min_valid, int reanchor) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_seq) return;
    const double inv_n = 1.0 / ((double)seqs[i].g.H * seqs[i].g.W);
    const float vf = (float)(result[8 * i + 6] * inv_n);
    const int count = fsk[i] + 1;
    unsigned f = 0;
    if (count >= max_frames || vf < min_valid) f |= 1u;          // keyframe due
    if (vf < min_valid) f |= 4u;                                  // low overlap
    if (result[8 * i + 7] > 0.0 || *health != 0) f |= 2u;         // diverged
    flags[i] = f;
    fsk[i] = (reanchor && (f & 1u)) ? 0 : count;
}

// re-anchoring on the frame just tracked, predicated on the device flag of
// the tile's sequence: the frame becomes the keyframe image, its normals the
// normal-integration targets; pose linearisation points and messages reset,
// log-depths kept (the graph of a frame step has no branches)
__global__ __launch_bounds__(256) void k_batch_keyframe_apply(const SeqDesc* __restrict__ seqs,
                                                              const int2* __restrict__ work, int parity,
                                                              const unsigned* __restrict__ flags) {
    const SeqDesc* d;
    int u, v, item;
    const bool in_img = batch_pixel(seqs, work, d, u, v, item);
    const int seq = work[blockIdx.x].y;
    if (!in_img || !(flags[seq] & 1u)) return;
    float* X = parity ? d->X1 : d->X0;
    float* X2 = parity ? d->X0 : d->X1;
    keyframe_prep_pixel(d->g, d->frame, d->normals, d->Is, d->cxt, d->cyt, X, X2, u, v);
}

__global__ void k_set_ints(int* __restrict__ p, int n, int value) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

// the iteration block of a frame step in one launch: the n_passes non-final
// passes that follow the prologue, with a grid-wide barrier between passes
// (the prologue and the final pass, which writes the canonical messages, are
// launches of their own). The grid is co-resident (cooperative launch) and a
// multiple of 8 workgroups, so workgroup b, which runs items b, b + G,
// b + 2G, ..., stays with the work list's range of its XCD. Every workgroup
// reaches every barrier: pixels outside an image skip the arithmetic, not the
// barrier.
__global__ __launch_bounds__(256) void k_batch_persistent(const SeqDesc* __restrict__ seqs,
                                                          const int2* __restrict__ work, int n_work, int parity,
                                                          int n_passes, Strengths s, int* __restrict__ health) {
    cg::grid_group grid = cg::this_grid();
    for (int pass = 0; pass < n_passes; ++pass) {
        const int par = parity ^ (pass & 1);
        for (int w = blockIdx.x; w < n_work; w += gridDim.x) {
            const int2 wi = work[w];
            const SeqDesc* d = &seqs[wi.y];
            const int tile = wi.x - d->tile_base;
            const int u = (tile % d->tiles_x) * (int)blockDim.x + (int)threadIdx.x;
            const int v = (tile / d->tiles_x) * (int)blockDim.y + (int)threadIdx.y;
            if (u < d->g.W && v < d->g.H) {
                const float* X = par ? d->X1 : d->X0;
                float* Y = par ? d->X0 : d->X1;
                iterate_pixel_pf<false, false, false, true>(d->g, s, d->in, X, Y, d->var_ll, d->valid, health, u, v);
            }
        }
        if (pass + 1 < n_passes) grid.sync();
    }
}

hipError_t launch_batch_frame_step(const BatchLaunch& b, int n_iters, hipStream_t st) {
    const dim3 blk(b.tile_x, b.tile_y), grid(b.n_work);
    hipLaunchKernelGGL(k_clear_int, dim3(1), dim3(64), 0, st, b.health);
    hipLaunchKernelGGL(k_batch_frame_prep, grid, blk, 0, st, b.seqs, b.work);
    int parity = b.parity;
    if (n_iters > 0) {
        hipLaunchKernelGGL(k_batch_prologue, grid, blk, 0, st, b.seqs, b.work, parity, b.s, b.health);
        parity ^= 1;
        for (int it = 0; it < n_iters; ++it) {
            if (it == n_iters - 1)
                hipLaunchKernelGGL(k_batch_iterate<true>, grid, blk, 0, st, b.seqs, b.work, parity, b.s, b.health);
            else
                hipLaunchKernelGGL(k_batch_iterate<false>, grid, blk, 0, st, b.seqs, b.work, parity, b.s, b.health);
            parity ^= 1;
        }
    }
    launch_batch_stats(b, parity, st);
    return launch_batch_keyframe(b, parity, st);
}

hipError_t launch_set_ints(int* p, int n, int value, hipStream_t st) {
    hipLaunchKernelGGL(k_set_ints, dim3((n + 255) / 256), dim3(256), 0, st, p, n, value);
    return hipGetLastError();
}

hipError_t launch_batch_keyframe(const BatchLaunch& b, int parity, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_keyframe_test, dim3((b.n_seq + 63) / 64), dim3(64), 0, st, b.seqs, b.n_seq, b.result,
                       b.health, b.fsk, b.flags, b.kf_max_frames, b.kf_min_valid, b.reanchor);
    if (b.reanchor)
        hipLaunchKernelGGL(k_batch_keyframe_apply, dim3(b.n_work), dim3(b.tile_x, b.tile_y), 0, st, b.seqs, b.work,
                           parity, b.flags);
    return hipGetLastError();
}

int batch_persistent_grid(const BatchLaunch& b) {
    int per_cu = 0, dev = 0, n_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_batch_persistent),
                                                     b.tile_x * b.tile_y, 0) != hipSuccess)
        return 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    int g = per_cu * n_cu;
    if (g > b.n_work) g = b.n_work;
    if (g >= 8) g -= g % 8;
    return g;
}

hipError_t launch_batch_frame_step_persistent(const BatchLaunch& b, int n_iters, int grid_blocks, hipStream_t st) {
    const dim3 blk(b.tile_x, b.tile_y), grid(b.n_work);
    hipLaunchKernelGGL(k_clear_int, dim3(1), dim3(64), 0, st, b.health);
    hipLaunchKernelGGL(k_batch_frame_prep, grid, blk, 0, st, b.seqs, b.work);
    hipLaunchKernelGGL(k_batch_prologue, grid, blk, 0, st, b.seqs, b.work, b.parity, b.s, b.health);
    const SeqDesc* seqs = b.seqs;
    const int2* work = b.work;
    int n_work = b.n_work, parity = b.parity ^ 1, n_passes = n_iters - 1;
    Strengths s = b.s;
    int* health = b.health;
    if (n_passes > 0) {
        void* args[] = {&seqs, &work, &n_work, &parity, &n_passes, &s, &health};
        hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_batch_persistent), dim3(grid_blocks),
                                                  blk, args, 0, st);
        if (e != hipSuccess) return e;
    }
    const int fin = b.parity ^ 1 ^ (n_passes & 1);
    hipLaunchKernelGGL(k_batch_iterate<true>, grid, blk, 0, st, b.seqs, b.work, fin, b.s, b.health);
    const int par = fin ^ 1;
    launch_batch_stats(b, par, st);
    return launch_batch_keyframe(b, par, st);
}

hipError_t launch_batch_passes(const BatchLaunch& b, int n_iters, bool prologue, bool final_last, hipStream_t st) {
    const dim3 blk(b.tile_x, b.tile_y), grid(b.n_work);
    int parity = b.parity;
    if (prologue) {
        hipLaunchKernelGGL(k_batch_prologue, grid, blk, 0, st, b.seqs, b.work, parity, b.s, b.health);
        parity ^= 1;
    }
    for (int it = 0; it < n_iters; ++it) {
        if (final_last && it == n_iters - 1)
            hipLaunchKernelGGL(k_batch_iterate<true>, grid, blk, 0, st, b.seqs, b.work, parity, b.s, b.health);
        else
            hipLaunchKernelGGL(k_batch_iterate<false>, grid, blk, 0, st, b.seqs, b.work, parity, b.s, b.health);
        parity ^= 1;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// launchers

static dim3 grid2d(const Geo& g, dim3 b) { return dim3((g.W + b.x - 1) / b.x, (g.H + b.y - 1) / b.y); }
static const dim3 kBlock(64, 1);
// fused passes: 64 x 4 tiles keep the vertical neighbours' points and partials
// in the same workgroup's cache lines (measured 1.15x against 1.24x of the
// algorithmic bytes for 64 x 1 at 640x480, same duration)
static const dim3 kBlockFused(64, 4);

hipError_t launch_frame_prep(const Geo& g, const float* src, long src_pitch, float* It, float* Gx, float* Gy,
                             hipStream_t st, int* clear) {
    hipLaunchKernelGGL(k_frame_prep, grid2d(g, kBlock), kBlock, 0, st, g, src, src_pitch, It, Gx, Gy, clear);
    return hipGetLastError();
}

hipError_t launch_keyframe_prep(const Geo& g, const float* img, const float* normals, float* Is, float* cxt,
                                float* cyt, float* X, float* X2, hipStream_t st) {
    hipLaunchKernelGGL(k_keyframe_prep, grid2d(g, kBlock), kBlock, 0, st, g, img, normals, Is, cxt, cyt, X, X2);
    return hipGetLastError();
}

hipError_t launch_init_state(const Geo& g, float* X, float ell0, hipStream_t st) {
    hipLaunchKernelGGL(k_init_state, grid2d(g, kBlock), kBlock, 0, st, g, X, ell0);
    return hipGetLastError();
}

hipError_t launch_pf_iteration(const Geo& g, const Strengths& s, const Inputs& in, float* X, double* marg,
                               double* M, float* var_ll, float* valid, float beta, int* health, hipStream_t st) {
    hipLaunchKernelGGL(k_pf_linearise, grid2d(g, kBlock), kBlock, 0, st, g, s, in, X, marg, valid, health);
    hipLaunchKernelGGL(k_pf_messages, grid2d(g, kBlock), kBlock, 0, st, g, s, in, X, marg, M, beta, health);
    hipLaunchKernelGGL(k_pf_update, grid2d(g, kBlock), kBlock, 0, st, g, s, in, X, M, var_ll, valid, health);
    return hipGetLastError();
}

hipError_t launch_fu_prologue(const Geo& g, const Strengths& s, const Inputs& in, const float* X, float* Y,
                              int* health, hipStream_t st) {
    hipLaunchKernelGGL(k_fu_prologue, grid2d(g, kBlockFused), kBlockFused, 0, st, g, s, in, X, Y, health);
    return hipGetLastError();
}

hipError_t launch_fu_iterate(const Geo& g, const Strengths& s, const Inputs& in, const float* X, float* Y,
                             bool final_pass, float* var_ll, float* valid, int* health, hipStream_t st) {
    static int n_cu = 0;
    if (n_cu == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu < 1)
            n_cu = 256;
    }
    const dim3 t = grid2d(g, kBlockFused);
    const int ntiles = (int)(t.x * t.y);
    const dim3 grid((unsigned)std::min(ntiles, n_cu));
    if (final_pass)
        hipLaunchKernelGGL(k_fu_iterate<true>, grid, kBlockFused, 0, st, g, s, in, X, Y, var_ll, valid, health,
                           (int)t.x, ntiles);
    else
        hipLaunchKernelGGL(k_fu_iterate<false>, grid, kBlockFused, 0, st, g, s, in, X, Y, var_ll, valid, health,
                           (int)t.x, ntiles);
    return hipGetLastError();
}

hipError_t launch_fu_segment_tape(const Geo& g, const Strengths& s, const Inputs& in, const float* X0, float* seg,
                                  long seg_stride, int len, float* tA, float* tB, double* marg, long marg_stride,
                                  float* M, long M_stride, double* bel, long bel_stride, float* var_ll, float* valid,
                                  int* health, hipStream_t st) {
    if (len < 1) return hipSuccess;
    const dim3 grid = grid2d(g, kBlockFused);
    hipLaunchKernelGGL(k_fu_prologue_tape, grid, kBlockFused, 0, st, g, s, in, X0, tA, marg, health);
    float* t[2] = {tA, tB};
    for (int k = 0; k + 1 < len; ++k)
        hipLaunchKernelGGL(k_fu_rot_tape, grid, kBlockFused, 0, st, g, s, in, t[k & 1], t[(k + 1) & 1],
                           seg + seg_stride * (k + 1), M + M_stride * k, bel + bel_stride * k,
                           marg + marg_stride * (k + 1), health);
    const int k = len - 1;
    hipLaunchKernelGGL(k_fu_final_tape, grid, kBlockFused, 0, st, g, s, in, t[k & 1], t[(k + 1) & 1],
                       M + M_stride * k, bel + bel_stride * k, var_ll, valid, health);
    return hipGetLastError();
}

hipError_t launch_valid_only(const Geo& g, const Strengths& s, const Inputs& in, const float* X, float* valid,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_valid_only, grid2d(g, kBlock), kBlock, 0, st, g, s, in, X, valid);
    return hipGetLastError();
}

int stats_blocks(const Geo& g) { return stat_tiles(g.H, g.W); }

hipError_t launch_frame_stats(const Geo& g, const float* X, const float* valid, int use_valid, double* partial,
                              double* result, hipStream_t st, const int* health) {
    const int nb = stats_blocks(g);
    hipLaunchKernelGGL(k_frame_stats, dim3(nb), dim3(RED_THREADS), 0, st, g, X, valid, use_valid, partial);
    hipLaunchKernelGGL(k_frame_final, dim3(1), dim3(RED_THREADS), 0, st, nb, partial, result, health);
    return hipGetLastError();
}

hipError_t launch_outputs(const Geo& g, const float* X, const float* var_ll, int have_var, float* inv_depth,
                          float* inv_var, hipStream_t st) {
    hipLaunchKernelGGL(k_outputs, grid2d(g, kBlock), kBlock, 0, st, g, X, var_ll, have_var, inv_depth, inv_var);
    return hipGetLastError();
}

hipError_t launch_pack_state(const Geo& g, const float* X, float* dense, int to_dense, hipStream_t st) {
    hipLaunchKernelGGL(k_pack_state, grid2d(g, kBlock), kBlock, 0, st, g, X, dense, to_dense);
    return hipGetLastError();
}

hipError_t launch_copy_plane(const Geo& g, const float* dense, float* plane, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_plane, grid2d(g, kBlock), kBlock, 0, st, g, dense, plane);
    return hipGetLastError();
}

}  // namespace pv
