// HIP kernels of the quadtree identity topology (PixVOD, arXiv 2606.03989,
// Fig. 2, Sec. 3.3, Sec. 4.2) for gfx950.
//
// The synchronous iteration of Sec. 4.1 in the same rotated form as the grid's
// fused schedule: a sender turns its belief and its stored message from a
// factor into a partial message (independent of the receiver's linearisation
// point); the receiver completes it with the factor residual at both points,
// updates and relinearises its variable, then sends its next partials. Each
// iteration is two launches over the same buffers, one lane per pixel and one
// lane per node (all levels in one launch, each workgroup inside one level).
//
// Where partials live: a variable's partial towards its parent, and a node's
// partials towards its children, stay in the sender's own slots (coalesced
// writes from the wide lower levels; the parent gathers four children from
// two adjacent rows). Normal-integration partials go into the receiver's
// slot, as on the grid. At frame ends the same slots hold the canonical
// messages, each stored at the variable that receives it.
#include "gbp_tree.h"
#include "gbp_device.hpp"

#include <cmath>

namespace pv {

namespace {

__device__ inline void load_part27(const float* __restrict__ base, long stride, long p, float part[27]) {
#pragma unroll
    for (int k = 0; k < 27; ++k) part[k] = base[(long)k * stride + p];
}

__device__ inline void store_msg27(float* __restrict__ base, long stride, long p, const float m[27]) {
#pragma unroll
    for (int k = 0; k < 27; ++k) base[(long)k * stride + p] = m[k];
}

// receiver-side completion of an identity partial (h, Lambda') with the
// residual r seen by the receiver: eta = h - Lambda' r; the message is added
// to the pose block of the belief and kept at storage precision
template <int LD>
__device__ inline void complete_identity(const float part[27], const double r[6], double* L, double* eta,
                                         float msg[27]) {
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        double e = (double)part[a];
#pragma unroll
        for (int b = 0; b < 6; ++b) e -= (double)part[6 + s6(a, b)] * r[b];
        eta[a] += e;
        msg[a] = (float)e;
    }
#pragma unroll
    for (int r_ = 0; r_ < 6; ++r_)
#pragma unroll
        for (int c = r_; c < 6; ++c) L[LD == 7 ? s7(r_, c) : s6(r_, c)] += (double)part[6 + s6(r_, c)];
#pragma unroll
    for (int k = 0; k < 21; ++k) msg[6 + k] = part[6 + k];
}

template <int LD>
__device__ inline void add_identity(const float m[27], double* L, double* eta) {
#pragma unroll
    for (int a = 0; a < 6; ++a) eta[a] += (double)m[a];
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = r; c < 6; ++c) L[LD == 7 ? s7(r, c) : s6(r, c)] += (double)m[6 + s6(r, c)];
}

// first-order transport of a stored identity message by the mean step m
__device__ inline void transport_identity(float msg[27], const double m[6]) {
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        double s = (double)msg[a];
#pragma unroll
        for (int b = 0; b < 6; ++b) s -= (double)msg[6 + s6(a, b)] * m[b];
        msg[a] = (float)s;
    }
}

// sender-side partial of an identity factor from the sender's pose marginal
// (P, p) minus the factor's stored message to the sender
__device__ inline bool identity_partial_from(double lamR, const double P[21], const double p[6], const float back[27],
                                             float part[27]) {
    double V[21], v[6], Lp[21], h[6];
#pragma unroll
    for (int k = 0; k < 21; ++k) V[k] = P[k] - (double)back[6 + k];
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = p[k] - (double)back[k];
    const bool ok = identity_partial(lamR, V, v, Lp, h);
#pragma unroll
    for (int k = 0; k < 6; ++k) part[k] = (float)h[k];
#pragma unroll
    for (int k = 0; k < 21; ++k) part[6 + k] = (float)Lp[k];
    return ok;
}

// pose prior of a node (Eq. prior) with precision lamP at Exp(tau) = (R, t):
// r = Log(Exp(xi_hat)^-1 Exp(tau)), J = I + ad(r)/2 + ad(r)^2/12
__device__ inline void node_prior(const Strengths& s, double lamP, const double tau[6], const double R[9],
                                  const double t[3], double L[21], double eta[6]) {
    double rp[6];
    if (s.prior_is_identity) {
#pragma unroll
        for (int k = 0; k < 6; ++k) rp[k] = tau[k];
    } else {
        double Rr[9], tr[3];
        se3_compose(s.prior_R, s.prior_t, R, t, Rr, tr);
        se3_log(Rr, tr, rp);
    }
    // J = [[A, 0], [B, A]]: A = I + W/2 + W^2/12, B = P/2 + (P W + W P)/12,
    // W = [theta]x and P = [rho]x of r
    const double w0 = rp[0], w1 = rp[1], w2 = rp[2], p0 = rp[3], p1 = rp[4], p2 = rp[5];
    const double Wm[9] = {0.0, -w2, w1, w2, 0.0, -w0, -w1, w0, 0.0};
    const double Pm[9] = {0.0, -p2, p1, p2, 0.0, -p0, -p1, p0, 0.0};
    double A[9], B[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double ww = 0.0, pw = 0.0, wp = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                ww += Wm[r * 3 + k] * Wm[k * 3 + c];
                pw += Pm[r * 3 + k] * Wm[k * 3 + c];
                wp += Wm[r * 3 + k] * Pm[k * 3 + c];
            }
            A[r * 3 + c] = (r == c ? 1.0 : 0.0) + 0.5 * Wm[r * 3 + c] + ww * (1.0 / 12.0);
            B[r * 3 + c] = 0.5 * Pm[r * 3 + c] + (pw + wp) * (1.0 / 12.0);
        }
    // column a of J: rows 0..2 from A (a < 3), rows 3..5 from B (a < 3) or A (a >= 3)
    double J[36];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            J[r * 6 + c] = A[r * 3 + c];
            J[r * 6 + c + 3] = 0.0;
            J[(r + 3) * 6 + c] = B[r * 3 + c];
            J[(r + 3) * 6 + c + 3] = A[r * 3 + c];
        }
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        double e = 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k) e += J[k * 6 + a] * rp[k];
        eta[a] = -lamP * e;
#pragma unroll
        for (int b = a; b < 6; ++b) {
            double g = 0.0;
#pragma unroll
            for (int k = 0; k < 6; ++k) g += J[k * 6 + a] * J[k * 6 + b];
            L[s6(a, b)] = lamP * g;
        }
    }
}

// per-workgroup level of a node launch (uniform across the workgroup)
struct Level {
    int l, H, W, off, b0;      // this level
    int Wp, offp;              // parent level
    int Hc, Wc, offc;          // child level
    double lamP, lamR_up, lamR_down;
};

__device__ inline Level level_of_block(const TreeGeo& t, int b) {
    Level v;
    v.l = 1;
#pragma unroll
    for (int k = 2; k <= kTreeMaxLevels; ++k)
        if (k <= t.L && b >= t.bstart[k]) v.l = k;
    // gather the fields with constant indices only (no dynamic indexing of
    // the kernel-argument structure)
    v.H = v.W = v.off = v.b0 = v.Wp = v.offp = v.Hc = v.Wc = v.offc = 0;
    v.lamP = v.lamR_up = v.lamR_down = 0.0;
#pragma unroll
    for (int k = 1; k <= kTreeMaxLevels; ++k)
        if (k == v.l) {
            v.H = t.Hl[k];
            v.W = t.Wl[k];
            v.off = t.off[k];
            v.b0 = t.bstart[k];
            v.Hc = t.Hl[k - 1];
            v.Wc = t.Wl[k - 1];
            v.offc = t.off[k - 1];
            v.lamP = t.lamP[k];
            v.lamR_up = t.lamR[k];
            v.lamR_down = t.lamR[k - 1];
            if (k < kTreeMaxLevels) {
                v.Wp = t.Wl[k + 1];
                v.offp = t.off[k + 1];
            }
        }
    return v;
}

__device__ inline void round6(double tau[6]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) tau[k] = (double)(float)tau[k];
}

// ---------------------------------------------------------------------------
// pixels

// sender side of a pixel: partial towards the parent (own slot) and the
// normal-integration partials (neighbours' slots) from the belief (L, eta)
__device__ inline bool pixel_emit(const Geo& g, const Strengths& s, const Inputs& in, int u, int v,
                                  const double L[28], const double eta[7], const float mup[27],
                                  const float mn[4][2], float* __restrict__ Y) {
    double P[21], p[6], D, dv;
    pose_marginal(L, eta, P, p);
    bool ok = depth_marginal(L, eta, D, dv);
    const long pi = pix_of(g, u, v);
    float part[27];
    ok = identity_partial_from(s.lamR, P, p, mup, part) && ok;
    store_msg27(Y + (long)TP_UP * g.plane, g.plane, pi, part);
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        int nu, nv;
        if (!neighbour(g, u, v, d, nu, nv)) continue;
        const long pj = pix_of(g, nu, nv);
        float* dn = Y + (long)(TP_MN + 2 * opposite(d)) * g.plane + pj;
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
    return ok;
}

__device__ inline void pixel_store_point(float* __restrict__ Y, const Geo& g, long p, const double tau[6], double ell) {
#pragma unroll
    for (int k = 0; k < 6; ++k) Y[(P_TAU + k) * g.plane + p] = (float)tau[k];
    Y[P_ELL * g.plane + p] = (float)ell;
}

__global__ __launch_bounds__(256) void k_tr_pixel_prologue(Geo g, TreeGeo t, Strengths s, Inputs in,
                                                           const float* __restrict__ X, float* __restrict__ Y,
                                                           int* __restrict__ health) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    if (u >= g.W || v >= g.H) return;
    const long p = pix_of(g, u, v);
    double tau[6], ell, R[9], tt[3], L[28], eta[7];
    load_point(X, g, p, tau, ell);
    se3_exp(tau, R, tt);
    unary_factors<true>(g, s, in, u, v, tau, R, tt, ell, L, eta);
    float mup[27], mn[4][2];
    load_part27(X + (long)TP_UP * g.plane, g.plane, p, mup);
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        mn[d][0] = X[(long)(TP_MN + 2 * d) * g.plane + p];
        mn[d][1] = X[(long)(TP_MN + 2 * d + 1) * g.plane + p];
        eta[6] += (double)mn[d][0];
        L[s7(6, 6)] += (double)mn[d][1];
    }
    add_identity<7>(mup, L, eta);
    const bool ok = pixel_emit(g, s, in, u, v, L, eta, mup, mn, Y);
    pixel_store_point(Y, g, p, tau, ell);
    if (!ok) atomicOr(health, 1);
}

template <bool FINAL>
__global__ __launch_bounds__(256) void k_tr_pixel_iterate(Geo g, TreeGeo t, Strengths s, Inputs in,
                                                          const float* __restrict__ X, const float* __restrict__ NX,
                                                          float* __restrict__ Y, float* __restrict__ var_ll,
                                                          float* __restrict__ valid, int* __restrict__ health) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    if (u >= g.W || v >= g.H) return;
    const long pi = pix_of(g, u, v);
    double tau[6], ell, R[9], tt[3], L[28], eta[7];
    load_point(X, g, pi, tau, ell);
    se3_exp(tau, R, tt);
    const bool val = unary_factors<true>(g, s, in, u, v, tau, R, tt, ell, L, eta);

    // the parent's partial for this child slot, completed at both points
    float mup[27];
    {
        const long pn = (long)t.off[1] + (long)(v >> 1) * t.Wl[1] + (u >> 1);
        const int q = ((v & 1) << 1) | (u & 1);
        double tp[6], Rp[9], trp[3], r[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) tp[k] = (double)NX[(long)(TN_TAU + k) * t.nplane + pn];
        se3_exp(tp, Rp, trp);
        se3_between(Rp, trp, R, tt, r);
        float part[27];
        load_part27(NX + (long)(TN_CH + 27 * q) * t.nplane, t.nplane, pn, part);
        complete_identity<7>(part, r, L, eta, mup);
    }
    // normal-integration partials in this pixel's slots
    float mn[4][2];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        mn[d][0] = mn[d][1] = 0.0f;
        int nu, nv;
        if (!neighbour(g, u, v, d, nu, nv)) continue;
        const long pj = pix_of(g, nu, nv);
        const double ellj = (double)X[(long)P_ELL * g.plane + pj];
        double rn;
        if (s.lamN > 0.0 && normal_residual(g, in, pi, pj, d, ell, ellj, rn)) {
            const float* sn = X + (long)(TP_MN + 2 * d) * g.plane + pi;
            const float nl = sn[g.plane];
            const double ne = (double)sn[0] - (double)nl * rn;
            eta[6] += ne;
            L[s7(6, 6)] += (double)nl;
            mn[d][0] = (float)ne;
            mn[d][1] = nl;
        }
    }
    // update: mean, relinearisation (Eq. var), transport of the stored messages
    double idg[7], m[7];
    bool ok = chol7(L, idg);
#pragma unroll
    for (int k = 0; k < 7; ++k) m[k] = eta[k];
    chol7_solve(L, idg, m);
    const double var = chol7_var_last(idg);
    {
        double R1[9], t1[3], Rm[9], tm[3];
        se3_exp(m, Rm, tm);
        se3_compose(R, tt, Rm, tm, R1, t1);
        se3_log(R1, t1, tau);
    }
    ell += m[6];
    transport_identity(mup, m);
#pragma unroll
    for (int d = 0; d < 4; ++d) mn[d][0] = (float)((double)mn[d][0] - (double)mn[d][1] * m[6]);
    round6(tau);
    ell = (double)(float)ell;
    pixel_store_point(Y, g, pi, tau, ell);
    if (FINAL) {
        store_msg27(Y + (long)TP_UP * g.plane, g.plane, pi, mup);
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            Y[(long)(TP_MN + 2 * d) * g.plane + pi] = mn[d][0];
            Y[(long)(TP_MN + 2 * d + 1) * g.plane + pi] = mn[d][1];
        }
        var_ll[pi] = (float)var;
        valid[pi] = val ? 1.0f : 0.0f;
    } else {
        se3_exp(tau, R, tt);
        unary_factors<true>(g, s, in, u, v, tau, R, tt, ell, L, eta);
        add_identity<7>(mup, L, eta);
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            eta[6] += (double)mn[d][0];
            L[s7(6, 6)] += (double)mn[d][1];
        }
        ok = pixel_emit(g, s, in, u, v, L, eta, mup, mn, Y) && ok;
    }
    if (!ok) atomicOr(health, 1);
}

// ---------------------------------------------------------------------------
// nodes

// sender side of a node: partials towards its parent and its children, in
// its own slots
__device__ inline bool node_emit(const TreeGeo& t, const Level& lv, int x, int y, long n, const double L[21],
                                 const double eta[6], const float msg[5][27], float* __restrict__ NY) {
    bool ok = true;
    float part[27];
    if (lv.l < t.L) {
        ok = identity_partial_from(lv.lamR_up, L, eta, msg[0], part) && ok;
        store_msg27(NY + (long)TN_UP * t.nplane, t.nplane, n, part);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int cx = 2 * x + (q & 1), cy = 2 * y + (q >> 1);
        if (cx >= lv.Wc || cy >= lv.Hc) continue;
        ok = identity_partial_from(lv.lamR_down, L, eta, msg[1 + q], part) && ok;
        store_msg27(NY + (long)(TN_CH + 27 * q) * t.nplane, t.nplane, n, part);
    }
    return ok;
}

template <bool PROLOGUE, bool FINAL>
__global__ __launch_bounds__(kTreeThreads) void k_tr_node(Geo g, TreeGeo t, Strengths s,
                                                          const float* __restrict__ X, const float* __restrict__ NX,
                                                          float* __restrict__ NY, int* __restrict__ health) {
    const Level lv = level_of_block(t, (int)blockIdx.x);
    const int i = ((int)blockIdx.x - lv.b0) * kTreeThreads + (int)threadIdx.x;
    if (i >= lv.H * lv.W) return;
    const int x = i % lv.W, y = i / lv.W;
    const long n = (long)lv.off + i;
    double tau[6], R[9], tt[3], L[21], eta[6];
    float msg[5][27];
    bool ok = true;
    if (PROLOGUE) {
#pragma unroll
        for (int k = 0; k < 6; ++k) tau[k] = (double)NX[(long)(TN_TAU + k) * t.nplane + n];
        se3_exp(tau, R, tt);
        node_prior(s, lv.lamP, tau, R, tt, L, eta);
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            load_part27(NX + (long)(TN_UP + 27 * k) * t.nplane, t.nplane, n, msg[k]);
            add_identity<6>(msg[k], L, eta);
        }
    } else {
        // --- every load issued before any use (its address depends only on
        // the node index): the node's pose, the parent's pose and its partial
        // for this child slot, the children's poses and partials towards this
        // node. A missing parent or child reads the node itself; its values
        // are discarded.
        float tnf[6], tpf[6], tcf[4][6];
        const bool has_par = lv.l < t.L;
        const long pp = has_par ? (long)lv.offp + (long)(y >> 1) * lv.Wp + (x >> 1) : n;
        const int qn = ((y & 1) << 1) | (x & 1);
        bool has_c[4];
#pragma unroll
        for (int k = 0; k < 6; ++k) tnf[k] = NX[(long)(TN_TAU + k) * t.nplane + n];
#pragma unroll
        for (int k = 0; k < 6; ++k) tpf[k] = NX[(long)(TN_TAU + k) * t.nplane + pp];
        load_part27(NX + (long)(TN_CH + 27 * qn) * t.nplane, t.nplane, pp, msg[0]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int cx = 2 * x + (q & 1), cy = 2 * y + (q >> 1);
            has_c[q] = cx < lv.Wc && cy < lv.Hc;
            const int cxc = has_c[q] ? cx : 2 * x, cyc = has_c[q] ? cy : 2 * y;
            if (lv.l == 1) {
                const long pc = pix_of(g, cxc, cyc);
#pragma unroll
                for (int k = 0; k < 6; ++k) tcf[q][k] = X[(long)(P_TAU + k) * g.plane + pc];
                load_part27(X + (long)TP_UP * g.plane, g.plane, pc, msg[1 + q]);
            } else {
                const long nc = (long)lv.offc + (long)cyc * lv.Wc + cxc;
#pragma unroll
                for (int k = 0; k < 6; ++k) tcf[q][k] = NX[(long)(TN_TAU + k) * t.nplane + nc];
                load_part27(NX + (long)TN_UP * t.nplane, t.nplane, nc, msg[1 + q]);
            }
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) tau[k] = (double)tnf[k];
        se3_exp(tau, R, tt);
        node_prior(s, lv.lamP, tau, R, tt, L, eta);
        // parent's partial for this child slot, completed in place
        if (has_par) {
            double tp[6], Rp[9], trp[3], r[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) tp[k] = (double)tpf[k];
            se3_exp(tp, Rp, trp);
            se3_between(Rp, trp, R, tt, r);
            complete_identity<6>(msg[0], r, L, eta, msg[0]);
        } else {
#pragma unroll
            for (int k = 0; k < 27; ++k) msg[0][k] = 0.0f;
        }
        // children's partials towards this node
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (!has_c[q]) {
#pragma unroll
                for (int k = 0; k < 27; ++k) msg[1 + q][k] = 0.0f;
                continue;
            }
            double tc[6], Rc[9], trc[3], r[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) tc[k] = (double)tcf[q][k];
            se3_exp(tc, Rc, trc);
            se3_between(Rc, trc, R, tt, r);
            complete_identity<6>(msg[1 + q], r, L, eta, msg[1 + q]);
        }
        // update: mean, relinearisation, transport
        double idg[6], m[6];
        ok = chol6(L, idg);
#pragma unroll
        for (int k = 0; k < 6; ++k) m[k] = eta[k];
        chol6_solve(L, idg, m);
        {
            double R1[9], t1[3], Rm[9], tm[3];
            se3_exp(m, Rm, tm);
            se3_compose(R, tt, Rm, tm, R1, t1);
            se3_log(R1, t1, tau);
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) transport_identity(msg[k], m);
        round6(tau);
        if (FINAL) {
#pragma unroll
            for (int k = 0; k < 6; ++k) NY[(long)(TN_TAU + k) * t.nplane + n] = (float)tau[k];
#pragma unroll
            for (int k = 0; k < 5; ++k) store_msg27(NY + (long)(TN_UP + 27 * k) * t.nplane, t.nplane, n, msg[k]);
            if (!ok) atomicOr(health, 1);
            return;
        }
        se3_exp(tau, R, tt);
        node_prior(s, lv.lamP, tau, R, tt, L, eta);
#pragma unroll
        for (int k = 0; k < 5; ++k) add_identity<6>(msg[k], L, eta);
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) NY[(long)(TN_TAU + k) * t.nplane + n] = (float)tau[k];
    ok = node_emit(t, lv, x, y, n, L, eta, msg, NY) && ok;
    if (!ok) atomicOr(health, 1);
}

__global__ void k_tr_clear(float* __restrict__ p, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

__global__ void k_tr_pack_pixels(Geo g, float* __restrict__ X, float* __restrict__ dense, int to_dense) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    if (u >= g.W || v >= g.H) return;
    const long p = pix_of(g, u, v), d = (long)v * g.W + u, N = (long)g.H * g.W;
    for (int k = 0; k < TP_PLANES; ++k) {
        if (to_dense) dense[(long)k * N + d] = X[(long)k * g.plane + p];
        else X[(long)k * g.plane + p] = dense[(long)k * N + d];
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// host side

bool make_tree_geo(int H, int W, double sigma_P, double sigma_R, TreeGeo* t) {
    *t = TreeGeo{};
    t->Hl[0] = H;
    t->Wl[0] = W;
    int L = 0;
    while (t->Hl[L] > 1 || t->Wl[L] > 1) {
        if (L == kTreeMaxLevels) return false;
        t->Hl[L + 1] = (t->Hl[L] + 1) / 2;
        t->Wl[L + 1] = (t->Wl[L] + 1) / 2;
        ++L;
    }
    if (L == 0) return false;
    t->L = L;
    t->off[0] = 0;
    t->off[1] = 0;
    t->bstart[1] = 0;
    for (int l = 1; l <= L; ++l) {
        const int n = t->Hl[l] * t->Wl[l];
        t->off[l + 1] = t->off[l] + n;
        t->bstart[l + 1] = t->bstart[l] + (n + kTreeThreads - 1) / kTreeThreads;
    }
    t->NT = t->off[L + 1];
    t->nblocks = t->bstart[L + 1];
    t->nplane = ((long)t->NT + 63) / 64 * 64;
    for (int l = 0; l <= L; ++l) {
        const double sp = std::ldexp(sigma_P, -l), sr = std::ldexp(sigma_R, -l);
        t->lamP[l] = 1.0 / (sp * sp);
        t->lamR[l] = 1.0 / (sr * sr);
    }
    return true;
}

static const dim3 kTreeBlock(64, 4);
static dim3 tree_grid2d(const Geo& g) {
    return dim3((g.W + kTreeBlock.x - 1) / kTreeBlock.x, (g.H + kTreeBlock.y - 1) / kTreeBlock.y);
}

hipError_t launch_tree_prologue(const Geo& g, const TreeGeo& t, const Strengths& s, const Inputs& in,
                                const float* X, const float* NX, float* Y, float* NY, int* health, hipStream_t st) {
    hipLaunchKernelGGL(k_tr_pixel_prologue, tree_grid2d(g), kTreeBlock, 0, st, g, t, s, in, X, Y, health);
    hipLaunchKernelGGL((k_tr_node<true, false>), dim3(t.nblocks), dim3(kTreeThreads), 0, st, g, t, s, X, NX, NY,
                       health);
    return hipGetLastError();
}

hipError_t launch_tree_iterate(const Geo& g, const TreeGeo& t, const Strengths& s, const Inputs& in,
                               const float* X, const float* NX, float* Y, float* NY, bool final_pass,
                               float* var_ll, float* valid, int* health, hipStream_t st) {
    if (final_pass) {
        hipLaunchKernelGGL(k_tr_pixel_iterate<true>, tree_grid2d(g), kTreeBlock, 0, st, g, t, s, in, X, NX, Y, var_ll,
                           valid, health);
        hipLaunchKernelGGL((k_tr_node<false, true>), dim3(t.nblocks), dim3(kTreeThreads), 0, st, g, t, s, X, NX, NY,
                           health);
    } else {
        hipLaunchKernelGGL(k_tr_pixel_iterate<false>, tree_grid2d(g), kTreeBlock, 0, st, g, t, s, in, X, NX, Y,
                           var_ll, valid, health);
        hipLaunchKernelGGL((k_tr_node<false, false>), dim3(t.nblocks), dim3(kTreeThreads), 0, st, g, t, s, X, NX, NY,
                           health);
    }
    return hipGetLastError();
}

hipError_t launch_tree_clear_nodes(const TreeGeo& t, float* NX, hipStream_t st) {
    const long n = (long)TN_PLANES * t.nplane;
    hipLaunchKernelGGL(k_tr_clear, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, NX, n);
    return hipGetLastError();
}

hipError_t launch_tree_pack_pixels(const Geo& g, float* X, float* dense, int to_dense, hipStream_t st) {
    const dim3 b(64, 1), gr((g.W + 63) / 64, g.H);
    hipLaunchKernelGGL(k_tr_pack_pixels, gr, b, 0, st, g, X, dense, to_dense);
    return hipGetLastError();
}

}  // namespace pv
