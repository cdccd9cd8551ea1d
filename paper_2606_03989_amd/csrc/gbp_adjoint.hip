// HIP kernels of the reverse sweep through unrolled GBP iterations (PixVOD,
// arXiv 2606.03989) for gfx950: one lane per pixel, FP32 cotangent planes (the
// state's cotangent in the state layout and the intermediate ones: Mb, Ub,
// Eb), FP64 algebra in registers.
//
// Reverse of one canonical iteration X -> X' (linearise + marginals, messages,
// update + relinearise + transport; Sec. 3.4 and Sec. 4.1), given the
// cotangent Xb' of X':
//   forward recompute  the fused passes that recompute X also keep its belief
//                      and marginals (64 planes), the information of its new
//                      messages (88 FP32 planes: exact, they are the FP32
//                      partials' values) and the belief of the update (35);
//   k_adj_update       reverse of the update at every pixel: cotangents of its
//                      four new messages (Mb, 116 planes) and of its unary
//                      information and point (Ub, 42 planes);
//   k_adj_edges        one lane per (pixel, direction): the pixel as the sender
//                      of its outgoing message and the receiver of its incoming
//                      one on that edge: cotangents of its marginals, of the
//                      residual's pose and log-depth arguments, and of the
//                      stored message the sender subtracted (gathered from the
//                      neighbours' Mb, no atomics; the four directions of a
//                      pixel are summed with lane shuffles);
//   k_adj_belief       reverse of the marginals and of the unary factors:
//                      completes Xb (cotangent of X) and accumulates the
//                      per-pixel parameter gradients. Every stored message
//                      enters the belief the same way, so its cotangent
//                      there is one 29-value slot-common part Cb per pixel;
//                      it is kept apart from the slot-specific part in Xb
//                      and added by the next reader (k_adj_update), instead
//                      of a read-modify-write of all four slots.
#include "gbp_adjoint.h"
#include "gbp_adjoint.hpp"

namespace pv {

constexpr int MSG_STRIDE = 29;   // per direction: eta 6, Lambda 21, normal eta, normal lambda
constexpr int UB_TAU = 35;       // Ub: L_bar 28, eta_bar 7, tau_bar 6, ell_bar 1
constexpr int UB_ELL = 41;
constexpr int EB_P = 0;          // Eb: P_bar 21, p_bar 6, D_bar, dv_bar, eps_bar 6, ell_bar
constexpr int EB_PV = 21;
constexpr int EB_D = 27;
constexpr int EB_DV = 28;
constexpr int EB_EPS = 29;
constexpr int EB_ELL = 35;

__device__ inline bool pixel_2d(const Geo& g, int& u, int& v) {
    u = blockIdx.x * blockDim.x + threadIdx.x;
    v = blockIdx.y * blockDim.y + threadIdx.y;
    return u < g.W && v < g.H;
}

// reverse of the update (k_pf_update): belief from the unary and the new
// messages, mean m, relinearisation, transport of the messages
__global__ __launch_bounds__(256, 2) void k_adj_update(Geo g, Strengths s, Inputs in, const float* __restrict__ X,
                                                    const float* __restrict__ M, const double* __restrict__ bel,
                                                    const float* __restrict__ Xb, const float* __restrict__ Cb,
                                                    float* __restrict__ Mb, float* __restrict__ Ub) {
    int u, v;
    if (!pixel_2d(g, u, v)) return;
    const long p = pix_of(g, u, v);
    const long pl = g.plane;
    double tau[6], ell, R[9], t[3], L[28], eta[7];
    load_point(X, g, p, tau, ell);
    se3_exp(tau, R, t);
    // the belief of the update (unary + new messages), kept by the recompute
#pragma unroll
    for (int k = 0; k < 28; ++k) L[k] = bel[(long)k * pl + p];
#pragma unroll
    for (int k = 0; k < 7; ++k) eta[k] = bel[(long)(28 + k) * pl + p];
    double idg[7], m[7];
    chol7(L, idg);
#pragma unroll
    for (int k = 0; k < 7; ++k) m[k] = eta[k];
    chol7_solve(L, idg, m);
    double Rm[9], tm[3], R1[9], t1[3], tn[6];
    se3_exp(m, Rm, tm);
    se3_compose(R, t, Rm, tm, R1, t1);
    se3_log(R1, t1, tn);

    // transport eta' = eta - Lambda m_p, ne' = ne - nl m6: contribution to m_bar
    double mb[7] = {0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        int nu, nv;
        if (!neighbour(g, u, v, d, nu, nv)) continue;
        const float* md = M + (long)d * LAM_STRIDE * pl + p;
        const float* xb = Xb + (long)(P_MID + d * MID_STRIDE) * pl + p;
        const float* cb = Cb + p;
        double Lam[21], eb[6], y[6];
#pragma unroll
        for (int k = 0; k < 21; ++k) Lam[k] = (double)md[k * pl];
#pragma unroll
        for (int a = 0; a < 6; ++a) eb[a] = (double)xb[a * pl] + (double)cb[a * pl];
        sym_mv6(Lam, eb, y);
#pragma unroll
        for (int a = 0; a < 6; ++a) mb[a] -= y[a];
        mb[6] -= (double)md[21 * pl] * ((double)Xb[(long)(P_MN + 2 * d) * pl + p] + (double)cb[27 * pl]);
    }
    // relinearisation tau' = Log(Exp(tau) Exp(m_p)):
    //   d tau' = Jl(tau')^-1 Jl(tau) d tau + Jr(tau')^-1 Jr(m_p) d m_p
    double tnb[6], a6[6], taub[6], b6[6], mpb[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) tnb[k] = (double)Xb[(long)(P_TAU + k) * pl + p];
    const double ellnb = (double)Xb[(long)P_ELL * pl + p];
    jac_invT_apply(tn, 1.0, tnb, a6);
    jac_T_apply(tau, 1.0, a6, taub);
    jac_invT_apply(tn, -1.0, tnb, b6);
    jac_T_apply(m, -1.0, b6, mpb);
#pragma unroll
    for (int k = 0; k < 6; ++k) mb[k] += mpb[k];
    mb[6] += ellnb;
    // m = B^-1 beta
    double betab[7], Bb[28];
#pragma unroll
    for (int k = 0; k < 7; ++k) betab[k] = mb[k];
    chol7_solve(L, idg, betab);
#pragma unroll
    for (int k = 0; k < 28; ++k) Bb[k] = 0.0;
    sym_outer_acc7(Bb, betab, m, -1.0);

    // cotangents of the four new messages: transport + belief
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        float* o = Mb + (long)d * MSG_STRIDE * pl + p;
        int nu, nv;
        if (!neighbour(g, u, v, d, nu, nv)) {
#pragma unroll
            for (int k = 0; k < MSG_STRIDE; ++k) o[k * pl] = 0.0f;
            continue;
        }
        const float* xb = Xb + (long)(P_MID + d * MID_STRIDE) * pl + p;
        const float* cb = Cb + p;
        double eb[6];
#pragma unroll
        for (int a = 0; a < 6; ++a) {
            eb[a] = (double)xb[a * pl] + (double)cb[a * pl];
            o[a * pl] = (float)(eb[a] + betab[a]);
        }
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
            for (int c = r; c < 6; ++c) {
                const double tr = (r == c) ? eb[r] * m[r] : eb[r] * m[c] + eb[c] * m[r];
                o[(6 + s6(r, c)) * pl] =
                    (float)(((double)xb[(6 + s6(r, c)) * pl] + (double)cb[(6 + s6(r, c)) * pl]) - tr + Bb[s7(r, c)]);
            }
        const double neb = (double)Xb[(long)(P_MN + 2 * d) * pl + p] + (double)cb[27 * pl];
        const double nlb = (double)Xb[(long)(P_MN + 2 * d + 1) * pl + p] + (double)cb[28 * pl];
        o[27 * pl] = (float)(neb + betab[6]);
        o[28 * pl] = (float)(nlb - neb * m[6] + Bb[s7(6, 6)]);
    }
    float* ub = Ub + p;
#pragma unroll
    for (int k = 0; k < 28; ++k) ub[k * pl] = (float)Bb[k];
#pragma unroll
    for (int k = 0; k < 7; ++k) ub[(28 + k) * pl] = (float)betab[k];
#pragma unroll
    for (int k = 0; k < 6; ++k) ub[(UB_TAU + k) * pl] = (float)taub[k];
    ub[UB_ELL * pl] = (float)ellnb;
}

// reverse of the message step (k_pf_messages), one lane per (pixel j,
// direction d): j as the receiver of the message in its slot d (residual
// cotangent) and as the sender of the message into its neighbour in direction
// d (its marginals and the stored message it subtracted). The four lanes of a
// pixel are adjacent; their contributions to j's marginal and perturbation
// cotangents are summed with lane shuffles and written by the d = 0 lane.
// Writes the sender part of j's slot-d cotangent to Xbo.
__global__ __launch_bounds__(256, 2) void k_adj_edges(Geo g, Strengths s, Inputs in, const float* __restrict__ X,
                                                   const double* __restrict__ marg, const float* __restrict__ M,
                                                   const float* __restrict__ Mb, float* __restrict__ Xbo,
                                                   float* __restrict__ Eb, double* __restrict__ gN) {
    const int d = threadIdx.x & 3;
    const int u = blockIdx.x * (blockDim.x >> 2) + (threadIdx.x >> 2);
    const int v = blockIdx.y;
    // every lane of a pixel takes part in the shuffles; lanes past the row end
    // work on a clamped copy and write nothing
    const bool inside = u < g.W;
    const int uc = inside ? u : g.W - 1;
    const long pj = pix_of(g, uc, v);
    const long pl = g.plane;
    double acc[37];   // P_bar 21, p_bar 6, D_bar, dv_bar, eps_bar 6, ell_bar, lamN_bar
#pragma unroll
    for (int k = 0; k < 37; ++k) acc[k] = 0.0;
    float* xo = Xbo + (long)(P_MID + d * MID_STRIDE) * pl + pj;
    float* xn = Xbo + (long)(P_MN + 2 * d) * pl + pj;
    int nu, nv;
    if (neighbour(g, uc, v, d, nu, nv)) {
        double tau[6], ell, R[9], t[3];
        load_point(X, g, pj, tau, ell);
        se3_exp(tau, R, t);
        const long pi = pix_of(g, nu, nv);
        const int o = opposite(d);
        const float* Mj = M + (long)d * LAM_STRIDE * pl + pj;
        const float* Mbj = Mb + (long)d * MSG_STRIDE * pl + pj;
        const float* Mi = M + (long)o * LAM_STRIDE * pl + pi;
        const float* Mbi = Mb + (long)o * MSG_STRIDE * pl + pi;
        // residual of the message into j from i, r = Log(Exp(tau_i)^-1 Exp(tau_j));
        // the message into i from j uses -r
        double ti[6], elli, Ri[9], tri[3], r[6];
        load_point(X, g, pi, ti, elli);
        se3_exp(ti, Ri, tri);
        se3_between(Ri, tri, R, t, r);
        // eta_new = h - Lp r on both sides: receiver r_bar = -Lp_j eb_j, sender
        // r_bar = -Lp_i eb_i with d(-r) = -d r, so eps_j += Jr(r)^-T (Lp_i eb_i - Lp_j eb_j)
        double rb[6];
        {
            double Lam[21], e[6], y1[6], y2[6];
#pragma unroll
            for (int k = 0; k < 21; ++k) Lam[k] = (double)Mj[k * pl];
#pragma unroll
            for (int a = 0; a < 6; ++a) e[a] = (double)Mbj[a * pl];
            sym_mv6(Lam, e, y1);
#pragma unroll
            for (int k = 0; k < 21; ++k) Lam[k] = (double)Mi[k * pl];
#pragma unroll
            for (int a = 0; a < 6; ++a) e[a] = (double)Mbi[a * pl];
            sym_mv6(Lam, e, y2);
#pragma unroll
            for (int a = 0; a < 6; ++a) rb[a] = y2[a] - y1[a];
        }
        jac_invT_apply(r, -1.0, rb, acc + 29);

        // sender: the partial of the message into i from j's variable-to-factor
        // message (j's marginal minus j's stored message from this factor)
        double V[21], vv[6], Lpb[21], hb[6], Vb[21], vb[6];
#pragma unroll
        for (int k = 0; k < 21; ++k) {
            V[k] = marg[(long)k * pl + pj] - (double)X[(long)(P_MID + d * MID_STRIDE + 6 + k) * pl + pj];
            Lpb[k] = (double)Mbi[(6 + k) * pl];
        }
#pragma unroll
        for (int a = 0; a < 6; ++a) {
            vv[a] = marg[(long)(21 + a) * pl + pj] - (double)X[(long)(P_MID + d * MID_STRIDE + a) * pl + pj];
            hb[a] = (double)Mbi[a * pl];
        }
        // eta_i = h - Lp (-r): Lp_bar += sym(hb r^T)
        sym_outer_acc6(Lpb, hb, r, 1.0);
        identity_partial_adjoint(s.lamR, V, vv, Lpb, hb, Vb, vb);
#pragma unroll
        for (int k = 0; k < 21; ++k) acc[k] = Vb[k];
#pragma unroll
        for (int a = 0; a < 6; ++a) acc[21 + a] = vb[a];
        if (inside) {
#pragma unroll
            for (int k = 0; k < 21; ++k) xo[(6 + k) * pl] = (float)(-Vb[k]);
#pragma unroll
            for (int a = 0; a < 6; ++a) xo[a * pl] = (float)(-vb[a]);
        }

        // normal-integration factor of the edge
        double nsb = 0.0, nlsb = 0.0;
        double rn_j, rn_i;
        if (s.lamN > 0.0 && normal_residual(g, in, pj, pi, d, ell, elli, rn_j)) {
            normal_residual(g, in, pi, pj, o, elli, ell, rn_i);
            // ne_new = h - lp rn: receiver j and sender j (rn_i depends on ell_j with -1)
            acc[35] = -(double)Mj[21 * pl] * (double)Mbj[27 * pl] + (double)Mi[21 * pl] * (double)Mbi[27 * pl];
            const double neb = (double)Mbi[27 * pl], nlb = (double)Mbi[28 * pl];
            const double ls = marg[27L * pl + pj] - (double)X[(long)(P_MN + 2 * d + 1) * pl + pj];
            const double vs = marg[28L * pl + pj] - (double)X[(long)(P_MN + 2 * d) * pl + pj];
            double lsb, vsb, lnb;
            normal_partial_adjoint(s.lamN, ls, vs, nlb - neb * rn_i, neb, lsb, vsb, lnb);
            acc[27] = lsb;
            acc[28] = vsb;
            acc[36] = lnb;
            nsb = -vsb;
            nlsb = -lsb;
        }
        if (inside) {
            xn[0] = (float)nsb;
            xn[pl] = (float)nlsb;
        }
    } else if (inside) {
        for (int k = 0; k < MID_STRIDE; ++k) xo[k * pl] = 0.0f;
        xn[0] = xn[pl] = 0.0f;
    }
    // sum over the four directions of the pixel (lanes 4q .. 4q + 3)
#pragma unroll
    for (int k = 0; k < 37; ++k) {
        acc[k] += __shfl_xor(acc[k], 1, 4);
        acc[k] += __shfl_xor(acc[k], 2, 4);
    }
    if (d == 0 && inside) {
        float* eb = Eb + pj;
#pragma unroll
        for (int k = 0; k < 21; ++k) eb[(EB_P + k) * pl] = (float)acc[k];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            eb[(EB_PV + k) * pl] = (float)acc[21 + k];
            eb[(EB_EPS + k) * pl] = (float)acc[29 + k];
        }
        eb[EB_D * pl] = (float)acc[27];
        eb[EB_DV * pl] = (float)acc[28];
        eb[EB_ELL * pl] = (float)acc[35];
        gN[pj] += acc[36];
    }
}

// reverse of the marginals and of the unary factors; completes Xbo (point
// planes) and writes the slot-common part Cbo
__global__ __launch_bounds__(256) void k_adj_belief(Geo g, Strengths s, Inputs in, const float* __restrict__ X,
                                                    const double* __restrict__ marg, const float* __restrict__ Ub,
                                                    const float* __restrict__ Eb,
                                                    float* __restrict__ Xbo, float* __restrict__ Cbo,
                                                    double* __restrict__ gsig, double* __restrict__ gk) {
    int u, v;
    if (!pixel_2d(g, u, v)) return;
    const long p = pix_of(g, u, v);
    const long pl = g.plane;
    double tau[6], ell, R[9], t[3], L[28], eta[7];
    load_point(X, g, p, tau, ell);
    se3_exp(tau, R, t);
    // the belief of the marginals (unary + stored messages), kept by the recompute
#pragma unroll
    for (int k = 0; k < 28; ++k) L[k] = marg[(long)(29 + k) * pl + p];
#pragma unroll
    for (int k = 0; k < 7; ++k) eta[k] = marg[(long)(57 + k) * pl + p];
    const float* eb = Eb + p;
    double Pb[21], pb[6];
#pragma unroll
    for (int k = 0; k < 21; ++k) Pb[k] = (double)eb[(EB_P + k) * pl];
#pragma unroll
    for (int k = 0; k < 6; ++k) pb[k] = (double)eb[(EB_PV + k) * pl];
    double BbS[28], ebS[7];
#pragma unroll
    for (int k = 0; k < 28; ++k) BbS[k] = 0.0;
#pragma unroll
    for (int k = 0; k < 7; ++k) ebS[k] = 0.0;
    marginals_adjoint(L, eta, Pb, pb, (double)eb[EB_D * pl], (double)eb[EB_DV * pl], BbS, ebS);

    const float* ub = Ub + p;
    double Lb[28], etab[7], epsb[6], taub[6];
#pragma unroll
    for (int k = 0; k < 28; ++k) Lb[k] = (double)ub[k * pl] + BbS[k];
#pragma unroll
    for (int k = 0; k < 7; ++k) etab[k] = (double)ub[(28 + k) * pl] + ebS[k];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        epsb[k] = (double)eb[(EB_EPS + k) * pl];
        taub[k] = (double)ub[(UB_TAU + k) * pl];
    }
    double ellb = (double)ub[UB_ELL * pl] + (double)eb[EB_ELL * pl];
    double sigb = 0.0, kb = 0.0;
    unary_adjoint(g, s, in, u, v, tau, R, t, ell, Lb, etab, epsb, taub, ellb, sigb, kb);
    double te[6];
    jac_T_apply(tau, -1.0, epsb, te);
#pragma unroll
    for (int k = 0; k < 6; ++k) Xbo[(long)(P_TAU + k) * pl + p] = (float)(taub[k] + te[k]);
    Xbo[(long)P_ELL * pl + p] = (float)ellb;
    // every stored message enters the belief: one slot-common cotangent
    float* cb = Cbo + p;
#pragma unroll
    for (int a = 0; a < 6; ++a) cb[a * pl] = (float)ebS[a];
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = r; c < 6; ++c) cb[(6 + s6(r, c)) * pl] = (float)BbS[s7(r, c)];
    cb[27 * pl] = (float)ebS[6];
    cb[28 * pl] = (float)BbS[s7(6, 6)];
    gsig[p] += sigb;
    gk[p] += kb;
}

// cotangents of the per-frame outputs: pose mean (Eq. estimator_avg) and the
// inverse-depth map rho = exp(-ell)
__global__ void k_adj_inject(Geo g, const float* __restrict__ Xend, float* __restrict__ Xb, PoseBar xb,
                             const float* __restrict__ rhob) {
    int u, v;
    if (!pixel_2d(g, u, v)) return;
    const long p = pix_of(g, u, v);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        float* q = Xb + (long)(P_TAU + k) * g.plane + p;
        *q = (float)((double)*q + xb.v[k]);
    }
    if (rhob) {
        const double rho = exp(-(double)Xend[(long)P_ELL * g.plane + p]);
        float* q = Xb + (long)P_ELL * g.plane + p;
        *q = (float)((double)*q - rho * (double)rhob[(long)v * g.W + u]);
    }
}

// per block: sums of two FP64 planes (deterministic two-stage reduction)
constexpr int SUM_THREADS = 256;

__global__ __launch_bounds__(SUM_THREADS) void k_sum2(Geo g, const double* __restrict__ a,
                                                      const double* __restrict__ b, double* __restrict__ partial) {
    __shared__ double sh[2][SUM_THREADS];
    double s0 = 0.0, s1 = 0.0;
    const long N = (long)g.H * g.W;
    for (long i = (long)blockIdx.x * SUM_THREADS + threadIdx.x; i < N; i += (long)gridDim.x * SUM_THREADS) {
        const long p = pix_of(g, (int)(i % g.W), (int)(i / g.W));
        s0 += a[p];
        s1 += b[p];
    }
    sh[0][threadIdx.x] = s0;
    sh[1][threadIdx.x] = s1;
    __syncthreads();
    for (int w = SUM_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < 2) partial[(long)blockIdx.x * 2 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void k_sum2_final(int nblocks, const double* __restrict__ partial, double* __restrict__ result) {
    const int k = threadIdx.x;
    if (k >= 2) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += partial[(long)b * 2 + k];
    result[k] = s;
}

// FP64 plane -> dense FP32 map
__global__ void k_plane_to_dense(Geo g, const double* __restrict__ src, float* __restrict__ dst) {
    int u, v;
    if (!pixel_2d(g, u, v)) return;
    dst[(long)v * g.W + u] = (float)src[pix_of(g, u, v)];
}

// ---------------------------------------------------------------------------
// launchers

static const dim3 kAdjBlock(64, 4);
static dim3 adj_grid(const Geo& g) { return dim3((g.W + 63) / 64, (g.H + 3) / 4); }

hipError_t launch_adj_update(const Geo& g, const Strengths& s, const Inputs& in, const float* X, const float* M,
                             const double* bel, const float* Xb, const float* Cb, float* Mb, float* Ub,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_adj_update, adj_grid(g), kAdjBlock, 0, st, g, s, in, X, M, bel, Xb, Cb, Mb, Ub);
    return hipGetLastError();
}

hipError_t launch_adj_edges(const Geo& g, const Strengths& s, const Inputs& in, const float* X, const double* marg,
                            const float* M, const float* Mb, float* Xbo, float* Eb, double* gN, hipStream_t st) {
    // one lane per (pixel, direction): 64 pixels of a row per 256-lane workgroup
    hipLaunchKernelGGL(k_adj_edges, dim3((g.W + 63) / 64, g.H), dim3(256), 0, st, g, s, in, X, marg, M, Mb, Xbo, Eb,
                       gN);
    return hipGetLastError();
}

hipError_t launch_adj_belief(const Geo& g, const Strengths& s, const Inputs& in, const float* X, const double* marg,
                             const float* Ub, const float* Eb, float* Xbo, float* Cbo, double* gsig, double* gk,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_adj_belief, adj_grid(g), kAdjBlock, 0, st, g, s, in, X, marg, Ub, Eb, Xbo, Cbo, gsig, gk);
    return hipGetLastError();
}

hipError_t launch_adj_inject(const Geo& g, const float* Xend, float* Xb, const PoseBar& xb, const float* rhob,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_adj_inject, adj_grid(g), kAdjBlock, 0, st, g, Xend, Xb, xb, rhob);
    return hipGetLastError();
}

int sum2_blocks(const Geo& g) {
    const long N = (long)g.H * g.W;
    long b = (N + SUM_THREADS * 8 - 1) / (SUM_THREADS * 8);
    if (b < 1) b = 1;
    if (b > 1024) b = 1024;
    return (int)b;
}

hipError_t launch_sum2(const Geo& g, const double* a, const double* b, double* partial, double* result,
                       hipStream_t st) {
    const int nb = sum2_blocks(g);
    hipLaunchKernelGGL(k_sum2, dim3(nb), dim3(SUM_THREADS), 0, st, g, a, b, partial);
    hipLaunchKernelGGL(k_sum2_final, dim3(1), dim3(64), 0, st, nb, partial, result);
    return hipGetLastError();
}

hipError_t launch_plane_to_dense(const Geo& g, const double* src, float* dst, hipStream_t st) {
    hipLaunchKernelGGL(k_plane_to_dense, adj_grid(g), kAdjBlock, 0, st, g, src, dst);
    return hipGetLastError();
}

}  // namespace pv
