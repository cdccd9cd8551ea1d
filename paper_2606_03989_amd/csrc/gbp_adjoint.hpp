// Reverse-mode building blocks of the per-pixel GBP iteration (PixVOD,
// arXiv 2606.03989), FP64 in registers.
//
// Each function is the hand-derived vector-Jacobian product of one forward
// block of gbp_device.hpp: given the cotangents of the block's outputs (the
// derivative of a scalar loss with respect to each output number) it adds the
// cotangents of the block's inputs. Conventions:
//   * a packed symmetric matrix (upper storage) is a list of independent
//     numbers; its cotangent holds dLoss/d(stored entry), so an off-diagonal
//     cotangent collects both positions the entry stands for;
//   * a pose cotangent is kept either against the tangent vector tau itself
//     or against a right perturbation eps of Exp(tau), T -> T Exp(eps), and
//     the two meet through the right Jacobian: tau_bar += Jr(tau)^T eps_bar;
//   * rounding to the FP32 storage precision is differentiated as the
//     identity, comparisons (valid warp window, Huber branch, bilinear cell)
//     as constants: the result is the derivative of the smooth piece the
//     iteration is on.
#pragma once

#include "gbp_device.hpp"

namespace pv {

// ---------------------------------------------------------------------------
// SE(3) Jacobians, tangent ordering [theta; rho] (Eq. exp_err)
//
// Left Jacobian Jl(xi) = [[V, 0], [Q, V]] with V = I + B W + C W^2 (the
// matrix that maps rho to the translation of Exp), Q(theta, rho) its
// rotation-translation coupling, and Jr(xi) = Jl(-xi). Only products of their
// transposes (and inverse transposes) with vectors are needed:
//   Jl^T [a; b]    = [V^T a + Q^T b; V^T b]
//   Jl^-T [a; b]   = [V^-T (a - Q^T V^-T b); V^-T b]
// with V^T = I - B W + C W^2, V^-T = I + W/2 + D W^2 and
//   Q = P/2 + C (WP + PW + WPW) + c2 (W^2 P + P W^2 - 3 WPW) + c3 (WPW^2 + W^2 PW),
// W = [theta]x, P = [rho]x, B = (1 - cos)/th^2, C = (th - sin)/th^3,
// D = (1 - th sin / (2 (1 - cos)))/th^2, c2 = (th^2 + 2 cos - 2)/(2 th^4),
// c3 = (2 th - 3 sin + th cos)/(2 th^5).

struct LieCoef {
    double B, C, D, c2, c3;
};

__device__ inline LieCoef lie_coef(double th2) {
    LieCoef k;
    if (th2 < 1e-2) {
        const double t4 = th2 * th2, t6 = t4 * th2, t8 = t4 * t4;
        k.B = 0.5 - th2 * (1.0 / 24.0) + t4 * (1.0 / 720.0) - t6 * (1.0 / 40320.0) + t8 * (1.0 / 3628800.0);
        k.C = 1.0 / 6.0 - th2 * (1.0 / 120.0) + t4 * (1.0 / 5040.0) - t6 * (1.0 / 362880.0) + t8 * (1.0 / 39916800.0);
        k.D = 1.0 / 12.0 + th2 * (1.0 / 720.0) + t4 * (1.0 / 30240.0) + t6 * (1.0 / 1209600.0) +
              t8 * (1.0 / 47900160.0);
        k.c2 = 1.0 / 24.0 - th2 * (1.0 / 720.0) + t4 * (1.0 / 40320.0) - t6 * (1.0 / 3628800.0) +
               t8 * (1.0 / 479001600.0);
        k.c3 = 1.0 / 120.0 - th2 * (1.0 / 2520.0) + t4 * (1.0 / 120960.0) - t6 * (1.0 / 9979200.0) +
               t8 * (1.0 / 1245404160.0);
    } else {
        const double th = sqrt(th2);
        double s, c;
        sincos(th, &s, &c);
        const double sh = sin(0.5 * th);
        const double omc = 2.0 * sh * sh;  // 1 - cos
        k.B = omc / th2;
        k.C = (th - s) / (th2 * th);
        k.D = (1.0 - th * s / (2.0 * omc)) / th2;
        k.c2 = (th2 - 2.0 * omc) / (2.0 * th2 * th2);
        k.c3 = (2.0 * th - 3.0 * s + th * c) / (2.0 * th2 * th2 * th);
    }
    return k;
}

// o = x + a (w x x) + b (w x (w x x))
__device__ inline void rodrigues_apply(const double w[3], double a, double b, const double x[3], double o[3]) {
    double u1[3], u2[3];
    skew_mul(w, x, u1);
    skew_mul(w, u1, u2);
#pragma unroll
    for (int k = 0; k < 3; ++k) o[k] = x[k] + a * u1[k] + b * u2[k];
}

// o = Q(w, p)^T x
__device__ inline void coupling_T_apply(const double w[3], const double p[3], const LieCoef& k, const double x[3],
                                        double o[3]) {
    double u1[3], u2[3], px[3], pw[3], pw2[3], wp[3], w2p[3], wpw[3], w2pw[3], wpw2[3];
    skew_mul(w, x, u1);    // W x
    skew_mul(w, u1, u2);   // W^2 x
    skew_mul(p, x, px);    // P x
    skew_mul(p, u1, pw);   // P W x
    skew_mul(p, u2, pw2);  // P W^2 x
    skew_mul(w, px, wp);   // W P x
    skew_mul(w, wp, w2p);  // W^2 P x
    skew_mul(w, pw, wpw);  // W P W x
    skew_mul(w, wpw, w2pw);
    skew_mul(w, pw2, wpw2);
    // (skew products transpose with reversed order and a sign per factor)
#pragma unroll
    for (int i = 0; i < 3; ++i)
        o[i] = -0.5 * px[i] + k.C * (pw[i] + wp[i] - wpw[i]) + k.c2 * (3.0 * wpw[i] - pw2[i] - w2p[i]) +
               k.c3 * (w2pw[i] + wpw2[i]);
}

// o = Jl(xi)^T x  (sgn = +1) or Jr(xi)^T x = Jl(-xi)^T x (sgn = -1)
__device__ inline void jac_T_apply(const double xi[6], double sgn, const double x[6], double o[6]) {
    const double w[3] = {sgn * xi[0], sgn * xi[1], sgn * xi[2]};
    const double p[3] = {sgn * xi[3], sgn * xi[4], sgn * xi[5]};
    const LieCoef k = lie_coef(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    double a[3], b[3], qb[3];
    rodrigues_apply(w, -k.B, k.C, x, a);
    rodrigues_apply(w, -k.B, k.C, x + 3, b);
    coupling_T_apply(w, p, k, x + 3, qb);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        o[i] = a[i] + qb[i];
        o[3 + i] = b[i];
    }
}

// o = Jl(xi)^-T x  (sgn = +1) or Jr(xi)^-T x (sgn = -1)
__device__ inline void jac_invT_apply(const double xi[6], double sgn, const double x[6], double o[6]) {
    const double w[3] = {sgn * xi[0], sgn * xi[1], sgn * xi[2]};
    const double p[3] = {sgn * xi[3], sgn * xi[4], sgn * xi[5]};
    const LieCoef k = lie_coef(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    double vb[3], qv[3], a[3];
    rodrigues_apply(w, 0.5, k.D, x + 3, vb);  // V^-T b
    coupling_T_apply(w, p, k, vb, qv);
#pragma unroll
    for (int i = 0; i < 3; ++i) a[i] = x[i] - qv[i];
    double top[3];
    rodrigues_apply(w, 0.5, k.D, a, top);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        o[i] = top[i];
        o[3 + i] = vb[i];
    }
}

// ---------------------------------------------------------------------------
// packed symmetric helpers

// cotangent of the packed entries of S read as a full matrix in (S a) . b-type
// products: out[s(r,c)] += f (a_r b_c + a_c b_r) for r < c, f a_r b_r for r = c
__device__ inline void sym_outer_acc6(double out[21], const double a[6], const double b[6], double f) {
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = r; c < 6; ++c)
            out[s6(r, c)] += (r == c) ? f * a[r] * b[r] : f * (a[r] * b[c] + a[c] * b[r]);
}

__device__ inline void sym_outer_acc7(double out[28], const double a[7], const double b[7], double f) {
#pragma unroll
    for (int r = 0; r < 7; ++r)
#pragma unroll
        for (int c = r; c < 7; ++c)
            out[s7(r, c)] += (r == c) ? f * a[r] * b[r] : f * (a[r] * b[c] + a[c] * b[r]);
}

// y = S x for a packed symmetric 6x6 S
__device__ inline void sym_mv6(const double S[21], const double x[6], double y[6]) {
#pragma unroll
    for (int r = 0; r < 6; ++r) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < 6; ++c) s += S[s6(r, c)] * x[c];
        y[r] = s;
    }
}

// ---------------------------------------------------------------------------
// unary factors (photometric + prior), reverse of unary_factors
//
// Given the cotangents (Lb, eb) of the unary information (L, eta) of pixel
// (u, v) at its linearisation point, adds:
//   eps_bar  cotangent of a right perturbation of Exp(tau) (photometric part,
//            and the prior when its mean is not the identity),
//   tau_bar  cotangent of tau itself (prior with identity mean),
//   ell_bar  log-depth,
//   sig_bar  the pixel's sigma_D (map entry), k_bar the Huber threshold.
__device__ inline void unary_adjoint(const Geo& g, const Strengths& s, const Inputs& in, int u, int v,
                                     const double tau[6], const double R[9], const double t[3], double ell,
                                     const double Lb[28], const double eb[7], double eps_bar[6],
                                     double tau_bar[6], double& ell_bar, double& sig_bar, double& k_bar) {
    // --- photometric (Eq. distrb_photo, warp Eq. warp)
    const double q0 = ((double)u - g.cx) / g.fx, q1 = ((double)v - g.cy) / g.fy;
    const double qt[3] = {q0, q1, 1.0};
    const double rho = exp(-ell);
    const double a0 = R[0] * q0 + R[1] * q1 + R[2] + rho * t[0];
    const double a1 = R[3] * q0 + R[4] * q1 + R[5] + rho * t[1];
    const double a2 = R[6] * q0 + R[7] * q1 + R[8] + rho * t[2];
    // the warp, its validity and the samples' loads, outside the validity
    // branches (clamped addresses; an invalid warp's values are unused) so
    // that the loads are not held back by them
    const double iz = rcp_nr(a2 > 0.0 ? a2 : 1.0);
    const double wx = g.fx * a0 * iz + g.cx, wy = g.fy * a1 * iz + g.cy;
    const bool warp_ok = a2 > 0.0 && wx >= -WARP_EPS && wx <= (g.W - 1) + WARP_EPS && wy >= -WARP_EPS &&
                         wy <= (g.H - 1) + WARP_EPS;
    const double x = warp_ok ? fmin(fmax(wx, 0.0), (double)(g.W - 1)) : 0.0;
    const double y = warp_ok ? fmin(fmax(wy, 0.0), (double)(g.H - 1)) : 0.0;
    int x0 = (int)floor(x), y0 = (int)floor(y);
    x0 = x0 > g.W - 2 ? g.W - 2 : (x0 < 0 ? 0 : x0);
    y0 = y0 > g.H - 2 ? g.H - 2 : (y0 < 0 ? 0 : y0);
    const long o = (long)y0 * g.pitch + x0, o2 = o + g.pitch;
    const long pix = (long)v * g.pitch + u;
    float smp[3][4];
    {
        const float* planes[3] = {in.It, in.Gx, in.Gy};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            smp[k][0] = planes[k][o];
            smp[k][1] = planes[k][o + 1];
            smp[k][2] = planes[k][o2];
            smp[k][3] = planes[k][o2 + 1];
        }
    }
    const float Isv = in.Is[pix];
    const float sigv = s.has_sigma_map ? in.sigD[pix] : 1.0f;
    if (warp_ok) {
        {
            // bilinear samples and their in-cell derivatives
            const double fx = x - x0, fy = y - y0;
            double val[3], dx[3], dy[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double c00 = smp[k][0], c10 = smp[k][1], c01 = smp[k][2], c11 = smp[k][3];
                val[k] = (1.0 - fy) * ((1.0 - fx) * c00 + fx * c10) + fy * ((1.0 - fx) * c01 + fx * c11);
                dx[k] = (1.0 - fy) * (c10 - c00) + fy * (c11 - c01);
                dy[k] = (1.0 - fx) * (c01 - c00) + fx * (c11 - c10);
            }
            const double gx = val[1], gy = val[2];
            const double r = (double)Isv - val[0];
            const double c[3] = {-gx * g.fx * iz, -gy * g.fy * iz, (gx * g.fx * a0 + gy * g.fy * a1) * iz * iz};
            double b[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) b[k] = R[k] * c[0] + R[3 + k] * c[1] + R[6 + k] * c[2];
            double J[7];
            skew_mul(qt, b, J);  // J_theta = q x b
            J[3] = rho * b[0];
            J[4] = rho * b[1];
            J[5] = rho * b[2];
            const double ct = c[0] * t[0] + c[1] * t[1] + c[2] * t[2];
            J[6] = -rho * ct;
            const double isig = s.has_sigma_map ? rcp_nr((double)sigv) : s.inv_sigD;
            const double lamD = isig * isig;
            const double M = fabs(r) * isig;
            double kappa = 1.0;
            const bool robust = M > s.huber_k;
            double iM = 0.0;
            if (robust) {
                iM = rcp_nr(M);
                kappa = s.huber_k * iM * (2.0 - s.huber_k * iM);
            }
            const double w = kappa * lamD;

            // L += w J J^T, eta -= w J r
            double eJ = 0.0;
#pragma unroll
            for (int a = 0; a < 7; ++a) eJ += eb[a] * J[a];
            double wbar = -r * eJ;
            double Jb[7];
#pragma unroll
            for (int a = 0; a < 7; ++a) {
                double sj = 0.0;
#pragma unroll
                for (int bb = 0; bb < 7; ++bb) sj += (bb == a ? 2.0 : 1.0) * Lb[s7(a, bb)] * J[bb];
                Jb[a] = w * (sj - r * eb[a]);
#pragma unroll
                for (int bb = a; bb < 7; ++bb) wbar += Lb[s7(a, bb)] * J[a] * J[bb];
            }
            double rbar = -w * eJ;
            // w = kappa(M, k) lamD, M = |r| / sigma
            const double kapbar = wbar * lamD;
            double isigbar = 2.0 * isig * wbar * kappa;
            if (robust) {
                const double k = s.huber_k;
                const double Mbar = kapbar * (2.0 * k * iM * iM) * (k * iM - 1.0);
                k_bar += kapbar * 2.0 * iM * (1.0 - k * iM);
                rbar += Mbar * isig * (r >= 0.0 ? 1.0 : -1.0);
                isigbar += Mbar * fabs(r);
            }
            sig_bar += -isigbar * isig * isig;
            const double Itbar = -rbar;
            // J_theta = q x b, J_rho = rho b, J6 = -rho c.t
            double bbar[3], t1[3];
            skew_mul(Jb, qt, t1);
#pragma unroll
            for (int k = 0; k < 3; ++k) bbar[k] = t1[k] + rho * Jb[3 + k];
            double rhobar = Jb[3] * b[0] + Jb[4] * b[1] + Jb[5] * b[2] - Jb[6] * ct;
            double cbar[3], tbar[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                cbar[k] = -Jb[6] * rho * t[k];
                tbar[k] = -Jb[6] * rho * c[k];
            }
            // b = R^T c under R -> R Exp(phi): db = b x phi
            double phibar[3];
            skew_mul(bbar, b, phibar);
#pragma unroll
            for (int k = 0; k < 3; ++k) cbar[k] += R[k * 3] * bbar[0] + R[k * 3 + 1] * bbar[1] + R[k * 3 + 2] * bbar[2];
            // c from (gx, gy, iz, a0, a1)
            const double gxbar = -g.fx * iz * cbar[0] + g.fx * a0 * iz * iz * cbar[2];
            const double gybar = -g.fy * iz * cbar[1] + g.fy * a1 * iz * iz * cbar[2];
            double izbar = -gx * g.fx * cbar[0] - gy * g.fy * cbar[1] + 2.0 * (gx * g.fx * a0 + gy * g.fy * a1) * iz * cbar[2];
            double abar[3] = {gx * g.fx * iz * iz * cbar[2], gy * g.fy * iz * iz * cbar[2], 0.0};
            // bilinear sample position (x, y) = clamp(warp)
            const double xbar = Itbar * dx[0] + gxbar * dx[1] + gybar * dx[2];
            const double ybar = Itbar * dy[0] + gxbar * dy[1] + gybar * dy[2];
            const double wxbar = (wx >= 0.0 && wx <= (double)(g.W - 1)) ? xbar : 0.0;
            const double wybar = (wy >= 0.0 && wy <= (double)(g.H - 1)) ? ybar : 0.0;
            abar[0] += g.fx * iz * wxbar;
            abar[1] += g.fy * iz * wybar;
            izbar += g.fx * a0 * wxbar + g.fy * a1 * wybar;
            abar[2] += -iz * iz * izbar;
            // a = R q + rho t under R -> R Exp(phi), t -> t + R nu
            rhobar += abar[0] * t[0] + abar[1] * t[1] + abar[2] * t[2];
#pragma unroll
            for (int k = 0; k < 3; ++k) tbar[k] += rho * abar[k];
            double Rta[3], t2[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) Rta[k] = R[k] * abar[0] + R[3 + k] * abar[1] + R[6 + k] * abar[2];
            skew_mul(qt, Rta, t2);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                eps_bar[k] += phibar[k] + t2[k];
                eps_bar[3 + k] += R[k] * tbar[0] + R[3 + k] * tbar[1] + R[6 + k] * tbar[2];
            }
            ell_bar += -rho * rhobar;
        }
    }

    // --- prior (Eq. prior): L_pp += lamP Jp^T Jp, eta_p -= lamP Jp^T rp,
    //     eta_6 -= lamP (ell - prior_ell), Jp = I + ad/2 + ad^2/12 at rp
    double rp[6];
    if (s.prior_is_identity) {
#pragma unroll
        for (int k = 0; k < 6; ++k) rp[k] = tau[k];
    } else {
        double Rr[9], tr[3];
        se3_compose(s.prior_R, s.prior_t, R, t, Rr, tr);
        se3_log(Rr, tr, rp);
    }
    // J = [[S, 0], [Q, S]] as in unary_factors: S = I + W/2 + W^2/12,
    // Q = P/2 + (PW + WP)/12 with W = [w]x, P = [q]x, rp = (w, q)
    const double w0 = rp[0], w1 = rp[1], w2 = rp[2], p0 = rp[3], p1 = rp[4], p2 = rp[5];
    const double Wm[9] = {0.0, -w2, w1, w2, 0.0, -w0, -w1, w0, 0.0};
    const double Pm[9] = {0.0, -p2, p1, p2, 0.0, -p0, -p1, p0, 0.0};
    double S[9], Q[9];
    {
        const double w[3] = {w0, w1, w2}, q[3] = {p0, p1, p2};
        const double th2 = w0 * w0 + w1 * w1 + w2 * w2;
        const double wq = w0 * p0 + w1 * p1 + w2 * p2;
        constexpr double c12 = 1.0 / 12.0;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double I = (r == c) ? 1.0 : 0.0;
                S[r * 3 + c] = I + 0.5 * Wm[r * 3 + c] + (w[r] * w[c] - I * th2) * c12;
                Q[r * 3 + c] = 0.5 * Pm[r * 3 + c] + (w[r] * q[c] + q[r] * w[c] - 2.0 * I * wq) * c12;
            }
    }
    const double lamP = s.lamP;
    // eta_p -= lamP J^T rp: rp_bar = -lamP J eb_p
    double rpb[6];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double e0 = 0.0, e1 = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            e0 += S[k * 3 + a] * eb[a];
            e1 += Q[k * 3 + a] * eb[a] + S[k * 3 + a] * eb[3 + a];
        }
        rpb[k] = -lamP * e0;
        rpb[3 + k] = -lamP * e1;
    }
    // L_pp += lamP J^T J: J_bar = lamP (J M - rp eb_p^T), M the pose block of
    // Lb with a doubled diagonal; S enters both diagonal blocks, Q the lower
    // left one (the upper right block of J is identically zero)
    double Sb[9], Qb[9];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double tl = 0.0, bl = 0.0, br = 0.0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double m_jc = (j == c ? 2.0 : 1.0) * Lb[s7(j, c)];
                const double m_j3c = Lb[s7(j, 3 + c)];
                const double m_3jc = Lb[s7(3 + j, c)];
                const double m_3j3c = (j == c ? 2.0 : 1.0) * Lb[s7(3 + j, 3 + c)];
                tl += S[k * 3 + j] * m_jc;
                bl += Q[k * 3 + j] * m_jc + S[k * 3 + j] * m_3jc;
                br += Q[k * 3 + j] * m_j3c + S[k * 3 + j] * m_3j3c;
            }
            Sb[k * 3 + c] = lamP * ((tl - rp[k] * eb[c]) + (br - rp[3 + k] * eb[3 + c]));
            Qb[k * 3 + c] = lamP * (bl - rp[3 + k] * eb[c]);
        }
    // through S(w) and Q(w, q), with W^T = -W and P^T = -P:
    //   W_bar = Sb/2 - (Sb W + W Sb)/12 - (P Qb + Qb P)/12,
    //   P_bar = Qb/2 - (Qb W + W Qb)/12
    {
        double Wb[9], Pb[9];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double sw = 0.0, pq = 0.0, qw = 0.0;
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    sw += Sb[r * 3 + j] * Wm[j * 3 + c] + Wm[r * 3 + j] * Sb[j * 3 + c];
                    pq += Pm[r * 3 + j] * Qb[j * 3 + c] + Qb[r * 3 + j] * Pm[j * 3 + c];
                    qw += Qb[r * 3 + j] * Wm[j * 3 + c] + Wm[r * 3 + j] * Qb[j * 3 + c];
                }
                Wb[r * 3 + c] = 0.5 * Sb[r * 3 + c] - (sw + pq) * (1.0 / 12.0);
                Pb[r * 3 + c] = 0.5 * Qb[r * 3 + c] - qw * (1.0 / 12.0);
            }
        rpb[0] += Wb[7] - Wb[5];
        rpb[1] += Wb[2] - Wb[6];
        rpb[2] += Wb[3] - Wb[1];
        rpb[3] += Pb[7] - Pb[5];
        rpb[4] += Pb[2] - Pb[6];
        rpb[5] += Pb[3] - Pb[1];
    }
    ell_bar += -lamP * eb[6];
    // both targets are updated unconditionally (one of the two increments is
    // zero): stores into tau_bar or eps_bar chosen by a branch would be merged
    // into stores through a selected pointer, which keeps both arrays in
    // scratch memory
    double dtau[6], deps[6];
    if (s.prior_is_identity) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            dtau[k] = rpb[k];
            deps[k] = 0.0;
        }
    } else {
        // rp = Log(Exp(prior)^-1 Exp(tau)): d rp = Jr(rp)^-1 eps
        jac_invT_apply(rp, -1.0, rpb, deps);
#pragma unroll
        for (int k = 0; k < 6; ++k) dtau[k] = 0.0;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        tau_bar[k] += dtau[k];
        eps_bar[k] += deps[k];
    }
}

// ---------------------------------------------------------------------------
// marginals of the belief (pose_marginal, depth_marginal), reverse
//
// Cotangents (Pb, pb) of the pose marginal and (Db, dvb) of the depth
// marginal of the belief (L, eta) are added to (Lb, eb).
__device__ inline void marginals_adjoint(const double L[28], const double eta[7], const double Pb[21],
                                         const double pb[6], double Db, double dvb, double Lb[28], double eb[7]) {
    const double i66 = rcp_nr(L[s7(6, 6)]);
    double b[6], bb[6];
#pragma unroll
    for (int r = 0; r < 6; ++r) {
        b[r] = L[s7(r, 6)];
        bb[r] = 0.0;
    }
    double L66b = 0.0;
    // P = L_pp - b b^T / L66, p = eta_p - b eta6 / L66
#pragma unroll
    for (int r = 0; r < 6; ++r) {
#pragma unroll
        for (int c = r; c < 6; ++c) {
            const double x = Pb[s6(r, c)];
            Lb[s7(r, c)] += x;
            if (r == c) {
                bb[r] -= 2.0 * x * b[r] * i66;
            } else {
                bb[r] -= x * b[c] * i66;
                bb[c] -= x * b[r] * i66;
            }
            L66b += x * b[r] * b[c] * i66 * i66;
        }
        eb[r] += pb[r];
        bb[r] -= pb[r] * eta[6] * i66;
        eb[6] -= pb[r] * b[r] * i66;
        L66b += pb[r] * b[r] * eta[6] * i66 * i66;
    }
    // D = L66 - b^T A^-1 b, dv = eta6 - b^T A^-1 eta_p with A = L_pp
    double A[21], idg[6], y[6], z[6];
#pragma unroll
    for (int r = 0; r < 6; ++r) {
#pragma unroll
        for (int c = r; c < 6; ++c) A[s6(r, c)] = L[s7(r, c)];
        y[r] = b[r];
        z[r] = eta[r];
    }
    chol6(A, idg);
    chol6_solve(A, idg, y);
    chol6_solve(A, idg, z);
    L66b += Db;
    eb[6] += dvb;
#pragma unroll
    for (int r = 0; r < 6; ++r) {
        bb[r] -= 2.0 * Db * y[r] + dvb * z[r];
        eb[r] -= dvb * y[r];
#pragma unroll
        for (int c = r; c < 6; ++c)
            Lb[s7(r, c)] += (r == c) ? (Db * y[r] * y[r] + dvb * y[r] * z[r])
                                     : (2.0 * Db * y[r] * y[c] + dvb * (y[r] * z[c] + y[c] * z[r]));
    }
#pragma unroll
    for (int r = 0; r < 6; ++r) Lb[s7(r, 6)] += bb[r];
    Lb[s7(6, 6)] += L66b;
}

// ---------------------------------------------------------------------------
// partial messages, reverse of identity_partial and normal_partial

// Identity factor: A = V + lamR I, Lp = lamR I - lamR^2 A^-1, h = lamR A^-1 v.
// V is the sender's variable-to-factor pose information before the shift;
// (Lpb, hb) -> (Vb, vb) (overwritten).
__device__ inline void identity_partial_adjoint(double lamR, const double V[21], const double v[6],
                                                const double Lpb[21], const double hb[6], double Vb[21],
                                                double vb[6]) {
    double A[21], Ai[21];
#pragma unroll
    for (int k = 0; k < 21; ++k) A[k] = V[k];
#pragma unroll
    for (int k = 0; k < 6; ++k) A[s6(k, k)] += lamR;
    sweep6_neg_inverse(A);
#pragma unroll
    for (int k = 0; k < 21; ++k) Ai[k] = -A[k];
    // cotangent of the packed inverse
    double Aib[21];
    const double l2 = lamR * lamR;
#pragma unroll
    for (int k = 0; k < 21; ++k) Aib[k] = -l2 * Lpb[k];
    sym_outer_acc6(Aib, hb, v, lamR);
    sym_mv6(Ai, hb, vb);
#pragma unroll
    for (int k = 0; k < 6; ++k) vb[k] *= lamR;
    // d(A^-1) = -A^-1 dA A^-1: with S the half-weight matrix of Aib,
    // G = A^-1 S A^-1 and Vb = -(diag G, 2 G off the diagonal)
    double T[36];
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            double x = 0.0;
#pragma unroll
            for (int k = 0; k < 6; ++k) x += (r == k ? 1.0 : 0.5) * Aib[s6(r, k)] * Ai[s6(k, c)];
            T[r * 6 + c] = x;
        }
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = r; c < 6; ++c) {
            double x = 0.0;
#pragma unroll
            for (int k = 0; k < 6; ++k) x += Ai[s6(r, k)] * T[k * 6 + c];
            Vb[s6(r, c)] = (r == c) ? -x : -2.0 * x;
        }
}

// Normal factor: lp = lamN ls / (lamN + ls), h = lamN vs / (lamN + ls);
// (lpb, hb) -> (lsb, vsb, lamNb)
__device__ inline void normal_partial_adjoint(double lamN, double ls, double vs, double lpb, double hb, double& lsb,
                                              double& vsb, double& lamNb) {
    const double id = rcp_nr(lamN + ls), id2 = id * id;
    lsb = (lpb * lamN * lamN - hb * lamN * vs) * id2;
    vsb = hb * lamN * id;
    lamNb = (lpb * ls * ls + hb * vs * ls) * id2;
}

}  // namespace pv
