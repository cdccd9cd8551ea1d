/*
 * FP64 CPU oracle for per-pixel GBP visual odometry and depth (PixVOD).
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
 * baseline leg of the benchmark, never by the product path. Shares no code
 * with the GPU library. Plain loops, OpenMP over pixels inside each phase.
 *
 * Paper references are to arXiv 2606.03989 (PixVOD): Sec. 3.1 Eq. (photo),
 * (warp); Sec. 3.3 Eqs. (distrb_photo), (prior), (regul), (gbpni); Sec. 3.4
 * Eq. (var) and the linearised energy; Sec. 4.1 implementation details
 * (synchronous schedule, stored messages, tangent-space projection, Huber
 * covariance weighting); Sec. 4.3 (warm start between target frames);
 * App. C.2 Eqs. (exp_err), (estimator_avg).
 *
 * Readings of points the paper leaves open are listed with the design notes
 * of the repository; the ones this file depends on are restated where used.
 */
#include "pixvod_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double eta[7]; double lam[49]; } g7;

#define OR_MAX_LEVELS 30

struct or_ctx {
    or_config cfg;
    int N;
    int have_kf, have_frame;
    double *I_s, *cxt, *cyt;           /* keyframe image, normal targets */
    double *I_t, *Gx, *Gy;             /* target frame and its gradients */
    double *sigD;                      /* per-pixel photometric sigma */
    double *prior_ell;                 /* per-pixel log-depth prior mean */
    double *tau, *ell;                 /* linearisation points */
    g7 *msg, *newmsg;                  /* 8 stored f2v messages per pixel */
    g7 *unary, *belief;
    double *mean, *var_ll;
    int *valid;
    double T_w_kf[16];
    double xi_last[6];
    int have_track;
    int frames_since_kf;
    int diverged;
    /* quadtree topology: node levels 1..L above the pixels (level 0) */
    int tree, L, NT;
    int lvH[OR_MAX_LEVELS + 1], lvW[OR_MAX_LEVELS + 1];
    int lvOff[OR_MAX_LEVELS + 2];      /* first node of level l >= 1 */
    double* ntau;                      /* node linearisation points */
    g7 *pmsg, *pnewmsg;                /* per pixel: message of the edge to its parent */
    g7 *nmsg, *nnewmsg;                /* per node: slot 0 parent edge, 1 + q child edges */
    g7 *nunary, *nbelief;
};

/* ------------------------------------------------------------------------ */
/* small dense linear algebra (row-major)                                    */

static void mat_mul(int n, int k, int m, const double* A, const double* B, double* C) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < m; ++j) {
            double s = 0.0;
            for (int l = 0; l < k; ++l) s += A[i * k + l] * B[l * m + j];
            C[i * m + j] = s;
        }
}

/* Cholesky factorisation A = L L^T of an n x n SPD matrix; returns 0 on success */
static int cholesky(int n, const double* A, double* L) {
    memset(L, 0, sizeof(double) * n * n);
    for (int j = 0; j < n; ++j) {
        double d = A[j * n + j];
        for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
        if (!(d > 0.0)) return -1;
        double ljj = sqrt(d);
        L[j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double s = A[i * n + j];
            for (int k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = s / ljj;
        }
    }
    return 0;
}

/* solve (L L^T) x = b in place */
static void chol_solve(int n, const double* L, double* b) {
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[i * n + k] * b[k];
        b[i] = s / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * b[k];
        b[i] = s / L[i * n + i];
    }
}

/* inverse of a general n x n matrix by Gauss-Jordan with partial pivoting */
static int mat_inverse(int n, const double* A, double* Ainv) {
    double M[72];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            M[i * 2 * n + j] = A[i * n + j];
            M[i * 2 * n + n + j] = (i == j) ? 1.0 : 0.0;
        }
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(M[r * 2 * n + c]) > fabs(M[p * 2 * n + c])) p = r;
        if (M[p * 2 * n + c] == 0.0) return -1;
        if (p != c)
            for (int j = 0; j < 2 * n; ++j) {
                double t = M[c * 2 * n + j];
                M[c * 2 * n + j] = M[p * 2 * n + j];
                M[p * 2 * n + j] = t;
            }
        double inv = 1.0 / M[c * 2 * n + c];
        for (int j = 0; j < 2 * n; ++j) M[c * 2 * n + j] *= inv;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            double f = M[r * 2 * n + c];
            for (int j = 0; j < 2 * n; ++j) M[r * 2 * n + j] -= f * M[c * 2 * n + j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Ainv[i * n + j] = M[i * 2 * n + n + j];
    return 0;
}

static void skew(const double w[3], double S[9]) {
    S[0] = 0.0;   S[1] = -w[2]; S[2] = w[1];
    S[3] = w[2];  S[4] = 0.0;   S[5] = -w[0];
    S[6] = -w[1]; S[7] = w[0];  S[8] = 0.0;
}

/* ------------------------------------------------------------------------ */
/* SE(3): Exp, Log, adjoint, right Jacobian (App. C.2 Eq. exp_err: tangent     */
/* [theta; rho], translation V(theta) rho)                                   */

void or_se3_exp(const double xi[6], double T[16]) {
    const double* w = xi;
    const double* rho = xi + 3;
    double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double A, B, C;   /* sin(t)/t, (1-cos t)/t^2, (t - sin t)/t^3 */
    if (th2 < 1e-2) {  /* Taylor series, truncation below 1e-19 */
        double t4 = th2 * th2, t6 = t4 * th2, t8 = t4 * t4;
        A = 1.0 - th2 / 6.0 + t4 / 120.0 - t6 / 5040.0 + t8 / 362880.0;
        B = 0.5 - th2 / 24.0 + t4 / 720.0 - t6 / 40320.0 + t8 / 3628800.0;
        C = 1.0 / 6.0 - th2 / 120.0 + t4 / 5040.0 - t6 / 362880.0 + t8 / 39916800.0;
    } else {
        double th = sqrt(th2), sh = sin(0.5 * th);
        A = sin(th) / th;
        B = 2.0 * sh * sh / th2;
        C = (th - sin(th)) / (th2 * th);
    }
    double S[9], S2[9];
    skew(w, S);
    mat_mul(3, 3, 3, S, S, S2);
    double R[9], V[9];
    for (int i = 0; i < 9; ++i) {
        double I = (i % 4 == 0) ? 1.0 : 0.0;
        R[i] = I + A * S[i] + B * S2[i];
        V[i] = I + B * S[i] + C * S2[i];
    }
    memset(T, 0, sizeof(double) * 16);
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) T[r * 4 + c] = R[r * 3 + c];
        T[r * 4 + 3] = V[r * 3 + 0] * rho[0] + V[r * 3 + 1] * rho[1] + V[r * 3 + 2] * rho[2];
    }
    T[15] = 1.0;
}

static void so3_log(const double R[9], double w[3]) {
    double tr = R[0] + R[4] + R[8];
    double v[3] = {R[7] - R[5], R[2] - R[6], R[3] - R[1]};   /* vee(R - R^T) = 2 sin(t) n */
    double s = 0.5 * sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    double c = 0.5 * (tr - 1.0);
    double th = atan2(s, c);
    if (th < 1e-4) {
        double f = 0.5 * (1.0 + th * th / 6.0 + 7.0 * th * th * th * th / 360.0);  /* t/(2 sin t) */
        for (int i = 0; i < 3; ++i) w[i] = f * v[i];
    } else if (th > M_PI - 1e-4) {
        /* near pi: axis from the symmetric part */
        double n[3];
        for (int i = 0; i < 3; ++i) {
            double d = (R[i * 4] + 1.0) * 0.5;
            n[i] = sqrt(d > 0.0 ? d : 0.0);
        }
        int k = (n[0] >= n[1] && n[0] >= n[2]) ? 0 : (n[1] >= n[2] ? 1 : 2);
        for (int i = 0; i < 3; ++i)
            if (i != k) n[i] = (R[i * 3 + k] + R[k * 3 + i]) / (4.0 * n[k]);
        double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (n[0] * v[0] + n[1] * v[1] + n[2] * v[2] < 0.0) nn = -nn;
        for (int i = 0; i < 3; ++i) w[i] = th * n[i] / nn;
    } else {
        double f = th / (2.0 * sin(th));
        for (int i = 0; i < 3; ++i) w[i] = f * v[i];
    }
}

void or_se3_log(const double T[16], double xi[6]) {
    double R[9], t[3];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) R[r * 3 + c] = T[r * 4 + c];
        t[r] = T[r * 4 + 3];
    }
    so3_log(R, xi);
    const double* w = xi;
    double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double D;  /* V^-1 = I - S/2 + D S^2, D = (1 - (t/2) cot(t/2)) / t^2 */
    if (th2 < 1e-2) {
        double t4 = th2 * th2, t6 = t4 * th2, t8 = t4 * t4;
        D = 1.0 / 12.0 + th2 / 720.0 + t4 / 30240.0 + t6 / 1209600.0 + t8 / 47900160.0;
    } else {
        double th = sqrt(th2), sh = sin(0.5 * th);
        D = (1.0 - th * sin(th) / (4.0 * sh * sh)) / th2;
    }
    double S[9], S2[9];
    skew(w, S);
    mat_mul(3, 3, 3, S, S, S2);
    for (int r = 0; r < 3; ++r) {
        double s = 0.0;
        for (int c = 0; c < 3; ++c) {
            double I = (r == c) ? 1.0 : 0.0;
            s += (I - 0.5 * S[r * 3 + c] + D * S2[r * 3 + c]) * t[c];
        }
        xi[3 + r] = s;
    }
}

static void se3_inverse(const double T[16], double Ti[16]) {
    memset(Ti, 0, sizeof(double) * 16);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) Ti[r * 4 + c] = T[c * 4 + r];
    for (int r = 0; r < 3; ++r)
        Ti[r * 4 + 3] = -(Ti[r * 4 + 0] * T[3] + Ti[r * 4 + 1] * T[7] + Ti[r * 4 + 2] * T[11]);
    Ti[15] = 1.0;
}

/* ad of xi = [theta; rho]: [[theta^, 0], [rho^, theta^]] */
static void se3_ad(const double xi[6], double ad[36]) {
    double St[9], Sr[9];
    skew(xi, St);
    skew(xi + 3, Sr);
    memset(ad, 0, sizeof(double) * 36);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            ad[r * 6 + c] = St[r * 3 + c];
            ad[(r + 3) * 6 + c] = Sr[r * 3 + c];
            ad[(r + 3) * 6 + c + 3] = St[r * 3 + c];
        }
}

/* right Jacobian from its defining series sum_n (-ad)^n / (n+1)! */
void or_se3_jr(const double xi[6], double J[36]) {
    double ad[36], P[36], Q[36];
    se3_ad(xi, ad);
    for (int i = 0; i < 36; ++i) {
        ad[i] = -ad[i];
        P[i] = (i % 7 == 0) ? 1.0 : 0.0;
        J[i] = P[i];
    }
    for (int n = 1; n < 60; ++n) {
        mat_mul(6, 6, 6, P, ad, Q);
        double mx = 0.0;
        for (int i = 0; i < 36; ++i) {
            P[i] = Q[i] / (double)(n + 1);
            J[i] += P[i];
            if (fabs(P[i]) > mx) mx = fabs(P[i]);
        }
        if (mx < 1e-20) break;
    }
}

/* prior-factor Jacobian: the inverse right Jacobian truncated after its
 * second-order term, I + ad/2 + ad^2/12 */
void or_prior_jacobian(const double xi[6], double J[36]) {
    double ad[36], ad2[36];
    se3_ad(xi, ad);
    mat_mul(6, 6, 6, ad, ad, ad2);
    for (int i = 0; i < 36; ++i) J[i] = ((i % 7 == 0) ? 1.0 : 0.0) + 0.5 * ad[i] + ad2[i] / 12.0;
}

/* ------------------------------------------------------------------------ */
/* photometric factor pieces                                                 */

/* covariance weighting equivalent to the Huber cost at whitened residual M:
 * kappa * M^2 / 2 equals the Huber energy (Sec. 3.3 Eq. distrb_photo, Sec. 4.1) */
double or_huber_weight(double M, double k) {
    M = fabs(M);
    if (M <= k) return 1.0;
    return 2.0 * k / M - (k * k) / (M * M);
}

static const double WARP_EPS = 1e-3;   /* pixels of tolerance on the image border */

int or_warp(const or_ctx* ctx, double u, double v, const double tau[6], double ell,
            double w[2], double Jw[14]) {
    const or_config* c = &ctx->cfg;
    double T[16];
    or_se3_exp(tau, T);
    double q[3] = {(u - c->cx) / c->fx, (v - c->cy) / c->fy, 1.0};
    double rho = exp(-ell);
    double a[3];
    for (int r = 0; r < 3; ++r)
        a[r] = T[r * 4 + 0] * q[0] + T[r * 4 + 1] * q[1] + T[r * 4 + 2] * q[2] + rho * T[r * 4 + 3];
    if (!(a[2] > 0.0)) return 0;
    w[0] = c->fx * a[0] / a[2] + c->cx;
    w[1] = c->fy * a[1] / a[2] + c->cy;
    /* dw/da */
    double dwda[6] = {c->fx / a[2], 0.0, -c->fx * a[0] / (a[2] * a[2]),
                      0.0, c->fy / a[2], -c->fy * a[1] / (a[2] * a[2])};
    /* da/d[dtheta, drho, dell]: -R[q]x, rho R, -rho t (3 x 7) */
    double R[9], Sq[9], RSq[9];
    for (int r = 0; r < 3; ++r)
        for (int cc = 0; cc < 3; ++cc) R[r * 3 + cc] = T[r * 4 + cc];
    skew(q, Sq);
    mat_mul(3, 3, 3, R, Sq, RSq);
    double dadx[21];
    for (int r = 0; r < 3; ++r) {
        for (int cc = 0; cc < 3; ++cc) {
            dadx[r * 7 + cc] = -RSq[r * 3 + cc];
            dadx[r * 7 + 3 + cc] = rho * R[r * 3 + cc];
        }
        dadx[r * 7 + 6] = -rho * T[r * 4 + 3];
    }
    mat_mul(2, 3, 7, dwda, dadx, Jw);
    return 1;
}

/* bilinear sample of an H x W image at (x, y) inside [0, W-1] x [0, H-1];
 * a single-row image (H = 1) is sampled linearly along x */
static double bilinear(const double* img, int H, int W, double x, double y) {
    if (H == 1) {
        int x0 = (int)floor(x);
        if (x0 > W - 2) x0 = W - 2;
        if (x0 < 0) x0 = 0;
        double fx = x - x0;
        return (1.0 - fx) * img[x0] + fx * img[x0 + 1];
    }
    int x0 = (int)floor(x), y0 = (int)floor(y);
    if (x0 > W - 2) x0 = W - 2;
    if (y0 > H - 2) y0 = H - 2;
    if (x0 < 0) x0 = 0;
    if (y0 < 0) y0 = 0;
    double fx = x - x0, fy = y - y0;
    const double* p = img + (size_t)y0 * W + x0;
    return (1.0 - fy) * ((1.0 - fx) * p[0] + fx * p[1]) + fy * ((1.0 - fx) * p[W] + fx * p[W + 1]);
}

static void add_outer(double lam[49], double eta[7], const double J[7], double r, double prec) {
    for (int a = 0; a < 7; ++a) {
        eta[a] -= J[a] * prec * r;
        for (int b = 0; b < 7; ++b) lam[a * 7 + b] += J[a] * prec * J[b];
    }
}

/* pose part of the prior factor, Eq. (prior): r = Log(Exp(xi_hat)^-1 Exp(tau))
 * with precision lamP, added to (eta, lam) */
static void add_pose_prior(const or_config* c, const double tau[6], double lamP, double eta[7],
                           double lam[49]) {
    double Tp[16], Tpi[16], Tt[16], Tr[16], rp[6];
    or_se3_exp(c->prior_xi, Tp);
    se3_inverse(Tp, Tpi);
    or_se3_exp(tau, Tt);
    mat_mul(4, 4, 4, Tpi, Tt, Tr);
    or_se3_log(Tr, rp);
    double Jp[36];
    or_prior_jacobian(rp, Jp);
    for (int k = 0; k < 6; ++k) {
        double row[7] = {0};
        for (int cc = 0; cc < 6; ++cc) row[cc] = Jp[k * 6 + cc];
        add_outer(lam, eta, row, rp[k], lamP);
    }
}

/* precision of a factor whose sigma is halved at each level above the
 * pixels: sigma_l = sigma 2^-l (Sec. 4.2) */
static double level_lambda(double sigma, int l) {
    double s = ldexp(sigma, -l);
    return 1.0 / (s * s);
}

/* photometric + prior unary factor of pixel i in information form */
static int unary_at(const or_ctx* ctx, int i, double eta[7], double lam[49], int* valid) {
    const or_config* c = &ctx->cfg;
    const int W = c->W, H = c->H;
    const int u = i % W, v = i / W;
    const double* tau = ctx->tau + 6 * (size_t)i;
    const double ell = ctx->ell[i];
    memset(eta, 0, sizeof(double) * 7);
    memset(lam, 0, sizeof(double) * 49);
    *valid = 0;

    /* photometric factor, Eq. (distrb_photo) with the warp of Eq. (warp) */
    double w[2], Jw[14];
    if (or_warp(ctx, (double)u, (double)v, tau, ell, w, Jw) &&
        w[0] >= -WARP_EPS && w[0] <= (W - 1) + WARP_EPS &&
        w[1] >= -WARP_EPS && w[1] <= (H - 1) + WARP_EPS) {
        double x = fmin(fmax(w[0], 0.0), (double)(W - 1));
        double y = fmin(fmax(w[1], 0.0), (double)(H - 1));
        double It = bilinear(ctx->I_t, H, W, x, y);
        double gx = bilinear(ctx->Gx, H, W, x, y);
        double gy = bilinear(ctx->Gy, H, W, x, y);
        double r = ctx->I_s[i] - It;
        double J[7];
        for (int k = 0; k < 7; ++k) J[k] = -(gx * Jw[k] + gy * Jw[7 + k]);
        double lamD = 1.0 / (ctx->sigD[i] * ctx->sigD[i]);
        double kappa = or_huber_weight(fabs(r) * sqrt(lamD), c->huber_k);
        add_outer(lam, eta, J, r, kappa * lamD);
        *valid = 1;
    }

    /* prior factor, Eq. (prior): r = [Log(Exp(xi_hat)^-1 Exp(tau)); ell - ell_hat] */
    double lamP = 1.0 / (c->sigma_P * c->sigma_P);
    add_pose_prior(c, tau, lamP, eta, lam);
    double row6[7] = {0, 0, 0, 0, 0, 0, 1.0};
    add_outer(lam, eta, row6, ell - ctx->prior_ell[i], lamP);
    return 0;
}

int or_unary(const or_ctx* ctx, int u, int v, double eta[7], double lam[49], int* valid) {
    if (!ctx->have_kf || !ctx->have_frame) return -1;
    return unary_at(ctx, v * ctx->cfg.W + u, eta, lam, valid);
}

/* ------------------------------------------------------------------------ */
/* factor-to-variable message by dense marginalisation                       */

int or_factor_message(int m, const double* r, const double* J, const double* prec,
                      const double eta_s[7], const double lam_s[49],
                      double eta_out[7], double lam_out[49]) {
    double L[196], h[14];
    for (int a = 0; a < 14; ++a) {
        h[a] = 0.0;
        for (int k = 0; k < m; ++k) h[a] -= J[k * 14 + a] * prec[k] * r[k];
        for (int b = 0; b < 14; ++b) {
            double s = 0.0;
            for (int k = 0; k < m; ++k) s += J[k * 14 + a] * prec[k] * J[k * 14 + b];
            L[a * 14 + b] = s;
        }
    }
    /* the sender's variable-to-factor message enters the sender block */
    for (int a = 0; a < 7; ++a) {
        h[7 + a] += eta_s[a];
        for (int b = 0; b < 7; ++b) L[(7 + a) * 14 + 7 + b] += lam_s[a * 7 + b];
    }
    /* marginalise the sender: Lrr - Lrs Lss^-1 Lsr, hr - Lrs Lss^-1 hs */
    double Lss[49], Lc[49];
    for (int a = 0; a < 7; ++a)
        for (int b = 0; b < 7; ++b) Lss[a * 7 + b] = L[(7 + a) * 14 + 7 + b];
    if (cholesky(7, Lss, Lc) != 0) return -1;
    double X[49], y[7];
    for (int col = 0; col < 7; ++col) {
        double b[7];
        for (int a = 0; a < 7; ++a) b[a] = L[(7 + a) * 14 + col];   /* Lsr column */
        chol_solve(7, Lc, b);
        for (int a = 0; a < 7; ++a) X[a * 7 + col] = b[a];
    }
    for (int a = 0; a < 7; ++a) y[a] = h[7 + a];
    chol_solve(7, Lc, y);
    for (int a = 0; a < 7; ++a) {
        double se = h[a];
        for (int k = 0; k < 7; ++k) se -= L[a * 14 + 7 + k] * y[k];
        eta_out[a] = se;
        for (int b = 0; b < 7; ++b) {
            double s = L[a * 14 + b];
            for (int k = 0; k < 7; ++k) s -= L[a * 14 + 7 + k] * X[k * 7 + b];
            lam_out[a * 7 + b] = s;
        }
    }
    /* an information matrix is symmetric; remove the rounding asymmetry of the product */
    for (int a = 0; a < 7; ++a)
        for (int b = a + 1; b < 7; ++b) {
            double sym = 0.5 * (lam_out[a * 7 + b] + lam_out[b * 7 + a]);
            lam_out[a * 7 + b] = sym;
            lam_out[b * 7 + a] = sym;
        }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* context                                                                   */

void or_default_config(or_config* c) {
    memset(c, 0, sizeof(*c));
    c->H = 24; c->W = 32;
    c->fx = c->fy = 30.0; c->cx = 16.0; c->cy = 12.0;
    /* leaf-level strengths of Sec. 4.2 */
    c->sigma_D = 5e-3; c->sigma_P = 1.0; c->sigma_R = 4e-4; c->sigma_N = 1e-3; c->huber_k = 400.0;
    c->init_inv_depth = 1.0;
    c->prior_log_depth = 0.0;
    c->kf_max_frames = 150;
    c->kf_min_valid_frac = 0.5;
    c->damping = 0.0;
}

int or_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of the OpenMP loops from now on (n >= 1); the CPU-baseline timing
 * runs one thread and all host threads in one process */
void or_set_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

or_ctx* or_create(const or_config* cfg) {
    if (!cfg || cfg->H < 1 || cfg->W < 2 || !(cfg->fx > 0) || !(cfg->fy > 0)) return NULL;
    if (cfg->topology != OR_TOPO_GRID && cfg->topology != OR_TOPO_QUADTREE) return NULL;
    or_ctx* x = (or_ctx*)calloc(1, sizeof(or_ctx));
    x->cfg = *cfg;
    x->N = cfg->H * cfg->W;
    size_t N = (size_t)x->N;
    x->I_s = calloc(N, sizeof(double));
    x->cxt = calloc(N, sizeof(double));
    x->cyt = calloc(N, sizeof(double));
    x->I_t = calloc(N, sizeof(double));
    x->Gx = calloc(N, sizeof(double));
    x->Gy = calloc(N, sizeof(double));
    x->sigD = calloc(N, sizeof(double));
    x->prior_ell = calloc(N, sizeof(double));
    x->tau = calloc(6 * N, sizeof(double));
    x->ell = calloc(N, sizeof(double));
    x->msg = calloc(8 * N, sizeof(g7));
    x->newmsg = calloc(8 * N, sizeof(g7));
    x->unary = calloc(N, sizeof(g7));
    x->belief = calloc(N, sizeof(g7));
    x->mean = calloc(7 * N, sizeof(double));
    x->var_ll = calloc(N, sizeof(double));
    x->valid = calloc(N, sizeof(int));
    for (size_t i = 0; i < N; ++i) {
        x->sigD[i] = cfg->sigma_D;
        x->prior_ell[i] = cfg->prior_log_depth;
        x->ell[i] = -log(cfg->init_inv_depth);
        x->var_ll[i] = NAN;
    }
    memset(x->T_w_kf, 0, sizeof(x->T_w_kf));
    for (int k = 0; k < 4; ++k) x->T_w_kf[k * 5] = 1.0;
    /* quadtree levels: level l >= 1 has ceil(H / 2^l) x ceil(W / 2^l) nodes,
     * the last level is the single root */
    x->lvH[0] = cfg->H;
    x->lvW[0] = cfg->W;
    x->L = 0;
    if (cfg->topology == OR_TOPO_QUADTREE) {
        x->tree = 1;
        while (x->lvH[x->L] > 1 || x->lvW[x->L] > 1) {
            x->lvH[x->L + 1] = (x->lvH[x->L] + 1) / 2;
            x->lvW[x->L + 1] = (x->lvW[x->L] + 1) / 2;
            x->L += 1;
        }
    }
    x->lvOff[1] = 0;
    for (int l = 1; l <= x->L; ++l) x->lvOff[l + 1] = x->lvOff[l] + x->lvH[l] * x->lvW[l];
    x->NT = x->lvOff[x->L + 1];
    if (x->tree) {
        size_t NT = (size_t)x->NT;
        x->ntau = calloc(6 * NT, sizeof(double));
        x->pmsg = calloc(N, sizeof(g7));
        x->pnewmsg = calloc(N, sizeof(g7));
        x->nmsg = calloc(5 * NT, sizeof(g7));
        x->nnewmsg = calloc(5 * NT, sizeof(g7));
        x->nunary = calloc(NT, sizeof(g7));
        x->nbelief = calloc(NT, sizeof(g7));
    }
    return x;
}

void or_destroy(or_ctx* x) {
    if (!x) return;
    free(x->I_s); free(x->cxt); free(x->cyt); free(x->I_t); free(x->Gx); free(x->Gy);
    free(x->sigD); free(x->prior_ell); free(x->tau); free(x->ell); free(x->msg); free(x->newmsg);
    free(x->unary); free(x->belief); free(x->mean); free(x->var_ll); free(x->valid);
    free(x->ntau); free(x->pmsg); free(x->pnewmsg); free(x->nmsg); free(x->nnewmsg);
    free(x->nunary); free(x->nbelief);
    free(x);
}

int or_set_sigma_D_map(or_ctx* x, const double* s) {
    for (int i = 0; i < x->N; ++i) x->sigD[i] = s ? s[i] : x->cfg.sigma_D;
    return 0;
}

/* current world pose of the camera: T_w_kf * Exp(xi_last)^-1 */
static void world_pose(const or_ctx* x, double out[16]) {
    double E[16], Ei[16];
    or_se3_exp(x->xi_last, E);
    se3_inverse(E, Ei);
    mat_mul(4, 4, 4, x->T_w_kf, Ei, out);
}

static int set_keyframe_impl(or_ctx* x, const float* img32, const double* img64,
                             const float* normals) {
    const or_config* c = &x->cfg;
    const int W = c->W;
    if (x->have_track) {            /* re-anchor: the new keyframe is the current camera */
        double Tw[16];
        world_pose(x, Tw);
        memcpy(x->T_w_kf, Tw, sizeof(Tw));
    }
    memset(x->xi_last, 0, sizeof(x->xi_last));
    x->have_track = 0;
    for (int i = 0; i < x->N; ++i) {
        x->I_s[i] = img64 ? img64[i] : (double)img32[i];
        /* normal integration targets (Eq. gbpni): the log-depth step to the
         * right/lower neighbour implied by the normal n at pixel a is
         * -n_x / (f_x n.q_a) (resp. -n_y / (f_y n.q_a)); the factor's residual
         * is (ell_b - ell_a) + c_a. Grazing normals deactivate the edge. */
        int u = i % W, v = i / W;
        double q[3] = {(u - c->cx) / c->fx, (v - c->cy) / c->fy, 1.0};
        double n[3] = {normals[3 * i], normals[3 * i + 1], normals[3 * i + 2]};
        double nq = n[0] * q[0] + n[1] * q[1] + n[2] * q[2];
        double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
        int ok = isfinite(nq) && fabs(nq) >= 1e-3 * qn;
        x->cxt[i] = ok ? n[0] / (c->fx * nq) : NAN;
        x->cyt[i] = ok ? n[1] / (c->fy * nq) : NAN;
        for (int k = 0; k < 6; ++k) x->tau[6 * (size_t)i + k] = 0.0;
    }
    memset(x->msg, 0, sizeof(g7) * 8 * (size_t)x->N);
    if (x->tree) {
        memset(x->ntau, 0, sizeof(double) * 6 * (size_t)x->NT);
        memset(x->pmsg, 0, sizeof(g7) * (size_t)x->N);
        memset(x->nmsg, 0, sizeof(g7) * 5 * (size_t)x->NT);
    }
    x->frames_since_kf = 0;
    x->have_kf = 1;
    x->diverged = 0;
    return 0;
}

int or_set_keyframe(or_ctx* x, const float* img, const float* normals) {
    return set_keyframe_impl(x, img, NULL, normals);
}

int or_set_keyframe64(or_ctx* x, const double* img, const float* normals) {
    return set_keyframe_impl(x, NULL, img, normals);
}

/* keyframe depth transfer (depth propagation, Sec. 3.3; re-anchoring, Sec.
 * 3.5): the 3-D point exp(ell) q of every pixel of the current keyframe is
 * moved into the camera of the frame just tracked by that frame's pose
 * estimate Exp(xi) (keyframe points to current camera) and splatted to the
 * nearest pixel of the new keyframe (rounding half up); where several land,
 * the nearest depth (compared at FP32) wins; pixels nothing lands on keep
 * their log-depth. The new log-depth is log of the point's depth z. */
int or_transfer_depth(or_ctx* x) {
    if (!x || !x->have_track) return -2;
    const or_config* c = &x->cfg;
    const int W = c->W, H = c->H, N = x->N;
    double T[16];
    or_se3_exp(x->xi_last, T);
    float* zb = (float*)malloc(sizeof(float) * (size_t)N);
    for (int j = 0; j < N; ++j) zb[j] = INFINITY;
    for (int i = 0; i < N; ++i) {
        const int u = i % W, v = i / W;
        const double d = exp(x->ell[i]);
        const double P[3] = {d * (u - c->cx) / c->fx, d * (v - c->cy) / c->fy, d};
        double Q[3];
        for (int r = 0; r < 3; ++r) Q[r] = T[r * 4] * P[0] + T[r * 4 + 1] * P[1] + T[r * 4 + 2] * P[2] + T[r * 4 + 3];
        if (!(Q[2] > 0.0)) continue;
        const double uu = c->fx * Q[0] / Q[2] + c->cx, vv = c->fy * Q[1] / Q[2] + c->cy;
        const double ju = floor(uu + 0.5), jv = floor(vv + 0.5);
        if (!(ju >= 0.0 && ju < (double)W && jv >= 0.0 && jv < (double)H)) continue;
        const int j = (int)jv * W + (int)ju;
        const float z = (float)Q[2];
        if (z < zb[j]) zb[j] = z;
    }
    for (int j = 0; j < N; ++j)
        if (zb[j] < INFINITY) x->ell[j] = log((double)zb[j]);
    free(zb);
    return 0;
}

static void set_frame_impl(or_ctx* x, const float* f32, const double* f64) {
    const int H = x->cfg.H, W = x->cfg.W;
    for (int i = 0; i < x->N; ++i) x->I_t[i] = f64 ? f64[i] : (double)f32[i];
    /* central differences inside, one-sided at the border */
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            const double* I = x->I_t;
            int i = v * W + u;
            if (u == 0) x->Gx[i] = I[i + 1] - I[i];
            else if (u == W - 1) x->Gx[i] = I[i] - I[i - 1];
            else x->Gx[i] = 0.5 * (I[i + 1] - I[i - 1]);
            if (H == 1) x->Gy[i] = 0.0;
            else if (v == 0) x->Gy[i] = I[i + W] - I[i];
            else if (v == H - 1) x->Gy[i] = I[i] - I[i - W];
            else x->Gy[i] = 0.5 * (I[i + W] - I[i - W]);
        }
    x->have_frame = 1;
}

int or_set_frame(or_ctx* x, const float* frame) {
    set_frame_impl(x, frame, NULL);
    return 0;
}

int or_set_frame64(or_ctx* x, const double* frame) {
    set_frame_impl(x, NULL, frame);
    return 0;
}

static int neighbour(const or_ctx* x, int i, int d) {
    const int W = x->cfg.W, H = x->cfg.H;
    int u = i % W, v = i / W;
    switch (d) {
        case OR_LEFT: return u > 0 ? i - 1 : -1;
        case OR_RIGHT: return u < W - 1 ? i + 1 : -1;
        case OR_UP: return v > 0 ? i - W : -1;
        default: return v < H - 1 ? i + W : -1;
    }
}

static int opposite(int d) { return d ^ 1; }

static void g7_zero(g7* g) { memset(g, 0, sizeof(*g)); }

/* message to the receiver (linearisation point t_recv) of the identity factor
 * (Eq. regul) it shares with a sender (t_send), given the sender's belief and
 * the factor's previous message to the sender:
 * r = Log(Exp(t_send)^-1 Exp(t_recv)), Jacobians +I (receiver) and -I (sender)
 * at consensus, or the exact Lie Jacobians J_r(r)^-1 and -J_l(r)^-1 */
static int identity_message(const or_config* c, const double* t_recv, const double* t_send, double lamR,
                            const g7* bel_send, const g7* back, g7* out) {
    double Ti[16], Tj[16], Tji[16], Trel[16], r[6];
    or_se3_exp(t_recv, Ti);
    or_se3_exp(t_send, Tj);
    se3_inverse(Tj, Tji);
    mat_mul(4, 4, 4, Tji, Ti, Trel);
    or_se3_log(Trel, r);
    double J[6 * 14];
    memset(J, 0, sizeof(J));
    if (c->full_jacobian) {
        double Jr[36], Ji[36], rn[6], Jl[36], Jli[36];
        or_se3_jr(r, Jr);
        mat_inverse(6, Jr, Ji);
        for (int k = 0; k < 6; ++k) rn[k] = -r[k];
        or_se3_jr(rn, Jl);                 /* J_l(r) = J_r(-r) */
        mat_inverse(6, Jl, Jli);
        for (int a = 0; a < 6; ++a)
            for (int b = 0; b < 6; ++b) {
                J[a * 14 + b] = Ji[a * 6 + b];
                J[a * 14 + 7 + b] = -Jli[a * 6 + b];
            }
    } else {
        for (int a = 0; a < 6; ++a) {
            J[a * 14 + a] = 1.0;
            J[a * 14 + 7 + a] = -1.0;
        }
    }
    double prec6[6] = {lamR, lamR, lamR, lamR, lamR, lamR};
    g7 v2f = *bel_send;
    for (int a = 0; a < 7; ++a) v2f.eta[a] -= back->eta[a];
    for (int a = 0; a < 49; ++a) v2f.lam[a] -= back->lam[a];
    return or_factor_message(6, r, J, prec6, v2f.eta, v2f.lam, out->eta, out->lam) ? -1 : 0;
}

static void g7_add(g7* b, const g7* m) {
    for (int a = 0; a < 7; ++a) b->eta[a] += m->eta[a];
    for (int a = 0; a < 49; ++a) b->lam[a] += m->lam[a];
}

static void g7_damp(g7* nm, const g7* om, double bta) {
    for (int a = 0; a < 7; ++a) nm->eta[a] = (1.0 - bta) * nm->eta[a] + bta * om->eta[a];
    for (int a = 0; a < 49; ++a) nm->lam[a] = (1.0 - bta) * nm->lam[a] + bta * om->lam[a];
}

/* Planted faults for the test-suite's check that the transport pins can fail
 * (the oracle's own build never defines OR_PLANTED_FAULT): 1 drops the
 * transport, 2 transports the identity-factor slots only, 3 transports with
 * the information of the message that was replaced. */
#ifndef OR_PLANTED_FAULT
#define OR_PLANTED_FAULT 0
#endif

/* first-order transport of a stored message into the tangent space moved by m */
static void g7_transport(g7* g, const double m[7]) {
    for (int a = 0; a < 7; ++a) {
        double s = 0.0;
        for (int bb = 0; bb < 7; ++bb) s += g->lam[a * 7 + bb] * m[bb];
        g->eta[a] -= s;
    }
}

/* storage emulation (test switch): FP32 rounding of a message */
static void g7_round32(g7* g) {
    for (int a = 0; a < 7; ++a) g->eta[a] = (double)(float)g->eta[a];
    for (int a = 0; a < 49; ++a) g->lam[a] = (double)(float)g->lam[a];
}

static double round32(double x) { return (double)(float)x; }

/* quadtree node helpers */
static int node_level(const or_ctx* x, int n) {
    int l = 1;
    while (n >= x->lvOff[l + 1]) ++l;
    return l;
}
static int node_at(const or_ctx* x, int l, int col, int row) { return x->lvOff[l] + row * x->lvW[l] + col; }

/* unary factor of a quadtree node: the pose prior of its level (Eq. prior,
 * sigma_P halved per level) and unit information on the inert 7th coordinate */
static void node_unary(const or_ctx* x, int l, const double* tau, g7* u) {
    memset(u, 0, sizeof(*u));
    add_pose_prior(&x->cfg, tau, level_lambda(x->cfg.sigma_P, l), u->eta, u->lam);
    u->lam[48] = 1.0;
}

/* one synchronous GBP iteration (Sec. 4.1, Sec. 4.3) */
static int iterate_once(or_ctx* x) {
    const or_config* c = &x->cfg;
    const int N = x->N, NT = x->NT, tree = x->tree;
    const double lamR = 1.0 / (c->sigma_R * c->sigma_R);
    const double lamN = 1.0 / (c->sigma_N * c->sigma_N);
    int fail = 0;

    /* L + B: unary factors at the linearisation points and beliefs */
#pragma omp parallel for schedule(static) reduction(| : fail)
    for (int i = 0; i < N; ++i) {
        g7* u = &x->unary[i];
        unary_at(x, i, u->eta, u->lam, &x->valid[i]);
        g7* b = &x->belief[i];
        *b = *u;
        for (int k = 0; k < 8; ++k) g7_add(b, &x->msg[8 * (size_t)i + k]);
        if (tree) g7_add(b, &x->pmsg[i]);
    }
#pragma omp parallel for schedule(static)
    for (int n = 0; n < NT; ++n) {
        node_unary(x, node_level(x, n), x->ntau + 6 * (size_t)n, &x->nunary[n]);
        x->nbelief[n] = x->nunary[n];
        for (int k = 0; k < 5; ++k) g7_add(&x->nbelief[n], &x->nmsg[5 * (size_t)n + k]);
    }

    /* F: factor-to-variable messages for every directed edge */
#pragma omp parallel for schedule(static) reduction(| : fail)
    for (int i = 0; i < N; ++i) {
        const double* ti = x->tau + 6 * (size_t)i;
        for (int d = 0; d < 4; ++d) {
            g7* out_id = &x->newmsg[8 * (size_t)i + d];
            g7* out_n = &x->newmsg[8 * (size_t)i + 4 + d];
            int j = neighbour(x, i, d);
            if (j < 0) { g7_zero(out_id); g7_zero(out_n); continue; }
            int dj = opposite(d);

            /* identity factor of the grid topology, Eq. (regul) */
            if (tree) g7_zero(out_id);
            else if (identity_message(c, ti, x->tau + 6 * (size_t)j, lamR, &x->belief[j],
                                      &x->msg[8 * (size_t)j + dj], out_id))
                fail = 1;

            /* normal integration factor, Eq. (gbpni): r = ell_b - ell_a + c_a,
             * a = left/upper pixel of the edge, b = right/lower pixel */
            int horizontal = (d == OR_LEFT || d == OR_RIGHT);
            int recv_is_b = (d == OR_LEFT || d == OR_UP);
            int a_idx = recv_is_b ? j : i;
            double ca = horizontal ? x->cxt[a_idx] : x->cyt[a_idx];
            if (!isfinite(ca) || lamN == 0.0) { g7_zero(out_n); continue; }
            double ell_a = recv_is_b ? x->ell[j] : x->ell[i];
            double ell_b = recv_is_b ? x->ell[i] : x->ell[j];
            double rn = ell_b - ell_a + ca;
            double Jn[14];
            memset(Jn, 0, sizeof(Jn));
            Jn[6] = recv_is_b ? 1.0 : -1.0;
            Jn[13] = -Jn[6];
            g7 v2f = x->belief[j];
            const g7* back = &x->msg[8 * (size_t)j + 4 + dj];
            for (int a = 0; a < 7; ++a) v2f.eta[a] -= back->eta[a];
            for (int a = 0; a < 49; ++a) v2f.lam[a] -= back->lam[a];
            if (or_factor_message(1, &rn, Jn, &lamN, v2f.eta, v2f.lam, out_n->eta, out_n->lam))
                fail = 1;
        }
        if (tree) {
            /* quadtree identity factor to the parent node of level 1 */
            const int W = c->W, u = i % W, v = i / W;
            const int p = node_at(x, 1, u / 2, v / 2), q = 2 * (v & 1) + (u & 1);
            if (identity_message(c, ti, x->ntau + 6 * (size_t)p, level_lambda(c->sigma_R, 0),
                                 &x->nbelief[p], &x->nmsg[5 * (size_t)p + 1 + q], &x->pnewmsg[i]))
                fail = 1;
            if (c->damping != 0.0) g7_damp(&x->pnewmsg[i], &x->pmsg[i], c->damping);
        }
        if (c->damping != 0.0)
            for (int k = 0; k < 8; ++k)
                g7_damp(&x->newmsg[8 * (size_t)i + k], &x->msg[8 * (size_t)i + k], c->damping);
    }
    /* quadtree nodes: messages of the edges to the parent and to the children;
     * the identity factor between levels l and l + 1 has sigma_R 2^-l */
#pragma omp parallel for schedule(static) reduction(| : fail)
    for (int n = 0; n < NT; ++n) {
        const int l = node_level(x, n);
        const int col = (n - x->lvOff[l]) % x->lvW[l], row = (n - x->lvOff[l]) / x->lvW[l];
        const double* tn = x->ntau + 6 * (size_t)n;
        g7* out = &x->nnewmsg[5 * (size_t)n];
        if (l < x->L) {
            const int pp = node_at(x, l + 1, col / 2, row / 2), qn = 2 * (row & 1) + (col & 1);
            if (identity_message(c, tn, x->ntau + 6 * (size_t)pp, level_lambda(c->sigma_R, l),
                                 &x->nbelief[pp], &x->nmsg[5 * (size_t)pp + 1 + qn], &out[0]))
                fail = 1;
        } else {
            g7_zero(&out[0]);
        }
        for (int q = 0; q < 4; ++q) {
            const int cc = 2 * col + (q & 1), cr = 2 * row + (q >> 1);
            if (cc >= x->lvW[l - 1] || cr >= x->lvH[l - 1]) { g7_zero(&out[1 + q]); continue; }
            const double* ts;
            const g7 *bel, *back;
            if (l == 1) {
                const int ch = cr * c->W + cc;
                ts = x->tau + 6 * (size_t)ch;
                bel = &x->belief[ch];
                back = &x->pmsg[ch];
            } else {
                const int ch = node_at(x, l - 1, cc, cr);
                ts = x->ntau + 6 * (size_t)ch;
                bel = &x->nbelief[ch];
                back = &x->nmsg[5 * (size_t)ch];
            }
            if (identity_message(c, tn, ts, level_lambda(c->sigma_R, l - 1), bel, back, &out[1 + q]))
                fail = 1;
        }
        if (c->damping != 0.0)
            for (int k = 0; k < 5; ++k) g7_damp(&out[k], &x->nmsg[5 * (size_t)n + k], c->damping);
    }

    if (c->store_fp32) {
#pragma omp parallel for schedule(static)
        for (int i = 0; i < N; ++i) {
            for (int k = 0; k < 8; ++k) g7_round32(&x->newmsg[8 * (size_t)i + k]);
            if (tree) g7_round32(&x->pnewmsg[i]);
        }
#pragma omp parallel for schedule(static)
        for (int n = 0; n < NT; ++n)
            for (int k = 0; k < 5; ++k) g7_round32(&x->nnewmsg[5 * (size_t)n + k]);
    }

    /* U: new beliefs, means, relinearisation and message transport */
#pragma omp parallel for schedule(static) reduction(| : fail)
    for (int i = 0; i < N; ++i) {
        g7* mi = &x->msg[8 * (size_t)i];
#if OR_PLANTED_FAULT == 3
        g7 replaced[8];
        memcpy(replaced, mi, 8 * sizeof(g7));
#endif
        memcpy(mi, &x->newmsg[8 * (size_t)i], 8 * sizeof(g7));
        g7 b = x->unary[i];
        for (int k = 0; k < 8; ++k) g7_add(&b, &mi[k]);
        if (tree) {
            x->pmsg[i] = x->pnewmsg[i];
            g7_add(&b, &x->pmsg[i]);
        }
        x->belief[i] = b;
        double Lc[49];
        double* m = x->mean + 7 * (size_t)i;
        if (cholesky(7, b.lam, Lc) != 0) {
            fail = 1;
            for (int a = 0; a < 7; ++a) m[a] = NAN;
            x->var_ll[i] = NAN;
            continue;
        }
        memcpy(m, b.eta, sizeof(double) * 7);
        chol_solve(7, Lc, m);
        double e6[7] = {0, 0, 0, 0, 0, 0, 1.0};
        chol_solve(7, Lc, e6);
        x->var_ll[i] = e6[6];
        if (c->frozen) continue;
        /* relinearise at the belief mean (Eq. var): tau <- Log(Exp(tau) Exp(m)) */
        double* ti = x->tau + 6 * (size_t)i;
        double T0[16], Tm[16], T1[16];
        or_se3_exp(ti, T0);
        or_se3_exp(m, Tm);
        mat_mul(4, 4, 4, T0, Tm, T1);
        or_se3_log(T1, ti);
        x->ell[i] += m[6];
        /* first-order transport of stored messages into the new tangent space */
#if OR_PLANTED_FAULT == 0
        for (int k = 0; k < 8; ++k) g7_transport(&mi[k], m);
#elif OR_PLANTED_FAULT == 2
        for (int k = 0; k < 4; ++k) g7_transport(&mi[k], m);
#elif OR_PLANTED_FAULT == 3
        for (int k = 0; k < 8; ++k) {
            g7 t = replaced[k];
            memcpy(t.eta, mi[k].eta, sizeof(t.eta));
            g7_transport(&t, m);
            memcpy(mi[k].eta, t.eta, sizeof(t.eta));
        }
#endif
        if (tree) g7_transport(&x->pmsg[i], m);
    }
#pragma omp parallel for schedule(static) reduction(| : fail)
    for (int n = 0; n < NT; ++n) {
        g7* mn = &x->nmsg[5 * (size_t)n];
        memcpy(mn, &x->nnewmsg[5 * (size_t)n], 5 * sizeof(g7));
        g7 b = x->nunary[n];
        for (int k = 0; k < 5; ++k) g7_add(&b, &mn[k]);
        x->nbelief[n] = b;
        double Lc[49], m[7];
        if (cholesky(7, b.lam, Lc) != 0) {
            fail = 1;
            continue;
        }
        memcpy(m, b.eta, sizeof(double) * 7);
        chol_solve(7, Lc, m);
        if (c->frozen) continue;
        double* tn = x->ntau + 6 * (size_t)n;
        double T0[16], Tm[16], T1[16];
        or_se3_exp(tn, T0);
        or_se3_exp(m, Tm);
        mat_mul(4, 4, 4, T0, Tm, T1);
        or_se3_log(T1, tn);
        for (int k = 0; k < 5; ++k) g7_transport(&mn[k], m);
    }
    if (c->store_fp32) {
#pragma omp parallel for schedule(static)
        for (int i = 0; i < N; ++i) {
            for (int k = 0; k < 6; ++k) x->tau[6 * (size_t)i + k] = round32(x->tau[6 * (size_t)i + k]);
            x->ell[i] = round32(x->ell[i]);
            for (int k = 0; k < 8; ++k) g7_round32(&x->msg[8 * (size_t)i + k]);
            if (tree) g7_round32(&x->pmsg[i]);
        }
#pragma omp parallel for schedule(static)
        for (int n = 0; n < NT; ++n) {
            for (int k = 0; k < 6; ++k) x->ntau[6 * (size_t)n + k] = round32(x->ntau[6 * (size_t)n + k]);
            for (int k = 0; k < 5; ++k) g7_round32(&x->nmsg[5 * (size_t)n + k]);
        }
    }
    if (fail) x->diverged = 1;
    return fail ? -1 : 0;
}

int or_iterate(or_ctx* x, int n_iters) {
    if (!x->have_kf || !x->have_frame) return -2;
    int rc = 0;
    for (int it = 0; it < n_iters; ++it)
        if (iterate_once(x)) rc = -1;
    return rc;
}

int or_track(or_ctx* x, const float* frame, int n_iters, or_track_out* out,
             double* inv_depth, double* inv_depth_var) {
    if (!x->have_kf) return -2;
    if (n_iters < 0) return -1;
    or_set_frame(x, frame);
    if (n_iters == 0)
        for (int i = 0; i < x->N; ++i) x->var_ll[i] = NAN;
    or_iterate(x, n_iters);
    const int N = x->N;
    /* pose estimate: mean of the per-pixel poses (Eq. estimator_avg) */
    double xi[6] = {0};
    int nvalid = 0, bad = 0;
    for (int i = 0; i < N; ++i) {
        for (int k = 0; k < 6; ++k) xi[k] += x->tau[6 * (size_t)i + k];
        nvalid += x->valid[i];
        if (!isfinite(x->ell[i])) bad = 1;
        for (int k = 0; k < 6; ++k) if (!isfinite(x->tau[6 * (size_t)i + k])) bad = 1;
    }
    for (int k = 0; k < 6; ++k) xi[k] /= (double)N;
    memcpy(x->xi_last, xi, sizeof(xi));
    x->have_track = 1;
    x->frames_since_kf += 1;
    if (n_iters == 0) {   /* no iteration: the overlap test uses the current point */
        nvalid = 0;
        for (int i = 0; i < N; ++i) {
            double e[7], l[49];
            int vv;
            unary_at(x, i, e, l, &vv);
            nvalid += vv;
        }
    }
    double vf = (double)nvalid / (double)N;
    if (inv_depth)
        for (int i = 0; i < N; ++i) inv_depth[i] = exp(-x->ell[i]);
    if (inv_depth_var)
        for (int i = 0; i < N; ++i) {
            double r = exp(-x->ell[i]);
            inv_depth_var[i] = r * r * x->var_ll[i];
        }
    if (out) {
        memcpy(out->xi, xi, sizeof(xi));
        world_pose(x, out->T_world);
        out->valid_fraction = vf;
        out->frames_since_keyframe = x->frames_since_kf;
        unsigned f = 0;
        if (x->frames_since_kf >= x->cfg.kf_max_frames || vf < x->cfg.kf_min_valid_frac)
            f |= OR_KEYFRAME_DUE;
        if (vf < x->cfg.kf_min_valid_frac) f |= OR_LOW_OVERLAP;
        if (bad || x->diverged) f |= OR_DIVERGED;
        out->flags = f;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* state exchange                                                            */

size_t or_state_doubles(const or_ctx* x) {
    return x->tree ? (size_t)x->N * 42 + (size_t)x->NT * 141 : (size_t)x->N * 123;
}

static int upper_index(int r, int c) { return r * 6 - r * (r - 1) / 2 + (c - r); }

/* identity message <-> 27 exchange values (eta 6, Lambda upper-packed 21) */
static void pack27(const g7* g, double* p) {
    for (int a = 0; a < 6; ++a) p[a] = g->eta[a];
    for (int r = 0; r < 6; ++r)
        for (int cc = r; cc < 6; ++cc) p[6 + upper_index(r, cc)] = g->lam[r * 7 + cc];
}
static void unpack27(const double* p, g7* g) {
    g7_zero(g);
    for (int a = 0; a < 6; ++a) g->eta[a] = p[a];
    for (int r = 0; r < 6; ++r)
        for (int cc = r; cc < 6; ++cc) {
            g->lam[r * 7 + cc] = p[6 + upper_index(r, cc)];
            g->lam[cc * 7 + r] = p[6 + upper_index(r, cc)];
        }
}

static int get_tree_state(const or_ctx* x, double* out) {
    for (int i = 0; i < x->N; ++i) {
        double* o = out + 42 * (size_t)i;
        for (int k = 0; k < 6; ++k) o[k] = x->tau[6 * (size_t)i + k];
        o[6] = x->ell[i];
        pack27(&x->pmsg[i], o + 7);
        for (int d = 0; d < 4; ++d) {
            const g7* g = &x->msg[8 * (size_t)i + 4 + d];
            o[34 + 2 * d] = g->eta[6];
            o[35 + 2 * d] = g->lam[48];
        }
    }
    double* nb = out + 42 * (size_t)x->N;
    for (int n = 0; n < x->NT; ++n) {
        double* o = nb + 141 * (size_t)n;
        for (int k = 0; k < 6; ++k) o[k] = x->ntau[6 * (size_t)n + k];
        for (int k = 0; k < 5; ++k) pack27(&x->nmsg[5 * (size_t)n + k], o + 6 + 27 * k);
    }
    return 0;
}

static int set_tree_state(or_ctx* x, const double* in) {
    for (int i = 0; i < x->N; ++i) {
        const double* o = in + 42 * (size_t)i;
        for (int k = 0; k < 6; ++k) x->tau[6 * (size_t)i + k] = o[k];
        x->ell[i] = o[6];
        unpack27(o + 7, &x->pmsg[i]);
        for (int d = 0; d < 4; ++d) {
            g7_zero(&x->msg[8 * (size_t)i + d]);
            g7* g = &x->msg[8 * (size_t)i + 4 + d];
            g7_zero(g);
            g->eta[6] = o[34 + 2 * d];
            g->lam[48] = o[35 + 2 * d];
        }
    }
    const double* nb = in + 42 * (size_t)x->N;
    for (int n = 0; n < x->NT; ++n) {
        const double* o = nb + 141 * (size_t)n;
        for (int k = 0; k < 6; ++k) x->ntau[6 * (size_t)n + k] = o[k];
        for (int k = 0; k < 5; ++k) unpack27(o + 6 + 27 * k, &x->nmsg[5 * (size_t)n + k]);
    }
    return 0;
}

int or_get_state(const or_ctx* x, double* out) {
    if (x->tree) return get_tree_state(x, out);
    for (int i = 0; i < x->N; ++i) {
        double* o = out + 123 * (size_t)i;
        for (int k = 0; k < 6; ++k) o[k] = x->tau[6 * (size_t)i + k];
        o[6] = x->ell[i];
        for (int d = 0; d < 4; ++d) {
            const g7* g = &x->msg[8 * (size_t)i + d];
            double* p = o + 7 + 27 * d;
            for (int a = 0; a < 6; ++a) p[a] = g->eta[a];
            for (int r = 0; r < 6; ++r)
                for (int cc = r; cc < 6; ++cc) p[6 + upper_index(r, cc)] = g->lam[r * 7 + cc];
        }
        for (int d = 0; d < 4; ++d) {
            const g7* g = &x->msg[8 * (size_t)i + 4 + d];
            o[115 + 2 * d] = g->eta[6];
            o[116 + 2 * d] = g->lam[48];
        }
    }
    return 0;
}

int or_set_state(or_ctx* x, const double* in) {
    if (x->tree) return set_tree_state(x, in);
    for (int i = 0; i < x->N; ++i) {
        const double* o = in + 123 * (size_t)i;
        for (int k = 0; k < 6; ++k) x->tau[6 * (size_t)i + k] = o[k];
        x->ell[i] = o[6];
        for (int d = 0; d < 4; ++d) {
            g7* g = &x->msg[8 * (size_t)i + d];
            g7_zero(g);
            const double* p = o + 7 + 27 * d;
            for (int a = 0; a < 6; ++a) g->eta[a] = p[a];
            for (int r = 0; r < 6; ++r)
                for (int cc = r; cc < 6; ++cc) {
                    g->lam[r * 7 + cc] = p[6 + upper_index(r, cc)];
                    g->lam[cc * 7 + r] = p[6 + upper_index(r, cc)];
                }
        }
        for (int d = 0; d < 4; ++d) {
            g7* g = &x->msg[8 * (size_t)i + 4 + d];
            g7_zero(g);
            g->eta[6] = o[115 + 2 * d];
            g->lam[48] = o[116 + 2 * d];
        }
    }
    return 0;
}

int or_tree_levels(const or_ctx* x, int* hw) {
    if (hw)
        for (int l = 0; l <= x->L; ++l) {
            hw[2 * l] = x->lvH[l];
            hw[2 * l + 1] = x->lvW[l];
        }
    return x->L;
}

int or_get_node_beliefs(const or_ctx* x, double* lam_out, double* eta_out) {
    for (int n = 0; n < x->NT; ++n) {
        if (lam_out) memcpy(lam_out + 49 * (size_t)n, x->nbelief[n].lam, sizeof(double) * 49);
        if (eta_out) memcpy(eta_out + 7 * (size_t)n, x->nbelief[n].eta, sizeof(double) * 7);
    }
    return 0;
}

int or_get_means(const or_ctx* x, double* out) {
    memcpy(out, x->mean, sizeof(double) * 7 * (size_t)x->N);
    return 0;
}

int or_get_beliefs(const or_ctx* x, double* lam_out, double* eta_out) {
    for (int i = 0; i < x->N; ++i) {
        if (lam_out) memcpy(lam_out + 49 * (size_t)i, x->belief[i].lam, sizeof(double) * 49);
        if (eta_out) memcpy(eta_out + 7 * (size_t)i, x->belief[i].eta, sizeof(double) * 7);
    }
    return 0;
}

int or_get_normal_targets(const or_ctx* x, double* cx_out, double* cy_out) {
    memcpy(cx_out, x->cxt, sizeof(double) * (size_t)x->N);
    memcpy(cy_out, x->cyt, sizeof(double) * (size_t)x->N);
    return 0;
}

/* prior factor means, Eq. (prior) and the log-depth prior of Sec. 3.3: the
 * pose mean for every pixel and, if given, a per-pixel log-depth mean (NULL
 * keeps the current ones). Temporal priors carry the previous frame's
 * estimates forward this way. */
int or_set_prior(or_ctx* x, const double xi[6], const double* log_depth) {
    if (!x) return -1;
    if (xi)
        for (int k = 0; k < 6; ++k) x->cfg.prior_xi[k] = xi[k];
    if (log_depth) memcpy(x->prior_ell, log_depth, sizeof(double) * (size_t)x->N);
    return 0;
}

/* the pose estimate of the last tracked frame (mean of the per-pixel poses)
 * and the current log-depths become the prior means */
int or_set_prior_from_state(or_ctx* x) {
    if (!x) return -1;
    double m[6] = {0, 0, 0, 0, 0, 0};
    for (int i = 0; i < x->N; ++i)
        for (int k = 0; k < 6; ++k) m[k] += x->tau[6 * (size_t)i + k];
    for (int k = 0; k < 6; ++k) x->cfg.prior_xi[k] = m[k] / (double)x->N;
    memcpy(x->prior_ell, x->ell, sizeof(double) * (size_t)x->N);
    return 0;
}

int or_get_gradients(const or_ctx* x, double* gx, double* gy) {
    memcpy(gx, x->Gx, sizeof(double) * (size_t)x->N);
    memcpy(gy, x->Gy, sizeof(double) * (size_t)x->N);
    return 0;
}

/* energy of the nonlinear model at the current linearisation points:
 * Huber photometric + prior + identity + normal terms, each 1/2 |r|^2_Lambda */
static void add_identity_energy(const double* ti, const double* tj, double lamR, double* E) {
    double Tj[16], Ti[16], Tji[16], Trel[16], r[6];
    or_se3_exp(ti, Ti);
    or_se3_exp(tj, Tj);
    se3_inverse(Tj, Tji);
    mat_mul(4, 4, 4, Tji, Ti, Trel);
    or_se3_log(Trel, r);
    for (int k = 0; k < 6; ++k) *E += 0.5 * lamR * r[k] * r[k];
}

static void add_prior_energy(const or_config* c, const double* ti, double lamP, double* E) {
    double Tp[16], Tpi[16], Tt[16], Tr[16], rp[6];
    or_se3_exp(c->prior_xi, Tp);
    se3_inverse(Tp, Tpi);
    or_se3_exp(ti, Tt);
    mat_mul(4, 4, 4, Tpi, Tt, Tr);
    or_se3_log(Tr, rp);
    for (int k = 0; k < 6; ++k) *E += 0.5 * lamP * rp[k] * rp[k];
}

double or_energy(const or_ctx* x) {
    const or_config* c = &x->cfg;
    const int W = c->W, H = c->H, N = x->N;
    double E = 0.0;
    const double lamR = 1.0 / (c->sigma_R * c->sigma_R);
    const double lamN = 1.0 / (c->sigma_N * c->sigma_N);
    const double lamP = 1.0 / (c->sigma_P * c->sigma_P);
    for (int i = 0; i < N; ++i) {
        const double* ti = x->tau + 6 * (size_t)i;
        int u = i % W, v = i / W;
        double w[2], Jw[14];
        if (x->have_frame && or_warp(x, u, v, ti, x->ell[i], w, Jw) &&
            w[0] >= -WARP_EPS && w[0] <= (W - 1) + WARP_EPS &&
            w[1] >= -WARP_EPS && w[1] <= (H - 1) + WARP_EPS) {
            double xx = fmin(fmax(w[0], 0.0), (double)(W - 1));
            double yy = fmin(fmax(w[1], 0.0), (double)(H - 1));
            double r = x->I_s[i] - bilinear(x->I_t, H, W, xx, yy);
            double M = fabs(r) / x->sigD[i];
            double k = c->huber_k;
            E += (M <= k) ? 0.5 * M * M : k * M - 0.5 * k * k;
        }
        add_prior_energy(c, ti, lamP, &E);
        double dl = x->ell[i] - x->prior_ell[i];
        E += 0.5 * lamP * dl * dl;
        if (x->tree)   /* quadtree edge to the parent */
            add_identity_energy(ti, x->ntau + 6 * (size_t)node_at(x, 1, u / 2, v / 2), lamR, &E);
        /* each edge once: towards the right and lower neighbours */
        for (int d = OR_RIGHT; d <= OR_DOWN; d += 2) {
            int j = neighbour(x, i, d);
            if (j < 0) continue;
            if (!x->tree) add_identity_energy(ti, x->tau + 6 * (size_t)j, lamR, &E);
            double ca = (d == OR_RIGHT) ? x->cxt[i] : x->cyt[i];
            if (isfinite(ca)) {
                double rn = x->ell[j] - x->ell[i] + ca;
                E += 0.5 * lamN * rn * rn;
            }
        }
    }
    /* quadtree nodes: level prior and the edge to the parent */
    for (int n = 0; n < x->NT; ++n) {
        const int l = node_level(x, n);
        const double* tn = x->ntau + 6 * (size_t)n;
        add_prior_energy(c, tn, level_lambda(c->sigma_P, l), &E);
        if (l < x->L) {
            const int col = (n - x->lvOff[l]) % x->lvW[l], row = (n - x->lvOff[l]) / x->lvW[l];
            add_identity_energy(tn, x->ntau + 6 * (size_t)node_at(x, l + 1, col / 2, row / 2),
                                level_lambda(c->sigma_R, l), &E);
        }
    }
    return E;
}
