// Per-pixel GBP algebra for gfx950, FP64 in registers.
//
// Method: PixVOD (arXiv 2606.03989). Storage is FP32 structure-of-arrays
// planes; every per-pixel 6x6 / 7x7 solve, marginalisation and message is
// evaluated in double precision (the information matrices span ~1 .. 1e8).
//
// Tangent ordering [theta(3); rho(3); logdepth], Exp of Eq. (exp_err),
// perturbations on the right (Eq. var), information form (eta, Lambda).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pv {

// ---------------------------------------------------------------------------
// plane indices of the 123-plane state
constexpr int P_TAU = 0;                 // 6 planes
constexpr int P_ELL = 6;
constexpr int P_MID = 7;                 // 4 x 27: eta(6) + upper-packed Lambda(21)
constexpr int P_MN = 115;                // 4 x 2: eta, lambda
constexpr int N_PLANES = 123;
constexpr int MID_STRIDE = 27;
constexpr int LAM_STRIDE = 22;           // reverse-sweep tape per slot: Lambda 21, normal lambda

enum { DIR_L = 0, DIR_R = 1, DIR_U = 2, DIR_D = 3 };

__host__ __device__ constexpr int opposite(int d) { return d ^ 1; }
__host__ __device__ constexpr int s6(int r, int c) {
    return r <= c ? r * 6 - r * (r - 1) / 2 + (c - r) : c * 6 - c * (c - 1) / 2 + (r - c);
}
__host__ __device__ constexpr int s7(int r, int c) {
    return r <= c ? r * 7 - r * (r - 1) / 2 + (c - r) : c * 7 - c * (c - 1) / 2 + (r - c);
}

// ---------------------------------------------------------------------------
// frame geometry and factor strengths, passed by value to every kernel
struct Geo {
    int H, W;
    int pitch;            // floats per row of every plane
    long plane;           // floats per plane (H * pitch)
    double fx, fy, cx, cy;
};

struct Strengths {
    double lamP;          // prior
    double lamR;          // identity
    double lamN;          // normal integration
    double lamD;          // photometric, used when no sigma map is bound
    double inv_sigD;      // 1 / sigma_D, likewise
    double huber_k;
    double prior_ell;
    double prior_R[9];    // Exp(prior_xi)^-1 rotation
    double prior_t[3];    // Exp(prior_xi)^-1 translation
    int prior_is_identity;
    int has_sigma_map;
    int has_prior_map;    // per-pixel log-depth prior means (in.prior_ell)
};

// inputs that stay fixed for a keyframe / a frame
struct Inputs {
    const float* Is;      // keyframe image
    const float* cxt;     // normal targets towards the right neighbour
    const float* cyt;     // normal targets towards the lower neighbour
    const float* sigD;    // per-pixel sigma_D (valid if has_sigma_map)
    const float* It;      // target frame
    const float* Gx;      // its central-difference gradients
    const float* Gy;
    const float* prior_ell;   // per-pixel log-depth prior mean (valid if has_prior_map)
};

// one sequence of a batch (device-resident descriptor)
struct SeqDesc {
    Geo g;
    Inputs in;
    float* X0;            // state ping-pong copies
    float* X1;
    float* var_ll;
    float* valid;
    const float* frame;   // dense target frame (H * W) of the current step
    const float* normals; // its normal map (H * W * 3), for re-anchoring on it
    float* It;            // frame-prep outputs (same planes as in.It, in.Gx, in.Gy)
    float* Gx;
    float* Gy;
    float* Is;            // keyframe-prep outputs (same planes as in.Is, in.cxt, in.cyt)
    float* cxt;
    float* cyt;
    int tile_base;        // natural index of the sequence's first work item
    int tiles_x;          // tiles per image row
    int n_tiles;
    int stat_base;        // first of the sequence's statistics records (one per 64 x 4 tile)
};

// arguments of the batched launches
struct BatchLaunch {
    const SeqDesc* seqs;  // device array, n_seq entries
    const int2* work;     // device array: (natural item index, sequence) per workgroup
    int n_work;
    int n_seq;
    int tile_x, tile_y;
    int parity;           // buffer holding the canonical state
    Strengths s;
    int* health;
    double* partial;      // 8 doubles per 64 x 4 statistics tile of every sequence
    int max_stat_tiles;   // statistics tiles of the largest image
    double* result;       // 8 doubles per sequence
    // keyframe test and re-anchoring on the device (Sec. 3.5)
    int* fsk;             // per sequence: frames tracked since its keyframe
    unsigned* flags;      // per sequence: flags of the frame just tracked
    int kf_max_frames;
    float kf_min_valid;
    int reanchor;         // re-anchor due sequences on the frame just tracked
};

// ---------------------------------------------------------------------------
// SE(3)

__device__ inline void skew_mul(const double w[3], const double v[3], double out[3]) {
    out[0] = w[1] * v[2] - w[2] * v[1];
    out[1] = w[2] * v[0] - w[0] * v[2];
    out[2] = w[0] * v[1] - w[1] * v[0];
}

// 1/x and 1/sqrt(x) in double precision: the hardware estimate refined by two
// Newton steps (quadratic convergence from the ~2^-22 estimate to rounding)
__device__ inline double rcp_nr(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

__device__ inline double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    double e = fma(-h * y, y, 0.5);
    y = fma(y, e, y);
    e = fma(-h * y, y, 0.5);
    return fma(y, e, y);
}

// R = I + A W + B W^2 and V = I + B W + C W^2 with W = [theta]x
__device__ inline void se3_exp(const double xi[6], double R[9], double t[3]) {
    const double w0 = xi[0], w1 = xi[1], w2 = xi[2];
    const double th2 = w0 * w0 + w1 * w1 + w2 * w2;
    double A, B, C;
    if (th2 < 1e-2) {
        const double t4 = th2 * th2, t6 = t4 * th2, t8 = t4 * t4;
        A = 1.0 - th2 * (1.0 / 6.0) + t4 * (1.0 / 120.0) - t6 * (1.0 / 5040.0) + t8 * (1.0 / 362880.0);
        B = 0.5 - th2 * (1.0 / 24.0) + t4 * (1.0 / 720.0) - t6 * (1.0 / 40320.0) + t8 * (1.0 / 3628800.0);
        C = 1.0 / 6.0 - th2 * (1.0 / 120.0) + t4 * (1.0 / 5040.0) - t6 * (1.0 / 362880.0) + t8 * (1.0 / 39916800.0);
    } else {
        const double th = sqrt(th2);
        double s, c;
        sincos(th, &s, &c);
        const double sh = sin(0.5 * th);
        A = s / th;
        B = 2.0 * sh * sh / th2;
        C = (th - s) / (th2 * th);
    }
    // W^2 = w w^T - th2 I
    const double W2[9] = {w0 * w0 - th2, w0 * w1, w0 * w2,
                          w1 * w0, w1 * w1 - th2, w1 * w2,
                          w2 * w0, w2 * w1, w2 * w2 - th2};
    const double Wm[9] = {0.0, -w2, w1, w2, 0.0, -w0, -w1, w0, 0.0};
    double V[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double I = (k % 4 == 0) ? 1.0 : 0.0;
        R[k] = I + A * Wm[k] + B * W2[k];
        V[k] = I + B * Wm[k] + C * W2[k];
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) t[r] = V[r * 3] * xi[3] + V[r * 3 + 1] * xi[4] + V[r * 3 + 2] * xi[5];
}

// theta / sin(theta) as a series in s^2 = sin^2(theta), valid for cos > 0:
// asin(s)/s = sum_k (2k)! / (4^k (k!)^2 (2k+1)) s^(2k); truncation < 2e-18
// for s <= 0.1
__device__ inline double asin_over_s(double s2) {
    double p = 143.0 / 10240.0;
    p = fma(p, s2, 231.0 / 13312.0);
    p = fma(p, s2, 63.0 / 2816.0);
    p = fma(p, s2, 35.0 / 1152.0);
    p = fma(p, s2, 5.0 / 112.0);
    p = fma(p, s2, 3.0 / 40.0);
    p = fma(p, s2, 1.0 / 6.0);
    return fma(p, s2, 1.0);
}

// w = Log(R); th2 receives theta^2
__device__ inline void so3_log(const double R[9], double w[3], double& th2) {
    const double v0 = R[7] - R[5], v1 = R[2] - R[6], v2 = R[3] - R[1];
    const double s2 = 0.25 * (v0 * v0 + v1 * v1 + v2 * v2);     // sin^2(theta)
    const double c = 0.5 * (R[0] + R[4] + R[8] - 1.0);          // cos(theta)
    if (s2 < 1e-2 && c > 0.0) {
        const double g = asin_over_s(s2);                       // theta / sin(theta)
        th2 = s2 * g * g;
        const double f = 0.5 * g;
        w[0] = f * v0;
        w[1] = f * v1;
        w[2] = f * v2;
        return;
    }
    const double s = sqrt(s2);
    const double th = atan2(s, c);
    th2 = th * th;
    if (th < 3.14149265358979) {
        const double f = th / (2.0 * s);
        w[0] = f * v0;
        w[1] = f * v1;
        w[2] = f * v2;
        return;
    }
    // near pi: axis from the diagonal (not reached by tracking motions); the
    // largest diagonal entry k picks the column, by selects rather than a
    // computed index so that R stays in registers
    double n[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double d = (R[i * 4] + 1.0) * 0.5;
        n[i] = sqrt(d > 0.0 ? d : 0.0);
    }
    const int k = (n[0] >= n[1] && n[0] >= n[2]) ? 0 : (n[1] >= n[2] ? 1 : 2);
    const double nk = (k == 0) ? n[0] : (k == 1 ? n[1] : n[2]);
    double m[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        // (R[i][k] + R[k][i]) / (4 n_k) for i != k
        const double rik = (k == 0) ? R[i * 3] : (k == 1 ? R[i * 3 + 1] : R[i * 3 + 2]);
        const double rki = (k == 0) ? R[i] : (k == 1 ? R[3 + i] : R[6 + i]);
        m[i] = (i == k) ? n[i] : (rik + rki) / (4.0 * nk);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) n[i] = m[i];
    double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    if (n[0] * v0 + n[1] * v1 + n[2] * v2 < 0.0) nn = -nn;
    w[0] = th * n[0] / nn;
    w[1] = th * n[1] / nn;
    w[2] = th * n[2] / nn;
}

// xi = Log([R | t]); translation part rho = V^-1 t, V^-1 = I - W/2 + D W^2
__device__ inline void se3_log(const double R[9], const double t[3], double xi[6]) {
    double th2;
    so3_log(R, xi, th2);
    double D;
    if (th2 < 1e-2) {
        const double t4 = th2 * th2, t6 = t4 * th2, t8 = t4 * t4;
        D = 1.0 / 12.0 + th2 * (1.0 / 720.0) + t4 * (1.0 / 30240.0) + t6 * (1.0 / 1209600.0) +
            t8 * (1.0 / 47900160.0);
    } else {
        const double th = sqrt(th2), sh = sin(0.5 * th);
        D = (1.0 - th * sin(th) / (4.0 * sh * sh)) / th2;
    }
    double wt[3], wwt[3];
    skew_mul(xi, t, wt);
    skew_mul(xi, wt, wwt);
    xi[3] = t[0] - 0.5 * wt[0] + D * wwt[0];
    xi[4] = t[1] - 0.5 * wt[1] + D * wwt[1];
    xi[5] = t[2] - 0.5 * wt[2] + D * wwt[2];
}

// [Ro | to] = [Ra | ta] * [Rb | tb]
__device__ inline void se3_compose(const double Ra[9], const double ta[3], const double Rb[9],
                                   const double tb[3], double Ro[9], double to[3]) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
            Ro[r * 3 + c] = Ra[r * 3] * Rb[c] + Ra[r * 3 + 1] * Rb[3 + c] + Ra[r * 3 + 2] * Rb[6 + c];
        to[r] = Ra[r * 3] * tb[0] + Ra[r * 3 + 1] * tb[1] + Ra[r * 3 + 2] * tb[2] + ta[r];
    }
}

// Log([Rj | tj]^-1 [Ri | ti]): the identity-factor residual of Eq. (regul)
__device__ inline void se3_between(const double Rj[9], const double tj[3], const double Ri[9],
                                   const double ti[3], double r[6]) {
    double R[9], t[3], d[3] = {ti[0] - tj[0], ti[1] - tj[1], ti[2] - tj[2]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int c = 0; c < 3; ++c) R[a * 3 + c] = Rj[a] * Ri[c] + Rj[3 + a] * Ri[3 + c] + Rj[6 + a] * Ri[6 + c];
        t[a] = Rj[a] * d[0] + Rj[3 + a] * d[1] + Rj[6 + a] * d[2];
    }
    se3_log(R, t, r);
}

// ---------------------------------------------------------------------------
// small symmetric linear algebra, packed upper storage

// in-place LDL^T-free Cholesky of a packed 6x6 SPD matrix; A <- L (lower in the
// same packed slots, L(r,c) stored at s6(c,r)); returns false on a
// non-positive pivot. inv_diag receives 1/L(k,k).
__device__ inline bool chol6(double A[21], double inv_diag[6]) {
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double d = A[s6(j, j)];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= A[s6(j, k)] * A[s6(j, k)];
        ok = ok && (d > 0.0);
        const double dd = d > 0.0 ? d : 1e-300;
        const double il = rsqrt_nr(dd);
        A[s6(j, j)] = dd * il;
        inv_diag[j] = il;
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            double s = A[s6(i, j)];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= A[s6(i, k)] * A[s6(j, k)];
            A[s6(i, j)] = s * il;
        }
    }
    return ok;
}

__device__ inline void chol6_solve(const double L[21], const double inv_diag[6], double b[6]) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double s = b[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L[s6(i, k)] * b[k];
        b[i] = s * inv_diag[i];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        double s = b[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) s -= L[s6(k, i)] * b[k];
        b[i] = s * inv_diag[i];
    }
}

// inverse of the SPD matrix from its Cholesky factor: Ainv (packed) = L^-T L^-1
__device__ inline void chol6_inverse(const double L[21], const double inv_diag[6], double Ai[21]) {
    // X = L^-1 (lower triangular), packed the same way as L
    double X[21];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        X[s6(j, j)] = inv_diag[j];
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            double s = 0.0;
#pragma unroll
            for (int k = j; k < i; ++k) s -= L[s6(i, k)] * X[s6(k, j)];
            X[s6(i, j)] = s * inv_diag[i];
        }
    }
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = r; c < 6; ++c) {
            double s = 0.0;
#pragma unroll
            for (int k = c; k < 6; ++k) s += X[s6(k, r)] * X[s6(k, c)];
            Ai[s6(r, c)] = s;
        }
}

__device__ inline bool chol7(double A[28], double inv_diag[7]) {
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        double d = A[s7(j, j)];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= A[s7(j, k)] * A[s7(j, k)];
        ok = ok && (d > 0.0);
        const double dd = d > 0.0 ? d : 1e-300;
        const double il = rsqrt_nr(dd);
        A[s7(j, j)] = dd * il;
        inv_diag[j] = il;
#pragma unroll
        for (int i = j + 1; i < 7; ++i) {
            double s = A[s7(i, j)];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= A[s7(i, k)] * A[s7(j, k)];
            A[s7(i, j)] = s * il;
        }
    }
    return ok;
}

__device__ inline void chol7_solve(const double L[28], const double inv_diag[7], double b[7]) {
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        double s = b[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L[s7(i, k)] * b[k];
        b[i] = s * inv_diag[i];
    }
#pragma unroll
    for (int i = 6; i >= 0; --i) {
        double s = b[i];
#pragma unroll
        for (int k = i + 1; k < 7; ++k) s -= L[s7(k, i)] * b[k];
        b[i] = s * inv_diag[i];
    }
}

// [A^-1]_66 from the Cholesky factor: |L^-T e_6|^2 = 1 / L66^2 (last row of L^-1
// has a single entry in its last column)
__device__ inline double chol7_var_last(const double inv_diag[7]) { return inv_diag[6] * inv_diag[6]; }

// ---------------------------------------------------------------------------
// photometric and prior factors

__device__ inline float plane_at(const float* p, const Geo& g, int u, int v) {
    return p[(long)v * g.pitch + u];
}

constexpr double WARP_EPS = 1e-3;

// per-pixel inputs of the unary factors: keyframe intensity, photometric sigma
// (when a map is bound) and log-depth prior mean (when a map is bound)
struct PixelInputs {
    float Is, sigD, prior_ell;
};

__device__ inline PixelInputs load_pixel_inputs(const Geo& g, const Strengths& s, const Inputs& in, int u, int v) {
    const long pix = (long)v * g.pitch + u;
    PixelInputs r;
    r.Is = in.Is[pix];
    r.sigD = s.has_sigma_map ? in.sigD[pix] : 0.0f;
    r.prior_ell = s.has_prior_map ? in.prior_ell[pix] : 0.0f;
    return r;
}

// The photometric factor of pixel (u, v) (Eq. distrb_photo, warp of Eq. warp,
// Huber covariance weighting) at the linearisation point (R, t) = Exp(tau),
// ell, as the pieces that enter a belief: the 1 x 7 Jacobian J, the weight
// w = kappa lamD and the residual r; valid is the valid-warp flag (an invalid
// warp leaves the factor out).
struct Photo {
    double J[7];
    double w, r;
    bool valid;
};

// The factor in two halves, so that a caller can put independent work
// between the sample loads and their use: photometric_begin computes the
// warp and issues the twelve bilinear-sample loads (at clamped addresses,
// also for an invalid warp, whose values are then unused), photometric_end
// forms the factor. photometric() is the two in a row.
struct PhotoPre {
    double q0, q1, rho, a0, a1, iz, fx, fy;
    float s[12];           // I_t, G_x, G_y at the four corners (o, o + 1, o + pitch, o + pitch + 1)
    bool valid;
};

__device__ inline PhotoPre photometric_begin(const Geo& g, const Inputs& in, int u, int v, const double R[9],
                                             const double t[3], double ell) {
    PhotoPre p;
    p.q0 = ((double)u - g.cx) / g.fx;
    p.q1 = ((double)v - g.cy) / g.fy;
    p.rho = exp(-ell);
    p.a0 = R[0] * p.q0 + R[1] * p.q1 + R[2] + p.rho * t[0];
    p.a1 = R[3] * p.q0 + R[4] * p.q1 + R[5] + p.rho * t[1];
    const double a2 = R[6] * p.q0 + R[7] * p.q1 + R[8] + p.rho * t[2];
    p.iz = rcp_nr(a2 > 0.0 ? a2 : 1.0);
    const double wx = g.fx * p.a0 * p.iz + g.cx, wy = g.fy * p.a1 * p.iz + g.cy;
    p.valid = a2 > 0.0 && wx >= -WARP_EPS && wx <= (g.W - 1) + WARP_EPS && wy >= -WARP_EPS &&
              wy <= (g.H - 1) + WARP_EPS;
    const double x = p.valid ? fmin(fmax(wx, 0.0), (double)(g.W - 1)) : 0.0;
    const double y = p.valid ? fmin(fmax(wy, 0.0), (double)(g.H - 1)) : 0.0;
    int x0 = (int)floor(x), y0 = (int)floor(y);
    x0 = x0 > g.W - 2 ? g.W - 2 : (x0 < 0 ? 0 : x0);
    y0 = y0 > g.H - 2 ? g.H - 2 : (y0 < 0 ? 0 : y0);
    p.fx = x - x0;
    p.fy = y - y0;
    const long o = (long)y0 * g.pitch + x0;
    const long o2 = o + g.pitch;
    const long off[4] = {o, o + 1, o2, o2 + 1};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        p.s[c] = in.It[off[c]];
        p.s[4 + c] = in.Gx[off[c]];
        p.s[8 + c] = in.Gy[off[c]];
    }
    return p;
}

// SEL: formed without branches (an invalid warp's pieces are computed from
// its clamped samples and replaced by zeros, the Huber weight chosen by a
// select), which lets the caller's independent work be scheduled under the
// sample loads; the values are those of the branchy form.
template <bool SEL = false>
__device__ inline Photo photometric_end(const PhotoPre& p, const Geo& g, const Strengths& s, const double R[9],
                                        const double t[3], const PixelInputs& pin) {
    Photo f;
    f.valid = false;
    f.w = 0.0;
    f.r = 0.0;
#pragma unroll
    for (int a = 0; a < 7; ++a) f.J[a] = 0.0;
    if (!SEL && !p.valid) return f;
    f.valid = true;
    const double fx = p.fx, fy = p.fy, iz = p.iz, rho = p.rho, q0 = p.q0, q1 = p.q1;
    const double It = (1.0 - fy) * ((1.0 - fx) * p.s[0] + fx * p.s[1]) + fy * ((1.0 - fx) * p.s[2] + fx * p.s[3]);
    const double gx = (1.0 - fy) * ((1.0 - fx) * p.s[4] + fx * p.s[5]) + fy * ((1.0 - fx) * p.s[6] + fx * p.s[7]);
    const double gy = (1.0 - fy) * ((1.0 - fx) * p.s[8] + fx * p.s[9]) + fy * ((1.0 - fx) * p.s[10] + fx * p.s[11]);
    f.r = (double)pin.Is - It;
    // c = -g^T dw/da  (row 3-vector)
    const double c0 = -gx * g.fx * iz, c1 = -gy * g.fy * iz;
    const double c2 = (gx * g.fx * p.a0 + gy * g.fy * p.a1) * iz * iz;
    // J_theta = c.(-R [q]x d) = -(R^T c).(q x d) = -((R^T c) x q).d with b = R^T c
    const double b0 = R[0] * c0 + R[3] * c1 + R[6] * c2;
    const double b1 = R[1] * c0 + R[4] * c1 + R[7] * c2;
    const double b2 = R[2] * c0 + R[5] * c1 + R[8] * c2;
    f.J[0] = -(b1 * 1.0 - b2 * q1);
    f.J[1] = -(b2 * q0 - b0 * 1.0);
    f.J[2] = -(b0 * q1 - b1 * q0);
    f.J[3] = rho * b0;
    f.J[4] = rho * b1;
    f.J[5] = rho * b2;
    f.J[6] = -rho * (c0 * t[0] + c1 * t[1] + c2 * t[2]);
    const double isig = s.has_sigma_map ? rcp_nr((double)pin.sigD) : s.inv_sigD;
    const double lamD = isig * isig;
    const double M = fabs(f.r) * isig;
    double kappa = 1.0;
    if constexpr (SEL) {
        const double iM = rcp_nr(M > s.huber_k ? M : 1.0);
        kappa = (M > s.huber_k) ? s.huber_k * iM * (2.0 - s.huber_k * iM) : 1.0;
    } else if (M > s.huber_k) {
        const double iM = rcp_nr(M);
        kappa = s.huber_k * iM * (2.0 - s.huber_k * iM);
    }
    f.w = kappa * lamD;
    if constexpr (SEL) {
        const bool ok = p.valid;
        f.valid = ok;
#pragma unroll
        for (int a = 0; a < 7; ++a) f.J[a] = ok ? f.J[a] : 0.0;
        f.w = ok ? f.w : 0.0;
        f.r = ok ? f.r : 0.0;
    }
    return f;
}

template <bool SEL = false>
__device__ inline Photo photometric(const Geo& g, const Strengths& s, const Inputs& in, int u, int v,
                                    const double R[9], const double t[3], double ell, const PixelInputs& pin) {
    return photometric_end<SEL>(photometric_begin(g, in, u, v, R, t, ell), g, s, R, t, pin);
}

// L += w J^T J, eta -= w J r for a valid photometric factor (SEL: an invalid
// factor, zero from photometric_end<true>, adds exact zeros)
template <bool SEL = false>
__device__ inline void add_photometric(const Photo& f, double L[28], double eta[7]) {
    if (!SEL && !f.valid) return;
#pragma unroll
    for (int a = 0; a < 7; ++a) {
        const double wJa = f.w * f.J[a];
        eta[a] -= wJa * f.r;
#pragma unroll
        for (int b = a; b < 7; ++b) L[s7(a, b)] += wJa * f.J[b];
    }
}

// Adds the prior factor (Eq. prior) at the linearisation point tau,
// (R, t) = Exp(tau), ell to (L, eta).
__device__ inline void add_prior(const Strengths& s, const double tau[6], const double R[9], const double t[3],
                                 double ell, const PixelInputs& pin, double L[28], double eta[7]) {
    // --- prior: r = [Log(Exp(prior)^-1 Exp(tau)); ell - prior_ell],
    //     J = blockdiag(I + ad/2 + ad^2/12, 1)
    double rp[6];
    if (s.prior_is_identity) {
#pragma unroll
        for (int k = 0; k < 6; ++k) rp[k] = tau[k];
    } else {
        double Rr[9], tr[3];
        se3_compose(s.prior_R, s.prior_t, R, t, Rr, tr);
        se3_log(Rr, tr, rp);
    }
    // J = [[S, 0], [Q, S]] with, for rp = (w, q), W = [w]x, P = [q]x and
    // [a]x [b]x = b a^T - (a.b) I:
    //   S = I + W/2 + W^2/12 = I + W/2 + (w w^T - |w|^2 I)/12,
    //   Q = P/2 + (PW + WP)/12 = P/2 + (w q^T + q w^T - 2 (w.q) I)/12
    double S[9], Q[9];
    {
        const double w0 = rp[0], w1 = rp[1], w2 = rp[2], p0 = rp[3], p1 = rp[4], p2 = rp[5];
        const double w[3] = {w0, w1, w2}, q[3] = {p0, p1, p2};
        const double Wm[9] = {0.0, -w2, w1, w2, 0.0, -w0, -w1, w0, 0.0};
        const double Pm[9] = {0.0, -p2, p1, p2, 0.0, -p0, -p1, p0, 0.0};
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
    // J^T J = [[S^T S + Q^T Q, Q^T S], [S^T Q, S^T S]],
    // J^T rp = [S^T rp_w + Q^T rp_q; S^T rp_q]
    const double lamP = s.lamP;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double e0 = 0.0, e1 = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            e0 += S[k * 3 + a] * rp[k] + Q[k * 3 + a] * rp[3 + k];
            e1 += S[k * 3 + a] * rp[3 + k];
        }
        eta[a] -= lamP * e0;
        eta[3 + a] -= lamP * e1;
#pragma unroll
        for (int b = a; b < 3; ++b) {
            double ss = 0.0, qq = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                ss += S[k * 3 + a] * S[k * 3 + b];
                qq += Q[k * 3 + a] * Q[k * 3 + b];
            }
            L[s7(a, b)] += lamP * (ss + qq);
            L[s7(3 + a, 3 + b)] += lamP * ss;
        }
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            double qs = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) qs += Q[k * 3 + a] * S[k * 3 + b];
            L[s7(a, 3 + b)] += lamP * qs;
        }
    }
    const double pell = s.has_prior_map ? (double)pin.prior_ell : s.prior_ell;
    eta[6] -= lamP * (ell - pell);
    L[s7(6, 6)] += lamP;
}

// the unary belief (photometric + prior) from a photometric factor's pieces
template <bool SEL = false>
__device__ inline void unary_from(const Strengths& s, const Photo& f, const double tau[6], const double R[9],
                                  const double t[3], double ell, const PixelInputs& pin, double L[28],
                                  double eta[7]) {
#pragma unroll
    for (int k = 0; k < 28; ++k) L[k] = 0.0;
#pragma unroll
    for (int k = 0; k < 7; ++k) eta[k] = 0.0;
    add_photometric<SEL>(f, L, eta);
    add_prior(s, tau, R, t, ell, pin, L, eta);
}

// (L, eta) = photometric + prior factors of pixel (u, v) at tau, ell; returns
// the valid-warp flag
template <bool SEL = false>
__device__ inline bool unary_factors(const Geo& g, const Strengths& s, const Inputs& in, int u, int v,
                                     const double tau[6], const double R[9], const double t[3],
                                     double ell, const PixelInputs& pin, double L[28], double eta[7]) {
    const Photo f = photometric<SEL>(g, s, in, u, v, R, t, ell, pin);
    unary_from<SEL>(s, f, tau, R, t, ell, pin, L, eta);
    return f.valid;
}

template <bool SEL = false>
__device__ inline bool unary_factors(const Geo& g, const Strengths& s, const Inputs& in, int u, int v,
                                     const double tau[6], const double R[9], const double t[3],
                                     double ell, double L[28], double eta[7]) {
    return unary_factors<SEL>(g, s, in, u, v, tau, R, t, ell, load_pixel_inputs(g, s, in, u, v), L, eta);
}

// ---------------------------------------------------------------------------
// marginals of a pixel belief

// pose marginal (depth eliminated): P = L_pp - L_p6 L_6p / L_66
__device__ inline void pose_marginal(const double L[28], const double eta[7], double P[21], double p[6]) {
    const double i66 = rcp_nr(L[s7(6, 6)]);
#pragma unroll
    for (int r = 0; r < 6; ++r) {
        const double lr = L[s7(r, 6)] * i66;
        p[r] = eta[r] - lr * eta[6];
#pragma unroll
        for (int c = r; c < 6; ++c) P[s6(r, c)] = L[s7(r, c)] - lr * L[s7(c, 6)];
    }
}

// depth marginal (pose eliminated): D = L_66 - L_6p L_pp^-1 L_p6
__device__ inline bool depth_marginal(const double L[28], const double eta[7], double& D, double& dv) {
    double A[21], idg[6], y[6], z[6];
#pragma unroll
    for (int r = 0; r < 6; ++r) {
#pragma unroll
        for (int c = r; c < 6; ++c) A[s6(r, c)] = L[s7(r, c)];
        y[r] = L[s7(r, 6)];
        z[r] = eta[r];
    }
    const bool ok = chol6(A, idg);
    chol6_solve(A, idg, y);
    chol6_solve(A, idg, z);
    double sy = 0.0, sz = 0.0;
#pragma unroll
    for (int r = 0; r < 6; ++r) {
        sy += L[s7(r, 6)] * y[r];
        sz += y[r] * eta[r];
    }
    D = L[s7(6, 6)] - sy;
    dv = eta[6] - sz;
    return ok;
}

// ---------------------------------------------------------------------------
// grid access

__device__ inline long pix_of(const Geo& g, int u, int v) { return (long)v * g.pitch + u; }

__device__ inline bool neighbour(const Geo& g, int u, int v, int d, int& nu, int& nv) {
    nu = u + (d == DIR_L ? -1 : (d == DIR_R ? 1 : 0));
    nv = v + (d == DIR_U ? -1 : (d == DIR_D ? 1 : 0));
    return nu >= 0 && nu < g.W && nv >= 0 && nv < g.H;
}

__device__ inline void load_point(const float* __restrict__ X, const Geo& g, long p, double tau[6], double& ell) {
#pragma unroll
    for (int k = 0; k < 6; ++k) tau[k] = (double)X[(P_TAU + k) * g.plane + p];
    ell = (double)X[P_ELL * g.plane + p];
}

// normal-integration target and the residual seen by a receiver at pixel i
// whose neighbour j lies in direction d; false if the edge is inactive.
// Eq. (gbpni): r = (ell_b - ell_a) + c_a with a the left/upper pixel.
__device__ inline bool normal_residual(const Geo& g, const Inputs& in, long pi, long pj, int d,
                                       double ell_i, double ell_j, double& r_recv) {
    float c;
    double sgn;
    if (d == DIR_L) { c = in.cxt[pj]; sgn = 1.0; }         // a = j, b = i
    else if (d == DIR_R) { c = in.cxt[pi]; sgn = -1.0; }   // a = i, b = j
    else if (d == DIR_U) { c = in.cyt[pj]; sgn = 1.0; }
    else { c = in.cyt[pi]; sgn = -1.0; }
    if (!isfinite(c)) return false;
    // receiver's Jacobian is +1 when it is b: r_recv = (ell_b - ell_a + c) * (+1 if b)
    r_recv = (sgn > 0.0) ? (ell_i - ell_j + (double)c) : (ell_i - ell_j - (double)c);
    return true;
}

__device__ inline bool normal_active(const Geo& g, const Inputs& in, long pi, long pj, int d) {
    float c = (d == DIR_L) ? in.cxt[pj] : (d == DIR_R) ? in.cxt[pi] : (d == DIR_U) ? in.cyt[pj] : in.cyt[pi];
    return isfinite(c);
}

__device__ inline void load_messages(const float* __restrict__ X, const Geo& g, long p, float mid[4][27],
                                     float mn[4][2]) {
#pragma unroll
    for (int d = 0; d < 4; ++d) {
#pragma unroll
        for (int k = 0; k < 27; ++k) mid[d][k] = X[(long)(P_MID + d * MID_STRIDE + k) * g.plane + p];
        mn[d][0] = X[(long)(P_MN + 2 * d) * g.plane + p];
        mn[d][1] = X[(long)(P_MN + 2 * d + 1) * g.plane + p];
    }
}

// B += messages (embedded: identity -> pose block, normal -> depth entry)
__device__ inline void add_messages(double L[28], double eta[7], const float mid[4][27], const float mn[4][2]) {
#pragma unroll
    for (int d = 0; d < 4; ++d) {
#pragma unroll
        for (int a = 0; a < 6; ++a) eta[a] += (double)mid[d][a];
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
            for (int c = r; c < 6; ++c) L[s7(r, c)] += (double)mid[d][6 + s6(r, c)];
    }
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        eta[6] += (double)mn[d][0];
        L[s7(6, 6)] += (double)mn[d][1];
    }
}

// ---------------------------------------------------------------------------
// factor-to-variable messages, split into the part the sender computes from
// its variable-to-factor message (the "partial", independent of the
// receiver's linearisation point) and the receiver's completion with the
// factor residual at both linearisation points.
//
// Identity factor (Eq. regul) with Jacobians +I / -I: for the sender's
// variable-to-factor pose marginal (V, v) and A = lamR I + V,
//   Lambda' = lamR I - lamR^2 A^-1,   h = lamR A^-1 v,   eta' = h - Lambda' r.
// A^-1 comes from symmetric Gauss-Jordan elimination (the sweep operator on
// each pivot in turn), which leaves -A^-1 in the packed storage; every pivot
// is a Schur complement of A, so a non-positive one means A is not SPD.
__device__ inline bool sweep6_neg_inverse(double A[21]) {
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double D = A[s6(k, k)];
        ok = ok && (D > 0.0);
        const double iD = rcp_nr(D > 0.0 ? D : 1e-300);
        double r[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) r[i] = (i == k) ? 0.0 : A[s6(i, k)] * iD;
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j = i; j < 6; ++j)
                if (i != k && j != k) A[s6(i, j)] = fma(-A[s6(i, k)], r[j], A[s6(i, j)]);
#pragma unroll
        for (int i = 0; i < 6; ++i)
            if (i != k) A[s6(i, k)] = r[i];
        A[s6(k, k)] = -iD;
    }
    return ok;
}

__device__ inline bool identity_partial(double lamR, double V[21], const double v[6], double Lp[21],
                                        double h[6]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) V[s6(k, k)] += lamR;
    const bool ok = sweep6_neg_inverse(V);          // V <- -A^-1
    const double l2 = lamR * lamR;
#pragma unroll
    for (int r = 0; r < 6; ++r) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < 6; ++c) s = fma(V[s6(r, c)], v[c], s);
        h[r] = -lamR * s;
#pragma unroll
        for (int c = r; c < 6; ++c) Lp[s6(r, c)] = fma(l2, V[s6(r, c)], r == c ? lamR : 0.0);
    }
    return ok;
}

// Normal-integration factor (Eq. gbpni): sender's depth marginal (ls, vs),
//   lambda' = lamN ls / (lamN + ls),  h = lamN vs / (lamN + ls),
//   eta' = h - lambda' r_recv with r_recv the residual as seen by the receiver.
__device__ inline void normal_partial(double lamN, double ls, double vs, double& lp, double& h) {
    const double inv = rcp_nr(lamN + ls);
    lp = lamN * ls * inv;
    h = lamN * vs * inv;
}

}  // namespace pv
