/*
 * FP64 CPU oracle for per-pixel Gaussian Belief Propagation visual odometry
 * (PixVOD, arXiv 2606.03989).
 *
 * TEST INFRASTRUCTURE ONLY. This library is the parity authority that the GPU
 * path is checked against. Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product path never does.
 * It shares no code with the GPU library.
 *
 * What it computes (one synchronous GBP iteration, flooding schedule, Sec. 3.4
 * and Sec. 4.1 of the paper):
 *   L  linearise every pixel's unary factors at its linearisation point:
 *      photometric factor (Eq. distrb_photo, warp Eq. warp) with Huber
 *      covariance weighting, and the pose/log-depth prior (Eq. prior);
 *   B  belief = unary + all stored factor-to-variable messages;
 *   F  every factor-to-variable message is recomputed: the variable-to-factor
 *      message of the sender (its belief minus the factor's message to it) is
 *      combined with the linearised factor over both variables and the sender
 *      is marginalised out (dense Schur complement); identity factors
 *      (Eq. regul) couple the pose blocks of 4-neighbours, normal integration
 *      factors (Eq. gbpni) couple their log-depths;
 *   U  new belief, its mean in the tangent space, relinearisation of the
 *      variable at the mean (Eq. var) and first-order transport of the stored
 *      messages into the new tangent space (Sec. 4.1).
 * Per frame, after the iterations: the pose estimate is the mean of the
 * per-pixel poses (Eq. estimator_avg), the inverse-depth map exp(-log depth).
 *
 * Every 7-D Gaussian is stored in information form (eta, Lambda) over the
 * tangent vector [dtheta(3); drho(3); dlogdepth] at the pixel's current
 * linearisation point. Pose tangent ordering is [rotation; translation] with
 * Exp([theta; rho]) = [[R(theta), V(theta) rho], [0, 1]] (Eq. exp_err) and
 * perturbations applied on the right, T = Tbar * Exp(delta).
 */
#ifndef PIXVOD_ORACLE_H
#define PIXVOD_ORACLE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* neighbour directions; message slot d holds the message from the factor on
 * the edge towards the neighbour in direction d */
enum { OR_LEFT = 0, OR_RIGHT = 1, OR_UP = 2, OR_DOWN = 3 };

/* flags reported per frame */
enum { OR_KEYFRAME_DUE = 1u, OR_DIVERGED = 2u, OR_LOW_OVERLAP = 4u };

typedef struct {
    int H, W;
    double fx, fy, cx, cy;
    /* factor strengths: Lambda = sigma^-2 (Sec. 4.2); huber_k in whitened units */
    double sigma_D, sigma_P, sigma_R, sigma_N, huber_k;
    double init_inv_depth;            /* inverse depth of every pixel at creation */
    double prior_xi[6];               /* prior pose mean (identity by default) */
    double prior_log_depth;           /* prior log-depth mean (0 = depth 1) */
    int kf_max_frames;                /* re-anchoring: frame count limit */
    double kf_min_valid_frac;         /* re-anchoring: overlap limit */
    double damping;                   /* message damping beta, 0 = none */
    /* test switches */
    int frozen;                       /* never relinearise: linear GBP */
    int full_jacobian;                /* identity factor with exact Lie Jacobians */
    int topology;                     /* identity factors: OR_TOPO_GRID or OR_TOPO_QUADTREE */
    int store_fp32;                   /* storage emulation: every new message is rounded to
                                       * FP32 before the update uses it, and the linearisation
                                       * points and stored messages after every iteration */
} or_config;

/* identity-factor topologies (Sec. 3.3, Fig. 2): the 4-neighbour pixel grid,
 * or the quadtree of pose variables above the pixels, where each node of
 * level l >= 1 (a ceil(H/2^l) x ceil(W/2^l) array) joins the 2 x 2 block of
 * level l - 1 below it; sigma_P and sigma_R halve per level (Sec. 4.2) */
enum { OR_TOPO_GRID = 0, OR_TOPO_QUADTREE = 1 };

typedef struct {
    double xi[6];            /* mean over pixels of the pose tangent (Eq. estimator_avg) */
    double T_world[16];      /* row-major T_world<-current */
    double valid_fraction;   /* pixels whose warp landed in the image, last iteration */
    int frames_since_keyframe;
    unsigned flags;
} or_track_out;

typedef struct or_ctx or_ctx;

/* library-level; H >= 1 (a single row is a chain, used by the tree tests), W >= 2 */
void or_default_config(or_config* cfg);
or_ctx* or_create(const or_config* cfg);
void or_destroy(or_ctx* ctx);
int or_threads(void);
void or_set_threads(int n);

/* per-pixel sigma_D map (H*W); NULL restores the constant cfg.sigma_D */
int or_set_sigma_D_map(or_ctx* ctx, const double* sigma_map);

/* keyframe image (H*W) and its normals (H*W*3, keyframe camera frame).
 * Resets pose linearisation points to identity and all messages to zero;
 * log-depths are kept. */
int or_set_keyframe(or_ctx* ctx, const float* img, const float* normals);

/* one target frame (H*W), n_iters synchronous iterations; inv_depth and
 * inv_depth_var may be NULL (H*W doubles otherwise) */
int or_track(or_ctx* ctx, const float* frame, int n_iters, or_track_out* out,
             double* inv_depth, double* inv_depth_var);

/* keyframe depth transfer before re-anchoring on the frame just tracked: the
 * log-depths of the current keyframe are forward-warped into that frame with
 * its pose estimate (nearest-pixel splat, nearest depth wins, pixels nothing
 * lands on keep theirs); then call or_set_keyframe with the new keyframe.
 * -2 before a tracked frame. */
int or_transfer_depth(or_ctx* ctx);

/* double-precision image variants (exact synthetic constructions in tests) */
int or_set_keyframe64(or_ctx* ctx, const double* img, const float* normals);
int or_set_frame64(or_ctx* ctx, const double* frame);

/* iterations on the current frame without the per-frame bookkeeping */
int or_iterate(or_ctx* ctx, int n_iters);
/* stage a target frame (gradient images) without iterating */
int or_set_frame(or_ctx* ctx, const float* frame);

/* state in the exchange layout.
 * Grid: per pixel 123 doubles,
 * [tau(6), logdepth, 4 x (identity eta(6), Lambda upper-packed row-major(21)),
 *  4 x (normal eta, normal lambda)], pixels in row-major order.
 * Quadtree: per pixel 42 doubles [tau(6), logdepth, message of the edge to the
 * parent (eta 6, Lambda 21), 4 x (normal eta, lambda)], then per node of
 * levels 1..L (level-major, row-major within a level) 141 doubles [tau(6),
 * message of the edge to the parent (27; zero at the root), for child slot
 * q = 2 (y & 1) + (x & 1): message of the edge to that child (27; zero where
 * the child lies outside its level)]. Every message is the one the factor
 * sends to the variable that stores it. */
size_t or_state_doubles(const or_ctx* ctx);
int or_get_state(const or_ctx* ctx, double* out);
int or_set_state(or_ctx* ctx, const double* in);

/* prior means (Eq. prior; log-depth prior of Sec. 3.3): pose mean xi (NULL
 * keeps it) and per-pixel log-depth means (H*W, NULL keeps them) */
int or_set_prior(or_ctx* ctx, const double xi[6], const double* log_depth);
/* temporal priors: the mean of the current per-pixel poses and the current
 * log-depths become the prior means */
int or_set_prior_from_state(or_ctx* ctx);

/* frozen mode: per-pixel belief mean (7 doubles per pixel) of the last iteration */
int or_get_means(const or_ctx* ctx, double* out);
/* quadtree: number of node levels L above the pixels (0 for the grid) and,
 * if hw is not NULL, hw[2l], hw[2l+1] = rows, columns of level l = 0..L */
int or_tree_levels(const or_ctx* ctx, int* hw);
/* quadtree: last iteration's node beliefs (49 + 7 doubles per node, node
 * order of the exchange layout; the 7th coordinate is an inert placeholder) */
int or_get_node_beliefs(const or_ctx* ctx, double* lam_out, double* eta_out);

/* last iteration's belief information matrices (49 doubles per pixel) */
int or_get_beliefs(const or_ctx* ctx, double* lam_out, double* eta_out);
/* normal-integration targets (c_x, c_y per pixel; NaN = inactive edge) */
int or_get_normal_targets(const or_ctx* ctx, double* cx_out, double* cy_out);
/* central-difference gradient images of the staged frame */
int or_get_gradients(const or_ctx* ctx, double* gx_out, double* gy_out);
/* squared-whitened energy of the linearised-at-the-current-point model */
double or_energy(const or_ctx* ctx);

/* --- building blocks exposed for the pinning tests ----------------------- */
void or_se3_exp(const double xi[6], double T[16]);
void or_se3_log(const double T[16], double xi[6]);
void or_se3_jr(const double xi[6], double J[36]);          /* right Jacobian, power series */
void or_prior_jacobian(const double xi[6], double J[36]);  /* I + ad/2 + ad^2/12 */
double or_huber_weight(double M, double k);
/* warp of pixel (u,v) under (tau, logdepth): w, dw/d[delta(6), dlogdepth] (2x7 row-major);
 * returns 1 if a_z > 0 */
int or_warp(const or_ctx* ctx, double u, double v, const double tau[6], double ell,
            double w[2], double Jw[14]);
/* unary (photometric + prior) information of pixel (u,v) at the current state */
int or_unary(const or_ctx* ctx, int u, int v, double eta[7], double lam[49], int* valid);
/* generic factor-to-variable message: factor with m residuals r, Jacobian J
 * (m x 14 over [x_recv; x_send]) and diagonal precision prec; sender's
 * variable-to-factor message (eta_s, lam_s). Returns 0 on success. */
int or_factor_message(int m, const double* r, const double* J, const double* prec,
                      const double eta_s[7], const double lam_s[49],
                      double eta_out[7], double lam_out[49]);

#ifdef __cplusplus
}
#endif
#endif
