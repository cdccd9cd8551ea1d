/*
 * pixvod: per-pixel Gaussian Belief Propagation visual odometry and depth on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: PixVOD (arXiv 2606.03989). Every pixel holds a stacked variable of a
 * camera pose in SE(3) and a log-depth (Sec. 3.3). Its photometric factor
 * (Eq. distrb_photo) compares the keyframe intensity with the target frame
 * sampled at the warp of Eq. (warp); a prior factor (Eq. prior) anchors pose
 * and log-depth; camera-motion identity factors (Eq. regul) tie the poses of
 * 4-neighbours together, and normal-integration factors (Eq. gbpni) tie their
 * log-depths to a surface-normal map. Inference is synchronous Gaussian
 * Belief Propagation with relinearisation at the current means (Sec. 3.4,
 * Sec. 4.1) against a fixed keyframe (Sec. 3.5); the per-frame camera pose is
 * the mean of the per-pixel poses (App. C.2, Eq. estimator_avg).
 *
 * Conventions shared by every entry point:
 *   - Images are H x W row-major float32, pixel centres at integer (u, v).
 *   - A pose tangent is [theta(3); rho(3)] with
 *     Exp = [[R(theta), V(theta) rho], [0, 1]] (App. C.2, Eq. exp_err); the
 *     per-pixel pose maps keyframe-camera points into the current camera.
 *   - Every call returns a PIXVOD_* status; nothing throws across the ABI.
 *     Arguments are validated before any GPU work is issued.
 *   - Buffers passed in are owned by the caller. `where` says whether a
 *     pointer is host memory (PIXVOD_HOST) or device memory on the context's
 *     device (PIXVOD_DEVICE). Device pointers are used in stream order on the
 *     context's stream.
 *   - A context is used by one thread at a time; there is no internal locking.
 *   - Numerical divergence is reported as a flag, not as an error.
 */
#ifndef PIXVOD_H
#define PIXVOD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
enum {
    PIXVOD_OK = 0,
    PIXVOD_EINVAL = -1,   /* invalid argument */
    PIXVOD_ESTATE = -2,   /* call not valid in the context's current state */
    PIXVOD_EHIP = -3,     /* a HIP runtime call failed */
    PIXVOD_ENOMEM = -4,   /* device allocation failed */
    PIXVOD_ENODEV = -5    /* no usable gfx950 device */
};

/* memory location of a buffer argument */
enum { PIXVOD_HOST = 0, PIXVOD_DEVICE = 1 };

/* per-frame flags */
enum {
    PIXVOD_KEYFRAME_DUE = 1u,  /* re-anchoring test fired (Sec. 3.5) */
    PIXVOD_DIVERGED = 2u,      /* non-finite state or a non-positive pivot */
    PIXVOD_LOW_OVERLAP = 4u    /* valid-warp fraction below kf_min_valid_frac */
};

/* iteration schedules; both compute the same synchronous iteration */
enum {
    PIXVOD_SCHED_FUSED = 0,       /* one pass over the state per iteration */
    PIXVOD_SCHED_PER_FACTOR = 1   /* one kernel per GBP step */
};

/* camera-motion identity topologies (Sec. 3.3, Fig. 2) */
enum {
    PIXVOD_TOPO_GRID = 0,       /* identity factors between 4-neighbour pixels */
    PIXVOD_TOPO_QUADTREE = 1    /* hierarchical quadtree of pose variables */
};

typedef struct pixvod_ctx pixvod_ctx;

/* pinhole intrinsics in pixels */
typedef struct {
    float fx, fy, cx, cy;
} pixvod_intrinsics;

/* Factor strengths (Sec. 4.2: Lambda = sigma^-2 I, Huber threshold in
 * whitened units) and tracking parameters. pixvod_default_params() fills the
 * paper's leaf-level values (5e-3, 1, 4e-4, 1e-3, 400). */
typedef struct {
    float sigma_D;             /* photometric noise (intensity units) */
    float sigma_P;             /* pose / log-depth prior */
    float sigma_R;             /* camera-motion identity factor */
    float sigma_N;             /* normal-integration factor */
    float huber_k;             /* Huber threshold on the whitened residual */
    float init_inv_depth;      /* inverse depth of every pixel at creation */
    float prior_xi[6];         /* prior pose mean (identity by default) */
    float prior_log_depth;     /* prior log-depth mean (0 = depth 1) */
    int32_t kf_max_frames;     /* re-anchoring: frames per keyframe */
    float kf_min_valid_frac;   /* re-anchoring: minimum overlap */
    float damping;             /* message damping beta; only the per-factor
                                * schedule supports beta != 0 */
} pixvod_params;

/* result of one tracked frame */
typedef struct {
    double xi_rel[6];          /* mean per-pixel pose, T_current<-keyframe */
    double T_world[16];        /* row-major T_world<-current =
                                * T_world<-keyframe * Exp(xi_rel)^-1 */
    float* inv_depth;          /* caller buffer (H*W) or NULL: exp(-log depth) */
    float* inv_depth_var;      /* caller buffer (H*W) or NULL: delta-method
                                * variance of the inverse depth from the final
                                * belief; NaN when n_iters == 0 */
    int32_t out_where;         /* PIXVOD_HOST / PIXVOD_DEVICE for the two maps */
    float valid_fraction;      /* pixels whose warp landed in the image during
                                * the last iteration */
    int32_t frames_since_keyframe;
    uint32_t flags;            /* PIXVOD_KEYFRAME_DUE | DIVERGED | LOW_OVERLAP */
} pixvod_track_out;

/* Fills the paper's default parameters (Sec. 4.2) with init_inv_depth 1,
 * kf_max_frames 150, kf_min_valid_frac 0.5, damping 0. */
void pixvod_default_params(pixvod_params* params);

/* Creates a context for H x W frames (H, W >= 2; fx, fy > 0) on the current
 * HIP device. params == NULL selects the defaults. All device state is owned
 * by the context: 123 float32 planes per pixel (pose 6, log-depth 1, four
 * identity messages of 27 values and four normal messages of 2 values) in
 * two ping-pong copies, plus the keyframe and frame inputs. Returns
 * PIXVOD_ENODEV without a usable GPU, PIXVOD_ENOMEM if allocation fails. */
int pixvod_create(int H, int W, const pixvod_intrinsics* K, const pixvod_params* params,
                  pixvod_ctx** out_ctx);

/* Releases every device allocation of the context. NULL is accepted. */
int pixvod_destroy(pixvod_ctx* ctx);

/* Uses `hip_stream` (a hipStream_t, e.g. torch's current stream) for all
 * later work; NULL restores the context's own stream. */
int pixvod_set_stream(pixvod_ctx* ctx, void* hip_stream);

/* Selects PIXVOD_SCHED_FUSED (default) or PIXVOD_SCHED_PER_FACTOR.
 * PIXVOD_EINVAL for the fused schedule when params.damping != 0. */
int pixvod_set_schedule(pixvod_ctx* ctx, int schedule);

/* Identity-factor topology (Sec. 3.3; the hierarchy of Fig. 2 with the
 * per-level strengths of Sec. 4.2). PIXVOD_TOPO_GRID (default) ties each pixel
 * pose to its 4 neighbours. PIXVOD_TOPO_QUADTREE adds levels l = 1..L of 6-D
 * pose variables, level l a ceil(H/2^l) x ceil(W/2^l) array ending in one
 * root; each node is tied by an identity factor to the up to four variables
 * of the 2 x 2 block below it (pixels at level 1) and carries a pose prior.
 * The prior of level l has sigma_P 2^-l, the identity factor between levels l
 * and l + 1 has sigma_R 2^-l (params.sigma_P and sigma_R are the leaf
 * values); the lateral pixel identity factors are dropped, the photometric,
 * prior and normal-integration factors stay. The pose estimate remains the
 * mean of the pixel poses (Eq. estimator_avg). Device memory: 141 float32
 * planes per node (pose 6, the message of the edge to the parent 27, the
 * messages of the four child edges 4 x 27) in two copies, about 0.33 nodes per
 * pixel. Quadtree contexts run the fused schedule only (damping 0).
 * PIXVOD_ESTATE after the first pixvod_set_keyframe; PIXVOD_EINVAL for the
 * per-factor schedule or damping. */
int pixvod_set_topology(pixvod_ctx* ctx, int topology);

/* Level sizes: *n_levels = L + 1 (1 for the grid); hw (2 * (L + 1) ints, may
 * be NULL) receives rows, columns of levels 0 (pixels) .. L (root). */
int pixvod_tree_levels(const pixvod_ctx* ctx, int* n_levels, int* hw);

/* Keyframe anchoring (Sec. 3.5): `img` (H*W) becomes the reference image and
 * `normals` (H*W*3, unit normals in the keyframe camera frame) define the
 * normal-integration targets of Eq. (gbpni). Pose linearisation points are
 * reset to identity and every message to zero; log-depths are kept. After a
 * tracked frame, the world pose of the keyframe becomes that frame's world
 * pose (re-anchoring on the frame just tracked). */
int pixvod_set_keyframe(pixvod_ctx* ctx, const float* img, const float* normals, int where);

/* Re-anchoring with depth transfer (depth propagation, Sec. 3.3): as
 * pixvod_set_keyframe, but first the current log-depths are forward-warped
 * into the frame just tracked, which `img` should be: each keyframe pixel's
 * 3-D point exp(log depth) q is moved by the last pose estimate
 * (Eq. estimator_avg) and splatted to the nearest pixel (rounding half up);
 * the nearest depth (compared at FP32) wins, and pixels no point lands on keep
 * their log-depth. One extra H x W plane is allocated on first use.
 * PIXVOD_ESTATE before a tracked frame. */
int pixvod_set_keyframe_transfer(pixvod_ctx* ctx, const float* img, const float* normals, int where);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * re-anchoring with depth transfer as pixvod_set_keyframe_transfer, with the
 * same arguments and results, but its z-buffer is a static device array of
 * 2^21 entries that each GPU holds for the lifetime of the process instead of
 * a plane allocated on first use; nothing is allocated, and with device
 * pointers (PIXVOD_DEVICE) nothing is copied through the host either.
 * PIXVOD_EINVAL when H times the row pitch (W rounded up to a multiple of 64)
 * exceeds 2^21 (1920 x 1080 fits); PIXVOD_ESTATE before a tracked frame.
 * Every context on a GPU shares that GPU's array: calls on one GPU that
 * overlap in time (different streams or threads) race. */
int pixvod_set_keyframe_transfer_noalloc(pixvod_ctx* ctx, const float* img, const float* normals, int where);

/* Optional per-pixel photometric sigma map (H*W); NULL restores the constant
 * params.sigma_D. */
int pixvod_set_sigma_map(pixvod_ctx* ctx, const float* sigma_D_map, int where);

/* Tracks one target frame (H*W): n_iters >= 0 synchronous GBP iterations
 * warm-started from the previous frame's state (Sec. 4.3), then the pose
 * estimate, output maps, keyframe test and flags. Returns after the pose is
 * on the host; device output maps are written in stream order.
 * With pixvod_set_graph enabled, the fused schedule on the grid topology
 * captures the frame step (prologue, n_iters passes, frame reductions) once
 * as a HIP graph per starting state buffer and replays it; it is captured
 * again whenever a kernel argument changes (parameters, bound maps, n_iters,
 * profiling). Results are identical to launching the passes one by one.
 * PIXVOD_ESTATE before the first pixvod_set_keyframe. */
int pixvod_track(pixvod_ctx* ctx, const float* frame, int where, int n_iters,
                 pixvod_track_out* out);

/* Prior means (Eq. prior; the log-depth prior of Sec. 3.3). xi: the pose mean
 * of every pixel's prior factor (6 doubles, host; NULL keeps the current one);
 * log_depth: per-pixel log-depth prior means (H*W floats at `where`; NULL keeps
 * the current ones, initially params.prior_log_depth everywhere). A new
 * keyframe returns the pose mean to params.prior_xi and keeps the log-depth
 * means. */
int pixvod_set_prior(pixvod_ctx* ctx, const double xi[6], const float* log_depth, int where);

/* Temporal priors (motion continuity and depth propagation, Sec. 3.3): the
 * last tracked frame's pose estimate and the current per-pixel log-depths
 * become the prior means for the next frames. ESTATE before the first frame
 * tracked on the current keyframe. */
int pixvod_set_prior_from_state(pixvod_ctx* ctx);

/* Runs n_iters iterations on the last staged frame without per-frame
 * bookkeeping (benchmarks and tests). */
int pixvod_iterate(pixvod_ctx* ctx, int n_iters);

/* State exchange: 123 planes of H*W float32 in plane-major order
 * [pose 0..5, log-depth, for d in {left, right, up, down}: identity message
 * eta(6) + Lambda upper-packed row-major(21), for d: normal eta, lambda].
 * Slot d of pixel i holds the message from the factor on the edge towards
 * the neighbour in direction d; slots of edges that leave the image are 0.
 * Quadtree contexts: 42 planes of H*W [pose 0..5, log-depth, message of the
 * edge to the parent (eta 6, Lambda 21), for d: normal eta, lambda], then 141
 * planes of NT nodes (levels 1..L in order, row-major within a level)
 * [pose 0..5, message of the edge to the parent (27; zero at the root), for
 * child slot q = 2 (y & 1) + (x & 1): message of that child's edge (27; zero
 * for a child outside its level)]. Every message is the one its factor sends
 * to the variable that stores it. pixvod_state_bytes gives the size. */
int pixvod_state_bytes(const pixvod_ctx* ctx, size_t* bytes);
int pixvod_get_state(pixvod_ctx* ctx, void* dst, int where);
int pixvod_set_state(pixvod_ctx* ctx, const void* src, int where);

/* Kernel timing for benchmarks. With profiling enabled, the context records
 * a HIP event pair on its stream around each run of consecutive launches of
 * one pass kind below (per frame: the prologue, the n_iters - 1 fused passes,
 * the last pass; all per-factor iterations); pixvod_profile_read() waits for
 * the stream, returns the summed duration in milliseconds and the launch
 * count of one pass kind, and resets that kind. Durations of a run include
 * the gaps between its launches. */
enum {
    PIXVOD_PROF_FUSED_ITERATE = 0,    /* one fused iteration pass (not the last of a frame) */
    PIXVOD_PROF_FUSED_FINAL = 1,      /* the last fused pass of a frame */
    PIXVOD_PROF_FUSED_PROLOGUE = 2,   /* the per-frame prologue of the fused schedule */
    PIXVOD_PROF_PER_FACTOR = 3,       /* one per-factor iteration (three kernels) */
    PIXVOD_PROF_KINDS = 4
};
int pixvod_profile_enable(pixvod_ctx* ctx, int enable);
/* With profiling enabled, replayed frame steps time their passes with event
 * nodes captured in the graph; where the runtime cannot capture them the
 * frame steps of a profiled context launch their passes one by one. */

/* enable != 0: pixvod_track replays the captured frame step; 0 (default):
 * every pass is launched on its own. */
int pixvod_set_graph(pixvod_ctx* ctx, int enable);
int pixvod_profile_read(pixvod_ctx* ctx, int kind, double* total_ms, int64_t* launches);

/* ---------------------------------------------------------------------------
 * Batches: many independent sequences of mixed resolution advanced together.
 * Every pass of the fused schedule is one launch over a work list of
 * (sequence, tile) items; a frame step (frame preparation, prologue, n_iters
 * passes, per-sequence reductions) is captured once as a HIP graph and
 * replayed. Per-pixel arithmetic is the single-sequence code and the pose
 * sums are reduced over the same fixed 64 x 4 pixel tiles in the same order
 * as in a single context, so results (states, pose means, world poses) are
 * identical to per-sequence contexts and independent of the tile shape.
 * All sequences share one parameter set and the fused schedule (damping 0).
 */
typedef struct pixvod_batch pixvod_batch;

/* n >= 1 sequences with sizes H[i] x W[i] (>= 2) and intrinsics K[i]. */
int pixvod_batch_create(int n, const int* H, const int* W, const pixvod_intrinsics* K,
                        const pixvod_params* params, pixvod_batch** out_batch);
int pixvod_batch_destroy(pixvod_batch* b);
int pixvod_batch_set_stream(pixvod_batch* b, void* hip_stream);

/* Keyframes for m listed sequences (seq_ids[k], images imgs[k], normals
 * normals[k]), with the semantics of pixvod_set_keyframe. */
int pixvod_batch_set_keyframes(pixvod_batch* b, int m, const int* seq_ids, const float* const* imgs,
                               const float* const* normals, int where);

/* One frame per sequence (frames[i], H[i]*W[i]); n_iters >= 1 iterations for
 * all sequences; outs[i] receives sequence i's result (maps written when its
 * pointers are set). Requires every sequence to have a keyframe. */
int pixvod_batch_track(pixvod_batch* b, const float* const* frames, int where, int n_iters,
                       pixvod_track_out* outs);

/* As pixvod_batch_track, and inside the same frame step the keyframe test
 * (Sec. 3.5) runs on the device: every sequence whose test fires on the frame
 * just tracked is re-anchored on it by a kernel predicated on that sequence's
 * device flag, as pixvod_set_keyframe would (the frame becomes the keyframe
 * image, normals[i] (H[i]*W[i]*3, unit normals in that frame's camera) give
 * the normal-integration targets, pose linearisation points and messages
 * reset, log-depths kept, the keyframe's world pose becomes the frame's).
 * outs[i].flags carries PIXVOD_KEYFRAME_DUE for the re-anchored sequences;
 * the maps are those of the frame just tracked. Device frames and normals
 * (PIXVOD_DEVICE) are read in place until the call returns. */
int pixvod_batch_track_reanchor(pixvod_batch* b, const float* const* frames, const float* const* normals,
                                int where, int n_iters, pixvod_track_out* outs);

/* Runs the iteration block of each frame step (prologue and n_iters passes)
 * as one persistent cooperative launch with a grid-wide barrier between the
 * passes (enable = 1) instead of one captured launch per pass (0, default).
 * Results are identical; the grid is the co-resident maximum for the tile. */
int pixvod_batch_set_persistent(pixvod_batch* b, int enable);

/* Tile shape of the work list (tile_x * tile_y <= 256, both >= 1). */
int pixvod_batch_set_tile(pixvod_batch* b, int tile_x, int tile_y);

/* Times every candidate tile shape on n_iters passes over the current frames
 * (the state is restored afterwards), selects the fastest and returns it. */
int pixvod_batch_autotune(pixvod_batch* b, int n_iters, int* tile_x, int* tile_y);

/* Average duration (ms) of the last frame step, timed with HIP events. */
int pixvod_batch_last_step_ms(pixvod_batch* b, double* ms);

/* Per-sequence state in the exchange layout of pixvod_get_state; set_state
 * replaces sequence seq's canonical state (its keyframe and frame counter are
 * kept). */
int pixvod_batch_get_state(pixvod_batch* b, int seq, void* dst, int where);
int pixvod_batch_set_state(pixvod_batch* b, int seq, const void* src, int where);

/* ---------------------------------------------------------------------------
 * Differentiation: unrolled tracking with a hand-written adjoint.
 * A forward pass runs n_frames target frames of one keyframe with n_iters
 * synchronous iterations each (per-factor semantics, fused kernels), starting
 * every time from the state set by pixvod_unroll_set_keyframe: pose
 * linearisation points at the identity, messages zero, log-depth
 * -log(init_inv_depth). No re-anchoring happens inside the unroll. It records
 * the canonical state every ckpt_every iterations (and at every frame start)
 * on a device tape. The outputs per frame are the pose estimate xi (mean of
 * the per-pixel pose tangents, Eq. estimator_avg) and the inverse-depth map.
 * The backward pass walks the tape in reverse: for each checkpoint segment it
 * recomputes the segment's states, then runs the reverse of every iteration
 * (vector-Jacobian products of the marginals, the message step with its
 * Schur complements, the update with its relinearisation and transport, and
 * the photometric and prior factors), and returns the gradient of
 *   sum_f xi_bar[f] . xi[f] + sum_f sum_i inv_depth_bar[f][i] inv_depth[f][i]
 * with respect to the per-pixel photometric sigma map (Eq. distrb_photo), the
 * normal-integration sigma (Eq. gbpni) and the Huber threshold. Any loss of
 * the outputs is handled by passing its output cotangents. Stored FP32
 * roundings are differentiated as the identity and discrete decisions (valid
 * warp window, Huber branch, interpolation cell) as constants.
 * The unroll always uses a sigma map; damping must be 0.
 */
typedef struct pixvod_unroll pixvod_unroll;

/* H, W >= 2; 1 <= n_iters; 1 <= ckpt_every; 1 <= max_frames. Device memory
 * holds max_frames * ceil(n_iters / ckpt_every) checkpoints of the state
 * (123 * H * W floats each, rows padded to 64 floats) and ckpt_every states of
 * one recomputed segment. */
int pixvod_unroll_create(int H, int W, const pixvod_intrinsics* K, const pixvod_params* params, int max_frames,
                         int n_iters, int ckpt_every, pixvod_unroll** out_unroll);
int pixvod_unroll_destroy(pixvod_unroll* u);
int pixvod_unroll_set_stream(pixvod_unroll* u, void* hip_stream);

/* keyframe image (H*W) and normals (H*W*3), as pixvod_set_keyframe */
int pixvod_unroll_set_keyframe(pixvod_unroll* u, const float* img, const float* normals, int where);

/* Replaces the state the forward passes start from (after
 * pixvod_unroll_set_keyframe, which resets it) with `state` in the exchange
 * layout of pixvod_get_state (123 * H * W floats at `where`); the keyframe is
 * kept. A forward pass from a given state makes the reverse sweep of a few
 * iterations comparable with differences of the same iterations from the
 * same state. PIXVOD_ESTATE before a keyframe. */
int pixvod_unroll_set_state(pixvod_unroll* u, const float* state, int where);

/* frames: n_frames * H * W (1 <= n_frames <= max_frames), copied; sigma_map:
 * H * W photometric sigmas (> 0); sigma_N > 0 and huber_k > 0 replace the
 * creation parameters. xi_out (host, n_frames * 6 doubles) and inv_depth_out
 * (n_frames * H * W floats at out_where) may be NULL. */
int pixvod_unroll_forward(pixvod_unroll* u, const float* frames, int n_frames, int where, const float* sigma_map,
                          int sigma_where, double sigma_N, double huber_k, double* xi_out, float* inv_depth_out,
                          int out_where);

/* Cotangents of the last forward's outputs: xi_bar (host, n_frames * 6) and
 * inv_depth_bar (n_frames * H * W at `where`), either may be NULL (zero).
 * Gradients: grad_sigma_map (H * W floats at grad_where, may be NULL),
 * grad_sigma_N and grad_huber_k (host doubles, may be NULL). Needs a forward
 * pass since the last keyframe; may be called several times per forward. */
int pixvod_unroll_backward(pixvod_unroll* u, const double* xi_bar, const float* inv_depth_bar, int where,
                           float* grad_sigma_map, int grad_where, double* grad_sigma_N, double* grad_huber_k);

/* Durations (ms, HIP events on the stream) of the last forward and backward. */
int pixvod_unroll_last_ms(const pixvod_unroll* u, double* forward_ms, double* backward_ms);

/* ---------------------------------------------------------------------------
 * Centralised baseline: direct tracking with every pixel accessible at once
 * (Sec. 3.1, Eq. photo), solved by IRLS Gauss-Newton as the paper's
 * centralised comparison (Sec. 4.4). Unknowns: one global pose xi (right
 * perturbation) and a log-depth per keyframe pixel. The energy is Eq. (photo)
 * with the per-pixel model's factors at exact consensus: photometric factors
 * with the Huber covariance weighting frozen at the current residuals, each
 * pixel's log-depth prior, the normal-integration factors and one prior
 * factor on the pose; there are no identity factors. Each IRLS iteration solves the Gauss-Newton normal equations
 * (6 + H*W unknowns; the depth block is diagonal plus sigma_N^-2 times the
 * graph Laplacian of the active normal edges) by preconditioned conjugate
 * gradients in FP64 (block-Jacobi: the 6x6 pose block and the depth
 * diagonal) until the residual norm falls below cg_tol times its initial
 * value or max_cg iterations, then sets xi <- Log(Exp(xi) Exp(d_xi)),
 * ell <- ell + d_ell. Parameters as pixvod_params (sigma_R unused; a constant
 * sigma_D). Device memory: 17 FP64 and 6 FP32 planes of H x W.
 */
typedef struct pixvod_central pixvod_central;

typedef struct {
    int32_t cg_iters;          /* CG iterations over the call's IRLS iterations */
    int32_t last_cg_iters;     /* those of the last IRLS iteration */
    double last_rel_residual;  /* its final residual norm / initial norm */
    float valid_fraction;      /* pixels whose warp landed in the image (last linearisation) */
    uint32_t flags;            /* PIXVOD_DIVERGED for a non-finite pose */
} pixvod_central_stats;

/* H, W >= 2, H*W <= 2^26; max_cg >= 1; 0 < cg_tol < 1. The initial point is
 * the identity pose and log-depth -log(params.init_inv_depth). */
int pixvod_central_create(int H, int W, const pixvod_intrinsics* K, const pixvod_params* params, int max_cg,
                          double cg_tol, pixvod_central** out);
int pixvod_central_destroy(pixvod_central* c);
int pixvod_central_set_stream(pixvod_central* c, void* hip_stream);
/* keyframe image (H*W) and normals (H*W*3); the pose restarts at the
 * identity, log-depths are kept */
int pixvod_central_set_keyframe(pixvod_central* c, const float* img, const float* normals, int where);
/* current point: xi (6 doubles, host) and log-depths (H*W doubles, host,
 * row-major); either may be NULL */
int pixvod_central_set_point(pixvod_central* c, const double xi[6], const double* log_depth);
int pixvod_central_get_point(pixvod_central* c, double xi[6], double* log_depth);
/* n_iters >= 0 IRLS iterations on `frame` (H*W) from the current point
 * (warm start); xi_out (host, may be NULL), inv_depth (H*W at out_where, may
 * be NULL), stats (may be NULL). ESTATE before a keyframe. Synchronous: the
 * host reads the CG stop test between chunks of 16 CG iterations on the
 * solver's stream. */
int pixvod_central_track(pixvod_central* c, const float* frame, int where, int n_iters, double xi_out[6],
                         float* inv_depth, int out_where, pixvod_central_stats* stats);
/* duration (ms, HIP events) of the last call's IRLS iterations */
int pixvod_central_last_ms(const pixvod_central* c, double* ms);

/* Per-context message of the last failure; ctx == NULL gives the last
 * failure of a call that had no context (e.g. pixvod_create). */
const char* pixvod_last_error(const pixvod_ctx* ctx);

/* Library version string. */
const char* pixvod_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PIXVOD_H */
