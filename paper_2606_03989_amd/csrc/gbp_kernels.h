// Launchers of the GBP kernels (host-side declarations).
#pragma once

#include <hip/hip_runtime.h>

namespace pv {

struct Geo;
struct Strengths;
struct Inputs;
struct SeqDesc;
struct BatchLaunch;

// target frame and its gradients; `clear` (may be NULL) is set to 0 on the way
hipError_t launch_frame_prep(const Geo& g, const float* src, long src_pitch, float* It, float* Gx, float* Gy,
                             hipStream_t st, int* clear = nullptr);
hipError_t launch_keyframe_prep(const Geo& g, const float* img, const float* normals, float* Is, float* cxt,
                                float* cyt, float* X, float* X2, hipStream_t st);
hipError_t launch_init_state(const Geo& g, float* X, float ell0, hipStream_t st);
hipError_t launch_pf_iteration(const Geo& g, const Strengths& s, const Inputs& in, float* X, double* marg,
                               double* M, float* var_ll, float* valid, float beta, int* health, hipStream_t st);
hipError_t launch_fu_prologue(const Geo& g, const Strengths& s, const Inputs& in, const float* X, float* Y,
                              int* health, hipStream_t st);
hipError_t launch_fu_iterate(const Geo& g, const Strengths& s, const Inputs& in, const float* X, float* Y,
                             bool final_pass, float* var_ll, float* valid, int* health, hipStream_t st);
// the recompute of a checkpoint segment of len iterations from its canonical
// state X0, with the tape of every iteration k: the marginals (29 FP64 planes)
// followed by the belief they come from (35) at marg + k * marg_stride, the
// information of the new messages (88 FP32) at M + k * M_stride and the
// belief of the update (35 FP64) at bel + k * bel_stride. The canonical states
// after iterations 1 .. len - 1 go to seg + k * seg_stride; tA and tB are
// state-sized work buffers (tB receives the last canonical state). One
// prologue, len - 1 rotated passes (update of k and prologue of k + 1) and a
// final pass.
hipError_t launch_fu_segment_tape(const Geo& g, const Strengths& s, const Inputs& in, const float* X0, float* seg,
                                  long seg_stride, int len, float* tA, float* tB, double* marg, long marg_stride,
                                  float* M, long M_stride, double* bel, long bel_stride, float* var_ll, float* valid,
                                  int* health, hipStream_t st);
hipError_t launch_valid_only(const Geo& g, const Strengths& s, const Inputs& in, const float* X, float* valid,
                             hipStream_t st);
// statistics records of an image: one per 64 x 4 pixel tile
int stats_blocks(const Geo& g);
// result (9 doubles): the six pose sums, valid count, non-finite count, and
// the health flag *health when given
hipError_t launch_frame_stats(const Geo& g, const float* X, const float* valid, int use_valid, double* partial,
                              double* result, hipStream_t st, const int* health = nullptr);
hipError_t launch_outputs(const Geo& g, const float* X, const float* var_ll, int have_var, float* inv_depth,
                          float* inv_var, hipStream_t st);
hipError_t launch_pack_state(const Geo& g, const float* X, float* dense, int to_dense, hipStream_t st);
hipError_t launch_copy_plane(const Geo& g, const float* dense, float* plane, hipStream_t st);

// one frame step of a batch: clear health, frame prep, prologue, n passes,
// per-sequence statistics, keyframe test and re-anchoring (canonical state
// ends in buffer parity ^ (n > 0 ? (n + 1) & 1 : 0))
hipError_t launch_batch_frame_step(const BatchLaunch& b, int n_iters, hipStream_t st);
// p[0 .. n) = value
hipError_t launch_set_ints(int* p, int n, int value, hipStream_t st);
// keyframe test of the frame just tracked and, if b.reanchor, re-anchoring of
// the due sequences on it (canonical state in buffer `parity`)
hipError_t launch_batch_keyframe(const BatchLaunch& b, int parity, hipStream_t st);
// the same frame step with the iteration block as one persistent cooperative
// launch of grid_blocks workgroups (batch_persistent_grid: the co-resident
// maximum, a multiple of 8; 0 if it cannot be determined)
int batch_persistent_grid(const BatchLaunch& b);
hipError_t launch_batch_frame_step_persistent(const BatchLaunch& b, int n_iters, int grid_blocks, hipStream_t st);
// bare passes (autotuning and timing)
hipError_t launch_batch_passes(const BatchLaunch& b, int n_iters, bool prologue, bool final_last, hipStream_t st);

}  // namespace pv
