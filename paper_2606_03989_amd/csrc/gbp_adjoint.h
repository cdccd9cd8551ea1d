// Launchers of the reverse-sweep kernels (host-side declarations).
#pragma once

#include <hip/hip_runtime.h>

namespace pv {

struct Geo;
struct Strengths;
struct Inputs;

// cotangent added to each pixel's pose tangent (the pose output's cotangent
// divided by the pixel count)
struct PoseBar {
    double v[6];
};

// Cb: the slot-common cotangent of the stored messages (29 FP32 planes, a
// slot's layout: eta 6, Lambda 21, normal eta, normal lambda), added to every
// existing slot of Xb by its reader
// M: the tape of the new messages' information, LAM_STRIDE FP32 planes per slot
hipError_t launch_adj_update(const Geo& g, const Strengths& s, const Inputs& in, const float* X, const float* M,
                             const double* bel, const float* Xb, const float* Cb, float* Mb, float* Ub,
                             hipStream_t st);
hipError_t launch_adj_edges(const Geo& g, const Strengths& s, const Inputs& in, const float* X, const double* marg,
                            const float* M, const float* Mb, float* Xbo, float* Eb, double* gN, hipStream_t st);
hipError_t launch_adj_belief(const Geo& g, const Strengths& s, const Inputs& in, const float* X, const double* marg,
                             const float* Ub, const float* Eb, float* Xbo, float* Cbo, double* gsig, double* gk,
                             hipStream_t st);
hipError_t launch_adj_inject(const Geo& g, const float* Xend, float* Xb, const PoseBar& xb, const float* rhob,
                             hipStream_t st);
int sum2_blocks(const Geo& g);
hipError_t launch_sum2(const Geo& g, const double* a, const double* b, double* partial, double* result,
                       hipStream_t st);
hipError_t launch_plane_to_dense(const Geo& g, const double* src, float* dst, hipStream_t st);

}  // namespace pv
