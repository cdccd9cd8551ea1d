// Keyframe depth transfer by forward warping (host-side declarations).
#pragma once

#include <hip/hip_runtime.h>

namespace pv {

struct Geo;

// rotation (row-major) and translation of Exp(xi): keyframe points to the
// camera of the frame just tracked
struct Pose {
    double R[9];
    double t[3];
};

// forward-warps the log-depth plane of the state X in place; zbuf is one
// pitched plane of scratch
hipError_t launch_depth_transfer(const Geo& g, const Pose& p, float* X, unsigned* zbuf, hipStream_t st);

}  // namespace pv
