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

// The allocation-free variant's z-buffer: a device array of
// kTransferScratchMax entries (8 MiB, room for a 1920 x 1080 frame's pitched
// plane) that lives as long as the process. transfer_scratch_init(device),
// called with that device current, looks up its address once per device;
// transfer_scratch(device) returns it (nullptr before the lookup).
constexpr long kTransferScratchMax = 1L << 21;
constexpr int kMaxDevices = 64;
hipError_t transfer_scratch_init(int device);
unsigned* transfer_scratch(int device);

}  // namespace pv
