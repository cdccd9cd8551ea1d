// Keyframe depth transfer (PixVOD, arXiv 2606.03989: depth propagation of
// Sec. 3.3 at the re-anchoring of Sec. 3.5) for gfx950.
//
// Before the frame just tracked becomes the keyframe, every pixel's 3-D point
// exp(ell) q of the current keyframe is moved into that frame's camera by its
// pose estimate and splatted to the nearest pixel (rounding half up). A
// 32-bit atomicMin on the FP32 depth bits (positive floats order as unsigned
// integers) keeps the nearest point; a second pass turns the winners into
// log-depths and leaves the pixels nothing landed on as they were.
#include "gbp_transfer.h"
#include "gbp_device.hpp"

#include <mutex>

namespace pv {

namespace {

constexpr unsigned kInfBits = 0x7f800000u;

__global__ void k_tf_clear(Geo g, unsigned* __restrict__ zb) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    if (u >= g.W || v >= g.H) return;
    zb[pix_of(g, u, v)] = kInfBits;
}

__global__ void k_tf_splat(Geo g, Pose p, const float* __restrict__ X, unsigned* __restrict__ zb) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    if (u >= g.W || v >= g.H) return;
    const double d = exp((double)X[(long)P_ELL * g.plane + pix_of(g, u, v)]);
    const double P0 = d * ((double)u - g.cx) / g.fx, P1 = d * ((double)v - g.cy) / g.fy, P2 = d;
    const double Q0 = p.R[0] * P0 + p.R[1] * P1 + p.R[2] * P2 + p.t[0];
    const double Q1 = p.R[3] * P0 + p.R[4] * P1 + p.R[5] * P2 + p.t[1];
    const double Q2 = p.R[6] * P0 + p.R[7] * P1 + p.R[8] * P2 + p.t[2];
    if (!(Q2 > 0.0)) return;
    const double ju = floor(g.fx * Q0 / Q2 + g.cx + 0.5), jv = floor(g.fy * Q1 / Q2 + g.cy + 0.5);
    if (!(ju >= 0.0 && ju < (double)g.W && jv >= 0.0 && jv < (double)g.H)) return;
    const float z = (float)Q2;
    atomicMin(zb + pix_of(g, (int)ju, (int)jv), __float_as_uint(z));
}

__global__ void k_tf_gather(Geo g, const unsigned* __restrict__ zb, float* __restrict__ X) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    if (u >= g.W || v >= g.H) return;
    const long pi = pix_of(g, u, v);
    const unsigned b = zb[pi];
    if (b != kInfBits) X[(long)P_ELL * g.plane + pi] = (float)log((double)__uint_as_float(b));
}

std::mutex g_scratch_mutex;
unsigned* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

// z-buffer of the allocation-free re-anchoring entry point: each device holds
// its own copy for the process's lifetime, shared by every call on it. Host
// code uses the address looked up by transfer_scratch_init, never the name.
static __device__ __align__(256) unsigned scratch[kTransferScratchMax];

hipError_t transfer_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<unsigned*>(ptr);
    return hipSuccess;
}

unsigned* transfer_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    return g_scratch_ptr[device];
}

hipError_t launch_depth_transfer(const Geo& g, const Pose& p, float* X, unsigned* zbuf, hipStream_t st) {
    const dim3 b(64, 4), gr((g.W + 63) / 64, (g.H + 3) / 4);
    hipLaunchKernelGGL(k_tf_clear, gr, b, 0, st, g, zbuf);
    hipLaunchKernelGGL(k_tf_splat, gr, b, 0, st, g, p, X, zbuf);
    hipLaunchKernelGGL(k_tf_gather, gr, b, 0, st, g, zbuf, X);
    return hipGetLastError();
}

}  // namespace pv
