// Quadtree identity topology (PixVOD, arXiv 2606.03989, Fig. 2, Sec. 3.3,
// Sec. 4.2): host-side geometry and launchers.
//
// Level 0 is the pixel array; level l >= 1 holds ceil(H / 2^l) x ceil(W / 2^l)
// 6-D pose nodes, node (x, y) joined by an identity factor (Eq. regul) to each
// existing node (2x + a, 2y + b), a, b in {0, 1}, of level l - 1 (child slot
// q = 2b + a), up to the single root at level L. Every node carries a pose
// prior (Eq. prior). sigma_P and sigma_R halve per level: the prior of level l
// has sigma_P 2^-l, the identity factor between levels l and l + 1 has
// sigma_R 2^-l. Pixels keep their photometric, prior and normal-integration
// factors; the identity factor to their level-1 parent replaces the four
// lateral ones.
#pragma once

#include <hip/hip_runtime.h>

namespace pv {

struct Geo;
struct Strengths;
struct Inputs;

constexpr int kTreeMaxLevels = 24;

// pixel planes of the quadtree state (inside the 123-plane pixel buffers)
constexpr int TP_UP = 7;        // 27: message of the parent edge / the pixel's partial towards its parent
constexpr int TP_MN = 34;       // 4 x 2: normal messages / partials (receiver slots, as the grid)
constexpr int TP_PLANES = 42;
// node planes (node-major planes of nplane floats)
constexpr int TN_TAU = 0;       // 6
constexpr int TN_UP = 6;        // 27: message of the parent edge / partial towards the parent
constexpr int TN_CH = 33;       // 4 x 27: messages of the child edges / partials towards the children
constexpr int TN_PLANES = 141;
// lanes per node workgroup: one wave, so that at one wave per SIMD (the node
// update's register use) each SIMD takes the next workgroup as soon as its
// own wave ends, and a level is padded to a multiple of 64 nodes only
constexpr int kTreeThreads = 64;

struct TreeGeo {
    int L;                              // node levels above the pixels
    int NT;                             // nodes
    long nplane;                        // floats per node plane (NT rounded up to 64)
    int nblocks;                        // workgroups of a node launch
    int off[kTreeMaxLevels + 2];        // first node of level l >= 1; off[L + 1] = NT
    int Hl[kTreeMaxLevels + 1];         // rows of level l (Hl[0] = H)
    int Wl[kTreeMaxLevels + 1];         // columns of level l (Wl[0] = W)
    int bstart[kTreeMaxLevels + 2];     // first workgroup of level l >= 1; bstart[L + 1] = nblocks
    double lamP[kTreeMaxLevels + 1];    // prior precision of level l
    double lamR[kTreeMaxLevels + 1];    // identity precision of the edge between levels l and l + 1
};

// levels and per-level strengths; false if the image needs more than
// kTreeMaxLevels levels
bool make_tree_geo(int H, int W, double sigma_P, double sigma_R, TreeGeo* t);

// per-frame prologue: beliefs of the canonical state (X, NX) and the first
// partials (Y, NY)
hipError_t launch_tree_prologue(const Geo& g, const TreeGeo& t, const Strengths& s, const Inputs& in,
                                const float* X, const float* NX, float* Y, float* NY, int* health, hipStream_t st);
// one iteration: complete the partials in (X, NX), update, relinearise, then
// the next partials (or, final_pass, the canonical state and the per-pixel
// outputs) into (Y, NY)
hipError_t launch_tree_iterate(const Geo& g, const TreeGeo& t, const Strengths& s, const Inputs& in,
                               const float* X, const float* NX, float* Y, float* NY, bool final_pass,
                               float* var_ll, float* valid, int* health, hipStream_t st);
// node buffers to zero (keyframe reset) and the state exchange of the pixel
// part (42 planes, pitched <-> dense H x W)
hipError_t launch_tree_clear_nodes(const TreeGeo& t, float* NX, hipStream_t st);
hipError_t launch_tree_pack_pixels(const Geo& g, float* X, float* dense, int to_dense, hipStream_t st);

}  // namespace pv
