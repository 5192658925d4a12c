// Shared device-side definitions of lib7dgs (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sd7.h"

namespace sd7 {

// Rasterizer constants (FP32 values; see sd7.h).
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;
constexpr float kZNear = 0.2f;
constexpr float kDilation = 0.3f;
constexpr float kJClamp = 1.3f;
constexpr int kTile = SD7_TILE;
constexpr uint32_t kCulled = 0xFFFFFFFFu;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.69314718055994531f;
constexpr float kNegHalfLog2e = -0.72134752044448170f;
constexpr float kNegLog2e = -1.4426950408889634f;

constexpr int kBlock = 256;        // threads per block of the per-Gaussian kernels
constexpr int kSortPerThread = 8;  // radix-sort elements per thread of a work tile
constexpr int kSortItems = 256 * kSortPerThread;  // elements per radix-sort work tile
static_assert(kSortItems == SD7_PAIR_ROUND, "a frame's arena share is a whole number of work tiles");
constexpr int kScanItems = 4096;   // elements per scan work tile
constexpr int kSplatFloats = 12;   // floats per splat record

// Per-frame descriptor, built on the host and copied into the workspace.
struct FrameDev {
    const float* mu_p;
    const float* mu_t;
    const float* mu_d;
    const float* L;
    const float* alpha;
    const float* sh;
    float* image;
    float* final_T;
    uint32_t* last;
    const float* dL_dimage;
    float* g_mu_p;
    float* g_mu_t;
    float* g_mu_d;
    float* g_L;
    float* g_alpha;
    float* g_sh;
    float* g_lambda;     // optional [2]: dL/dlambda_t, dL/dlambda_d (accumulated)
    uint32_t* ncontrib;  // optional per-pixel contributor count
    const float* agr;    // optional AGR weights (SD7_AGR_WEIGHTS floats)
    uint32_t n;        // Gaussians
    uint32_t g0;       // first Gaussian in the concatenated per-Gaussian arrays
    uint32_t W, H;
    uint32_t tiles_x, tiles_y;
    uint32_t t0;       // first tile in the concatenated tile arrays
    uint32_t nch;      // binning chunks (the kept Gaussians are cut into this many)
    uint32_t d_mode;   // 1: Gaussian i is conditioned on unit(mu_p,i - c)
    uint32_t m0;       // first entry of the frame's [chunk][tile] count matrix
    uint32_t keep_sliced;  // 1: the fused slice/projection writes the sliced statistics
    float R[9];
    float c[3];
    float fx, fy, cx, cy;
    float t;
    float d[3];
    float lambda_t, lambda_d;
    float bg[3];
    float limx, limy;  // view-ray ratio clamps of J: 1.3 x (W/2) / fx, 1.3 x (H/2) / fy
};

// Third word of a raw buffer resource on gfx9-class GPUs (32-bit data format,
// no swizzle): range-checked loads at byte offsets below the record count.
constexpr int kBufferWord3 = 0x00020000;
constexpr uint32_t kMaxCountTiles = 32768;  // tiles per frame the counting binner takes (more: radix binner)
constexpr uint32_t kGroup = 8;              // tiles per side of a counting-binner group (one lane per tile)

// Prefix of launch blocks over the frames of a call (kernel argument).
struct BlockMap {
    uint32_t start[SD7_MAX_FRAMES + 1];
    int nf;
};

__device__ __forceinline__ int frame_of_block(const BlockMap& bm, uint32_t b)
{
    int lo = 0, hi = bm.nf - 1;
    while (lo < hi) {  // largest f with start[f] <= b
        int mid = (lo + hi + 1) >> 1;
        if (bm.start[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Frames of a call grouped by scene (same parameter arrays): group g owns
// frame[first[g]] .. frame[first[g + 1] - 1] and the work units start[g] ..
// start[g + 1] - 1 (kernel argument).  A unit is one (block of kBlock
// Gaussians, frame) of the group, numbered Gaussian block by Gaussian block
// and, within one, frame by frame.
struct SceneGroups {
    uint32_t start[SD7_MAX_FRAMES + 1];
    uint8_t first[SD7_MAX_FRAMES + 1];
    uint8_t frame[SD7_MAX_FRAMES];
    int ng;
};

// The fused slice/projection grid is a whole number of rounds of
// kSliceResident blocks, the blocks that are resident on the chip at once
// (three per CU, set by their 48 KiB of LDS, on 256 CUs), each taking an
// equal share of the units, about kSliceUnitsPerBlock of them or more.  Every
// block then does the same work and no round runs partly filled.
constexpr uint32_t kSliceResident = 768;
constexpr uint32_t kSliceUnitsPerBlock = 8;

__device__ __forceinline__ int group_of_unit(const SceneGroups& sg, uint32_t b)
{
    int lo = 0, hi = sg.ng - 1;
    while (lo < hi) {  // largest g with start[g] <= b
        int mid = (lo + hi + 1) >> 1;
        if (sg.start[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// A segment of a segmented sort: one frame's elements.
struct SortSeg {
    uint32_t in_base;    // first element in the input arrays
    uint32_t out_base;   // first element in the output arrays
    uint32_t len;        // elements read
    uint32_t wt0;        // first work tile
    uint32_t nwt;        // work tiles
    uint32_t cnt_excl;   // elements counted (scattered) by earlier segments
    uint32_t pad[2];
};

// Device-side sizes written by the setup kernels.
struct SortTotals {
    uint32_t wt;         // total work tiles
    uint32_t hist_len;   // 256 * wt
    uint32_t pad[2];
};

__device__ __forceinline__ int seg_of_tile(const SortSeg* segs, int nseg, uint32_t w)
{
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (segs[mid].wt0 <= w) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Workgroups of a launch go to the 8 XCDs round-robin in launch order.  This
// maps launch index i (of nb) to a logical index such that every XCD runs one
// contiguous range of logical blocks, whose shared data then stays in that
// XCD's L2.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t i, uint32_t nb)
{
    const uint32_t x = i % kXcds, k = i / kXcds, q = nb / kXcds, rem = nb % kXcds;
    return x * q + min(x, rem) + k;
}

__device__ __forceinline__ uint64_t lanemask_lt()
{
    const uint32_t lane = __lane_id();
    return lane == 0 ? 0ull : ((~0ull) >> (64 - lane));
}

}  // namespace sd7
