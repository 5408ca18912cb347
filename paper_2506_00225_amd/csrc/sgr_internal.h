// Internal definitions shared by the HIP kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sgr.h"

namespace sgr {

constexpr int kTile = 16;          // tile edge in pixels (16x16 = 256 pixels = 4 wave64)
constexpr int kBlock = 256;        // threads per tile workgroup
constexpr int kMaxK = 32;          // top-k limit
constexpr int kMaxC = 256;         // class limit (u8 indices)
constexpr int kAccStride = 257;    // LDS class-major stride: conflict-free for consecutive pixels
constexpr uint32_t kInvalid = 0xffffffffu;
constexpr int kRegBlock = 32;      // classes per register accumulator vector
constexpr int kMaxRegC = 128;      // classes that fit the register accumulators (4 vectors)
constexpr int kMaxPasses = 4;      // class ranges the LDS class sums may be split into
// Class-rank table of a visible pair whose top-k list has 16 entries over at
// most 128 classes, 8 words: the 128-bit class mask (words 0-3); words 4-5,
// nibble r = stored list position of the class of rank r (its r-th
// smallest class); words 6-7 unused (padding).  A pixel finds its label's
// rank with one mask lookup and a popcount, and from it the list position
// (lists with a repeated class are flagged in the record, have zero
// nibbles, and are never looked up).
constexpr int kRankWords = 8;

// Top-k entries are stored grouped by accumulator block (class / 32), in
// their original order inside a block, so a compositing kernel can walk a
// Gaussian's classes one register vector at a time (the records are built
// in build_record).
// counters[] slots at the start of the workspace
enum Counter : int {
    kStatus = 0,      // bit 1: capacity exceeded
    kNumVisible = 1,  // visible (view, Gaussian) pairs
    kNumKeys = 2,     // tile keys (saturates at capacity+1 for the status check)
    kWork = 3,        // reserved
    kDone = 4,        // persistent-kernel finished-block count
    kKeysLo = 5,      // exact key count, low 32 bits (the scan total)
    kNumCounters = 16
};

// Per-view table on the device (64-byte aligned rows).
struct alignas(16) ViewDev {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    int32_t width, height, tiles_x, tiles_y;
    int32_t tile_off;   // first global tile of this view
    int32_t pad0;
    int64_t pix_off;    // first pixel of this view in the per-pixel workspace arrays
};

// Projected record of one (view, Gaussian) pair, 48 bytes.
//   r0 = (ix, iy as int bits, hx, hy): pixel-space mean = (ix + fx, iy + fy),
//        integer part exact, fraction f in [0,1) to fp32 precision, stored
//        as h = 0.5 - f (fp32), so a pixel centre's offset from the mean is
//        (px - ix) + hx
//   r1 = (ca, cb, cc, o): exponent of the splat in base 2,
//        log2 G = -(ca*u^2 + cc*dy^2), u = dx + cb*dy, with
//        ca = a/(2 ln 2), cb = b/a, cc = (c - b^2/a)/(2 ln 2) for the conic
//        Q = a dx^2 + 2 b dx dy + c dy^2 (both terms are non-negative, so
//        fp32 evaluation has no cancellation)
//   r2 = (col_lo | col_hi << 16, row_lo | row_hi << 16, z, 0)
struct Proj {
    float4 r0, r1, r2;
};

__host__ __device__ inline int64_t div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Tile launches are padded to a multiple of 8 workgroups.  Workgroup i runs
// on XCD i % 8; mapping it to tile (i % 8) * (grid / 8) + i / 8 gives each
// XCD a contiguous run of tiles, so neighbouring tiles (which share
// Gaussians) hit the same L2.  Tiles past the real count exit at once.
__device__ inline int xcd_remap(int bid, int grid8) {
    const int per = grid8 >> 3;
    return (bid & 7) * per + (bid >> 3);
}
__device__ inline int tile_of_block(int bid, int grid8, int linear) { return linear ? bid : xcd_remap(bid, grid8); }

}  // namespace sgr
