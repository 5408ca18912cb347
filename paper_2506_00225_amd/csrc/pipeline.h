// Workspace plan, kernel argument blocks and launchers of the pipeline.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "sgr_internal.h"

namespace sgr {

constexpr int kViewChunk = 16;
constexpr int kMaxAdamSegs = SGR_MAX_ADAM_SEGMENTS;  // segments of one Adam launch

// Workspace layout of one frame: a pure function of the call arguments.
struct Plan {
    int64_t n = 0, vn = 0, cap = 0, num_tiles = 0, num_pixels = 0;
    int V = 0, k = 0, kpad = 0, C = 0, nv_slot = 0;
    int tile_bits = 0, tile_passes = 0;
    int radix_bits = 8;  // widest radix digit (6 or 8)
    // status bit set on the device when a semantic index is >= C
    static constexpr uint32_t kBadIndex = 8u;
    sgr_config cfg{};
    std::vector<ViewDev> view_table;
    // byte offsets
    size_t counters = 0, views = 0;
    size_t count = 0, zbits = 0, gp_of_lin = 0;
    // Records of visible pairs are kept in (view, Gaussian id) order, the
    // order the compaction finds them in; order[r] is the record of the pair
    // at depth rank r (front to back, per view), toff is indexed by depth
    // rank, tcount (tiles touched) both by depth rank and (tcount_rec) by
    // record, and every record array by record.
    size_t vis_k0 = 0, vis_v0 = 0, vis_k1 = 0, vis_v1 = 0, order = 0, pair_lin = 0;
    size_t srec = 0, scol = 0, ssv = 0, ssi = 0, tcount = 0, tcount_rec = 0, toff = 0;
    // class-rank table of each visible pair (kRankWords words), kept when the
    // top-k lists have 16 entries over at most 128 classes
    bool ranked = false;
    size_t srk = 0;
    size_t sorig = 0;  // original list index of each stored top-k position [vis][kpad] (bytes)
    size_t keys0 = 0, vals0 = 0, keys1 = 0, vals1 = 0, owner = 0, ranges = 0, heads = 0;
    size_t sorted_keys = 0, sorted_vals = 0;
    size_t hist = 0, partial = 0;
    size_t block_vis = 0;  // visible pairs per block of 256 (view, Gaussian) pairs
    size_t pix_T = 0, pix_last = 0;
    size_t slots = 0, touched = 0, g2d = 0;
    size_t tile_part = 0;
    size_t map_table = 0, grad_table = 0, loss_table = 0;
    size_t total = 0;
};

sgr_status make_plan(int64_t n, const sgr_camera* cams, int32_t V, const sgr_config* cfg, int64_t cap, Plan* P);

// One bias-corrected Adam update (bc1 = 1 - b1^t, bc2 = 1 - b2^t) of a
// parameter p with moments m, v and gradient g, the parameter clamped to
// [lo, hi].  The Adam launch and the gather with Adam share it, so both give
// the same bits.
struct AdamParams {
    float lr, b1, b2, eps, bc1, bc2;
};
inline AdamParams adam_params(float lr, float b1, float b2, float eps, int step) {
    return AdamParams{lr, b1, b2, eps, 1.f - powf(b1, (float)step), 1.f - powf(b2, (float)step)};
}
__device__ __forceinline__ void adam_update(float g, float& m, float& v, float& p, float lo, float hi,
                                            const AdamParams& h) {
    // One fixed evaluation: the two fused multiply-adds are written out and
    // nothing else is contracted, so every kernel that applies the step (the
    // plain one, the one fused into the gather) gives the same bits.
#pragma clang fp contract(off)
    m = fmaf(h.b1, m, (1.f - h.b1) * g);
    v = fmaf(h.b2, v, ((1.f - h.b2) * g) * g);
    p = fminf(fmaxf(p - h.lr * (m / h.bc1) / (sqrtf(v / h.bc2) + h.eps), lo), hi);
}

struct ProjectArgs {
    const float *means, *scales, *quats, *opacity;
    const ViewDev* views;
    int64_t n, vn;
    float alpha_min, z_near, lowpass;
    uint32_t *count, *zbits, *gp_of_lin;
    uint32_t* block_vis;  // visible pairs of each block of 256 pairs (the compaction's prefix)
    // With init set, the projection launch also initialises the frame: it
    // clears the counters and the tile ranges and stores the view table (one
    // chunk of at most kViewChunk views, passed as a kernel argument, which
    // the projection reads instead of the table it is storing).
    int init;
    uint32_t* counters;
    uint2* ranges;
    int64_t num_tiles;
    ViewDev* views_out;
};

struct GatherArgs {
    // visible pairs per block of 256 (view, Gaussian) pairs (ProjectArgs::block_vis), or with
    // partial_scanned their exclusive prefix sums
    const uint32_t* partial;
    int partial_scanned;
    ProjectArgs proj;
    const uint32_t* count;
    const float *rgb, *sem_val;
    const uint8_t* sem_idx;
    int64_t n;
    int k, kpad, C;
    uint32_t* counters;
    Proj* srec;
    float4* scol;
    float* ssv;
    uint8_t* ssi;
    uint32_t* srk;  // class-rank table [vis][kRankWords], or nullptr
    uint8_t* sorig; // original list index of each stored position [vis][kpad]
    uint32_t *tcount, *gp_of_lin;  // tcount by record
    uint32_t* pair_lin;  // view * n + id of each record
    uint32_t* zkeys;     // fp32 depth bits of each record: the depth sort's keys
};

struct KeyArgs {
    const uint32_t *toff, *tcount;  // by depth rank
    const uint32_t* order;          // record of each depth rank
    const Proj* srec;
    const ViewDev* views;
    const uint32_t* counters;
    int64_t cap;
    uint32_t *keys, *owner;
    uint32_t* heads;  // [cap / kKeyChunk + 1]: owner of each chunk's first key
    // the tile sort's first-pass counts (radix_first_pass layout), written
    // here so the sort needs no histogram launch for that pass
    uint32_t* hist0;
    uint32_t hist_bins;
    int hist_block_major;
};

constexpr int kKeyChunk = 2048;  // keys emitted per workgroup

sgr_status launch_project(const Plan& P, const sgr_gaussians* g, char* ws, hipStream_t st,
                          const float* d_poses = nullptr);
sgr_status launch_bin(const Plan& P, char* ws, int64_t* d_num_keys, hipStream_t st);
sgr_status launch_forward(const Plan& P, const sgr_maps* out, char* ws, hipStream_t st);
sgr_status launch_backward_tiles(const Plan& P, const sgr_map_grads* dL, char* ws, hipStream_t st);
// With adam (six segments: means, scales, quats, opacity, rgb, sem_val) the
// per-Gaussian gradients update the parameters where they are formed
// instead of being written to out.
sgr_status launch_backward_gather(const Plan& P, const sgr_gaussians* g, const sgr_grads* out, char* ws,
                                  hipStream_t st, const sgr_adam_segment* adam = nullptr,
                                  const AdamParams* hp = nullptr);
sgr_status launch_score(const Plan& P, uint32_t* n_empty, double* entropy_sum, char* ws, hipStream_t st);
sgr_status launch_forward_dense(const Plan& P, const float* dense, const sgr_maps* out, char* ws, hipStream_t st);
sgr_status launch_forward_loss(const Plan& P, const sgr_maps* out, const sgr_loss_view* lv, const sgr_loss_config* lc,
                               double* loss, char* ws, hipStream_t st);
sgr_status launch_score_maps(const float* sem, const int32_t* n_contrib, int W, int H, int C, uint32_t* n_empty,
                             double* entropy_sum, char* scratch, hipStream_t st);
size_t score_maps_scratch_bytes(int W, int H);

}  // namespace sgr
