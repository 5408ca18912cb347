// C ABI: argument validation (host only, before any HIP call), workspace
// planning and dispatch.
#include <cmath>
#include <mutex>

#include "pipeline.h"
#include "render_common.h"
#include "sort.h"

namespace sgr {

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

static bool finite_cam(const sgr_camera& c) {
    for (int i = 0; i < 9; i++)
        if (!std::isfinite(c.R[i])) return false;
    for (int i = 0; i < 3; i++)
        if (!std::isfinite(c.t[i])) return false;
    return std::isfinite(c.fx) && std::isfinite(c.fy) && std::isfinite(c.cx) && std::isfinite(c.cy) && c.fx != 0.f &&
           c.fy != 0.f;
}

sgr_status make_plan(int64_t n, const sgr_camera* cams, int32_t V, const sgr_config* cfg, int64_t cap, Plan* P) {
    if (!cams || !cfg || !P || n < 0 || V < 1 || cap < 1) return SGR_EINVAL;
    if (cfg->num_classes < 1 || cfg->num_classes > kMaxC || cfg->top_k < 1 || cfg->top_k > kMaxK) return SGR_EINVAL;
    if (!(cfg->alpha_min > 0.f) || !(cfg->alpha_max > cfg->alpha_min) || !(cfg->alpha_max < 1.f) ||
        !(cfg->t_min > 0.f) || !(cfg->t_min < 1.f) || !(cfg->z_near > 0.f) || !std::isfinite(cfg->z_near) ||
        !(cfg->lowpass >= 0.f) || !std::isfinite(cfg->lowpass))
        return SGR_EINVAL;
    if ((cfg->tile_w != 0 && cfg->tile_w != kTile) || (cfg->tile_h != 0 && cfg->tile_h != kTile))
        return SGR_EUNSUPPORTED;
    if (cfg->sem_accumulators < SGR_ACC_AUTO || cfg->sem_accumulators > SGR_ACC_REGISTERS) return SGR_EINVAL;
    if (cfg->sem_accumulators == SGR_ACC_REGISTERS && cfg->num_classes > kMaxRegC) return SGR_EUNSUPPORTED;
    if (cfg->tile_order < SGR_TILES_AUTO || cfg->tile_order > SGR_TILES_LINEAR || cfg->score_workgroups < 0)
        return SGR_EINVAL;
    if (cfg->sem_passes < 0 || cfg->sem_passes > kMaxPasses) return SGR_EINVAL;
    if (cfg->bwd_batch != 0 && cfg->bwd_batch != 32 && cfg->bwd_batch != 44 && cfg->bwd_batch != 56)
        return SGR_EINVAL;
    if (cfg->radix_bits != 0 && cfg->radix_bits != 6 && cfg->radix_bits != 8) return SGR_EINVAL;
    const int64_t vn = n * (int64_t)V;
    if (vn >= (int64_t)1 << 31 || cap >= (int64_t)1 << 31) return SGR_EINVAL;
    P->n = n;
    P->V = V;
    P->vn = vn;
    P->cap = cap;
    P->k = cfg->top_k;
    P->kpad = (cfg->top_k + 3) & ~3;
    P->C = cfg->num_classes;
    P->cfg = *cfg;
    P->view_table.assign(V, ViewDev{});
    int64_t tiles = 0, pixels = 0;
    for (int v = 0; v < V; v++) {
        const sgr_camera& c = cams[v];
        if (c.width < 1 || c.height < 1 || c.width > 32767 || c.height > 32767 || !finite_cam(c)) return SGR_EINVAL;
        ViewDev& d = P->view_table[v];
        memcpy(d.R, c.R, sizeof(d.R));
        memcpy(d.t, c.t, sizeof(d.t));
        d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy;
        d.width = c.width;
        d.height = c.height;
        d.tiles_x = (int32_t)div_up(c.width, kTile);
        d.tiles_y = (int32_t)div_up(c.height, kTile);
        d.tile_off = (int32_t)tiles;
        d.pix_off = pixels;
        tiles += (int64_t)d.tiles_x * d.tiles_y;
        pixels += (int64_t)c.width * c.height;
        if (tiles >= (int64_t)1 << 30 || pixels >= (int64_t)1 << 40) return SGR_EINVAL;
    }
    P->num_tiles = tiles;
    P->num_pixels = pixels;
    int bits = 1;
    while (((int64_t)1 << bits) < tiles) bits++;
    P->tile_bits = bits;
    P->radix_bits = cfg->radix_bits > 0 ? cfg->radix_bits : 8;
    P->tile_passes = radix_passes(bits, P->radix_bits);

    const int NV = 10 + P->k;
    const size_t vns = (size_t)vn, caps = (size_t)cap;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + std::max<size_t>(bytes, 1), 256);
        return at;
    };
    P->counters = take(sizeof(uint32_t) * kNumCounters);
    P->views = take(sizeof(ViewDev) * V);
    P->map_table = take(sizeof(MapPtrs) * V);
    P->grad_table = take(sizeof(GradPtrs) * V);
    P->loss_table = take(sizeof(LossPtrs) * V);
    P->count = take(4 * vns);
    P->zbits = take(4 * vns);
    P->gp_of_lin = take(4 * vns);
    P->vis_k0 = take(4 * vns);
    P->vis_v0 = take(4 * vns);
    P->vis_k1 = take(4 * vns);
    P->vis_v1 = take(4 * vns);
    P->order = P->vis_v0;  // the 4-pass depth sort ends in the *0 buffers
    P->pair_lin = take(4 * vns);
    P->srec = take(sizeof(Proj) * vns);
    P->scol = take(16 * vns);
    P->ssv = take(4 * (size_t)P->k * vns);
    P->ssi = take((size_t)P->kpad * vns);
    P->sorig = take((size_t)P->kpad * vns);
    P->ranked = P->k == 16 && P->C <= 128;
    if (P->ranked) P->srk = take(4 * (size_t)kRankWords * vns);
    P->tcount = take(4 * vns);
    P->tcount_rec = take(4 * vns);
    P->toff = take(4 * vns);
    P->keys0 = take(4 * caps);
    P->vals0 = take(4 * caps);
    P->keys1 = take(4 * caps);
    P->vals1 = take(4 * caps);
    P->owner = take(4 * caps);
    P->heads = take(4 * (caps / kKeyChunk + 2));
    P->ranges = take(8 * (size_t)tiles);
    const uint32_t big = (uint32_t)std::max<int64_t>(vn, cap);
    const size_t hist_words = radix_hist_words(big);
    P->hist = take(4 * hist_words);
    P->partial = take(4 * scan_partial_words(std::max<size_t>(big, hist_words)));
    P->block_vis = take(4 * (size_t)div_up((int64_t)vns, 256));
    P->pix_T = take(4 * (size_t)pixels);
    P->pix_last = take(4 * (size_t)pixels);
    P->slots = take(4 * (size_t)NV * caps);
    P->touched = take(caps);
    P->g2d = take(4 * (size_t)NV * vns);
    P->tile_part = take((sizeof(double) + sizeof(uint32_t)) * (size_t)tiles);
    P->total = o;
    const bool odd = (P->tile_passes & 1) != 0;
    P->sorted_keys = odd ? P->keys1 : P->keys0;
    P->sorted_vals = odd ? P->vals1 : P->vals0;
    return SGR_OK;
}

// ------------------------------------------------------------------ small device helpers

struct BytePayload {
    uint32_t words[480];
    uint32_t nwords;
};

__global__ void copy_payload(BytePayload p, uint32_t* dst) {
    for (uint32_t i = threadIdx.x; i < p.nwords; i += blockDim.x) dst[i] = p.words[i];
}

// Words [0, n1) of the payload to dst1, the rest to dst2.
__global__ void copy_payload2(BytePayload p, uint32_t n1, uint32_t* dst1, uint32_t* dst2) {
    for (uint32_t i = threadIdx.x; i < p.nwords; i += blockDim.x) {
        if (i < n1) dst1[i] = p.words[i];
        else dst2[i - n1] = p.words[i];
    }
}

// Host -> device copy carried in kernel arguments (no host staging buffer,
// safe to capture in a graph).  bytes must be a multiple of 4.
void upload_bytes(void* dst, const void* src, size_t bytes, hipStream_t st) {
    const uint32_t* s = (const uint32_t*)src;
    uint32_t* d = (uint32_t*)dst;
    size_t words = bytes / 4;
    for (size_t off = 0; off < words; off += 480) {
        BytePayload p;
        p.nwords = (uint32_t)std::min<size_t>(480, words - off);
        memcpy(p.words, s + off, 4 * p.nwords);
        copy_payload<<<1, 256, 0, st>>>(p, d + off);
    }
}

// Two host -> device copies in one launch when they fit one payload.
void upload_pair(void* dst1, const void* src1, size_t bytes1, void* dst2, const void* src2, size_t bytes2,
                 hipStream_t st) {
    const size_t w1 = bytes1 / 4, w2 = bytes2 / 4;
    if (w1 + w2 > 480) {
        upload_bytes(dst1, src1, bytes1, st);
        upload_bytes(dst2, src2, bytes2, st);
        return;
    }
    BytePayload p;
    p.nwords = (uint32_t)(w1 + w2);
    memcpy(p.words, src1, 4 * w1);
    memcpy(p.words + w1, src2, 4 * w2);
    copy_payload2<<<1, 256, 0, st>>>(p, (uint32_t)w1, (uint32_t*)dst1, (uint32_t*)dst2);
}

__global__ void zero_u32(uint32_t* p) { *p = 0u; }

static std::mutex g_dev_mu;
static int g_cu[64];
static size_t g_lds[64];

static int current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    return dev;
}

int device_cu_count() {
    const int dev = current_device();
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (!g_cu[dev]) {
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0) cu = 256;
        g_cu[dev] = cu;
    }
    return g_cu[dev];
}

size_t device_max_lds() {
    const int dev = current_device();
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (!g_lds[dev]) {
        int b = 0;
        if (hipDeviceGetAttribute(&b, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || b <= 0)
            b = 65536;
        g_lds[dev] = std::min<size_t>((size_t)b, kMaxLds);
    }
    return g_lds[dev];
}

size_t score_maps_scratch_bytes(int W, int H) {
    const size_t grid = (size_t)div_up((int64_t)W * H, kBlock);
    return align_up((sizeof(double) + sizeof(uint32_t)) * grid + sizeof(uint32_t), 256);
}

// Scratch of sgr_score_maps_noalloc: one static device array per GPU (the
// runtime gives each device its own copy), so that entry point never
// allocates.  Host code must not pass `scratch` itself to a kernel (in host
// code the name is a host-side stand-in, not a device address): the address
// is looked up once per device with hipGetSymbolAddress and kept here.
static __device__ __align__(256) unsigned char scratch[SGR_NOALLOC_SCRATCH_BYTES];
static void* g_scratch_ptr[64];
static_assert((sizeof(double) + sizeof(uint32_t)) * (SGR_NOALLOC_MAX_PIXELS / kBlock) + sizeof(uint32_t) + 255 <=
                  SGR_NOALLOC_SCRATCH_BYTES,
              "the static scratch holds the partial sums of the largest view it accepts");

// Device address of this device's `scratch`, looked up on the first call on
// the device (with that device current); nullptr if the lookup fails.
static void* noalloc_scratch() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace sgr

using namespace sgr;

static bool gaussians_ok(const sgr_gaussians* g) {
    if (!g || g->n < 0) return false;
    if (g->n == 0) return true;
    return g->means && g->scales && g->quats && g->opacity && g->rgb && g->sem_val && g->sem_idx;
}

static sgr_status prepare(const sgr_gaussians* g, const sgr_camera* cams, int32_t V, const sgr_config* cfg,
                          int64_t cap, void* ws, size_t ws_bytes, Plan* P) {
    if (!gaussians_ok(g)) return SGR_EINVAL;
    const sgr_status s = make_plan(g->n, cams, V, cfg, cap, P);
    if (s != SGR_OK) return s;
    if (!ws || ws_bytes < P->total || ((uintptr_t)ws & 255u)) return SGR_EINVAL;
    return SGR_OK;
}

extern "C" {

size_t sgr_workspace_size(int64_t n, const sgr_camera* cams, int32_t num_views, const sgr_config* cfg,
                          int64_t key_capacity) {
    Plan P;
    if (make_plan(n, cams, num_views, cfg, key_capacity, &P) != SGR_OK) return 0;
    return P.total;
}

sgr_status sgr_workspace_layout(int64_t n, const sgr_camera* cams, int32_t num_views, const sgr_config* cfg,
                                int64_t key_capacity, sgr_layout* out) {
    if (!out) return SGR_EINVAL;
    Plan P;
    const sgr_status s = make_plan(n, cams, num_views, cfg, key_capacity, &P);
    if (s != SGR_OK) return s;
    out->total_bytes = P.total;
    out->counters = P.counters;
    out->views = P.views;
    out->proj_count = P.count;
    out->proj_zbits = P.zbits;
    out->pair_rec = P.srec;
    out->pair_lin = P.pair_lin;
    out->order = P.order;
    out->sorted_keys = P.sorted_keys;
    out->sorted_vals = P.sorted_vals;
    out->key_owner = P.owner;
    out->ranges = P.ranges;
    out->tile_offsets = P.toff;
    out->num_tiles = P.num_tiles;
    out->num_pixels = P.num_pixels;
    out->vn = P.vn;
    return SGR_OK;
}

sgr_status sgr_project(const sgr_gaussians* g, const sgr_camera* cams, int32_t num_views, const sgr_config* cfg,
                       int64_t key_capacity, void* workspace, size_t workspace_bytes, void* stream) {
    Plan P;
    sgr_status s = prepare(g, cams, num_views, cfg, key_capacity, workspace, workspace_bytes, &P);
    if (s != SGR_OK) return s;
    return launch_project(P, g, (char*)workspace, (hipStream_t)stream);
}

sgr_status sgr_bin(const sgr_gaussians* g, const sgr_camera* cams, int32_t num_views, const sgr_config* cfg,
                   int64_t key_capacity, int64_t* d_num_keys, void* workspace, size_t workspace_bytes,
                   void* stream) {
    Plan P;
    sgr_status s = prepare(g, cams, num_views, cfg, key_capacity, workspace, workspace_bytes, &P);
    if (s != SGR_OK) return s;
    return launch_bin(P, (char*)workspace, d_num_keys, (hipStream_t)stream);
}

sgr_status sgr_render_forward(const sgr_gaussians* g, const sgr_camera* cams, int32_t num_views,
                              const sgr_config* cfg, int64_t key_capacity, const sgr_maps* out, void* workspace,
                              size_t workspace_bytes, void* stream) {
    if (!out) return SGR_EINVAL;
    Plan P;
    sgr_status s = prepare(g, cams, num_views, cfg, key_capacity, workspace, workspace_bytes, &P);
    if (s != SGR_OK) return s;
    return launch_forward(P, out, (char*)workspace, (hipStream_t)stream);
}

sgr_status sgr_render_forward_dense(const sgr_gaussians* g, const float* dense_sem, const sgr_camera* cams,
                                    int32_t num_views, const sgr_config* cfg, int64_t key_capacity,
                                    const sgr_maps* out, void* workspace, size_t workspace_bytes, void* stream) {
    if (!out || !dense_sem) return SGR_EINVAL;
    Plan P;
    sgr_status s = prepare(g, cams, num_views, cfg, key_capacity, workspace, workspace_bytes, &P);
    if (s != SGR_OK) return s;
    return launch_forward_dense(P, dense_sem, out, (char*)workspace, (hipStream_t)stream);
}

sgr_status sgr_render_forward_loss(const sgr_gaussians* g, const sgr_camera* cams, int32_t num_views,
                                   const sgr_config* cfg, int64_t key_capacity, const sgr_maps* out,
                                   const sgr_loss_view* lv, const sgr_loss_config* lc, double* loss, void* workspace,
                                   size_t workspace_bytes, void* stream) {
    if (!lv || !lc || !loss) return SGR_EINVAL;
    const float w[] = {lc->w_depth, lc->w_rgb, lc->w_sil, lc->w_sem, lc->lambda_hd, lc->lambda_cos, lc->sqrt_eps};
    for (float x : w)
        if (!(x >= 0.f) || !std::isfinite(x)) return SGR_EINVAL;
    if (!std::isfinite(lc->sil_thresh) || !(lc->ce_floor > 0.f) || !std::isfinite(lc->entropy_tau)) return SGR_EINVAL;
    Plan P;
    sgr_status s = prepare(g, cams, num_views, cfg, key_capacity, workspace, workspace_bytes, &P);
    if (s != SGR_OK) return s;
    return launch_forward_loss(P, out, lv, lc, loss, (char*)workspace, (hipStream_t)stream);
}

sgr_status sgr_render_backward(const sgr_gaussians* g, const sgr_camera* cams, int32_t num_views,
                               const sgr_config* cfg, int64_t key_capacity, const sgr_map_grads* dL,
                               const sgr_grads* out, void* workspace, size_t workspace_bytes, void* stream) {
    if (!dL || !out) return SGR_EINVAL;
    Plan P;
    sgr_status s = prepare(g, cams, num_views, cfg, key_capacity, workspace, workspace_bytes, &P);
    if (s != SGR_OK) return s;
    if ((s = launch_backward_tiles(P, dL, (char*)workspace, (hipStream_t)stream)) != SGR_OK) return s;
    return launch_backward_gather(P, g, out, (char*)workspace, (hipStream_t)stream);
}

sgr_status sgr_render_backward_tiles(const sgr_gaussians* g, const sgr_camera* cams, int32_t num_views,
                                     const sgr_config* cfg, int64_t key_capacity, const sgr_map_grads* dL,
                                     void* workspace, size_t workspace_bytes, void* stream) {
    if (!dL) return SGR_EINVAL;
    Plan P;
    sgr_status s = prepare(g, cams, num_views, cfg, key_capacity, workspace, workspace_bytes, &P);
    if (s != SGR_OK) return s;
    return launch_backward_tiles(P, dL, (char*)workspace, (hipStream_t)stream);
}

sgr_status sgr_render_backward_gather(const sgr_gaussians* g, const sgr_camera* cams, int32_t num_views,
                                      const sgr_config* cfg, int64_t key_capacity, const sgr_grads* out,
                                      void* workspace, size_t workspace_bytes, void* stream) {
    if (!out) return SGR_EINVAL;
    Plan P;
    sgr_status s = prepare(g, cams, num_views, cfg, key_capacity, workspace, workspace_bytes, &P);
    if (s != SGR_OK) return s;
    return launch_backward_gather(P, g, out, (char*)workspace, (hipStream_t)stream);
}

sgr_status sgr_render_backward_gather_adam(const sgr_gaussians* g, const sgr_camera* cams, int32_t num_views,
                                           const sgr_config* cfg, int64_t key_capacity,
                                           const sgr_adam_segment* segments, float lr, float beta1, float beta2,
                                           float eps, int32_t step, void* workspace, size_t workspace_bytes,
                                           void* stream) {
    if (!segments || step < 1 || !(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
        !(eps > 0.f))
        return SGR_EINVAL;
    Plan P;
    sgr_status s = prepare(g, cams, num_views, cfg, key_capacity, workspace, workspace_bytes, &P);
    if (s != SGR_OK) return s;
    const int64_t want[6] = {3 * P.n, 3 * P.n, 4 * P.n, P.n, 3 * P.n, (int64_t)P.k * P.n};
    for (int i = 0; i < 6; i++) {
        const sgr_adam_segment& sg = segments[i];
        if (sg.n != want[i] || (sg.n > 0 && (!sg.p || !sg.m || !sg.v)) || !(sg.lo <= sg.hi)) return SGR_EINVAL;
    }
    const AdamParams h = adam_params(lr, beta1, beta2, eps, step);
    return launch_backward_gather(P, g, nullptr, (char*)workspace, (hipStream_t)stream, segments, &h);
}

sgr_status sgr_score_views(const sgr_gaussians* g, const sgr_camera* cams, int32_t num_views,
                           const sgr_config* cfg, int64_t key_capacity, uint32_t* n_empty, double* entropy_sum,
                           void* workspace, size_t workspace_bytes, void* stream) {
    if (!n_empty || !entropy_sum) return SGR_EINVAL;
    Plan P;
    sgr_status s = prepare(g, cams, num_views, cfg, key_capacity, workspace, workspace_bytes, &P);
    if (s != SGR_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    if ((s = launch_project(P, g, (char*)workspace, st)) != SGR_OK) return s;
    if ((s = launch_bin(P, (char*)workspace, nullptr, st)) != SGR_OK) return s;
    return launch_score(P, n_empty, entropy_sum, (char*)workspace, st);
}

sgr_status sgr_score_poses(const sgr_gaussians* g, const sgr_camera* intrinsics, int32_t num_views, const float* poses,
                           const sgr_config* cfg, int64_t key_capacity, uint32_t* n_empty, double* entropy_sum,
                           void* workspace, size_t workspace_bytes, void* stream) {
    if (!intrinsics || !poses || !n_empty || !entropy_sum || num_views < 1) return SGR_EINVAL;
    std::vector<sgr_camera> cams((size_t)num_views, *intrinsics);
    for (sgr_camera& c : cams) {  // placeholders until the device poses are copied in
        for (int i = 0; i < 9; i++) c.R[i] = (i % 4 == 0) ? 1.f : 0.f;
        for (int i = 0; i < 3; i++) c.t[i] = 0.f;
    }
    Plan P;
    sgr_status s = prepare(g, cams.data(), num_views, cfg, key_capacity, workspace, workspace_bytes, &P);
    if (s != SGR_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    if ((s = launch_project(P, g, (char*)workspace, st, poses)) != SGR_OK) return s;
    if ((s = launch_bin(P, (char*)workspace, nullptr, st)) != SGR_OK) return s;
    return launch_score(P, n_empty, entropy_sum, (char*)workspace, st);
}

size_t sgr_score_maps_workspace_size(int32_t width, int32_t height) {
    if (width < 1 || height < 1) return 0;
    return score_maps_scratch_bytes(width, height);
}

sgr_status sgr_score_maps(const float* sem, const int32_t* n_contrib, int32_t width, int32_t height,
                          int32_t num_classes, uint32_t* n_empty, double* entropy_sum, void* workspace,
                          size_t workspace_bytes, void* stream) {
    if (!sem || !n_contrib || !n_empty || !entropy_sum || width < 1 || height < 1 || num_classes < 1 ||
        num_classes > kMaxC)
        return SGR_EINVAL;
    if (!workspace || workspace_bytes < score_maps_scratch_bytes(width, height) || ((uintptr_t)workspace & 255u))
        return SGR_EINVAL;
    return launch_score_maps(sem, n_contrib, width, height, num_classes, n_empty, entropy_sum, (char*)workspace,
                             (hipStream_t)stream);
}

sgr_status sgr_score_maps_noalloc(const float* sem, const int32_t* n_contrib, int32_t width, int32_t height,
                                  int32_t num_classes, uint32_t* n_empty, double* entropy_sum, void* stream) {
    if (!sem || !n_contrib || !n_empty || !entropy_sum || width < 1 || height < 1 || num_classes < 1 ||
        num_classes > kMaxC)
        return SGR_EINVAL;
    if ((int64_t)width * height > SGR_NOALLOC_MAX_PIXELS) return SGR_EUNSUPPORTED;
    void* ptr = noalloc_scratch();
    if (!ptr) return SGR_EHIP;
    // the same launches as sgr_score_maps; its counter is cleared by a kernel
    // at the start of every call, the partial sums are written before read
    return launch_score_maps(sem, n_contrib, width, height, num_classes, n_empty, entropy_sum, (char*)ptr,
                             (hipStream_t)stream);
}

sgr_status sgr_read_status(const void* workspace, void* stream, int64_t* num_visible, int64_t* num_keys) {
    if (!workspace) return SGR_EINVAL;
    uint32_t c[kNumCounters];
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return SGR_EHIP;
    if (hipMemcpy(c, workspace, sizeof(c), hipMemcpyDeviceToHost) != hipSuccess) return SGR_EHIP;
    if (num_visible) *num_visible = c[kNumVisible];
    if (num_keys) *num_keys = c[kKeysLo];
    if (c[kStatus] & SGR_ECAPACITY) return SGR_ECAPACITY;
    if (c[kStatus] & Plan::kBadIndex) return SGR_EINVAL;
    return SGR_OK;
}

const char* sgr_status_string(int32_t s) {
    // an int, not the enum: a caller may hand in any code, and a value
    // outside the enumerators is not a valid sgr_status in C++
    switch (s) {
        case SGR_OK: return "ok";
        case SGR_EINVAL: return "invalid argument";
        case SGR_ECAPACITY: return "tile key capacity exceeded";
        case SGR_EHIP: return "HIP runtime error";
        case SGR_EUNSUPPORTED: return "unsupported configuration";
    }
    return "unknown status";
}

}  // extern "C"
