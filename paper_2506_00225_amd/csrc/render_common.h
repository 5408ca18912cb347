// Shared pieces of the compositing kernels.
#pragma once

#include "pipeline.h"

namespace sgr {

constexpr int kFwdBatch = 128;     // Gaussians staged per forward batch (two culling ballots)
static_assert(kFwdBatch == 128, "the forward culls a batch with two 64-lane ballots");
constexpr size_t kMaxLds = 160 * 1024;

// LDS floats of a class-major accumulator tile, rounded up so that what
// follows it stays 16-byte aligned.
__host__ __device__ inline int acc_floats(int C) { return (C * kAccStride + 3) & ~3; }

// Semantic accumulators held in registers: NB vectors of 32 classes.  A
// class index is wave-uniform during a blend (every lane composites the same
// Gaussian), so an update is a uniform-indexed register read-modify-write.
typedef float v32f __attribute__((ext_vector_type(32)));
// References to the kernel's own vector variables (an aggregate of vectors
// would be placed in scratch memory): blocks past NB are never touched.
template <int NB>
struct RegAcc {
    v32f &a0, &a1, &a2, &a3;
};

// The entries of block B (classes 32 B .. 32 B + 31) from position m on.
template <int B, int KM, int KWM>
__device__ __forceinline__ void acc_run(v32f& acc, const float (&vv)[KM], const uint32_t (&wd)[KWM], int k, float w,
                                        int& m) {
    while (m < k) {
        const uint32_t c = (wd[m >> 2] >> (8 * (m & 3))) & 0xffu;
        if ((int)(c / kRegBlock) != B) break;
        acc[c % kRegBlock] = fmaf(vv[m], w, acc[c % kRegBlock]);
        m++;
    }
}

// acc[class] += v_m * w for the k entries of one Gaussian, stored grouped by
// block (class / 32): the entries of a block are consecutive, so each block
// is one uniform loop over one register vector.  sv: the k values (LDS),
// wd: the class bytes, four per word, in scalar registers.
template <int NB, int KT, int KM, int KWM>
__device__ __forceinline__ void reg_accumulate(RegAcc<NB>& A, const float* sv, const uint32_t (&wd)[KWM], int k,
                                               float w) {
    float vv[KM];
    if constexpr (KT > 0 && (KT & 3) == 0) {  // 16-byte aligned rows of KT values
#pragma unroll
        for (int m = 0; m < KM; m += 4) {
            const float4 v4 = *(const float4*)(sv + m);
            vv[m] = v4.x; vv[m + 1] = v4.y; vv[m + 2] = v4.z; vv[m + 3] = v4.w;
        }
    } else {
#pragma unroll
        for (int m = 0; m < KM; m++) vv[m] = m < k ? sv[m] : 0.f;
    }
    // The trip counts are hidden from the optimiser: unrolled, the block
    // loops' exits would merge copies of whole vectors.
    int kk = k;
    asm volatile("" : "+s"(kk));
    int m = 0;
    acc_run<0>(A.a0, vv, wd, kk, w, m);
    if constexpr (NB > 1) acc_run<1>(A.a1, vv, wd, kk, w, m);
    if constexpr (NB > 2) acc_run<2>(A.a2, vv, wd, kk, w, m);
    if constexpr (NB > 3) acc_run<3>(A.a3, vv, wd, kk, w, m);
}

template <int NB>
__device__ __forceinline__ void reg_zero(RegAcc<NB>& A) {
    A.a0 = 0.f;
    if constexpr (NB > 1) A.a1 = 0.f;
    if constexpr (NB > 2) A.a2 = 0.f;
    if constexpr (NB > 3) A.a3 = 0.f;
}

// Per-view pointer tables.  With one view the entry travels inline in the
// kernel arguments, so no upload launch precedes the kernel; with more it is
// a table in the workspace.
template <class T>
struct ViewTable {
    const T* table;  // [V] in the workspace, or nullptr: use `one`
    T one;
    __device__ __forceinline__ T operator[](int v) const { return table ? table[v] : one; }
};

struct MapPtrs {
    float *rgb, *depth, *sil, *sem, *t_final;
    int32_t* n_contrib;
};

struct LossPtrs {  // one view's loss targets and gradient outputs
    const float *rgb, *depth;
    const int32_t* label;
    const float* sem;
    float *g_rgb, *g_depth, *g_sil, *g_sem, *g_sem_at_label;
};

struct LossK {  // fused-loss kernel arguments
    ViewTable<LossPtrs> views;
    float w_depth, w_rgb, w_sil, w_sem, sil_thresh, ce_floor, lambda_hd, lambda_cos, tau, sqrt_eps;
    double* tile_loss;  // [num_tiles]
};

struct GradPtrs {
    const float *rgb, *depth, *sil, *sem;
    const int32_t* sem_label;  // sparse semantic gradient (when sem is NULL)
    const float* sem_at_label;
};

struct TileArgs {
    const ViewDev* views;
    int V;
    int64_t num_tiles;
    int k, kpad, C;
    const uint2* ranges;
    const uint32_t *svals, *owner;  // the pair of sorted key s: owner[svals[s]]
    const Proj* srec;
    const float4* scol;
    const float* ssv;
    const uint8_t* ssi;
    const uint32_t* srk;  // class-rank table [vis][kRankWords] (k = 16, C <= 128), or nullptr
    uint32_t* counters;
    float* pix_T;
    uint32_t* pix_last;
    float alpha_min, alpha_max, t_min;
    int linear_tiles;  // 1: workgroup i takes tile i; 0: XCD-contiguous runs
    ViewTable<MapPtrs> maps;
    ViewTable<LossPtrs> loss_views;  // label-only class sums: each view's label map
};

struct TileResult {
    float T;
    int ncon;
    bool inside;
    int v, px, py, tx, ty;
    uint32_t last;
    float c[3];
    float d, s;
    int lab;    // label-only class sums: the pixel's label (-1 if none) ...
    float ql;   // ... and its class sum
};

struct ScoreOut {
    double* tile_h;
    uint32_t* tile_e;
    uint32_t* n_empty;
    double* entropy_sum;
};

// Pixel layout of a 16x16 tile over 256 threads: wave w covers the 8x8
// quadrant (w & 1, w >> 1), lane l the pixel (l & 7, l >> 3) inside it, so a
// small Gaussian touches few waves.  slot_of gives the thread (and LDS
// column) that owns tile pixel (lx, ly).
__host__ __device__ inline int tile_px(int t) { return ((t >> 6) & 1) * 8 + (t & 7); }
__host__ __device__ inline int tile_py(int t) { return ((t >> 7) & 1) * 8 + ((t >> 3) & 7); }
__host__ __device__ inline int slot_of(int lx, int ly) {
    return (((ly >> 3) << 1) | (lx >> 3)) * 64 + ((ly & 7) << 3) + (lx & 7);
}

__device__ inline int view_of_tile(const ViewDev* views, int V, int gt) {
    int lo = 0, hi = V - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].tile_off <= gt) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// alpha = min(alpha_max, o G) at the centre of pixel (px, py).  The offset
// from the mean is formed from the record's integer part and its stored
// 0.5 - fraction (exact up to one rounding), and log2 G = -(ca u^2 + cc dy^2) with
// u = dx + cb dy has no cancellation.  dx, dy are pixel centre minus mean.
__device__ __forceinline__ float eval_alpha(const float4& q0, const float4& q1, int px, int py, float amax,
                                            float* G, float* dx, float* dy) {
    const float ddx = (float)(px - __float_as_int(q0.x)) + q0.z;
    const float ddy = (float)(py - __float_as_int(q0.y)) + q0.w;
    const float u = fmaf(q1.y, ddy, ddx);
    const float e = fmaf(q1.x * u, u, q1.z * ddy * ddy);
    const float g = __builtin_amdgcn_exp2f(-e);  // v_exp_f32; e >= 0 here
    *G = g;
    *dx = ddx;
    *dy = ddy;
    return fminf(amax, q1.w * g);
}

// eval_alpha that also returns u = dx + cb dy (the backward's whitened
// offsets start from it).
__device__ __forceinline__ float eval_alpha_u(const float4& q0, const float4& q1, int px, int py, float amax,
                                              float* G, float* dx, float* dy, float* u) {
    const float ddx = (float)(px - __float_as_int(q0.x)) + q0.z;
    const float ddy = (float)(py - __float_as_int(q0.y)) + q0.w;
    const float uu = fmaf(q1.y, ddy, ddx);
    const float e = fmaf(q1.x * uu, uu, q1.z * ddy * ddy);
    const float g = __builtin_amdgcn_exp2f(-e);  // v_exp_f32; e >= 0 here
    *G = g;
    *dx = ddx;
    *dy = ddy;
    *u = uu;
    return fminf(amax, q1.w * g);
}

// Whether an entry can reach alpha >= alpha_min at some pixel centre of the
// block of pixels [bx0, bx1] x [by0, by1] (already clipped to the entry's
// rectangle).  The exponent e = ca u^2 + cc dy^2 (u = dx + cb dy, the form
// eval_alpha evaluates) is minimised over the continuous box spanned by the
// block's pixel centres, a lower bound of its minimum over the pixels, and
// compared with log2(o / alpha_min) plus slack for rounding.  It only answers
// false where no pixel of the block passes the alpha cutoff, so skipping
// such an entry changes no result.  (The rectangle is the box of the whole
// ellipse; a block near one of its corners often misses the ellipse.)
__device__ __forceinline__ bool conic_meets_block(const float4& q0, const float4& q1, int bx0, int bx1, int by0,
                                                  int by1, float amin) {
    const float x0 = (float)(bx0 - __float_as_int(q0.x)) + q0.z;
    const float x1 = x0 + (float)(bx1 - bx0);
    const float y0 = (float)(by0 - __float_as_int(q0.y)) + q0.w;
    const float y1 = y0 + (float)(by1 - by0);
    const float ca = q1.x, cb = q1.y, cc = q1.z;
    // along a row y: u = dx + cb y is smallest at dx = -cb y
    const float xa = fminf(fmaxf(-cb * y0, x0), x1), xb = fminf(fmaxf(-cb * y1, x0), x1);
    const float ua = fmaf(cb, y0, xa), ub = fmaf(cb, y1, xb);
    const float ea = fmaf(ca * ua, ua, cc * y0 * y0), eb = fmaf(ca * ub, ub, cc * y1 * y1);
    // along a column x: e is smallest at dy = -ca cb x / (ca cb^2 + cc)
    const float k = -ca * cb * __builtin_amdgcn_rcpf(fmaf(ca * cb, cb, cc));
    const float yc = fminf(fmaxf(k * x0, y0), y1), yd = fminf(fmaxf(k * x1, y0), y1);
    const float uc = fmaf(cb, yc, x0), ud = fmaf(cb, yd, x1);
    const float ec = fmaf(ca * uc, uc, cc * yc * yc), ed = fmaf(ca * ud, ud, cc * yd * yd);
    const bool inside = x0 <= 0.f && x1 >= 0.f && y0 <= 0.f && y1 >= 0.f;  // the mean's own pixel box
    const float emin = inside ? 0.f : fminf(fminf(ea, eb), fminf(ec, ed));
    const float E = __log2f(q1.w / amin);
    return emin <= E + 1e-3f * (1.f + fabsf(E));
}

// Writes the tile's class-major LDS columns (one per pixel, stride 257) as
// [H][W][C] rows: each tile row is one contiguous run of 16 C floats.
__device__ __forceinline__ void write_rows_from_lds(const float* smem, float* out, const ViewDev& vw, int C, int tx,
                                                    int ty) {
    const int x0 = tx * kTile, y0 = ty * kTile;
    const int wcols = min(kTile, vw.width - x0), hrows = min(kTile, vw.height - y0);
    const int row_elems = kTile * C;
    const int dl = kBlock / C, dc = kBlock % C;
    for (int row = 0; row < hrows; row++) {
        float* dst = out + ((int64_t)(y0 + row) * vw.width + x0) * C;
        int lx = threadIdx.x / C, c = threadIdx.x % C;
        for (int e = threadIdx.x; e < row_elems; e += kBlock) {
            if (lx < wcols) dst[e] = smem[c * kAccStride + slot_of(lx, row)];
            lx += dl;
            c += dc;
            if (c >= C) { c -= C; lx++; }
        }
    }
}

TileArgs make_tile_args(const Plan& P, char* ws);
size_t fwd_lds_bytes(int C, int k, int kpad, int sem_mode);
int device_cu_count();
size_t device_max_lds();
void upload_bytes(void* dst, const void* src, size_t bytes, hipStream_t st);

// Fills `t` from the host entries: inline for one view, else uploaded to
// `dst` in the workspace.
template <class T>
void set_view_table(ViewTable<T>& t, const std::vector<T>& entries, char* dst, hipStream_t st) {
    if (entries.size() == 1) {
        t.table = nullptr;
        t.one = entries[0];
    } else {
        upload_bytes(dst, entries.data(), sizeof(T) * entries.size(), st);
        t.table = (const T*)dst;
        t.one = T{};
    }
}
void upload_pair(void* dst1, const void* src1, size_t bytes1, void* dst2, const void* src2, size_t bytes2,
                 hipStream_t st);

__global__ void zero_u32(uint32_t* p);

}  // namespace sgr
