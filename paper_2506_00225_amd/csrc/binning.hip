// Projection (EWA splat), visibility compaction with the compositing records,
// the depth sort of the records,
// per-tile key emission and tile ranges.
#include "pipeline.h"
#include "sort.h"

namespace sgr {

// --------------------------------------------------------------- views

struct ViewChunk {
    ViewDev v[kViewChunk];
    int32_t first, count;
};

// Camera tables travel as kernel arguments (graph-capturable, no host copy).
__global__ void upload_views(ViewChunk chunk, ViewDev* views) {
    const int j = threadIdx.x;
    if (j < chunk.count) views[chunk.first + j] = chunk.v[j];
}

// Clears the counters and tile ranges; block 0 also stores one chunk of the
// view table (count 0: none).
__global__ void init_frame(uint32_t* counters, uint2* ranges, int64_t num_tiles, ViewChunk chunk, ViewDev* views) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < kNumCounters) counters[i] = 0;
    if (i < num_tiles) ranges[i] = make_uint2(0u, 0u);
    if (blockIdx.x == 0 && threadIdx.x < chunk.count) views[chunk.first + threadIdx.x] = chunk.v[threadIdx.x];
}

__global__ void publish_num_keys(const uint32_t* counters, int64_t* d_num_keys) {
    d_num_keys[0] = (int64_t)counters[kKeysLo];
}

// --------------------------------------------------------------- projection

// Projection of Gaussian i into view vw.  Everything that decides binning
// (the camera-space point, the 2D covariance, the pixel rectangle, the depth
// key) is evaluated in double precision with the same operation order as the
// FP64 reference and no contraction into FMA, so the tile keys agree bit for
// bit; the compositing record is then rounded to fp32.  Returns the number
// of tiles the pixel rectangle touches (0: culled).
// Where the projection takes Gaussian i's parameters from: the arrays, read
// where each is first used (so a pair behind the camera reads only its
// mean), or values loaded beforehand.
struct ParamsAt {
    const ProjectArgs& a;
    int64_t i;
    __device__ float mean(int r) const { return a.means[3 * i + r]; }
    __device__ float quat(int r) const { return a.quats[4 * i + r]; }
    __device__ float scale(int r) const { return a.scales[3 * i + r]; }
    __device__ float opacity() const { return a.opacity[i]; }
};
struct GeomIn {
    float m[3], q[4], s[3], o, rgb[3];
    uint32_t count;
    __device__ float mean(int r) const { return m[r]; }
    __device__ float quat(int r) const { return q[r]; }
    __device__ float scale(int r) const { return s[r]; }
    __device__ float opacity() const { return o; }
};

template <typename In>
__device__ __forceinline__ uint32_t project_pair(const ProjectArgs& a, const ViewDev& vw, int v, const In& in,
                                                 uint32_t* zbits, Proj* rec) {
#pragma clang fp contract(off)
    uint32_t count = 0;
    const double m0 = in.mean(0), m1 = in.mean(1), m2 = in.mean(2);
    double p[3];
#pragma unroll
    for (int r = 0; r < 3; r++)
        p[r] = (double)vw.R[3 * r] * m0 + (double)vw.R[3 * r + 1] * m1 + (double)vw.R[3 * r + 2] * m2 +
               (double)vw.t[r];
    const float zf = (float)p[2];
    *zbits = __float_as_uint(zf);
    if (!(p[2] > (double)a.z_near)) return 0;
    const double q0 = in.quat(0), q1 = in.quat(1), q2 = in.quat(2), q3 = in.quat(3);
    const double qn = sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
    const double w = q0 / qn, x = q1 / qn, y = q2 / qn, z = q3 / qn;
    double Rq[9];
    Rq[0] = 1 - 2 * (y * y + z * z); Rq[1] = 2 * (x * y - w * z);     Rq[2] = 2 * (x * z + w * y);
    Rq[3] = 2 * (x * y + w * z);     Rq[4] = 1 - 2 * (x * x + z * z); Rq[5] = 2 * (y * z - w * x);
    Rq[6] = 2 * (x * z - w * y);     Rq[7] = 2 * (y * z + w * x);     Rq[8] = 1 - 2 * (x * x + y * y);
    const double s[3] = {(double)in.scale(0), (double)in.scale(1), (double)in.scale(2)};
    double S3[9];
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            double acc = 0;
#pragma unroll
            for (int e = 0; e < 3; e++) acc += Rq[3 * r + e] * s[e] * s[e] * Rq[3 * c + e];
            S3[3 * r + c] = acc;
        }
    const double fx = vw.fx, fy = vw.fy, zz = p[2];
    const double J[6] = {fx / zz, 0, -fx * p[0] / (zz * zz), 0, fy / zz, -fy * p[1] / (zz * zz)};
    double T[6];
#pragma unroll
    for (int r = 0; r < 2; r++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            double acc = 0;
#pragma unroll
            for (int e = 0; e < 3; e++) acc += J[3 * r + e] * (double)vw.R[3 * e + c];
            T[3 * r + c] = acc;
        }
    double S2[4];
#pragma unroll
    for (int r = 0; r < 2; r++)
#pragma unroll
        for (int c = 0; c < 2; c++) {
            double acc = 0;
#pragma unroll
            for (int e = 0; e < 3; e++)
#pragma unroll
                for (int f = 0; f < 3; f++) acc += T[3 * r + e] * S3[3 * e + f] * T[3 * c + f];
            S2[2 * r + c] = acc;
        }
    const double lp = a.lowpass;
    S2[0] += lp;
    S2[3] += lp;
    const double sxx = S2[0], sxy = 0.5 * (S2[1] + S2[2]), syy = S2[3];
    const double det = sxx * syy - sxy * sxy;
    const double o = in.opacity();
    if (!(det > 0 && o >= (double)a.alpha_min)) return 0;
    const double mx = fx * p[0] / zz + (double)vw.cx, my = fy * p[1] / zz + (double)vw.cy;
    const double qmax = 2.0 * log(o / (double)a.alpha_min);
    const double ex = sqrt(qmax * sxx), ey = sqrt(qmax * syy);
    double clo = ceil(mx - ex - 0.5), chi = floor(mx + ex - 0.5);
    double rlo = ceil(my - ey - 0.5), rhi = floor(my + ey - 0.5);
    if (clo < 0) clo = 0;
    if (chi > vw.width - 1) chi = vw.width - 1;
    if (rlo < 0) rlo = 0;
    if (rhi > vw.height - 1) rhi = vw.height - 1;
    // Reading: a projected mean 2^30 px or more from the image origin is
    // culled (the record's integer part could not hold it; such a Gaussian
    // reaches the image only through a footprint of the same size).  The
    // FP64 reference applies the same test.
    if (!(clo <= chi && rlo <= rhi && fabs(mx) < 1073741824.0 && fabs(my) < 1073741824.0)) return 0;
    const int c0 = (int)clo, c1 = (int)chi, r0 = (int)rlo, r1 = (int)rhi;
    count = (uint32_t)((c1 / kTile - c0 / kTile + 1) * (r1 / kTile - r0 / kTile + 1));
    if (rec) {
        const double ixd = floor(mx), iyd = floor(my);
        const double a_ = syy / det;  // conic entries
        const double kInv2Ln2 = 0.72134752044448170368;  // 1 / (2 ln 2)
        // the pixel-centre offset 0.5 - fraction, rounded once here rather than at every use
        rec->r0 = make_float4(__int_as_float((int)ixd), __int_as_float((int)iyd), 0.5f - (float)(mx - ixd),
                              0.5f - (float)(my - iyd));
        rec->r1 = make_float4((float)(a_ * kInv2Ln2), (float)(-sxy / syy), (float)(kInv2Ln2 / syy), (float)o);
        rec->r2 = make_float4(__uint_as_float((uint32_t)c0 | ((uint32_t)c1 << 16)),
                              __uint_as_float((uint32_t)r0 | ((uint32_t)r1 << 16)), zf, __int_as_float(v));
    }
    return count;
}

// One thread per (view, Gaussian): tile count and depth key only; the
// compositing record is recomputed later for the visible pairs alone.  Each
// workgroup also counts its visible pairs (block_vis), which is all the
// compaction needs for its prefix sums.
__global__ __launch_bounds__(256, 6) void project_kernel(ProjectArgs a, ViewChunk ch) {
    const int64_t lin = blockIdx.x * 256ll + threadIdx.x;
    if (a.init) {
        const int64_t nclear = a.num_tiles > kNumCounters ? a.num_tiles : kNumCounters;
        for (int64_t z = lin; z < nclear; z += (int64_t)gridDim.x * 256) {
            if (z < kNumCounters) a.counters[z] = 0;
            if (z < a.num_tiles) a.ranges[z] = make_uint2(0u, 0u);
        }
        if (blockIdx.x == 0 && threadIdx.x < ch.count) a.views_out[ch.first + threadIdx.x] = ch.v[threadIdx.x];
    }
    uint32_t cnt = 0;
    if (lin < a.vn) {
        const int v = (int)(lin / a.n);
        const int64_t i = lin - (int64_t)v * a.n;
        a.gp_of_lin[lin] = kInvalid;
        uint32_t zb;
        cnt = project_pair(a, a.init ? ch.v[v] : a.views[v], v, ParamsAt{a, i}, &zb, nullptr);
        a.count[lin] = cnt;
        a.zbits[lin] = zb;
    }
    const int nvis = __syncthreads_count(cnt != 0u);
    if (threadIdx.x == 0) a.block_vis[blockIdx.x] = (uint32_t)nvis;
}

// --------------------------------------------------------------- gather

// Record g of the visible pair lin (= view * n + id), built in two halves
// (build_topk, build_geom).  Bit 31 of the
// record's view word flags a Gaussian whose top-k list repeats a class (the
// LDS-accumulator forward then adds its values one at a time).  The top-k
// values and classes are stored grouped by accumulator block (class /
// kRegBlock; list order within a block); the projection backward undoes the
// grouping.  rv and rb are this thread's LDS rows (GATHER_ROW_* below): the
// stored list is scattered there and read back in order.
template <int KM>
struct GatherRow {
    static constexpr int kVals = KM + 1;               // floats per row (odd: no bank conflicts)
    static constexpr int kBytes = ((KM + 3) & ~3) + 4;  // class / list-index bytes per row
};

// The values and class indices (four per word) of pair lin's top-k list.
template <int KT>
struct TopkIn {
    static constexpr int KM = KT > 0 ? KT : kMaxK;
    float vin[KM];
    uint32_t words[(KM + 3) / 4];
};
template <int KT>
__device__ __forceinline__ void load_topk(const GatherArgs& a, uint32_t lin, TopkIn<KT>& t) {
    const int v = (int)(lin / (uint64_t)a.n);
    const int64_t i = (int64_t)lin - (int64_t)v * a.n;
    const int k = KT > 0 ? KT : a.k;
    constexpr int KM = KT > 0 ? KT : kMaxK;
    constexpr int KWM = (KM + 3) / 4;
    const float* sv = a.sem_val + i * k;
    float* vin = t.vin;
    if constexpr (KT > 0 && (KT & 3) == 0) {
#pragma unroll
        for (int m = 0; m < KT; m += 4) {
            const float4 v4 = *(const float4*)(sv + m);
            vin[m] = v4.x; vin[m + 1] = v4.y; vin[m + 2] = v4.z; vin[m + 3] = v4.w;
        }
    } else {
#pragma unroll
        for (int m = 0; m < KM; m++) vin[m] = m < k ? sv[m] : 0.f;
    }
    uint32_t* words = t.words;
    const uint8_t* si = a.sem_idx + i * k;
    if constexpr (KT > 0 && (KT & 3) == 0) {
#pragma unroll
        for (int w = 0; w < KWM; w++) words[w] = *(const uint32_t*)(si + 4 * w);
    } else {
#pragma unroll
        for (int w = 0; w < KWM; w++) {
            uint32_t word = 0;
#pragma unroll
            for (int b = 0; b < 4; b++)
                if (4 * w + b < k) word |= (uint32_t)si[4 * w + b] << (8 * b);
            words[w] = word;
        }
    }
}

// The top-k half of record g from its loaded list: stored values, classes,
// list indices and the class-rank table.  Returns whether the list repeats
// a class.
template <int KT>
__device__ __forceinline__ bool build_topk(const GatherArgs& a, uint32_t g, const TopkIn<KT>& t, float* rv,
                                           uint8_t* rc, uint8_t* ro) {
    const int k = KT > 0 ? KT : a.k;
    const int kw = (KT > 0 ? ((KT + 3) & ~3) : a.kpad) >> 2;
    constexpr int KM = KT > 0 ? KT : kMaxK;
    constexpr int KWM = (KM + 3) / 4;
    const float* vin = t.vin;
    const uint32_t* words = t.words;
    bool bad = false, dup = false;
    uint32_t cls[KM];
    uint64_t cnt = 0;  // entries per accumulator block, one byte per block (at most 8 blocks, 32 entries)
#pragma unroll
    for (int m = 0; m < KM; m++) {
        cls[m] = 0u;
        if (m < k) {
            cls[m] = (words[m >> 2] >> (8 * (m & 3))) & 0xffu;
            if ((int)cls[m] >= a.C) {  // never index past the class accumulators
                bad = true;
                cls[m] = 0u;
            }
            cnt += 1ull << (8 * (cls[m] / kRegBlock));
        }
    }
#pragma unroll
    for (int m = 0; m < KM; m++)
#pragma unroll
        for (int q = 0; q < KM; q++)
            if (q < m && m < k) dup |= cls[q] == cls[m];
    // stored position of entry m: the entries of lower blocks (an exclusive
    // prefix of the byte counts: the multiply adds every lower byte into
    // each byte, and no byte exceeds 32), then the block's earlier entries
    uint64_t run = cnt * 0x0101010101010100ull;
    uint32_t pos[KM];
    uint32_t* rcw = (uint32_t*)rc;
    uint32_t* row = (uint32_t*)ro;
#pragma unroll
    for (int w = 0; w < KWM; w++)
        if (w < kw) { rcw[w] = 0u; row[w] = 0u; }  // padding bytes past k stay 0
#pragma unroll
    for (int m = 0; m < KM; m++) {
        if (m < k) {
            const uint32_t sh = 8u * (cls[m] / kRegBlock);
            pos[m] = (uint32_t)(run >> sh) & 0xffu;
            run += 1ull << sh;
            rv[pos[m]] = vin[m];
            rc[pos[m]] = (uint8_t)cls[m];
            ro[pos[m]] = (uint8_t)m;
        }
    }
    float* dv = a.ssv + (size_t)g * k;
    if constexpr (KT > 0 && (KT & 3) == 0) {
#pragma unroll
        for (int m = 0; m < KT; m += 4) *(float4*)(dv + m) = make_float4(rv[m], rv[m + 1], rv[m + 2], rv[m + 3]);
    } else {
        for (int m = 0; m < k; m++) dv[m] = rv[m];
    }
    // classes in stored order, and the list index each stored position came
    // from (the projection backward writes the top-k value gradients back in
    // list order)
    uint32_t* di = (uint32_t*)(a.ssi + (size_t)g * a.kpad);
    uint32_t* dorig = (uint32_t*)(a.sorig + (size_t)g * a.kpad);
#pragma unroll
    for (int w = 0; w < KWM; w++)
        if (w < kw) {
            di[w] = rcw[w];
            dorig[w] = row[w];
        }
    if constexpr (KT == 16) {
        if (a.srk) {
            // class-rank table of the stored list (classes < 128 here): the
            // class mask, and for each rank the stored position of its class
            uint32_t mk[4] = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int m = 0; m < 16; m++) {
                const uint32_t c = cls[m] & 127u;
#pragma unroll
                for (int w = 0; w < 4; w++) mk[w] |= (c >> 5) == (uint32_t)w ? 1u << (c & 31u) : 0u;
            }
            const uint32_t n0 = __builtin_popcount(mk[0]), n1 = n0 + __builtin_popcount(mk[1]),
                           n2 = n1 + __builtin_popcount(mk[2]);
            uint64_t perm = 0;
#pragma unroll
            for (int m = 0; m < 16; m++) {
                const uint32_t c = cls[m] & 127u, w = c >> 5;
                const uint32_t base = w == 0 ? 0u : (w == 1 ? n0 : (w == 2 ? n1 : n2));
                const uint32_t mw = w == 0 ? mk[0] : (w == 1 ? mk[1] : (w == 2 ? mk[2] : mk[3]));
                const uint32_t rank = base + __builtin_popcount(mw & ((1u << (c & 31u)) - 1u));
                perm |= dup ? 0ull : (uint64_t)pos[m] << (4 * (rank & 15u));
            }
            uint4* dst = (uint4*)(a.srk + (size_t)g * kRankWords);
            dst[0] = make_uint4(mk[0], mk[1], mk[2], mk[3]);
            dst[1] = make_uint4((uint32_t)perm, (uint32_t)(perm >> 32), 0u, 0u);
        }
    }
    if (bad) atomicOr(&a.counters[kStatus], Plan::kBadIndex);
    return dup;
}

// The parameters, colour and tile count of pair lin.
__device__ __forceinline__ void load_geom(const GatherArgs& a, uint32_t lin, GeomIn& t) {
    const int v = (int)(lin / (uint64_t)a.n);
    const int64_t i = (int64_t)lin - (int64_t)v * a.n;
    const ProjectArgs& pa = a.proj;
#pragma unroll
    for (int r = 0; r < 3; r++) {
        t.m[r] = pa.means[3 * i + r];
        t.s[r] = pa.scales[3 * i + r];
        t.rgb[r] = a.rgb[3 * i + r];
    }
#pragma unroll
    for (int r = 0; r < 4; r++) t.q[r] = pa.quats[4 * i + r];
    t.o = pa.opacity[i];
    t.count = a.count[lin];
}

// The geometric half of record g from its loaded parameters: the
// projection (the compositing record, colour and depth) and the pair's tile
// count and depth key.
__device__ __forceinline__ void build_geom(const GatherArgs& a, uint32_t g, uint32_t lin, bool dup, const GeomIn& t) {
    const int v = (int)(lin / (uint64_t)a.n);
    Proj p;
    uint32_t zb;
    project_pair(a.proj, a.proj.views[v], v, t, &zb, &p);
    a.zkeys[g] = zb;
    a.pair_lin[g] = lin;
    a.scol[g] = make_float4(t.rgb[0], t.rgb[1], t.rgb[2], p.r2.z);
    p.r2.w = __uint_as_float(__float_as_uint(p.r2.w) | (dup ? 0x80000000u : 0u));
    a.srec[g] = p;
    a.tcount[g] = t.count;
    a.gp_of_lin[lin] = g;
}

// Compaction of the visible pairs with their records, in (view, Gaussian id)
// order: a workgroup takes kScanTile consecutive pairs, lists the visible
// ones in LDS, and builds their records with every lane busy.  Records are
// numbered in that order (partial[b]: visible pairs of the projection's
// block b of 256 pairs; each workgroup adds up those before its own), so
// the parameter reads run forward
// through memory; the depth sort then orders record numbers.  The last
// workgroup writes the visible count.
constexpr int kGatherThreads = 256;
constexpr uint32_t kGatherSumBlocks = 512;  // above this many workgroups the block counts are scanned first
constexpr int kGatherItems = kScanTile / kGatherThreads;

template <int KT>
__global__ __launch_bounds__(kGatherThreads, KT > 0 ? 3 : 1) void compact_gather(GatherArgs a) {
    constexpr int NW = kGatherThreads / 64;
    __shared__ uint32_t wsum[NW];
    __shared__ uint32_t s_before, s_nloc;
    __shared__ uint32_t s_lin[kScanTile];
    constexpr int KM = KT > 0 ? KT : kMaxK;
    using Row = GatherRow<KM>;
    __shared__ float s_rv[kGatherThreads * Row::kVals];
    __shared__ __align__(4) uint8_t s_rc[kGatherThreads * Row::kBytes];
    __shared__ __align__(4) uint8_t s_ro[kGatherThreads * Row::kBytes];
    __shared__ uint8_t s_dup[kScanTile];
    const int64_t vn = a.proj.vn;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    {
        // visible pairs before this workgroup's block: the projection's
        // counts of the 256-pair blocks before it (summed here when there
        // are few workgroups, else scanned beforehand)
        uint32_t before = 0;
        const uint32_t nb = blockIdx.x * (kScanTile / 256);
        if (a.partial_scanned) {
            if (tid == 0) before = a.partial[nb];
        } else {
            for (uint32_t b = tid; b < nb; b += kGatherThreads) before += a.partial[b];
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) before += __shfl_xor(before, o, 64);
        if (lane == 0) wsum[w] = before;
        __syncthreads();
        if (tid == 0) {
            uint32_t t = 0;
            for (int j = 0; j < NW; j++) t += wsum[j];
            s_before = t;
        }
        __syncthreads();
    }
    const int64_t base = blockIdx.x * (int64_t)kScanTile + tid * kGatherItems;
    uint32_t f[kGatherItems], s = 0;
#pragma unroll
    for (int r = 0; r < kGatherItems; r++) {
        const int64_t i = base + r;
        f[r] = (i < vn && a.count[i] != 0u) ? 1u : 0u;
        s += f[r];
    }
    // block exclusive scan of the flags
    uint32_t x = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint32_t pre = x - s;
    for (int j = 0; j < w; j++) pre += wsum[j];
    if (tid == kGatherThreads - 1) {
        s_nloc = pre + s;
        if (blockIdx.x == gridDim.x - 1) a.counters[kNumVisible] = s_before + pre + s;  // every visible pair
    }
#pragma unroll
    for (int r = 0; r < kGatherItems; r++)
        if (f[r]) s_lin[pre++] = (uint32_t)(base + r);
    __syncthreads();
    const uint32_t nloc = s_nloc, before = s_before;
    // two passes over this thread's records (the same ones in both), each
    // with fewer live registers than one pass that did both halves; each
    // loads the next record's inputs before it builds the current one
    if constexpr (KT > 0) {
        TopkIn<KT> cur, nxt;
        if ((uint32_t)tid < nloc) load_topk<KT>(a, s_lin[tid], cur);
        for (uint32_t j = tid; j < nloc; j += kGatherThreads) {
            if (j + kGatherThreads < nloc) load_topk<KT>(a, s_lin[j + kGatherThreads], nxt);
            s_dup[j] = build_topk<KT>(a, before + j, cur, s_rv + tid * Row::kVals, s_rc + tid * Row::kBytes,
                                      s_ro + tid * Row::kBytes) ? 1 : 0;
            cur = nxt;
        }
    } else {  // (a run-time list length: lists of up to kMaxK entries, loaded one at a time)
        for (uint32_t j = tid; j < nloc; j += kGatherThreads) {
            TopkIn<KT> cur;
            load_topk<KT>(a, s_lin[j], cur);
            s_dup[j] = build_topk<KT>(a, before + j, cur, s_rv + tid * Row::kVals, s_rc + tid * Row::kBytes,
                                      s_ro + tid * Row::kBytes) ? 1 : 0;
        }
    }
    {
        GeomIn cur, nxt;
        if ((uint32_t)tid < nloc) load_geom(a, s_lin[tid], cur);
        for (uint32_t j = tid; j < nloc; j += kGatherThreads) {
            if (j + kGatherThreads < nloc) load_geom(a, s_lin[j + kGatherThreads], nxt);
            build_geom(a, before + j, s_lin[j], s_dup[j] != 0, cur);
            cur = nxt;
        }
    }
}

// --------------------------------------------------------------- keys

// Keys are emitted in depth order, in chunks of kKeyChunk consecutive keys,
// one chunk per workgroup, so a pair near the camera that covers thousands
// of tiles is spread over many workgroups.  The scan of the pairs' key counts
// records, for every chunk, the depth rank of the pair that owns its first
// key (the pair at depth rank r, record order[r], owns keys [toff[r], toff[r]
// + tcount[r])) in heads.

// Workgroup q emits keys [q C, q C + C) (C = kKeyChunk): the pairs that own
// them, heads[q] onwards, go to LDS (offsets, tile rectangle and record),
// and each key finds its owner there (marks and a max-scan over the chunk's
// positions, below).  A pair owns at least
// one key, so at most C + 1 pairs meet a chunk; longer runs (pairs with none)
// are taken in windows of that size.  owner[e] is the record of key e's
// pair.
__global__ __launch_bounds__(256) void emit_keys(KeyArgs a) {
    static_assert(kKeyChunk == kRadixTileSmall && kKeyChunk == kRadixTileMid,
                  "a chunk of keys is a block of the tile sort (when hist0 is set)");
    constexpr int W = kKeyChunk + 1;
    __shared__ uint32_t off[W + 1];
    __shared__ uint32_t s_hist[256];  // counts of the sort's first digit among this chunk's keys
    __shared__ int32_t info[W][4];  // first global tile of the rect, rect width in tiles, view width in tiles, record
    __shared__ uint32_t s_own[kKeyChunk];  // owner (window index) of each key of the window's range
    __shared__ uint32_t s_wmax[4];
    const uint32_t nv = a.counters[kNumVisible];
    const uint64_t K = min((uint64_t)a.counters[kKeysLo], (uint64_t)a.cap);
    const uint64_t e0 = (uint64_t)blockIdx.x * kKeyChunk;
    if (e0 >= K || nv == 0) return;
    const uint64_t e1 = min(e0 + kKeyChunk, K);
    const uint32_t dmask = a.hist_bins - 1u;
    for (uint32_t d = threadIdx.x; d < a.hist_bins; d += 256) s_hist[d] = 0u;  // (read after the loop's barriers)
    uint32_t w0 = a.heads[blockIdx.x];
    // the pairs that own this chunk's keys end with the owner of the next
    // chunk's first key (recorded when that chunk exists)
    const uint32_t wend = e1 < K ? min(nv, a.heads[blockIdx.x + 1] + 1) : nv;
    while (true) {
        // window of pairs [w0, w0 + nw)
        const uint32_t nw = min((uint32_t)W, wend - w0);
        for (uint32_t i = threadIdx.x; i < nw; i += 256) {
            const uint32_t r = w0 + i, g = a.order[r];
            off[i] = a.toff[r];
            const float4 r2 = a.srec[g].r2;
            const uint32_t rx = __float_as_uint(r2.x), ry = __float_as_uint(r2.y);
            const int v = __float_as_int(r2.w) & 0x7fffffff;
            const int tx0 = (int)(rx & 0xffffu) / kTile, tx1 = (int)(rx >> 16) / kTile;
            const int ty0 = (int)(ry & 0xffffu) / kTile;
            const ViewDev& vw = a.views[v];
            info[i][0] = vw.tile_off + ty0 * vw.tiles_x + tx0;
            info[i][1] = tx1 - tx0 + 1;
            info[i][2] = vw.tiles_x;
            info[i][3] = (int32_t)g;
            if (i == nw - 1) off[nw] = a.toff[r] + a.tcount[r];
        }
        __syncthreads();
        // keys of this chunk owned by the window's pairs
        const uint64_t k0 = max(e0, (uint64_t)off[0]), k1 = min(e1, (uint64_t)off[nw]);
        const uint32_t nk = (uint32_t)(k1 - k0);  // at most kKeyChunk
        // owner of key k0 + p (the last pair j with off[j] <= k0 + p): each
        // pair with keys here marks where its keys start (one pair per
        // position), then an inclusive max-scan carries the marks forward
        for (uint32_t q = threadIdx.x; q < kKeyChunk; q += 256) s_own[q] = 0;
        __syncthreads();
        for (uint32_t j = threadIdx.x; j < nw; j += 256) {
            const uint64_t b = max((uint64_t)off[j], k0);
            if (b < k1 && off[j + 1] > b) s_own[b - k0] = j;
        }
        __syncthreads();
        {
            constexpr int PT = kKeyChunk / 256;  // positions per thread, in order
            uint32_t own[PT], m = 0;
#pragma unroll
            for (int u = 0; u < PT; u++) {
                m = max(m, s_own[threadIdx.x * PT + u]);
                own[u] = m;
            }
            // exclusive max over the threads before this one
            const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
            uint32_t x = m;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = __shfl_up(x, o, 64);
                if (lane >= o) x = max(x, y);
            }
            if (lane == 63) s_wmax[wv] = x;
            uint32_t before = __shfl_up(x, 1, 64);
            if (lane == 0) before = 0;
            __syncthreads();
            for (int w = 0; w < wv; w++) before = max(before, s_wmax[w]);
#pragma unroll
            for (int u = 0; u < PT; u++) s_own[threadIdx.x * PT + u] = max(own[u], before);
        }
        __syncthreads();
        for (uint32_t p = threadIdx.x; p < nk; p += 256) {
            const uint64_t e = k0 + p;
            const int lo = (int)s_own[p];
            const uint32_t local = (uint32_t)(e - off[lo]);
            const uint32_t wdt = (uint32_t)info[lo][1];
            const uint32_t gt = (uint32_t)info[lo][0] + (local / wdt) * (uint32_t)info[lo][2] + local % wdt;
            a.keys[e] = gt;
            a.owner[e] = (uint32_t)info[lo][3];
            if (a.hist0) atomicAdd(&s_hist[gt & dmask], 1u);
        }
        // the same for every thread: taken as a scalar, so the loop exit is uniform
        const int more = __builtin_amdgcn_readfirstlane((uint64_t)off[nw] < e1 && w0 + nw < wend ? 1 : 0);
        __syncthreads();  // the window is read before it is replaced
        if (!more) break;
        w0 += nw;
    }
    // this block's first-digit counts (the loop ended at a barrier)
    if (!a.hist0) return;
    const uint32_t nblk = (uint32_t)div_up((int64_t)K, kKeyChunk);
    for (uint32_t d = threadIdx.x; d < a.hist_bins; d += 256)
        a.hist0[a.hist_block_major ? blockIdx.x * a.hist_bins + d : d * nblk + blockIdx.x] = s_hist[d];
}

// [start, end) of every non-empty tile.  (The compositing kernels find the
// pair of sorted key s as owner[svals[s]], inside their staging prefetch.)
__global__ __launch_bounds__(256) void tile_ranges(const uint32_t* __restrict__ skeys, uint2* __restrict__ ranges,
                                                   const uint32_t* __restrict__ counters, uint32_t cap) {
    // four consecutive keys per thread (one 16-byte load; the sorted keys
    // are 16-byte aligned), with the keys either side of them
    const uint32_t s0 = (blockIdx.x * 256u + threadIdx.x) * 4u;
    const uint32_t K = min(counters[kKeysLo], cap);
    if (counters[kStatus] & SGR_ECAPACITY) return;
    if (s0 >= K) return;
    uint32_t k[6];
    if (s0 + 4u <= K) {
        const uint4 q = *reinterpret_cast<const uint4*>(skeys + s0);
        k[1] = q.x; k[2] = q.y; k[3] = q.z; k[4] = q.w;
    } else {
#pragma unroll
        for (uint32_t u = 0; u < 4u; u++) k[1 + u] = s0 + u < K ? skeys[s0 + u] : 0u;
    }
    k[0] = s0 > 0u ? skeys[s0 - 1u] : 0u;
    k[5] = s0 + 4u < K ? skeys[s0 + 4u] : 0u;
#pragma unroll
    for (uint32_t u = 0; u < 4u; u++) {
        const uint32_t s = s0 + u;
        if (s >= K) break;
        const uint32_t key = k[1 + u];
        if (s == 0u || k[u] != key) ranges[key].x = s;
        if (s == K - 1u || k[2 + u] != key) ranges[key].y = s + 1u;
    }
}

// --------------------------------------------------------------- launchers

// R and t of view v from poses[v][12] (R row-major, then t).
__global__ __launch_bounds__(256) void set_view_poses(ViewDev* views, const float* __restrict__ poses, int V) {
    const int v = blockIdx.x * 256 + threadIdx.x;
    if (v >= V) return;
    for (int c = 0; c < 9; c++) views[v].R[c] = poses[12 * v + c];
    for (int c = 0; c < 3; c++) views[v].t[c] = poses[12 * v + 9 + c];
}

sgr_status launch_project(const Plan& P, const sgr_gaussians* g, char* ws, hipStream_t st, const float* d_poses) {
    ViewDev* views = (ViewDev*)(ws + P.views);
    uint32_t* counters = (uint32_t*)(ws + P.counters);
    // camera table, as kernel arguments: the first chunk with the counter
    // clear, any further chunks on their own
    auto chunk = [&](int first) {
        ViewChunk ch;
        memset(&ch, 0, sizeof(ch));
        ch.first = first;
        ch.count = std::min(kViewChunk, P.V - first);
        for (int j = 0; j < ch.count; j++) ch.v[j] = P.view_table[first + j];
        return ch;
    };
    // With one chunk of views and host poses (and some pair to project), the
    // projection launch initialises the frame itself; otherwise a separate
    // launch does, and further chunks and device poses follow it.
    const bool fold = P.V <= kViewChunk && !d_poses && P.vn > 0;
    if (!fold) {
        const int64_t nthreads = std::max<int64_t>(P.num_tiles, kNumCounters);
        init_frame<<<(unsigned)div_up(nthreads, 256), 256, 0, st>>>(counters, (uint2*)(ws + P.ranges), P.num_tiles,
                                                                    chunk(0), views);
        for (int first = kViewChunk; first < P.V; first += kViewChunk)
            upload_views<<<1, kViewChunk, 0, st>>>(chunk(first), views);
        if (d_poses) set_view_poses<<<(unsigned)div_up(P.V, 256), 256, 0, st>>>(views, d_poses, P.V);
    }
    ProjectArgs pa;
    pa.means = g->means; pa.scales = g->scales; pa.quats = g->quats; pa.opacity = g->opacity;
    pa.views = views; pa.n = P.n; pa.vn = P.vn;
    pa.alpha_min = P.cfg.alpha_min; pa.z_near = P.cfg.z_near; pa.lowpass = P.cfg.lowpass;
    pa.count = (uint32_t*)(ws + P.count); pa.zbits = (uint32_t*)(ws + P.zbits);
    pa.gp_of_lin = (uint32_t*)(ws + P.gp_of_lin);
    pa.block_vis = (uint32_t*)(ws + P.block_vis);
    pa.init = fold ? 1 : 0;
    pa.counters = counters; pa.ranges = (uint2*)(ws + P.ranges); pa.num_tiles = P.num_tiles; pa.views_out = views;
    if (P.vn == 0) return hipGetLastError() == hipSuccess ? SGR_OK : SGR_EHIP;
    project_kernel<<<(unsigned)div_up(P.vn, 256), 256, 0, st>>>(pa, chunk(0));
    // compaction of visible pairs with their records, then the depth sort
    // of record numbers
    uint32_t* partial = (uint32_t*)(ws + P.partial);
    GatherArgs ga;
    ga.partial = pa.block_vis; ga.proj = pa; ga.count = pa.count;
    ga.rgb = g->rgb; ga.sem_val = g->sem_val; ga.sem_idx = g->sem_idx;
    ga.n = P.n; ga.k = P.k; ga.kpad = P.kpad; ga.C = P.C; ga.counters = counters;
    ga.srec = (Proj*)(ws + P.srec); ga.scol = (float4*)(ws + P.scol); ga.ssv = (float*)(ws + P.ssv);
    ga.ssi = (uint8_t*)(ws + P.ssi); ga.srk = P.ranked ? (uint32_t*)(ws + P.srk) : nullptr;
    ga.sorig = (uint8_t*)(ws + P.sorig); ga.tcount = (uint32_t*)(ws + P.tcount_rec); ga.gp_of_lin = pa.gp_of_lin;
    ga.pair_lin = (uint32_t*)(ws + P.pair_lin); ga.zkeys = (uint32_t*)(ws + P.vis_k0);
    {
        const uint32_t nblk = (uint32_t)div_up(P.vn, kScanTile);
        // Each compaction workgroup needs the visible pairs before its block.
        // With few workgroups each adds up the counts itself; with many (a
        // batch of views), summing them all would grow with the square of
        // the count, so an exclusive scan of the counts comes first.
        ga.partial_scanned = nblk > kGatherSumBlocks ? 1 : 0;
        if (ga.partial_scanned) {
            const uint32_t nvb = (uint32_t)div_up(P.vn, 256);
            scan_exclusive(pa.block_vis, pa.block_vis, host_count(nvb), nvb, partial, nullptr, 0, nullptr, st);
        }
        if (P.k == 16) compact_gather<16><<<nblk, kGatherThreads, 0, st>>>(ga);
        else if (P.k == 3) compact_gather<3><<<nblk, kGatherThreads, 0, st>>>(ga);
        else compact_gather<0><<<nblk, kGatherThreads, 0, st>>>(ga);
    }
    // (fp32 depth bits, record) pairs; records are numbered in id order, so
    // a stable sort on the bits alone gives the (depth, id) order.  32 bits
    // in 4 (8-bit digits) or 6 (6-bit digits) passes: the record numbers end
    // in the *0 buffers (P.order).  The last pass also writes each pair's
    // tile count by depth rank.
    const int passes = radix_sort((uint32_t*)(ws + P.vis_k0), (uint32_t*)(ws + P.vis_v0), (uint32_t*)(ws + P.vis_k1),
                                  (uint32_t*)(ws + P.vis_v1), true, device_count(counters + kNumVisible, 0),
                                  (uint32_t)P.vn, 32, (uint32_t*)(ws + P.hist), partial, st, P.radix_bits,
                                  ga.tcount, (uint32_t*)(ws + P.tcount));
    if (passes & 1) return SGR_EUNSUPPORTED;
    return hipGetLastError() == hipSuccess ? SGR_OK : SGR_EHIP;
}

sgr_status launch_bin(const Plan& P, char* ws, int64_t* d_num_keys, hipStream_t st) {
    uint32_t* counters = (uint32_t*)(ws + P.counters);
    uint32_t* partial = (uint32_t*)(ws + P.partial);
    uint32_t* tcount = (uint32_t*)(ws + P.tcount);
    uint32_t* toff = (uint32_t*)(ws + P.toff);
    const uint32_t* order = (const uint32_t*)(ws + P.order);
    // key offsets of the pairs in depth order; the total is the key count K.
    // The scan also records, for every chunk of kKeyChunk keys, the depth
    // rank of the pair that owns its first key.
    scan_exclusive(tcount, toff, device_count(counters + kNumVisible, 0), (uint32_t)P.vn, partial,
                   counters + kKeysLo, (uint32_t)P.cap, counters + kStatus, st, (uint32_t*)(ws + P.heads),
                   (uint32_t)kKeyChunk);
    KeyArgs ka;
    ka.toff = toff; ka.tcount = tcount; ka.order = order; ka.srec = (const Proj*)(ws + P.srec); ka.views = (const ViewDev*)(ws + P.views);
    ka.counters = counters; ka.cap = P.cap;
    ka.keys = (uint32_t*)(ws + P.keys0); ka.owner = (uint32_t*)(ws + P.owner);
    ka.heads = (uint32_t*)(ws + P.heads);
    // When the tile sort's blocks are the chunks of emission, the emission
    // counts the first digit of each block (the sort then has no histogram
    // launch for that pass); larger sorts take longer blocks.
    const RadixFirstPass fp = radix_first_pass((uint32_t)P.cap, P.tile_bits, P.radix_bits);
    const bool counted = fp.tile == (uint32_t)kKeyChunk && P.vn > 0;
    ka.hist0 = counted ? (uint32_t*)(ws + P.hist) : nullptr;
    ka.hist_bins = fp.bins;
    ka.hist_block_major = fp.block_major;
    if (P.vn > 0) emit_keys<<<(unsigned)div_up(P.cap, kKeyChunk), 256, 0, st>>>(ka);
    const int passes = radix_sort((uint32_t*)(ws + P.keys0), (uint32_t*)(ws + P.vals0), (uint32_t*)(ws + P.keys1),
                                  (uint32_t*)(ws + P.vals1), true, device_count(counters + kKeysLo, (uint32_t)P.cap),
                                  (uint32_t)P.cap, P.tile_bits, (uint32_t*)(ws + P.hist), partial, st, P.radix_bits,
                                  nullptr, nullptr, counted);
    if (passes != P.tile_passes) return SGR_EUNSUPPORTED;
    tile_ranges<<<(unsigned)div_up(P.cap, 1024), 256, 0, st>>>((const uint32_t*)(ws + P.sorted_keys),
                                                              (uint2*)(ws + P.ranges), counters, (uint32_t)P.cap);
    if (d_num_keys) publish_num_keys<<<1, 1, 0, st>>>(counters, d_num_keys);
    return hipGetLastError() == hipSuccess ? SGR_OK : SGR_EHIP;
}

}  // namespace sgr
