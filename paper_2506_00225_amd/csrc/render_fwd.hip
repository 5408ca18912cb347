// Front-to-back compositing (Eq. 1, Eq. 3) per 16x16 tile, and the
// persistent candidate-view scorer (Eq. 4-6) built on the same tile body.
#include "pipeline.h"
#include "render_common.h"

namespace sgr {

// Classes [lo, lo + cnt) of the tile's pixels from LDS rows (stride 257)
// into the [H][W][C] map: each pixel's run of cnt classes is contiguous.
__device__ __forceinline__ void write_rows_range(const float* smem, float* out, const ViewDev& vw, int C, int lo,
                                                 int cnt, int tx, int ty) {
    const int x0 = tx * kTile, y0 = ty * kTile;
    const int wcols = min(kTile, vw.width - x0), hrows = min(kTile, vw.height - y0);
    const int row_elems = kTile * cnt;
    const int dl = kBlock / cnt, dc = kBlock % cnt;
    for (int row = 0; row < hrows; row++) {
        float* dst = out + ((int64_t)(y0 + row) * vw.width + x0) * C + lo;
        int lx = threadIdx.x / cnt, c = threadIdx.x % cnt;
        for (int e = threadIdx.x; e < row_elems; e += kBlock) {
            if (lx < wcols) dst[lx * C + c] = smem[c * kAccStride + slot_of(lx, row)];
            lx += dl;
            c += dc;
            if (c >= cnt) { c -= cnt; lx++; }
        }
    }
}

// Per-tile compositing.  One thread per pixel (256 = 4 wave64).  Batches of
// the tile's front-to-back list are staged in LDS; every lane reads the
// same record (an LDS broadcast).  Semantic accumulators (SEM):
//   0  none;
//   1  LDS, class-major with a 257-float stride: the 64 lanes of a wave
//      update 64 consecutive floats of one class row, conflict-free;
//   2  the thread's own row of the output map (when LDS is too small);
//   3  registers, NB vectors of 32 classes (C <= 128): no LDS, so more
//      waves fit on a CU;
//   4  only the class sum at the pixel's label (a cross-entropy target
//      needs no other class): one register per pixel, no LDS.
// Every mode adds a blend's values in the same order with the same fused
// multiply-add, so they give the same bits.
//
// NPASS > 1 (SEM == 1): the LDS holds `rows` class rows and this call
// accumulates only classes [lo, lo + cnt); the caller walks the tile once
// per class range.  Half the LDS per workgroup lets two workgroups share a
// CU, at the price of recompositing the geometry in every pass.
template <int KT, int SEM, int NB, int NPASS = 1>
__device__ __forceinline__ void composite_tile(const TileArgs& a, int gt, float* smem, TileResult& res,
                                               RegAcc<NB>& racc, int lo = 0, int cnt = 0, int rows = 0) {
    const int tid = threadIdx.x;
    const int k = KT > 0 ? KT : a.k;
    const int kw = (KT > 0 ? ((KT + 3) & ~3) : a.kpad) >> 2;  // index words per Gaussian
    const int C = a.C;
    if constexpr (NPASS == 1) {
        lo = 0;
        cnt = C;
        rows = C;
    }
    float* acc = smem;                                   // [rows][257] when SEM == 1
    float* bat = smem + (SEM == 1 ? acc_floats(rows) : 0);
    float4* s_r0 = (float4*)bat;
    float4* s_r1 = s_r0 + kFwdBatch;
    float4* s_r2 = s_r1 + kFwdBatch;
    float4* s_col = s_r2 + kFwdBatch;
    float* s_sv = (float*)(s_col + kFwdBatch);
    uint32_t* s_si = (uint32_t*)(s_sv + kFwdBatch * k);
    // Label-only sums with k = 16 and C <= 128: each staged entry also
    // carries its classes as a 128-bit mask, four (mask word, classes in
    // lower words) pairs and a zero pair, and (distinct classes) its values
    // in class order, so a pixel finds its label's value with one mask
    // lookup and one read instead of 16 compares.
    constexpr bool RANKED = SEM == 4 && KT == 16;
    uint2* s_lm = (uint2*)(s_si + kFwdBatch * kw);  // [kFwdBatch][5]
    const bool ranked = RANKED && C <= 128;

    const int v = view_of_tile(a.views, a.V, gt);
    const ViewDev& vw = a.views[v];
    const int local = gt - vw.tile_off;
    const int tx = local % vw.tiles_x, ty = local / vw.tiles_x;
    const int px = tx * kTile + tile_px(tid), py = ty * kTile + tile_py(tid);
    const bool inside = px < vw.width && py < vw.height;
    const uint2 rg = a.ranges[gt];
    const uint32_t start = rg.x, end = rg.y;

    if (SEM == 1)
        for (int i = tid; i < cnt * kAccStride; i += kBlock) acc[i] = 0.f;
    if constexpr (SEM == 3) reg_zero(racc);
    int lab = -1;
    float ql = 0.f;
    if (SEM == 4) {
        const int32_t* lm = a.loss_views[v].label;
        if (inside && lm) lab = lm[(int64_t)py * vw.width + px];
        // taken here, so the compositing loop does not wait on the batch
        // prefetch loads issued after it
        asm volatile("" : "+v"(lab));
    }
    // the label's mask word (4: the zero pair, for no label or one >= 128),
    // its bit and the bits below it
    const int lword = (lab >= 0 && lab < 128) ? (lab >> 5) : 4;
    const uint32_t lbit = (uint32_t)lab & 31u, lbelow = (1u << lbit) - 1u;
    float* gacc = nullptr;  // SEM == 2: the thread's own row of the output map
    if (SEM == 2 && inside && a.maps[v].sem) {
        gacc = a.maps[v].sem + ((int64_t)py * vw.width + px) * C;
        for (int c = 0; c < C; c++) gacc[c] = 0.f;
    }

    float T = 1.f, cr = 0.f, cg = 0.f, cb = 0.f, dd = 0.f, ss = 0.f;
    int ncon = 0;
    uint32_t last = start;
    bool done = !inside;
    const float amin = a.alpha_min, amax = a.alpha_max, tmin = a.t_min;
    const int wv = tid >> 6, lane = tid & 63;
    const int wx0 = tx * kTile + (wv & 1) * 8, wy0 = ty * kTile + (wv >> 1) * 8;  // this wave's 8x8 block

    // Staging registers: thread j < kFwdBatch carries list entry j's record
    // and colour, thread kFwdBatch + j its top-k values and class indices.
    // The next batch is fetched into them while the current one is composited.
    constexpr int KM = KT > 0 ? KT : kMaxK;
    constexpr int KWM = (KM + 3) / 4;
    // With the class sums in LDS in one pass and k fixed at compile time, a
    // staged entry carries its classes as byte offsets of their accumulator
    // rows (class * 257 * 4), so a blend does no index decoding.
    constexpr bool OFFS = SEM == 1 && NPASS == 1 && KT > 0;
    constexpr int KIDX = OFFS ? KM : KWM;  // index words per staged entry
    // One register array serves both roles (record: r0, r1, r2, colour as
    // 16 words; semantics: KM values then KIDX index words).
    constexpr int KSTG = (KM + KIDX) > 16 ? (KM + KIDX) : 16;
    uint32_t stg[KSTG];
#pragma unroll
    for (int q = 0; q < KSTG; q++) stg[q] = 0u;
    auto fetch = [&](uint32_t f0, int fn) {
        if (tid < kFwdBatch) {
            if (tid < fn) {
                const uint32_t g = a.owner[a.svals[f0 + tid]];
                const float4* rp = (const float4*)(a.srec + g);
                const float4 r[4] = {rp[0], rp[1], rp[2], a.scol[g]};
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    stg[4 * q] = __float_as_uint(r[q].x);
                    stg[4 * q + 1] = __float_as_uint(r[q].y);
                    stg[4 * q + 2] = __float_as_uint(r[q].z);
                    stg[4 * q + 3] = __float_as_uint(r[q].w);
                }
            }
        } else if (SEM != 0 && tid - kFwdBatch < fn) {
            const uint32_t g = a.owner[a.svals[f0 + tid - kFwdBatch]];
            const float* sv = a.ssv + (size_t)g * k;
            if constexpr (KT > 0 && (KT & 3) == 0) {
#pragma unroll
                for (int m = 0; m < KM; m += 4) {
                    const float4 v4 = *(const float4*)(sv + m);
                    stg[m] = __float_as_uint(v4.x);
                    stg[m + 1] = __float_as_uint(v4.y);
                    stg[m + 2] = __float_as_uint(v4.z);
                    stg[m + 3] = __float_as_uint(v4.w);
                }
            } else {
#pragma unroll
                for (int m = 0; m < KM; m++)
                    if (m < k) stg[m] = __float_as_uint(sv[m]);
            }
            const uint32_t* si = (const uint32_t*)(a.ssi) + (size_t)g * kw;
            if constexpr (OFFS) {
#pragma unroll
                for (int mw = 0; mw < KWM; mw++) {
                    const uint32_t word = si[mw];
#pragma unroll
                    for (int b = 0; b < 4; b++)
                        if (mw * 4 + b < KM) stg[KM + mw * 4 + b] = ((word >> (8 * b)) & 0xffu) * (kAccStride * 4);
                }
            } else {
#pragma unroll
                for (int m = 0; m < KWM; m++)
                    if (m < kw) stg[KM + m] = si[m];
            }
        }
    };

    if (start < end) fetch(start, (int)min((uint32_t)kFwdBatch, end - start));
    for (uint32_t b0 = start; b0 < end; b0 += kFwdBatch) {
        if (__builtin_amdgcn_readfirstlane(__syncthreads_count(done)) == kBlock) break;
        const int nb = (int)min((uint32_t)kFwdBatch, end - b0);
        if (tid < kFwdBatch) {
            if (tid < nb) {
                s_r0[tid] = make_float4(__uint_as_float(stg[0]), __uint_as_float(stg[1]), __uint_as_float(stg[2]),
                                        __uint_as_float(stg[3]));
                s_r1[tid] = make_float4(__uint_as_float(stg[4]), __uint_as_float(stg[5]), __uint_as_float(stg[6]),
                                        __uint_as_float(stg[7]));
                s_r2[tid] = make_float4(__uint_as_float(stg[8]), __uint_as_float(stg[9]), __uint_as_float(stg[10]),
                                        __uint_as_float(stg[11]));
                s_col[tid] = make_float4(__uint_as_float(stg[12]), __uint_as_float(stg[13]),
                                         __uint_as_float(stg[14]), __uint_as_float(stg[15]));
            }
        } else if (SEM != 0) {
            const int j = tid - kFwdBatch;
            if (RANKED && ranked && j < nb) {
                // class mask, classes in lower words, and the values in class
                // order when the classes are distinct (list order otherwise)
                uint32_t mk[4] = {0u, 0u, 0u, 0u};
#pragma unroll
                for (int m = 0; m < 16; m++) {
                    const uint32_t c = (stg[KM + (m >> 2)] >> (8 * (m & 3))) & 0xffu;
                    const uint32_t bit = 1u << (c & 31u), wsel = c >> 5;
#pragma unroll
                    for (int q = 0; q < 4; q++) mk[q] |= wsel == (uint32_t)q ? bit : 0u;
                }
                uint32_t below[4], nset = 0;
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    below[q] = nset;
                    nset += __builtin_popcount(mk[q]);
                    s_lm[j * 5 + q] = make_uint2(mk[q], below[q]);
                }
                s_lm[j * 5 + 4] = make_uint2(0u, 0u);
                const bool distinct = nset == 16u;
#pragma unroll
                for (int m = 0; m < 16; m++) {
                    const uint32_t c = (stg[KM + (m >> 2)] >> (8 * (m & 3))) & 0xffu;
                    const uint32_t wsel = c >> 5, lowbits = (1u << (c & 31u)) - 1u;
                    uint32_t word = mk[0], pre = below[0];
#pragma unroll
                    for (int q = 1; q < 4; q++) {
                        word = wsel == (uint32_t)q ? mk[q] : word;
                        pre = wsel == (uint32_t)q ? below[q] : pre;
                    }
                    const uint32_t pos = distinct ? pre + __builtin_popcount(word & lowbits) : (uint32_t)m;
                    s_sv[j * 16 + pos] = __uint_as_float(stg[m]);
                }
#pragma unroll
                for (int m = 0; m < KWM; m++) s_si[j * kw + m] = stg[KM + m];
            } else if (j < nb) {
#pragma unroll
                for (int m = 0; m < KM; m++)
                    if (m < k) s_sv[j * k + m] = __uint_as_float(stg[m]);
                if constexpr (OFFS) {
#pragma unroll
                    for (int m = 0; m < KM; m++) s_si[j * KM + m] = stg[KM + m];
                } else {
#pragma unroll
                    for (int m = 0; m < KWM; m++)
                        if (m < kw) s_si[j * kw + m] = stg[KM + m];
                }
            }
        }
        __syncthreads();
        if (b0 + kFwdBatch < end) fetch(b0 + kFwdBatch, (int)min((uint32_t)kFwdBatch, end - b0 - kFwdBatch));

        // Entries that can reach a pixel of this wave's block (pixel
        // rectangle, then ellipse), as two 64-bit masks (entries lane and
        // 64 + lane).
        bool h0 = false, h1 = false;
#pragma unroll
        for (int half = 0; half < 2; half++) {
            const int j = half * 64 + lane;
            if (j < nb) {
                const float4 q2 = s_r2[j];
                const uint32_t rx = __float_as_uint(q2.x), ry = __float_as_uint(q2.y);
                const int bx0 = max(wx0, (int)(rx & 0xffffu)), bx1 = min(wx0 + 7, (int)(rx >> 16));
                const int by0 = max(wy0, (int)(ry & 0xffffu)), by1 = min(wy0 + 7, (int)(ry >> 16));
                bool h = bx0 <= bx1 && by0 <= by1;
                if (h) h = conic_meets_block(s_r0[j], s_r1[j], bx0, bx1, by0, by1, amin);
                if (half == 0) h0 = h; else h1 = h;
            }
        }
        uint64_t mlo = __ballot(h0), mhi = __ballot(h1);
        auto next = [&]() -> int {
            if (mlo) {
                const int j = __builtin_ctzll(mlo);
                mlo &= mlo - 1;
                return j;
            }
            if (mhi) {
                const int j = 64 + __builtin_ctzll(mhi);
                mhi &= mhi - 1;
                return j;
            }
            return -1;
        };
        // Every lane takes every entry of the wave's mask, with w = 0 where
        // it does not blend (outside the rectangle, alpha below the cutoff,
        // terminated): adding 0 leaves a sum's bits unchanged, so lanes need
        // no branches; an entry no lane blends is skipped as a whole.  The
        // next entry's record is loaded before this one's updates.
        if (__ballot(!done) == 0) continue;
        int jn = next();
        float4 n0 = {}, n1 = {}, n2 = {};
        if (jn >= 0) {
            n0 = s_r0[jn];
            n1 = s_r1[jn];
            n2 = s_r2[jn];
        }
        while (jn >= 0) {
            const int j = jn;
            const float4 q0 = n0, q1 = n1, q2 = n2;
            jn = next();
            if (jn >= 0) {
                n0 = s_r0[jn];
                n1 = s_r1[jn];
                n2 = s_r2[jn];
            }
            const uint32_t rx = __float_as_uint(q2.x), ry = __float_as_uint(q2.y);
            const bool inr = !done && px >= (int)(rx & 0xffffu) && px <= (int)(rx >> 16) &&
                             py >= (int)(ry & 0xffffu) && py <= (int)(ry >> 16);
            float G, dx, dy;
            const float alpha = eval_alpha(q0, q1, px, py, amax, &G, &dx, &dy);
            const bool pass = inr && alpha >= amin;
            const float Tn = T * (1.f - alpha);
            const bool blend = pass && !(Tn < tmin);
            done = done || (pass && Tn < tmin);
            const float w = blend ? alpha * T : 0.f;
            if (SEM == 3 || __ballot(blend) != 0) {
                const float4 col = s_col[j];
                cr = fmaf(col.x, w, cr);
                cg = fmaf(col.y, w, cg);
                cb = fmaf(col.z, w, cb);
                dd = fmaf(col.w, w, dd);
                ss += w;
                if constexpr (SEM == 3) {
                    const float* sv = s_sv + j * k;
                    const uint32_t* si = s_si + j * kw;
                    uint32_t wd[KWM];
#pragma unroll
                    for (int q = 0; q < KWM; q++) wd[q] = q < kw ? __builtin_amdgcn_readfirstlane(si[q]) : 0u;
                    reg_accumulate<NB, KT, KM, KWM>(racc, sv, wd, k, w);
                } else if constexpr (OFFS) {
                    // k values and k row offsets, then (distinct classes) all
                    // reads before all updates; repeated classes in order
                    const float* sv = s_sv + j * KT;
                    const uint32_t* so = s_si + j * KT;
                    float vals[KT];
                    uint32_t off[KT];
                    if constexpr ((KT & 3) == 0) {
#pragma unroll
                        for (int m = 0; m < KT; m += 4) {
                            const float4 v4 = *(const float4*)(sv + m);
                            const uint4 o4 = *(const uint4*)(so + m);
                            vals[m] = v4.x; vals[m + 1] = v4.y; vals[m + 2] = v4.z; vals[m + 3] = v4.w;
                            off[m] = o4.x; off[m + 1] = o4.y; off[m + 2] = o4.z; off[m + 3] = o4.w;
                        }
                    } else {
#pragma unroll
                        for (int m = 0; m < KT; m++) {
                            vals[m] = sv[m];
                            off[m] = so[m];
                        }
                    }
                    char* col_base = (char*)(acc + tid);
                    if ((__float_as_uint(q2.w) >> 31) == 0u) {
                        float cur[KT];
#pragma unroll
                        for (int m = 0; m < KT; m++) cur[m] = *(float*)(col_base + off[m]);
#pragma unroll
                        for (int m = 0; m < KT; m++) *(float*)(col_base + off[m]) = fmaf(vals[m], w, cur[m]);
                    } else {
#pragma unroll
                        for (int m = 0; m < KT; m++) {
                            float* q = (float*)(col_base + off[m]);
                            *q = fmaf(vals[m], w, *q);
                        }
                    }
                } else if constexpr (SEM == 4) {
                    // the label's sum: entries of other classes add 0, in
                    // list order (repeated classes add in turn)
                    const float* sv = s_sv + j * k;
                    const uint32_t* si = s_si + j * kw;
                    if (RANKED && ranked && (__float_as_uint(q2.w) >> 31) == 0u) {
                        // distinct classes: the one update the list would make
                        // (the others add exact zeros), with the label's value
                        // found through the class mask
                        const uint2 mw = s_lm[j * 5 + lword];
                        const uint32_t pos = mw.y + __builtin_popcount(mw.x & lbelow);
                        const float vl = s_sv[j * 16 + (pos & 15u)];
                        ql = fmaf((mw.x >> lbit) & 1u ? vl : 0.f, w, ql);
                    } else if constexpr (KT > 0 && (KT & 15) == 0) {
                        // whole rows first (16-byte loads), then selects
#pragma unroll
                        for (int m0 = 0; m0 < KT; m0 += 16) {
                            const uint4 wd = *(const uint4*)(si + m0 / 4);
                            float vv[16];
#pragma unroll
                            for (int q = 0; q < 16; q += 4) {
                                const float4 v4 = *(const float4*)(sv + m0 + q);
                                vv[q] = v4.x; vv[q + 1] = v4.y; vv[q + 2] = v4.z; vv[q + 3] = v4.w;
                            }
                            const uint32_t ww[4] = {wd.x, wd.y, wd.z, wd.w};
#pragma unroll
                            for (int q = 0; q < 16; q++)
                                ql = fmaf((int)((ww[q >> 2] >> (8 * (q & 3))) & 0xffu) == lab ? vv[q] : 0.f, w, ql);
                        }
                    } else {
#pragma unroll
                        for (int mw = 0; mw < (KT > 0 ? (KT + 3) / 4 : kMaxK / 4); mw++) {
                            if (KT == 0 && mw >= kw) break;
                            const uint32_t word = si[mw];
#pragma unroll
                            for (int b = 0; b < 4; b++) {
                                const int m = mw * 4 + b;
                                if (m < k) {
                                    const float v = sv[m];
                                    ql = fmaf((int)((word >> (8 * b)) & 0xffu) == lab ? v : 0.f, w, ql);
                                }
                            }
                        }
                    }
                } else if constexpr (SEM != 0) {
                    const float* sv = s_sv + j * k;
                    const uint32_t* si = s_si + j * kw;
#pragma unroll
                    for (int mw = 0; mw < (KT > 0 ? (KT + 3) / 4 : kMaxK / 4); mw++) {
                        if (KT == 0 && mw >= kw) break;
                        const uint32_t word = si[mw];
#pragma unroll
                        for (int b = 0; b < 4; b++) {
                            const int m = mw * 4 + b;
                            if (m < k) {
                                const uint32_t cl = (word >> (8 * b)) & 0xffu;
                                if (SEM == 1) {
                                    const uint32_t rel = cl - (uint32_t)lo;
                                    if (NPASS == 1 || rel < (uint32_t)cnt)
                                        acc[rel * kAccStride + tid] = fmaf(sv[m], w, acc[rel * kAccStride + tid]);
                                } else if (gacc && blend) {
                                    gacc[cl] = fmaf(sv[m], w, gacc[cl]);
                                }
                            }
                        }
                    }
                }
            }
            T = blend ? Tn : T;
            ncon += blend ? 1 : 0;
            last = blend ? b0 + j + 1 : last;
            if (__ballot(!done) == 0) break;
        }
    }
    res.T = T;
    res.ncon = ncon;
    res.inside = inside;
    res.v = v;
    res.px = px;
    res.py = py;
    res.tx = tx;
    res.ty = ty;
    res.last = last;
    res.c[0] = cr; res.c[1] = cg; res.c[2] = cb;
    res.d = dd;
    res.s = ss;
    res.lab = lab;
    res.ql = ql;
}

__device__ __forceinline__ float sgnf(float x) { return x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f); }

// The mapping loss of one pixel and its gradient with respect to the maps
// (Sec. 3.1), fused after the tile's compositing.  Geometry: the
// silhouette-masked depth and colour L1 and |S - 1|.  Semantics (LDS class
// sums, SEM == 1): each thread turns its own class column into dL/dP, from
// a dense target g (entropy mask, Hellinger + cosine) or a label
// (cross-entropy).  The tile's summed loss goes to tile_loss[gt].
template <int SEM, int NPASS = 1>
__device__ __forceinline__ void loss_epilogue(const TileArgs& a, const LossK& lk, const TileResult& r,
                                              const ViewDev& vw, int gt, float* smem, int lab = -1,
                                              float q_label = 0.f) {
    __shared__ double s_part[kBlock / 64];
    const int tid = threadIdx.x;
    const LossPtrs& L = lk.views[r.v];
    const float inv_p = 1.f / ((float)vw.width * (float)vw.height);
    const int64_t pix = (int64_t)r.py * vw.width + r.px;
    double lpx = 0.0;
    if (r.inside) {
        const float m = r.s > lk.sil_thresh ? 1.f : 0.f;
        float lg = 0.f;
        if (L.depth) {
            const float rd = r.d - L.depth[pix];
            lg += m * lk.w_depth * fabsf(rd);
            if (L.g_depth) L.g_depth[pix] = m * lk.w_depth * sgnf(rd) * inv_p;
        } else if (L.g_depth) {
            L.g_depth[pix] = 0.f;
        }
#pragma unroll
        for (int ch = 0; ch < 3; ch++) {
            if (L.rgb) {
                const float rc = r.c[ch] - L.rgb[3 * pix + ch];
                lg += m * lk.w_rgb * fabsf(rc);
                if (L.g_rgb) L.g_rgb[3 * pix + ch] = m * lk.w_rgb * sgnf(rc) * inv_p;
            } else if (L.g_rgb) {
                L.g_rgb[3 * pix + ch] = 0.f;
            }
        }
        const float rs = r.s - 1.f;
        lg += lk.w_sil * fabsf(rs);
        if (L.g_sil) L.g_sil[pix] = lk.w_sil * sgnf(rs) * inv_p;
        lpx = (double)lg;
    }
    if constexpr ((SEM == 1 && NPASS > 1) || SEM == 4) {
        // class passes or label-only sums: only the cross-entropy term, from
        // the label's class sum; its gradient in the one-class form
        if (r.inside && L.label) {
            float gl = 0.f;
            if (lab >= 0 && lab < a.C) {
                lpx -= (double)(lk.w_sem * logf(fmaxf(q_label, lk.ce_floor)));
                gl = q_label > lk.ce_floor ? -lk.w_sem * inv_p / q_label : 0.f;
            } else {
                atomicOr(&a.counters[kStatus], Plan::kBadIndex);
            }
            if (L.g_sem_at_label) L.g_sem_at_label[pix] = gl;
        } else if (r.inside && L.g_sem_at_label) {
            L.g_sem_at_label[pix] = 0.f;
        }
    }
    if constexpr (SEM == 1 && NPASS == 1) {
        const int C = a.C;
        __syncthreads();  // class sums final
        if (a.maps[r.v].sem) {
            write_rows_from_lds(smem, a.maps[r.v].sem, vw, C, r.tx, r.ty);
            __syncthreads();  // every column read before it is overwritten
        }
        float* col = smem + tid;  // this pixel's classes, stride kAccStride
        if (r.inside && L.sem) {
            if (L.g_sem_at_label) L.g_sem_at_label[pix] = 0.f;  // dense target: no single-class form
            const float* g = L.sem + pix * C;
            const float e = lk.sqrt_eps;
            float H = 0.f, gg = 0.f, qq = 0.f, gq = 0.f, dd = 0.f;
            for (int c = 0; c < C; c++) {
                const float gc = g[c], qc = col[c * kAccStride];
                if (gc > 0.f) H -= gc * logf(gc);
                gg += gc * gc;
                qq += qc * qc;
                gq += gc * qc;
                const float d = sqrtf(gc + e) - sqrtf(qc + e);
                dd += d * d;
            }
            if (H < lk.tau && gg > 0.f && qq > 0.f) {
                const float ng = sqrtf(gg), nq = sqrtf(qq), root = sqrtf(dd);
                const float cosv = gq / (ng * nq);
                const float kSqrt2 = 1.41421356237309504880f;
                lpx += (double)(lk.w_sem * (lk.lambda_hd * root / kSqrt2 + lk.lambda_cos * (1.f - cosv)));
                const float s = lk.w_sem * inv_p;
                const float a_hd = root > 0.f ? -lk.lambda_hd / (2.f * kSqrt2 * root) : 0.f;
                const float a_g = -lk.lambda_cos / (ng * nq), a_q = lk.lambda_cos * cosv / (nq * nq);
                for (int c = 0; c < C; c++) {
                    const float gc = g[c], qc = col[c * kAccStride];
                    const float sq = sqrtf(qc + e);
                    const float d = sqrtf(gc + e) - sq;
                    col[c * kAccStride] = s * (a_hd * d / sq + a_g * gc + a_q * qc);
                }
            } else {
                for (int c = 0; c < C; c++) col[c * kAccStride] = 0.f;
            }
        } else if (r.inside && L.label) {
            const int lab = L.label[pix];
            float gl = 0.f;
            if (lab >= 0 && lab < C) {
                const float q = col[lab * kAccStride];
                lpx -= (double)(lk.w_sem * logf(fmaxf(q, lk.ce_floor)));
                gl = q > lk.ce_floor ? -lk.w_sem * inv_p / q : 0.f;
            } else {
                atomicOr(&a.counters[kStatus], Plan::kBadIndex);
            }
            if (L.g_sem_at_label) L.g_sem_at_label[pix] = gl;
            if (L.g_sem) {
                for (int c = 0; c < C; c++) col[c * kAccStride] = 0.f;
                if (lab >= 0 && lab < C) col[lab * kAccStride] = gl;
            }
        } else {
            if (r.inside && L.g_sem_at_label) L.g_sem_at_label[pix] = 0.f;
            if (L.g_sem)
                for (int c = 0; c < C; c++) col[c * kAccStride] = 0.f;
        }
        __syncthreads();
        if (L.g_sem) write_rows_from_lds(smem, L.g_sem, vw, C, r.tx, r.ty);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) lpx += __shfl_xor(lpx, o, 64);
    if ((tid & 63) == 0) s_part[tid >> 6] = lpx;
    __syncthreads();
    if (tid == 0) lk.tile_loss[gt] = ((s_part[0] + s_part[1]) + s_part[2]) + s_part[3];
}

// Classes 32 B .. 32 B + 31 of a wave's 8x8 pixel block to the [H][W][C]
// map through the wave's 64 x 33 LDS buffer: lane l stores its pixel's 32
// sums, then each store instruction covers four pixels' runs of 32 classes
// (16 lanes x 2 floats each) instead of 64 scattered floats.  Same-wave LDS
// accesses complete in order, so no barrier is needed.
template <int B>
__device__ __forceinline__ void write_sem_block(const v32f& acc, float* buf, float* out, const ViewDev& vw, int C,
                                                bool pairs, int wx0, int wy0, int lane) {
#pragma unroll
    for (int c = 0; c < kRegBlock; c++) buf[lane * 33 + c] = acc[c];
    for (int rr = 0; rr < 16; rr++) {
        const int p = rr * 4 + (lane >> 4);
        const int c2 = (lane & 15) * 2;
        const int cls = B * kRegBlock + c2;
        const int x = wx0 + (p & 7), y = wy0 + (p >> 3);
        if (x < vw.width && y < vw.height && cls < C) {
            float* dst = out + ((int64_t)y * vw.width + x) * C + cls;
            const float v0 = buf[p * 33 + c2], v1 = buf[p * 33 + c2 + 1];
            if (cls + 1 < C) {
                if (pairs) {
                    *(float2*)dst = make_float2(v0, v1);
                } else {
                    dst[0] = v0;
                    dst[1] = v1;
                }
            } else {
                dst[0] = v0;
            }
        }
    }
}

template <int KT, int SEM, int NB, bool LOSS, int NPASS = 1>
__device__ __forceinline__ void render_fwd_body(const TileArgs& a, const LossK& lk) {
    extern __shared__ __align__(16) float smem[];
    const int gt = tile_of_block(blockIdx.x, gridDim.x, a.linear_tiles);
    if (gt >= a.num_tiles) return;
    if (a.counters[kStatus] & SGR_ECAPACITY) return;
    TileResult r;
    v32f acc0, acc1, acc2, acc3;
    RegAcc<NB> racc{acc0, acc1, acc2, acc3};
    int lab = -1;        // fused cross-entropy under class passes: the pixel's label ...
    float q_label = 0.f; // ... and its class sum, taken in the pass that holds it
    if constexpr (NPASS == 1) {
        composite_tile<KT, SEM, NB>(a, gt, smem, r, racc);
    } else {
        static_assert(SEM == 1, "class passes use the LDS class sums");
        const int C = a.C, cpp = (C + NPASS - 1) / NPASS;
        for (int pass = 0; pass < NPASS; pass++) {
            const int lo = pass * cpp, cnt = min(cpp, C - lo);
            composite_tile<KT, 1, NB, NPASS>(a, gt, smem, r, racc, lo, cnt, cpp);
            __syncthreads();
            float* out = a.maps[r.v].sem;
            if (out) write_rows_range(smem, out, a.views[r.v], C, lo, cnt, r.tx, r.ty);
            if constexpr (LOSS) {
                if (pass == 0 && r.inside && lk.views[r.v].label)
                    lab = lk.views[r.v].label[(int64_t)r.py * a.views[r.v].width + r.px];
                if ((uint32_t)(lab - lo) < (uint32_t)cnt) q_label = smem[(lab - lo) * kAccStride + threadIdx.x];
            }
            __syncthreads();  // before the next pass clears the rows
        }
    }
    const ViewDev& vw = a.views[r.v];
    if (r.inside) {
        const int64_t pix = (int64_t)r.py * vw.width + r.px;
        const MapPtrs& o = a.maps[r.v];
        if (o.rgb) { o.rgb[3 * pix] = r.c[0]; o.rgb[3 * pix + 1] = r.c[1]; o.rgb[3 * pix + 2] = r.c[2]; }
        if (o.depth) o.depth[pix] = r.d;
        if (o.sil) o.sil[pix] = r.s;
        if (o.t_final) o.t_final[pix] = r.T;
        if (o.n_contrib) o.n_contrib[pix] = r.ncon;
        a.pix_T[vw.pix_off + pix] = r.T;
        a.pix_last[vw.pix_off + pix] = r.last;
    }
    if constexpr (LOSS) {
        if constexpr (SEM == 4) {
            lab = r.lab;
            q_label = r.ql;
        }
        loss_epilogue<SEM, NPASS>(a, lk, r, vw, gt, smem, lab, q_label);
        return;
    }
    if (SEM == 1 && NPASS == 1) {
        float* out = a.maps[r.v].sem;
        if (!out) return;
        __syncthreads();
        write_rows_from_lds(smem, out, vw, a.C, r.tx, r.ty);
    }
    if (SEM == 3) {
        // Each wave writes its 8x8 block, 32 classes at a time, through a
        // 64 x 33 LDS transpose: one store then covers four pixels' runs of
        // 32 classes instead of 64 scattered floats.
        float* out = a.maps[r.v].sem;
        if (!out) return;
        __syncthreads();  // the staging area becomes the transpose buffers
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        float* buf = smem + wv * (64 * 33);
        const int C = a.C;
        const bool pairs = (C & 1) == 0 && ((uintptr_t)out & 7u) == 0;  // 8-byte aligned class pairs
        const int wx0 = r.tx * kTile + (wv & 1) * 8, wy0 = r.ty * kTile + (wv >> 1) * 8;
        write_sem_block<0>(racc.a0, buf, out, vw, C, pairs, wx0, wy0, lane);
        if constexpr (NB > 1) write_sem_block<1>(racc.a1, buf, out, vw, C, pairs, wx0, wy0, lane);
        if constexpr (NB > 2) write_sem_block<2>(racc.a2, buf, out, vw, C, pairs, wx0, wy0, lane);
        if constexpr (NB > 3) write_sem_block<3>(racc.a3, buf, out, vw, C, pairs, wx0, wy0, lane);
    }
}

template <int KT, int SEM, int NB, bool LOSS, int NPASS = 1>
__global__ __launch_bounds__(kBlock) void render_fwd_kernel(TileArgs a, LossK lk) {
    render_fwd_body<KT, SEM, NB, LOSS, NPASS>(a, lk);
}

// Label-only class sums keep no class sums in LDS, so registers bound the
// workgroups per CU: the kernel is held to 80 VGPRs, six waves per SIMD
// (the few values this costs are kept in scratch, reloaded once per staged
// batch, outside the compositing loop).
template <int KT>
__global__ __launch_bounds__(kBlock, 6) void render_fwd_label_kernel(TileArgs a, LossK lk) {
    render_fwd_body<KT, 4, 1, true, 1>(a, lk);
}

// ------------------------------------------------------------------ scoring

// Persistent: a grid of about one workgroup per CU walks the (view, tile)
// items with a static stride.  Items are numbered so that the workgroups of
// one XCD (workgroup i runs on XCD i % 8) cover one contiguous run of tiles.
// Each item's silhouette count and semantic accumulators are composited, and
// the tile's empty-pixel count and summed entropy go to a fixed slot.  The
// last workgroup to finish reduces the slots of each view in tile order
// (FP64), so the scores are deterministic.  The loop bounds depend only on
// blockIdx and the grid, so every lane of every wave takes the same trip
// count through the barriers.
// Z += x and sxl += x log2 x over classes 32 B .. 32 B + 31 (those < C), with
// x the class sum clipped to [0.001, 1], in class order.
template <int B>
__device__ __forceinline__ void entropy_terms(const v32f& acc, int C, float lg_lo, float& Z, float& sxl) {
#pragma unroll
    for (int c = 0; c < kRegBlock; c++) {
        if (B * kRegBlock + c < C) {
            const float x = fminf(fmaxf(acc[c], 0.001f), 1.f);
            const float lx = (x == 0.001f) ? lg_lo : __log2f(x);
            Z += x;
            sxl += x * lx;
        }
    }
}

template <int KT, int SEM, int NB, int NPASS = 1>
__global__ __launch_bounds__(kBlock) void score_persistent_kernel(TileArgs a, ScoreOut so) {
    extern __shared__ __align__(16) float smem[];
    __shared__ double s_h[4];
    __shared__ uint32_t s_e[4];
    __shared__ int s_last;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const bool ok = !(a.counters[kStatus] & SGR_ECAPACITY);
    const int C = a.C;
    const float ln2 = 0.69314718055994530942f;
    const float lg_lo = -9.9657842846620870436f;  // log2(0.001)
    const int T = (int)a.num_tiles;
    const int per = (T + 7) >> 3;       // tiles per XCD run
    const int G = (int)gridDim.x;       // a multiple of 8
    const int items = ok ? per * 8 : 0;
    for (int item = (int)blockIdx.x; item < items; item += G) {
        const int gt = a.linear_tiles ? item : (item & 7) * per + (item >> 3);
        if (gt >= T) continue;
        TileResult r;
        v32f acc0, acc1, acc2, acc3;
        RegAcc<NB> racc{acc0, acc1, acc2, acc3};
        double h = 0.0;
        if constexpr (NPASS > 1) {
            // class passes: Z and sum x log2 x grow pass by pass, in class order
            const int cpp = (C + NPASS - 1) / NPASS;
            float Z = 0.f, sxl = 0.f;
            for (int pass = 0; pass < NPASS; pass++) {
                const int lo = pass * cpp, cnt = min(cpp, C - lo);
                composite_tile<KT, 1, NB, NPASS>(a, gt, smem, r, racc, lo, cnt, cpp);
                if (r.inside)
                    for (int c = 0; c < cnt; c++) {
                        const float x = fminf(fmaxf(smem[c * kAccStride + tid], 0.001f), 1.f);
                        const float lx = (x == 0.001f) ? lg_lo : __log2f(x);
                        Z += x;
                        sxl += x * lx;
                    }
                __syncthreads();
            }
            if (r.inside) h = (double)(ln2 * (__log2f(Z) - sxl / Z));
        } else {
        composite_tile<KT, SEM, NB>(a, gt, smem, r, racc);
        __syncthreads();
        if (r.inside) {
            float Z = 0.f, sxl = 0.f;
            if constexpr (SEM == 3) {
                entropy_terms<0>(racc.a0, C, lg_lo, Z, sxl);
                if constexpr (NB > 1) entropy_terms<1>(racc.a1, C, lg_lo, Z, sxl);
                if constexpr (NB > 2) entropy_terms<2>(racc.a2, C, lg_lo, Z, sxl);
                if constexpr (NB > 3) entropy_terms<3>(racc.a3, C, lg_lo, Z, sxl);
            } else {
                for (int c = 0; c < C; c++) {
                    const float x = fminf(fmaxf(smem[c * kAccStride + tid], 0.001f), 1.f);
                    const float lx = (x == 0.001f) ? lg_lo : __log2f(x);
                    Z += x;
                    sxl += x * lx;
                }
            }
            h = (double)(ln2 * (__log2f(Z) - sxl / Z));
        }
        }
        const uint64_t em = __ballot(r.inside && r.ncon == 0);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) h += __shfl_xor(h, o, 64);
        if (lane == 0) {
            s_h[w] = h;
            s_e[w] = (uint32_t)__popcll(em);
        }
        __syncthreads();
        if (tid == 0) {
            so.tile_h[gt] = ((s_h[0] + s_h[1]) + s_h[2]) + s_h[3];
            so.tile_e[gt] = s_e[0] + s_e[1] + s_e[2] + s_e[3];
        }
        __syncthreads();
    }
    __threadfence();
    __syncthreads();
    if (tid == 0) s_last = (atomicAdd(&a.counters[kDone], 1u) == gridDim.x - 1);
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    for (int v = tid; v < a.V; v += kBlock) {
        const ViewDev& vw = a.views[v];
        const int t0 = vw.tile_off, nt = vw.tiles_x * vw.tiles_y;
        double hs = 0.0;
        uint32_t es = 0;
        if (ok) {
            const volatile double* th = so.tile_h;
            const volatile uint32_t* te = so.tile_e;
            for (int t = 0; t < nt; t++) {
                hs += th[t0 + t];
                es += te[t0 + t];
            }
        }
        so.entropy_sum[v] = ok ? hs : 0.0;
        so.n_empty[v] = ok ? es : 0u;
    }
}

// ------------------------------------------------------------------ plain scoring from dense maps

__global__ __launch_bounds__(kBlock) void score_maps_kernel(const float* __restrict__ sem,
                                                            const int32_t* __restrict__ ncon, int64_t P, int C,
                                                            double* __restrict__ blk_h, uint32_t* __restrict__ blk_e,
                                                            uint32_t* done, uint32_t* n_empty, double* entropy_sum) {
    __shared__ double s_h[4];
    __shared__ uint32_t s_e[4];
    __shared__ int s_last;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t p = blockIdx.x * (int64_t)kBlock + tid;
    const float ln2 = 0.69314718055994530942f;
    const float lg_lo = -9.9657842846620870436f;
    double h = 0.0;
    bool empty = false;
    if (p < P) {
        const float* row = sem + p * C;
        float Z = 0.f, sxl = 0.f;
        for (int c = 0; c < C; c++) {
            const float x = fminf(fmaxf(row[c], 0.001f), 1.f);
            const float lx = (x == 0.001f) ? lg_lo : __log2f(x);
            Z += x;
            sxl += x * lx;
        }
        h = (double)(ln2 * (__log2f(Z) - sxl / Z));
        empty = ncon[p] == 0;
    }
    const uint64_t em = __ballot(empty);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) h += __shfl_xor(h, o, 64);
    if (lane == 0) { s_h[w] = h; s_e[w] = (uint32_t)__popcll(em); }
    __syncthreads();
    if (tid == 0) {
        blk_h[blockIdx.x] = ((s_h[0] + s_h[1]) + s_h[2]) + s_h[3];
        blk_e[blockIdx.x] = s_e[0] + s_e[1] + s_e[2] + s_e[3];
        __threadfence();
        s_last = (atomicAdd(done, 1u) == gridDim.x - 1);
    }
    __syncthreads();
    if (!s_last || tid != 0) return;
    __threadfence();
    double hs = 0.0;
    uint32_t es = 0;
    const volatile double* bh = blk_h;
    const volatile uint32_t* be = blk_e;
    for (unsigned b = 0; b < gridDim.x; b++) { hs += bh[b]; es += be[b]; }
    entropy_sum[0] = hs;
    n_empty[0] = es;
    *done = 0;
}

// ------------------------------------------------------------------ launchers

template <typename K>
static void set_lds(K kernel, size_t bytes) {
    if (bytes > 65536)
        (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// LDS of a forward launch: the staging area, plus the class-major
// accumulators (mode 1) or, for mode 3, room for the four waves' 64 x 33
// transpose buffers that reuse the staging area at the end.
size_t fwd_lds_bytes(int C, int k, int kpad, int sem_mode) {
    // per staged entry: records, k values, and the class indices as bytes
    // or (LDS class sums) as one 4-byte row offset each
    size_t b = (size_t)kFwdBatch * (4 * sizeof(float4) + k * sizeof(float) + (sem_mode == 1 ? std::max(kpad, 4 * k) : kpad));
    if (sem_mode == 1) b += (size_t)acc_floats(C) * sizeof(float);
    if (sem_mode == 3) b = std::max(b, (size_t)4 * 64 * 33 * sizeof(float));
    if (sem_mode == 4 && k == 16) b += (size_t)kFwdBatch * 5 * sizeof(uint2);  // class masks
    return b;
}

// Classes per pass when the class sums are split into `passes` ranges.
static int class_rows(int C, int passes) { return (C + passes - 1) / passes; }

// Class passes of an LDS launch: the configured count, else the fewest
// whose rows fit the LDS; 0 if none fits.
static int lds_passes(const Plan& P) {
    const size_t cap = device_max_lds();
    if (P.cfg.sem_passes > 0)
        return fwd_lds_bytes(class_rows(P.C, P.cfg.sem_passes), P.k, P.kpad, 1) <= cap ? P.cfg.sem_passes : 0;
    for (int p = 1; p <= kMaxPasses; p++)
        if (fwd_lds_bytes(class_rows(P.C, p), P.k, P.kpad, 1) <= cap) return p;
    return 0;
}

// 0: no semantics; 1: LDS accumulators; 2: accumulate into the output map;
// 3: register accumulators.  Automatic placement prefers LDS, which measures
// faster on gfx950 at C = 102 (a register update costs four VALU operations
// and a scalar index decode against two VALU and two LDS operations).
static int sem_mode_for(const Plan& P, bool want_sem) {
    if (!want_sem) return 0;
    const int acc = P.cfg.sem_accumulators;
    if (acc == SGR_ACC_REGISTERS) return 3;
    if (lds_passes(P) > 0) return 1;
    return (acc == SGR_ACC_AUTO && P.C <= kMaxRegC) ? 3 : 2;
}

TileArgs make_tile_args(const Plan& P, char* ws) {
    TileArgs a;
    memset(&a, 0, sizeof(a));
    a.views = (const ViewDev*)(ws + P.views);
    a.V = P.V;
    a.num_tiles = P.num_tiles;
    a.k = P.k;
    a.kpad = P.kpad;
    a.C = P.C;
    a.ranges = (const uint2*)(ws + P.ranges);
    a.svals = (const uint32_t*)(ws + P.sorted_vals);
    a.owner = (const uint32_t*)(ws + P.owner);
    a.srec = (const Proj*)(ws + P.srec);
    a.scol = (const float4*)(ws + P.scol);
    a.ssv = (const float*)(ws + P.ssv);
    a.ssi = (const uint8_t*)(ws + P.ssi);
    a.srk = P.ranked ? (const uint32_t*)(ws + P.srk) : nullptr;
    a.counters = (uint32_t*)(ws + P.counters);
    a.pix_T = (float*)(ws + P.pix_T);
    a.pix_last = (uint32_t*)(ws + P.pix_last);
    a.alpha_min = P.cfg.alpha_min;
    a.alpha_max = P.cfg.alpha_max;
    a.t_min = P.cfg.t_min;
    a.linear_tiles = P.cfg.tile_order == SGR_TILES_LINEAR ? 1 : 0;
    return a;
}

template <int KT, int SEM, int NB, bool LOSS = false, int NPASS = 1>
static void fwd_launch(const TileArgs& a, unsigned grid, size_t lds, hipStream_t st, const LossK& lk = LossK{}) {
    set_lds(render_fwd_kernel<KT, SEM, NB, LOSS, NPASS>, lds);
    render_fwd_kernel<KT, SEM, NB, LOSS, NPASS><<<grid, kBlock, lds, st>>>(a, lk);
}

template <int KT, bool LOSS>
static void fwd_launch_lds(int passes, const TileArgs& a, unsigned grid, size_t lds, hipStream_t st,
                           const LossK& lk = LossK{}) {
    if (passes == 1) fwd_launch<KT, 1, 1, LOSS>(a, grid, lds, st, lk);
    else if (passes == 2) fwd_launch<KT, 1, 1, LOSS, 2>(a, grid, lds, st, lk);
    else if (passes == 3) fwd_launch<KT, 1, 1, LOSS, 3>(a, grid, lds, st, lk);
    else fwd_launch<KT, 1, 1, LOSS, 4>(a, grid, lds, st, lk);
}

template <int KT>
static void fwd_dispatch_sem(int sem, int nb, int passes, const TileArgs& a, unsigned grid, size_t lds,
                             hipStream_t st) {
    if (sem == 0) fwd_launch<KT, 0, 1>(a, grid, lds, st);
    else if (sem == 1) fwd_launch_lds<KT, false>(passes, a, grid, lds, st);
    else if (sem == 2) fwd_launch<KT, 2, 1>(a, grid, lds, st);
    else if (nb == 1) fwd_launch<KT, 3, 1>(a, grid, lds, st);
    else if (nb == 2) fwd_launch<KT, 3, 2>(a, grid, lds, st);
    else if (nb == 3) fwd_launch<KT, 3, 3>(a, grid, lds, st);
    else fwd_launch<KT, 3, 4>(a, grid, lds, st);
}

sgr_status launch_forward(const Plan& P, const sgr_maps* out, char* ws, hipStream_t st) {
    TileArgs a = make_tile_args(P, ws);
    bool want_sem = false;
    std::vector<MapPtrs> mp(P.V);
    for (int v = 0; v < P.V; v++) {
        mp[v] = MapPtrs{out[v].rgb, out[v].depth, out[v].sil, out[v].sem, out[v].t_final, out[v].n_contrib};
        want_sem |= out[v].sem != nullptr;
    }
    set_view_table(a.maps, mp, ws + P.map_table, st);
    const int sem = sem_mode_for(P, want_sem);
    const int nb = (P.C + kRegBlock - 1) / kRegBlock;
    const int passes = sem == 1 ? lds_passes(P) : 1;
    const size_t lds = fwd_lds_bytes(class_rows(P.C, passes), P.k, P.kpad, sem);
    const unsigned grid = (unsigned)(div_up(P.num_tiles, 8) * 8);
    if (P.k == 16) fwd_dispatch_sem<16>(sem, nb, passes, a, grid, lds, st);
    else if (P.k == 3) fwd_dispatch_sem<3>(sem, nb, passes, a, grid, lds, st);
    else fwd_dispatch_sem<0>(sem, nb, passes, a, grid, lds, st);
    return hipGetLastError() == hipSuccess ? SGR_OK : SGR_EHIP;
}

// A persistent grid of as many workgroups as fit on the device at once.
template <int KT, int SEM, int NB, int NPASS = 1>
static sgr_status score_launch(const Plan& P, const TileArgs& a, const ScoreOut& so, size_t lds, hipStream_t st) {
    set_lds(score_persistent_kernel<KT, SEM, NB, NPASS>, lds);
    static int per_cu = 0;  // per instantiation; the dynamic LDS size is fixed by C and k
    static size_t per_cu_lds = 0;
    if (per_cu == 0 || per_cu_lds != lds) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, score_persistent_kernel<KT, SEM, NB, NPASS>, kBlock,
                                                         lds) != hipSuccess)
            return SGR_EHIP;
        per_cu = std::max(1, n);
        per_cu_lds = lds;
    }
    const int64_t resident = (int64_t)device_cu_count() * per_cu;
    const int64_t want = std::min<int64_t>(P.num_tiles, P.cfg.score_workgroups > 0 ? P.cfg.score_workgroups : resident);
    const unsigned grid = (unsigned)(div_up(want, 8) * 8);
    score_persistent_kernel<KT, SEM, NB, NPASS><<<grid, kBlock, lds, st>>>(a, so);
    return hipGetLastError() == hipSuccess ? SGR_OK : SGR_EHIP;
}

// Per-view loss: the view's tile slots summed in a fixed order, over P.
__global__ __launch_bounds__(256) void loss_reduce_kernel(const ViewDev* views, const double* tile_loss,
                                                          const uint32_t* counters, double* loss) {
    __shared__ double s_part[4];
    const ViewDev& vw = views[blockIdx.x];
    const bool ok = !(counters[kStatus] & SGR_ECAPACITY);
    const int nt = vw.tiles_x * vw.tiles_y;
    double s = 0.0;
    if (ok)
        for (int t = threadIdx.x; t < nt; t += 256) s += tile_loss[vw.tile_off + t];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0)
        loss[blockIdx.x] = ok ? (((s_part[0] + s_part[1]) + s_part[2]) + s_part[3]) / ((double)vw.width * vw.height)
                              : 0.0;
}

sgr_status launch_forward_loss(const Plan& P, const sgr_maps* out, const sgr_loss_view* lv, const sgr_loss_config* lc,
                               double* loss, char* ws, hipStream_t st) {
    TileArgs a = make_tile_args(P, ws);
    bool want_sem = false, dense_sem = false, sem_map = false;
    std::vector<MapPtrs> mp(P.V);
    std::vector<LossPtrs> lp(P.V);
    for (int v = 0; v < P.V; v++) {
        if (out) mp[v] = MapPtrs{out[v].rgb, out[v].depth, out[v].sil, out[v].sem, out[v].t_final, out[v].n_contrib};
        else mp[v] = MapPtrs{};
        lp[v] = LossPtrs{lv[v].rgb, lv[v].depth, lv[v].label, lv[v].sem,
                         lv[v].g_rgb, lv[v].g_depth, lv[v].g_sil, lv[v].g_sem, lv[v].g_sem_at_label};
        want_sem |= mp[v].sem != nullptr || lv[v].label != nullptr || lv[v].sem != nullptr || lv[v].g_sem != nullptr ||
                    lv[v].g_sem_at_label != nullptr;
        dense_sem |= lv[v].sem != nullptr || lv[v].g_sem != nullptr;
        sem_map |= mp[v].sem != nullptr;
    }
    LossK lk;
    if (P.V == 1) {
        set_view_table(a.maps, mp, nullptr, st);
        set_view_table(lk.views, lp, nullptr, st);
    } else {
        upload_pair(ws + P.map_table, mp.data(), sizeof(MapPtrs) * P.V, ws + P.loss_table, lp.data(),
                    sizeof(LossPtrs) * P.V, st);
        a.maps.table = (const MapPtrs*)(ws + P.map_table);
        a.maps.one = MapPtrs{};
        lk.views.table = (const LossPtrs*)(ws + P.loss_table);
        lk.views.one = LossPtrs{};
    }
    lk.w_depth = lc->w_depth; lk.w_rgb = lc->w_rgb; lk.w_sil = lc->w_sil; lk.w_sem = lc->w_sem;
    lk.sil_thresh = lc->sil_thresh; lk.ce_floor = lc->ce_floor;
    lk.lambda_hd = lc->lambda_hd; lk.lambda_cos = lc->lambda_cos;
    lk.tau = lc->entropy_tau > 0.f ? lc->entropy_tau : logf((float)P.k);
    lk.sqrt_eps = lc->sqrt_eps;
    lk.tile_loss = (double*)(ws + P.tile_part);
    a.loss_views = lk.views;
    // Cross-entropy targets only, no dense semantic map or gradient asked
    // for: each pixel needs only its label's class sum (mode 4).
    const bool label_only = want_sem && !dense_sem && !sem_map;
    const int sem = !want_sem ? 0 : label_only ? 4 : 1;
    // the dense target terms and the dense gradient need every class of a
    // pixel at once: one pass
    const int passes = sem != 1 ? 1 : dense_sem ? 1 : lds_passes(P);
    if (passes == 0) return SGR_EUNSUPPORTED;
    const size_t lds = fwd_lds_bytes(class_rows(P.C, passes), P.k, P.kpad, sem);
    if (lds > device_max_lds()) return SGR_EUNSUPPORTED;
    const unsigned grid = (unsigned)(div_up(P.num_tiles, 8) * 8);
    if (P.k == 16) {
        if (sem == 1) fwd_launch_lds<16, true>(passes, a, grid, lds, st, lk);
        else if (sem == 4) render_fwd_label_kernel<16><<<grid, kBlock, lds, st>>>(a, lk);
        else fwd_launch<16, 0, 1, true>(a, grid, lds, st, lk);
    } else if (P.k == 3) {
        if (sem == 1) fwd_launch_lds<3, true>(passes, a, grid, lds, st, lk);
        else if (sem == 4) render_fwd_label_kernel<3><<<grid, kBlock, lds, st>>>(a, lk);
        else fwd_launch<3, 0, 1, true>(a, grid, lds, st, lk);
    } else {
        if (sem == 1) fwd_launch_lds<0, true>(passes, a, grid, lds, st, lk);
        else if (sem == 4) render_fwd_label_kernel<0><<<grid, kBlock, lds, st>>>(a, lk);
        else fwd_launch<0, 0, 1, true>(a, grid, lds, st, lk);
    }
    loss_reduce_kernel<<<P.V, 256, 0, st>>>((const ViewDev*)(ws + P.views), lk.tile_loss,
                                            (const uint32_t*)(ws + P.counters), loss);
    return hipGetLastError() == hipSuccess ? SGR_OK : SGR_EHIP;
}

sgr_status launch_score(const Plan& P, uint32_t* n_empty, double* entropy_sum, char* ws, hipStream_t st) {
    TileArgs a = make_tile_args(P, ws);
    ScoreOut so;
    so.tile_h = (double*)(ws + P.tile_part);
    so.tile_e = (uint32_t*)(ws + P.tile_part + sizeof(double) * P.num_tiles);
    so.n_empty = n_empty;
    so.entropy_sum = entropy_sum;
    const int sem = sem_mode_for(P, true) == 3 ? 3 : 1;
    const int passes = sem == 1 ? lds_passes(P) : 1;
    if (passes == 0) return SGR_EUNSUPPORTED;
    const size_t lds = fwd_lds_bytes(class_rows(P.C, passes), P.k, P.kpad, sem == 3 ? 0 : 1);
    if (lds > device_max_lds()) return SGR_EUNSUPPORTED;
    const int nb = (P.C + kRegBlock - 1) / kRegBlock;
    if (P.k == 16) {
        if (sem == 1 && passes == 2) return score_launch<16, 1, 1, 2>(P, a, so, lds, st);
        if (sem == 1 && passes == 3) return score_launch<16, 1, 1, 3>(P, a, so, lds, st);
        if (sem == 1 && passes == 4) return score_launch<16, 1, 1, 4>(P, a, so, lds, st);
        if (sem == 1) return score_launch<16, 1, 1>(P, a, so, lds, st);
        if (nb == 1) return score_launch<16, 3, 1>(P, a, so, lds, st);
        if (nb == 2) return score_launch<16, 3, 2>(P, a, so, lds, st);
        if (nb == 3) return score_launch<16, 3, 3>(P, a, so, lds, st);
        return score_launch<16, 3, 4>(P, a, so, lds, st);
    }
    if (sem == 1 && passes == 2) return score_launch<0, 1, 1, 2>(P, a, so, lds, st);
    if (sem == 1 && passes == 3) return score_launch<0, 1, 1, 3>(P, a, so, lds, st);
    if (sem == 1 && passes == 4) return score_launch<0, 1, 1, 4>(P, a, so, lds, st);
    if (sem == 1) return score_launch<0, 1, 1>(P, a, so, lds, st);
    if (nb == 1) return score_launch<0, 3, 1>(P, a, so, lds, st);
    if (nb == 2) return score_launch<0, 3, 2>(P, a, so, lds, st);
    if (nb == 3) return score_launch<0, 3, 3>(P, a, so, lds, st);
    return score_launch<0, 3, 4>(P, a, so, lds, st);
}

sgr_status launch_score_maps(const float* sem, const int32_t* n_contrib, int W, int H, int C, uint32_t* n_empty,
                             double* entropy_sum, char* scratch, hipStream_t st) {
    const int64_t P = (int64_t)W * H;
    const unsigned grid = (unsigned)div_up(P, kBlock);
    double* bh = (double*)scratch;
    uint32_t* be = (uint32_t*)(scratch + sizeof(double) * grid);
    uint32_t* done = (uint32_t*)(scratch + (sizeof(double) + sizeof(uint32_t)) * grid);
    zero_u32<<<1, 1, 0, st>>>(done);
    score_maps_kernel<<<grid, kBlock, 0, st>>>(sem, n_contrib, P, C, bh, be, done, n_empty, entropy_sum);
    return hipGetLastError() == hipSuccess ? SGR_OK : SGR_EHIP;
}

}  // namespace sgr
