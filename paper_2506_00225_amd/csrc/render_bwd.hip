// Backward pass: reverse compositing per tile with an atomic-free per-tile
// reduction into one gradient slot per (tile, Gaussian) key, a fixed-order
// sum of each Gaussian's slots, and the chain rule to 3D parameters.
#include "pipeline.h"
#include "render_common.h"

namespace sgr {

// Keys per batch, each culled by one lane of a 64-lane ballot.  44 keeps the
// LDS of the one-class semantic gradient at 25.5 KB, so six workgroups share
// a CU, as many as 80 VGPRs allow (48 would take 28 KB and allow five).
constexpr int kBwdBatch = 44;
static_assert(kBwdBatch <= 64, "the backward culls a batch with one 64-lane ballot");

// Sum over the 64 lanes of a wave; the total lands in lane 63.  Row-wise
// inclusive scan with row_shr (zero fill), then row_bcast:15 / row_bcast:31
// carry the row totals upward.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_f(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROWMASK, 0xf, true));
}
__device__ __forceinline__ float wave_sum_lane63(float x) {
    x += dpp_f<0x111, 0xf>(x);  // row_shr:1
    x += dpp_f<0x112, 0xf>(x);  // row_shr:2
    x += dpp_f<0x114, 0xf>(x);  // row_shr:4
    x += dpp_f<0x118, 0xf>(x);  // row_shr:8
    x += dpp_f<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
    x += dpp_f<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
    return x;
}

struct BwdArgs {
    TileArgs t;
    ViewTable<GradPtrs> grads;
    float* slots;              // [cap][nvals]
    uint8_t* touched;          // [cap]
    const uint32_t* svals;     // sorted emission index of each key
    int nvals;                 // 10 + k
    int semgeo;
};

constexpr int kBwdThreads = 256;  // 4 waves, one pixel per lane, 8x8 pixel block per wave
constexpr int kBwdWaves = kBwdThreads / 64;

template <int CTRL>
__device__ __forceinline__ float dpp_perm(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, false));
}

// Transposed wave reduction of NP (16 or 32) values per lane.  Each step
// halves the number of registers while doubling the lanes each partial sum
// covers: permlane32 and permlane16 swaps pair lanes 32 and 16 apart, then
// row rotate-by-8, half-row mirror and quad permutes pair lanes 8, 4 and 2
// apart, the lane's own bit choosing which value it keeps.  About 70
// instructions for 32 values instead of 6 DPP steps per value.  On return
// every lane holds the full 64-lane sum of value
//   NP = 32: 16 b1 + 8 b2 + 4 b3 + 2 b4 + b5,   NP = 16: 8 b2 + 4 b3 + 2 b4 + b5
// (b_i = bit i of the lane id); see transposed_value_index.
// Values from index NREAL on are zero in every lane: swaps of two such
// values are skipped.
template <int NP, int NREAL = NP>
__device__ __forceinline__ float wave_transpose_sum(float (&v)[NP], int lane) {
    static_assert(NP == 16 || NP == 32, "16 or 32 values");
    float r1[NP / 2];
#pragma unroll
    for (int i = 0; i < NP / 2; i++) {
        if (2 * i >= NREAL) {
            r1[i] = 0.f;
            continue;
        }
        const auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[2 * i]), __float_as_uint(v[2 * i + 1]),
                                                       false, false);
        r1[i] = __uint_as_float(s[0]) + __uint_as_float(s[1]);
    }
    float r2[NP / 4];
#pragma unroll
    for (int i = 0; i < NP / 4; i++) {
        if (4 * i >= NREAL) {
            r2[i] = 0.f;
            continue;
        }
        const auto s = __builtin_amdgcn_permlane16_swap(__float_as_uint(r1[2 * i]), __float_as_uint(r1[2 * i + 1]),
                                                       false, false);
        r2[i] = __uint_as_float(s[0]) + __uint_as_float(s[1]);
    }
    const bool h8 = lane & 8, h4 = lane & 4, h2 = lane & 2;
    float r3[NP / 8];
#pragma unroll
    for (int i = 0; i < NP / 8; i++) {
        const float keep = h8 ? r2[2 * i + 1] : r2[2 * i], send = h8 ? r2[2 * i] : r2[2 * i + 1];
        r3[i] = keep + dpp_perm<0x128>(send);  // row_ror:8 (lane ^ 8 within a row)
    }
    float r4[NP / 16];
#pragma unroll
    for (int i = 0; i < NP / 16; i++) {
        const float keep = h4 ? r3[2 * i + 1] : r3[2 * i], send = h4 ? r3[2 * i] : r3[2 * i + 1];
        r4[i] = keep + dpp_perm<0x141>(send);  // row_half_mirror
    }
    float x;
    if constexpr (NP == 32) {
        const float keep = h2 ? r4[1] : r4[0], send = h2 ? r4[0] : r4[1];
        x = keep + dpp_perm<0x4e>(send);  // quad_perm [2,3,0,1]
    } else {
        x = r4[0] + dpp_perm<0x4e>(r4[0]);
    }
    return x + dpp_perm<0xb1>(x);  // quad_perm [1,0,3,2]
}

template <int NP>
__device__ __forceinline__ int transposed_value_index(int lane) {
    const int b1 = (lane >> 1) & 1, b2 = (lane >> 2) & 1, b3 = (lane >> 3) & 1, b4 = (lane >> 4) & 1,
              b5 = (lane >> 5) & 1;
    return NP == 32 ? 16 * b1 + 8 * b2 + 4 * b3 + 2 * b4 + b5 : 8 * b2 + 4 * b3 + 2 * b4 + b5;
}

// Per-key value layout (slots): 0,1 mean2d; 2,3,4 the 2D covariance
// Sigma2 (xx, both off-diagonal entries together, yy); 5 opacity; 6,7,8 rgb;
// 9 depth; 10.. semantic values.  With Q = d^T A d (A = Sigma2^-1, d the
// offset from the mean) and u = A d, dQ/dmean = -2 u and dQ/dSigma2 = -u u^T,
// so per pixel the first five are dQ ux, dQ uy, dQ ux^2, dQ ux uy, dQ uy^2
// (u in units of 2 ln 2, dQ = dL/dQ), scaled once per key.  Summing in this
// whitened frame keeps float32 rounding relative to the gradient itself:
// summing dQ d d^T and multiplying by A on both sides afterwards would scale
// the sum's rounding by the conic's condition number (thousands for the
// thin, long splats of a room scene).
// SPARSE: no view has a dense dL/dsem; each pixel's semantic gradient is one
// (class, value) pair (or none), held in registers instead of a 257-float
// LDS column per class, which leaves room for more workgroups per CU.
// RANKED (SPARSE, k = 16, C <= 128, semantic gradient kept off geometry): a
// pixel finds its label's position in a key's list through the key's class
// rank table (mask word, popcount, nibble) and adds its value into that
// position's per-wave LDS bin; bins of one wave are written by one wave
// only, one add instruction per key, which the LDS applies in a fixed lane
// order, so sums are reproducible bit for bit.  The wave reduction then
// carries only the ten geometry values.
// With k fixed at compile time the one-class kernel is held to 80 VGPRs for
// six waves per SIMD, matching the six workgroups its LDS allows.
template <int KT, bool SPARSE, bool RANKED = false, int NB = kBwdBatch>
__global__ __launch_bounds__(kBwdThreads, (KT == 16 || KT == 3) ? (SPARSE ? 6 : 5) : 1) void render_bwd_kernel(BwdArgs b) {
    static_assert(!RANKED || (KT == 16 && SPARSE), "the rank lookup needs k = 16 and a one-class gradient");
    static_assert(NB <= 64, "the backward culls a batch with one 64-lane ballot");
    extern __shared__ __align__(16) float smem[];
    const TileArgs& a = b.t;
    const int gt = tile_of_block(blockIdx.x, gridDim.x, a.linear_tiles);
    if (gt >= a.num_tiles) return;
    if (a.counters[kStatus] & SGR_ECAPACITY) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index, held in a scalar register
    const int k = KT > 0 ? KT : a.k;
    const int kw = (KT > 0 ? ((KT + 3) & ~3) : a.kpad) >> 2;
    const int C = a.C;
    constexpr int NVMAX = 10 + (KT > 0 ? KT : kMaxK);
    // padded value count of the transposed reduction (0: per-value DPP sums);
    // RANKED reduces the ten geometry values only
    constexpr int NP = RANKED ? 16 : ((KT > 0 && NVMAX <= 16) ? 16 : ((KT > 0 && NVMAX <= 32) ? 32 : 0));
    constexpr int NREG = NP > 0 ? NP : NVMAX;
    constexpr int NRED = RANKED ? 10 : NVMAX;  // values that go through the wave reduction
    const int NV = 10 + k;

    constexpr int KM = KT > 0 ? KT : kMaxK;  // register bound on k
    constexpr int KWM = (KM + 3) / 4;         // ... and on the index words
    float* gp = smem;  // [C][257] dL/dsem of the tile's pixels, column = owning thread (dense mode)
    float4* s_r0 = (float4*)(smem + (SPARSE ? 0 : acc_floats(C)));
    float4* s_r1 = s_r0 + NB;
    float4* s_r2 = s_r1 + NB;
    float4* s_col = s_r2 + NB;
    uint32_t* s_e = (uint32_t*)(s_col + NB);                   // emission index of each key
    float* s_sv = (float*)(s_e + NB);                          // top-k values (not RANKED)
    uint32_t* s_si = (uint32_t*)(s_sv + (RANKED ? 0 : NB * k));
    uint2* s_lm = (uint2*)(s_si + NB * kw);                    // RANKED: [NB][4] (mask word, classes below)
    uint2* s_pm = s_lm + (RANKED ? 4 * NB : 0);                // RANKED: [NB] rank -> list position
    float* part = (float*)(s_pm + (RANKED ? NB : 0));          // [waves][NB][NV]
    uint32_t* flag = (uint32_t*)(part + kBwdWaves * NB * NV);  // [waves][NB]
    uint32_t* s_tk = flag + kBwdWaves * NB;  // [NB]: the batch's blended keys (index | wave mask << 8)
    __shared__ uint32_t s_maxlast;
    __shared__ int s_ntk;

    const int v = view_of_tile(a.views, a.V, gt);
    const ViewDev& vw = a.views[v];
    const int local = gt - vw.tile_off;
    const int tx = local % vw.tiles_x, ty = local / vw.tiles_x;
    const int px = tx * kTile + tile_px(tid), py = ty * kTile + tile_py(tid);
    const bool inside = px < vw.width && py < vw.height;
    const uint2 rg = a.ranges[gt];
    const uint32_t start = rg.x, end = rg.y;
    const GradPtrs gr = b.grads[v];
    const int64_t pix = (int64_t)py * vw.width + px;

    float T = 1.f;
    uint32_t last = start;
    float gC0 = 0.f, gC1 = 0.f, gC2 = 0.f, gD = 0.f, gS = 0.f;
    if (inside) {
        T = a.pix_T[vw.pix_off + pix];
        last = a.pix_last[vw.pix_off + pix];
        if (gr.rgb) { gC0 = gr.rgb[3 * pix]; gC1 = gr.rgb[3 * pix + 1]; gC2 = gr.rgb[3 * pix + 2]; }
        if (gr.depth) gD = gr.depth[pix];
        if (gr.sil) gS = gr.sil[pix];
    }
    int lab = -1;  // sparse semantic gradient of this pixel: gl at class lab
    float gl = 0.f;
    if (inside && gr.sem_label && !gr.sem) {
        lab = gr.sem_label[pix];
        gl = gr.sem_at_label ? gr.sem_at_label[pix] : 0.f;
    }
    // RANKED: the label's mask word, its bit and the bits below it (a label
    // of 128 or more is in no list: classes are below C <= 128 here)
    const bool haslab = lab >= 0 && lab < 128;
    const int lword = haslab ? (lab >> 5) : 0;
    const uint32_t lbit = (uint32_t)lab & 31u, lbelow = (1u << lbit) - 1u;
    if (tid == 0) s_maxlast = start;
    if constexpr (!SPARSE) {
        const int x0 = tx * kTile, y0 = ty * kTile;
        const int wcols = min(kTile, vw.width - x0), hrows = min(kTile, vw.height - y0);
        const int row_elems = kTile * C;
        const int dl = kBwdThreads / C, dc = kBwdThreads % C;
        for (int row = 0; row < kTile; row++) {
            const int64_t rowpix = (int64_t)(y0 + row) * vw.width + x0;
            const float* src = gr.sem ? gr.sem + rowpix * C : nullptr;
            int cx = tid / C, c = tid % C;
            for (int e = tid; e < row_elems; e += kBwdThreads) {
                float val = 0.f;
                if (row < hrows && cx < wcols) {
                    if (src) val = src[e];
                    else if (gr.sem_label && gr.sem_label[rowpix + cx] == c)
                        val = gr.sem_at_label ? gr.sem_at_label[rowpix + cx] : 0.f;
                }
                gp[c * kAccStride + slot_of(cx, row)] = val;
                cx += dl;
                c += dc;
                if (c >= C) { c -= C; cx++; }
            }
        }
    }
    __syncthreads();
    if (inside && last > start) atomicMax(&s_maxlast, last);
    __syncthreads();
    const uint32_t maxlast = __builtin_amdgcn_readfirstlane(s_maxlast);
    // this wave's bound on blended list positions
    uint32_t wlast = inside ? last : start;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wlast = max(wlast, (uint32_t)__shfl_xor((int)wlast, o, 64));
    wlast = __builtin_amdgcn_readfirstlane(wlast);
    const float amin = a.alpha_min, amax = a.alpha_max;
    const float k2ln2 = 1.38629436111989061883f;    // 2 ln 2
    const float k2ln2sq = 1.92181205567280529356f;  // (2 ln 2)^2
    const int wx0 = tx * kTile + (wv & 1) * 8, wy0 = ty * kTile + (wv >> 1) * 8;  // this wave's 8x8 block
    float R = 0.f;

    // Staging registers: the four waves each carry a quarter of the next
    // batch while the current one is composited.  For key j: lane j of wave
    // 0 holds r0 and r1, of wave 1 r2, the colour and the emission index, of
    // waves 2 and 3 each half of the top-k values and class words.
    constexpr int VH = (KM + 1) / 2, WH = (KWM + 1) / 2;  // values / words of the first half
    constexpr int NSTG = (VH + WH) > 9 ? (VH + WH) : 9;
    uint32_t stg[NSTG];
#pragma unroll
    for (int q = 0; q < NSTG; q++) stg[q] = 0u;
    const int role = tid >> 6, rl = tid & 63;
    auto put4 = [&](int at, const float4& v) {
        stg[at] = __float_as_uint(v.x); stg[at + 1] = __float_as_uint(v.y);
        stg[at + 2] = __float_as_uint(v.z); stg[at + 3] = __float_as_uint(v.w);
    };
    auto get4 = [&](int at) {
        return make_float4(__uint_as_float(stg[at]), __uint_as_float(stg[at + 1]), __uint_as_float(stg[at + 2]),
                           __uint_as_float(stg[at + 3]));
    };
    auto fetch = [&](uint32_t f0, int fn) {
        if (rl >= fn) return;
        const uint32_t e = b.svals[f0 + rl], g = a.owner[e];  // emission index, pair
        if (role == 0) {
            const float4* rp = (const float4*)(a.srec + g);
            put4(0, rp[0]);
            put4(4, rp[1]);
        } else if (role == 1) {
            const float4* rp = (const float4*)(a.srec + g);
            put4(0, rp[2]);
            put4(4, a.scol[g]);
            stg[8] = e;
        } else if constexpr (RANKED) {
            // wave 2: the class words and the rank -> position nibbles; wave 3: the mask
            const uint32_t* rk = a.srk + (size_t)g * kRankWords;
            if (role == 2) {
                const uint4 w4 = *(const uint4*)((const uint32_t*)(a.ssi) + (size_t)g * 4);
                stg[0] = w4.x; stg[1] = w4.y; stg[2] = w4.z; stg[3] = w4.w;
                stg[4] = rk[4];
                stg[5] = rk[5];
            } else {
                const uint4 m4 = *(const uint4*)rk;
                stg[0] = m4.x; stg[1] = m4.y; stg[2] = m4.z; stg[3] = m4.w;
            }
        } else {
            const int v0 = role == 2 ? 0 : VH, w0 = role == 2 ? 0 : WH;
            const float* sv = a.ssv + (size_t)g * k;
            const uint32_t* si = (const uint32_t*)(a.ssi) + (size_t)g * kw;
#pragma unroll
            for (int m = 0; m < VH; m++)
                if (v0 + m < k && v0 + m < KM) stg[m] = __float_as_uint(sv[v0 + m]);
#pragma unroll
            for (int m = 0; m < WH; m++)
                if (w0 + m < kw && w0 + m < KWM) stg[VH + m] = si[w0 + m];
        }
    };

    int64_t bend = maxlast;
    uint32_t b0 = (uint32_t)max((int64_t)start, bend - NB);
    if (bend > (int64_t)start) fetch(b0, (int)(bend - b0));
    while (bend > (int64_t)start) {
        const int nb = (int)(bend - b0);
        if (rl < nb) {
            if (role == 0) {
                s_r0[rl] = get4(0);
                s_r1[rl] = get4(4);
            } else if (role == 1) {
                s_r2[rl] = get4(0);
                s_col[rl] = get4(4);
                s_e[rl] = stg[8];
            } else if constexpr (RANKED) {
                if (role == 2) {
#pragma unroll
                    for (int m = 0; m < 4; m++) s_si[rl * 4 + m] = stg[m];
                    s_pm[rl] = make_uint2(stg[4], stg[5]);
                } else {
                    uint32_t below = 0u;
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        s_lm[rl * 4 + q] = make_uint2(stg[q], below);
                        below += __builtin_popcount(stg[q]);
                    }
                }
            } else {
                const int v0 = role == 2 ? 0 : VH, w0 = role == 2 ? 0 : WH;
#pragma unroll
                for (int m = 0; m < VH; m++)
                    if (v0 + m < k && v0 + m < KM) s_sv[rl * k + v0 + m] = __uint_as_float(stg[m]);
#pragma unroll
                for (int m = 0; m < WH; m++)
                    if (w0 + m < kw && w0 + m < KWM) s_si[rl * kw + w0 + m] = stg[VH + m];
            }
        }
        __syncthreads();
        const int64_t nend = b0;
        const uint32_t nb0 = (uint32_t)max((int64_t)start, nend - NB);
        if (nend > (int64_t)start) fetch(nb0, (int)(nend - nb0));

        // Keys of this batch that can touch this wave's pixels: before the
        // wave's last blend and with a pixel rectangle meeting its block.
        bool hit = false;
        if (lane < nb) {
            const float4 q2 = s_r2[lane];
            const uint32_t rx = __float_as_uint(q2.x), ry = __float_as_uint(q2.y);
            const int bx0 = max(wx0, (int)(rx & 0xffffu)), bx1 = min(wx0 + 7, (int)(rx >> 16));
            const int by0 = max(wy0, (int)(ry & 0xffffu)), by1 = min(wy0 + 7, (int)(ry >> 16));
            hit = b0 + lane < wlast && bx0 <= bx1 && by0 <= by1;
            if (hit) hit = conic_meets_block(s_r0[lane], s_r1[lane], bx0, bx1, by0, by1, amin);
            if (!hit) flag[wv * NB + lane] = 0u;
        }
        uint64_t todo = __ballot(hit);
        while (todo) {  // back to front
            const int j = 63 - __builtin_clzll(todo);
            todo &= ~(1ull << j);
            const uint32_t s = b0 + j;
            const float4 q0 = s_r0[j], q1 = s_r1[j], q2 = s_r2[j];
            const uint32_t rx = __float_as_uint(q2.x), ry = __float_as_uint(q2.y);
            float G, dx, dy, uu;
            const float alpha = eval_alpha_u(q0, q1, px, py, amax, &G, &dx, &dy, &uu);
            const bool act = s < last && px >= (int)(rx & 0xffffu) && px <= (int)(rx >> 16) &&
                             py >= (int)(ry & 0xffffu) && py <= (int)(ry >> 16) && alpha >= amin;
            const uint64_t any = __ballot(act);
            if (any) {
                float val[NREG];
#pragma unroll
                for (int q = 0; q < NREG; q++) val[q] = 0.f;
                const float4 col = s_col[j];
                // the key's class words; the pixel's dL/dsem at its top-k
                // classes (dense form) and their sum weighted by the key's
                // values (only when the semantic loss reaches alpha)
                uint32_t cw[KWM];
                const float* sv = s_sv + (RANKED ? 0 : j * k);
                {
                    const uint32_t* si = s_si + j * kw;
#pragma unroll
                    for (int mw = 0; mw < KWM; mw++) cw[mw] = (KT > 0 || mw < kw) ? si[mw] : 0u;
                }
                float sg[KM];
                float es = 0.f;
                if constexpr (!SPARSE) {
#pragma unroll
                    for (int m = 0; m < KM; m++) {
                        if (m < k) {
                            const uint32_t cls = (cw[m >> 2] >> (8 * (m & 3))) & 0xffu;
                            sg[m] = gp[cls * kAccStride + tid];
                            es += sv[m] * sg[m];
                        }
                    }
                } else if (!RANKED && b.semgeo) {
#pragma unroll
                    for (int m = 0; m < KM; m++) {
                        if (m < k) {
                            const uint32_t cls = (cw[m >> 2] >> (8 * (m & 3))) & 0xffu;
                            es += sv[m] * ((int)cls == lab ? gl : 0.f);
                        }
                    }
                }
                const float om = 1.f - alpha;
                const float rom = __builtin_amdgcn_rcpf(om);
                const float Tf = T * rom;  // transmittance in front of this Gaussian
                const float w = act ? alpha * Tf : 0.f;  // blend weight; 0 where this pixel does not blend
                float e = col.x * gC0 + col.y * gC1 + col.z * gC2 + col.w * gD + gS;
                if (!RANKED && b.semgeo) e += es;  // (the ranked kernel runs only with semgeo off)
                const float dalpha = Tf * e - R * rom;
                if (act) {
                    T = Tf;
                    R += e * w;
                }
                // alpha = min(alpha_max, o G): no gradient through the clamp
                // (o G < alpha_max exactly when alpha < alpha_max)
                const bool free = act && alpha < amax;
                const float dQ = free ? dalpha * (-0.5f * alpha) : 0.f;
                val[5] = free ? dalpha * G : 0.f;
                // per pixel, with u = A d / (2 ln 2) = (ca uu, cb ux + cc dy):
                // dQ ux, dQ uy, dQ ux^2, dQ ux uy, dQ uy^2; the key's mean
                // and Sigma2 gradients are these sums, scaled once
                const float ux = q1.x * uu;
                const float uy = fmaf(q1.y, ux, q1.z * dy);
                val[0] = dQ * ux;
                val[1] = dQ * uy;
                val[2] = val[0] * ux;
                val[3] = val[0] * uy;
                val[4] = val[1] * uy;
                val[6] = w * gC0;
                val[7] = w * gC1;
                val[8] = w * gC2;
                val[9] = w * gD;
                if constexpr (RANKED) {
                    // semantic values go to the per-wave bins below
                } else if constexpr (SPARSE) {
                    // one class per pixel: w gl where the key's class is the
                    // label (no class where the pixel does not blend); the
                    // label is kept in one register, so each class costs a
                    // compare and a select
                    const float wg = w * gl;
                    int labm = act ? lab : -1;
                    asm volatile("" : "+v"(labm));
#pragma unroll
                    for (int m = 0; m < KM; m++)
                        if (m < k) val[10 + m] = (int)((cw[m >> 2] >> (8 * (m & 3))) & 0xffu) == labm ? wg : 0.f;
                } else {
#pragma unroll
                    for (int m = 0; m < KM; m++)
                        if (m < k) val[10 + m] = w * sg[m];
                }
                float* dst = part + (wv * NB + j) * NV;
                const bool one = (any & (any - 1)) == 0;
                if (one) {
                    // one active lane: its values are the wave's sums
                    if (act) {
#pragma unroll
                        for (int q = 0; q < NREG; q++)
                            if (q < NV && q < NRED) dst[q] = val[q];
                    }
                }
                // Two separate regions, the single-lane one first: the
                // reduction's in-place lane swaps then need no copies of the
                // values for a single-lane store after them.
                __builtin_amdgcn_sched_barrier(0);
                if (one) {
                } else if constexpr (NP > 0) {
                    const float sum = wave_transpose_sum<NP, (RANKED ? 10 : (KT > 0 ? 10 + KT : NP))>(val, lane);
                    const int q = transposed_value_index<NP>(lane);
                    if ((lane & (NP == 32 ? 1 : 3)) == 0 && q < NV && q < NRED) dst[q] = sum;
                } else {
#pragma unroll
                    for (int q = 0; q < NREG; q++) {
                        if (q < NV) {
                            const float sum = wave_sum_lane63(val[q]);
                            if (lane == 63) dst[q] = sum;
                        }
                    }
                }
                if constexpr (RANKED) {
                    // the wave's semantic bins of this key: cleared, then each
                    // blending lane whose label is in the key's list adds w gl
                    // at that class's list position (in order: one wave's LDS
                    // operations complete in issue order)
                    float* sb = dst + 10;
                    if (lane < 16) sb[lane] = 0.f;
                    const float wg = w * gl;
                    if ((__float_as_uint(q2.w) >> 31) == 0u) {  // distinct classes
                        const uint2 mw = s_lm[j * 4 + lword];
                        const uint2 pm = s_pm[j];
                        const uint32_t rank = mw.y + __builtin_popcount(mw.x & lbelow);
                        const uint64_t perm = ((uint64_t)pm.y << 32) | pm.x;
                        const uint32_t slot = (uint32_t)(perm >> ((4u * rank) & 63u)) & 15u;
                        if (act && haslab && ((mw.x >> lbit) & 1u)) atomicAdd(sb + slot, wg);
                    } else {
                        // a list with a repeated class: each of its positions
                        // that holds the label gets w gl
                        const uint32_t* si = s_si + j * 4;
#pragma unroll
                        for (int m = 0; m < 16; m++) {
                            const uint32_t cls = (si[m >> 2] >> (8 * (m & 3))) & 0xffu;
                            if (act && (int)cls == lab) atomicAdd(sb + m, wg);
                        }
                    }
                }
            }
            if (lane == 0) flag[wv * NB + j] = any ? 1u : 0u;
        }
        __syncthreads();
        // The keys of the batch some wave blended, with the mask of those
        // waves, listed once by wave 0 (it also writes every key's touched
        // flag); then the block sums only those keys' partials.
        if (wv == 0) {
            uint32_t wm = 0u;
            if (lane < nb) {
#pragma unroll
                for (int w = 0; w < kBwdWaves; w++) wm |= flag[w * NB + lane] != 0u ? 1u << w : 0u;
                b.touched[s_e[lane]] = wm ? 1 : 0;
            }
            const uint64_t tm = __ballot(wm != 0u);
            if (wm) s_tk[__popcll(tm & ((1ull << lane) - 1ull))] = (uint32_t)lane | (wm << 8);
            if (lane == 0) s_ntk = (int)__popcll(tm);
        }
        __syncthreads();
        const int ntk = __builtin_amdgcn_readfirstlane(s_ntk);
        for (int idx = tid; idx < ntk * NV; idx += kBwdThreads) {
            const int at = idx / NV, q = idx - at * NV;
            const uint32_t tk = s_tk[at];
            const int j = (int)(tk & 0xffu);
            const uint32_t wm = tk >> 8;
            float sum = 0.f;
#pragma unroll
            for (int w = 0; w < kBwdWaves; w++)
                if ((wm >> w) & 1u) sum += part[(w * NB + j) * NV + q];
            // with u in units of 2 ln 2: dL/dmean = -2 (2 ln 2) sum dQ u;
            // dL/dSigma2 = -(2 ln 2)^2 sum dQ u u^T, its two off-diagonal
            // entries together in slot 3
            if (q < 2) sum *= -2.f * k2ln2;
            else if (q == 3) sum *= -2.f * k2ln2sq;
            else if (q < 5) sum *= -k2ln2sq;
            b.slots[(size_t)s_e[j] * NV + q] = sum;
        }
        __syncthreads();
        bend = nend;
        b0 = nb0;
    }
    for (uint32_t s = maxlast + tid; s < end; s += kBwdThreads) b.touched[b.svals[s]] = 0;
}

// Sum of each visible pair's key slots.  A pair with a short key segment is summed by its own lane in
// emission order; long segments (a Gaussian near the camera can cover
// thousands of tiles) are taken one at a time by the whole wave: lane l sums
// keys l, l+64, ... and the wave reduces in a fixed pattern.  Either way the
// result does not depend on timing.  Most lanes of the launch are idle (one
// per possible pair), so the bound of 8 waves per SIMD (at most 64 registers)
// lets the whole grid be resident at once.
constexpr uint32_t kShortSeg = 16;

// Bit i set when byte i of x is nonzero.
__device__ __forceinline__ uint32_t nonzero_nibble(uint32_t x) {
    const uint32_t t = (((x & 0x7f7f7f7fu) + 0x7f7f7f7fu) | x) & 0x80808080u;
    return ((t >> 7) | (t >> 14) | (t >> 21) | (t >> 28)) & 0xfu;
}

template <int KT>
__global__ __launch_bounds__(256, KT > 0 ? 8 : 1) void gather_slots(const float* __restrict__ slots,
                                                    const uint8_t* __restrict__ touched,
                                                    const uint32_t* __restrict__ toff,
                                                    const uint32_t* __restrict__ tcount,
                                                    const uint32_t* __restrict__ order,
                                                    const uint32_t* __restrict__ counters, int nv_rt,
                                                    float* __restrict__ g2d) {
    constexpr int NVMAX = 10 + (KT > 0 ? KT : kMaxK);
    const int NV = KT > 0 ? 10 + KT : nv_rt;
    const uint32_t nvis = counters[kNumVisible];
    const bool ok = !(counters[kStatus] & SGR_ECAPACITY);
    // Pairs are taken by depth rank r (their keys are the emission range
    // [toff[r], toff[r] + tcount[r])), so the nearest ones (the longest
    // segments) are adjacent; striding ranks across all the workgroups the
    // launch could need (one lane per possible pair, most of them idle)
    // spreads them over the machine instead of queueing them in a few waves.
    // The sums go to the pair's record g = order[r].
    const uint32_t r = threadIdx.x * gridDim.x + blockIdx.x;
    const int lane = threadIdx.x & 63;
    const bool valid = r < nvis;
    uint32_t e0 = 0, e1 = 0, g = 0;
    if (valid) g = order[r];
    if (valid && ok) {
        e0 = toff[r];
        e1 = e0 + tcount[r];
    }
    const bool longseg = e1 - e0 > kShortSeg;
    if (valid && !longseg) {
        // the segment's touched flags, at most 16 bytes, from the (at most
        // five) aligned words that hold them, all loaded before any slot
        uint32_t mask = 0u;
        if (e1 > e0) {
            const uint32_t* tw = reinterpret_cast<const uint32_t*>(touched);
            const uint32_t w0 = e0 >> 2, wl = (e1 - 1u) >> 2;
            uint32_t bits = 0u;
#pragma unroll
            for (uint32_t j = 0; j < 5; j++)
                if (w0 + j <= wl) bits |= nonzero_nibble(tw[w0 + j]) << (4 * j);
            mask = (bits >> (e0 & 3u)) & ((1u << (e1 - e0)) - 1u);
        }
        float acc[NVMAX];
#pragma unroll
        for (int q = 0; q < NVMAX; q++) acc[q] = 0.f;
        while (mask) {  // the touched slots in emission order
            const float* sl = slots + (size_t)(e0 + (uint32_t)__builtin_ctz(mask)) * NV;
            mask &= mask - 1u;
#pragma unroll
            for (int q = 0; q < NVMAX; q++)
                if (q < NV) acc[q] += sl[q];
        }
#pragma unroll
        for (int q = 0; q < NVMAX; q++)
            if (q < NV) g2d[(size_t)g * NV + q] = acc[q];
    }
    uint64_t lm = __ballot(valid && longseg);
    while (lm) {
        const int src = __ffsll((long long)lm) - 1;
        lm &= lm - 1;
        const uint32_t s0 = __shfl(e0, src, 64), s1 = __shfl(e1, src, 64);
        const uint32_t gsrc = __shfl(g, src, 64);
        float acc[NVMAX];
#pragma unroll
        for (int q = 0; q < NVMAX; q++) acc[q] = 0.f;
        for (uint32_t e = s0 + lane; e < s1; e += 64) {
            if (!touched[e]) continue;
            const float* sl = slots + (size_t)e * NV;
#pragma unroll
            for (int q = 0; q < NVMAX; q++)
                if (q < NV) acc[q] += sl[q];
        }
#pragma unroll
        for (int q = 0; q < NVMAX; q++) {
            if (q < NV) {
                const float sum = wave_sum_lane63(acc[q]);
                if (lane == 63) g2d[(size_t)gsrc * NV + q] = sum;
            }
        }
    }
}

struct ProjBwdArgs {
    const float *means, *scales, *quats, *opacity;
    const ViewDev* views;
    int64_t n;
    int V, k, NV, C;
    float lowpass;
    const uint32_t* gp_of_lin;
    const float* g2d;
    const uint8_t* sorig;      // [vis][kpad]: list index of each stored top-k position
    int kpad;
    sgr_adam_segment seg[6];   // with Adam: means, scales, quats, opacity, rgb, sem_val
    AdamParams h;
    const uint32_t* counters;
    float *d_means, *d_scales, *d_quats, *d_opacity, *d_rgb, *d_sem;
};

// Chain rule from each (view, Gaussian) pair's 2D gradient to the 3D
// parameters, in float32 (the gradients need 1e-3; the binning, which must
// match an FP64 reference bit for bit, is the part kept in FP64), summed
// over views in view order.
//
// With ADAM the gradients are not written: each block stages its 256
// Gaussians' gradients of one parameter tensor in LDS, a contiguous range of
// that tensor, and the block applies the Adam update to the range with
// coalesced loads of p, m and v.  Those rows are loaded one or two tensors
// ahead of their update (the means' and scales' under the chain rule), so
// their latency overlaps the work before it.
constexpr int kAdamChunk = 8;

template <int WM>
__device__ __forceinline__ void adam_rows(const sgr_adam_segment& sg, const float* st, int64_t i0, int cnt, int w,
                                          const AdamParams& h) {
    const int ws = w | 1;  // odd row stride: the rows were written without bank conflicts
    const int tot = cnt * w;
    const int64_t base = i0 * w;
    // at most kAdamChunk elements per thread in flight (24 registers): the
    // widest rows (the top-k values) would otherwise hold 48
    constexpr int CH = WM < kAdamChunk ? WM : kAdamChunk;
    __syncthreads();  // the rows are staged, and every thread has read its parameters
#pragma unroll
    for (int u0 = 0; u0 < WM; u0 += CH) {
        float m[CH], v[CH], p[CH];
#pragma unroll
        for (int u = 0; u < CH; u++) {
            const int e = (int)threadIdx.x + 256 * (u0 + u);
            if (u0 + u < WM && e < tot) {
                m[u] = sg.m[base + e];
                v[u] = sg.v[base + e];
                p[u] = sg.p[base + e];
            }
        }
#pragma unroll
        for (int u = 0; u < CH; u++) {
            const int e = (int)threadIdx.x + 256 * (u0 + u);
            if (u0 + u < WM && e < tot) {
                const int t = e / w, c = e - t * w;
                adam_update(st[t * ws + c], m[u], v[u], p[u], sg.lo, sg.hi, h);
                sg.m[base + e] = m[u];
                sg.v[base + e] = v[u];
                sg.p[base + e] = p[u];
            }
        }
    }
    __syncthreads();  // before the rows are overwritten
}

// The same update split in two, so a tensor's rows can be loaded before
// the work that precedes their update: the block's m, v and p rows of one
// tensor (WM elements per thread), then, once its gradients are staged in
// st, the update and the stores.
template <int WM>
struct AdamRows {
    float m[WM], v[WM], p[WM];
};
template <int WM, int U0 = 0>  // (elements U0 .. U0 + WM - 1 of each thread)
__device__ __forceinline__ void adam_load(const sgr_adam_segment& sg, int64_t i0, int cnt, int w, AdamRows<WM>& r) {
    const int tot = cnt * w;
    const int64_t base = i0 * w;
#pragma unroll
    for (int u = 0; u < WM; u++) {
        const int e = (int)threadIdx.x + 256 * (U0 + u);
        if (e < tot) {
            r.m[u] = sg.m[base + e];
            r.v[u] = sg.v[base + e];
            r.p[u] = sg.p[base + e];
        }
    }
}
template <int WM, int U0 = 0>
__device__ __forceinline__ void adam_apply(const sgr_adam_segment& sg, const float* st, int64_t i0, int cnt, int w,
                                           const AdamParams& h, AdamRows<WM>& r) {
    const int ws = w | 1;
    const int tot = cnt * w;
    const int64_t base = i0 * w;
#pragma unroll
    for (int u = 0; u < WM; u++) {
        const int e = (int)threadIdx.x + 256 * (U0 + u);
        if (e < tot) {
            const int t = e / w, c = e - t * w;
            adam_update(st[t * ws + c], r.m[u], r.v[u], r.p[u], sg.lo, sg.hi, h);
            sg.m[base + e] = r.m[u];
            sg.v[base + e] = r.v[u];
            sg.p[base + e] = r.p[u];
        }
    }
}

// a0 b0 + a1 b1 + a2 b2 (+ c) as a fixed chain of fused multiply-adds
__device__ __forceinline__ float fdot3(float a0, float b0, float a1, float b1, float a2, float b2) {
#pragma clang fp contract(off)
    return fmaf(a2, b2, fmaf(a1, b1, a0 * b0));
}
__device__ __forceinline__ float fdot3c(float a0, float b0, float a1, float b1, float a2, float b2, float c) {
    return fmaf(a2, b2, fmaf(a1, b1, fmaf(a0, b0, c)));
}

template <int KT, bool ADAM>
__global__ __launch_bounds__(256) void project_backward_kernel(ProjBwdArgs a) {
    // The fused multiply-adds are written out and nothing else is contracted
    // (no choice left to the compiler): the kernel with the Adam step and the
    // one without compute the same gradients bit for bit.
#pragma clang fp contract(off)
    const int64_t i0 = blockIdx.x * 256ll, i = i0 + threadIdx.x;
    if (!ADAM && i >= a.n) return;
    // with ADAM every thread reaches the block's barriers; one past the end
    // reads the last Gaussian's parameters and takes no view
    const bool live = i < a.n;
    const int64_t il = live ? i : a.n - 1;
    const bool ok = live && !(a.counters[kStatus] & SGR_ECAPACITY);
    const int cnt = (int)min<int64_t>(256, a.n - i0);
    // the Adam rows of the means and scales are loaded first, under the
    // chain rule (the parameters it reads are stored only after the block's
    // next barrier)
    AdamRows<3> r_means, r_scales;
    if (ADAM) {
        adam_load<3>(a.seg[0], i0, cnt, 3, r_means);
        adam_load<3>(a.seg[1], i0, cnt, 3, r_scales);
    }
    float gm[3] = {0, 0, 0}, gs[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0};
    float go = 0.f, grgb[3] = {0.f, 0.f, 0.f};
    constexpr int KM = KT > 0 ? KT : kMaxK;
    const int k = KT > 0 ? KT : a.k;
    const float m0 = a.means[3 * il], m1 = a.means[3 * il + 1], m2 = a.means[3 * il + 2];
    const float q0 = a.quats[4 * il], q1 = a.quats[4 * il + 1], q2 = a.quats[4 * il + 2], q3 = a.quats[4 * il + 3];
    const float qn = sqrtf(fmaf(q3, q3, fmaf(q2, q2, fmaf(q1, q1, q0 * q0))));
    const float qw = q0 / qn, qx = q1 / qn, qy = q2 / qn, qz = q3 / qn;
    float Rq[9];
    Rq[0] = fmaf(-2.f, fmaf(qy, qy, qz * qz), 1.f);
    Rq[1] = 2.f * fmaf(qx, qy, -(qw * qz));
    Rq[2] = 2.f * fmaf(qx, qz, qw * qy);
    Rq[3] = 2.f * fmaf(qx, qy, qw * qz);
    Rq[4] = fmaf(-2.f, fmaf(qx, qx, qz * qz), 1.f);
    Rq[5] = 2.f * fmaf(qy, qz, -(qw * qx));
    Rq[6] = 2.f * fmaf(qx, qz, -(qw * qy));
    Rq[7] = 2.f * fmaf(qy, qz, qw * qx);
    Rq[8] = fmaf(-2.f, fmaf(qx, qx, qy * qy), 1.f);
    const float s[3] = {a.scales[3 * il], a.scales[3 * il + 1], a.scales[3 * il + 2]};
    float M[9], S3[9];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) M[3 * r + c] = Rq[3 * r + c] * s[c];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) S3[3 * r + c] = fdot3(M[3 * r], M[3 * c], M[3 * r + 1], M[3 * c + 1], M[3 * r + 2], M[3 * c + 2]);
    float dS3[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int v = 0; v < a.V && ok; v++) {
        const uint32_t g = a.gp_of_lin[(int64_t)v * a.n + i];
        if (g == kInvalid) continue;
        const float* d2 = a.g2d + (size_t)g * a.NV;
        const ViewDev& vw = a.views[v];
        float W[9];
        for (int r = 0; r < 9; r++) W[r] = vw.R[r];
        float p[3];
        for (int r = 0; r < 3; r++) p[r] = fdot3c(W[3 * r], m0, W[3 * r + 1], m1, W[3 * r + 2], m2, vw.t[r]);
        const float fx = vw.fx, fy = vw.fy, x = p[0], y = p[1], z = p[2];
        const float J[6] = {fx / z, 0, -fx * x / (z * z), 0, fy / z, -fy * y / (z * z)};
        float T[6];
        for (int r = 0; r < 2; r++)
            for (int c = 0; c < 3; c++) T[3 * r + c] = fdot3(J[3 * r], W[c], J[3 * r + 1], W[3 + c], J[3 * r + 2], W[6 + c]);
        float TS3[6];
        for (int r = 0; r < 2; r++)
            for (int c = 0; c < 3; c++)
                TS3[3 * r + c] = fdot3(T[3 * r], S3[c], T[3 * r + 1], S3[3 + c], T[3 * r + 2], S3[6 + c]);
        // the slots carry dL/dSigma2 itself (the low-pass term is a constant)
        const float dS2[4] = {d2[2], 0.5f * d2[3], 0.5f * d2[3], d2[4]};
        for (int r = 0; r < 3; r++)
            for (int c = 0; c < 3; c++)
                dS3[3 * r + c] = fmaf(T[3 + r], fmaf(dS2[3], T[3 + c], dS2[2] * T[c]),
                                      fmaf(T[r], fmaf(dS2[1], T[3 + c], dS2[0] * T[c]), dS3[3 * r + c]));
        float dT[6];
        for (int r = 0; r < 2; r++)
            for (int c = 0; c < 3; c++) dT[3 * r + c] = 2.0f * fmaf(dS2[2 * r + 1], TS3[3 + c], dS2[2 * r] * TS3[c]);
        float dJ[6];
        for (int r = 0; r < 2; r++)
            for (int c = 0; c < 3; c++) dJ[3 * r + c] = fdot3(dT[3 * r], W[3 * c], dT[3 * r + 1], W[3 * c + 1], dT[3 * r + 2], W[3 * c + 2]);
        const float z2 = z * z, z3 = z2 * z;
        float dp[3];
        dp[0] = dJ[2] * (-fx / z2);
        dp[1] = dJ[5] * (-fy / z2);
        dp[2] = fmaf(dJ[5], 2.0f * fy * y / z3, fmaf(dJ[4], -fy / z2, fmaf(dJ[2], 2.0f * fx * x / z3, dJ[0] * (-fx / z2))));
        const float gmx = d2[0], gmy = d2[1];
        dp[0] += gmx * fx / z;
        dp[1] += gmy * fy / z;
        dp[2] += -gmx * fx * x / z2 - gmy * fy * y / z2 + d2[9];
        for (int c = 0; c < 3; c++) gm[c] = fdot3c(W[c], dp[0], W[3 + c], dp[1], W[6 + c], dp[2], gm[c]);
        go += d2[5];
        grgb[0] += d2[6];
        grgb[1] += d2[7];
        grgb[2] += d2[8];
    }
    // Sigma3 = M M^T, M = Rq diag(s): dM = 2 dS3 M
    float dM[9];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) dM[3 * r + c] = 2.0f * fdot3(dS3[3 * r], M[c], dS3[3 * r + 1], M[3 + c], dS3[3 * r + 2], M[6 + c]);
    for (int c = 0; c < 3; c++) gs[c] = fdot3(dM[c], Rq[c], dM[3 + c], Rq[3 + c], dM[6 + c], Rq[6 + c]);
    float dR[9];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) dR[3 * r + c] = dM[3 * r + c] * s[c];
    float dq[4];
    // dL/dq of R(q) (the derivative of each rotation entry in q), left to right
    dq[0] = 2.0f * fmaf(qx, dR[7], fmaf(-qy, dR[6], fmaf(-qx, dR[5], fmaf(qz, dR[3], fmaf(qy, dR[2], -qz * dR[1])))));
    dq[1] = 2.0f * fmaf(-2.0f * qx, dR[8], fmaf(qw, dR[7], fmaf(qz, dR[6], fmaf(-qw, dR[5],
                   fmaf(-2.0f * qx, dR[4], fmaf(qy, dR[3], fmaf(qz, dR[2], qy * dR[1])))))));
    dq[2] = 2.0f * fmaf(-2.0f * qy, dR[8], fmaf(qz, dR[7], fmaf(-qw, dR[6], fmaf(qz, dR[5],
                   fmaf(qx, dR[3], fmaf(qw, dR[2], fmaf(qx, dR[1], -2.0f * qy * dR[0])))))));
    dq[3] = 2.0f * fmaf(qy, dR[7], fmaf(qx, dR[6], fmaf(qy, dR[5], fmaf(-2.0f * qz, dR[4],
                   fmaf(qw, dR[3], fmaf(qx, dR[2], fmaf(-qw, dR[1], -2.0f * qz * dR[0])))))));
    const float dot = fmaf(dq[3], qz, fmaf(dq[2], qy, fmaf(dq[1], qx, dq[0] * qw)));
    const float qh[4] = {qw, qx, qy, qz};
    for (int c = 0; c < 4; c++) gq[c] = fmaf(-qh[c], dot, dq[c]) / qn;
    if (!ADAM) {
        if (a.d_means) for (int c = 0; c < 3; c++) a.d_means[3 * i + c] = gm[c];
        if (a.d_scales) for (int c = 0; c < 3; c++) a.d_scales[3 * i + c] = gs[c];
        if (a.d_quats) for (int c = 0; c < 4; c++) a.d_quats[4 * i + c] = gq[c];
        if (a.d_opacity) a.d_opacity[i] = go;
        if (a.d_rgb) for (int c = 0; c < 3; c++) a.d_rgb[3 * i + c] = grgb[c];
    }
    constexpr int kRow = (KM | 1) > 5 ? (KM | 1) : 5;  // widest staged row: quats (4 | 1) or the top-k values
    __shared__ float st[ADAM ? 256 * kRow : 1];
    const int tid = threadIdx.x;
    if (ADAM) {
        // each tensor's update with the next tensors' rows already in flight
        AdamRows<4> r_quats;
        AdamRows<1> r_opac;
        AdamRows<3> r_rgb;
        for (int c = 0; c < 3; c++) st[tid * 3 + c] = gm[c];
        adam_load<4>(a.seg[2], i0, cnt, 4, r_quats);
        __syncthreads();  // the rows are staged, and every thread has read its parameters
        adam_apply<3>(a.seg[0], st, i0, cnt, 3, a.h, r_means);
        __syncthreads();
        for (int c = 0; c < 3; c++) st[tid * 3 + c] = gs[c];
        adam_load<1>(a.seg[3], i0, cnt, 1, r_opac);
        __syncthreads();
        adam_apply<3>(a.seg[1], st, i0, cnt, 3, a.h, r_scales);
        __syncthreads();
        for (int c = 0; c < 4; c++) st[tid * 5 + c] = gq[c];
        adam_load<3>(a.seg[4], i0, cnt, 3, r_rgb);
        __syncthreads();
        adam_apply<4>(a.seg[2], st, i0, cnt, 4, a.h, r_quats);
        __syncthreads();
        st[tid] = go;
        __syncthreads();
        adam_apply<1>(a.seg[3], st, i0, cnt, 1, a.h, r_opac);
        __syncthreads();
        for (int c = 0; c < 3; c++) st[tid * 3 + c] = grgb[c];
        __syncthreads();
        adam_apply<3>(a.seg[4], st, i0, cnt, 3, a.h, r_rgb);
        __syncthreads();
    }
    if (ADAM || a.d_sem) {
        // the top-k value gradients in stored order, summed over views (after
        // the chain rule, so its registers are free), then written to the list
        // positions they came from (the same for every view of a Gaussian)
        // with a fixed k the first half of the value rows is loaded first
        constexpr int SH = KT > 0 ? (KM + 1) / 2 : 1;
        AdamRows<SH> r_sem0;
        AdamRows<KM - SH> r_sem1;
        if (ADAM && KT > 0) adam_load<SH>(a.seg[5], i0, cnt, k, r_sem0);
        float gsem[KM];
#pragma unroll
        for (int p = 0; p < KM; p++) gsem[p] = 0.f;
        uint32_t gany = kInvalid;
        for (int v = 0; v < a.V && ok; v++) {
            const uint32_t g = a.gp_of_lin[(int64_t)v * a.n + i];
            if (g == kInvalid) continue;
            gany = g;
            const float* d2 = a.g2d + (size_t)g * a.NV + 10;
#pragma unroll
            for (int p = 0; p < KM; p++)
                if (p < k) gsem[p] += d2[p];
        }
        float* ds = ADAM ? st + tid * (k | 1) : a.d_sem + i * k;
        if (gany == kInvalid) {
            for (int m = 0; m < k; m++) ds[m] = 0.f;
        } else {
            const uint32_t* so = (const uint32_t*)(a.sorig + (size_t)gany * a.kpad);
#pragma unroll
            for (int p = 0; p < KM; p++)
                if (p < k) ds[(so[p >> 2] >> (8 * (p & 3))) & 0xffu] = gsem[p];
        }
        if (ADAM && KT > 0) {
            adam_load<KM - SH, SH>(a.seg[5], i0, cnt, k, r_sem1);
            __syncthreads();
            adam_apply<SH>(a.seg[5], st, i0, cnt, k, a.h, r_sem0);
            adam_apply<KM - SH, SH>(a.seg[5], st, i0, cnt, k, a.h, r_sem1);
        } else if (ADAM) {
            adam_rows<KM>(a.seg[5], st, i0, cnt, k, a.h);
        }
    }
}

// ------------------------------------------------------------------ launcher

static size_t bwd_lds_bytes(int C, int k, int kpad, bool sparse, bool ranked, int nb) {
    size_t b = (size_t)nb * (4 * sizeof(float4) + sizeof(uint32_t) + kpad);
    // the top-k values (not kept by the ranked kernel), or the class rank
    // tables: four (mask word, classes below) pairs and the position nibbles
    b += ranked ? (size_t)nb * 5 * sizeof(uint2) : (size_t)nb * k * sizeof(float);
    b += (size_t)kBwdWaves * nb * (10 + k) * sizeof(float) + kBwdWaves * nb * sizeof(uint32_t);
    b += (size_t)nb * sizeof(uint32_t);  // the list of blended keys
    if (!sparse) b += (size_t)acc_floats(C) * sizeof(float);
    return b;
}

template <typename K>
static void set_lds_b(K kernel, size_t bytes) {
    if (bytes > 65536)
        (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int KT, bool SPARSE, bool RANKED = false, int NB = kBwdBatch>
static void bwd_launch_nb(const BwdArgs& b, unsigned grid, size_t lds, hipStream_t st) {
    set_lds_b(render_bwd_kernel<KT, SPARSE, RANKED, NB>, lds);
    render_bwd_kernel<KT, SPARSE, RANKED, NB><<<grid, kBwdThreads, lds, st>>>(b);
}

// The staging batch is a speed choice (cfg.bwd_batch): 32, 44 (the default)
// or 56 keys, trading LDS per workgroup (workgroups per CU) against barriers
// per key.  Only the common k = 16 kernels carry the three sizes.
template <int KT, bool SPARSE, bool RANKED = false>
static void bwd_launch(const BwdArgs& b, unsigned grid, size_t lds, int nb, hipStream_t st) {
    if constexpr (KT == 16) {
        if (nb == 32) return bwd_launch_nb<KT, SPARSE, RANKED, 32>(b, grid, lds, st);
        if (nb == 56) return bwd_launch_nb<KT, SPARSE, RANKED, 56>(b, grid, lds, st);
    }
    bwd_launch_nb<KT, SPARSE, RANKED, kBwdBatch>(b, grid, lds, st);
}

sgr_status launch_backward_tiles(const Plan& P, const sgr_map_grads* dL, char* ws, hipStream_t st) {
    BwdArgs b;
    memset(&b, 0, sizeof(b));
    b.t = make_tile_args(P, ws);
    std::vector<GradPtrs> gpt(P.V);
    bool sparse = true;  // no view carries a dense semantic gradient
    for (int v = 0; v < P.V; v++) {
        gpt[v] = GradPtrs{dL[v].rgb, dL[v].depth, dL[v].sil, dL[v].sem, dL[v].sem_label, dL[v].sem_at_label};
        sparse &= dL[v].sem == nullptr;
    }
    set_view_table(b.grads, gpt, ws + P.grad_table, st);
    b.slots = (float*)(ws + P.slots);
    b.touched = (uint8_t*)(ws + P.touched);
    b.svals = (const uint32_t*)(ws + P.sorted_vals);
    b.nvals = 10 + P.k;
    b.semgeo = P.cfg.sem_grad_to_geometry;
    // one-class semantic gradient kept off geometry, k = 16, C <= 128: the
    // label's list position comes from the class rank tables
    const bool ranked = sparse && P.ranked && !b.semgeo;
    const int nb = (P.k == 16 && P.cfg.bwd_batch > 0) ? P.cfg.bwd_batch : kBwdBatch;
    const size_t lds = bwd_lds_bytes(P.C, P.k, P.kpad, sparse, ranked, nb);
    if (lds > device_max_lds()) return SGR_EUNSUPPORTED;
    const unsigned grid = (unsigned)(div_up(P.num_tiles, 8) * 8);
    if (P.k == 16) {
        if (ranked) bwd_launch<16, true, true>(b, grid, lds, nb, st);
        else if (sparse) bwd_launch<16, true>(b, grid, lds, nb, st);
        else bwd_launch<16, false>(b, grid, lds, nb, st);
    } else if (P.k == 3) {
        if (sparse) bwd_launch<3, true>(b, grid, lds, nb, st); else bwd_launch<3, false>(b, grid, lds, nb, st);
    } else {
        if (sparse) bwd_launch<0, true>(b, grid, lds, nb, st); else bwd_launch<0, false>(b, grid, lds, nb, st);
    }
    return hipGetLastError() == hipSuccess ? SGR_OK : SGR_EHIP;
}

sgr_status launch_backward_gather(const Plan& P, const sgr_gaussians* g, const sgr_grads* out, char* ws,
                                  hipStream_t st, const sgr_adam_segment* adam, const AdamParams* hp) {
    const uint32_t* counters = (const uint32_t*)(ws + P.counters);
    const int nvals = 10 + P.k;
    const unsigned ggrid = (unsigned)div_up(P.vn, 256);
    if (ggrid > 0) {
        const float* slots = (const float*)(ws + P.slots);
        const uint8_t* touched = (const uint8_t*)(ws + P.touched);
        const uint32_t* toff = (const uint32_t*)(ws + P.toff);
        const uint32_t* tcount = (const uint32_t*)(ws + P.tcount);
        float* g2d = (float*)(ws + P.g2d);
        const uint32_t* order = (const uint32_t*)(ws + P.order);
        if (P.k == 16) gather_slots<16><<<ggrid, 256, 0, st>>>(slots, touched, toff, tcount, order, counters, nvals, g2d);
        else if (P.k == 3) gather_slots<3><<<ggrid, 256, 0, st>>>(slots, touched, toff, tcount, order, counters, nvals, g2d);
        else gather_slots<0><<<ggrid, 256, 0, st>>>(slots, touched, toff, tcount, order, counters, nvals, g2d);
    }
    ProjBwdArgs pa;
    pa.means = g->means; pa.scales = g->scales; pa.quats = g->quats; pa.opacity = g->opacity;
    pa.views = (const ViewDev*)(ws + P.views);
    pa.n = P.n; pa.V = P.V; pa.k = P.k; pa.NV = nvals; pa.C = P.C;
    pa.lowpass = P.cfg.lowpass;
    pa.gp_of_lin = (const uint32_t*)(ws + P.gp_of_lin);
    pa.g2d = (const float*)(ws + P.g2d);
    pa.sorig = (const uint8_t*)(ws + P.sorig);
    pa.kpad = P.kpad;
    memset(pa.seg, 0, sizeof(pa.seg));
    pa.h = hp ? *hp : AdamParams{};
    if (adam)
        for (int s = 0; s < 6; s++) pa.seg[s] = adam[s];
    pa.counters = counters;
    pa.d_means = out ? out->means : nullptr; pa.d_scales = out ? out->scales : nullptr;
    pa.d_quats = out ? out->quats : nullptr; pa.d_opacity = out ? out->opacity : nullptr;
    pa.d_rgb = out ? out->rgb : nullptr; pa.d_sem = out ? out->sem_val : nullptr;
    const unsigned pgrid = (unsigned)div_up(P.n, 256);
    if (pgrid > 0) {
        if (adam) {
            if (P.k == 16) project_backward_kernel<16, true><<<pgrid, 256, 0, st>>>(pa);
            else if (P.k == 3) project_backward_kernel<3, true><<<pgrid, 256, 0, st>>>(pa);
            else project_backward_kernel<0, true><<<pgrid, 256, 0, st>>>(pa);
        } else {
            if (P.k == 16) project_backward_kernel<16, false><<<pgrid, 256, 0, st>>>(pa);
            else if (P.k == 3) project_backward_kernel<3, false><<<pgrid, 256, 0, st>>>(pa);
            else project_backward_kernel<0, false><<<pgrid, 256, 0, st>>>(pa);
        }
    }
    return hipGetLastError() == hipSuccess ? SGR_OK : SGR_EHIP;
}

}  // namespace sgr
