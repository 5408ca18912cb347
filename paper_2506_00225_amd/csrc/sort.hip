// Prefix scans and the stable LSD radix sort used for depth ordering and
// tile binning.  Reduce-then-scan everywhere: no kernel waits on another
// workgroup, so nothing here can spin.
#include "sort.h"

namespace sgr {

__device__ __forceinline__ uint32_t count_of(const CountSpec& c) {
    uint32_t n = c.d_n ? *c.d_n : c.host_n;
    if (c.cap && n > c.cap) n = c.cap;
    if (c.radix_blocks) n = c.radix_blocks * (uint32_t)div_up(n, c.radix_tile);
    return n;
}

// Block-wide exclusive scan of one value per thread (256 threads).
__device__ __forceinline__ uint32_t block_exscan(uint32_t v, uint32_t* wsum, uint32_t* total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const uint32_t s = wsum[j];
        pre += (j < w) ? s : 0u;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return pre + x - v;
}

__global__ __launch_bounds__(256) void scan_block_sums(const uint32_t* __restrict__ in, CountSpec cs,
                                                       uint32_t* __restrict__ partial) {
    __shared__ uint32_t wsum[4];
    const uint32_t n = count_of(cs);
    const uint32_t nblk = (uint32_t)div_up(n, kScanTile);
    if (blockIdx.x >= nblk) return;
    const uint32_t base = blockIdx.x * kScanTile;
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < kScanItems; r++) {
        const uint32_t i = base + r * 256 + threadIdx.x;
        if (i < n) s += in[i];
    }
    uint32_t tot;
    block_exscan(s, wsum, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// Exclusive scan of `in` into `out` (may alias) from the block sums: each
// workgroup adds up the sums of the blocks before it (integers, so the
// order does not matter), which saves a separate scan of the sums.  The last
// block writes the total (and the saturating capacity check).  With `heads`
// set, the scan is of per-item run lengths, and for every chunk of `chunk`
// positions below `cap` the item whose run holds the chunk's first position
// is recorded in heads[chunk index].
__global__ __launch_bounds__(256) void scan_apply(const uint32_t* in, CountSpec cs,
                                                  const uint32_t* __restrict__ partial, uint32_t* out,
                                                  uint32_t* __restrict__ total_out, uint32_t cap,
                                                  uint32_t* __restrict__ status, uint32_t* __restrict__ heads,
                                                  uint32_t chunk) {
    __shared__ uint32_t wsum[4];
    const uint32_t n = count_of(cs);
    const uint32_t nblk = (uint32_t)div_up(n, kScanTile);
    if (blockIdx.x >= nblk) {
        if (nblk == 0 && blockIdx.x == 0 && threadIdx.x == 0 && total_out) *total_out = 0;  // empty input
        return;
    }
    uint32_t before = 0;
    for (uint32_t i = threadIdx.x; i < blockIdx.x; i += 256) before += partial[i];
    uint32_t prefix;
    block_exscan(before, wsum, &prefix);
    const uint32_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    uint32_t v[kScanItems], s = 0;
#pragma unroll
    for (int r = 0; r < kScanItems; r++) {
        const uint32_t i = base + r;
        v[r] = i < n ? in[i] : 0u;
        s += v[r];
    }
    uint32_t tot;
    uint32_t pre = block_exscan(s, wsum, &tot) + prefix;
#pragma unroll
    for (int r = 0; r < kScanItems; r++) {
        const uint32_t i = base + r;
        if (i < n) {
            out[i] = pre;
            if (heads && v[r] > 0u && pre < cap) {
                const uint64_t last = min((uint64_t)pre + v[r], (uint64_t)cap) - 1;
                for (uint64_t q = ((uint64_t)pre + chunk - 1) / chunk; q * chunk <= last; q++) heads[q] = i;
            }
        }
        pre += v[r];
    }
    if (blockIdx.x == nblk - 1 && threadIdx.x == 0) {
        const uint32_t total = prefix + tot;
        if (total_out) *total_out = total;
        if (status && total > cap) atomicOr(status, (uint32_t)SGR_ECAPACITY);
    }
}

// Note: scan_block_sums reads items strided by 256 while scan_apply reads
// kScanItems consecutive items per thread; both cover the same kScanTile
// items per block, which is all the block sums need.

void scan_exclusive(const uint32_t* in, uint32_t* out, CountSpec cs, uint32_t max_n, uint32_t* partial,
                    uint32_t* total_out, uint32_t cap, uint32_t* status, hipStream_t st, uint32_t* heads,
                    uint32_t chunk) {
    const uint32_t nblk_max = (uint32_t)div_up(max_n, kScanTile);
    if (nblk_max == 0) return;
    scan_block_sums<<<nblk_max, 256, 0, st>>>(in, cs, partial);
    scan_apply<<<nblk_max, 256, 0, st>>>(in, cs, partial, out, total_out, cap, status, heads, chunk);
}

// ------------------------------------------------------------------ radix

// Per-block counts of the digit (key >> shift) & (2^dbits - 1): digit-major
// (hist[d * nblk + b], the order of the scan over them) or, BLOCK_MAJOR,
// hist[b * 2^dbits + d].
// DBITS: the digit width if fixed at compile time (8), else 0 and dbits.
template <bool BLOCK_MAJOR, int ITEMS, int DBITS>
__global__ __launch_bounds__(256) void radix_hist(const uint32_t* __restrict__ keys, CountSpec cs, int shift,
                                                  int dbits_rt, uint32_t* __restrict__ hist) {
    const int dbits = DBITS > 0 ? DBITS : dbits_rt;
    constexpr uint32_t TILE = 256u * ITEMS;
    __shared__ uint32_t cnt[256];
    const uint32_t n = count_of(cs);
    const uint32_t nblk = (uint32_t)div_up(n, TILE);
    if (blockIdx.x >= nblk) return;
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * TILE;
    uint32_t kr[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; r++) {
        const uint32_t i = base + r * 256 + threadIdx.x;
        kr[r] = i < n ? keys[i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < ITEMS; r++) {
        const uint32_t i = base + r * 256 + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(kr[r] >> shift) & ((1u << dbits) - 1u)], 1u);
    }
    __syncthreads();
    const uint32_t bins = 1u << dbits;
    if (DBITS == 8 || threadIdx.x < bins) {  // (every thread when the digit has 8 bits)
        if (BLOCK_MAJOR) hist[blockIdx.x * bins + threadIdx.x] = cnt[threadIdx.x];
        else hist[threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
    }
}

// Stable scatter of one digit of at most 8 bits.  Items are taken in index order, 256
// per round; within a wave the rank among equal digits comes from eight
// ballots, across the four waves from per-digit wave counts in LDS.
// SCANNED: hist holds the exclusive scan over (digit, block).  Otherwise it
// holds the raw counts, block-major, and each workgroup forms its own starting offsets:
// the counts of its digit in earlier blocks plus, over all blocks, the counts
// of smaller digits (used when there are few blocks; it saves three scan
// launches per pass).  With cdst set, cdst[out position] = csrc[value]
// (a value-indexed array carried into sorted order).
template <bool SCANNED, int ITEMS, int DBITS>
__global__ __launch_bounds__(256) void radix_scatter(const uint32_t* __restrict__ kin,
                                                     const uint32_t* __restrict__ vin,
                                                     uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                     CountSpec cs, int shift, int dbits_rt,
                                                     const uint32_t* __restrict__ hist,
                                                     const uint32_t* __restrict__ csrc, uint32_t* __restrict__ cdst) {
    const int dbits = DBITS > 0 ? DBITS : dbits_rt;
    constexpr uint32_t TILE = 256u * ITEMS;
    __shared__ uint32_t run[256];
    __shared__ uint32_t wc[4][256];
    const uint32_t n = count_of(cs);
    const uint32_t nblk = (uint32_t)div_up(n, TILE);
    if (blockIdx.x >= nblk) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t bins = 1u << dbits, mask = bins - 1u;
    const bool has_bin = DBITS == 8 || (uint32_t)tid < bins;  // thread tid owns digit tid
    if constexpr (SCANNED) {
        run[tid] = has_bin ? hist[tid * nblk + blockIdx.x] : 0u;
    } else {
        uint32_t before = 0, all = 0;
#pragma unroll 32
        for (uint32_t b = 0; b < nblk; b++) {  // coalesced: the digits of block b are adjacent
            const uint32_t c = has_bin ? hist[b * bins + tid] : 0u;
            all += c;
            before += b < blockIdx.x ? c : 0u;
        }
        uint32_t tot;
        run[tid] = block_exscan(all, wc[0], &tot) + before;  // wc[0] as scratch, cleared below
    }
#pragma unroll
    for (int j = 0; j < 4; j++) wc[j][tid] = 0;
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint32_t base = blockIdx.x * TILE;
    // Every round's items are loaded up front, so the rounds (each ends at
    // a barrier) do not each wait out a global load.  (With 16 items a
    // thread this costs one or two waves per SIMD, and still measured
    // faster.)
    uint32_t kr[ITEMS], vr[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; r++) {
        const uint32_t i = base + r * 256 + tid;
        kr[r] = i < n ? kin[i] : 0u;
        vr[r] = i < n ? (vin ? vin[i] : i) : 0u;
    }
#pragma unroll
    for (int r = 0; r < ITEMS; r++) {
        const uint32_t i = base + r * 256 + tid;
        const bool valid = i < n;
        const uint32_t key = kr[r];
        const uint32_t val = vr[r];
        const uint32_t d = (key >> shift) & mask;
        uint64_t match = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            if (b < dbits) {
                const bool bit = (d >> b) & 1u;
                const uint64_t bb = __ballot(bit);
                match &= bit ? bb : ~bb;
            }
        }
        const uint32_t rank = __popcll(match & lt);
        if (valid && rank == 0) wc[w][d] = __popcll(match);
        __syncthreads();
        if (valid) {
            uint32_t off = run[d] + rank;
            for (int j = 0; j < w; j++) off += wc[j][d];
            kout[off] = key;
            vout[off] = val;
            if (cdst) cdst[off] = csrc[val];
        }
        __syncthreads();
        run[tid] += wc[0][tid] + wc[1][tid] + wc[2][tid] + wc[3][tid];
        wc[0][tid] = 0; wc[1][tid] = 0; wc[2][tid] = 0; wc[3][tid] = 0;
        __syncthreads();
    }
}

int radix_sort(uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b, uint32_t* vals_b, bool vals_identity,
               CountSpec cs, uint32_t max_n, int bits, uint32_t* hist, uint32_t* partial, hipStream_t st,
               int max_digit, const uint32_t* carry_src, uint32_t* carry_dst, bool hist0_ready) {
    const uint32_t tile = radix_block_items(max_n);
    const bool mid = tile == (uint32_t)kRadixTileMid;  // (the small path's tile may be the same size)
    const uint32_t nblk_max = (uint32_t)div_up(max_n, tile);
    if (nblk_max == 0) return 0;
    // few: small tiles (more workgroups for a small sort) and offsets formed in the scatter
    const uint32_t nblk_small = (uint32_t)div_up(max_n, kRadixTileSmall);
    // passes of at most max_digit bits, the bits spread evenly (12 bits in
    // 8-bit digits: two 6-bit digits, whose 64 buckets keep the scatter's
    // writes in longer runs)
    const int passes = radix_passes(bits, max_digit);
    const int dbits = passes > 0 ? (bits + passes - 1) / passes : 8;
    const uint32_t bins = 1u << dbits;
    uint32_t *ki = keys_a, *vi = vals_a, *ko = keys_b, *vo = vals_b;
    CountSpec hs = cs;
    hs.radix_blocks = bins;
    hs.radix_tile = tile;
    const bool few = nblk_small <= kRadixFewBlocks;
    for (int p = 0; p < passes; p++) {
        const uint32_t* vin = (p == 0 && vals_identity) ? nullptr : vi;
        const int sh = dbits * p;
        const bool lastp = p == passes - 1;
        const uint32_t* cs_ = lastp ? carry_src : nullptr;
        uint32_t* cd_ = lastp ? carry_dst : nullptr;
        const bool counted = p == 0 && hist0_ready;  // the producer wrote this pass's counts
        if (few) {
            if (dbits == 8) {
                if (!counted) radix_hist<true, kRadixItemsSmall, 8><<<nblk_small, 256, 0, st>>>(ki, cs, sh, 8, hist);
                radix_scatter<false, kRadixItemsSmall, 8>
                    <<<nblk_small, 256, 0, st>>>(ki, vin, ko, vo, cs, sh, 8, hist, cs_, cd_);
            } else {
                if (!counted)
                    radix_hist<true, kRadixItemsSmall, 0><<<nblk_small, 256, 0, st>>>(ki, cs, sh, dbits, hist);
                radix_scatter<false, kRadixItemsSmall, 0>
                    <<<nblk_small, 256, 0, st>>>(ki, vin, ko, vo, cs, sh, dbits, hist, cs_, cd_);
            }
        } else {
            if (!counted) {
                if (mid) {
                    if (dbits == 8) radix_hist<false, kRadixItemsMid, 8><<<nblk_max, 256, 0, st>>>(ki, cs, sh, 8, hist);
                    else radix_hist<false, kRadixItemsMid, 0><<<nblk_max, 256, 0, st>>>(ki, cs, sh, dbits, hist);
                } else {
                    if (dbits == 8) radix_hist<false, kRadixItems, 8><<<nblk_max, 256, 0, st>>>(ki, cs, sh, 8, hist);
                    else radix_hist<false, kRadixItems, 0><<<nblk_max, 256, 0, st>>>(ki, cs, sh, dbits, hist);
                }
            }
            scan_exclusive(hist, hist, hs, bins * nblk_max, partial, nullptr, 0, nullptr, st);
            if (mid) {
                if (dbits == 8)
                    radix_scatter<true, kRadixItemsMid, 8>
                        <<<nblk_max, 256, 0, st>>>(ki, vin, ko, vo, cs, sh, 8, hist, cs_, cd_);
                else
                    radix_scatter<true, kRadixItemsMid, 0>
                        <<<nblk_max, 256, 0, st>>>(ki, vin, ko, vo, cs, sh, dbits, hist, cs_, cd_);
            } else {
                if (dbits == 8)
                    radix_scatter<true, kRadixItems, 8>
                        <<<nblk_max, 256, 0, st>>>(ki, vin, ko, vo, cs, sh, 8, hist, cs_, cd_);
                else
                    radix_scatter<true, kRadixItems, 0>
                        <<<nblk_max, 256, 0, st>>>(ki, vin, ko, vo, cs, sh, dbits, hist, cs_, cd_);
            }
        }
        uint32_t* t;
        t = ki; ki = ko; ko = t;
        t = vi; vi = vo; vo = t;
    }
    return passes;
}

}  // namespace sgr
