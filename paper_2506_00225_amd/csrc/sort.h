// Scan and radix-sort launchers (device code in sort.hip).
#pragma once

#include <algorithm>

#include "sgr_internal.h"

namespace sgr {

constexpr int kScanItems = 8;
constexpr int kScanTile = 256 * kScanItems;
// Blocks of the radix sorts.  Small sorts (up to kRadixFewBlocks blocks of
// kRadixTileSmall items) form each scatter workgroup's digit offsets from
// the raw per-block counts instead of a scan; the others scan the counts,
// with blocks of kRadixTileMid items up to kRadixMidMax items and of
// kRadixTile beyond (fewer, longer blocks keep the count tables and their
// scans small for sorts of tens of millions of keys).
constexpr int kRadixItems = 16;
constexpr int kRadixTile = 256 * kRadixItems;
constexpr int kRadixItemsMid = 8;
constexpr int kRadixTileMid = 256 * kRadixItemsMid;
constexpr uint32_t kRadixMidMax = 1u << 23;
constexpr int kRadixItemsSmall = 8;
constexpr int kRadixTileSmall = 256 * kRadixItemsSmall;
constexpr uint32_t kRadixFewBlocks = 512;

// Element count of a scan or sort: *d_n if d_n is set (device-resident,
// known only on the GPU), else host_n; clamped to cap when cap != 0.
// radix_blocks: if set, the count is radix_blocks digit bins times the number
// of radix blocks of radix_tile items that n makes.
struct CountSpec {
    const uint32_t* d_n;
    uint32_t host_n;
    uint32_t cap;
    uint32_t radix_blocks;
    uint32_t radix_tile;
};

inline CountSpec host_count(uint32_t n) { return CountSpec{nullptr, n, 0, 0, 0}; }
inline CountSpec device_count(const uint32_t* d, uint32_t cap) { return CountSpec{d, 0, cap, 0, 0}; }

// Items per radix block of a sort of at most max_n items.
inline uint32_t radix_block_items(uint32_t max_n) {
    if (div_up(max_n, kRadixTileSmall) <= (int64_t)kRadixFewBlocks) return kRadixTileSmall;
    return max_n <= kRadixMidMax ? kRadixTileMid : kRadixTile;
}

// Exclusive scan of in[0..n) into out (may alias in).  max_n bounds n and
// sizes the grid; partial needs div_up(max_n, kScanTile) words.  The total
// goes to *total_out (if set); total > cap sets SGR_ECAPACITY in *status.
// With heads set, heads[q] receives the item whose run [out[i], out[i] +
// in[i]) holds position q * chunk, for every such position below cap.
void scan_exclusive(const uint32_t* in, uint32_t* out, CountSpec cs, uint32_t max_n, uint32_t* partial,
                    uint32_t* total_out, uint32_t cap, uint32_t* status, hipStream_t st,
                    uint32_t* heads = nullptr, uint32_t chunk = 0);

// Passes of a radix sort of `bits` key bits with digits of at most
// max_digit (<= 8) bits.
inline int radix_passes(int bits, int max_digit) { return (bits + max_digit - 1) / max_digit; }

// Stable LSD radix sort of (key, value) pairs on the low `bits` key bits,
// at most max_digit (<= 8) bits per pass (spread evenly), ping-ponging
// between the a and b buffers.  Returns the pass count
// (radix_passes(bits, max_digit)): the result is in the a buffers when it is
// even, else in b.  vals_identity: the a values are not read; value i is
// taken to be i.  With carry_dst set, carry_dst[i] = carry_src[sorted value
// i] (written by the last pass).  With hist0_ready, the producer of the keys
// has already written the first pass's counts into hist (the layout of
// radix_first_pass), and that pass's histogram launch is skipped.
int radix_sort(uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b, uint32_t* vals_b, bool vals_identity,
               CountSpec cs, uint32_t max_n, int bits, uint32_t* hist, uint32_t* partial, hipStream_t st,
               int max_digit = 8, const uint32_t* carry_src = nullptr, uint32_t* carry_dst = nullptr,
               bool hist0_ready = false);

// The first pass's counts as radix_sort expects them, for a producer that
// writes them itself: per block of `tile` keys (the key count clamped to the
// sort's, as CountSpec gives it), the counts of key & (bins - 1);
// block-major (hist[b * bins + d]) when the sort takes few blocks, else
// digit-major (hist[d * nblk + b], nblk the blocks of the clamped count).
struct RadixFirstPass {
    uint32_t bins;
    int block_major;
    uint32_t tile;
};
inline RadixFirstPass radix_first_pass(uint32_t max_n, int bits, int max_digit) {
    const int passes = radix_passes(bits, max_digit);
    const int dbits = passes > 0 ? (bits + passes - 1) / passes : 8;
    return RadixFirstPass{1u << dbits, div_up(max_n, kRadixTileSmall) <= (int64_t)kRadixFewBlocks ? 1 : 0,
                          radix_block_items(max_n)};
}

inline size_t radix_hist_words(uint32_t max_n) {
    return 256u * (size_t)div_up(max_n, std::min(kRadixTileSmall, kRadixTileMid));
}
inline size_t scan_partial_words(size_t max_n) { return (size_t)div_up((int64_t)max_n, kScanTile) + 1; }

}  // namespace sgr
