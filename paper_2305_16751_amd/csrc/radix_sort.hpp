// Stable LSD radix sort of (key, u32 payload) pairs, one kernel launch per
// 8-bit digit ("onesweep": the digit offsets of every tile come from a
// decoupled look-back over the tiles before it, so each pass reads and writes
// the data once).  The per-digit histograms of every pass are computed up
// front, fused into the kernel that produces the keys.
//
// This realises the sorts of the paper's algorithm (Sec. 4: the per-axis
// sorts of coordinates and the sort of the expanded list; Sec. 5: its order).
// Stability is what carries the secondary orders: a list emitted in
// (last coordinate, queries first, ID) order and stably sorted by the
// bitstring tuple ends up in the Sec. 5 order.
#pragma once

#include "device_common.hpp"

namespace domagg {

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kMaxPasses = 8;  // 64-bit keys


// ---------------------------------------------------------------------------
// Fused histogram: add the digits of `key` for passes [0, passes) to the
// LDS histogram s_hist[passes][256].  All lanes of the wavefront must call
// it together; lanes with valid = false contribute nothing.  From pass
// peel_from on, lanes sharing the first valid lane's digit are added with
// one atomic (skewed digits, such as the high digits of the tree-node keys,
// would otherwise serialise on one LDS address).
// rb: the digit width (<= 8; rows stay 256 bins wide).
template <class K>
__device__ __forceinline__ void hist_add(uint32_t *s_hist, K key, bool valid, int passes,
                                         int peel_from = 0, int rb = kRadixBits) {
    const uint64_t act = __ballot(valid);
    if (act == 0) return;
    const int leader = __ffsll((unsigned long long)act) - 1;
    const int lane = lane_id();
    const uint32_t dmask = (1u << rb) - 1u;
    for (int p = 0; p < passes; ++p) {
        const uint32_t d = (uint32_t)(key >> (rb * p)) & dmask;
        if (p < peel_from) {  // digits known to be spread: one LDS atomic per lane
            if (valid) atomicAdd(&s_hist[p * kRadix + d], 1u);
            continue;
        }
        const uint32_t d0 = read_lane_u32(d, leader);
        const uint64_t same = __ballot(valid && d == d0);
        if (lane == leader) atomicAdd(&s_hist[p * kRadix + d0], (uint32_t)__popcll(same));
        if (valid && d != d0) atomicAdd(&s_hist[p * kRadix + d], 1u);
    }
}

// Writes the block's LDS histogram to part[blockIdx.x][passes * 256].
__device__ __forceinline__ void hist_flush(const uint32_t *s_hist, uint32_t *part, int passes) {
    for (int i = threadIdx.x; i < passes * kRadix; i += blockDim.x)
        part[(size_t)blockIdx.x * passes * kRadix + i] = s_hist[i];
}

// Exclusive sum over a block of BLOCK threads; *total gets the block sum.
template <int BLOCK>
__device__ __forceinline__ uint32_t block_excl_sum(uint32_t v, uint32_t *s_tmp, uint32_t *total) {
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    const uint32_t incl = wave_sum_scan_incl(v);
    if (lane == kWave - 1) s_tmp[wave] = incl;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < BLOCK / kWave; ++w) {
        const uint32_t t = s_tmp[w];
        pre += (w < wave) ? t : 0u;
        tot += t;
    }
    __syncthreads();
    if (total) *total = tot;
    return pre + incl - v;
}

// First stage of the histogram reduction: block (p, c) sums rows
// [c*rows, (c+1)*rows) of part[nblocks][passes][256] into part2[c][passes][256].
__global__ __launch_bounds__(kRadix) void hist_partial_kernel(const uint32_t *__restrict__ part,
                                                              int nblocks, int passes, int rows,
                                                              uint32_t *__restrict__ part2) {
    const int p = blockIdx.x, c = blockIdx.y, d = threadIdx.x;
    const int b0 = c * rows, b1 = min(nblocks, b0 + rows);
    uint32_t sum = 0;
    for (int b = b0; b < b1; ++b) sum += part[((size_t)b * passes + p) * kRadix + d];
    part2[((size_t)c * passes + p) * kRadix + d] = sum;
}

// One block per pass: sums the per-block partial histograms and scans them
// into exclusive digit bases.  counts/bases are [passes][256].
__global__ __launch_bounds__(kRadix) void hist_reduce_kernel(const uint32_t *__restrict__ part,
                                                             int nblocks, int passes,
                                                             uint32_t *__restrict__ counts,
                                                             uint32_t *__restrict__ bases) {
    __shared__ uint32_t s_tmp[kRadix / kWave];
    const int p = blockIdx.x, d = threadIdx.x;
    uint32_t sum = 0;
    for (int b = 0; b < nblocks; ++b) sum += part[((size_t)b * passes + p) * kRadix + d];
    const uint32_t ex = block_excl_sum<kRadix>(sum, s_tmp, nullptr);
    counts[p * kRadix + d] = sum;
    bases[p * kRadix + d] = ex;
}

// Standalone histogram of an existing key array (used when the producer
// could not fuse it).
template <class K, int BLOCK>
__global__ __launch_bounds__(BLOCK) void hist_kernel(const K *__restrict__ keys, uint64_t n,
                                                     int passes, uint32_t *__restrict__ part) {
    __shared__ uint32_t s_hist[kMaxPasses * kRadix];
    for (int i = threadIdx.x; i < passes * kRadix; i += BLOCK) s_hist[i] = 0;
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * BLOCK;
    for (uint64_t base = (uint64_t)blockIdx.x * BLOCK; base < n; base += stride) {
        const uint64_t i = base + threadIdx.x;
        const bool valid = i < n;
        const K k = valid ? keys[i] : K(0);
        hist_add(s_hist, k, valid, passes);
    }
    __syncthreads();
    hist_flush(s_hist, part, passes);
}

// ---------------------------------------------------------------------------
// Look-back words of the digit passes: the flag in the top two bits, the
// count below.  32-bit words when every count fits in 30 bits (n < 2^30),
// else 64-bit.
template <class S>
struct DigitWord {
    static constexpr int kShift = sizeof(S) * 8 - 2;
    static constexpr S kMask = (S(1) << kShift) - 1;
    __device__ static S make(uint32_t flag, uint64_t count) { return (S(flag) << kShift) | S(count); }
    __device__ static uint32_t flag(S w) { return (uint32_t)(w >> kShift); }
    __device__ static uint32_t count(S w) { return (uint32_t)(w & kMask); }
};

// ---------------------------------------------------------------------------
// One digit pass.  A workgroup takes the next tile from a ticket counter (so
// every tile it waits on belongs to a workgroup that is already running),
// ranks its keys by digit within each wavefront (ballot matching, stable in
// index order), publishes its per-digit counts, looks back over earlier tiles
// for the per-digit offsets (one thread per digit), stages keys and then
// payloads in LDS in local digit order and writes them out in runs.
//
// n < 2^32 - 2*TILE.  status: [tiles][256] words of type S, zero before the
// launch; ticket: zero before the launch.  digit_base: [256] exclusive bases
// of the pass's digits over the whole array.  ROLE only names the
// instantiation (0: per-point coordinate sorts, 1: the sort of the expanded
// records) so the two show up separately in profiles.  VT: the payload type
// (u32, or u64 for the last-axis sort that carries each point's rank).
// HAS_VAL = false: keys only (a record packed into one word: its digits sit
// at `shift` within the word), vin / vout unused.  RBITS: the digit width
// (status words and digit bases are [2^RBITS] per tile / pass).
template <class K, class S, int BLOCK, int ITEMS, int ROLE = 0, class VT = uint32_t, bool HAS_VAL = true,
          int RBITS = kRadixBits>
__global__ __launch_bounds__(BLOCK) void onesweep_kernel(
    const K *__restrict__ kin, const VT *__restrict__ vin, K *__restrict__ kout,
    VT *__restrict__ vout, uint32_t n, int shift, const uint32_t *__restrict__ digit_base,
    S *__restrict__ status, uint32_t *__restrict__ ticket) {
    constexpr int TILE = BLOCK * ITEMS;
    constexpr int WAVES = BLOCK / kWave;
    constexpr int RADIX = 1 << RBITS;
    using W = DigitWord<S>;
    static_assert(BLOCK >= RADIX, "one thread per digit");
    static_assert(RBITS >= 4 && RBITS <= 10, "");
    static_assert(ITEMS <= 32, "");

    __shared__ union {
        K keys[TILE];
        VT vals[TILE];
    } s_stage;
    __shared__ uint32_t s_whist[WAVES][RADIX];  // counts, then exclusive over waves
    __shared__ uint32_t s_dstart[RADIX];        // tile-local start of each digit
    __shared__ uint32_t s_goff[RADIX];          // global start minus local start
    __shared__ uint32_t s_tmp[WAVES];
    __shared__ uint32_t s_tile;

    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    for (int i = tid; i < WAVES * RADIX; i += BLOCK) (&s_whist[0][0])[i] = 0;
    if (tid == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint64_t wbase = (uint64_t)tile * TILE + (uint64_t)wave * kWave * ITEMS;

    // Wave-striped loads: item i of lane l is element wbase + 64 i + l, so
    // ranking items in order i keeps index order within the wavefront.
    K key[ITEMS];
    VT val[ITEMS];
    uint32_t loc[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint64_t idx = wbase + (uint64_t)i * kWave + lane;
        if (idx < n) {
            key[i] = kin[idx];
            if constexpr (HAS_VAL) val[i] = vin[idx];
        } else {
            key[i] = ~K(0);  // the largest digit at every shift: sorts after all real keys of the tile
            val[i] = VT(0);
        }
    }

    const uint64_t below_mask = lanemask_lt();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t d = (uint32_t)(key[i] >> shift) & (RADIX - 1);
        const uint64_t peers = match_digit<RBITS>(d);
        const uint32_t below = (uint32_t)__popcll(peers & below_mask);
        const uint32_t cnt = s_whist[wave][d];
        loc[i] = cnt + below;
        if (below == 0) s_whist[wave][d] = cnt + (uint32_t)__popcll(peers);
    }
    __syncthreads();

    uint32_t count = 0;
    if (tid < RADIX) {
#pragma unroll
        for (int w = 0; w < WAVES; ++w) {
            const uint32_t c = s_whist[w][tid];
            s_whist[w][tid] = count;
            count += c;
        }
        store_agent(&status[(uint64_t)tile * RADIX + tid],
                    W::make(tile == 0 ? kFlagInclusive : kFlagAggregate, count));
    }
    const uint32_t dstart = block_excl_sum<BLOCK>(tid < RADIX ? count : 0u, s_tmp, nullptr);
    if (tid < RADIX) {
        s_dstart[tid] = dstart;
        uint32_t excl = 0;
        if (tile > 0) {
            // Walk back over earlier tiles, four words per round trip (the
            // loads are issued together; a word not yet published is polled
            // on its own), until an inclusive word; tile 0's always is.
            constexpr int kDepth = 4;
            int64_t t = (int64_t)tile - 1;
            bool done = false;
            while (!done) {
                S w[kDepth];
#pragma unroll
                for (int k = 0; k < kDepth; ++k)
                    w[k] = (t - k >= 0) ? load_agent(&status[(uint64_t)(t - k) * RADIX + tid]) : S(0);
#pragma unroll
                for (int k = 0; k < kDepth; ++k) {
                    if (done || t - k < 0) continue;
                    while (W::flag(w[k]) == 0) {
                        __builtin_amdgcn_s_sleep(2);
                        w[k] = load_agent(&status[(uint64_t)(t - k) * RADIX + tid]);
                    }
                    excl += W::count(w[k]);
                    done = W::flag(w[k]) == kFlagInclusive;
                }
                t -= kDepth;
            }
            store_agent(&status[(uint64_t)tile * RADIX + tid], W::make(kFlagInclusive, excl + count));
        }
        s_goff[tid] = digit_base[tid] + excl - dstart;
    }
    __syncthreads();

#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t d = (uint32_t)(key[i] >> shift) & (RADIX - 1);
        const uint32_t lp = s_dstart[d] + s_whist[wave][d] + loc[i];
        s_stage.keys[lp] = key[i];
        loc[i] = lp;
    }
    __syncthreads();

    uint32_t gpos[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t p = (uint32_t)(i * BLOCK + tid);
        const K k = s_stage.keys[p];
        const uint32_t d = (uint32_t)(k >> shift) & (RADIX - 1);
        const uint32_t g = s_goff[d] + p;
        gpos[i] = g;
        if (g < n) kout[g] = k;
    }
    if constexpr (HAS_VAL) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) s_stage.vals[loc[i]] = val[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t p = (uint32_t)(i * BLOCK + tid);
            if (gpos[i] < n) vout[gpos[i]] = s_stage.vals[p];
        }
    }
}

}  // namespace domagg
