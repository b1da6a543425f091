// Single-pass segmented scan with decoupled look-back (the segmented scan of
// Sec. 2.2: maximal runs of equal tags are scanned independently).
//
// A Problem supplies the element type staged through LDS and the monoid:
//   using V;   using Raw;
//   V    identity() const;           V combine(V earlier, V later) const;
//   Raw  load(uint64_t i) const;     element i in scan order (a reverse scan
//                                    maps i to the mirrored memory position)
//   bool head(const Raw &prev, const Raw &cur) const;   cur starts a segment
//   V    value(const Raw &prev, bool has_prev, const Raw &cur, uint64_t i) const;
//   void emit(uint64_t i, const Raw &cur, V v, V excl, V incl, bool last) const;
// Element 0 always starts a segment; `last` says the element ends its segment.
//
// status holds 2 * tiles * (1 or 2) words, zero before the launch (tiles =
// ceil(n / (BLOCK * ITEMS))).
//
// Each workgroup takes a tile from a ticket counter, stages it in LDS with
// coalesced loads, scans ITEMS consecutive elements per thread, combines
// threads with a wavefront scan on DPP and the wavefronts through LDS, and
// gets its carry-in from the tiles before it: a tile containing a segment
// start publishes its inclusive value at once; only a tile that begins
// inside a segment walks back, stopping at the first inclusive status.
#pragma once

#include "device_common.hpp"

namespace domagg {

template <class P, int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void seg_scan_kernel(P p, uint64_t n,
                                                         uint64_t *__restrict__ status,
                                                         uint32_t *__restrict__ ticket) {
    using V = typename P::V;
    using Raw = typename P::Raw;
    constexpr int TILE = BLOCK * ITEMS;
    constexpr int WAVES = BLOCK / kWave;
    static_assert(ITEMS % 2 == 0 && ITEMS <= 30, "");
    // one pad slot per ITEMS elements keeps the per-thread (blocked) LDS reads
    // spread over the banks
    auto pidx = [](int li) { return li + li / ITEMS; };

    __shared__ Raw s_raw[TILE + TILE / ITEMS];
    __shared__ Raw s_pred, s_succ;
    __shared__ V s_wval[WAVES], s_wpre[WAVES];
    __shared__ uint32_t s_wflag[WAVES], s_wpref[WAVES];
    __shared__ V s_carry;
    __shared__ uint32_t s_tile;

    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    if (tid == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint64_t base = (uint64_t)tile * TILE;
    // status: [tiles] inclusive-or-aggregate words, then [tiles] aggregate words
    uint64_t *const aggs = status + ((n + TILE - 1) / TILE) * ScanStatusWords<V>::kWords;

#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int li = j * BLOCK + tid;
        const uint64_t i = base + li;
        if (i < n) s_raw[pidx(li)] = p.load(i);
    }
    if (tid == 0 && base > 0) s_pred = p.load(base - 1);
    if (tid == BLOCK - 1 && base + TILE < n) s_succ = p.load(base + TILE);
    __syncthreads();

    const int l0 = tid * ITEMS;
    V v[ITEMS];
    uint32_t heads = 0;  // bit j: item j starts a segment; bit ITEMS: the next element does
    uint32_t tflag = 0;
    V acc = p.identity();
    Raw prev = (l0 == 0) ? s_pred : s_raw[pidx(l0 - 1)];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const uint64_t i = base + l0 + j;
        if (i < n) {
            const Raw cur = s_raw[pidx(l0 + j)];
            const bool has_prev = i > 0;
            const bool hd = !has_prev || p.head(prev, cur);
            v[j] = p.value(prev, has_prev, cur, i);
            if (hd) {
                heads |= 1u << j;
                tflag = 1;
                acc = p.identity();
            }
            acc = p.combine(acc, v[j]);
            prev = cur;
        } else {
            // past the end: marks the previous element as the last of its segment
            v[j] = p.identity();
            heads |= 1u << j;
        }
    }
    {
        const uint64_t inext = base + l0 + ITEMS;
        if (inext >= n) {
            heads |= 1u << ITEMS;
        } else {
            const Raw nxt = (l0 + ITEMS == TILE) ? s_succ : s_raw[pidx(l0 + ITEMS)];
            if (p.head(prev, nxt)) heads |= 1u << ITEMS;
        }
    }

    // Wavefront scan of the per-thread (flag, aggregate) pairs.
    uint32_t f = tflag;
    V a = acc;
    wave_seg_scan_incl(p, f, a);
    // every lane takes part in the permutes; lane 0 then drops what it read
    const int src = lane ? lane - 1 : 0;
    const V up_v = read_lane(a, src);
    const uint32_t up_f = read_lane_u32(f, src);
    const V ex_v = lane ? up_v : p.identity();
    const uint32_t ex_f = lane ? up_f : 0u;
    if (lane == kWave - 1) {
        s_wval[wave] = a;
        s_wflag[wave] = f;
    }
    __syncthreads();

    // Wavefront 0 combines the wavefront totals, publishes the tile's status
    // and looks back.  Every lane computes the same values; lane 0 writes.
    if (wave == 0) {
        V run = p.identity();
        uint32_t rf = 0;
        for (int w = 0; w < WAVES; ++w) {
            if (lane == 0) {
                s_wpre[w] = run;
                s_wpref[w] = rf;
            }
            run = s_wflag[w] ? s_wval[w] : p.combine(run, s_wval[w]);
            rf |= s_wflag[w];
        }
        // run = the tile's value at its end, counted from its last segment
        // start (rf = 1) or from its beginning (rf = 0)
        const bool first_is_head = (base == 0) || p.head(s_pred, s_raw[0]);
        if (lane == 0) {
            if (!rf) publish_status(aggs, tile, kFlagAggregate, run);
            publish_status(status, tile, rf ? kFlagInclusive : kFlagAggregate, run);
        }
        V carry = p.identity();
        if (!first_is_head) {
            // Find the nearest earlier tile with an inclusive value, 64 tiles
            // per round trip (lane l reads tile hi - l), then fold the
            // aggregates of the tiles after it left to right, 64 per round
            // trip.  Every inclusive value is therefore the same left fold
            // from its segment's start whatever the timing, so floating-point
            // results do not depend on scheduling.
            int64_t hi = (int64_t)tile - 1, t0 = -1;
            V incl_v = p.identity();
            for (;;) {
                const int64_t t = hi - lane;
                V pv = p.identity();
                uint32_t fl = 0;
                if (t >= 0) fl = wait_status<V>(status, (uint32_t)t, pv);
                const uint64_t im = __ballot(fl == kFlagInclusive);
                if (im) {
                    const int l = __ffsll((unsigned long long)im) - 1;  // nearest
                    t0 = hi - l;
                    incl_v = read_lane(pv, l);
                    break;
                }
                hi -= kWave;
            }
            carry = incl_v;
            for (int64_t w0 = t0 + 1; w0 < (int64_t)tile; w0 += kWave) {
                const int64_t t = w0 + lane;
                V av = p.identity();
                if (t < (int64_t)tile) (void)wait_status<V>(aggs, (uint32_t)t, av);
                const int cnt = (int)(((int64_t)tile - w0) < kWave ? ((int64_t)tile - w0) : kWave);
                for (int k = 0; k < cnt; ++k) carry = p.combine(carry, read_lane(av, k));
            }
            if (!rf && lane == 0) publish_status(status, tile, kFlagInclusive, p.combine(carry, run));
        }
        if (lane == 0) s_carry = carry;
    }
    __syncthreads();

    V run = s_carry;
    run = s_wpref[wave] ? s_wpre[wave] : p.combine(run, s_wpre[wave]);
    run = ex_f ? ex_v : p.combine(run, ex_v);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const uint64_t i = base + l0 + j;
        if (i < n) {
            if ((heads >> j) & 1u) run = p.identity();
            const V excl = run;
            run = p.combine(run, v[j]);
            p.emit(i, s_raw[pidx(l0 + j)], v[j], excl, run, (heads >> (j + 1)) & 1u);
        }
    }
}

}  // namespace domagg
