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
// and optionally
//   void pre(uint64_t i, const Raw &cur) const;   element-wise outputs that do
//                                    not depend on the scan, written while
//                                    the tile is staged (consecutive threads,
//                                    consecutive elements: coalesced stores)
// Element 0 always starts a segment; `last` says the element ends its segment.
// combine must be associative; with an integral V it must also be exact, as
// integer sums and maxima are: the look-back then folds tile aggregates in a
// tree rather than strictly left to right.
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

#include <type_traits>
#include <utility>

#include "device_common.hpp"

namespace domagg {

template <class P, class = void>
struct HasPre : std::false_type {};
template <class P>
struct HasPre<P, std::void_t<decltype(std::declval<const P &>().pre(uint64_t(0),
                                                                    std::declval<const typename P::Raw &>()))>>
    : std::true_type {};

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
    __shared__ V s_wval[WAVES];
    __shared__ uint32_t s_wflag[WAVES];
    __shared__ V s_carry;
    __shared__ uint32_t s_tile;

    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    if (tid == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint64_t base = (uint64_t)tile * TILE;
    // status: [tiles] inclusive-or-aggregate words, then [tiles] aggregate words
    uint64_t *const aggs = status + ((n + TILE - 1) / TILE) * ScanStatusWords<V>::kWords;

    {
        // every load of the tile in flight before the first LDS store: the
        // indices are clamped into [0, n), so no load is predicated (a
        // predicated load followed by its store waited once per item)
        Raw rr[ITEMS];
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint64_t i = base + (uint64_t)j * BLOCK + tid;
            rr[j] = p.load(i < n ? i : n - 1);
        }
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int li = j * BLOCK + tid;
            if (base + li < n) {
                s_raw[pidx(li)] = rr[j];
                if constexpr (HasPre<P>::value) p.pre(base + (uint64_t)li, rr[j]);
            }
        }
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

    // This wavefront's prefix within the tile: the combined totals of the
    // wavefronts before it, and whether a segment starts among them.
    V wpre = p.identity();
    uint32_t wpref = 0;
    for (int w = 0; w < wave; ++w) {
        wpre = s_wflag[w] ? s_wval[w] : p.combine(wpre, s_wval[w]);
        wpref |= s_wflag[w];
    }
    // The thread's items depend on the tile's carry-in only if no segment
    // starts in the tile before them; all other threads emit at once, while
    // wavefront 0 is still looking back.
    const bool needs_carry = !(wpref || ex_f);
    auto emit_items = [&](V run) {
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
    };

    // Wavefront 0 combines the wavefront totals, publishes the tile's status
    // and looks back.  Every lane computes the same values; lane 0 writes.
    if (wave == 0) {
        V run = p.identity();
        uint32_t rf = 0;
        for (int w = 0; w < WAVES; ++w) {
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
            // Find the nearest earlier tile with an inclusive value, then fold
            // the aggregates of the tiles after it left to right.  Each lane
            // reads kDepth tiles per round trip (lane l, slot k: distance
            // 64 k + l), their loads issued together, so a round trip covers
            // 64 kDepth tiles.  Every inclusive value is the same left fold
            // from its segment's start whatever the timing, so floating-point
            // results do not depend on scheduling.
            constexpr int kDepth = 4;
            int64_t hi = (int64_t)tile - 1, t0 = -1;
            V incl_v = p.identity();
            for (;;) {
                V pv[kDepth];
                uint32_t fl[kDepth];
#pragma unroll
                for (int k = 0; k < kDepth; ++k) {
                    const int64_t t = hi - lane - kWave * k;
                    pv[k] = p.identity();
                    fl[k] = t >= 0 ? try_status<V>(status, (uint32_t)t, pv[k]) : kFlagAggregate;
                }
                // Only the published run of tiles nearest to this one
                // matters: stop at its first inclusive value, and poll again
                // only while that run is cut short by an unpublished tile.
                bool found = false;
#pragma unroll
                for (int k = 0; k < kDepth; ++k) {
                    if (found) continue;
                    const int64_t t = hi - lane - kWave * k;
                    for (;;) {
                        const uint64_t pub = __ballot(fl[k] != 0);
                        const uint64_t inc = __ballot(t >= 0 && fl[k] == kFlagInclusive);
                        const int run = pub == ~0ull ? kWave : __ffsll((unsigned long long)~pub) - 1;
                        const uint64_t near = inc & (run == kWave ? ~0ull : ((1ull << run) - 1ull));
                        if (near) {
                            const int l = __ffsll((unsigned long long)near) - 1;  // nearest
                            t0 = hi - l - kWave * k;
                            incl_v = read_uniform_lane(pv[k], l);
                            found = true;
                            break;
                        }
                        if (run == kWave) break;  // 64 aggregates: on to the next slot
                        __builtin_amdgcn_s_sleep(1);
                        if (fl[k] == 0) fl[k] = try_status<V>(status, (uint32_t)t, pv[k]);
                    }
                }
                if (found) break;
                hi -= kWave * kDepth;
            }
            carry = incl_v;
            for (int64_t w0 = t0 + 1; w0 < (int64_t)tile; w0 += kWave * kDepth) {
                V av[kDepth];
                uint32_t fl[kDepth];
#pragma unroll
                for (int k = 0; k < kDepth; ++k) {
                    const int64_t t = w0 + kWave * k + lane;
                    av[k] = p.identity();
                    fl[k] = t < (int64_t)tile ? try_status<V>(aggs, (uint32_t)t, av[k]) : kFlagAggregate;
                }
#pragma unroll
                for (int k = 0; k < kDepth; ++k) {
                    const int64_t t = w0 + kWave * k + lane;
                    while (fl[k] == 0) {
                        __builtin_amdgcn_s_sleep(1);
                        fl[k] = try_status<V>(aggs, (uint32_t)t, av[k]);
                    }
                }
#pragma unroll
                for (int k = 0; k < kDepth; ++k) {
                    const int64_t left = (int64_t)tile - (w0 + kWave * k);
                    const int cnt = left <= 0 ? 0 : (left < kWave ? (int)left : kWave);
                    if constexpr (std::is_integral<V>::value) {
                        // Integer values: every grouping gives the left fold's
                        // result exactly, so the wavefront folds the 64
                        // aggregates as a tree (blocks of 2, 4, ... lanes, in
                        // tile order) instead of one after another.
                        V x = lane < cnt ? av[k] : p.identity();
#pragma unroll
                        for (int off = 1; off < kWave; off <<= 1) {
                            const V y = read_lane(x, lane ^ off);
                            x = (lane & off) ? p.combine(y, x) : p.combine(x, y);
                        }
                        carry = p.combine(carry, x);
                    } else {
                        for (int l = 0; l < cnt; ++l) carry = p.combine(carry, read_uniform_lane(av[k], l));
                    }
                }
            }
            if (!rf && lane == 0) publish_status(status, tile, kFlagInclusive, p.combine(carry, run));
        }
        if (lane == 0) s_carry = carry;
    }
    if (!needs_carry) emit_items(ex_f ? ex_v : p.combine(wpre, ex_v));
    __syncthreads();
    if (needs_carry) emit_items(p.combine(p.combine(s_carry, wpre), ex_v));
}

}  // namespace domagg
