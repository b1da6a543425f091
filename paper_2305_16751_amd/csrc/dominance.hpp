// The dominance-specific kernels and scan problems:
//   - order-preserving keys of one coordinate axis (Sec. 4, the coordinate
//     list of each axis) with the radix histogram fused in;
//   - dense ranks from a sorted axis (Sec. 4, the shift / less / sum-scan
//     steps, and the broadcast of the number of distinct values);
//   - per-point record counts and their offsets (the sizes of the flat map:
//     a data point yields the product over the expanded axes of
//     |P0(rank)| = L - popcount, a query of |P1(rank)| = popcount, Lemma 2);
//   - the flat map itself, load-balanced over output records (Sec. 5: the
//     last axis is not expanded);
//   - the segmented scan of the weights over the sorted records and the
//     regrouping of query partials (Sec. 4), and its transpose for the
//     gradient.
#pragma once

#include <type_traits>

#include "device_common.hpp"
#include "radix_sort.hpp"

namespace domagg {

// ---------------------------------------------------------------------------
// Points are numbered by slot: queries first (slot = query row), then data
// (slot = nQ + data row).  Sorting a coordinate stably by value therefore
// puts queries before data on equal values, the tie rule of Sec. 5, and
// keeps row order among equals (IDs break ties, Sec. 2.1).

__device__ __forceinline__ uint32_t ordered_key(float x) {
    uint32_t u = __float_as_uint(x);
    if (x == 0.0f) u = 0u;  // -0 and +0 are the same real number
    return (u >> 31) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ uint32_t ordered_key(int32_t x) { return (uint32_t)x ^ 0x80000000u; }
__device__ __forceinline__ bool is_nan(float x) { return x != x; }
__device__ __forceinline__ bool is_nan(int32_t) { return false; }

// The point a list position holds before a coordinate sort: slot p (queries
// first), or with data_first the data points first (slot nQ + p for p < nD),
// so that a stable sort puts data before queries on equal coordinates (the
// tie rule of <= on the last axis).
__device__ __forceinline__ uint32_t slot_at(uint64_t p, uint32_t nQ, uint32_t n, bool data_first) {
    if (!data_first) return (uint32_t)p;
    const uint32_t nD = n - nQ;
    return p < nD ? nQ + (uint32_t)p : (uint32_t)p - nD;
}

// keys[p] = (instance << 32 | ordered coordinate) or the ordered coordinate
// of the point s at position p (slot_at); vals[p] = its internal slot,
// ppos[s] (or s while ppos is not yet known).  Fused histogram of `passes`
// digits; NaN raises *nan_flag.
template <class K, class C, int BLOCK>
__global__ __launch_bounds__(BLOCK) void extract_keys_kernel(
    const C *__restrict__ q, const C *__restrict__ d, int m, int axis, uint32_t nQ, uint32_t n,
    const uint32_t *__restrict__ inst_of_slot, const uint32_t *__restrict__ ppos, K *__restrict__ keys,
    uint32_t *__restrict__ vals, int passes, uint32_t *__restrict__ hist_part, uint32_t *__restrict__ nan_flag,
    bool data_first) {
    __shared__ uint32_t s_hist[kMaxPasses * kRadix];
    for (int i = threadIdx.x; i < passes * kRadix; i += BLOCK) s_hist[i] = 0;
    __syncthreads();
    bool saw_nan = false;
    // U points per thread and round, every load issued before the first is
    // used (indices clamped below n)
    constexpr int U = 4;
    const uint64_t stride = (uint64_t)gridDim.x * BLOCK * U;
    for (uint64_t b = (uint64_t)blockIdx.x * BLOCK * U; b < n; b += stride) {
        C xs[U];
        uint32_t ps[U], is[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t p0 = b + (uint64_t)u * BLOCK + threadIdx.x;
            const uint64_t s = slot_at(p0 < n ? p0 : (uint64_t)n - 1, nQ, n, data_first);
            xs[u] = (s < nQ) ? q[s * m + axis] : d[(s - nQ) * m + axis];
            ps[u] = ppos ? ppos[s] : (uint32_t)s;
            is[u] = (sizeof(K) == 8 && inst_of_slot) ? inst_of_slot[s] : 0u;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t p = b + (uint64_t)u * BLOCK + threadIdx.x;
            const bool valid = p < n;
            K key = 0;
            if (valid) {
                const C x = xs[u];
                saw_nan |= is_nan(x);
                key = (K)ordered_key(x);
                if constexpr (sizeof(K) == 8) key |= (K)is[u] << 32;
                keys[p] = key;
                vals[p] = ps[u];
            }
            // (the low digits of coordinate keys are spread; the top one, with
            // the sign and exponent, and the instance digits are skewed)
            hist_add(s_hist, key, valid, passes, sizeof(K) == 8 ? 3 : passes - 1);
        }
    }
    if (saw_nan) atomicOr(nan_flag, 1u);
    __syncthreads();
    hist_flush(s_hist, hist_part, passes);
}

// m = 2: keys of the last (real) axis as above, with 64-bit payloads that
// carry what the flat map needs of each point, so that the count pass reads
// it in sequence instead of gathering it:
//   bit 63 query, bits 32..62 first-axis rank, bits 0..31 the record payload
//   (query: its internal row, with kQueryFlag unless records carry weights;
//   data: its internal row, or its weight bits when records carry weights).
// pr[s] = rank << 32 | internal slot (from the first axis's rank pass); w:
// weights in input order (records carrying weights) or null.
template <class K, class C, class W, int BLOCK>
__global__ __launch_bounds__(BLOCK) void extract_sigma_kernel(
    const C *__restrict__ q, const C *__restrict__ d, int axis, uint32_t nQ, uint32_t n,
    const uint32_t *__restrict__ inst_of_slot, const uint64_t *__restrict__ pr, const W *__restrict__ w,
    bool carry_weights, K *__restrict__ keys, uint64_t *__restrict__ vals, int passes,
    uint32_t *__restrict__ hist_part, uint32_t *__restrict__ nan_flag, bool data_first) {
    __shared__ uint32_t s_hist[kMaxPasses * kRadix];
    for (int i = threadIdx.x; i < passes * kRadix; i += BLOCK) s_hist[i] = 0;
    __syncthreads();
    bool saw_nan = false;
    // U points per thread and round, every load issued before the first is
    // used (indices clamped below n)
    constexpr int U = 4;
    const uint64_t stride = (uint64_t)gridDim.x * BLOCK * U;
    for (uint64_t b = (uint64_t)blockIdx.x * BLOCK * U; b < n; b += stride) {
        C xs[U];
        uint64_t rss[U];
        uint32_t wbs[U], is[U], ss[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t p0 = b + (uint64_t)u * BLOCK + threadIdx.x;
            const uint64_t s = slot_at(p0 < n ? p0 : (uint64_t)n - 1, nQ, n, data_first);
            ss[u] = (uint32_t)s;
            xs[u] = (s < nQ) ? q[s * 2 + axis] : d[(s - nQ) * 2 + axis];
            rss[u] = pr[s];
            // (weights exist only with data: n > nQ, so the clamped index is in bounds)
            wbs[u] = 0;
            if (carry_weights && w && n > nQ) __builtin_memcpy(&wbs[u], &w[s >= nQ ? s - nQ : 0], 4);
            is[u] = (sizeof(K) == 8 && inst_of_slot) ? inst_of_slot[s] : 0u;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t p = b + (uint64_t)u * BLOCK + threadIdx.x;
            const bool valid = p < n;
            K key = 0;
            if (valid) {
                const bool isq = ss[u] < nQ;
                const C x = xs[u];
                saw_nan |= is_nan(x);
                key = (K)ordered_key(x);
                if constexpr (sizeof(K) == 8) key |= (K)is[u] << 32;
                const uint64_t rs = rss[u];
                const uint32_t sp = (uint32_t)rs, r = (uint32_t)(rs >> 32);
                uint32_t payload;
                if (isq) {
                    payload = carry_weights ? sp : (kQueryFlag | sp);
                } else if (carry_weights) {
                    payload = wbs[u];
                } else {
                    payload = sp - nQ;
                }
                keys[p] = key;
                vals[p] = ((uint64_t)((isq ? 0x80000000u : 0u) | r) << 32) | payload;
            }
            // (the low digits of coordinate keys are spread; the top one, with
            // the sign and exponent, and the instance digits are skewed)
            hist_add(s_hist, key, valid, passes, sizeof(K) == 8 ? 3 : passes - 1);
        }
    }
    if (saw_nan) atomicOr(nan_flag, 1u);
    __syncthreads();
    hist_flush(s_hist, hist_part, passes);
}

// The basic variant (Sec. 4): every axis is expanded, and inside a tuple's
// run of records data precede queries.  The point order the flat map follows
// is then data first, then queries (slot order otherwise), with no
// coordinate read: keys[p] = the instance (64-bit keys) or 0, slots[p] = the
// internal slot of the point at position p.
template <class K>
__global__ void basic_order_kernel(uint32_t nQ, uint32_t n, const uint32_t *__restrict__ inst_of_slot,
                                   const uint32_t *__restrict__ ppos, K *__restrict__ keys,
                                   uint32_t *__restrict__ slots) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        const uint32_t s = slot_at(p, nQ, n, true);
        K key = 0;
        if constexpr (sizeof(K) == 8) key = inst_of_slot ? (K)inst_of_slot[s] << 32 : K(0);
        keys[p] = key;
        slots[p] = ppos[s];
    }
}

// inst_of_slot[s]: the instance owning slot s (largest k with off[k] <= row).
__global__ void instance_of_slot_kernel(const int64_t *__restrict__ q_off,
                                        const int64_t *__restrict__ d_off, int64_t n_inst,
                                        uint32_t nQ, uint32_t n, uint32_t *__restrict__ out) {
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t *off = s < nQ ? q_off : d_off;
    const int64_t row = s < nQ ? (int64_t)s : (int64_t)(s - nQ);
    int64_t lo = 0, hi = n_inst;  // off[lo] <= row < off[hi]
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (off[mid] <= row) lo = mid; else hi = mid;
    }
    out[s] = (uint32_t)lo;
}

template <class T>
__global__ void fill_kernel(T *__restrict__ p, uint64_t n, T v) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// Clears a scan's or a sort pass's look-back words and its ticket counter
// (a kernel rather than a memset, so the clear is safe inside a HIP graph).
__global__ void clear_lookback_kernel(uint64_t *__restrict__ status, uint64_t words,
                                      uint32_t *__restrict__ ticket) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride)
        status[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *ticket = 0;
}

// ---------------------------------------------------------------------------
// Dense ranks (Sec. 4): over a list sorted by (instance, coordinate), the
// value is 1 where the coordinate differs from its predecessor (the first
// element compares with -inf); its inclusive sum restarted at every instance
// is the 1-based rank.  The last element of each instance holds K, the number
// of distinct coordinates.  rank[slot] receives the 0-based rank.
//
// Internal numbering (POS, first expanded axis only).  Every later stage
// numbers points by their order on this axis instead of by input row: data
// point d becomes dpos = the number of data points before it in the sorted
// list, query q becomes qpos likewise, and the internal slot is qpos or
// nQ + dpos (queries first, as for input slots).  Instance ranges are kept
// (positions of instance k lie in [off[k], off[k+1])).  This is a relabelling
// only; the method's lists are unchanged.  What it buys: the records of a
// tree node on this axis come from a contiguous rank range, so their data
// and query labels fall in a narrow window, and the scans' weight gathers and
// partial stores stay in cache instead of striding over all of HBM.  The
// count of data points rides in the high half of the scan value.

template <class K, bool POS = false>
struct RankProblem {
    using V = typename std::conditional<POS, uint64_t, uint32_t>::type;
    struct Raw {
        K key;
        uint32_t slot;
    };
    const K *keys;
    const uint32_t *slots;
    uint32_t *rank;
    uint32_t *kcount;  // [n_inst]
    uint32_t n;        // points: slots read from the sorted list are checked against it
    uint32_t n_inst;
    // POS only
    uint32_t nQ;
    const int64_t *doff, *qoff;  // instance offsets of data and queries, or null (one instance)
    uint32_t *ppos;              // [n] by input slot: the internal slot (or null, see pr)
    uint64_t *pr;                // or [n] by input slot: rank << 32 | internal slot (m = 2)
    uint32_t *cdf_d, *cdf_q;     // or null; one instance: data / queries of rank below r, at [r]
    uint32_t *dinv, *qinv;       // [nD], [nQ]: input row of each position
    // <= on this axis: the queries' ranks move up by one (slots below nq_le
    // are queries; 0 for strict dominance)
    uint32_t nq_le;

    __device__ static uint32_t inst(const Raw &r) {
        if constexpr (sizeof(K) == 8) return (uint32_t)(r.key >> 32);
        else return 0u;
    }
    __device__ V identity() const { return V(0); }
    __device__ V combine(V a, V b) const { return a + b; }
    __device__ Raw load(uint64_t i) const { return Raw{keys[i], slots[i]}; }
    __device__ bool head(const Raw &prev, const Raw &cur) const { return inst(prev) != inst(cur); }
    __device__ V value(const Raw &prev, bool has_prev, const Raw &cur, uint64_t) const {
        const V distinct = (!has_prev || prev.key != cur.key) ? V(1) : V(0);
        if constexpr (POS) return distinct | ((uint64_t)(cur.slot >= nQ) << 32);
        else return distinct;
    }
    __device__ void emit(uint64_t i, const Raw &cur, V v, V excl, V incl, bool last) const {
        const uint32_t r = (uint32_t)incl - 1u;
        const uint32_t ins = inst(cur);
        if (cur.slot >= n || ins >= n_inst) return;  // only if the sort were wrong
        if constexpr (POS) {
            if (cdf_d && ((uint32_t)v & 1u) && r < n) {
                // the first point of rank r: the points before it have ranks below r
                const uint32_t dbefore = (uint32_t)(excl >> 32);
                cdf_d[r] = dbefore;
                cdf_q[r] = (uint32_t)i - dbefore;
            }
            // data points up to and including element i, in this instance
            const uint64_t cd = incl >> 32;
            const uint64_t dbase = doff ? (uint64_t)doff[ins] : 0ull;
            uint32_t sp;
            if (cur.slot >= nQ) {
                const uint32_t p = (uint32_t)(dbase + cd - 1u);
                if (p >= n - nQ) return;
                dinv[p] = cur.slot - nQ;
                sp = nQ + p;
            } else {
                // element i is the (i - dbase - qbase)-th of its instance,
                // cd of those before it are data
                const uint32_t p = (uint32_t)(i - dbase - cd);
                if (p >= nQ) return;
                qinv[p] = cur.slot;
                sp = p;
            }
            const uint32_t rq = r + (cur.slot < nq_le ? 1u : 0u);
            if (pr) pr[cur.slot] = ((uint64_t)rq << 32) | sp;
            else ppos[cur.slot] = sp;
            rank[sp] = rq;
        } else {
            rank[cur.slot] = r + (cur.slot < nq_le ? 1u : 0u);
        }
        if (last) kcount[ins] = (uint32_t)incl;
    }
};

// dst[p] = src[idx[p]]: inputs into internal order (idx is a permutation of
// [0, n); an index outside it would mean a wrong sort and reads 0 instead).
template <class T>
__global__ void gather_kernel(const T *__restrict__ src, const uint32_t *__restrict__ idx, T *__restrict__ dst,
                              uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        const uint32_t i = idx[p];
        dst[p] = i < n ? src[i] : T(0);
    }
}

// Records that carry their weights: rw[s] = rank of the first axis (low
// half) | bits of the weight of data point s - nQ, taken from input row
// dinv[s - nQ] (high half; 0 for queries or without weights).  W: a 4-byte
// weight type.
template <class W>
__global__ void pack_rank_weight_kernel(const uint32_t *__restrict__ rank0, const uint32_t *__restrict__ dinv,
                                        const W *__restrict__ w, uint32_t nQ, uint64_t n, uint64_t *__restrict__ rw) {
    static_assert(sizeof(W) == 4, "");
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += stride) {
        uint32_t wb = 0;
        if (w && s >= nQ) {
            const uint32_t row = dinv[s - nQ];
            if (row < n - nQ) __builtin_memcpy(&wb, &w[row], 4);  // (dinv is a permutation of the data rows)
        }
        rw[s] = (uint64_t)rank0[s] | ((uint64_t)wb << 32);
    }
}

// dst[idx[p]] = src[p]: results back into input order (idx is a permutation
// of [0, n); an index outside it is dropped).
template <class T>
__global__ void scatter_kernel(const T *__restrict__ src, const uint32_t *__restrict__ idx, T *__restrict__ dst,
                               uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        const uint32_t i = idx[p];
        if (i < n) dst[i] = src[p];
    }
}

// ---------------------------------------------------------------------------
// Flat-map sizes.  Over the points in last-axis order (slot list `slots`,
// sorted keys carry the instance), the value is the number of records the
// point yields; the exclusive sums are the record offsets, off[n] = E.  As a
// side effect the point's ranks, payload and instance are laid out in that
// order for the emitter.

template <class K, int NAX, bool INL = false>
struct CountProblem {
    using V = uint64_t;
    struct Raw {
        K key;
        uint32_t slot;
    };
    const K *keys;
    const uint32_t *slots;
    const uint32_t *rank;   // [NAX][n] by slot
    const uint8_t *ltab;    // [NAX][n_inst]
    uint32_t n_inst, nQ, n;
    uint64_t *off;          // [n + 1]
    uint32_t *rs;           // [NAX][n] by position
    uint32_t *pay;          // [n] by position: record payload of the point
    uint32_t *inst_s;       // [n] by position, or null
    // INL: first-axis rank and weight bits packed by slot (rank low, weight
    // high); wv[i] receives the weight bits of data points
    const uint64_t *rw;
    uint32_t *wv;

    __device__ static uint32_t inst(const Raw &r) {
        if constexpr (sizeof(K) == 8) return (uint32_t)(r.key >> 32);
        else return 0u;
    }
    __device__ V identity() const { return 0ull; }
    __device__ V combine(V a, V b) const { return a + b; }
    __device__ Raw load(uint64_t i) const { return Raw{keys[i], slots[i]}; }
    __device__ bool head(const Raw &, const Raw &) const { return false; }
    __device__ V value(const Raw &, bool, const Raw &cur, uint64_t i) const {
        const bool isq = cur.slot < nQ;
        const uint32_t ins = inst(cur);
        if (cur.slot >= n || ins >= n_inst) return 0ull;  // only if the sort were wrong: no records
        uint64_t c = 1;
#pragma unroll
        for (int a = 0; a < NAX; ++a) {
            uint32_t r;
            if (INL && a == 0) {
                const uint64_t x = rw[cur.slot];  // one gather for the rank and the weight
                r = (uint32_t)x;
                if (!isq) wv[i] = (uint32_t)(x >> 32);
            } else {
                r = rank[(uint64_t)a * n + cur.slot];
            }
            const uint32_t L = ltab[(uint64_t)a * n_inst + ins];
            const uint32_t pc = (uint32_t)__popc(r);
            c *= isq ? pc : (L - pc);
            rs[(uint64_t)a * n + i] = r;
        }
        pay[i] = isq ? (kQueryFlag | cur.slot) : (cur.slot - nQ);
        if (inst_s) inst_s[i] = ins;
        return c;
    }
    __device__ void emit(uint64_t i, const Raw &, V, V excl, V incl, bool) const {
        off[i] = excl;
        if (i == (uint64_t)n - 1) off[n] = incl;
    }
};

// ---------------------------------------------------------------------------
// The flat map (Sec. 4 with Sec. 5).  Output record o belongs to the point k
// with off[k] <= o < off[k+1]; its index t = o - off[k] enumerates the
// product of the point's per-axis prefix sets (mixed radix, last expanded
// axis fastest).  On axis a the t_a-th element of P0 (data) or P1 (query) of
// the L_a-bit rank r is the prefix of length j, where j is the position,
// counted from the most significant digit, of the t_a-th 0 (data) or 1
// (query) digit of r.  That bitstring is stored as the tree node id
// (1 << j) | (r >> (L_a - j)), which is unique across lengths.  Points are in
// last-axis order and the record sort is stable, which yields the Sec. 5
// order inside every segment.

// m = 2 with the last-axis sort's 64-bit payloads (extract_sigma_kernel):
// the same counts, offsets and laid-out state, read in sequence.
template <class K, bool INL>
struct CountProblemSigma {
    using V = uint64_t;
    struct Raw {
        K key;
        uint64_t v;
    };
    const K *keys;
    const uint64_t *vals;
    const uint8_t *ltab;  // [n_inst]
    uint32_t n_inst, n;
    uint64_t *off;        // [n + 1]
    uint32_t *rs;         // [n] by position: first-axis rank
    uint32_t *pay;        // [n] by position: kQueryFlag | query row, or data row (0 with weights)
    uint32_t *inst_s;     // [n] by position, or null
    uint32_t *wv;         // INL: [n] by position, weight bits of data points

    __device__ static uint32_t inst(const Raw &r) {
        if constexpr (sizeof(K) == 8) return (uint32_t)(r.key >> 32);
        else return 0u;
    }
    __device__ V identity() const { return 0ull; }
    __device__ V combine(V a, V b) const { return a + b; }
    __device__ Raw load(uint64_t i) const { return Raw{keys[i], vals[i]}; }
    __device__ bool head(const Raw &, const Raw &) const { return false; }
    // the point's state in last-axis order (while the tile is staged)
    __device__ void pre(uint64_t i, const Raw &cur) const {
        const bool isq = (cur.v >> 63) != 0;
        const uint32_t r = (uint32_t)(cur.v >> 32) & 0x7fffffffu;
        const uint32_t payload = (uint32_t)cur.v;
        const uint32_t ins = inst(cur);
        if (ins >= n_inst) return;  // only if the sort were wrong
        rs[i] = r;
        if (isq) {
            pay[i] = kQueryFlag | (payload & ~kQueryFlag);
        } else {
            pay[i] = INL ? 0u : payload;
            if (INL) wv[i] = payload;
        }
        if (inst_s) inst_s[i] = ins;
    }
    __device__ V value(const Raw &, bool, const Raw &cur, uint64_t) const {
        const bool isq = (cur.v >> 63) != 0;
        const uint32_t r = (uint32_t)(cur.v >> 32) & 0x7fffffffu;
        const uint32_t ins = inst(cur);
        if (ins >= n_inst) return 0ull;  // only if the sort were wrong: no records
        const uint32_t L = ltab[ins];
        const uint32_t pc = (uint32_t)__popc(r);
        return isq ? pc : (L - pc);
    }
    __device__ void emit(uint64_t i, const Raw &, V, V excl, V incl, bool) const {
        off[i] = excl;
        if (i == (uint64_t)n - 1) off[n] = incl;
    }
};

// Key-length classes.  The sort only has to bring equal keys together (any
// order of the segments will do) and keep the last-axis order inside them.
// A node id at level j has j + 1 significant bits, so shallow levels need
// fewer 8-bit digit passes.  With classes, the flat map writes each record
// into the region of its class -- the number of digits covering its key,
// clamped below so that there are at most kMaxClasses -- keeping last-axis
// order inside the region, and each region is sorted with its own number of
// passes.  Class c of cls_passes[c] passes is written to buffer A when that
// number is odd and to B when it is even, so that every region ends in B.
constexpr int kMaxClasses = 4;

struct EmitArgs {
    const uint64_t *off;      // [n + 1]
    const uint32_t *rs;       // [NAX][n]
    const uint32_t *pay;      // [n]
    const uint32_t *inst_s;   // [n] or null
    const uint8_t *ltab;      // [NAX][n_inst]
    const uint32_t *chunk_k;  // [chunks]: the point holding each chunk's first record
    uint32_t n, n_inst;
    uint64_t E;
    int field_shift[3];
    int inst_shift;
    int passes;               // digit passes (the largest class's, with classes)
    uint32_t *hist_part;
    unsigned long long *data_records;
    // classes (ncls = 1: records are written in last-axis order to buffer A)
    int ncls;
    int cls_c0;                          // digit count of class 0
    int cls_passes[kMaxClasses];
    int cls_row0[kMaxClasses];           // first histogram row of each class
    int hist_rows;                       // sum of cls_passes
    int rbits;                           // digit width of the record sort (<= 8)
    int sort_lo;                         // key bits below the sorted digits (a batch's instance id)
    uint32_t skew;                       // bit p: digit pass p holds a node field's top bits (skewed)
    int lmax0;                           // field width of the first expanded axis (the classes' level masks)
    uint64_t cls_base[kMaxClasses];      // region starts
    uint32_t cls_mask[kMaxClasses];      // first-axis levels of each class (bit L-1-j for level j)
    const uint32_t *cls_off;             // [chunks][kMaxClasses]: records of each class before the chunk
    uint32_t *error;                     // set when a chunk's records disagree with its class counts
    // records carrying weights (flag_shift >= 0): a data record's payload is
    // its weight bits wv[k]; a query record's payload is its row and its key
    // has bit flag_shift set (above every digit the sort looks at)
    const uint32_t *wv;
    int flag_shift;
    // packed records (pk_a non-null): one 64-bit word per record, the key
    // shifted up by pk_shift above the payload; written to pk_a (to pk_b for
    // classes whose region lives in buffer B) instead of the key and payload
    // arrays
    uint64_t *pk_a, *pk_b;
    int pk_shift;
    bool pk_labels;  // the payload is a flagged label (else 32 raw bits)
};

// A record as one 64-bit word: key above pay_bits payload bits.  A flagged
// label keeps its query flag in the top payload bit (see RecSrc).
template <class K>
__device__ __forceinline__ uint64_t pack_record(K key, uint32_t pay, int pay_bits, bool labels) {
    uint64_t p = pay;
    if (labels && (pay & kQueryFlag)) p = (1ull << (pay_bits - 1)) | (pay & ~kQueryFlag);
    return ((uint64_t)key << pay_bits) | p;
}

// Sum of the 16-bit fields of `packed` below field q (q <= 4).
__device__ __forceinline__ uint32_t packed_prefix(uint64_t packed, int q) {
    const uint64_t x = packed & (q >= 4 ? ~0ull : ((1ull << (16 * q)) - 1ull));
    return (uint32_t)(x & 0xffffu) + (uint32_t)((x >> 16) & 0xffffu) + (uint32_t)((x >> 32) & 0xffffu) +
           (uint32_t)(x >> 48);
}

// Key-length class of a record key: the number of rb-bit digits that cover
// its significant bits, less c0 (shorter keys share class 0).  The digit
// count exceeds c0 + k exactly when the key has more than (c0 + k) * rb
// significant bits, so the class is a sum of three comparisons (no division;
// keys of a plan never need more than kMaxClasses classes).
static_assert(kMaxClasses == 4, "three class thresholds");
template <class K>
__device__ __forceinline__ int key_class(K key, int c0, int rb) {
    const int bits = (int)(sizeof(K) * 8) - (sizeof(K) == 8 ? __clzll((long long)key) : __clz((int)key));
    const int t0 = c0 * rb;
    return (int)(bits > t0) + (int)(bits > t0 + rb) + (int)(bits > t0 + 2 * rb);
}

// chunk_k[c] = the point k with off[k] <= c * chunk < off[k+1].
__global__ void chunk_start_kernel(const uint64_t *__restrict__ off, uint32_t n, int chunk_shift,
                                   uint32_t *__restrict__ chunk_k) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        const uint64_t lo = off[k], hi = off[k + 1];
        const uint64_t mask = (1ull << chunk_shift) - 1;
        for (uint64_t c = (lo + mask) >> chunk_shift; (c << chunk_shift) < hi; ++c) chunk_k[c] = (uint32_t)k;
    }
}

// Per-point state of the walk, cached in LDS for the points of one chunk.
template <int NAX>
struct PointCache {
    static constexpr int kCap = 480;  // (points per chunk: about CHUNK / 12 for uniform inputs)
    uint32_t off[kCap + 1];  // low words of the record offsets (taken relative to off[0])
    uint32_t pay[kCap];
    uint32_t wv[kCap];
    uint32_t inst[kCap];
    uint32_t rank[NAX > 0 ? NAX : 1][kCap];
};

// Per-point walk over the product of prefix sets.  For each expanded axis
// the remaining digits to visit are kept as a mask over the L-digit rank
// string (bit L-1-j is digit j counted from the top); the last axis moves
// fastest, like the offsets of the count pass.
template <int NAX>
struct PointWalk {
    uint32_t r[3], L[3], full[3], rem[3];
    uint32_t payload, inst;  // payload: what the point's records carry
    bool isq;
    uint64_t kbase;  // the key bits every record of the point shares: instance and query flag

    // lsingle: the levels of every axis (8 bits each) when there is one
    // instance, else ~0u (then they are read per point)
    __device__ void set(const EmitArgs &a, uint32_t pay, uint32_t wbits, uint32_t ins, const uint32_t *ranks,
                        uint32_t lsingle) {
        isq = (pay & kQueryFlag) != 0u;
        payload = a.flag_shift < 0 ? pay : (isq ? (pay & ~kQueryFlag) : wbits);
        inst = ins;
        kbase = (a.inst_s ? (uint64_t)ins << a.inst_shift : 0ull) |
                ((a.flag_shift >= 0 && isq) ? 1ull << a.flag_shift : 0ull);
#pragma unroll
        for (int ax = 0; ax < NAX; ++ax) {
            r[ax] = ranks[ax];
            L[ax] = lsingle != ~0u ? (lsingle >> (8 * ax)) & 0xffu : a.ltab[(uint64_t)ax * a.n_inst + inst];
            const uint32_t mask = (L[ax] >= 32u) ? 0xffffffffu : ((1u << L[ax]) - 1u);
            full[ax] = isq ? (r[ax] & mask) : (~r[ax] & mask);
            rem[ax] = full[ax];
        }
    }
    // point k of the chunk (index idx among its points), from the LDS cache or global memory
    __device__ void load(const EmitArgs &a, const PointCache<NAX> *pc, bool cached, uint32_t klo, uint32_t idx,
                         uint32_t lsingle) {
        uint32_t rk[3] = {0, 0, 0};
        uint32_t pay, wb, ins;
        if (cached) {
            pay = pc->pay[idx];
            wb = pc->wv[idx];
            ins = pc->inst[idx];
#pragma unroll
            for (int ax = 0; ax < NAX; ++ax) rk[ax] = pc->rank[ax][idx];
        } else {
            const uint32_t k = klo + idx;
            pay = a.pay[k];
            wb = a.wv ? a.wv[k] : 0u;
            ins = a.inst_s ? a.inst_s[k] : 0u;
#pragma unroll
            for (int ax = 0; ax < NAX; ++ax) rk[ax] = a.rs[(uint64_t)ax * a.n + k];
        }
        set(a, pay, wb, ins, rk, lsingle);
    }
    // positions the walk at the point's t-th record
    __device__ void seek(uint32_t t) {
#pragma unroll
        for (int ax = NAX - 1; ax >= 0; --ax) {
            const uint32_t c = (uint32_t)__popc(full[ax]);
            uint32_t ta = t;
            if (ax > 0) {
                ta = t % c;
                t /= c;
            }
            for (uint32_t i = 0; i < ta; ++i) rem[ax] &= ~(1u << (31u - __clz(rem[ax])));
        }
    }
    template <class K>
    __device__ K key(const int *field_shift) const {
        K key = (K)kbase;
#pragma unroll
        for (int ax = 0; ax < NAX; ++ax) {
            const uint32_t top = 31u - (uint32_t)__clz(rem[ax]);  // highest remaining digit
            const uint32_t j = L[ax] - 1u - top;                 // its position from the top
            // (a 64-bit shift: the prefix of length 0 shifts by L, which may be 32)
            const uint32_t node = (1u << j) | (uint32_t)((uint64_t)r[ax] >> (L[ax] - j));
            key |= (K)node << field_shift[ax];
        }
        return key;
    }
    // advances to the next record; returns false when the point is exhausted
    __device__ bool next() {
#pragma unroll
        for (int ax = NAX - 1; ax >= 0; --ax) {
            rem[ax] &= ~(1u << (31u - __clz(rem[ax])));
            if (rem[ax]) return true;
            rem[ax] = full[ax];
        }
        return false;
    }
};


// Records of each class among the records [ta, tb) of one point, packed in
// 16-bit fields.  The walk visits the first axis slowest and its levels in
// increasing order (the highest remaining digit of the rank string first),
// and classes are increasing ranges of first-axis levels, so the records of
// class q are indices [R s_q, R (s_q + n_q)): n_q levels of the point fall
// in class q, s_q in the classes before it, R = records per first-axis level.
template <int NAX>
__device__ __forceinline__ uint64_t point_class_counts(const EmitArgs &a, uint32_t pay, const uint32_t *ranks,
                                                       uint32_t ins, uint32_t ta, uint32_t tb) {
    const bool isq = (pay & kQueryFlag) != 0u;
    uint32_t full0 = 0, R = 1;
#pragma unroll
    for (int ax = 0; ax < NAX; ++ax) {
        // (in a batch the instance's own widths; the class masks are over the
        // first axis's field width, so its digit string is aligned to it)
        const uint32_t L = a.inst_s ? a.ltab[(uint64_t)ax * a.n_inst + (ins < a.n_inst ? ins : 0u)] : a.ltab[ax];
        const uint32_t mask = L >= 32u ? 0xffffffffu : ((1u << L) - 1u);
        const uint32_t full = isq ? (ranks[ax] & mask) : (~ranks[ax] & mask);
        if (ax == 0) full0 = L <= (uint32_t)a.lmax0 ? full << ((uint32_t)a.lmax0 - L) : full;
        else R *= (uint32_t)__popc(full);
    }
    uint64_t packed = 0;
    uint32_t s = 0;
#pragma unroll
    for (int q = 0; q < kMaxClasses; ++q) {
        const uint32_t nq = (uint32_t)__popc(full0 & a.cls_mask[q]);
        const uint32_t lo = R * s, hi = R * (s + nq);
        const uint32_t x0 = ta < lo ? lo : (ta > hi ? hi : ta);
        const uint32_t x1 = tb < lo ? lo : (tb > hi ? hi : tb);
        packed |= (uint64_t)(x1 - x0) << (16 * q);
        s += nq;
    }
    return packed;
}

// m = 2, one instance: the digit histograms of the record keys of every
// class and pass, without looking at a single record.  The records of tree
// node t = (1 << j) | P are the data points whose rank has prefix P then a
// 0 digit and the queries whose rank has prefix P then a 1 digit (Lemma 2's
// prefix sets), i.e. two rank ranges, counted from the rank CDFs: cdf_d[x] =
// data points of rank below x (x < K; nD from K on), cdf_q likewise.  Rows
// of the histogram as in the flat map: class q, pass p -> row0[q] + p.
__global__ __launch_bounds__(256) void node_hist_kernel(const uint32_t *__restrict__ cdf_d,
                                                        const uint32_t *__restrict__ cdf_q, uint32_t K, uint32_t nD,
                                                        uint32_t nQ, int L, EmitArgs a) {
    __shared__ uint32_t s_hist[26 * kRadix];
    const int rows = a.hist_rows;
    for (int i = threadIdx.x; i < rows * kRadix; i += blockDim.x) s_hist[i] = 0;
    __syncthreads();
    auto cd = [&](uint64_t x) { return x < K ? cdf_d[x] : nD; };
    auto cq = [&](uint64_t x) { return x < K ? cdf_q[x] : nQ; };
    const uint64_t nodes = 1ull << L;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x + 1; t < nodes; t += stride) {
        const int j = 63 - __clzll((long long)t);
        const uint64_t P = t ^ (1ull << j);
        const uint64_t half = 1ull << (L - j - 1);
        const uint64_t lo = P << (L - j);
        const uint32_t cnt = (cd(lo + half) - cd(lo)) + (cq(lo + 2 * half) - cq(lo + half));
        if (cnt == 0) continue;
        const int q = key_class((uint32_t)t, a.cls_c0, a.rbits);
        int row0 = 0;
#pragma unroll
        for (int c = 0; c < kMaxClasses; ++c)
            if (c < q) row0 += a.cls_passes[c];
        int np = a.cls_passes[0];
#pragma unroll
        for (int c = 1; c < kMaxClasses; ++c)
            if (c == q) np = a.cls_passes[c];
        const uint32_t dmask = (1u << a.rbits) - 1u;
        for (int p = 0; p < np; ++p)
            atomicAdd(&s_hist[(row0 + p) * kRadix + ((uint32_t)(t >> (a.rbits * p)) & dmask)], cnt);
    }
    __syncthreads();
    if (rows) hist_flush(s_hist, a.hist_part, rows);
}

// Digit histograms from the points, for any m and batches whose instance id
// is below the sorted bits.  A point's records are the tuples of its per-axis
// node sets (Lemma 2's prefix sets, one node per selected level), and the
// digit of pass p of a record's key is the OR of its nodes' slices in the
// pass's bit window.  A node whose bits all lie below the window has a zero
// slice, so per axis the nodes split into one zero group (counted) and the
// nodes reaching into the window (taken one by one); every combination of
// groups adds the product of the group sizes to its digit.  The combination
// of zero groups only is summed over the wavefront first (it is the common
// digit 0 of the high passes).  Work per point: the sum over classes and
// passes of the combinations, far below one update per record and pass.

// Every combination of the axes AX.. (the digit and multiplicity so far);
// `picked`: an axis before AX took a reaching node.
template <int AX, int NAX>
__device__ __forceinline__ void point_hist_combos(uint32_t *row, const uint32_t *hi, const uint32_t *zero,
                                                  const uint32_t *r, const uint32_t *L, const int *fs, int w0,
                                                  uint32_t dmask, uint32_t digit, uint32_t mult, bool picked) {
    if constexpr (AX == NAX) {
        if (picked) atomicAdd(&row[digit], mult);
    } else {
        if (zero[AX]) point_hist_combos<AX + 1, NAX>(row, hi, zero, r, L, fs, w0, dmask, digit, mult * zero[AX], picked);
        for (uint32_t m = hi[AX]; m; m &= m - 1u) {
            const uint32_t b = (uint32_t)__ffs(m) - 1u;  // (lowest remaining) digit L-1-j of the rank string: level j
            const uint32_t j = L[AX] - 1u - b;
            const uint32_t node = (1u << j) | (j ? (r[AX] >> (L[AX] - j)) : 0u);
            const uint32_t sl = (uint32_t)((((uint64_t)node) << fs[AX]) >> w0) & dmask;
            point_hist_combos<AX + 1, NAX>(row, hi, zero, r, L, fs, w0, dmask, digit | sl, mult, true);
        }
    }
}

template <int NAX>
__global__ __launch_bounds__(256) void point_hist_kernel(EmitArgs a) {
    static_assert(NAX >= 1 && NAX <= 3, "");
    __shared__ uint32_t s_hist[26 * kRadix];
    const int rows = a.hist_rows;
    for (int i = threadIdx.x; i < rows * kRadix; i += blockDim.x) s_hist[i] = 0;
    __syncthreads();
    const int lane = lane_id();
    const int rb = a.rbits;
    const uint32_t dmask = (1u << rb) - 1u;
    const bool cls = a.ncls > 1;
    const int ncls = cls ? a.ncls : 1;
    int fs[NAX];
#pragma unroll
    for (int ax = 0; ax < NAX; ++ax) fs[ax] = a.field_shift[ax];
    // every lane of a wavefront runs the same rounds (wavefront sums below)
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k0 = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~(uint64_t)(kWave - 1)); k0 < a.n;
         k0 += stride) {
        const uint64_t k = k0 + (uint64_t)lane;
        bool valid = k < a.n;
        uint32_t r[NAX], L[NAX], sel[NAX];
        uint32_t ins = 0, pay = 0;
        if (valid) {
            pay = a.pay[k];
            if (a.inst_s) ins = a.inst_s[k];
            if (ins >= a.n_inst) valid = false;  // only if the sort were wrong
        }
        const bool isq = (pay & kQueryFlag) != 0u;
#pragma unroll
        for (int ax = 0; ax < NAX; ++ax) {
            r[ax] = valid ? a.rs[(uint64_t)ax * a.n + k] : 0u;
            L[ax] = valid ? (uint32_t)a.ltab[(uint64_t)ax * a.n_inst + ins] : 0u;
            const uint32_t mask = L[ax] >= 32u ? 0xffffffffu : ((1u << L[ax]) - 1u);
            sel[ax] = isq ? (r[ax] & mask) : (~r[ax] & mask);
            if (sel[ax] == 0u) valid = false;  // no records
        }
        // the class masks are over the first axis's field width: aligned to
        // this point's own width
        const uint32_t align = L[0] <= (uint32_t)a.lmax0 ? (uint32_t)a.lmax0 - L[0] : 0u;
        for (int c = 0; c < ncls; ++c) {
            const uint32_t f0 = cls ? (sel[0] & (a.cls_mask[c] >> align)) : sel[0];
            const bool vc = valid && f0 != 0u;
            const int np = cls ? a.cls_passes[c] : a.passes;
            uint32_t *rowp = s_hist + (cls ? a.cls_row0[c] : 0) * kRadix;
            for (int p = 0; p < np; ++p, rowp += kRadix) {
                const int w0 = a.sort_lo + rb * p;
                uint32_t hi[NAX], zero[NAX];
                uint32_t allz = vc ? 1u : 0u;
#pragma unroll
                for (int ax = 0; ax < NAX; ++ax) {
                    const uint32_t sx = ax == 0 ? f0 : sel[ax];
                    uint32_t h = 0;
                    if (fs[ax] < w0 + rb) {
                        const int kk = w0 > fs[ax] ? w0 - fs[ax] : 0;  // levels j >= kk reach past w0
                        if (kk < (int)L[ax]) {
                            const uint32_t nb = L[ax] - (uint32_t)kk;
                            h = sx & (nb >= 32u ? 0xffffffffu : ((1u << nb) - 1u));
                        }
                    }
                    hi[ax] = h;
                    zero[ax] = (uint32_t)(__popc(sx) - __popc(h));
                    allz *= zero[ax];
                }
                const uint32_t tot = wave_sum_scan_incl(allz);
                if (lane == kWave - 1 && tot) atomicAdd(&rowp[0], tot);
                if (vc) point_hist_combos<0, NAX>(rowp, hi, zero, r, L, fs, w0, dmask, 0u, 1u, false);
            }
        }
    }
    __syncthreads();
    if (rows) hist_flush(s_hist, a.hist_part, rows);
}

// The flat map (Sec. 4 with Sec. 5).  Record o belongs to the point k with
// off[k] <= o < off[k+1]; its index t = o - off[k] enumerates the product of
// the point's per-axis prefix sets, last expanded axis fastest.  On axis a
// the t_a-th element of P0 (data) or P1 (query) of the L_a-digit rank r is
// the prefix of length j, j being the position from the top of the t_a-th 0
// (data) or 1 (query) digit of r; it is stored as the tree node id
// (1 << j) | (first j digits of r), unique across lengths.  Points come in
// last-axis order and the record sort is stable, which yields the Sec. 5
// order inside every segment.
//
// A block takes chunks of CHUNK consecutive records (a fixed share of them)
// and loads the state of each chunk's points into LDS with coalesced
// reads.  Each thread produces ITEMS consecutive records (one
// search for its first, then a walk) and stages them in LDS.  Without
// classes the block then writes them out in place.  With classes, each
// thread first counts its records per class from its points (closed form,
// see point_class_counts); one block scan of those counts gives every record
// its slot in a class-split staging, and the block writes each class's run
// into its region at the chunk's class offset, computed beforehand for every
// chunk by chunk_class_kernel and chunk_offsets_kernel.  The digit
// histograms of every pass (of every class) are accumulated on the way, or
// come from node_hist_kernel.

// The record sort's digit histograms from the emitted records, in one
// streaming pass (instead of inside the flat map's per-record loop): every
// record of class q (its region of buffer A or B) adds the digits of its key
// for the class's passes to rows row0[q] .. row0[q] + passes[q] - 1.
// Without classes all records are in A, with `passes` rows.
struct RecHistArgs {
    const uint64_t *pk[2];  // packed records in buffers A and B, or null
    const void *keys[2];    // keys (K) in A and B when not packed
    uint64_t E;
    int ncls;               // 1: no classes
    uint64_t cls_base[kMaxClasses];
    int cls_passes[kMaxClasses];
    int cls_row0[kMaxClasses];
    int cls_in_b[kMaxClasses];  // the region lives in buffer B
    int passes;             // without classes; with classes the largest class's
    int pay_bits;
    int rows;
    int rbits;              // digit width (<= 8)
    int sort_lo;            // key bits below the sorted digits
    uint32_t skew;          // bit p: pass p's digit is skewed (holds a field's top bits)
    uint32_t *hist_part;    // [gridDim.x][rows][256]
};

// Adds the digits of `key` for passes [0, np) to histogram rows row0 + p.
// On the passes in `skew` (digits concentrated on few values) the lanes that
// share the first active lane's row and digit are added with one atomic; the
// spread digits of the other passes take one LDS atomic per lane.  All lanes
// of the wavefront call it, for max_np passes.
template <class K>
__device__ __forceinline__ void hist_add_rows_skew(uint32_t *s_hist, K key, bool valid, int row0, int np,
                                                   int max_np, uint32_t skew, int rb) {
    const int lane = lane_id();
    const uint32_t dmask = (1u << rb) - 1u;
    for (int p = 0; p < max_np; ++p) {
        const bool v = valid && p < np;
        const uint32_t idx = (uint32_t)(row0 + p) * kRadix + ((uint32_t)(key >> (rb * p)) & dmask);
        if (!((skew >> p) & 1u)) {
            if (v) atomicAdd(&s_hist[idx], 1u);
            continue;
        }
        const uint64_t act = __ballot(v);
        if (act == 0) continue;
        const int leader = __ffsll((unsigned long long)act) - 1;
        const uint32_t i0 = read_lane_u32(idx, leader);
        const uint64_t same = __ballot(v && idx == i0);
        if (lane == leader) atomicAdd(&s_hist[i0], (uint32_t)__popcll(same));
        if (v && idx != i0) atomicAdd(&s_hist[idx], 1u);
    }
}

template <class K, bool PK>
__global__ __launch_bounds__(256) void record_hist_kernel(RecHistArgs a) {
    __shared__ uint32_t s_hist[26 * kRadix];
    for (int i = threadIdx.x; i < a.rows * kRadix; i += blockDim.x) s_hist[i] = 0;
    __syncthreads();
    // every lane of a wavefront runs the same iterations (the histogram adds
    // are wavefront operations); U records per lane, loads issued together
    constexpr int U = 4;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * U;
    const uint64_t wbase = ((uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~(uint64_t)(kWave - 1))) * U;
    const int lane = lane_id();
    for (uint64_t b = wbase; b < a.E; b += stride) {
        K key[U];
        int q[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t i0 = b + (uint64_t)u * kWave + lane;
            const uint64_t i = i0 < a.E ? i0 : a.E - 1;
            int c = 0;
#pragma unroll
            for (int t = 1; t < kMaxClasses; ++t)
                if (t < a.ncls && i >= a.cls_base[t]) c = t;
            q[u] = c;
            const int buf = a.ncls > 1 ? a.cls_in_b[c] : 0;
            if constexpr (PK) key[u] = (K)(a.pk[buf][i] >> (a.pay_bits + a.sort_lo));
            else key[u] = static_cast<const K *>(a.keys[buf])[i] >> a.sort_lo;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool valid = b + (uint64_t)u * kWave + lane < a.E;
            const int c = q[u];
            const int row0 = a.ncls > 1 ? a.cls_row0[c] : 0;
            const int np = a.ncls > 1 ? a.cls_passes[c] : a.passes;
            hist_add_rows_skew(s_hist, key[u], valid, row0, np, a.passes, a.skew, a.rbits);
        }
    }
    __syncthreads();
    hist_flush(s_hist, a.hist_part, a.rows);
}

// Exclusive sum of packed 16-bit counters over a block (each field's block
// total must stay below 2^16); *total gets the packed block sums.
template <int BLOCK>
__device__ __forceinline__ uint64_t block_excl_sum_packed(uint64_t v, uint64_t *s_tmp, uint64_t *total) {
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    // inclusive wavefront sum by DPP moves (rows, then across rows)
    uint64_t incl = v;
    incl += dpp_val<kDppRowShr1, 0xf>(incl, (uint64_t)0);
    incl += dpp_val<kDppRowShr2, 0xf>(incl, (uint64_t)0);
    incl += dpp_val<kDppRowShr4, 0xf>(incl, (uint64_t)0);
    incl += dpp_val<kDppRowShr8, 0xf>(incl, (uint64_t)0);
    incl += dpp_val<kDppRowBcast15, 0xa>(incl, (uint64_t)0);
    incl += dpp_val<kDppRowBcast31, 0xc>(incl, (uint64_t)0);
    if (lane == kWave - 1) s_tmp[wave] = incl;
    __syncthreads();
    uint64_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < BLOCK / kWave; ++w) {
        const uint64_t t = s_tmp[w];
        pre += (w < wave) ? t : 0ull;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return pre + incl - v;
}

// Sum of `v` over the wavefront, in every lane (every lane must be active).
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
    v += dpp_val<kDppRowShr1, 0xf>(v, (uint64_t)0);
    v += dpp_val<kDppRowShr2, 0xf>(v, (uint64_t)0);
    v += dpp_val<kDppRowShr4, 0xf>(v, (uint64_t)0);
    v += dpp_val<kDppRowShr8, 0xf>(v, (uint64_t)0);
    // lane 16 r + 15 holds the sum of row r
    return read_uniform_lane(v, 15) + read_uniform_lane(v, 31) + read_uniform_lane(v, 47) + read_uniform_lane(v, 63);
}

// Records of each class in every chunk of the flat map, from the points'
// closed-form class counts (the emitter's chunks, without producing them):
// cnt[c] in packed 16-bit fields (a chunk holds at most 2^16 - 1 records),
// which must start at zero.  One thread per point; a point's records in the
// chunk of its first record are summed over the lanes that share that chunk
// (consecutive points, so a wavefront spans few chunks) and added with one
// atomic; the rare points whose records run into later chunks add those
// parts one by one.
constexpr int kChunkGroup = 1024;  // chunks per group of the offset sums

__device__ __forceinline__ void unpack_class_counts(uint64_t v, uint64_t &w01, uint64_t &w23) {
    w01 = (v & 0xffffull) | (((v >> 16) & 0xffffull) << 32);
    w23 = ((v >> 32) & 0xffffull) | ((v >> 48) << 32);
}

template <int NAX>
__global__ __launch_bounds__(256) void chunk_class_kernel(EmitArgs a, int chunk_shift,
                                                          unsigned long long *__restrict__ cnt) {
    const int lane = lane_id();
    // U points per lane and round, their loads issued together (indices
    // clamped below n); every lane of a wavefront runs the same rounds
    // (wavefront sums below)
    constexpr int U = 2;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * U;
    const uint64_t base0 = ((uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~(uint64_t)(kWave - 1))) * U;
    for (uint64_t kb = base0; kb < a.n; kb += stride) {
        uint64_t bs[U], es[U];
        uint32_t pays[U], inss[U], rks[U][NAX > 0 ? NAX : 1];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t k0 = kb + (uint64_t)u * kWave + lane;
            const uint64_t k = k0 < a.n ? k0 : (uint64_t)a.n - 1;
            bs[u] = a.off[k];
            es[u] = a.off[k + 1];
            pays[u] = a.pay[k];
            inss[u] = a.inst_s ? a.inst_s[k] : 0u;
#pragma unroll
            for (int ax = 0; ax < NAX; ++ax) rks[u][ax] = a.rs[(uint64_t)ax * a.n + k];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t k = kb + (uint64_t)u * kWave + lane;
            const uint64_t b = bs[u], e = es[u];
            const bool has = k < a.n && e > b;
            const uint64_t c0 = b >> chunk_shift;
            uint64_t v = 0, end0 = 0;
            if (has) {
                end0 = (c0 + 1) << chunk_shift;
                if (end0 > e) end0 = e;
                v = point_class_counts<NAX>(a, pays[u], rks[u], inss[u], 0u, (uint32_t)(end0 - b));
            }
            // sum over the lanes sharing a first chunk, one atomic per chunk
            uint64_t todo = __ballot(has);
            while (todo) {
                const int leader = __ffsll((unsigned long long)todo) - 1;
                const uint64_t cl = read_uniform_lane(c0, leader);
                const uint64_t same = __ballot(has && c0 == cl);
                const uint64_t sum = wave_sum_u64(((same >> lane) & 1ull) ? v : 0ull);
                if (lane == leader) atomicAdd(&cnt[cl], (unsigned long long)sum);
                todo &= ~same;
            }
            // records past the first chunk (points straddling chunk ends)
            if (has && end0 < e) {
                for (uint64_t lo = end0; lo < e; lo += (1ull << chunk_shift)) {
                    const uint64_t hi = (lo + (1ull << chunk_shift) < e) ? lo + (1ull << chunk_shift) : e;
                    atomicAdd(&cnt[lo >> chunk_shift],
                              (unsigned long long)point_class_counts<NAX>(a, pays[u], rks[u], inss[u],
                                                                          (uint32_t)(lo - b), (uint32_t)(hi - b)));
                }
            }
        }
    }
}

// Class sums of each group of kChunkGroup chunks (one workgroup per group):
// gsum[2 g] holds classes 0 and 1, gsum[2 g + 1] classes 2 and 3, in 32-bit
// fields (every class has fewer than 2^32 records).
__global__ __launch_bounds__(256) void chunk_group_kernel(const unsigned long long *__restrict__ cnt, uint64_t nchunks,
                                                          unsigned long long *__restrict__ gsum) {
    constexpr int BLOCK = 256;
    __shared__ uint64_t s_tmp[BLOCK / kWave];
    const uint64_t c0 = (uint64_t)blockIdx.x * kChunkGroup;
    uint64_t s01 = 0, s23 = 0;
#pragma unroll
    for (int i = 0; i < kChunkGroup / BLOCK; ++i) {
        const uint64_t c = c0 + (uint64_t)i * BLOCK + threadIdx.x;
        uint64_t w01 = 0, w23 = 0;
        if (c < nchunks) unpack_class_counts(cnt[c], w01, w23);
        s01 += w01;
        s23 += w23;
    }
    uint64_t t01, t23;
    block_excl_sum_packed<BLOCK>(s01, s_tmp, &t01);
    block_excl_sum_packed<BLOCK>(s23, s_tmp, &t23);
    if (threadIdx.x == 0) {
        gsum[2 * blockIdx.x] = t01;
        gsum[2 * blockIdx.x + 1] = t23;
    }
}

// Exclusive sums of the per-chunk class counts: off[c] = (records of class
// q in the chunks before c, q = 0..3); tot[q] = all records of class q.
// One workgroup per group of kChunkGroup chunks (kChunkGroup / 256 chunks
// per thread); a group's start is the sum of the groups before it.
__global__ __launch_bounds__(256) void chunk_offsets_kernel(const unsigned long long *__restrict__ cnt,
                                                            const unsigned long long *__restrict__ gsum,
                                                            uint64_t nchunks, uint4 *__restrict__ off,
                                                            unsigned long long *__restrict__ tot) {
    constexpr int BLOCK = 256, PER = kChunkGroup / BLOCK;
    __shared__ uint64_t s_tmp[BLOCK / kWave];
    __shared__ uint64_t s_base[2];
    const uint64_t g = blockIdx.x;
    const uint64_t ngroups = (nchunks + kChunkGroup - 1) / kChunkGroup;
    if (threadIdx.x < kWave) {
        // groups before this one (and, for group 0, all of them: the totals)
        const uint64_t upto = g == 0 ? ngroups : g;
        uint64_t b01 = 0, b23 = 0;
        for (uint64_t h = threadIdx.x; h < upto; h += kWave) {
            b01 += gsum[2 * h];
            b23 += gsum[2 * h + 1];
        }
        b01 = wave_sum_u64(b01);
        b23 = wave_sum_u64(b23);
        if (threadIdx.x == 0) {
            if (g == 0) {
                tot[0] = (uint32_t)b01;
                tot[1] = b01 >> 32;
                tot[2] = (uint32_t)b23;
                tot[3] = b23 >> 32;
                b01 = b23 = 0;
            }
            s_base[0] = b01;
            s_base[1] = b23;
        }
    }
    const uint64_t c0 = g * kChunkGroup + (uint64_t)threadIdx.x * PER;
    uint64_t v[PER];
    uint64_t s01 = 0, s23 = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        v[i] = c0 + i < nchunks ? cnt[c0 + i] : 0ull;
        uint64_t w01, w23;
        unpack_class_counts(v[i], w01, w23);
        s01 += w01;
        s23 += w23;
    }
    uint64_t t01, t23;
    uint64_t r01 = block_excl_sum_packed<BLOCK>(s01, s_tmp, &t01);  // (plain 64-bit sums: 32-bit fields never carry)
    uint64_t r23 = block_excl_sum_packed<BLOCK>(s23, s_tmp, &t23);
    r01 += s_base[0];
    r23 += s_base[1];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        if (c0 + i < nchunks)
            off[c0 + i] = make_uint4((uint32_t)r01, (uint32_t)(r01 >> 32), (uint32_t)r23, (uint32_t)(r23 >> 32));
        uint64_t w01, w23;
        unpack_class_counts(v[i], w01, w23);
        r01 += w01;
        r23 += w23;
    }
}

// HIST: the kernel builds the record sort's digit histograms (a.hist_part);
// without it they come from elsewhere and the LDS for them is not reserved.
template <class K, int NAX, int BLOCK, int ITEMS, bool CLS, bool HIST = true>
__global__ __launch_bounds__(BLOCK) void emit_kernel(EmitArgs a, K *__restrict__ keys_a, uint32_t *__restrict__ vals_a,
                                                     K *__restrict__ keys_b, uint32_t *__restrict__ vals_b) {
    constexpr int CHUNK = BLOCK * ITEMS;
    // histogram rows: passes of every class (up to 1+2+3+4 for 32-bit keys)
    constexpr int kRows = !HIST ? 1 : CLS ? (sizeof(K) == 4 ? 10 : 26) : kMaxPasses;
    using PC = PointCache<NAX>;
    __shared__ PC s_pc;
    __shared__ K s_keys[CHUNK];
    __shared__ uint32_t s_pay[CHUNK];
    __shared__ uint32_t s_hist[HIST ? kRows * kRadix : 1];
    __shared__ unsigned long long s_data;
    __shared__ uint64_t s_scan[BLOCK / kWave];
    __shared__ uint64_t s_cdst[kMaxClasses];  // destination of the chunk's first slot of each class, minus its run start
    // packed records: where staged record i of class q goes (s_cptr[q][i]),
    // for i below s_clim[q] (the rest would fall outside the record array)
    __shared__ uint64_t *s_cptr[kMaxClasses];
    __shared__ uint32_t s_clim[kMaxClasses];
    __shared__ uint32_t s_next[2];            // the block's next chunk's point range
    __shared__ uint16_t s_tfirst[BLOCK];      // cached chunks: the point holding each thread's first record (< kCap)
    const int rows = (HIST && a.hist_part) ? (CLS ? a.hist_rows : a.passes) : 0;
    for (int i = threadIdx.x; i < rows * kRadix; i += BLOCK) s_hist[i] = 0;
    if (threadIdx.x == 0) s_data = 0;
    uint32_t my_data = 0;
    const bool with_inst = a.inst_s != nullptr;
    // the two most significant digits of the node keys are skewed toward 0
    const int peel_from = a.passes > 2 ? a.passes - 2 : 0;
    // per class: first histogram row (bits 0-7) and passes (bits 8-15), in
    // a register, so that a lane's class selects them without memory access
    uint64_t cls_info = 0;
#pragma unroll
    for (int q = 0; q < kMaxClasses; ++q)
        cls_info |= (uint64_t)((uint32_t)a.cls_row0[q] | ((uint32_t)a.cls_passes[q] << 8)) << (16 * q);

    // the key without the query flag of records that carry weights
    const K kmask = a.flag_shift >= 0 ? ~(K(1) << a.flag_shift) : ~K(0);
    // one instance: the levels of every axis, read once
    uint32_t lsingle = ~0u;
    if (!with_inst) {
        lsingle = 0;
#pragma unroll
        for (int ax = 0; ax < NAX; ++ax) lsingle |= (uint32_t)a.ltab[ax] << (8 * ax);
    }
    // class region starts
    __shared__ uint64_t s_cls_base[kMaxClasses];
    if (threadIdx.x < kMaxClasses) s_cls_base[threadIdx.x] = a.cls_base[threadIdx.x];

    const uint64_t nchunks = (a.E + CHUNK - 1) / CHUNK;
    // Block b takes chunks b, b + G, b + 2G, ... (G = gridDim.x; every chunk
    // holds CHUNK records and its class offsets are precomputed, so there is
    // no ordering between chunks).  The state of a chunk's points is loaded
    // into registers while the previous chunk's records are stored, and
    // moved into LDS when the chunk starts; a chunk whose points do not fit
    // the cache reads them from global memory during its walk.
    constexpr uint32_t kCap = PC::kCap;
    static_assert(kCap <= 2 * BLOCK, "at most two point slots per thread");
    const uint32_t *off_lo = reinterpret_cast<const uint32_t *>(a.off);  // low words: offsets within a chunk fit 32 bits
    const uint32_t i0 = threadIdx.x, i1 = threadIdx.x + BLOCK, i2 = threadIdx.x + 2 * BLOCK;
    // the prefetched state (slots i0, i1; offsets also at i2 and i0 + 1,
    // i1 + 1) and class offset
    uint32_t pf0 = 0, pf1 = 0, pf2 = 0, pg0 = 0, pg1 = 0, py0 = 0, py1 = 0, pw0 = 0, pw1 = 0, pn0 = 0, pn1 = 0;
    uint32_t pcoff = 0;
    uint32_t pr0[NAX > 0 ? NAX : 1], pr1[NAX > 0 ? NAX : 1];
#pragma unroll
    for (int ax = 0; ax < (NAX > 0 ? NAX : 1); ++ax) pr0[ax] = pr1[ax] = 0;
    // point range [klo, khi] of chunk c (khi < n: the point holding the next
    // chunk's first record, or the last point)
    auto chunk_lo = [&](uint64_t c) -> uint32_t { return a.chunk_k[c]; };
    auto chunk_hi = [&](uint64_t c) -> uint32_t { return (c + 1 < nchunks) ? a.chunk_k[c + 1] : a.n - 1; };
    auto prefetch = [&](uint64_t c, uint32_t klo, uint32_t khi) {
        if constexpr (CLS) pcoff = a.cls_off[c * kMaxClasses + (threadIdx.x & (kMaxClasses - 1))];
        const uint32_t npts = khi - klo + 1;
        if (npts > kCap) return;
        // clamped indices: every load in bounds (klo + npts <= n), only the LDS stores are predicated
        const uint32_t j0 = i0 < npts ? i0 : npts - 1, j1 = i1 < npts ? i1 : npts - 1;
        pf0 = off_lo[2ull * (klo + (i0 <= npts ? i0 : npts))];
        pf1 = off_lo[2ull * (klo + (i1 <= npts ? i1 : npts))];
        pf2 = off_lo[2ull * (klo + (i2 <= npts ? i2 : npts))];
        pg0 = off_lo[2ull * (klo + (i0 + 1 <= npts ? i0 + 1 : npts))];  // the ends of points i0, i1
        pg1 = off_lo[2ull * (klo + (i1 + 1 <= npts ? i1 + 1 : npts))];
        py0 = a.pay[klo + j0];
        py1 = a.pay[klo + j1];
        if (a.wv) {
            pw0 = a.wv[klo + j0];
            pw1 = a.wv[klo + j1];
        }
        if (with_inst) {
            pn0 = a.inst_s[klo + j0];
            pn1 = a.inst_s[klo + j1];
        }
#pragma unroll
        for (int ax = 0; ax < NAX; ++ax) {
            pr0[ax] = a.rs[(uint64_t)ax * a.n + klo + j0];
            pr1[ax] = a.rs[(uint64_t)ax * a.n + klo + j1];
        }
    };
    uint64_t c = blockIdx.x;
    uint32_t klo = 0, khi = 0;
    if (c < nchunks) {
        klo = chunk_lo(c);
        khi = chunk_hi(c);
        prefetch(c, klo, khi);
    }
    for (; c < nchunks; c += gridDim.x) {
        const uint64_t cn = c + gridDim.x;
        const uint64_t o0 = c * CHUNK;
        const uint64_t o1 = (o0 + CHUNK < a.E) ? o0 + CHUNK : a.E;
        const uint32_t npts = khi - klo + 1;
        const uint32_t nrec = (uint32_t)(o1 - o0);
        uint32_t nklo = 0, nkhi = 0;
        uint64_t tot = 0;  // the chunk's records per class (packed)
        uint32_t cpre1 = 0, cpre2 = 0, cpre3 = 0;  // and in the classes below 1, 2 and 3
        // one copy of the chunk's code for cached and one for uncached points
        // (a run-time choice inside the loops below would make every wait
        // for LDS also wait for global memory)
        auto chunk = [&](auto cached_c) {
            constexpr bool cached = decltype(cached_c)::value;
            if (cached) {
                // (the previous chunk's walk is over: its last barrier came after it)
                if (i0 <= npts) s_pc.off[i0] = pf0;
                if (i1 <= npts) s_pc.off[i1] = pf1;
                if (i2 <= npts) s_pc.off[i2] = pf2;
                if (i0 < npts) {
                    s_pc.pay[i0] = py0;
                    s_pc.wv[i0] = pw0;
                    s_pc.inst[i0] = pn0;
#pragma unroll
                    for (int ax = 0; ax < NAX; ++ax) s_pc.rank[ax][i0] = pr0[ax];
                }
                if (i1 < npts) {
                    s_pc.pay[i1] = py1;
                    s_pc.wv[i1] = pw1;
                    s_pc.inst[i1] = pn1;
#pragma unroll
                    for (int ax = 0; ax < NAX; ++ax) s_pc.rank[ax][i1] = pr1[ax];
                }
                // each point marks the threads whose first record (o0 + ITEMS t)
                // it holds: records [fs, fe), low words, taken relative to o0
                auto mark = [&](uint32_t i, uint32_t fs, uint32_t fe) {
                    const int32_t ds = (int32_t)(fs - (uint32_t)o0), de = (int32_t)(fe - (uint32_t)o0);
                    const int32_t tlo = ds <= 0 ? 0 : (ds + ITEMS - 1) / ITEMS;
                    int32_t thi = de <= 0 ? 0 : (de + ITEMS - 1) / ITEMS;
                    if (thi > BLOCK) thi = BLOCK;
                    for (int32_t t = tlo; t < thi; ++t) s_tfirst[t] = (uint16_t)i;
                };
                if (i0 < npts) mark(i0, pf0, pg0);
                if (i1 < npts) mark(i1, pf1, pg1);
            }
            // (thread q < classes) records of class q in the chunks before this one
            const uint32_t coff = pcoff;
            __syncthreads();  // point cache written; every thread done with the previous chunk's staging
            // (the uncached reads are 64-bit: a select between the LDS and the
            // global address would make one flat load, which waits on both)
            const uint32_t obase = cached ? s_pc.off[0] : (uint32_t)a.off[klo];
            auto offr = [&](uint32_t i) -> uint32_t {
                return (cached ? s_pc.off[i] : (uint32_t)a.off[klo + i]) - obase;
            };

            const uint64_t r0 = o0 + (uint64_t)threadIdx.x * ITEMS;
            PointWalk<NAX> pw;
            uint32_t idx = 0, left = 0;
            if (r0 < o1) {
                const uint32_t rel = (uint32_t)r0 - obase;
                if (cached) {
                    idx = s_tfirst[threadIdx.x];
                } else {
                    uint32_t lo = 0, hi = npts;  // offr(lo) <= rel < offr(hi)
                    while (hi - lo > 1) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (offr(mid) <= rel) lo = mid; else hi = mid;
                    }
                    idx = lo;
                }
                pw.load(a, &s_pc, cached, klo, idx, lsingle);
                const uint32_t t = rel - offr(idx);
                left = offr(idx + 1) - offr(idx) - t;  // records left in this point
                pw.seek(t);
            }

            // With classes: this thread's records per class, from its points
            // (before they are produced), scanned over the block.  That gives
            // each record's slot in the class-split staging and the chunk's
            // counts per class.
            uint64_t mine = 0, expect = 0;
            if constexpr (CLS) {
                if (r0 < o1) {
                    uint32_t need = (uint32_t)((o1 - r0) < (uint64_t)ITEMS ? (o1 - r0) : (uint64_t)ITEMS);
                    uint32_t k = idx, ta = offr(idx + 1) - offr(idx) - left;
                    while (need) {
                        const uint32_t pcnt = offr(k + 1) - offr(k);
                        const uint32_t tb = (pcnt - ta < need) ? pcnt : ta + need;
                        if (tb > ta) {
                            uint32_t rk[NAX > 0 ? NAX : 1];
                            uint32_t pay, ins = 0;
                            if (cached) {
                                pay = s_pc.pay[k];
                                if (with_inst) ins = s_pc.inst[k];
#pragma unroll
                                for (int ax = 0; ax < NAX; ++ax) rk[ax] = s_pc.rank[ax][k];
                            } else {
                                pay = a.pay[klo + k];
                                if (with_inst) ins = a.inst_s[klo + k];
#pragma unroll
                                for (int ax = 0; ax < NAX; ++ax) rk[ax] = a.rs[(uint64_t)ax * a.n + klo + k];
                            }
                            expect += point_class_counts<NAX>(a, pay, rk, ins, ta, tb);
                            need -= tb - ta;
                        }
                        ++k;
                        ta = 0;
                    }
                }
                mine = block_excl_sum_packed<BLOCK>(expect, s_scan, &tot);
                cpre1 = packed_prefix(tot, 1);
                cpre2 = packed_prefix(tot, 2);
                cpre3 = packed_prefix(tot, 3);
                // destination of the chunk's first staged record of each class,
                // minus its staging position
                if (threadIdx.x < (unsigned)a.ncls) {
                    const int q = threadIdx.x;
                    const uint64_t cd = s_cls_base[q] + coff - packed_prefix(tot, q);
                    s_cdst[q] = cd;
                    if (a.pk_a) {
                        uint64_t *const out = ((cls_info >> (16 * q + 8)) & 1u) ? a.pk_a : a.pk_b;
                        const bool in = cd < a.E;  // (always, unless the class totals were wrong)
                        s_cptr[q] = in ? out + cd : out;
                        s_clim[q] = in ? (uint32_t)((a.E - cd) < (uint64_t)CHUNK ? (a.E - cd) : (uint64_t)CHUNK) : 0u;
                    }
                }
            }

            // (thread 0) the next chunk's point range: loaded now, passed on
            // through LDS once this chunk's records are produced
            uint32_t tlo = 0, thi = 0;
            if (threadIdx.x == 0 && cn < nchunks) {
                tlo = chunk_lo(cn);
                thi = chunk_hi(cn);
            }
            uint64_t seen = 0;  // records produced per class (checked against the expectation)
#pragma unroll 1
            for (int j = 0; j < ITEMS; ++j) {
                const bool valid = r0 + j < o1;
                K key = 0;
                if (valid) {
                    key = pw.template key<K>(a.field_shift);
                    uint32_t lp = threadIdx.x * ITEMS + j;
                    if constexpr (CLS) {
                        const int q = key_class((key & kmask) >> a.sort_lo, a.cls_c0, a.rbits);
                        // (the prefix of class q as a sum of masked steps: selects, no branches)
                        const uint32_t pre = (cpre1 & (0u - (uint32_t)(q > 0))) +
                                             ((cpre2 - cpre1) & (0u - (uint32_t)(q > 1))) +
                                             ((cpre3 - cpre2) & (0u - (uint32_t)(q > 2)));
                        lp = pre + ((uint32_t)(mine >> (16 * q)) & 0xffffu);
                        mine += 1ull << (16 * q);
                        seen += 1ull << (16 * q);
                    }
                    if (lp < (uint32_t)CHUNK) {
                        s_keys[lp] = key;
                        s_pay[lp] = pw.payload;
                    }
                    my_data += pw.isq ? 0u : 1u;
                    if (--left) {
                        pw.next();
                    } else if (r0 + j + 1 < o1) {
                        // next point with records (points without records have equal offsets)
                        do {
                            ++idx;
                            left = offr(idx + 1) - offr(idx);
                        } while (left == 0);
                        pw.load(a, &s_pc, cached, klo, idx, lsingle);
                    }
                }
                // (the digits the sort reads: above the instance bits of a batch)
                const K hkey = (key & kmask) >> a.sort_lo;
                if constexpr (!CLS) {
                    if (rows) hist_add(s_hist, hkey, valid, a.passes, peel_from, a.rbits);
                } else {
                    const int q = valid ? key_class(hkey, a.cls_c0, a.rbits) : 0;
                    const uint32_t ci = (uint32_t)(cls_info >> (16 * q));
                    if (rows)
                        hist_add_rows_skew(s_hist, hkey, valid, (int)(ci & 0xffu), (int)((ci >> 8) & 0xffu),
                                           a.passes, a.skew, a.rbits);
                }
            }
            if constexpr (CLS) {
                if (seen != expect) atomicOr(a.error, 1u);  // records disagree with the class counts: reported
            }
            if (threadIdx.x == 0) {
                s_next[0] = tlo;
                s_next[1] = thi;
            }
        };
        if (npts <= kCap) chunk(std::true_type{});
        else chunk(std::false_type{});
        __syncthreads();  // staging complete
        nklo = s_next[0];
        nkhi = s_next[1];
        // the next chunk's points, loaded while this chunk's records are stored
        if (cn < nchunks) prefetch(cn, nklo, nkhi);
        if (a.pk_a) {
            // packed records: one 64-bit word per record (the payload kind is
            // uniform, so each kind gets a loop of its own)
            auto store_packed = [&](auto labels_c) {
                constexpr bool LABELS = decltype(labels_c)::value;
                for (uint32_t i = threadIdx.x; i < nrec; i += BLOCK) {
                    const uint64_t w = pack_record(s_keys[i], s_pay[i], a.pk_shift, LABELS);
                    if constexpr (CLS) {
                        const int q = (int)(a.ncls > 1 && i >= cpre1) + (int)(a.ncls > 2 && i >= cpre2) +
                                      (int)(a.ncls > 3 && i >= cpre3);
                        if (i >= s_clim[q]) continue;  // only if the class totals were wrong
                        // (a pointer read from LDS: taken as global memory, so the
                        // store is a global one and not a flat one)
                        using GPtr = __attribute__((address_space(1))) uint64_t *;
                        ((GPtr)s_cptr[q])[i] = w;
                    } else {
                        if (o0 + i >= a.E) continue;
                        a.pk_a[o0 + i] = w;
                    }
                }
            };
            if (a.pk_labels) store_packed(std::true_type{});
            else store_packed(std::false_type{});
        } else if constexpr (!CLS) {
            for (uint32_t i = threadIdx.x; i < nrec; i += BLOCK) {
                keys_a[o0 + i] = s_keys[i];
                vals_a[o0 + i] = s_pay[i];
            }
        } else {
            for (uint32_t i = threadIdx.x; i < nrec; i += BLOCK) {
                const int q = (int)(a.ncls > 1 && i >= cpre1) + (int)(a.ncls > 2 && i >= cpre2) +
                              (int)(a.ncls > 3 && i >= cpre3);
                const uint64_t dst = s_cdst[q] + i;
                if (dst >= a.E) continue;  // only if the class totals were wrong
                if ((cls_info >> (16 * q + 8)) & 1u) {
                    keys_a[dst] = s_keys[i];
                    vals_a[dst] = s_pay[i];
                } else {
                    keys_b[dst] = s_keys[i];
                    vals_b[dst] = s_pay[i];
                }
            }
        }
        klo = nklo;
        khi = nkhi;
    }
    __syncthreads();
    if (rows) hist_flush(s_hist, a.hist_part, rows);
    if (my_data) atomicAdd(&s_data, (unsigned long long)my_data);
    __syncthreads();
    if (threadIdx.x == 0 && s_data) atomicAdd(a.data_records, s_data);
}

// ---------------------------------------------------------------------------
// Regrouping (Sec. 4: the sort by ID and the scan tagged by ID).  Every
// partial aggregate of a point goes to a place of its own that depends only
// on the point and on the record's tuple of tree levels (j_1, ..., j_{m-1}),
// read off the key (the level of node (1 << j) | prefix is its highest set
// bit): a point has at most one record per level tuple, and one exactly when
// every j_a is a 1-digit of its axis-a rank (a query) or a 0-digit (a data
// point).  The scan stores each partial with a plain store, and a second pass
// folds each point's partials in level-tuple order -- no atomics, and the
// same fold order on every run.  Two layouts of those places:
//   slot mode     part[slot][row], slot = the level tuple in mixed radix over
//                 the per-axis field widths (all tuples, valid or not): no
//                 per-point state is read while scanning;
//   compact mode  part[base(row) + t], t = the record's index among the
//                 point's records (the valid tuples in the same order), base
//                 = exclusive sum of the record counts of the rows before it:
//                 exactly one place per record, for wide tables that would be
//                 mostly empty (m = 4 with wide ranks).

struct SlotMap {
    int nax;
    int field_shift[3];
    uint32_t field_mask[3];
    uint32_t radix[3];
    uint32_t n_slots;  // product of the radices; stores to slots beyond it are dropped
    template <class K>
    __device__ __forceinline__ uint32_t level(K key, int a) const {
        const uint32_t node = (uint32_t)(key >> field_shift[a]) & field_mask[a];
        return 31u - (uint32_t)__clz(node);
    }
    template <class K>
    __device__ __forceinline__ uint32_t slot(K key) const {
        uint32_t sl = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (a < nax) sl = sl * radix[a] + level(key, a);
        return sl;
    }
    // Compact mode.  st = {base, fa_1, fa_2, fa_3} of the record's point:
    // fa_a holds the digits of the axis-a rank that select prefixes (1-digits
    // for a query, 0-digits for a data point), left-aligned (digit j at bit
    // 31 - j).  On axis a the record is the t_a-th selected digit from the top
    // (t_a = selected digits above its level); the point's records are
    // numbered in mixed radix over the per-axis counts, first axis slowest,
    // which is the order of the flat map's walk and of the level tuples.
    template <class K>
    __device__ __forceinline__ uint64_t compact(K key, const uint4 &st) const {
        const uint32_t fa[3] = {st.y, st.z, st.w};
        uint32_t t = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (a < nax) {
                const uint32_t j = level(key, a);
                const uint32_t c = (uint32_t)__popc(fa[a]);
                const uint32_t ta = j ? (uint32_t)__popc(fa[a] >> (32u - j)) : 0u;
                t = t * c + ta;
            }
        }
        return (uint64_t)st.x + t;
    }
};

// Records per point of the compact layout: product over axes of the
// selected digits.
__device__ __forceinline__ uint32_t compact_count(const uint4 &st, int nax) {
    uint32_t c = 1;
    const uint32_t fa[3] = {st.y, st.z, st.w};
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (a < nax) c *= (uint32_t)__popc(fa[a]);
    return c;
}

enum { OP_SUM = 0, OP_MAX = 1, OP_COUNT = 2 };

template <class V>
__device__ __forceinline__ V lowest();
template <> __device__ __forceinline__ int32_t lowest<int32_t>() { return INT32_MIN; }
template <> __device__ __forceinline__ int64_t lowest<int64_t>() { return INT64_MIN; }
template <> __device__ __forceinline__ float lowest<float>() { return -__builtin_inff(); }
template <> __device__ __forceinline__ double lowest<double>() { return -__builtin_inf(); }

// The value F is accumulated in: the output type, except fp32 sums, which
// carry a compensated pair (F32c) through the scans and the fold.
template <class Out, int OP>
struct AccumOf {
    using type = Out;
};
template <>
struct AccumOf<float, OP_SUM> {
    using type = F32c;
};

template <class A, int OP>
struct Monoid {
    __device__ static A identity() {
        if constexpr (OP == OP_MAX) return lowest<A>();
        else return A(0);
    }
    __device__ static A combine(A a, A b) {
        if constexpr (OP == OP_MAX) return b > a ? b : a;
        else return a + b;
    }
};
template <>
struct Monoid<F32c, OP_SUM> {
    __device__ static F32c identity() { return F32c{0.0f, 0.0f}; }
    __device__ static F32c combine(F32c a, F32c b) { return f32c_add(a, b); }
};

template <class A, class X>
__device__ __forceinline__ A acc_from(X x) {
    if constexpr (std::is_same<A, F32c>::value) return F32c{(float)x, 0.0f};
    else return A(x);
}
template <class Out, class A>
__device__ __forceinline__ Out acc_out(A a) {
    if constexpr (std::is_same<A, F32c>::value) return (Out)(a.hi + a.lo);
    else return (Out)a;
}

// The sorted records as the scans read them: two arrays (key, 32-bit
// payload), or one array of packed 64-bit words (key above pay_bits payload
// bits).  Packed label payloads (plan records) keep the query flag in their
// top payload bit and are returned in the 32-bit form (kQueryFlag | row);
// packed weight payloads (records that carry weights) take all 32 bits.
// PK (the layout) and LABELS (the payload kind) are compile-time choices:
// a run-time branch inside the scans' load loops made the compiler wait for
// every load before the next one was issued.  The records are read once per
// scan, so the loads are non-temporal: they leave L2 to the lines of the
// scattered partial stores, whose bytes combine there (forward scan at
// f32_2d_16m 2.69 -> 2.65 ms).
template <class K, bool PK>
struct RecSrc {
    const K *keys;
    const uint32_t *vals;
    const uint64_t *packed;
    int pay_bits;   // packed: payload bits (32 for weight payloads)
    template <bool LABELS = true>
    __device__ __forceinline__ void get(uint64_t i, K &k, uint32_t &pay) const {
        if constexpr (PK) {
            const uint64_t w = __builtin_nontemporal_load(&packed[i]);
            k = (K)(w >> pay_bits);
            if constexpr (LABELS) {
                const uint32_t row = (uint32_t)w & ((1u << (pay_bits - 1)) - 1u);
                pay = ((w >> (pay_bits - 1)) & 1u) ? (kQueryFlag | row) : row;
            } else {
                pay = (uint32_t)w;
            }
        } else {
            k = __builtin_nontemporal_load(&keys[i]);
            pay = __builtin_nontemporal_load(&vals[i]);
        }
    }
};

// Where a scan puts the partial aggregates of one kind of point (queries in
// the forward, data in the backward; both in the forward that also reports
// data totals).  part == null: not stored.
template <class Out>
struct PartDest {
    Out *part;
    const uint4 *cstate;  // compact mode: [rows] state of the rows, or null (slot mode)
    uint64_t stride;      // rows (slot mode)
    uint64_t cap;         // entries of part: stores at or beyond it are dropped
    template <class K, class A>
    __device__ __forceinline__ void store(const SlotMap &sm, K key, uint32_t row, A v) const {
        if (!part || row >= stride) return;  // (rows are below stride by construction)
        uint64_t at;
        if (cstate) {
            at = sm.compact(key, cstate[row]);
        } else {
            const uint32_t sl = sm.slot(key);
            at = (uint64_t)sl * stride + row;
        }
        if (at < cap) part[at] = acc_out<Out>(v);
    }
};

// Forward: the segmented scan of the weights over the sorted records.
// Segments are runs of equal keys (the bitstring tuple, Sec. 5).  Queries
// carry the unit e; at a query record the scan value is F over the data
// records before it in its segment, i.e. over the data points that share
// this tuple and lie strictly below it on the last axis.  Each such partial
// goes to its place of the regrouping (q); with dq.part set, the inclusive
// value at every data record goes to its place too (the partial aggregates
// the construction also carries at data records).  Payloads and w use the
// internal numbering of the points.
//
// INL: the records carry the weights (a data record's payload is its weight
// bits, a query record's key has bit flag_shift set and its payload is the
// query's row), so the scan reads them in sequence instead of gathering.
template <class K, class W, class Out, int OP, bool INL = false, bool PK = false>
struct ForwardProblem {
    using V = typename AccumOf<Out, OP>::type;
    struct Raw {
        K key;
        uint32_t payload;
    };
    RecSrc<K, PK> rec;
    const W *w;  // unused for COUNT and INL
    PartDest<Out> q, d;
    uint64_t nw;     // weights (|D|): payloads are checked against it
    SlotMap sm;
    int flag_shift;  // INL

    __device__ bool is_query(const Raw &r) const {
        if constexpr (INL) return ((r.key >> flag_shift) & K(1)) != K(0);
        else return (r.payload & kQueryFlag) != 0u;
    }
    __device__ V identity() const { return Monoid<V, OP>::identity(); }
    __device__ V combine(V a, V b) const { return Monoid<V, OP>::combine(a, b); }
    __device__ Raw load(uint64_t i) const {
        Raw r;
        rec.template get<!INL>(i, r.key, r.payload);  // (records carrying weights hold raw weight bits)
        return r;
    }
    __device__ bool head(const Raw &prev, const Raw &cur) const {
        if constexpr (INL) return ((prev.key ^ cur.key) & ~(K(1) << flag_shift)) != K(0);
        else return prev.key != cur.key;
    }
    __device__ V value(const Raw &, bool, const Raw &cur, uint64_t) const {
        if (is_query(cur)) return identity();
        if constexpr (OP == OP_COUNT) {
            return V(1);
        } else if constexpr (INL) {
            static_assert(sizeof(W) == 4, "");
            W x;
            __builtin_memcpy(&x, &cur.payload, 4);
            return acc_from<V>(x);
        } else {
            return cur.payload < nw ? acc_from<V>(w[cur.payload]) : identity();  // (always below |D|)
        }
    }
    __device__ void emit(uint64_t, const Raw &cur, V, V, V incl, bool) const {
        if (is_query(cur)) {
            q.store(sm, cur.key, INL ? cur.payload : (cur.payload & ~kQueryFlag), incl);
        } else if constexpr (!INL) {
            d.store(sm, cur.key, cur.payload, incl);
        }
    }
};

// Backward of the sum: the same records scanned from the end.  Queries carry
// grad_out, data carry 0; at a data record the exclusive value is the sum of
// grad_out over the queries after it in its segment, i.e. the queries sharing
// the tuple and lying strictly above it on the last axis (equal last
// coordinates put queries first, so they come before the data record and are
// not counted).  Those partials go to the data point's places of the
// regrouping (internal numbering).
template <class K, class G, bool PK = false>
struct BackwardProblem {
    using V = typename AccumOf<G, OP_SUM>::type;
    struct Raw {
        K key;
        uint32_t payload;
    };
    RecSrc<K, PK> rec;
    const G *g;
    PartDest<G> d;
    uint64_t ng;  // |Q|
    SlotMap sm;
    uint64_t E;

    __device__ V identity() const { return Monoid<V, OP_SUM>::identity(); }
    __device__ V combine(V a, V b) const { return Monoid<V, OP_SUM>::combine(a, b); }
    __device__ Raw load(uint64_t i) const {
        Raw r;
        rec.template get<true>(E - 1 - i, r.key, r.payload);
        return r;
    }
    __device__ bool head(const Raw &prev, const Raw &cur) const { return prev.key != cur.key; }
    __device__ V value(const Raw &, bool, const Raw &cur, uint64_t) const {
        if (!(cur.payload & kQueryFlag)) return identity();
        const uint32_t q = cur.payload & ~kQueryFlag;
        return q < ng ? acc_from<V>(g[q]) : identity();  // (always below |Q|)
    }
    __device__ void emit(uint64_t, const Raw &cur, V, V excl, V, bool) const {
        if (cur.payload & kQueryFlag) return;
        d.store(sm, cur.key, cur.payload, excl);
    }
};

// Folds each row's partials in level-tuple order: out[inv[o]] = F over the
// partials of row o (point slot_base + o).
struct RegroupArgs {
    const uint32_t *inv;           // [nout]: output index of row o, or null (identity)
    const uint32_t *rank;          // [nax][n] by point slot (slot mode)
    const uint32_t *inst_of_slot;  // [n] or null (slot mode)
    const uint8_t *ltab;           // [nax][n_inst] (slot mode)
    const uint4 *cstate;           // [nout] state of the rows (compact mode)
    uint64_t cap;                  // entries of the compact table
    uint32_t n, n_inst;
    uint32_t slot_base;
    uint32_t digit;
    uint32_t radix[3];
    uint64_t nout;
};

// Slot mode: a row's valid slots are the level tuples whose digits of the
// point's ranks equal `digit` (1 for queries, 0 for data) and lie below the
// instance's widths.
template <class Out, int OP, int NAX>
__global__ __launch_bounds__(256) void regroup_kernel(RegroupArgs a, const Out *__restrict__ part,
                                                      Out *__restrict__ out) {
    using A = typename AccumOf<Out, OP>::type;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t o = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; o < a.nout; o += stride) {
        const uint32_t s = a.slot_base + (uint32_t)o;
        const uint32_t ins = a.inst_of_slot ? a.inst_of_slot[s] : 0u;
        uint32_t x[3] = {0, 0, 0}, L[3] = {0, 0, 0};
#pragma unroll
        for (int ax = 0; ax < NAX; ++ax) {
            const uint32_t r = a.rank[(uint64_t)ax * a.n + s];
            L[ax] = a.ltab[(uint64_t)ax * a.n_inst + (ins < a.n_inst ? ins : 0u)];
            x[ax] = a.digit ? r : ~r;
        }
        // digit j of the L-digit string x, counted from the top, is bit L-1-j
        auto ok = [&](int ax, uint32_t j) { return j < L[ax] && ((x[ax] >> (L[ax] - 1u - j)) & 1u); };
        A acc = Monoid<A, OP>::identity();
        auto add = [&](Out v) { acc = Monoid<A, OP>::combine(acc, acc_from<A>(v)); };
        if constexpr (NAX == 0) {
            add(part[o]);
        } else if constexpr (NAX == 1) {
            // 8 slots per round, loaded before any is folded, folded in
            // slot order as above; only valid slots are loaded (neighbouring
            // rows share their high rank digits, so whole lines of invalid
            // partials are never fetched)
            constexpr uint32_t kU = 8;
            const uint32_t R = a.radix[0];
            for (uint32_t j0 = 0; j0 < R; j0 += kU) {
                Out v[kU];
                bool use[kU];
#pragma unroll
                for (uint32_t u = 0; u < kU; ++u) {
                    use[u] = j0 + u < R && ok(0, j0 + u);
                    v[u] = use[u] ? part[(uint64_t)(j0 + u) * a.nout + o] : Out();
                }
#pragma unroll
                for (uint32_t u = 0; u < kU; ++u)
                    if (use[u]) add(v[u]);
            }
        } else if constexpr (NAX == 2) {
            // per first-axis level, the second axis's slots 8 at a time as above
            constexpr uint32_t kU = 8;
            const uint32_t R1 = a.radix[1];
            for (uint32_t j0 = 0; j0 < a.radix[0]; ++j0) {
                if (!ok(0, j0)) continue;
                const Out *row = part + (uint64_t)j0 * R1 * a.nout + o;
                for (uint32_t j1 = 0; j1 < R1; j1 += kU) {
                    Out v[kU];
                    bool use[kU];
#pragma unroll
                    for (uint32_t u = 0; u < kU; ++u) {
                        use[u] = j1 + u < R1 && ok(1, j1 + u);
                        v[u] = use[u] ? row[(uint64_t)(j1 + u) * a.nout] : Out();
                    }
#pragma unroll
                    for (uint32_t u = 0; u < kU; ++u)
                        if (use[u]) add(v[u]);
                }
            }
        } else {
            for (uint32_t j0 = 0; j0 < a.radix[0]; ++j0) {
                const bool v0 = ok(0, j0);
                for (uint32_t j1 = 0; j1 < a.radix[1]; ++j1) {
                    const bool v1 = v0 && ok(1, j1);
                    for (uint32_t j2 = 0; j2 < a.radix[2]; ++j2)
                        if (v1 && ok(2, j2))
                            add(part[(((uint64_t)j0 * a.radix[1] + j1) * a.radix[2] + j2) * a.nout + o]);
                }
            }
        }
        const uint64_t dst = a.inv ? (uint64_t)a.inv[o] : o;
        if (dst < a.nout) out[dst] = acc_out<Out>(acc);  // (inv is a permutation of the rows)
    }
}

// Compact mode: row o's partials are part[base, base + count) in level-tuple
// order.  One wavefront folds one row: lane l takes partials l, l + 64, ...
// of the run in order (the wavefront's loads are consecutive), then the
// lanes' values are combined by a butterfly over lane distances 32, 16, ..,
// 1.  The grouping depends only on the run's length, so results repeat bit
// for bit; every F here is commutative (fp32 sums through F32c, whose
// addition is symmetric), so both lanes of a butterfly pair hold the same
// value.
template <class A>
__device__ __forceinline__ A lane_xor(A v, int mask) {
    const int src = lane_id() ^ mask;
    if constexpr (std::is_same<A, F32c>::value) {
        return F32c{__uint_as_float(read_lane_u32(__float_as_uint(v.hi), src)),
                    __uint_as_float(read_lane_u32(__float_as_uint(v.lo), src))};
    } else if constexpr (sizeof(A) == 8) {
        uint64_t u;
        __builtin_memcpy(&u, &v, 8);
        u = read_lane_u64(u, src);
        A r;
        __builtin_memcpy(&r, &u, 8);
        return r;
    } else {
        static_assert(sizeof(A) == 4, "");
        uint32_t u;
        __builtin_memcpy(&u, &v, 4);
        u = read_lane_u32(u, src);
        A r;
        __builtin_memcpy(&r, &u, 4);
        return r;
    }
}

template <class Out, int OP>
__global__ __launch_bounds__(256) void regroup_compact_kernel(RegroupArgs a, int nax, const Out *__restrict__ part,
                                                              Out *__restrict__ out) {
    using A = typename AccumOf<Out, OP>::type;
    const int lane = lane_id();
    const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x / kWave);
    // every lane of a wavefront takes the same rows (the butterfly below)
    for (uint64_t o = (uint64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; o < a.nout; o += nwaves) {
        const uint4 st = a.cstate[o];
        const uint32_t cnt = compact_count(st, nax);
        uint64_t end = (uint64_t)st.x + cnt;
        if (end > a.cap) end = a.cap;  // (counts add up to the table size by construction)
        A acc = Monoid<A, OP>::identity();
        uint64_t i = (uint64_t)st.x + (uint64_t)lane;
        // 4 partials per lane and round, loaded before any is folded
        for (; i + 3 * kWave < end; i += 4 * kWave) {
            Out v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = part[i + (uint64_t)u * kWave];
#pragma unroll
            for (int u = 0; u < 4; ++u) acc = Monoid<A, OP>::combine(acc, acc_from<A>(v[u]));
        }
        for (; i < end; i += kWave) acc = Monoid<A, OP>::combine(acc, acc_from<A>(part[i]));
#pragma unroll
        for (int m = kWave / 2; m >= 1; m >>= 1) acc = Monoid<A, OP>::combine(acc, lane_xor(acc, m));
        if (lane == 0) {
            const uint64_t dst = a.inv ? (uint64_t)a.inv[o] : o;
            if (dst < a.nout) out[dst] = acc_out<Out>(acc);  // (inv is a permutation of the rows)
        }
    }
}

// State of the compact layout for every point slot: {base, fa_1, fa_2, fa_3}
// (see SlotMap::compact), base = exclusive sum of the record counts of the
// slots before it of the same kind (queries: slots < nQ; data: the rest), as a
// segmented scan restarted at slot nQ.  fa_a = the selecting digits of the
// axis-a rank, left-aligned: a query selects its 1-digits, a data point its
// 0-digits (Lemma 2's prefix sets P1 and P0), over the L_a digits of its
// instance.
struct CompactStateProblem {
    using V = uint64_t;
    using Raw = uint32_t;
    const uint32_t *rank;          // [nax][n] by slot
    const uint32_t *inst_of_slot;  // [n] or null
    const uint8_t *ltab;           // [nax][n_inst]
    uint32_t n, nQ, n_inst;
    int nax;
    uint4 *cstate;                 // [n]

    __device__ uint4 state(uint32_t s) const {
        const uint32_t ins = inst_of_slot ? inst_of_slot[s] : 0u;
        const bool isq = s < nQ;
        uint32_t fa[3] = {0, 0, 0};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (a < nax) {
                const uint32_t L = ltab[(uint64_t)a * n_inst + (ins < n_inst ? ins : 0u)];
                const uint32_t r = rank[(uint64_t)a * n + s];
                const uint32_t mask = L >= 32u ? 0xffffffffu : ((1u << L) - 1u);
                const uint32_t full = (isq ? r : ~r) & mask;
                fa[a] = L ? full << (32u - L) : 0u;
            }
        }
        return make_uint4(0u, fa[0], fa[1], fa[2]);
    }
    __device__ V identity() const { return 0ull; }
    __device__ V combine(V a, V b) const { return a + b; }
    __device__ Raw load(uint64_t i) const { return (uint32_t)i; }
    __device__ bool head(const Raw &, const Raw &cur) const { return cur == nQ; }
    __device__ V value(const Raw &, bool, const Raw &cur, uint64_t) const {
        return compact_count(state(cur), nax);
    }
    __device__ void emit(uint64_t, const Raw &cur, V, V excl, V, bool) const {
        uint4 st = state(cur);
        st.x = (uint32_t)excl;
        cstate[cur] = st;
    }
};

}  // namespace domagg

namespace domagg {

// ---------------------------------------------------------------------------
// The final list of Sec. 4 (instructions 6m+6 .. 6m+9): every record once,
// in nondecreasing ID order (data row i has ID i, query row j has ID
// |D| + j), each carrying the total of its ID -- the query's result, or for
// a data point F over the partial aggregates at its own records.

// inv[perm[i]] = i (perm a permutation of [0, n); other indices dropped).
__global__ void invert_perm_kernel(const uint32_t *__restrict__ perm, uint64_t n, uint32_t *__restrict__ inv) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t p = perm[i];
        if (p < n) inv[p] = (uint32_t)i;
    }
}

// Records per ID (the size of the point's product of prefix sets) and their
// exclusive sums: off[id] = the list position of ID id's first entry,
// off[n] = E.
struct IdCountProblem {
    using V = uint64_t;
    using Raw = uint32_t;
    const uint32_t *drow_pos;      // [nD] internal position of each data row, or null (identity)
    const uint32_t *qrow_pos;      // [nQ] likewise for queries
    const uint32_t *rank;          // [nax][n] by internal slot
    const uint32_t *inst_of_slot;  // [n] or null
    const uint8_t *ltab;           // [nax][n_inst]
    uint32_t n, nD, nQ, n_inst;
    int nax;
    uint64_t *off;                 // [n + 1]

    __device__ V identity() const { return 0ull; }
    __device__ V combine(V a, V b) const { return a + b; }
    __device__ Raw load(uint64_t i) const { return (uint32_t)i; }
    __device__ bool head(const Raw &, const Raw &) const { return false; }
    __device__ V value(const Raw &, bool, const Raw &id, uint64_t) const {
        const bool isq = id >= nD;
        uint32_t slot;
        if (isq) {
            const uint32_t j = id - nD;
            slot = qrow_pos ? qrow_pos[j] : j;
        } else {
            slot = nQ + (drow_pos ? drow_pos[id] : id);
        }
        if (slot >= n) return 0ull;  // (positions are below |D| and |Q| by construction)
        const uint32_t ins = inst_of_slot ? inst_of_slot[slot] : 0u;
        uint64_t c = 1;
        for (int a = 0; a < nax; ++a) {
            const uint32_t r = rank[(uint64_t)a * n + slot];
            const uint32_t L = ltab[(uint64_t)a * n_inst + (ins < n_inst ? ins : 0u)];
            const uint32_t pc = (uint32_t)__popc(r);
            c *= isq ? pc : (L > pc ? L - pc : 0u);
        }
        return c;
    }
    __device__ void emit(uint64_t i, const Raw &, V, V excl, V incl, bool) const {
        off[i] = excl;
        if (i == (uint64_t)n - 1) off[n] = incl;
    }
};

// ids[off[id] .. off[id + 1]) = id.
__global__ void id_fill_kernel(const uint64_t *__restrict__ off, uint32_t n, uint64_t cap,
                               int64_t *__restrict__ ids) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; id < n; id += stride) {
        uint64_t hi = off[id + 1];
        if (hi > cap) hi = cap;  // (off[n] = E = cap by construction)
        for (uint64_t i = off[id]; i < hi; ++i) ids[i] = (int64_t)id;
    }
}

// Instructions 6m+7 .. 6m+9 over the list sorted by ID: H = the IDs shifted
// right by one; the value is e wherever the ID equals H (neutral_if_eq),
// else the ID's total (its first entry, where the complete aggregate sits
// after the reversal of 6m+6); the segmented scan tagged by ID then carries
// it to every entry of the run.
template <class Out, int OP>
struct BroadcastProblem {
    using V = typename AccumOf<Out, OP>::type;
    struct Raw {
        int64_t id;
    };
    const int64_t *ids;  // [E]
    const Out *tot_d;    // [nD] totals of the data rows
    const Out *tot_q;    // [nQ] totals of the queries
    uint64_t nD, nQ;
    Out *vals;           // [E]

    __device__ V identity() const { return Monoid<V, OP>::identity(); }
    __device__ V combine(V a, V b) const { return Monoid<V, OP>::combine(a, b); }
    __device__ Raw load(uint64_t i) const { return Raw{ids[i]}; }
    __device__ bool head(const Raw &prev, const Raw &cur) const { return prev.id != cur.id; }
    __device__ V value(const Raw &prev, bool has_prev, const Raw &cur, uint64_t) const {
        if (has_prev && prev.id == cur.id) return identity();  // neutral_if_eq
        const uint64_t id = (uint64_t)cur.id;
        if (id < nD) return acc_from<V>(tot_d[id]);
        if (id - nD < nQ) return acc_from<V>(tot_q[id - nD]);
        return identity();  // (IDs are below |D| + |Q| by construction)
    }
    __device__ void emit(uint64_t i, const Raw &, V, V, V incl, bool) const { vals[i] = acc_out<Out>(incl); }
};

}  // namespace domagg
