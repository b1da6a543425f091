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

// keys[s] = (instance << 32 | ordered coordinate) or the ordered coordinate;
// vals[s] = the point's internal slot, ppos[s] (or s while ppos is not yet
// known).  Fused histogram of `passes` digits; NaN raises *nan_flag.
template <class K, class C, int BLOCK>
__global__ __launch_bounds__(BLOCK) void extract_keys_kernel(
    const C *__restrict__ q, const C *__restrict__ d, int m, int axis, uint32_t nQ, uint32_t n,
    const uint32_t *__restrict__ inst_of_slot, const uint32_t *__restrict__ ppos, K *__restrict__ keys,
    uint32_t *__restrict__ vals, int passes, uint32_t *__restrict__ hist_part, uint32_t *__restrict__ nan_flag) {
    __shared__ uint32_t s_hist[kMaxPasses * kRadix];
    for (int i = threadIdx.x; i < passes * kRadix; i += BLOCK) s_hist[i] = 0;
    __syncthreads();
    bool saw_nan = false;
    const uint64_t stride = (uint64_t)gridDim.x * BLOCK;
    for (uint64_t b = (uint64_t)blockIdx.x * BLOCK; b < n; b += stride) {
        const uint64_t s = b + threadIdx.x;
        const bool valid = s < n;
        K key = 0;
        if (valid) {
            const C x = (s < nQ) ? q[s * m + axis] : d[(s - nQ) * m + axis];
            saw_nan |= is_nan(x);
            key = (K)ordered_key(x);
            if constexpr (sizeof(K) == 8) {
                if (inst_of_slot) key |= (K)inst_of_slot[s] << 32;
            }
            keys[s] = key;
            vals[s] = ppos ? ppos[s] : (uint32_t)s;
        }
        hist_add(s_hist, key, valid, passes);
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
    uint32_t *__restrict__ hist_part, uint32_t *__restrict__ nan_flag) {
    __shared__ uint32_t s_hist[kMaxPasses * kRadix];
    for (int i = threadIdx.x; i < passes * kRadix; i += BLOCK) s_hist[i] = 0;
    __syncthreads();
    bool saw_nan = false;
    const uint64_t stride = (uint64_t)gridDim.x * BLOCK;
    for (uint64_t b = (uint64_t)blockIdx.x * BLOCK; b < n; b += stride) {
        const uint64_t s = b + threadIdx.x;
        const bool valid = s < n;
        K key = 0;
        if (valid) {
            const bool isq = s < nQ;
            const C x = isq ? q[s * 2 + axis] : d[(s - nQ) * 2 + axis];
            saw_nan |= is_nan(x);
            key = (K)ordered_key(x);
            if constexpr (sizeof(K) == 8) {
                if (inst_of_slot) key |= (K)inst_of_slot[s] << 32;
            }
            const uint64_t rs = pr[s];
            const uint32_t sp = (uint32_t)rs, r = (uint32_t)(rs >> 32);
            uint32_t payload;
            if (isq) {
                payload = carry_weights ? sp : (kQueryFlag | sp);
            } else if (carry_weights) {
                payload = 0;
                if (w) __builtin_memcpy(&payload, &w[s - nQ], 4);
            } else {
                payload = sp - nQ;
            }
            keys[s] = key;
            vals[s] = ((uint64_t)((isq ? 0x80000000u : 0u) | r) << 32) | payload;
        }
        hist_add(s_hist, key, valid, passes);
    }
    if (saw_nan) atomicOr(nan_flag, 1u);
    __syncthreads();
    hist_flush(s_hist, hist_part, passes);
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
            if (pr) pr[cur.slot] = ((uint64_t)r << 32) | sp;
            else ppos[cur.slot] = sp;
            rank[sp] = r;
        } else {
            rank[cur.slot] = r;
        }
        if (last) kcount[ins] = (uint32_t)incl;
    }
};

// dst[p] = src[idx[p]]: inputs into internal order.
template <class T>
__global__ void gather_kernel(const T *__restrict__ src, const uint32_t *__restrict__ idx, T *__restrict__ dst,
                              uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) dst[p] = src[idx[p]];
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
        if (w && s >= nQ) __builtin_memcpy(&wb, &w[dinv[s - nQ]], 4);
        rw[s] = (uint64_t)rank0[s] | ((uint64_t)wb << 32);
    }
}

// dst[idx[p]] = src[p]: results back into input order.
template <class T>
__global__ void scatter_kernel(const T *__restrict__ src, const uint32_t *__restrict__ idx, T *__restrict__ dst,
                               uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) dst[idx[p]] = src[p];
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
    __device__ V value(const Raw &, bool, const Raw &cur, uint64_t i) const {
        const bool isq = (cur.v >> 63) != 0;
        const uint32_t r = (uint32_t)(cur.v >> 32) & 0x7fffffffu;
        const uint32_t payload = (uint32_t)cur.v;
        const uint32_t ins = inst(cur);
        if (ins >= n_inst) return 0ull;  // only if the sort were wrong: no records
        const uint32_t L = ltab[ins];
        const uint32_t pc = (uint32_t)__popc(r);
        rs[i] = r;
        if (isq) {
            pay[i] = kQueryFlag | (payload & ~kQueryFlag);
        } else {
            pay[i] = INL ? 0u : payload;
            if (INL) wv[i] = payload;
        }
        if (inst_s) inst_s[i] = ins;
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
    uint64_t cls_base[kMaxClasses];      // region starts
    uint32_t cls_mask[kMaxClasses];      // first-axis levels of each class (bit L-1-j for level j)
    unsigned long long *cls_status;      // [chunks][kMaxClasses] look-back words
    uint32_t *ticket;
    uint32_t *error;                     // set when a chunk's records disagree with its class counts
    // records carrying weights (flag_shift >= 0): a data record's payload is
    // its weight bits wv[k]; a query record's payload is its row and its key
    // has bit flag_shift set (above every digit the sort looks at)
    const uint32_t *wv;
    int flag_shift;
};

// Sum of the 16-bit fields of `packed` below field q (q <= 4).
__device__ __forceinline__ uint32_t packed_prefix(uint64_t packed, int q) {
    const uint64_t x = packed & (q >= 4 ? ~0ull : ((1ull << (16 * q)) - 1ull));
    return (uint32_t)(x & 0xffffu) + (uint32_t)((x >> 16) & 0xffffu) + (uint32_t)((x >> 32) & 0xffffu) +
           (uint32_t)(x >> 48);
}

template <class K>
__device__ __forceinline__ int key_class(K key, int c0) {
    const int bits = (int)(sizeof(K) * 8) - (sizeof(K) == 8 ? __clzll((long long)key) : __clz((int)key));
    const int nominal = (bits + kRadixBits - 1) / kRadixBits;
    return (nominal > c0 ? nominal : c0) - c0;
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
    static constexpr int kCap = 512;
    uint32_t off[kCap + 1];  // record offsets relative to the chunk's first point
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

    __device__ void set(const EmitArgs &a, uint32_t pay, uint32_t wbits, uint32_t ins, const uint32_t *ranks) {
        isq = (pay & kQueryFlag) != 0u;
        payload = a.flag_shift < 0 ? pay : (isq ? (pay & ~kQueryFlag) : wbits);
        inst = ins;
#pragma unroll
        for (int ax = 0; ax < NAX; ++ax) {
            r[ax] = ranks[ax];
            L[ax] = a.ltab[(uint64_t)ax * a.n_inst + inst];
            const uint32_t mask = (L[ax] >= 32u) ? 0xffffffffu : ((1u << L[ax]) - 1u);
            full[ax] = isq ? (r[ax] & mask) : (~r[ax] & mask);
            rem[ax] = full[ax];
        }
    }
    // point k of the chunk (index idx among its points), from the LDS cache or global memory
    __device__ void load(const EmitArgs &a, const PointCache<NAX> *pc, bool cached, uint32_t klo, uint32_t idx) {
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
        set(a, pay, wb, ins, rk);
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
    __device__ K key(int inst_shift, bool with_inst, const int *field_shift, int flag_shift) const {
        K key = with_inst ? ((K)inst << inst_shift) : K(0);
        if (flag_shift >= 0 && isq) key |= K(1) << flag_shift;
#pragma unroll
        for (int ax = 0; ax < NAX; ++ax) {
            const uint32_t top = 31u - (uint32_t)__clz(rem[ax]);  // highest remaining digit
            const uint32_t j = L[ax] - 1u - top;                 // its position from the top
            const uint32_t node = (1u << j) | (j ? (r[ax] >> (L[ax] - j)) : 0u);
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
                                                       uint32_t ta, uint32_t tb) {
    const bool isq = (pay & kQueryFlag) != 0u;
    uint32_t full0 = 0, R = 1;
#pragma unroll
    for (int ax = 0; ax < NAX; ++ax) {
        const uint32_t L = a.ltab[ax];
        const uint32_t mask = L >= 32u ? 0xffffffffu : ((1u << L) - 1u);
        const uint32_t full = isq ? (ranks[ax] & mask) : (~ranks[ax] & mask);
        if (ax == 0) full0 = full;
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

// Records per class over all points (one instance).
template <int NAX>
__global__ __launch_bounds__(256) void class_count_kernel(EmitArgs a, unsigned long long *__restrict__ cls_tot) {
    __shared__ unsigned long long s_tot[kMaxClasses];
    if (threadIdx.x < kMaxClasses) s_tot[threadIdx.x] = 0;
    __syncthreads();
    unsigned long long acc[kMaxClasses] = {0, 0, 0, 0};
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < a.n; k += stride) {
        uint32_t rk[NAX > 0 ? NAX : 1];
#pragma unroll
        for (int ax = 0; ax < NAX; ++ax) rk[ax] = a.rs[(uint64_t)ax * a.n + k];
        const uint64_t pc = point_class_counts<NAX>(a, a.pay[k], rk, 0u, 0xffffffffu);
#pragma unroll
        for (int q = 0; q < kMaxClasses; ++q) acc[q] += (pc >> (16 * q)) & 0xffffu;
    }
#pragma unroll
    for (int q = 0; q < kMaxClasses; ++q)
        if (acc[q]) atomicAdd(&s_tot[q], acc[q]);
    __syncthreads();
    if (threadIdx.x < kMaxClasses && s_tot[threadIdx.x]) atomicAdd(cls_tot + threadIdx.x, s_tot[threadIdx.x]);
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
        const int q = key_class((uint32_t)t, a.cls_c0);
        int row0 = 0;
#pragma unroll
        for (int c = 0; c < kMaxClasses; ++c)
            if (c < q) row0 += a.cls_passes[c];
        int np = a.cls_passes[0];
#pragma unroll
        for (int c = 1; c < kMaxClasses; ++c)
            if (c == q) np = a.cls_passes[c];
        for (int p = 0; p < np; ++p)
            atomicAdd(&s_hist[(row0 + p) * kRadix + ((uint32_t)(t >> (kRadixBits * p)) & (kRadix - 1))], cnt);
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
// A block takes a chunk of CHUNK consecutive records (from a ticket, so that
// every chunk it waits on is held by a running block) and loads the state of
// the chunk's points into LDS with coalesced reads.  Each thread produces
// ITEMS consecutive records (one search for its first, then a walk) and
// stages them in LDS.  Without classes the block then writes them out in
// place.  With classes, each thread first counts its records per class from
// its points (closed form, see point_class_counts); one block scan of those
// counts gives every record its slot in a class-split staging and the
// chunk's counts, which are published before the walk.  After the walk,
// wavefront 0 looks back over earlier chunks for each class's offset and the
// block writes each class's run into its region.  The digit histograms of
// every pass (of every class) are accumulated on the way.

// Adds the digits of `key` for passes [0, np) to histogram rows row0 + p;
// lanes sharing the first active lane's row and digit are added with one
// atomic.  All lanes of the wavefront call it, for max_np passes.
template <class K>
__device__ __forceinline__ void hist_add_rows(uint32_t *s_hist, K key, bool valid, int row0, int np, int max_np) {
    const int lane = lane_id();
    for (int p = 0; p < max_np; ++p) {
        const bool v = valid && p < np;
        const uint64_t act = __ballot(v);
        if (act == 0) continue;
        const int leader = __ffsll((unsigned long long)act) - 1;
        const uint32_t idx = (uint32_t)(row0 + p) * kRadix + ((uint32_t)(key >> (kRadixBits * p)) & (kRadix - 1));
        const uint32_t i0 = read_lane_u32(idx, leader);
        const uint64_t same = __ballot(v && idx == i0);
        if (lane == leader) atomicAdd(&s_hist[i0], (uint32_t)__popcll(same));
        if (v && idx != i0) atomicAdd(&s_hist[idx], 1u);
    }
}

// Exclusive sum of packed 16-bit counters over a block (each field's block
// total must stay below 2^16); *total gets the packed block sums.
template <int BLOCK>
__device__ __forceinline__ uint64_t block_excl_sum_packed(uint64_t v, uint64_t *s_tmp, uint64_t *total) {
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    uint64_t incl = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint64_t o = read_lane_u64(incl, lane >= d ? lane - d : 0);
        if (lane >= d) incl += o;
    }
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

template <class K, int NAX, int BLOCK, int ITEMS, bool CLS>
__global__ __launch_bounds__(BLOCK) void emit_kernel(EmitArgs a, K *__restrict__ keys_a, uint32_t *__restrict__ vals_a,
                                                     K *__restrict__ keys_b, uint32_t *__restrict__ vals_b) {
    constexpr int CHUNK = BLOCK * ITEMS;
    // histogram rows: passes of every class (up to 1+2+3+4 for 32-bit keys)
    constexpr int kRows = CLS ? (sizeof(K) == 4 ? 10 : 26) : kMaxPasses;
    using PC = PointCache<NAX>;
    using DW = DigitWord<unsigned long long>;
    __shared__ PC s_pc;
    __shared__ K s_keys[CHUNK];
    __shared__ uint32_t s_pay[CHUNK];
    __shared__ uint32_t s_hist[kRows * kRadix];
    __shared__ unsigned long long s_data;
    __shared__ uint64_t s_scan[BLOCK / kWave];
    __shared__ uint64_t s_cdst[kMaxClasses];  // destination of the chunk's first slot of each class, minus its run start
    __shared__ uint32_t s_chunk;
    // (with classes the histograms may come from elsewhere: hist_part null)
    const int rows = a.hist_part ? (CLS ? a.hist_rows : a.passes) : 0;
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

    const uint64_t nchunks = (a.E + CHUNK - 1) / CHUNK;
    for (;;) {
        __syncthreads();  // previous chunk done with LDS
        if (threadIdx.x == 0) s_chunk = atomicAdd(a.ticket, 1u);
        __syncthreads();
        const uint64_t c = s_chunk;
        if (c >= nchunks) break;
        const uint64_t o0 = c * CHUNK;
        const uint64_t o1 = (o0 + CHUNK < a.E) ? o0 + CHUNK : a.E;
        const uint32_t klo = a.chunk_k[c];
        const uint32_t khi = (c + 1 < nchunks) ? a.chunk_k[c + 1] : a.n - 1;  // may be one past
        const uint32_t npts = khi - klo + 1;
        const bool cached = npts <= (uint32_t)PC::kCap;
        const uint64_t obase = a.off[klo];
        if (cached) {
            for (uint32_t i = threadIdx.x; i <= npts; i += BLOCK) s_pc.off[i] = (uint32_t)(a.off[klo + i] - obase);
            for (uint32_t i = threadIdx.x; i < npts; i += BLOCK) {
                s_pc.pay[i] = a.pay[klo + i];
                s_pc.wv[i] = a.wv ? a.wv[klo + i] : 0u;
                s_pc.inst[i] = with_inst ? a.inst_s[klo + i] : 0u;
#pragma unroll
                for (int ax = 0; ax < NAX; ++ax) s_pc.rank[ax][i] = a.rs[(uint64_t)ax * a.n + klo + i];
            }
        }
        __syncthreads();
        auto offr = [&](uint32_t i) -> uint32_t {
            return cached ? s_pc.off[i] : (uint32_t)(a.off[klo + i] - obase);
        };
        const uint32_t nrec = (uint32_t)(o1 - o0);

        const uint64_t r0 = o0 + (uint64_t)threadIdx.x * ITEMS;
        PointWalk<NAX> pw;
        uint32_t idx = 0, left = 0;
        if (r0 < o1) {
            const uint32_t rel = (uint32_t)(r0 - obase);
            uint32_t lo = 0, hi = npts;  // offr(lo) <= rel < offr(hi)
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (offr(mid) <= rel) lo = mid; else hi = mid;
            }
            idx = lo;
            pw.load(a, &s_pc, cached, klo, idx);
            const uint32_t t = rel - offr(idx);
            left = offr(idx + 1) - offr(idx) - t;  // records left in this point
            pw.seek(t);
        }

        // With classes: this thread's records per class, from its points
        // (before they are produced), scanned over the block.  That gives
        // each record's slot in the class-split staging and the chunk's
        // counts, which are published at once so that later chunks can look
        // past this one while its records are still being produced.
        uint64_t mine = 0, tot = 0, expect = 0;
        if constexpr (CLS) {
            if (r0 < o1) {
                uint32_t need = (uint32_t)((o1 - r0) < (uint64_t)ITEMS ? (o1 - r0) : (uint64_t)ITEMS);
                uint32_t k = idx, ta = offr(idx + 1) - offr(idx) - left;
                while (need) {
                    const uint32_t pcnt = offr(k + 1) - offr(k);
                    const uint32_t tb = (pcnt - ta < need) ? pcnt : ta + need;
                    if (tb > ta) {
                        uint32_t rk[NAX > 0 ? NAX : 1];
                        uint32_t pay;
                        if (cached) {
                            pay = s_pc.pay[k];
#pragma unroll
                            for (int ax = 0; ax < NAX; ++ax) rk[ax] = s_pc.rank[ax][k];
                        } else {
                            pay = a.pay[klo + k];
#pragma unroll
                            for (int ax = 0; ax < NAX; ++ax) rk[ax] = a.rs[(uint64_t)ax * a.n + klo + k];
                        }
                        expect += point_class_counts<NAX>(a, pay, rk, ta, tb);
                        need -= tb - ta;
                    }
                    ++k;
                    ta = 0;
                }
            }
            mine = block_excl_sum_packed<BLOCK>(expect, s_scan, &tot);
            if (threadIdx.x < (unsigned)a.ncls) {
                const int q = threadIdx.x;
                store_agent(&a.cls_status[c * kMaxClasses + q],
                            DW::make(c == 0 ? kFlagInclusive : kFlagAggregate, (uint32_t)(tot >> (16 * q)) & 0xffffu));
            }
        }

        uint64_t seen = 0;  // records produced per class (checked against the expectation)
#pragma unroll 1
        for (int j = 0; j < ITEMS; ++j) {
            const bool valid = r0 + j < o1;
            K key = 0;
            if (valid) {
                key = pw.template key<K>(a.inst_shift, with_inst, a.field_shift, a.flag_shift);
                uint32_t lp = threadIdx.x * ITEMS + j;
                if constexpr (CLS) {
                    const int q = key_class(key & kmask, a.cls_c0);
                    lp = packed_prefix(tot, q) + ((uint32_t)(mine >> (16 * q)) & 0xffffu);
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
                    pw.load(a, &s_pc, cached, klo, idx);
                }
            }
            if constexpr (!CLS) {
                if (rows) hist_add(s_hist, key, valid, a.passes, peel_from);
            } else {
                const int q = valid ? key_class(key & kmask, a.cls_c0) : 0;
                const uint32_t ci = (uint32_t)(cls_info >> (16 * q));
                if (rows) hist_add_rows(s_hist, key, valid, (int)(ci & 0xffu), (int)((ci >> 8) & 0xffu), a.passes);
            }
        }
        if constexpr (CLS) {
            if (seen != expect) atomicOr(a.error, 1u);  // records disagree with the class counts: reported
            // Class offsets from the chunks before this one, by wavefront 0
            // after its share of the records (by then the chunks before have
            // mostly published inclusive words): lane 16 q + k reads chunk
            // hi - k for class q, 16 chunks per class per round trip; a
            // class's walk ends at the nearest inclusive word (chunk 0
            // publishes one at once).
            if (threadIdx.x < kWave) {
                const int lane = threadIdx.x, q = lane >> 4, k = lane & 15;
                const bool act = q < a.ncls;
                const uint32_t count = act ? ((uint32_t)(tot >> (16 * q)) & 0xffffu) : 0u;
                unsigned long long *st = a.cls_status;
                uint64_t excl = 0;
                bool done = !act || c == 0;
                int64_t hi = (int64_t)c - 1;
                constexpr int kDepth = 4;  // chunks per lane and round trip (loads issued together)
                while (__ballot(!done)) {
                    unsigned long long w[kDepth];
#pragma unroll
                    for (int d = 0; d < kDepth; ++d) {
                        const int64_t t = hi - k - 16 * d;
                        w[d] = (!done && t >= 0) ? load_agent(&st[(uint64_t)t * kMaxClasses + q]) : DW::make(1, 0);
                    }
#pragma unroll
                    for (int d = 0; d < kDepth; ++d) {
                        const int64_t t = hi - k - 16 * d;
                        while (DW::flag(w[d]) == 0) {
                            __builtin_amdgcn_s_sleep(2);
                            w[d] = load_agent(&st[(uint64_t)t * kMaxClasses + q]);
                        }
                    }
#pragma unroll
                    for (int d = 0; d < kDepth; ++d) {
                        const int64_t t = hi - k - 16 * d;
                        const uint64_t im = __ballot(!done && t >= 0 && DW::flag(w[d]) == kFlagInclusive);
                        const uint32_t gm = (uint32_t)(im >> (16 * q)) & 0xffffu;
                        const int k0 = gm ? __ffs(gm) - 1 : 15;  // nearest inclusive chunk of the class
                        const uint64_t v =
                            row_sum_u64((!done && t >= 0 && k <= k0) ? (uint64_t)(w[d] & DW::kMask) : 0ull);
                        if (!done) {
                            excl += v;
                            done = gm != 0;
                        }
                    }
                    hi -= 16 * kDepth;
                }
                if (act && k == 0) {
                    if (c > 0) store_agent(&st[c * kMaxClasses + q], DW::make(kFlagInclusive, excl + count));
                    s_cdst[q] = a.cls_base[q] + excl - packed_prefix(tot, q);
                }
            }
        }
        __syncthreads();
        if constexpr (!CLS) {
            for (uint32_t i = threadIdx.x; i < nrec; i += BLOCK) {
                keys_a[o0 + i] = s_keys[i];
                vals_a[o0 + i] = s_pay[i];
            }
        } else {
            for (uint32_t i = threadIdx.x; i < nrec; i += BLOCK) {
                int q = 0;
#pragma unroll
                for (int t = 1; t < kMaxClasses; ++t)
                    if (t < a.ncls && i >= packed_prefix(tot, t)) q = t;
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
    }
    __syncthreads();
    if (rows) hist_flush(s_hist, a.hist_part, rows);
    if (my_data) atomicAdd(&s_data, (unsigned long long)my_data);
    __syncthreads();
    if (threadIdx.x == 0 && s_data) atomicAdd(a.data_records, s_data);
}

// ---------------------------------------------------------------------------
// Regrouping (Sec. 4: the sort by ID and the scan tagged by ID).  A record's
// slot is its tuple of tree levels (j_1, ..., j_{m-1}), read off the key (the
// level of node (1 << j) | prefix is its highest set bit), in mixed radix over
// the per-axis field widths.  A query has at most one record per slot, and
// one exactly when every j_a is a 1-digit of its axis-a rank (a 0-digit for
// data).  So the scan can store each partial at part[slot][row] with a plain
// store, and a second pass folds each row's valid slots in slot order -- no
// atomics, and the same fold order on every run.

struct SlotMap {
    int nax;
    int field_shift[3];
    uint32_t field_mask[3];
    uint32_t radix[3];
    uint32_t n_slots;  // product of the radices; stores to slots beyond it are dropped
    template <class K>
    __device__ __forceinline__ uint32_t slot(K key) const {
        uint32_t sl = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (a < nax) {
                const uint32_t node = (uint32_t)(key >> field_shift[a]) & field_mask[a];
                sl = sl * radix[a] + (31u - (uint32_t)__clz(node));
            }
        }
        return sl;
    }
};

enum { OP_SUM = 0, OP_MAX = 1, OP_COUNT = 2 };

template <class V>
__device__ __forceinline__ V lowest();
template <> __device__ __forceinline__ int32_t lowest<int32_t>() { return INT32_MIN; }
template <> __device__ __forceinline__ int64_t lowest<int64_t>() { return INT64_MIN; }
template <> __device__ __forceinline__ float lowest<float>() { return -__builtin_inff(); }
template <> __device__ __forceinline__ double lowest<double>() { return -__builtin_inf(); }

template <class V, int OP>
struct Monoid {
    __device__ static V identity() {
        if constexpr (OP == OP_MAX) return lowest<V>();
        else return V(0);
    }
    __device__ static V combine(V a, V b) {
        if constexpr (OP == OP_MAX) return b > a ? b : a;
        else return a + b;
    }
};

// Forward: the segmented scan of the weights over the sorted records.
// Segments are runs of equal keys (the bitstring tuple, Sec. 5).  Queries
// carry the unit e; at a query record the scan value is F over the data
// records before it in its segment, i.e. over the data points that share
// this tuple and lie strictly below it on the last axis.  Each such partial
// goes to part[slot * nQ + query] (slot mode) or is F-combined atomically
// into out[query] (atomic mode, for very sparse slot tables).  Payloads and
// w use the internal numbering of the points.
//
// INL: the records carry the weights (a data record's payload is its weight
// bits, a query record's key has bit flag_shift set and its payload is the
// query's row), so the scan reads them in sequence instead of gathering.
template <class K, class W, class Acc, int OP, bool INL = false>
struct ForwardProblem {
    using V = Acc;
    struct Raw {
        K key;
        uint32_t payload;
    };
    const K *keys;
    const uint32_t *vals;
    const W *w;  // unused for COUNT and INL
    V *out;      // atomic mode target
    V *part;     // slot mode target, or null
    uint64_t stride;
    uint64_t nw;     // weights (|D|): payloads are checked against it
    SlotMap sm;
    int flag_shift;  // INL

    __device__ bool is_query(const Raw &r) const {
        if constexpr (INL) return ((r.key >> flag_shift) & K(1)) != K(0);
        else return (r.payload & kQueryFlag) != 0u;
    }
    __device__ V identity() const { return Monoid<V, OP>::identity(); }
    __device__ V combine(V a, V b) const { return Monoid<V, OP>::combine(a, b); }
    __device__ Raw load(uint64_t i) const { return Raw{keys[i], vals[i]}; }
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
            return V(x);
        } else {
            return cur.payload < nw ? V(w[cur.payload]) : identity();  // (always below |D|)
        }
    }
    __device__ void emit(uint64_t, const Raw &cur, V, V, V incl, bool) const {
        if (!is_query(cur)) return;
        const uint32_t q = INL ? cur.payload : (cur.payload & ~kQueryFlag);
        if (q >= stride) return;  // (rows are < stride = |Q| by construction)
        if (part) {
            const uint32_t sl = sm.slot(cur.key);
            if (sl < sm.n_slots) part[(uint64_t)sl * stride + q] = incl;
        } else if (incl != identity()) {
            if constexpr (OP == OP_MAX) atomic_max(out + q, incl);
            else atomic_sum(out + q, incl);
        }
    }
};

// Backward of the sum: the same records scanned from the end.  Queries carry
// grad_out, data carry 0; at a data record the exclusive value is the sum of
// grad_out over the queries after it in its segment, i.e. the queries sharing
// the tuple and lying strictly above it on the last axis (equal last
// coordinates put queries first, so they come before the data record and are
// not counted).  Those partials go to part[slot * nD + data position], or
// are summed atomically into grad[data position] (internal numbering).
template <class K, class G>
struct BackwardProblem {
    using V = G;
    struct Raw {
        K key;
        uint32_t payload;
    };
    const K *keys;
    const uint32_t *vals;
    const G *g;
    G *grad;
    G *part;
    uint64_t stride;
    uint64_t ng;  // |Q|
    SlotMap sm;
    uint64_t E;

    __device__ G identity() const { return G(0); }
    __device__ G combine(G a, G b) const { return a + b; }
    __device__ Raw load(uint64_t i) const {
        const uint64_t q = E - 1 - i;
        return Raw{keys[q], vals[q]};
    }
    __device__ bool head(const Raw &prev, const Raw &cur) const { return prev.key != cur.key; }
    __device__ G value(const Raw &, bool, const Raw &cur, uint64_t) const {
        if (!(cur.payload & kQueryFlag)) return G(0);
        const uint32_t q = cur.payload & ~kQueryFlag;
        return q < ng ? g[q] : G(0);  // (always below |Q|)
    }
    __device__ void emit(uint64_t, const Raw &cur, G, G excl, G, bool) const {
        if (cur.payload & kQueryFlag) return;
        if (cur.payload >= stride) return;  // (rows are < stride = |D| by construction)
        if (part) {
            const uint32_t sl = sm.slot(cur.key);
            if (sl < sm.n_slots) part[(uint64_t)sl * stride + cur.payload] = excl;
        } else if (excl != G(0)) {
            atomic_sum(grad + cur.payload, excl);
        }
    }
};

// Folds each row's valid slots in slot order: out[o] = F over part[slot][o].
// Row o is point slot_base + o; its valid slots are the level tuples whose
// digits of the point's ranks equal `digit` (1 for queries, 0 for data) and
// lie below the instance's widths.
struct RegroupArgs {
    const uint32_t *inv;           // [nout]: output index of row o, or null (identity)
    const uint32_t *rank;          // [nax][n] by point slot
    const uint32_t *inst_of_slot;  // [n] or null
    const uint8_t *ltab;           // [nax][n_inst]
    uint32_t n, n_inst;
    uint32_t slot_base;
    uint32_t digit;
    uint32_t radix[3];
    uint64_t nout;
};

template <class V, int OP, int NAX>
__global__ __launch_bounds__(256) void regroup_kernel(RegroupArgs a, const V *__restrict__ part,
                                                      V *__restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t o = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; o < a.nout; o += stride) {
        const uint32_t s = a.slot_base + (uint32_t)o;
        const uint32_t ins = a.inst_of_slot ? a.inst_of_slot[s] : 0u;
        uint32_t x[3] = {0, 0, 0}, L[3] = {0, 0, 0};
#pragma unroll
        for (int ax = 0; ax < NAX; ++ax) {
            const uint32_t r = a.rank[(uint64_t)ax * a.n + s];
            L[ax] = a.ltab[(uint64_t)ax * a.n_inst + ins];
            x[ax] = a.digit ? r : ~r;
        }
        // digit j of the L-digit string x, counted from the top, is bit L-1-j
        auto ok = [&](int ax, uint32_t j) { return j < L[ax] && ((x[ax] >> (L[ax] - 1u - j)) & 1u); };
        V acc = Monoid<V, OP>::identity();
        if constexpr (NAX == 0) {
            acc = part[o];
        } else if constexpr (NAX == 1) {
            for (uint32_t j = 0; j < a.radix[0]; ++j)
                if (ok(0, j)) acc = Monoid<V, OP>::combine(acc, part[(uint64_t)j * a.nout + o]);
        } else if constexpr (NAX == 2) {
            for (uint32_t j0 = 0; j0 < a.radix[0]; ++j0) {
                const bool v0 = ok(0, j0);
                for (uint32_t j1 = 0; j1 < a.radix[1]; ++j1)
                    if (v0 && ok(1, j1))
                        acc = Monoid<V, OP>::combine(acc, part[((uint64_t)j0 * a.radix[1] + j1) * a.nout + o]);
            }
        } else {
            for (uint32_t j0 = 0; j0 < a.radix[0]; ++j0) {
                const bool v0 = ok(0, j0);
                for (uint32_t j1 = 0; j1 < a.radix[1]; ++j1) {
                    const bool v1 = v0 && ok(1, j1);
                    for (uint32_t j2 = 0; j2 < a.radix[2]; ++j2)
                        if (v1 && ok(2, j2))
                            acc = Monoid<V, OP>::combine(
                                acc, part[(((uint64_t)j0 * a.radix[1] + j1) * a.radix[2] + j2) * a.nout + o]);
                }
            }
        }
        out[a.inv ? a.inv[o] : o] = acc;
    }
}

}  // namespace domagg
