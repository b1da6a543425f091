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
// vals[s] = s.  Fused histogram of `passes` digits; NaN raises *nan_flag.
template <class K, class C, int BLOCK>
__global__ __launch_bounds__(BLOCK) void extract_keys_kernel(
    const C *__restrict__ q, const C *__restrict__ d, int m, int axis, uint32_t nQ, uint32_t n,
    const uint32_t *__restrict__ inst_of_slot, K *__restrict__ keys, uint32_t *__restrict__ vals,
    int passes, uint32_t *__restrict__ hist_part, uint32_t *__restrict__ nan_flag) {
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
            vals[s] = (uint32_t)s;
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

template <class K>
struct RankProblem {
    using V = uint32_t;
    struct Raw {
        K key;
        uint32_t slot;
    };
    const K *keys;
    const uint32_t *slots;
    uint32_t *rank;
    uint32_t *kcount;  // [n_inst]

    __device__ static uint32_t inst(const Raw &r) {
        if constexpr (sizeof(K) == 8) return (uint32_t)(r.key >> 32);
        else return 0u;
    }
    __device__ V identity() const { return 0u; }
    __device__ V combine(V a, V b) const { return a + b; }
    __device__ Raw load(uint64_t i) const { return Raw{keys[i], slots[i]}; }
    __device__ bool head(const Raw &prev, const Raw &cur) const { return inst(prev) != inst(cur); }
    __device__ V value(const Raw &prev, bool has_prev, const Raw &cur, uint64_t) const {
        return (!has_prev || prev.key != cur.key) ? 1u : 0u;
    }
    __device__ void emit(uint64_t, const Raw &cur, V, V, V incl, bool last) const {
        rank[cur.slot] = incl - 1u;
        if (last) kcount[inst(cur)] = incl;
    }
};

// ---------------------------------------------------------------------------
// Flat-map sizes.  Over the points in last-axis order (slot list `slots`,
// sorted keys carry the instance), the value is the number of records the
// point yields; the exclusive sums are the record offsets, off[n] = E.  As a
// side effect the point's ranks, payload and instance are laid out in that
// order for the emitter.

template <class K, int NAX>
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
        uint64_t c = 1;
#pragma unroll
        for (int a = 0; a < NAX; ++a) {
            const uint32_t r = rank[(uint64_t)a * n + cur.slot];
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

struct EmitArgs {
    const uint64_t *off;     // [n + 1]
    const uint32_t *rs;      // [NAX][n]
    const uint32_t *pay;     // [n]
    const uint32_t *inst_s;  // [n] or null
    const uint8_t *ltab;     // [NAX][n_inst]
    uint32_t n, n_inst;
    uint64_t E;
    int field_shift[3];
    int inst_shift;
    int passes;
    uint32_t *hist_part;
    unsigned long long *data_records;
};

// the t-th set digit of the L-digit string x counted from its most
// significant digit; returns its position from the top (0-based)
__device__ __forceinline__ uint32_t select_from_top(uint32_t x, uint32_t L, uint32_t t) {
    uint32_t y = __brev(x) >> (32u - L);
    for (uint32_t i = 0; i < t; ++i) y &= y - 1u;
    return (uint32_t)(__ffs(y) - 1);
}

template <class K, int NAX, int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void emit_kernel(EmitArgs a, K *__restrict__ keys_out,
                                                     uint32_t *__restrict__ vals_out) {
    constexpr int CHUNK = BLOCK * ITEMS;
    __shared__ uint32_t s_off[CHUNK + 1];
    __shared__ uint32_t s_hist[kMaxPasses * kRadix];
    __shared__ uint32_t s_klo, s_khi;
    __shared__ unsigned long long s_data;
    for (int i = threadIdx.x; i < a.passes * kRadix; i += BLOCK) s_hist[i] = 0;
    if (threadIdx.x == 0) s_data = 0;
    uint32_t my_data = 0;

    const uint64_t nchunks = (a.E + CHUNK - 1) / CHUNK;
    for (uint64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const uint64_t o0 = c * CHUNK;
        const uint64_t o1 = (o0 + CHUNK < a.E) ? o0 + CHUNK : a.E;
        __syncthreads();
        if (threadIdx.x < 2) {
            // largest k with off[k] <= target
            const uint64_t target = threadIdx.x == 0 ? o0 : o1 - 1;
            uint32_t lo = 0, hi = a.n;  // off[lo] <= target < off[hi]
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (a.off[mid] <= target) lo = mid; else hi = mid;
            }
            if (threadIdx.x == 0) s_klo = lo; else s_khi = lo;
        }
        __syncthreads();
        const uint32_t klo = s_klo, khi = s_khi;
        const uint32_t npts = khi - klo + 1;
        const bool cached = npts <= (uint32_t)CHUNK;
        const uint64_t obase = a.off[klo];
        if (cached)
            for (uint32_t i = threadIdx.x; i < npts; i += BLOCK) s_off[i] = (uint32_t)(a.off[klo + i] - obase);
        __syncthreads();

        uint32_t lo_hint = 0;
#pragma unroll 1
        for (int j = 0; j < ITEMS; ++j) {
            const uint64_t o = o0 + (uint64_t)j * BLOCK + threadIdx.x;
            const bool valid = o < o1;
            K key = 0;
            if (valid) {
                const uint32_t rel = (uint32_t)(o - obase);
                uint32_t lo = lo_hint, hi = npts;  // (relative) off[lo] <= rel < off[hi]
                if (cached) {
                    while (hi - lo > 1) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (s_off[mid] <= rel) lo = mid; else hi = mid;
                    }
                } else {
                    while (hi - lo > 1) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (a.off[klo + mid] - obase <= rel) lo = mid; else hi = mid;
                    }
                }
                lo_hint = lo;
                const uint32_t k = klo + lo;
                uint32_t t = rel - (cached ? s_off[lo] : (uint32_t)(a.off[k] - obase));
                const uint32_t p = a.pay[k];
                const bool isq = (p & kQueryFlag) != 0u;
                const uint32_t ins = a.inst_s ? a.inst_s[k] : 0u;
                if (a.inst_s) key = (K)ins << a.inst_shift;
#pragma unroll
                for (int ax = NAX - 1; ax >= 0; --ax) {
                    const uint32_t r = a.rs[(uint64_t)ax * a.n + k];
                    const uint32_t L = a.ltab[(uint64_t)ax * a.n_inst + ins];
                    const uint32_t pc = (uint32_t)__popc(r);
                    const uint32_t cnt = isq ? pc : (L - pc);
                    uint32_t ta;
                    if (ax == 0) {
                        ta = t;
                    } else {
                        ta = t % cnt;
                        t /= cnt;
                    }
                    const uint32_t mask = (L >= 32u) ? 0xffffffffu : ((1u << L) - 1u);
                    const uint32_t x = isq ? r : (~r & mask);
                    const uint32_t jlev = select_from_top(x, L, ta);
                    const uint32_t node = (1u << jlev) | (jlev ? (r >> (L - jlev)) : 0u);
                    key |= (K)node << a.field_shift[ax];
                }
                keys_out[o] = key;
                vals_out[o] = p;
                my_data += isq ? 0u : 1u;
            }
            hist_add(s_hist, key, valid, a.passes);
        }
    }
    __syncthreads();
    hist_flush(s_hist, a.hist_part, a.passes);
    if (my_data) atomicAdd(&s_data, (unsigned long long)my_data);
    __syncthreads();
    if (threadIdx.x == 0 && s_data) atomicAdd(a.data_records, s_data);
}

// ---------------------------------------------------------------------------
// Forward: the segmented scan of the weights over the sorted records.
// Segments are runs of equal keys (the bitstring tuple, Sec. 5).  Queries
// carry the unit e; at a query record the scan value is F over the data
// records before it in its segment, i.e. over the data points that share
// this tuple and lie strictly below it on the last axis.  Those partials are
// then F-reduced into out[query] (the regrouping by ID).

enum { OP_SUM = 0, OP_MAX = 1, OP_COUNT = 2 };

template <class V>
__device__ __forceinline__ V lowest();
template <> __device__ __forceinline__ int32_t lowest<int32_t>() { return INT32_MIN; }
template <> __device__ __forceinline__ int64_t lowest<int64_t>() { return INT64_MIN; }
template <> __device__ __forceinline__ float lowest<float>() { return -__builtin_inff(); }
template <> __device__ __forceinline__ double lowest<double>() { return -__builtin_inf(); }

template <class K, class W, class Acc, int OP>
struct ForwardProblem {
    using V = Acc;
    struct Raw {
        K key;
        uint32_t payload;
    };
    const K *keys;
    const uint32_t *vals;
    const W *w;  // unused for COUNT
    V *out;

    __device__ V identity() const {
        if constexpr (OP == OP_MAX) return lowest<V>();
        else return V(0);
    }
    __device__ V combine(V a, V b) const {
        if constexpr (OP == OP_MAX) return b > a ? b : a;
        else return a + b;
    }
    __device__ Raw load(uint64_t i) const { return Raw{keys[i], vals[i]}; }
    __device__ bool head(const Raw &prev, const Raw &cur) const { return prev.key != cur.key; }
    __device__ V value(const Raw &, bool, const Raw &cur, uint64_t) const {
        if (cur.payload & kQueryFlag) return identity();
        if constexpr (OP == OP_COUNT) return V(1);
        else return V(w[cur.payload]);
    }
    __device__ void emit(uint64_t, const Raw &cur, V, V, V incl, bool) const {
        if ((cur.payload & kQueryFlag) && incl != identity()) {
            V *dst = out + (cur.payload & ~kQueryFlag);
            if constexpr (OP == OP_MAX) atomic_max(dst, incl);
            else atomic_sum(dst, incl);
        }
    }
};

// Backward of the sum: the same records scanned from the end.  Queries carry
// grad_out, data carry 0; at a data record the exclusive value is the sum of
// grad_out over the queries after it in its segment, i.e. the queries sharing
// the tuple and lying strictly above it on the last axis (equal last
// coordinates put queries first, so they come before the data record and are
// not counted).  Those partials are summed into grad[data row].
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
    uint64_t E;

    __device__ G identity() const { return G(0); }
    __device__ G combine(G a, G b) const { return a + b; }
    __device__ Raw load(uint64_t i) const {
        const uint64_t q = E - 1 - i;
        return Raw{keys[q], vals[q]};
    }
    __device__ bool head(const Raw &prev, const Raw &cur) const { return prev.key != cur.key; }
    __device__ G value(const Raw &, bool, const Raw &cur, uint64_t) const {
        return (cur.payload & kQueryFlag) ? g[cur.payload & ~kQueryFlag] : G(0);
    }
    __device__ void emit(uint64_t, const Raw &cur, G, G excl, G, bool) const {
        if (!(cur.payload & kQueryFlag) && excl != G(0)) atomic_sum(grad + cur.payload, excl);
    }
};

}  // namespace domagg
