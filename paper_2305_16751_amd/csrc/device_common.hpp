// Device-side building blocks shared by the kernels: wave64 lane masks,
// digit matching across a wavefront, agent-scope status words for decoupled
// look-back, wavefront scans on DPP/permute, and compensated fp32 sums.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace domagg {

constexpr int kWave = 64;

// Query records carry this bit in their 32-bit payload; the remaining bits
// are the query's row.  Data records carry their data row.
constexpr uint32_t kQueryFlag = 0x80000000u;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int l = lane_id();
    return l ? (~0ull >> (64 - l)) : 0ull;
}

// Number of set bits of `mask` at lanes below the calling lane.
__device__ __forceinline__ uint32_t count_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Lanes of the (fully active) wavefront holding the same BITS-bit digit:
// for every bit, the ballot of the lanes that have it set, complemented in
// lanes where it is clear -- an XNOR with the lane's bit spread over a word
// (written on 32-bit halves, so each bit costs a few plain bit operations
// instead of a 64-bit select).
template <int BITS>
__device__ __forceinline__ uint64_t match_digit(uint32_t d) {
    uint32_t lo = ~0u, hi = ~0u;
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        const uint32_t s = (uint32_t)((int32_t)(d << (31 - b)) >> 31);  // all ones where bit b is set
        const uint64_t bal = __ballot(s != 0u);
        lo &= ~((uint32_t)bal ^ s);
        hi &= ~((uint32_t)(bal >> 32) ^ s);
    }
    return ((uint64_t)hi << 32) | lo;
}

// ---------------------------------------------------------------------------
// Agent-scope (all XCDs) relaxed loads and stores.  Each status word carries
// its own flag, so no fence is needed between a value and its flag.

template <class T>
__device__ __forceinline__ T load_agent(const T *p) {
    return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T, class U>
__device__ __forceinline__ void store_agent(T *p, U u) {
    const T v = (T)u;
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Bit casts between scan values and their 32/64-bit images.

template <class V>
__device__ __forceinline__ uint64_t to_bits(V v) {
    if constexpr (sizeof(V) == 4) {
        uint32_t u;
        __builtin_memcpy(&u, &v, 4);
        return u;
    } else {
        uint64_t u;
        __builtin_memcpy(&u, &v, 8);
        return u;
    }
}
template <class V>
__device__ __forceinline__ V from_bits(uint64_t u) {
    V v;
    if constexpr (sizeof(V) == 4) {
        uint32_t w = (uint32_t)u;
        __builtin_memcpy(&v, &w, 4);
    } else {
        __builtin_memcpy(&v, &u, 8);
    }
    return v;
}

// ---------------------------------------------------------------------------
// Look-back status of one tile of a scan: flag 0 = not yet published,
// 1 = the tile's own aggregate (it needs its predecessors), 2 = inclusive
// prefix up to and including the tile.  A 32-bit value is packed with its
// flag into one 64-bit word; a 64-bit value is split over two words that
// each carry the flag, and a reader accepts the pair only when both flags
// agree (each word only ever holds one aggregate and one inclusive image).

constexpr uint32_t kFlagAggregate = 1u;
constexpr uint32_t kFlagInclusive = 2u;

template <class V>
struct ScanStatusWords {
    static constexpr int kWords = sizeof(V) == 4 ? 1 : 2;
};

template <class V>
__device__ __forceinline__ void publish_status(uint64_t *st, uint32_t tile, uint32_t flag, V v) {
    const uint64_t b = to_bits(v);
    if constexpr (sizeof(V) == 4) {
        store_agent(st + tile, ((uint64_t)flag << 32) | (b & 0xffffffffull));
    } else {
        store_agent(st + 2ull * tile, ((uint64_t)flag << 32) | (b & 0xffffffffull));
        store_agent(st + 2ull * tile + 1, ((uint64_t)flag << 32) | (b >> 32));
    }
}

// One read of a tile's status: its flag (0 = not yet published) and value.
template <class V>
__device__ __forceinline__ uint32_t try_status(const uint64_t *st, uint32_t tile, V &v) {
    if constexpr (sizeof(V) == 4) {
        const uint64_t w = load_agent(st + tile);
        v = from_bits<V>(w & 0xffffffffull);
        return (uint32_t)(w >> 32);
    } else {
        const uint64_t w0 = load_agent(st + 2ull * tile);
        const uint64_t w1 = load_agent(st + 2ull * tile + 1);
        const uint32_t f0 = (uint32_t)(w0 >> 32), f1 = (uint32_t)(w1 >> 32);
        v = from_bits<V>((w0 & 0xffffffffull) | (w1 << 32));
        return f0 == f1 ? f0 : 0u;
    }
}

// Spins until the tile's status is published; returns its flag and value.
template <class V>
__device__ __forceinline__ uint32_t wait_status(const uint64_t *st, uint32_t tile, V &v) {
    for (;;) {
        if constexpr (sizeof(V) == 4) {
            const uint64_t w = load_agent(st + tile);
            const uint32_t f = (uint32_t)(w >> 32);
            if (f) {
                v = from_bits<V>(w & 0xffffffffull);
                return f;
            }
        } else {
            const uint64_t w0 = load_agent(st + 2ull * tile);
            const uint64_t w1 = load_agent(st + 2ull * tile + 1);
            const uint32_t f0 = (uint32_t)(w0 >> 32), f1 = (uint32_t)(w1 >> 32);
            if (f0 && f0 == f1) {
                v = from_bits<V>((w0 & 0xffffffffull) | (w1 << 32));
                return f0;
            }
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// ---------------------------------------------------------------------------
// Wavefront scans.  The row-local steps use DPP row_shr:1,2,4,8 (16-lane
// rows); the cross-row steps use DPP row_bcast:15 (the last lane of rows 0
// and 2 combined into rows 1 and 3) and row_bcast:31 (lane 31 combined into
// rows 2 and 3).  Lanes a step does not write keep `old`, which is the
// operator's identity, so every step is a plain combine.  Defining
// DOMAGG_WAVE_SCAN_BPERMUTE replaces the DPP moves by ds_bpermute with the
// same source lanes.

constexpr int kDppRowShr1 = 0x111;
constexpr int kDppRowShr2 = 0x112;
constexpr int kDppRowShr4 = 0x114;
constexpr int kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v, uint32_t old) {
#ifndef DOMAGG_WAVE_SCAN_BPERMUTE
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROW_MASK, 0xf, false);
#else
    const int l = lane_id();
    const int row = l >> 4;
    int src;
    bool take;
    if constexpr (CTRL >= kDppRowShr1 && CTRL <= kDppRowShr8 + 7) {
        constexpr int k = CTRL - 0x110;
        src = l - k;
        take = (l & 15) >= k;
    } else if constexpr (CTRL == kDppRowBcast15) {
        src = (l & ~15) - 1;
        take = row == 1 || row == 3;
    } else {
        src = 31;
        take = row >= 2;
    }
    (void)ROW_MASK;
    const uint32_t x = (uint32_t)__builtin_amdgcn_ds_bpermute((src < 0 ? 0 : src) << 2, (int)v);
    return take ? x : old;
#endif
}

template <int CTRL, int ROW_MASK, class V>
__device__ __forceinline__ V dpp_val(V v, V old) {
    if constexpr (sizeof(V) == 4) {
        return from_bits<V>(dpp_u32<CTRL, ROW_MASK>((uint32_t)to_bits(v), (uint32_t)to_bits(old)));
    } else {
        const uint64_t b = to_bits(v), o = to_bits(old);
        const uint32_t lo = dpp_u32<CTRL, ROW_MASK>((uint32_t)b, (uint32_t)o);
        const uint32_t hi = dpp_u32<CTRL, ROW_MASK>((uint32_t)(b >> 32), (uint32_t)(o >> 32));
        return from_bits<V>((uint64_t)lo | ((uint64_t)hi << 32));
    }
}

template <int CTRL, int ROW_MASK, class Op, class V>
__device__ __forceinline__ void seg_step(const Op &op, uint32_t &flag, V &v) {
    const V pv = dpp_val<CTRL, ROW_MASK>(v, op.identity());
    const uint32_t pf = dpp_u32<CTRL, ROW_MASK>(flag, 0u);
    if (!flag) v = op.combine(pv, v);
    flag |= pf;
}

// Inclusive segmented scan across the wavefront of (flag, value) pairs with
// the operator (fa, a) . (fb, b) = (fa | fb, fb ? b : F(a, b)).
template <class Op, class V>
__device__ __forceinline__ void wave_seg_scan_incl(const Op &op, uint32_t &flag, V &v) {
    seg_step<kDppRowShr1, 0xf>(op, flag, v);
    seg_step<kDppRowShr2, 0xf>(op, flag, v);
    seg_step<kDppRowShr4, 0xf>(op, flag, v);
    seg_step<kDppRowShr8, 0xf>(op, flag, v);
    seg_step<kDppRowBcast15, 0xa>(op, flag, v);
    seg_step<kDppRowBcast31, 0xc>(op, flag, v);
}

// Inclusive sum scan of u32 across the wavefront.
__device__ __forceinline__ uint32_t wave_sum_scan_incl(uint32_t v) {
    v += dpp_u32<kDppRowShr1, 0xf>(v, 0u);
    v += dpp_u32<kDppRowShr2, 0xf>(v, 0u);
    v += dpp_u32<kDppRowShr4, 0xf>(v, 0u);
    v += dpp_u32<kDppRowShr8, 0xf>(v, 0u);
    v += dpp_u32<kDppRowBcast15, 0xa>(v, 0u);
    v += dpp_u32<kDppRowBcast31, 0xc>(v, 0u);
    return v;
}

// Sum of a 64-bit value over each 16-lane row, returned to every lane of
// the row (every lane must be active).
__device__ __forceinline__ uint64_t read_lane_u64(uint64_t v, int src);
__device__ __forceinline__ uint64_t row_sum_u64(uint64_t v) {
    v += dpp_val<kDppRowShr1, 0xf>(v, (uint64_t)0);
    v += dpp_val<kDppRowShr2, 0xf>(v, (uint64_t)0);
    v += dpp_val<kDppRowShr4, 0xf>(v, (uint64_t)0);
    v += dpp_val<kDppRowShr8, 0xf>(v, (uint64_t)0);
    return read_lane_u64(v, (lane_id() & ~15) + 15);
}

// Value of `v` at lane `src` (ds_bpermute; every lane must be active).
__device__ __forceinline__ uint32_t read_lane_u32(uint32_t v, int src) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)v);
}

__device__ __forceinline__ uint64_t read_lane_u64(uint64_t v, int src) {
    const uint32_t lo = read_lane_u32((uint32_t)v, src);
    const uint32_t hi = read_lane_u32((uint32_t)(v >> 32), src);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// Value of `v` at a lane index that is the same for the whole wavefront
// (v_readlane into a scalar register: no LDS round trip).
template <class V>
__device__ __forceinline__ V read_uniform_lane(V v, int src) {
    if constexpr (sizeof(V) == 4) {
        return from_bits<V>((uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)to_bits(v), src));
    } else {
        const uint64_t b = to_bits(v);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, src);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), src);
        return from_bits<V>((uint64_t)lo | ((uint64_t)hi << 32));
    }
}

template <class V>
__device__ __forceinline__ V read_lane(V v, int src) {
    if constexpr (sizeof(V) == 4) {
        return from_bits<V>(read_lane_u32((uint32_t)to_bits(v), src));
    } else {
        const uint64_t b = to_bits(v);
        const uint32_t lo = read_lane_u32((uint32_t)b, src);
        const uint32_t hi = read_lane_u32((uint32_t)(b >> 32), src);
        return from_bits<V>((uint64_t)lo | ((uint64_t)hi << 32));
    }
}

// ---------------------------------------------------------------------------
// Compensated fp32 sum.  A value is the unevaluated pair hi + lo with
// |lo| <= ulp(hi) / 2; adding two of them is Knuth's TwoSum on the high parts
// followed by a renormalisation (Fast2Sum), all in fp32 arithmetic.  Long
// chains of fp32 additions (a segment that spans thousands of scan tiles, a
// carry folded across all of them) then keep an error of a few units in the
// last place of the result instead of one that grows with the chain.  The
// sequence of additions is what fixes the result, so results repeat bit for
// bit whenever the order of additions does.
struct F32c {
    float hi, lo;
};

__device__ __forceinline__ F32c f32c_add(F32c a, F32c b) {
    const float s = a.hi + b.hi;
    const float bb = s - a.hi;
    const float err = (a.hi - (s - bb)) + (b.hi - bb);
    const float lo = a.lo + b.lo + err;
    const float hi = s + lo;
    return F32c{hi, lo - (hi - s)};
}

}  // namespace domagg
