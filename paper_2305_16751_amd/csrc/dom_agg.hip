// C-ABI of the dominance aggregation library (declared in include/dom_agg.h).
//
// Host orchestration of the paper's construction (Sec. 4 with Sec. 5):
//   plan:     per axis 1..m-1: order-preserving keys -> stable radix sort ->
//             dense ranks; axis m: keys -> stable radix sort (the point order
//             of Sec. 5); record counts and offsets; flat map; stable radix
//             sort of the records by bitstring tuple.
//   forward:  segmented scan of the weights + regrouping into out[query].
//   backward: reverse segmented scan of grad_out + regrouping into grad[data].
// Every step runs in the kernels of dominance.hpp, radix_sort.hpp and
// seg_scan.hpp; this file only sizes, allocates, orders and checks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <limits>
#include <memory>
#include <type_traits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "dom_agg.h"
#include "dominance.hpp"
#include "seg_scan.hpp"
#include "tuner.hpp"

using namespace domagg;

namespace {

// ---------------------------------------------------------------------------
// Errors: internal failures throw; every exported function catches.

struct Failure {
    dom_agg_status status;
    std::string msg;
};

thread_local std::string t_last_error;

[[noreturn]] void fail(dom_agg_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    throw Failure{st, buf};
}

#define HIPCHK(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) fail(DOM_AGG_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

template <class F>
dom_agg_status guarded(F &&f) {
    try {
        f();
        t_last_error.clear();
        return DOM_AGG_OK;
    } catch (const Failure &e) {
        t_last_error = e.msg;
        return e.status;
    } catch (const std::bad_alloc &) {
        t_last_error = "host allocation failed";
        return DOM_AGG_ENOMEM;
    } catch (...) {
        t_last_error = "unexpected internal error";
        return DOM_AGG_EHIP;
    }
}

// ---------------------------------------------------------------------------
// Device memory: through the registered hook, else hipMalloc/hipFree; or,
// inside dom_agg_run_static, from the static workspace (below).

dom_agg_alloc_fn g_alloc = nullptr;
dom_agg_release_fn g_release = nullptr;
void *g_alloc_ctx = nullptr;

// A bump allocator over one device's static workspace, active on the calling
// thread for the duration of one dom_agg_run_static call.  Nothing is freed
// during the call; the next call starts again at the beginning.
struct Arena {
    char *base;
    size_t cap, used;
};
thread_local Arena *t_arena = nullptr;

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    bool from_arena = false;

    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept { *this = std::move(o); }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            reset();
            p = o.p;
            bytes = o.bytes;
            stream = o.stream;
            from_arena = o.from_arena;
            o.p = nullptr;
            o.bytes = 0;
            o.from_arena = false;
        }
        return *this;
    }
    ~DevBuf() { reset(); }
    void reset() {
        if (p && !from_arena) {
            if (g_release) g_release(p, stream, g_alloc_ctx);
            else (void)hipFree(p);
        }
        p = nullptr;
        bytes = 0;
        from_arena = false;
    }
    void alloc(size_t b, hipStream_t s) {
        reset();
        if (b == 0) return;
        stream = s;
        if (t_arena) {
            const size_t at = (t_arena->used + 255) & ~(size_t)255;
            if (at > t_arena->cap || b > t_arena->cap - at)
                fail(DOM_AGG_ETOOBIG, "the call needs more than the %zu-byte static workspace", t_arena->cap);
            p = t_arena->base + at;
            bytes = b;
            from_arena = true;
            t_arena->used = at + b;
            return;
        }
        void *q = nullptr;
        if (g_alloc) {
            q = g_alloc(b, (void *)s, g_alloc_ctx);
        } else if (hipMalloc(&q, b) != hipSuccess) {
            (void)hipGetLastError();
            q = nullptr;
        }
        if (!q) fail(DOM_AGG_ENOMEM, "device allocation of %zu bytes failed", b);
        p = q;
        bytes = b;
    }
    template <class T>
    T *as() const { return static_cast<T *>(p); }
};

// ---------------------------------------------------------------------------
// Optional per-kernel event timing.

struct TimedLaunch {
    const char *name;
    hipEvent_t a, b;
};
struct KernelTotal {
    const char *name;
    double ms;
    int64_t launches;
};

std::mutex g_tmu;
bool g_timing = false;
std::vector<TimedLaunch> g_pending;
std::vector<hipEvent_t> g_event_pool;
std::vector<KernelTotal> g_totals;
thread_local bool t_capturing = false;

hipEvent_t take_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    return e;
}

// DOM_AGG_SYNC_CHECK=1: synchronise after every launch and name the kernel in
// the error, to attribute a device fault (slow; for debugging only).
bool sync_check() {
    static const bool on = [] {
        const char *e = std::getenv("DOM_AGG_SYNC_CHECK");
        return e && e[0] == '1';
    }();
    return on;
}

template <class F>
void launch(const char *name, hipStream_t s, F &&f) {
    bool timed;
    {
        std::lock_guard<std::mutex> lk(g_tmu);
        timed = g_timing && !t_capturing;
    }
    if (sync_check() && !t_capturing) {
        f();
        const hipError_t e1 = hipGetLastError();
        const hipError_t e2 = hipStreamSynchronize(s);
        if (e1 != hipSuccess || e2 != hipSuccess)
            fail(DOM_AGG_EHIP, "kernel %s: %s", name, hipGetErrorString(e1 != hipSuccess ? e1 : e2));
        return;
    }
    if (!timed) {
        f();
        HIPCHK(hipGetLastError());
        return;
    }
    hipEvent_t a, b;
    {
        std::lock_guard<std::mutex> lk(g_tmu);
        a = take_event();
        b = take_event();
    }
    HIPCHK(hipEventRecord(a, s));
    f();
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(b, s));
    std::lock_guard<std::mutex> lk(g_tmu);
    g_pending.push_back({name, a, b});
}

// ---------------------------------------------------------------------------
// Device check: the library is built for gfx950 only.

void require_gfx950(int *device) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        fail(DOM_AGG_ENODEV, "no HIP device is available");
    }
    static std::mutex mu;
    static std::map<int, bool> ok;
    std::lock_guard<std::mutex> lk(mu);
    auto it = ok.find(dev);
    if (it == ok.end()) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
            (void)hipGetLastError();
            fail(DOM_AGG_ENODEV, "cannot query HIP device %d", dev);
        }
        it = ok.emplace(dev, std::strncmp(prop.gcnArchName, "gfx950", 6) == 0).first;
    }
    if (!it->second) fail(DOM_AGG_ENODEV, "device %d is not gfx950", dev);
    *device = dev;
}

// DOM_AGG_DIGIT_BITS=7 or 8 fixes the record sort's digit width (for
// measurement and tests; the tuner then searches tiles only, under keys of
// their own); 0 when unset.
int forced_digit_bits() {
    const char *e = std::getenv("DOM_AGG_DIGIT_BITS");
    if (!e || !e[0]) return 0;
    const int v = std::atoi(e);
    if (v != 7 && v != 8) fail(DOM_AGG_EINVAL, "DOM_AGG_DIGIT_BITS must be 7 or 8 (got \"%s\")", e);
    return v;
}

// DOM_AGG_COMPACT=1 regroups through the compact per-row layout even where
// the level-tuple slot table would be used (for measurement and tests).
bool compact_forced() {
    const char *e = std::getenv("DOM_AGG_COMPACT");
    return e && e[0] == '1';
}

// Where the record sort's digit histograms come from: the rank CDFs, one
// thread per tree node (m = 2, one instance); the points, in closed form; a
// streaming pass over the emitted records; or the flat map's per-record
// loop.  DOM_AGG_HIST=points / records / emit picks one of the last three
// where it applies (for measurement); 0 when unset.
enum class HistSource { kNodes, kPoints, kRecords, kEmit };

int hist_source_override() {
    const char *e = std::getenv("DOM_AGG_HIST");
    if (!e || !e[0]) return 0;
    if (!std::strcmp(e, "points")) return 1;
    if (!std::strcmp(e, "records")) return 2;
    if (!std::strcmp(e, "emit")) return 3;
    fail(DOM_AGG_EINVAL, "DOM_AGG_HIST must be points, records or emit (got \"%s\")", e);
}

// DOM_AGG_PACK=0 keeps records as separate key and payload arrays (for
// measurement); packing is on otherwise.
bool packing_enabled() {
    static const bool on = [] {
        const char *e = std::getenv("DOM_AGG_PACK");
        return !(e && e[0] == '0');
    }();
    return on;
}

int bits_for(uint64_t K) {
    int L = 0;
    while (L < 63 && (1ull << L) < K) ++L;
    return L;
}

uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

constexpr int kBlock = 256;
constexpr uint64_t kMaxRecords = (1ull << 32) - (1ull << 20);
// slot-mode regrouping is used when the level-tuple table is small and dense
// enough; beyond these, the compact layout (one place per record)
constexpr uint64_t kMaxSlots = 1024;
constexpr uint64_t kMaxSlotBytes = 64ull << 30;
constexpr size_t kMaxGraphs = 8;

}  // namespace

// ---------------------------------------------------------------------------
// The static workspace of dom_agg_run_static.  Every GPU the library runs on
// holds one copy of this array until the process ends.  Host code must not
// use the array's name as a device address: the address of each device's
// copy comes from hipGetSymbolAddress, taken once per device.

constexpr size_t kStaticScratchBytes = 256ull << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

char *static_scratch(int dev) {
    static std::mutex mu;
    static std::map<int, char *> ptrs;
    std::lock_guard<std::mutex> lk(mu);
    auto it = ptrs.find(dev);
    if (it != ptrs.end()) return it->second;
    void *ptr = nullptr;  // (the calling thread has `dev` current)
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        fail(DOM_AGG_EHIP, "hipGetSymbolAddress of the static workspace: %s", hipGetErrorString(e));
    }
    ptrs.emplace(dev, static_cast<char *>(ptr));
    return static_cast<char *>(ptr);
}

// Makes `a` the calling thread's allocator until the scope ends.
struct ArenaScope {
    explicit ArenaScope(Arena *a) { t_arena = a; }
    ~ArenaScope() { t_arena = nullptr; }
    ArenaScope(const ArenaScope &) = delete;
    ArenaScope &operator=(const ArenaScope &) = delete;
};

}  // namespace

// ---------------------------------------------------------------------------
// The plan.

struct dom_agg_plan_s {
    int device = 0;
    int m = 0, nax = 0;
    uint32_t flags = 0;
    // bit a: <= instead of < on axis a (DOM_AGG_LE(a))
    uint32_t le_mask = 0;
    // the basic variant of Sec. 4 (DOM_AGG_BASIC): every axis expanded
    bool basic = false;
    int64_t n_inst = 1, nD = 0, nQ = 0, n = 0;
    bool batched = false;
    int inst_bits = 0;
    int Lmax[3] = {0, 0, 0};
    int key_bits = 0;
    bool key64 = false;
    int field_shift[3] = {0, 0, 0};
    int inst_shift = 0;
    // bits at the bottom of the record key that the sort does not read: the
    // instance id in batches (Sec. 5 variant), whose records are emitted in
    // instance order, so a stable sort by the node fields alone keeps each
    // (tuple, instance) run together; 0 otherwise
    int sort_lo = 0;
    int64_t E = 0, E_D = 0;
    std::vector<int> rec_shifts;  // radix passes the record sort runs (without classes)
    int rbits = kRadixBits;       // the record sort's digit width (7 or 8; chosen by the tuner)
    // key-length classes of the record sort (ncls = 1: one sort over all records)
    int ncls = 1, cls_c0 = 0;
    int cls_passes[kMaxClasses] = {0, 0, 0, 0};
    int cls_row0[kMaxClasses] = {0, 0, 0, 0};
    int cls_rows = 0;
    uint32_t cls_mask[kMaxClasses] = {0, 0, 0, 0};
    uint64_t cls_tot[kMaxClasses] = {0, 0, 0, 0};
    TuneChoice tune;

    // per-point state, in last-axis order
    DevBuf off, rs, pay, inst_s;
    // per-point state by internal slot, kept for the regrouping: ranks,
    // instance, widths
    DevBuf rank, inst_of_slot, ltab;
    // internal numbering (points in first-axis order; m >= 2): input row of
    // each data / query position, and a buffer for inputs in that order
    bool permuted = false;
    DevBuf dinv, qinv, perm;
    // m = 2, one instance: rank CDFs of data and queries (the record sort's
    // digit histograms are counted from them per tree node)
    DevBuf cdf_d, cdf_q;
    uint32_t K0 = 0;
    // records as packed 64-bit words (key above pay_bits payload bits)
    bool packed = false;
    int pay_bits = 0;
    // records carrying weights (one-shot calls): requested, granted, the
    // query flag's bit in the record key, the weights and their dtype
    bool inline_req = false, inline_w = false;
    int flag_shift = -1;
    const void *w_src = nullptr;
    dom_agg_dtype w_dt = DOM_AGG_F32;
    DevBuf rw, wv;
    // regrouping: level-tuple slots (slot mode) or one place per record
    // (compact mode, with the per-slot state cstate)
    uint32_t n_slots = 1;
    bool use_slots = true;
    DevBuf part, cstate;
    // sorted records (KEEP)
    DevBuf rkeys, rvals;
    // look-back words and ticket of the forward/backward scans
    DevBuf scan_status, scan_ticket;
    uint64_t scan_words = 0;
    DevBuf ed_counter;

    // graph replay cache
    // graph replay cache (DOM_AGG_GRAPH): one instantiated graph per call
    // key (kind, op, dtypes, buffers), the oldest dropped beyond kMaxGraphs
    hipStream_t cap_stream = nullptr;
    std::vector<std::pair<std::vector<uintptr_t>, hipGraphExec_t>> graphs;
    int64_t graph_captures = 0;

    size_t workspace() const {
        return off.bytes + rs.bytes + pay.bytes + inst_s.bytes + rank.bytes + inst_of_slot.bytes + ltab.bytes +
               dinv.bytes + qinv.bytes + perm.bytes + rw.bytes + wv.bytes + cdf_d.bytes + cdf_q.bytes + part.bytes + cstate.bytes + rkeys.bytes + rvals.bytes + scan_status.bytes + scan_ticket.bytes + ed_counter.bytes;
    }
    SlotMap slot_map() const {
        SlotMap sm{};
        sm.nax = nax;
        for (int a = 0; a < 3; ++a) {
            sm.field_shift[a] = field_shift[a];
            sm.field_mask[a] = Lmax[a] >= 32 ? 0xffffffffu : ((1u << Lmax[a]) - 1u);
            sm.radix[a] = (uint32_t)std::max(Lmax[a], 1);
        }
        sm.n_slots = nax == 0 ? 1u : n_slots;
        return sm;
    }
};

namespace {

using Plan = dom_agg_plan_s;

// Pinned host staging for the plan's size reads: one buffer per host thread,
// grown on demand and kept for the life of the thread (a pinned allocation
// costs tens of microseconds, and its release can wait for the device, both
// while the device idles between a size read and the launches that follow
// it).  Every use reads the buffer after a stream synchronisation and is
// done with it before the next use.  Inside dom_agg_run_static: a fixed host
// buffer instead.
constexpr size_t kStaticHostBytes = 1u << 20;
thread_local unsigned char t_static_host[kStaticHostBytes];

struct PinnedStage {
    void *p = nullptr;
    size_t bytes = 0;
    // (at thread exit; a thread's thread-local objects go before any static
    // one, the runtime's included)
    ~PinnedStage() {
        if (p) (void)hipHostFree(p);
    }
};
thread_local PinnedStage t_pinned;

struct HostStage {
    void *get(size_t b) {
        if (t_arena) {
            if (b > kStaticHostBytes)
                fail(DOM_AGG_ETOOBIG, "the call needs more than %zu bytes of host staging", kStaticHostBytes);
            return t_static_host;
        }
        if (b > t_pinned.bytes) {
            if (t_pinned.p) (void)hipHostFree(t_pinned.p);
            t_pinned.p = nullptr;
            t_pinned.bytes = 0;
            size_t nb = 64u << 10;
            while (nb < b) nb <<= 1;
            HIPCHK(hipHostMalloc(&t_pinned.p, nb, hipHostMallocDefault));
            t_pinned.bytes = nb;
        }
        return t_pinned.p;
    }
};

unsigned grid_for(uint64_t n) {
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(ceil_div(n, kBlock), 8192));
}

// Workgroups of `kernel` (kBlock threads) resident on the current device at
// once, at most `work`.
template <class F>
unsigned resident_grid(F kernel, uint64_t work) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    // (the occupancy of a kernel on a device does not change: asked once)
    static std::mutex mu;
    static std::map<std::pair<const void *, int>, uint64_t> known;
    uint64_t g;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = known.find({reinterpret_cast<const void *>(kernel), dev});
        if (it == known.end()) {
            int cus = 0, per = 0;
            HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
            HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kBlock, 0));
            it = known.emplace(std::make_pair(reinterpret_cast<const void *>(kernel), dev),
                               (uint64_t)std::max(per, 1) * (uint64_t)std::max(cus, 1)).first;
        }
        g = it->second;
    }
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(g, work));
}

template <class T>
void fill(T *p, uint64_t n, T v, hipStream_t s) {
    if (!n) return;
    const unsigned grid = (unsigned)std::min<uint64_t>(ceil_div(n, kBlock), 4096);
    launch("fill", s, [&] { fill_kernel<T><<<grid, kBlock, 0, s>>>(p, n, v); });
}

void clear_lookback(uint64_t *status, uint64_t words, uint32_t *ticket, hipStream_t s) {
    const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(ceil_div(words, kBlock), 2048));
    launch("clear_lookback", s,
           [&] { clear_lookback_kernel<<<grid, kBlock, 0, s>>>(status, words, ticket); });
}

// ---------------------------------------------------------------------------
// Radix sort driver.

template <class K, int ROLE, int RB = kRadixBits>
const char *onesweep_name(int tile) {
    if constexpr (RB != kRadixBits) {
        static_assert(ROLE == 1 && RB == 7, "7-bit digits: record sort only");
        static const char *n7[2][2] = {{"onesweep_records_u32_t4096_d7", "onesweep_records_u32_t8192_d7"},
                                       {"onesweep_records_u64_t4096_d7", "onesweep_records_u64_t8192_d7"}};
        return n7[sizeof(K) == 8][tile == 8192];
    }
    static const char *names[2][2][3] = {
        {{"onesweep_points_u32_t2048", "onesweep_points_u32_t4096", "onesweep_points_u32_t8192"},
         {"onesweep_points_u64_t2048", "onesweep_points_u64_t4096", "onesweep_points_u64_t8192"}},
        {{"onesweep_records_u32_t2048", "onesweep_records_u32_t4096", "onesweep_records_u32_t8192"},
         {"onesweep_records_u64_t2048", "onesweep_records_u64_t4096", "onesweep_records_u64_t8192"}}};
    if (tile == 16384) return sizeof(K) == 8 ? "onesweep_records_u64_t16384" : "onesweep_records_u32_t16384";
    const int ti = tile == 2048 ? 0 : tile == 4096 ? 1 : 2;
    return names[ROLE][sizeof(K) == 8][ti];
}

template <class K, class S, int BLOCK, int ITEMS, int ROLE, class VT, int RB = kRadixBits>
void onesweep_launch(const K *kin, const VT *vin, K *kout, VT *vout, uint32_t n,
                     int shift, const uint32_t *bases, S *status, uint32_t *ticket, hipStream_t s) {
    // (status and ticket arrive cleared: one clear serves all passes of a sort)
    constexpr int TILE = BLOCK * ITEMS;
    const unsigned tiles = (unsigned)ceil_div(n, TILE);
    launch(onesweep_name<K, ROLE, RB>(TILE), s, [&] {
        onesweep_kernel<K, S, BLOCK, ITEMS, ROLE, VT, true, RB><<<tiles, BLOCK, 0, s>>>(
            kin, vin, kout, vout, n, shift, bases, status, ticket);
    });
}

// The tile a sort pass really uses (16384 only for the record sort with
// 32-bit keys; its 64-bit-key form would not fit the registers).
template <class K, int ROLE>
int effective_tile(int tile) {
    if (!valid_sort_tile(tile)) return 4096;
    if (tile == 16384 && (ROLE != 1 || sizeof(K) != 4)) return 8192;
    return tile;
}

template <class K, class S, int ROLE, class VT, int RB = kRadixBits>
void onesweep_dispatch(int tile, const K *kin, const VT *vin, K *kout, VT *vout, uint32_t n,
                       int shift, const uint32_t *bases, void *status, uint32_t *ticket, hipStream_t s) {
    S *st = static_cast<S *>(status);
    if constexpr (RB != kRadixBits) {
        // 7-bit digits: the two tile shapes the tuner tries with them
        if (tile == 8192)
            onesweep_launch<K, S, 512, 16, ROLE, VT, RB>(kin, vin, kout, vout, n, shift, bases, st, ticket, s);
        else
            onesweep_launch<K, S, 256, 16, ROLE, VT, RB>(kin, vin, kout, vout, n, shift, bases, st, ticket, s);
    } else if constexpr (sizeof(VT) == 8) {
        // 64-bit payloads: one tile shape
        onesweep_launch<K, S, 256, 16, ROLE, VT>(kin, vin, kout, vout, n, shift, bases, st, ticket, s);
    } else if (tile == 2048) {
        onesweep_launch<K, S, 256, 8, ROLE, VT>(kin, vin, kout, vout, n, shift, bases, st, ticket, s);
    } else if (tile == 8192) {
        onesweep_launch<K, S, 512, 16, ROLE, VT>(kin, vin, kout, vout, n, shift, bases, st, ticket, s);
    } else if (tile == 16384) {
        if constexpr (ROLE == 1 && sizeof(K) == 4)
            onesweep_launch<K, S, 512, 32, ROLE, VT>(kin, vin, kout, vout, n, shift, bases, st, ticket, s);
        else
            fail(DOM_AGG_EHIP, "internal: no 16384-element tile for this sort");
    } else {
        onesweep_launch<K, S, 256, 16, ROLE, VT>(kin, vin, kout, vout, n, shift, bases, st, ticket, s);
    }
}

// Sorts (kA, vA) by the listed digit shifts; returns true when the result
// ended up in (kB, vB).  bases: [passes][256] (pass p at shift lo + rb * p).
// rb: digit width, 8, or 7 for the record sort (tiles 4096 and 8192).
template <class K, int ROLE, class VT = uint32_t>
bool radix_sort(K *kA, VT *vA, K *kB, VT *vB, uint64_t n, const std::vector<int> &shifts,
                const uint32_t *bases, int tile, hipStream_t s, int rb = kRadixBits, int lo = 0) {
    if (n == 0 || shifts.empty()) return false;
    if (rb != kRadixBits && (ROLE != 1 || sizeof(VT) != 4 || rb != 7))
        fail(DOM_AGG_EHIP, "internal: %d-bit digits are for the record sort only", rb);
    tile = sizeof(VT) == 8 ? 4096 : effective_tile<K, ROLE>(tile);
    if (rb != kRadixBits) tile = tile == 8192 ? 8192 : 4096;
    const bool narrow = n < (1ull << 30);  // every digit count fits 30 bits
    // every pass gets its own look-back words (the tile count of the tile
    // shape the dispatch launches: TILE == tile) and, after all of them, its
    // own ticket; one clear before the first pass
    const uint64_t pass_words = ceil_div(ceil_div(n, (uint64_t)tile) * kRadix * (narrow ? 4 : 8), (uint64_t)8);
    const uint64_t np = shifts.size();
    DevBuf status;
    status.alloc((pass_words * np + ceil_div(np, (uint64_t)2) + 1) * 8, s);
    uint32_t *tickets = reinterpret_cast<uint32_t *>(status.as<uint64_t>() + pass_words * np);
    clear_lookback(status.as<uint64_t>(), pass_words * np + ceil_div(np, (uint64_t)2) + 1, tickets, s);
    bool inB = false;
    uint64_t pass = 0;
    for (int sh : shifts) {
        const K *ki = inB ? kB : kA;
        const VT *vi = inB ? vB : vA;
        K *ko = inB ? kA : kB;
        VT *vo = inB ? vA : vB;
        const uint32_t *b = bases + ((sh - lo) / rb) * kRadix;
        void *st = status.as<uint64_t>() + pass * pass_words;
        auto go = [&](auto s_c) {
            using S = decltype(s_c);
            if constexpr (ROLE == 1 && sizeof(VT) == 4) {
                if (rb == 7) {
                    onesweep_dispatch<K, S, ROLE, VT, 7>(tile, ki, vi, ko, vo, (uint32_t)n, sh, b, st,
                                                         tickets + pass, s);
                    return;
                }
            }
            onesweep_dispatch<K, S, ROLE, VT>(tile, ki, vi, ko, vo, (uint32_t)n, sh, b, st, tickets + pass, s);
        };
        if (narrow) go(uint32_t{});
        else go(uint64_t{});
        inB = !inB;
        ++pass;
    }
    // status/ticket are released stream-ordered (or by hipFree, which waits)
    return inB;
}

// Sorts packed 64-bit records (key above pay_bits payload bits) by the
// listed key digit shifts (digits of rb = 7 or 8 bits); returns true when
// the result ended up in B.
bool radix_sort_packed(uint64_t *A, uint64_t *B, uint64_t n, const std::vector<int> &shifts, int pay_bits,
                       const uint32_t *bases, int tile, hipStream_t s, int rb = kRadixBits, int lo = 0) {
    if (rb != 7 && rb != 8) fail(DOM_AGG_EHIP, "internal: %d-bit digits", rb);
    if (n == 0 || shifts.empty()) return false;
    tile = tile == 4096 ? 4096 : 8192;
    const bool narrow = n < (1ull << 30);
    const uint64_t pass_words = ceil_div(ceil_div(n, (uint64_t)tile) * kRadix * (narrow ? 4 : 8), (uint64_t)8);
    const uint64_t np = shifts.size();
    DevBuf status;
    status.alloc((pass_words * np + ceil_div(np, (uint64_t)2) + 1) * 8, s);
    uint32_t *tickets = reinterpret_cast<uint32_t *>(status.as<uint64_t>() + pass_words * np);
    clear_lookback(status.as<uint64_t>(), pass_words * np + ceil_div(np, (uint64_t)2) + 1, tickets, s);
    bool inB = false;
    uint64_t pass = 0;
    for (int sh : shifts) {
        const uint64_t *in = inB ? B : A;
        uint64_t *out = inB ? A : B;
        const uint32_t *b = bases + ((sh - lo) / rb) * kRadix;
        void *st = status.as<uint64_t>() + pass * pass_words;
        const unsigned tiles = (unsigned)ceil_div(n, (uint64_t)tile);
        const int shift = pay_bits + sh;
        auto go = [&](auto s_c) {
            using S = decltype(s_c);
            S *stw = static_cast<S *>(st);
            if (rb == 7 && tile == 4096)
                launch("onesweep_records_packed_t4096_d7", s, [&] {
                    onesweep_kernel<uint64_t, S, 256, 16, 1, uint32_t, false, 7><<<tiles, 256, 0, s>>>(
                        in, nullptr, out, nullptr, (uint32_t)n, shift, b, stw, tickets + pass);
                });
            else if (rb == 7)
                launch("onesweep_records_packed_t8192_d7", s, [&] {
                    onesweep_kernel<uint64_t, S, 512, 16, 1, uint32_t, false, 7><<<tiles, 512, 0, s>>>(
                        in, nullptr, out, nullptr, (uint32_t)n, shift, b, stw, tickets + pass);
                });
            else if (tile == 4096)
                launch("onesweep_records_packed_t4096", s, [&] {
                    onesweep_kernel<uint64_t, S, 256, 16, 1, uint32_t, false><<<tiles, 256, 0, s>>>(
                        in, nullptr, out, nullptr, (uint32_t)n, shift, b, stw, tickets + pass);
                });
            else
                launch("onesweep_records_packed_t8192", s, [&] {
                    onesweep_kernel<uint64_t, S, 512, 16, 1, uint32_t, false><<<tiles, 512, 0, s>>>(
                        in, nullptr, out, nullptr, (uint32_t)n, shift, b, stw, tickets + pass);
                });
        };
        if (narrow) go(uint32_t{});
        else go(uint64_t{});
        inB = !inB;
        ++pass;
    }
    return inB;
}

// Reduces part[nblocks][passes][256] to counts and exclusive bases [passes][256].
void reduce_hist(const uint32_t *part, int nblocks, int passes, uint32_t *counts, uint32_t *bases,
                 hipStream_t s) {
    const int R = std::max(1, std::min(64, nblocks));
    const int rows = (nblocks + R - 1) / R;
    DevBuf part2;
    part2.alloc((size_t)R * passes * kRadix * 4, s);
    launch("hist_reduce", s, [&] {
        hist_partial_kernel<<<dim3(passes, R), kRadix, 0, s>>>(part, nblocks, passes, rows, part2.as<uint32_t>());
    });
    launch("hist_reduce", s, [&] {
        hist_reduce_kernel<<<passes, kRadix, 0, s>>>(part2.as<uint32_t>(), R, passes, counts, bases);
    });
}

// Passes whose digit is not the same for every key (digits of rb bits from
// bit lo up).
std::vector<int> live_shifts(const uint32_t *counts, int passes, uint64_t n, int rb = kRadixBits, int lo = 0) {
    std::vector<int> sh;
    for (int p = 0; p < passes; ++p) {
        bool trivial = false;
        for (int d = 0; d < kRadix; ++d)
            if (counts[p * kRadix + d] == n) trivial = true;
        if (!trivial) sh.push_back(lo + p * rb);
    }
    return sh;
}

// ---------------------------------------------------------------------------
// Scan driver.

template <class Prob, int ITEMS>
void scan_launch(const char *name, const Prob &p, uint64_t n, uint64_t *status, uint64_t words_cap,
                 uint32_t *ticket, hipStream_t s) {
    if (n == 0) return;
    constexpr int TILE = kBlock * ITEMS;
    const uint64_t tiles = ceil_div(n, TILE);
    const uint64_t words = 2 * tiles * ScanStatusWords<typename Prob::V>::kWords;
    if (words > words_cap) fail(DOM_AGG_EHIP, "internal: scan status too small");
    clear_lookback(status, words, ticket, s);
    launch(name, s, [&] {
        seg_scan_kernel<Prob, kBlock, ITEMS><<<(unsigned)tiles, kBlock, 0, s>>>(p, n, status, ticket);
    });
}

// ---------------------------------------------------------------------------
// Plan construction, per-point part.

// Key-length classes of the record sort at digit width rb, over the key bits
// the sort reads (from sort_lo up; not for a basic-variant batch, whose
// instance bits sit above every node id, so nearly all keys would share one
// class).  Classes are merged from the short end until their histogram rows
// fit the flat map's LDS.  Returns false when the sort cannot run at this
// width (more digit passes than the kernels hold).
bool class_layout(Plan *P, int rb) {
    const int lo = P->sort_lo;
    const int cmax = std::max(1, (int)ceil_div(P->key_bits - lo, rb));
    if (cmax > kMaxPasses) return false;
    P->ncls = 1;
    P->cls_c0 = 0;
    P->cls_rows = 0;
    for (int q = 0; q < kMaxClasses; ++q) {
        P->cls_passes[q] = 0;
        P->cls_row0[q] = 0;
        P->cls_mask[q] = 0;
        P->cls_tot[q] = 0;
    }
    if ((P->batched && lo == 0) || P->nax < 1) return true;
    const int cmin = (int)ceil_div(P->field_shift[0] + 1 - lo, rb);
    const int cap = P->key64 ? 26 : 10;
    int nc = std::min(kMaxClasses, cmax - cmin + 1);
    while (nc >= 2 && nc * cmax - nc * (nc - 1) / 2 > cap) --nc;
    if (nc < 2) return true;
    P->ncls = nc;
    P->cls_c0 = cmax - nc + 1;
    int row = 0;
    for (int q = 0; q < nc; ++q) {
        P->cls_passes[q] = P->cls_c0 + q;
        P->cls_row0[q] = row;
        row += P->cls_passes[q];
    }
    P->cls_rows = row;
    const int L0 = P->Lmax[0];
    for (int j = 0; j < L0; ++j) {
        const int nominal = (int)ceil_div(P->field_shift[0] + j + 1 - lo, rb);
        const int q = std::max(nominal, P->cls_c0) - P->cls_c0;
        P->cls_mask[q] |= 1u << (L0 - 1 - j);
    }
    return true;
}

template <class C, class KP>
void build_points(Plan *P, const C *dq, const C *qq, const int64_t *doff, const int64_t *qoff,
                  hipStream_t s, HostStage &hs, DevBuf &sig_keys, DevBuf &sig_slots) {
    const uint32_t n = (uint32_t)P->n, nQ = (uint32_t)P->nQ;
    const int m = P->m, nax = P->nax;
    const int64_t ni = P->n_inst;

    DevBuf &inst_of_slot = P->inst_of_slot;
    DevBuf doff_dev, qoff_dev;
    if (P->batched) {
        doff_dev.alloc((ni + 1) * sizeof(int64_t), s);
        qoff_dev.alloc((ni + 1) * sizeof(int64_t), s);
        HIPCHK(hipMemcpyAsync(doff_dev.p, doff, (ni + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(qoff_dev.p, qoff, (ni + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
        inst_of_slot.alloc((size_t)n * sizeof(uint32_t), s);
        launch("instance_of_slot", s, [&] {
            instance_of_slot_kernel<<<(unsigned)ceil_div(n, kBlock), kBlock, 0, s>>>(
                qoff_dev.as<int64_t>(), doff_dev.as<int64_t>(), ni, nQ, n, inst_of_slot.as<uint32_t>());
        });
    }

    DevBuf &rank = P->rank;
    DevBuf kA, kB, vA, vB, kcount, nanflag, part, counts, bases, ppos, pr;
    // m = 2: the last axis is sorted with 64-bit payloads carrying each
    // point's rank and record payload (extract_sigma_kernel), after the key
    // layout is known; the count pass then reads them in sequence
    const bool sigv = nax == 1 && !P->basic;
    kA.alloc((size_t)n * sizeof(KP), s);
    kB.alloc((size_t)n * sizeof(KP), s);
    vA.alloc((size_t)n * 4, s);
    vB.alloc((size_t)n * 4, s);
    if (nax) {
        rank.alloc((size_t)nax * n * 4, s);
        kcount.alloc((size_t)nax * ni * 4, s);
        fill(kcount.as<uint32_t>(), (uint64_t)nax * ni, 0u, s);
        P->permuted = true;
        if (sigv) pr.alloc((size_t)n * 8, s);
        else ppos.alloc((size_t)n * 4, s);
        if (sigv && !P->batched) {
            P->cdf_d.alloc((size_t)n * 4, s);
            P->cdf_q.alloc((size_t)n * 4, s);
        }
        P->dinv.alloc((size_t)P->nD * 4, s);
        P->qinv.alloc((size_t)P->nQ * 4, s);
    }
    nanflag.alloc(4, s);
    fill(nanflag.as<uint32_t>(), 1, 0u, s);

    const int key_bits = 32 + (P->batched ? P->inst_bits : 0);
    const int passes = (int)ceil_div(key_bits, kRadixBits);
    const unsigned ext_blocks = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(ceil_div(n, kBlock), 1024));
    part.alloc((size_t)ext_blocks * passes * kRadix * 4, s);
    counts.alloc((size_t)passes * kRadix * 4, s);
    bases.alloc((size_t)passes * kRadix * 4, s);

    DevBuf scan_status, scan_ticket;
    scan_status.alloc((ceil_div(n, kBlock * 8) + 1) * sizeof(uint64_t) * 4, s);
    scan_ticket.alloc(16, s);

    // expanded axes first, the real (last) axis last
    for (int axis = 0; axis < (sigv ? 1 : m); ++axis) {
        // (the last axis with <=: data before queries on equal coordinates)
        const bool data_first = !P->basic && axis == m - 1 && ((P->le_mask >> axis) & 1u);
        launch("extract_keys", s, [&] {
            extract_keys_kernel<KP, C, kBlock><<<ext_blocks, kBlock, 0, s>>>(
                qq, dq, m, axis, nQ, n, inst_of_slot.as<uint32_t>(), axis > 0 ? ppos.as<uint32_t>() : nullptr,
                kA.as<KP>(), vA.as<uint32_t>(), passes, part.as<uint32_t>(), nanflag.as<uint32_t>(), data_first);
        });
        reduce_hist(part.as<uint32_t>(), (int)ext_blocks, passes, counts.as<uint32_t>(), bases.as<uint32_t>(), s);
        const size_t cb = (size_t)passes * kRadix * 4;
        uint32_t *h = static_cast<uint32_t *>(hs.get(cb + 4));
        HIPCHK(hipMemcpyAsync(h, counts.p, cb, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(h + passes * kRadix, nanflag.p, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (h[passes * kRadix]) fail(DOM_AGG_ENAN, "a coordinate on axis %d is NaN", axis);
        const std::vector<int> shifts = live_shifts(h, passes, n);
        const bool inB = radix_sort<KP, 0>(kA.as<KP>(), vA.as<uint32_t>(), kB.as<KP>(), vB.as<uint32_t>(), n,
                                        shifts, bases.as<uint32_t>(), P->tune.point_sort_tile, s);
        DevBuf &sk = inB ? kB : kA;
        DevBuf &sv = inB ? vB : vA;
        if (axis == 0 && nax > 0) {
            // ranks of the first axis, and the internal numbering of the points
            RankProblem<KP, true> rp{};
            rp.keys = sk.as<KP>();
            rp.slots = sv.as<uint32_t>();
            rp.rank = rank.as<uint32_t>();
            rp.kcount = kcount.as<uint32_t>();
            rp.n = n;
            rp.n_inst = (uint32_t)ni;
            rp.nQ = nQ;
            rp.doff = P->batched ? doff_dev.as<int64_t>() : nullptr;
            rp.qoff = P->batched ? qoff_dev.as<int64_t>() : nullptr;
            rp.ppos = ppos.as<uint32_t>();
            rp.pr = pr.as<uint64_t>();
            rp.cdf_d = P->cdf_d.as<uint32_t>();
            rp.cdf_q = P->cdf_q.as<uint32_t>();
            rp.dinv = P->dinv.as<uint32_t>();
            rp.qinv = P->qinv.as<uint32_t>();
            rp.nq_le = (P->le_mask & 1u) ? nQ : 0u;
            // (2048-element tiles: the rank scan's scattered per-point
            // stores want more resident tiles than its loads want long ones)
            scan_launch<RankProblem<KP, true>, 8>(
                "rank_scan", rp, n, scan_status.as<uint64_t>(), scan_status.bytes / 8,
                scan_ticket.as<uint32_t>(), s);
        } else if (axis < nax) {
            RankProblem<KP> rp{sk.as<KP>(), sv.as<uint32_t>(), rank.as<uint32_t>() + (size_t)axis * n,
                               kcount.as<uint32_t>() + (size_t)axis * ni, n, (uint32_t)ni};
            rp.nq_le = ((P->le_mask >> axis) & 1u) ? nQ : 0u;
            scan_launch<RankProblem<KP>, 8>(
                "rank_scan", rp, n, scan_status.as<uint64_t>(), scan_status.bytes / 8,
                scan_ticket.as<uint32_t>(), s);
        } else {
            sig_keys = std::move(sk);
            sig_slots = std::move(sv);
        }
    }
    if (P->basic) {
        // every axis was ranked; the flat map walks data first, then queries
        if (!ppos.p || nax != m) fail(DOM_AGG_EHIP, "internal: basic variant without internal slots");
        sig_keys.alloc((size_t)n * sizeof(KP), s);
        sig_slots.alloc((size_t)n * 4, s);
        launch("basic_order", s, [&] {
            basic_order_kernel<KP><<<grid_for(n), kBlock, 0, s>>>(nQ, n, inst_of_slot.as<uint32_t>(),
                                                                 ppos.as<uint32_t>(), sig_keys.as<KP>(),
                                                                 sig_slots.as<uint32_t>());
        });
    }

    // Bit widths per instance and axis (ceil(log2 K)), and the record key layout.
    std::vector<uint8_t> lt((size_t)nax * ni, 0);
    if (nax) {
        uint32_t *h = static_cast<uint32_t *>(hs.get((size_t)nax * ni * 4));
        HIPCHK(hipMemcpyAsync(h, kcount.p, (size_t)nax * ni * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        P->K0 = h[0];
        for (int a = 0; a < nax; ++a) {
            int lm = 0;
            for (int64_t k = 0; k < ni; ++k) {
                // (with <= the queries' ranks reach K: K + 1 values)
                const int L = bits_for((uint64_t)h[(size_t)a * ni + k] + ((P->le_mask >> a) & 1u));
                lt[(size_t)a * ni + k] = (uint8_t)L;
                lm = std::max(lm, L);
            }
            P->Lmax[a] = lm;
        }
    }
    // Key layout: node fields of the expanded axes (first axis highest).  In
    // a batch the instance id sits below them (not sorted on, see sort_lo),
    // except in the basic variant, whose points are not in instance order
    // (data of every instance first): there it sits above them.
    const bool inst_low = P->batched && !P->basic;
    P->sort_lo = inst_low ? P->inst_bits : 0;
    int sum = P->sort_lo;
    for (int a = nax - 1; a >= 0; --a) {
        P->field_shift[a] = sum;
        sum += P->Lmax[a];
    }
    P->inst_shift = P->batched && !inst_low ? sum : 0;
    P->key_bits = sum + (P->batched && !inst_low ? P->inst_bits : 0);
    if (P->key_bits > 64) fail(DOM_AGG_ETOOBIG, "record sort key needs %d bits (> 64)", P->key_bits);
    P->key64 = P->key_bits > 32;
    // Records as single 64-bit words when key and payload fit: 32 weight
    // bits with the query flag above the key's digits (records carrying
    // weights), else a flagged label of 1 + ceil(log2 max(|D|, |Q|)) bits.
    // Records carry their weights only when that packs (or packing is off):
    // a label record packs into fewer bytes than an unpacked weight record.
    const bool pack_ok = packing_enabled();
    P->pay_bits = 1 + bits_for((uint64_t)std::max<int64_t>(std::max(P->nD, P->nQ), 1));
    if (P->inline_req && nax > 0) {
        // the query flag goes one bit above the digits the record sort reads,
        // at either digit width
        int fs = 0;
        for (int rb : {7, 8})
            fs = std::max(fs, P->sort_lo + rb * std::max(1, (int)ceil_div(P->key_bits - P->sort_lo, rb)));
        const bool packs = pack_ok && fs + 1 + 32 <= 64;
        if (fs < 64 && (packs || !pack_ok)) {
            P->inline_w = true;
            P->flag_shift = fs;
            P->key64 = fs >= 32;
            P->packed = packs;
            if (packs) P->pay_bits = 32;
        }
    }
    if (!P->inline_w && pack_ok && P->key_bits + P->pay_bits <= 64) P->packed = true;
    DevBuf sig_vals64;
    if (sigv) {
        DevBuf wA, wB;
        wA.alloc((size_t)n * 8, s);
        wB.alloc((size_t)n * 8, s);
        launch("extract_keys", s, [&] {
            auto go = [&](auto *w) {
                using W = std::remove_const_t<std::remove_pointer_t<decltype(w)>>;
                extract_sigma_kernel<KP, C, W, kBlock><<<ext_blocks, kBlock, 0, s>>>(
                    qq, dq, 1, nQ, n, inst_of_slot.as<uint32_t>(), pr.as<uint64_t>(), w, P->inline_w, kA.as<KP>(),
                    wA.as<uint64_t>(), passes, part.as<uint32_t>(), nanflag.as<uint32_t>(),
                    ((P->le_mask >> 1) & 1u) != 0);
            };
            if (P->inline_w && P->w_dt == DOM_AGG_I32) go(static_cast<const int32_t *>(P->w_src));
            else go(P->inline_w ? static_cast<const float *>(P->w_src) : static_cast<const float *>(nullptr));
        });
        reduce_hist(part.as<uint32_t>(), (int)ext_blocks, passes, counts.as<uint32_t>(), bases.as<uint32_t>(), s);
        const size_t cb = (size_t)passes * kRadix * 4;
        uint32_t *h = static_cast<uint32_t *>(hs.get(cb + 4));
        HIPCHK(hipMemcpyAsync(h, counts.p, cb, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(h + passes * kRadix, nanflag.p, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (h[passes * kRadix]) fail(DOM_AGG_ENAN, "a coordinate on axis %d is NaN", m - 1);
        const std::vector<int> shifts = live_shifts(h, passes, n);
        const bool inB = radix_sort<KP, 0, uint64_t>(kA.as<KP>(), wA.as<uint64_t>(), kB.as<KP>(), wB.as<uint64_t>(),
                                                  n, shifts, bases.as<uint32_t>(), P->tune.point_sort_tile, s);
        sig_keys = std::move(inB ? kB : kA);
        sig_vals64 = std::move(inB ? wB : wA);
        pr.reset();
    }
    class_layout(P, P->rbits);
    {
        uint64_t S = 1;
        for (int a = 0; a < nax; ++a) S *= (uint64_t)std::max(P->Lmax[a], 1);
        const uint64_t rows = (uint64_t)std::max(P->nQ, P->nD);
        P->use_slots = nax == 0 || (S <= kMaxSlots && S * rows * 8 <= kMaxSlotBytes && !compact_forced());
        P->n_slots = (uint32_t)std::min<uint64_t>(S, 0xffffffffu);
    }

    if (nax) {
        P->ltab.alloc(lt.size(), s);
        HIPCHK(hipMemcpyAsync(P->ltab.p, lt.data(), lt.size(), hipMemcpyHostToDevice, s));
        P->rs.alloc((size_t)nax * n * 4, s);
    }
    P->off.alloc(((size_t)n + 1) * 8, s);
    P->pay.alloc((size_t)n * 4, s);
    if (P->batched) P->inst_s.alloc((size_t)n * 4, s);

    if (P->inline_w && !sigv) {
        // first-axis rank and weight bits side by side: the count scan's one
        // gather per point fetches both
        P->rw.alloc((size_t)n * 8, s);
        P->wv.alloc((size_t)n * 4, s);
        launch("pack_rank_weight", s, [&] {
            if (P->w_dt == DOM_AGG_I32)
                pack_rank_weight_kernel<int32_t><<<grid_for(n), kBlock, 0, s>>>(
                    rank.as<uint32_t>(), P->dinv.as<uint32_t>(), static_cast<const int32_t *>(P->w_src), nQ, n,
                    P->rw.as<uint64_t>());
            else
                pack_rank_weight_kernel<float><<<grid_for(n), kBlock, 0, s>>>(
                    rank.as<uint32_t>(), P->dinv.as<uint32_t>(), static_cast<const float *>(P->w_src), nQ, n,
                    P->rw.as<uint64_t>());
        });
    }
    if (sigv && P->inline_w) P->wv.alloc((size_t)n * 4, s);
    auto count_sigma = [&](auto inl_c) {
        constexpr bool INL = decltype(inl_c)::value;
        CountProblemSigma<KP, INL> cp{};
        cp.keys = sig_keys.as<KP>();
        cp.vals = sig_vals64.as<uint64_t>();
        cp.ltab = P->ltab.as<uint8_t>();
        cp.n_inst = (uint32_t)ni;
        cp.n = n;
        cp.off = P->off.as<uint64_t>();
        cp.rs = P->rs.as<uint32_t>();
        cp.pay = P->pay.as<uint32_t>();
        cp.inst_s = P->inst_s.as<uint32_t>();
        cp.wv = P->wv.as<uint32_t>();
        scan_launch<CountProblemSigma<KP, INL>, 8>("count_scan", cp, n, scan_status.as<uint64_t>(),
                                                   scan_status.bytes / 8, scan_ticket.as<uint32_t>(), s);
    };
    auto count = [&](auto nax_c) {
        constexpr int NAX = decltype(nax_c)::value;
        auto go = [&](auto inl_c) {
            constexpr bool INL = decltype(inl_c)::value;
            CountProblem<KP, NAX, INL> cp{sig_keys.as<KP>(), sig_slots.as<uint32_t>(), rank.as<uint32_t>(),
                                          P->ltab.as<uint8_t>(), (uint32_t)ni, nQ, n,
                                          P->off.as<uint64_t>(), P->rs.as<uint32_t>(), P->pay.as<uint32_t>(),
                                          P->inst_s.as<uint32_t>(), P->rw.as<uint64_t>(), P->wv.as<uint32_t>()};
            scan_launch<CountProblem<KP, NAX, INL>, sizeof(KP) == 4 ? 16 : 8>(
                "count_scan", cp, n, scan_status.as<uint64_t>(), scan_status.bytes / 8,
                scan_ticket.as<uint32_t>(), s);
        };
        if (NAX > 0 && P->inline_w) go(std::true_type{});
        else go(std::false_type{});
    };
    if (sigv) {
        if (P->inline_w) count_sigma(std::true_type{});
        else count_sigma(std::false_type{});
    } else {
        switch (nax) {
            case 0: count(std::integral_constant<int, 0>{}); break;
            case 1: count(std::integral_constant<int, 1>{}); break;
            case 2: count(std::integral_constant<int, 2>{}); break;
            default: count(std::integral_constant<int, 3>{}); break;
        }
    }
    sig_vals64.reset();
    uint64_t *h = static_cast<uint64_t *>(hs.get(8));
    HIPCHK(hipMemcpyAsync(h, P->off.as<uint64_t>() + n, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    P->E = (int64_t)*h;
    if ((uint64_t)P->E > kMaxRecords)
        fail(DOM_AGG_ETOOBIG, "flat map yields %lld records (limit %llu)", (long long)P->E,
             (unsigned long long)kMaxRecords);
}

// Digit passes of the record key whose digit is skewed: those holding the
// top bits of a tree-node field (node ids at level j have their leading 1 at
// bit j, so most ids are small) or instance bits.
uint32_t skewed_passes(const Plan *P) {
    uint32_t skew = 0;
    auto mark = [&](int lo, int hi) {  // bits [lo, hi)
        for (int p = 0; p < kMaxPasses; ++p)
            if (P->sort_lo + p * P->rbits < hi && P->sort_lo + (p + 1) * P->rbits > lo) skew |= 1u << p;
    };
    for (int a = 0; a < P->nax; ++a) {
        const int top = P->field_shift[a] + P->Lmax[a];  // one past the field's top bit
        if (P->Lmax[a] > 0) mark(top - 1, top);
    }
    if (P->batched && P->sort_lo == 0) mark(P->inst_shift, P->inst_shift + P->inst_bits);
    return skew;
}

// ---------------------------------------------------------------------------
// The flat map and the record sort.  With `probe`, the histogram is read back
// to find the live radix passes (stored in the plan); otherwise the stored
// passes are used with no host synchronisation before the sort.

template <class K>
void build_records(Plan *P, hipStream_t s, HostStage *hs, bool probe, DevBuf &outK, DevBuf &outV) {
    const uint64_t E = (uint64_t)P->E;
    const bool cls = P->ncls > 1;
    DevBuf kA, kB, vA, vB, part, counts, bases, cstat, ticket;
    const bool pk = P->packed;
    if (pk) {
        // packed words live in the key buffers; no payload arrays
        kA.alloc(E * 8, s);
        if (cls) kB.alloc(E * 8, s);
    } else {
        kA.alloc(E * sizeof(K), s);
        vA.alloc(E * 4, s);
        if (cls) {
            kB.alloc(E * sizeof(K), s);
            vB.alloc(E * 4, s);
        }
    }
    const int rb = P->rbits, lo = P->sort_lo;
    const int passes = cls ? P->cls_passes[P->ncls - 1] : std::max(1, (int)ceil_div(P->key_bits - lo, rb));
    const int rows = cls ? P->cls_rows : passes;
    if (rows > (sizeof(K) == 4 ? 10 : 26) || passes > kMaxPasses)
        fail(DOM_AGG_EHIP, "internal: %d histogram rows for %d-byte keys", rows, (int)sizeof(K));
    constexpr int EITEMS = 8;
    constexpr int CHUNK = kBlock * EITEMS;
    constexpr int CHUNK_SHIFT = 11;
    static_assert((1 << CHUNK_SHIFT) == CHUNK, "");
    const uint64_t nchunks = ceil_div(E, CHUNK);
    auto per_nax = [&](auto &&f) {
        switch (P->nax) {
            case 0: f(std::integral_constant<int, 0>{}); break;
            case 1: f(std::integral_constant<int, 1>{}); break;
            case 2: f(std::integral_constant<int, 2>{}); break;
            default: f(std::integral_constant<int, 3>{}); break;
        }
    };
    // The digit histograms: m = 2 with classes from the rank CDFs per tree
    // node (not with <= on the first axis: the CDFs are of the unshifted
    // ranks); otherwise from the points in closed form, unless the instance
    // id is among the sorted key bits (basic-variant batches) or there is no
    // expanded axis: then inside the flat map's per-record loop.  (Per record,
    // in the flat map or in a pass over the records, they cost 1.8 ms at
    // m = 3, |D| = |Q| = 2^20.)
    const bool can_points = P->nax >= 1 && P->inst_shift == 0;
    HistSource hsrc = (cls && P->cdf_d.p && P->m == 2 && !(P->le_mask & 1u)) ? HistSource::kNodes
                      : can_points                                            ? HistSource::kPoints
                                                                              : HistSource::kEmit;
    switch (hist_source_override()) {
        case 1: if (can_points) hsrc = HistSource::kPoints; break;
        case 2: hsrc = HistSource::kRecords; break;
        case 3: hsrc = HistSource::kEmit; break;
        default: break;
    }
    const bool node_hist = hsrc == HistSource::kNodes;
    const bool point_hist = hsrc == HistSource::kPoints;
    const bool sep_hist = hsrc == HistSource::kRecords;
    const bool emit_hist = hsrc == HistSource::kEmit;
    // the flat map's workgroups: as many as are resident at once (each takes
    // a fixed share of the chunks)
    unsigned grid = 1;
    per_nax([&](auto nax_c) {
        constexpr int NAX = decltype(nax_c)::value;
        if (cls && !emit_hist) grid = resident_grid(emit_kernel<K, NAX, kBlock, EITEMS, true, false>, nchunks);
        else if (cls) grid = resident_grid(emit_kernel<K, NAX, kBlock, EITEMS, true>, nchunks);
        else if (!emit_hist) grid = resident_grid(emit_kernel<K, NAX, kBlock, EITEMS, false, false>, nchunks);
        else grid = resident_grid(emit_kernel<K, NAX, kBlock, EITEMS, false>, nchunks);
    });
    DevBuf chunk_k;
    chunk_k.alloc(nchunks * 4, s);
    launch("chunk_start", s, [&] {
        const unsigned g = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(ceil_div(P->n, kBlock), 4096));
        chunk_start_kernel<<<g, kBlock, 0, s>>>(P->off.as<uint64_t>(), (uint32_t)P->n, CHUNK_SHIFT,
                                                chunk_k.as<uint32_t>());
    });
    part.alloc((size_t)grid * rows * kRadix * 4, s);
    counts.alloc((size_t)rows * kRadix * 4, s);
    bases.alloc((size_t)rows * kRadix * 4, s);
    if (!P->ed_counter.p) P->ed_counter.alloc(8, s);
    fill(P->ed_counter.as<unsigned long long>(), 1, 0ull, s);

    EmitArgs a{};
    a.off = P->off.as<uint64_t>();
    a.rs = P->rs.as<uint32_t>();
    a.pay = P->pay.as<uint32_t>();
    a.inst_s = P->inst_s.as<uint32_t>();
    a.ltab = P->ltab.as<uint8_t>();
    a.chunk_k = chunk_k.as<uint32_t>();
    a.n = (uint32_t)P->n;
    a.n_inst = (uint32_t)P->n_inst;
    a.E = E;
    for (int i = 0; i < 3; ++i) a.field_shift[i] = P->field_shift[i];
    a.inst_shift = P->inst_shift;
    a.passes = passes;
    a.hist_part = part.as<uint32_t>();
    a.data_records = P->ed_counter.as<unsigned long long>();
    a.wv = P->inline_w ? P->wv.as<uint32_t>() : nullptr;
    a.flag_shift = P->inline_w ? P->flag_shift : -1;
    a.pk_a = pk ? kA.as<uint64_t>() : nullptr;
    a.pk_b = pk && cls ? kB.as<uint64_t>() : nullptr;
    a.pk_shift = P->pay_bits;
    a.pk_labels = !P->inline_w;
    a.ncls = P->ncls;
    a.cls_c0 = P->cls_c0;
    a.hist_rows = rows;
    a.rbits = rb;
    a.sort_lo = lo;
    a.skew = skewed_passes(P);
    a.lmax0 = P->nax > 0 ? P->Lmax[0] : 0;
    for (int q = 0; q < kMaxClasses; ++q) {
        a.cls_passes[q] = P->cls_passes[q];
        a.cls_row0[q] = P->cls_row0[q];
        a.cls_mask[q] = P->cls_mask[q];
    }
    DevBuf npart;
    unsigned ngrid = 0;
    if (node_hist) {
        const uint64_t nodes = 1ull << P->Lmax[0];
        ngrid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(ceil_div(nodes, kBlock), 2048));
        npart.alloc((size_t)ngrid * rows * kRadix * 4, s);
        EmitArgs na = a;
        na.hist_part = npart.as<uint32_t>();
        launch("node_hist", s, [&] {
            node_hist_kernel<<<ngrid, kBlock, 0, s>>>(P->cdf_d.as<uint32_t>(), P->cdf_q.as<uint32_t>(), P->K0,
                                                     (uint32_t)P->nD, (uint32_t)P->nQ, P->Lmax[0], na);
        });
        a.hist_part = nullptr;  // the flat map skips its histograms
    }
    if (point_hist) {
        ngrid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(ceil_div(P->n, kBlock), 2048));
        npart.alloc((size_t)ngrid * rows * kRadix * 4, s);
        EmitArgs pa = a;
        pa.hist_part = npart.as<uint32_t>();
        per_nax([&](auto nax_c) {
            constexpr int NAX = decltype(nax_c)::value;
            if constexpr (NAX >= 1) {
                launch("point_hist", s, [&] { point_hist_kernel<NAX><<<ngrid, kBlock, 0, s>>>(pa); });
            }
        });
        a.hist_part = nullptr;
    }
    if (cls) {
        // Records of each class per chunk (closed form over the points), their
        // exclusive sums over the chunks (each chunk's class offsets, so the
        // emitter's chunks never wait on each other) and the class totals.
        static_assert(kBlock == 256, "chunk kernels use 256-thread workgroups");
        const uint64_t ngroups = ceil_div(nchunks, (uint64_t)kChunkGroup);
        DevBuf ccnt, gsum, tot;
        ccnt.alloc(nchunks * 8, s);
        gsum.alloc(ngroups * 16, s);
        tot.alloc(kMaxClasses * 8, s);
        cstat.alloc(nchunks * 16, s);
        fill(ccnt.as<unsigned long long>(), nchunks, 0ull, s);
        per_nax([&](auto nax_c) {
            constexpr int NAX = decltype(nax_c)::value;
            launch("chunk_class", s, [&] {
                chunk_class_kernel<NAX><<<grid_for(P->n), kBlock, 0, s>>>(a, CHUNK_SHIFT, ccnt.as<unsigned long long>());
            });
        });
        launch("chunk_offsets", s, [&] {
            chunk_group_kernel<<<(unsigned)ngroups, kBlock, 0, s>>>(ccnt.as<unsigned long long>(), nchunks,
                                                                    gsum.as<unsigned long long>());
        });
        launch("chunk_offsets", s, [&] {
            chunk_offsets_kernel<<<(unsigned)ngroups, kBlock, 0, s>>>(
                ccnt.as<unsigned long long>(), gsum.as<unsigned long long>(), nchunks, cstat.as<uint4>(),
                tot.as<unsigned long long>());
        });
        if (probe) {
            uint64_t *h = static_cast<uint64_t *>(hs->get(kMaxClasses * 8));
            HIPCHK(hipMemcpyAsync(h, tot.p, kMaxClasses * 8, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            uint64_t sum = 0;
            for (int q = 0; q < kMaxClasses; ++q) {
                P->cls_tot[q] = h[q];
                sum += h[q];
            }
            if (sum != E) fail(DOM_AGG_EHIP, "internal: class totals %llu != E %llu", (unsigned long long)sum,
                               (unsigned long long)E);
        }
        uint64_t base = 0;
        for (int q = 0; q < kMaxClasses; ++q) {
            a.cls_base[q] = base;
            base += P->cls_tot[q];
        }
    }
    ticket.alloc(16, s);
    fill(ticket.as<uint32_t>(), 2, 0u, s);  // (word 1: the error flag)
    a.cls_off = cstat.as<uint32_t>();
    a.error = ticket.as<uint32_t>() + 1;
    // (packed records: the key and payload arrays are not written)
    K *ka = pk ? nullptr : kA.as<K>(), *kb = pk ? nullptr : kB.as<K>();
    uint32_t *va = vA.as<uint32_t>(), *vb = vB.as<uint32_t>();
    if (sep_hist) a.hist_part = nullptr;  // (histograms after the flat map)
    per_nax([&](auto nax_c) {
        constexpr int NAX = decltype(nax_c)::value;
        launch("flatmap_emit", s, [&] {
            if (cls && !a.hist_part)
                emit_kernel<K, NAX, kBlock, EITEMS, true, false><<<grid, kBlock, 0, s>>>(a, ka, va, kb, vb);
            else if (cls)
                emit_kernel<K, NAX, kBlock, EITEMS, true><<<grid, kBlock, 0, s>>>(a, ka, va, kb, vb);
            else if (!a.hist_part)
                emit_kernel<K, NAX, kBlock, EITEMS, false, false><<<grid, kBlock, 0, s>>>(a, ka, va, nullptr, nullptr);
            else
                emit_kernel<K, NAX, kBlock, EITEMS, false><<<grid, kBlock, 0, s>>>(a, ka, va, nullptr, nullptr);
        });
    });
    if (node_hist || point_hist) {
        reduce_hist(npart.as<uint32_t>(), (int)ngrid, rows, counts.as<uint32_t>(), bases.as<uint32_t>(), s);
    } else if (sep_hist) {
        RecHistArgs h{};
        h.pk[0] = pk ? kA.as<uint64_t>() : nullptr;
        h.pk[1] = pk ? kB.as<uint64_t>() : nullptr;
        h.keys[0] = pk ? nullptr : kA.p;
        h.keys[1] = pk ? nullptr : kB.p;
        h.E = E;
        h.ncls = P->ncls;
        for (int q = 0; q < kMaxClasses; ++q) {
            h.cls_base[q] = a.cls_base[q];
            h.cls_passes[q] = P->cls_passes[q];
            h.cls_row0[q] = P->cls_row0[q];
            h.cls_in_b[q] = (P->cls_passes[q] & 1) ? 0 : 1;  // (see EmitArgs: odd-pass classes start in A)
        }
        h.passes = passes;
        h.pay_bits = P->pay_bits;
        h.rows = rows;
        h.rbits = rb;
        h.sort_lo = lo;
        h.skew = skewed_passes(P);
        const unsigned hgrid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(ceil_div(E, kBlock * 4), 1024));
        DevBuf hpart;
        hpart.alloc((size_t)hgrid * rows * kRadix * 4, s);
        h.hist_part = hpart.as<uint32_t>();
        launch("record_hist", s, [&] {
            if (pk) record_hist_kernel<K, true><<<hgrid, kBlock, 0, s>>>(h);
            else record_hist_kernel<K, false><<<hgrid, kBlock, 0, s>>>(h);
        });
        reduce_hist(hpart.as<uint32_t>(), (int)hgrid, rows, counts.as<uint32_t>(), bases.as<uint32_t>(), s);
    } else {
        reduce_hist(part.as<uint32_t>(), (int)grid, rows, counts.as<uint32_t>(), bases.as<uint32_t>(), s);
    }
    if (probe) {
        const size_t cb = (size_t)rows * kRadix * 4;
        uint32_t *h = static_cast<uint32_t *>(hs->get(cb + 12));
        HIPCHK(hipMemcpyAsync(h, counts.p, cb, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(h + rows * kRadix, P->ed_counter.p, 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(h + rows * kRadix + 2, ticket.as<uint32_t>() + 1, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (h[rows * kRadix + 2]) fail(DOM_AGG_EHIP, "internal: flat-map records disagree with their class counts");
        if (cls) {
            P->rec_shifts.clear();
            for (int p = 0; p < passes; ++p) P->rec_shifts.push_back(lo + p * rb);
        } else {
            P->rec_shifts = P->key_bits > lo ? live_shifts(h, passes, E, rb, lo) : std::vector<int>{};
        }
        uint64_t ed;
        std::memcpy(&ed, h + rows * kRadix, 8);
        P->E_D = (int64_t)ed;
    }
    if (cls) {
        // every region ends in B (see EmitArgs)
        for (int q = 0; q < P->ncls; ++q) {
            const uint64_t nq = P->cls_tot[q];
            if (nq == 0) continue;
            const int np = P->cls_passes[q];
            std::vector<int> shifts;
            for (int p = 0; p < np; ++p) shifts.push_back(lo + p * rb);
            const uint64_t b = a.cls_base[q];
            const uint32_t *cb = bases.as<uint32_t>() + (size_t)P->cls_row0[q] * kRadix;
            if (pk) {
                uint64_t *pa = kA.as<uint64_t>() + b, *pb = kB.as<uint64_t>() + b;
                if (np & 1)
                    radix_sort_packed(pa, pb, nq, shifts, P->pay_bits, cb, P->tune.record_sort_tile, s, rb, lo);
                else
                    radix_sort_packed(pb, pa, nq, shifts, P->pay_bits, cb, P->tune.record_sort_tile, s, rb, lo);
            } else if (np & 1)
                radix_sort<K, 1>(kA.as<K>() + b, vA.as<uint32_t>() + b, kB.as<K>() + b, vB.as<uint32_t>() + b, nq,
                                 shifts, cb, P->tune.record_sort_tile, s, rb, lo);
            else
                radix_sort<K, 1>(kB.as<K>() + b, vB.as<uint32_t>() + b, kA.as<K>() + b, vA.as<uint32_t>() + b, nq,
                                 shifts, cb, P->tune.record_sort_tile, s, rb, lo);
        }
        outK = std::move(kB);
        outV = std::move(vB);
        return;
    }
    bool inB = false;
    if (!P->rec_shifts.empty()) {
        if (pk) {
            kB.alloc(E * 8, s);
            inB = radix_sort_packed(kA.as<uint64_t>(), kB.as<uint64_t>(), E, P->rec_shifts, P->pay_bits,
                                    bases.as<uint32_t>(), P->tune.record_sort_tile, s, rb, lo);
        } else {
            kB.alloc(E * sizeof(K), s);
            vB.alloc(E * 4, s);
            inB = radix_sort<K, 1>(kA.as<K>(), vA.as<uint32_t>(), kB.as<K>(), vB.as<uint32_t>(), E, P->rec_shifts,
                                bases.as<uint32_t>(), P->tune.record_sort_tile, s, rb, lo);
        }
    }
    outK = std::move(inB ? kB : kA);
    outV = std::move(inB ? vB : vA);
}

// How the scans read the plan's sorted records: packed words (kp) or a key
// array (kp) and a payload array (vp).
template <class K, bool PK>
RecSrc<K, PK> rec_src(const Plan *P, const void *kp, const uint32_t *vp) {
    RecSrc<K, PK> r{};
    if (PK) {
        r.packed = static_cast<const uint64_t *>(kp);
        r.pay_bits = P->pay_bits;  // (label payloads unless the records carry weights)
    } else {
        r.keys = static_cast<const K *>(kp);
        r.vals = vp;
    }
    return r;
}

void records_for_call(Plan *P, hipStream_t s, DevBuf &k, DevBuf &v, const void **kp, const uint32_t **vp) {
    if (P->flags & DOM_AGG_RECOMPUTE) {
        if (P->key64) build_records<uint64_t>(P, s, nullptr, false, k, v);
        else build_records<uint32_t>(P, s, nullptr, false, k, v);
        *kp = k.p;
        *vp = v.as<uint32_t>();
    } else {
        *kp = P->rkeys.p;
        *vp = P->rvals.as<uint32_t>();
    }
}

// ---------------------------------------------------------------------------
// Forward and backward.

RegroupArgs regroup_args(const Plan *P, bool queries) {
    RegroupArgs r{};
    r.inv = P->permuted ? (queries ? P->qinv.as<uint32_t>() : P->dinv.as<uint32_t>()) : nullptr;
    r.cstate = P->cstate.p ? P->cstate.as<uint4>() + (queries ? 0 : P->nQ) : nullptr;
    r.cap = (uint64_t)(queries ? P->E - P->E_D : P->E_D);
    r.rank = P->rank.as<uint32_t>();
    r.inst_of_slot = P->inst_of_slot.as<uint32_t>();
    r.ltab = P->ltab.as<uint8_t>();
    r.n = (uint32_t)P->n;
    r.n_inst = (uint32_t)P->n_inst;
    r.slot_base = queries ? 0u : (uint32_t)P->nQ;
    r.digit = queries ? 1u : 0u;
    const SlotMap sm = P->slot_map();
    for (int a = 0; a < 3; ++a) r.radix[a] = sm.radix[a];
    r.nout = (uint64_t)(queries ? P->nQ : P->nD);
    return r;
}

template <class V, int OP>
void regroup(const Plan *P, bool queries, const V *part, V *out, hipStream_t s) {
    const RegroupArgs ra = regroup_args(P, queries);
    const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(ceil_div(ra.nout, kBlock), 8192));
    if (!P->use_slots) {
        // (one wavefront per row)
        const unsigned cgrid = (unsigned)std::max<uint64_t>(
            1, std::min<uint64_t>(ceil_div(ra.nout, (uint64_t)(kBlock / kWave)), 8192));
        launch("regroup", s,
               [&] { regroup_compact_kernel<V, OP><<<cgrid, kBlock, 0, s>>>(ra, P->nax, part, out); });
        return;
    }
    auto go = [&](auto nax_c) {
        constexpr int NAX = decltype(nax_c)::value;
        launch("regroup", s, [&] { regroup_kernel<V, OP, NAX><<<grid, kBlock, 0, s>>>(ra, part, out); });
    };
    switch (P->nax) {
        case 0: go(std::integral_constant<int, 0>{}); break;
        case 1: go(std::integral_constant<int, 1>{}); break;
        case 2: go(std::integral_constant<int, 2>{}); break;
        default: go(std::integral_constant<int, 3>{}); break;
    }
}

template <class V, int OP>
V host_identity() {
    if constexpr (OP == OP_MAX) {
        if constexpr (std::is_floating_point<V>::value) return -std::numeric_limits<V>::infinity();
        else return std::numeric_limits<V>::min();
    } else {
        return V(0);
    }
}

// The plan's per-call buffers, sized before any graph capture: inputs in
// internal order, and the table of the regrouping (slot or compact layout).
void ensure_part(Plan *P, size_t vbytes, hipStream_t s) {
    const size_t rows = (size_t)std::max(P->nQ, P->nD);
    if (P->permuted && P->perm.bytes < rows * 8) P->perm.alloc(rows * 8, s);
    if (P->nax == 0) return;
    const size_t places = (size_t)std::max(P->E - P->E_D, P->E_D);
    const size_t need = P->use_slots ? (size_t)P->n_slots * rows * vbytes : std::max<size_t>(places, 1) * vbytes;
    if (P->part.bytes < need) P->part.alloc(need, s);
}

// Where a scan stores the partials of queries (or data points): the
// regrouping table, or out itself when every point has one record (m = 1).
template <class V>
PartDest<V> part_dest(const Plan *P, bool queries, V *table) {
    PartDest<V> d{};
    d.part = table;
    d.stride = (uint64_t)(queries ? P->nQ : P->nD);
    if (P->nax > 0 && !P->use_slots) {
        d.cstate = P->cstate.as<uint4>() + (queries ? 0 : P->nQ);
        d.cap = (uint64_t)(queries ? P->E - P->E_D : P->E_D);
    } else {
        d.cstate = nullptr;
        d.cap = (uint64_t)(P->nax == 0 ? 1 : P->n_slots) * d.stride;
    }
    return d;
}

template <class T>
void gather(const T *src, const uint32_t *idx, T *dst, uint64_t n, hipStream_t s) {
    if (n == 0) return;
    launch("permute_in", s, [&] { gather_kernel<T><<<grid_for(n), kBlock, 0, s>>>(src, idx, dst, n); });
}

template <class T>
void scatter(const T *src, const uint32_t *idx, T *dst, uint64_t n, hipStream_t s) {
    if (n == 0) return;
    launch("permute_out", s, [&] { scatter_kernel<T><<<grid_for(n), kBlock, 0, s>>>(src, idx, dst, n); });
}

template <class K, class W, class V, int OP, bool INL, bool PK>
void forward_run_pk(Plan *P, const void *kp, const uint32_t *vp, const void *w, void *out, hipStream_t s) {
    ForwardProblem<K, W, V, OP, INL, PK> fp{};
    fp.rec = rec_src<K, PK>(P, kp, vp);
    fp.w = static_cast<const W *>(w);
    fp.flag_shift = P->flag_shift;
    fp.nw = (uint64_t)P->nD;
    if constexpr (OP != OP_COUNT && !INL) {
        if (P->permuted && P->nD > 0) {
            gather(static_cast<const W *>(w), P->dinv.as<uint32_t>(), P->perm.as<W>(), (uint64_t)P->nD, s);
            fp.w = P->perm.as<W>();
        }
    }
    V *const res = static_cast<V *>(out);
    fp.sm = P->slot_map();
    // m = 1: every query has exactly one record, so it is stored in place
    fp.q = part_dest<V>(P, true, P->nax == 0 ? res : P->part.as<V>());
    fp.d = PartDest<V>{};
    using FP = ForwardProblem<K, W, V, OP, INL, PK>;
    // (a name of its own when the records carry the weights: no weight is
    // gathered then, which the byte model of the timing report needs to know)
    const char *name = INL ? "forward_scan_inline" : "forward_scan";
    if (P->tune.scan_items == 8 || sizeof(K) == 8)
        scan_launch<FP, 8>(name, fp, (uint64_t)P->E, P->scan_status.as<uint64_t>(), P->scan_words,
                           P->scan_ticket.as<uint32_t>(), s);
    else
        scan_launch<FP, 16>(name, fp, (uint64_t)P->E, P->scan_status.as<uint64_t>(), P->scan_words,
                            P->scan_ticket.as<uint32_t>(), s);
    if (P->nax > 0) regroup<V, OP>(P, true, P->part.as<V>(), res, s);
}

template <class K, class W, class V, int OP, bool INL>
void forward_run(Plan *P, const void *kp, const uint32_t *vp, const void *w, void *out, hipStream_t s) {
    if (P->packed) forward_run_pk<K, W, V, OP, INL, true>(P, kp, vp, w, out, s);
    else forward_run_pk<K, W, V, OP, INL, false>(P, kp, vp, w, out, s);
}

// Records that carry weights were built for one (op, weight dtype); the
// scan then reads the weights from the records.
template <class K, class W, class V, int OP>
void forward_typed(Plan *P, const void *kp, const uint32_t *vp, const void *w, void *out, hipStream_t s) {
    if constexpr (OP == OP_COUNT || sizeof(W) == 4) {
        if (P->inline_w) return forward_run<K, W, V, OP, true>(P, kp, vp, w, out, s);
    }
    if (P->inline_w) fail(DOM_AGG_EHIP, "internal: records carry 4-byte weights");
    forward_run<K, W, V, OP, false>(P, kp, vp, w, out, s);
}

template <class K>
void forward_dispatch(Plan *P, dom_agg_op op, dom_agg_dtype wdt, const void *kp, const uint32_t *vp,
                      const void *w, void *out, hipStream_t s) {
    if (op == DOM_AGG_COUNT) return forward_typed<K, uint8_t, int64_t, OP_COUNT>(P, kp, vp, w, out, s);
    if (op == DOM_AGG_SUM) {
        switch (wdt) {
            case DOM_AGG_I32: return forward_typed<K, int32_t, int64_t, OP_SUM>(P, kp, vp, w, out, s);
            case DOM_AGG_I64: return forward_typed<K, int64_t, int64_t, OP_SUM>(P, kp, vp, w, out, s);
            case DOM_AGG_F32: return forward_typed<K, float, float, OP_SUM>(P, kp, vp, w, out, s);
            case DOM_AGG_F64: return forward_typed<K, double, double, OP_SUM>(P, kp, vp, w, out, s);
        }
    } else {
        switch (wdt) {
            case DOM_AGG_I32: return forward_typed<K, int32_t, int32_t, OP_MAX>(P, kp, vp, w, out, s);
            case DOM_AGG_I64: return forward_typed<K, int64_t, int64_t, OP_MAX>(P, kp, vp, w, out, s);
            case DOM_AGG_F32: return forward_typed<K, float, float, OP_MAX>(P, kp, vp, w, out, s);
            case DOM_AGG_F64: return forward_typed<K, double, double, OP_MAX>(P, kp, vp, w, out, s);
        }
    }
}

// The final list of Sec. 4 (instructions 6m+6 .. 6m+9): the forward scan
// keeping the partial aggregates of data records too, the regrouping of both
// kinds by point (their totals), the records per ID and their offsets, the
// IDs, and the broadcast of each ID's total along its run.
template <class K, class W, class V, int OP, bool PK>
void records_run_pk(Plan *P, const void *kp, const uint32_t *vp, const void *w, int64_t *ids, V *vals,
                 hipStream_t s) {
    const uint64_t nD = (uint64_t)P->nD, nQ = (uint64_t)P->nQ, n = (uint64_t)P->n, E = (uint64_t)P->E;
    const int nax = P->nax;
    DevBuf tq, td, totq, totd, wperm;
    totq.alloc(std::max<uint64_t>(nQ, 1) * sizeof(V), s);
    totd.alloc(std::max<uint64_t>(nD, 1) * sizeof(V), s);
    if (nax > 0) {
        const bool slots = P->use_slots;
        tq.alloc(std::max<uint64_t>(slots ? (uint64_t)P->n_slots * nQ : E - P->E_D, 1) * sizeof(V), s);
        td.alloc(std::max<uint64_t>(slots ? (uint64_t)P->n_slots * nD : P->E_D, 1) * sizeof(V), s);
    }
    ForwardProblem<K, W, V, OP, false, PK> fp{};
    fp.rec = rec_src<K, PK>(P, kp, vp);
    fp.w = static_cast<const W *>(w);
    fp.flag_shift = -1;
    fp.nw = nD;
    if constexpr (OP != OP_COUNT) {
        if (P->permuted && nD > 0) {
            wperm.alloc(nD * sizeof(W), s);
            gather(static_cast<const W *>(w), P->dinv.as<uint32_t>(), wperm.as<W>(), nD, s);
            fp.w = wperm.as<W>();
        }
    }
    fp.sm = P->slot_map();
    fp.q = part_dest<V>(P, true, nax == 0 ? totq.as<V>() : tq.as<V>());
    fp.d = part_dest<V>(P, false, nax == 0 ? totd.as<V>() : td.as<V>());
    using FP = ForwardProblem<K, W, V, OP, false, PK>;
    if (E > 0) {
        if (P->tune.scan_items == 8 || sizeof(K) == 8)
            scan_launch<FP, 8>("forward_scan", fp, E, P->scan_status.as<uint64_t>(), P->scan_words,
                               P->scan_ticket.as<uint32_t>(), s);
        else
            scan_launch<FP, 16>("forward_scan", fp, E, P->scan_status.as<uint64_t>(), P->scan_words,
                                P->scan_ticket.as<uint32_t>(), s);
    }
    if (nax > 0) {
        regroup<V, OP>(P, true, tq.as<V>(), totq.as<V>(), s);
        regroup<V, OP>(P, false, td.as<V>(), totd.as<V>(), s);
    }
    // records per ID, in ID order (data rows, then queries), and their offsets
    DevBuf drow, qrow, off, status, ticket;
    if (P->permuted) {
        drow.alloc(std::max<uint64_t>(nD, 1) * 4, s);
        qrow.alloc(std::max<uint64_t>(nQ, 1) * 4, s);
        launch("invert_perm", s, [&] {
            invert_perm_kernel<<<grid_for(nD), kBlock, 0, s>>>(P->dinv.as<uint32_t>(), nD, drow.as<uint32_t>());
        });
        launch("invert_perm", s, [&] {
            invert_perm_kernel<<<grid_for(nQ), kBlock, 0, s>>>(P->qinv.as<uint32_t>(), nQ, qrow.as<uint32_t>());
        });
    }
    off.alloc((n + 1) * 8, s);
    IdCountProblem ip{};
    ip.drow_pos = drow.as<uint32_t>();
    ip.qrow_pos = qrow.as<uint32_t>();
    ip.rank = P->rank.as<uint32_t>();
    ip.inst_of_slot = P->inst_of_slot.as<uint32_t>();
    ip.ltab = P->ltab.as<uint8_t>();
    ip.n = (uint32_t)n;
    ip.nD = (uint32_t)nD;
    ip.nQ = (uint32_t)nQ;
    ip.n_inst = (uint32_t)P->n_inst;
    ip.nax = nax;
    ip.off = off.as<uint64_t>();
    const uint64_t words = 2 * ceil_div(std::max(n, E), (uint64_t)kBlock * 8) * 2;
    status.alloc(words * 8, s);
    ticket.alloc(16, s);
    scan_launch<IdCountProblem, 8>("id_offsets", ip, n, status.as<uint64_t>(), words, ticket.as<uint32_t>(), s);
    launch("id_fill", s, [&] { id_fill_kernel<<<grid_for(n), kBlock, 0, s>>>(off.as<uint64_t>(), (uint32_t)n, E, ids); });
    BroadcastProblem<V, OP> bp{};
    bp.ids = ids;
    bp.tot_d = totd.as<V>();
    bp.tot_q = totq.as<V>();
    bp.nD = nD;
    bp.nQ = nQ;
    bp.vals = vals;
    scan_launch<BroadcastProblem<V, OP>, 8>("broadcast", bp, E, status.as<uint64_t>(), words, ticket.as<uint32_t>(),
                                            s);
}

template <class K, class W, class V, int OP>
void records_run(Plan *P, const void *kp, const uint32_t *vp, const void *w, int64_t *ids, V *vals,
                 hipStream_t s) {
    if (P->packed) records_run_pk<K, W, V, OP, true>(P, kp, vp, w, ids, vals, s);
    else records_run_pk<K, W, V, OP, false>(P, kp, vp, w, ids, vals, s);
}

template <class K>
void records_dispatch(Plan *P, dom_agg_op op, dom_agg_dtype wdt, const void *kp, const uint32_t *vp, const void *w,
                      int64_t *ids, void *vals, hipStream_t s) {
    if (op == DOM_AGG_COUNT)
        return records_run<K, uint8_t, int64_t, OP_COUNT>(P, kp, vp, w, ids, static_cast<int64_t *>(vals), s);
    if (op == DOM_AGG_SUM) {
        switch (wdt) {
            case DOM_AGG_I32: return records_run<K, int32_t, int64_t, OP_SUM>(P, kp, vp, w, ids, static_cast<int64_t *>(vals), s);
            case DOM_AGG_I64: return records_run<K, int64_t, int64_t, OP_SUM>(P, kp, vp, w, ids, static_cast<int64_t *>(vals), s);
            case DOM_AGG_F32: return records_run<K, float, float, OP_SUM>(P, kp, vp, w, ids, static_cast<float *>(vals), s);
            case DOM_AGG_F64: return records_run<K, double, double, OP_SUM>(P, kp, vp, w, ids, static_cast<double *>(vals), s);
        }
    } else {
        switch (wdt) {
            case DOM_AGG_I32: return records_run<K, int32_t, int32_t, OP_MAX>(P, kp, vp, w, ids, static_cast<int32_t *>(vals), s);
            case DOM_AGG_I64: return records_run<K, int64_t, int64_t, OP_MAX>(P, kp, vp, w, ids, static_cast<int64_t *>(vals), s);
            case DOM_AGG_F32: return records_run<K, float, float, OP_MAX>(P, kp, vp, w, ids, static_cast<float *>(vals), s);
            case DOM_AGG_F64: return records_run<K, double, double, OP_MAX>(P, kp, vp, w, ids, static_cast<double *>(vals), s);
        }
    }
}

template <class K, class G, bool PK>
void backward_typed_pk(Plan *P, const void *kp, const uint32_t *vp, const void *g, void *grad, hipStream_t s) {
    BackwardProblem<K, G, PK> bp{};
    bp.rec = rec_src<K, PK>(P, kp, vp);
    bp.g = static_cast<const G *>(g);
    if (P->permuted && P->nQ > 0) {
        gather(static_cast<const G *>(g), P->qinv.as<uint32_t>(), P->perm.as<G>(), (uint64_t)P->nQ, s);
        bp.g = P->perm.as<G>();
    }
    G *const res = static_cast<G *>(grad);
    bp.sm = P->slot_map();
    bp.d = part_dest<G>(P, false, P->nax == 0 ? res : P->part.as<G>());
    bp.ng = (uint64_t)P->nQ;
    bp.E = (uint64_t)P->E;
    if (P->tune.scan_items == 8 || sizeof(K) == 8)
        scan_launch<BackwardProblem<K, G, PK>, 8>("backward_scan", bp, (uint64_t)P->E, P->scan_status.as<uint64_t>(),
                                              P->scan_words, P->scan_ticket.as<uint32_t>(), s);
    else
        scan_launch<BackwardProblem<K, G, PK>, 16>("backward_scan", bp, (uint64_t)P->E, P->scan_status.as<uint64_t>(),
                                               P->scan_words, P->scan_ticket.as<uint32_t>(), s);
    if (P->nax > 0) regroup<G, OP_SUM>(P, false, P->part.as<G>(), res, s);
}

template <class K, class G>
void backward_typed(Plan *P, const void *kp, const uint32_t *vp, const void *g, void *grad, hipStream_t s) {
    if (P->packed) backward_typed_pk<K, G, true>(P, kp, vp, g, grad, s);
    else backward_typed_pk<K, G, false>(P, kp, vp, g, grad, s);
}

// Runs `body` directly, or through the plan's HIP graph in DOM_AGG_GRAPH mode.
template <class F>
void maybe_graph(Plan *P, const std::vector<uintptr_t> &key, hipStream_t s, F &&body) {
    if (!(P->flags & DOM_AGG_GRAPH) || (P->flags & DOM_AGG_RECOMPUTE)) {
        body(s);
        return;
    }
    hipGraphExec_t exec = nullptr;
    for (auto &g : P->graphs)
        if (g.first == key) exec = g.second;
    if (!exec) {
        if (P->graphs.size() >= kMaxGraphs) {
            (void)hipGraphExecDestroy(P->graphs.front().second);
            P->graphs.erase(P->graphs.begin());
        }
        if (!P->cap_stream) HIPCHK(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
        t_capturing = true;
        try {
            body(P->cap_stream);
        } catch (...) {
            t_capturing = false;
            hipGraph_t junk = nullptr;
            (void)hipStreamEndCapture(P->cap_stream, &junk);
            if (junk) (void)hipGraphDestroy(junk);
            throw;
        }
        t_capturing = false;
        HIPCHK(hipStreamEndCapture(P->cap_stream, &g));
        const hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIPCHK(e);
        P->graphs.emplace_back(key, exec);
        P->graph_captures++;
    }
    launch("graph_replay", s, [&] { HIPCHK(hipGraphLaunch(exec, s)); });
}


// ---------------------------------------------------------------------------
// Autotuner: times the record sort (flat map + radix passes) for each digit
// width and tile candidate, and the forward scan for each tile, on the plan's
// own records and keeps the fastest.  Results are cached per (device, record
// kind, key bits, ceil(log2 E)).  The sorted records depend on neither the
// digit width nor the tile, so the plan's records are kept as built; the
// per-width state (key-length classes, their totals, the live passes) is
// probed again for the width kept.

float time_ms(hipStream_t s, const std::function<void()> &f) {
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    HIPCHK(hipEventRecord(a, s));
    f();
    HIPCHK(hipEventRecord(b, s));
    HIPCHK(hipEventSynchronize(b));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms;
}

// The fastest of `reps` timed runs of f after one untimed run (which also
// takes the first launch of kernels not yet used in this process): one run
// alone is too noisy to rank candidates a few percent apart.
float best_of_ms(hipStream_t s, int reps, const std::function<void()> &f) {
    f();
    float best = 1e30f;
    for (int r = 0; r < reps; ++r) best = std::min(best, time_ms(s, f));
    return best;
}

// The cache's device name: architecture and compute-unit count.
std::string device_signature() {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    static std::mutex mu;
    static std::map<int, std::string> sig;
    std::lock_guard<std::mutex> lk(mu);
    auto it = sig.find(dev);
    if (it == sig.end()) {
        hipDeviceProp_t prop;
        HIPCHK(hipGetDeviceProperties(&prop, dev));
        it = sig.emplace(dev, std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount)).first;
    }
    return it->second;
}

// (records carrying weights, packed records and the basic variant are tuned
// separately: their keys and record widths differ; so are plans whose digit
// width DOM_AGG_DIGIT_BITS fixes)
TuneKey tune_key(const Plan *P) {
    const int kind = P->m | (P->inline_w ? 16 : 0) | (P->packed ? 32 : 0) | (P->basic ? 64 : 0) |
                     (P->batched ? 128 : 0) | (forced_digit_bits() << 8);
    return TuneKey{device_signature(), kind, P->key_bits, bits_for((uint64_t)P->E)};
}

// Builds the plan's records with the probe (class totals, live passes) and
// drops them.
void probe_records(Plan *P, hipStream_t s) {
    HostStage hs;
    DevBuf k, v;
    if (P->key64) build_records<uint64_t>(P, s, &hs, true, k, v);
    else build_records<uint32_t>(P, s, &hs, true, k, v);
}

// Applies a cached choice; called before the records are built, so that the
// plan's own record sort runs with it.
bool tune_lookup(Plan *P) {
    TuneCache &tc = TuneCache::get();
    if (!tc.enabled() || P->E <= 0) return false;
    TuneChoice c;
    if (!tc.lookup(tune_key(P), &c)) return false;
    if (c.digit_bits != P->rbits) {
        if (!class_layout(P, c.digit_bits)) return false;
        P->rbits = c.digit_bits;
    }
    P->tune.record_sort_tile = c.record_sort_tile;
    P->tune.scan_items = c.scan_items;
    P->tune.digit_bits = c.digit_bits;
    return true;
}

// Times the candidates (no cached choice yet) and stores the fastest.
void tune_plan(Plan *P, hipStream_t s) {
    TuneCache &tc = TuneCache::get();
    if (!tc.enabled() || P->E <= 0) return;
    const TuneKey key = tune_key(P);
    // the per-point state is still present here (plan construction)
    float best = 1e30f;
    int best_tile = P->tune.record_sort_tile, best_rb = P->rbits;
    int probed_rb = P->rbits;  // the width whose state the plan holds
    const int fdb = forced_digit_bits();
    for (int rb : {8, 7}) {
        if (fdb && rb != fdb) continue;
        if (rb != probed_rb) {
            if (!class_layout(P, rb)) continue;
            P->rbits = rb;
            probe_records(P, s);  // (also the first run at this width)
            probed_rb = rb;
        }
        for (int tile : {2048, 4096, 8192, 16384}) {
            if (effective_tile<uint32_t, 1>(tile) != tile || (P->key64 && tile == 16384)) continue;
            // (the packed sort's and the 7-bit sort's two tile shapes)
            if ((P->packed || rb == 7) && tile != 4096 && tile != 8192) continue;
            P->tune.record_sort_tile = tile;
            const float ms = best_of_ms(s, 2, [&] {
                DevBuf k, v;
                if (P->key64) build_records<uint64_t>(P, s, nullptr, false, k, v);
                else build_records<uint32_t>(P, s, nullptr, false, k, v);
            });
            if (ms < best) {
                best = ms;
                best_tile = tile;
                best_rb = rb;
            }
        }
    }
    if (best_rb != probed_rb) {
        if (!class_layout(P, best_rb)) fail(DOM_AGG_EHIP, "internal: digit width %d lost its layout", best_rb);
        P->rbits = best_rb;
        probe_records(P, s);
    }
    P->tune.record_sort_tile = best_tile;
    P->tune.digit_bits = best_rb;
    if (!P->key64 && P->rkeys.p && P->nQ > 0) {
        ensure_part(P, 8, s);
        DevBuf out;
        out.alloc((size_t)P->nQ * 8, s);
        best = 1e30f;
        int best_scan = P->tune.scan_items;
        for (int items : {8, 16}) {
            P->tune.scan_items = items;
            const float ms = best_of_ms(s, 2, [&] {
                forward_dispatch<uint32_t>(P, DOM_AGG_COUNT, DOM_AGG_I64, P->rkeys.p, P->rvals.as<uint32_t>(),
                                           nullptr, out.p, s);
            });
            if (ms < best) {
                best = ms;
                best_scan = items;
            }
        }
        P->tune.scan_items = best_scan;
    }
    tc.store(key, P->tune);
}


// Per-slot state of the compact regrouping layout (record counts, their
// exclusive sums per kind of point, and the selecting digits of the ranks).
void build_compact_state(Plan *P, hipStream_t s) {
    const uint64_t n = (uint64_t)P->n;
    P->cstate.alloc(n * sizeof(uint4), s);
    CompactStateProblem cp{};
    cp.rank = P->rank.as<uint32_t>();
    cp.inst_of_slot = P->inst_of_slot.as<uint32_t>();
    cp.ltab = P->ltab.as<uint8_t>();
    cp.n = (uint32_t)n;
    cp.nQ = (uint32_t)P->nQ;
    cp.n_inst = (uint32_t)P->n_inst;
    cp.nax = P->nax;
    cp.cstate = P->cstate.as<uint4>();
    const uint64_t words = 2 * ceil_div(n, (uint64_t)kBlock * 8) * ScanStatusWords<uint64_t>::kWords;
    DevBuf status, ticket;
    status.alloc(words * 8, s);
    ticket.alloc(16, s);
    scan_launch<CompactStateProblem, 8>("compact_state", cp, n, status.as<uint64_t>(), words,
                                        ticket.as<uint32_t>(), s);
}

// The DOM_AGG_LE bits valid for dimension m.
uint32_t le_flags(int m) {
    uint32_t f = 0;
    for (int a = 0; a < m && a < 4; ++a) f |= DOM_AGG_LE(a);
    return f;
}

// The basic variant expands every axis; the record key holds at most three
// tree-node fields.
void check_basic(int m, uint32_t flags) {
    if ((flags & DOM_AGG_BASIC) && m > 3)
        fail(DOM_AGG_EUNSUPPORTED, "the basic variant is provided for m <= 3 (m = %d)", m);
}

// Argument checks shared by dom_agg_plan and dom_agg_run (no HIP call).
void check_plan_args(int m, dom_agg_dtype coord_dtype, const void *d_coords, const void *q_coords, int64_t n_inst,
                     const int64_t *d_offsets, const int64_t *q_offsets) {
    if (m < 1 || m > 4) fail(DOM_AGG_EINVAL, "m = %d is outside [1, 4]", m);
    if (coord_dtype == DOM_AGG_F64 || coord_dtype == DOM_AGG_I64)
        fail(DOM_AGG_EUNSUPPORTED, "coordinates must be float32 or int32");
    if (coord_dtype != DOM_AGG_F32 && coord_dtype != DOM_AGG_I32)
        fail(DOM_AGG_EINVAL, "unknown coordinate dtype %d", (int)coord_dtype);
    if (n_inst < 1 || n_inst > (1ll << 30)) fail(DOM_AGG_EINVAL, "n_inst = %lld", (long long)n_inst);
    if (!d_offsets || !q_offsets) fail(DOM_AGG_EINVAL, "offsets are NULL");
    if (d_offsets[0] != 0 || q_offsets[0] != 0) fail(DOM_AGG_EINVAL, "offsets must start at 0");
    for (int64_t k = 0; k < n_inst; ++k)
        if (d_offsets[k + 1] < d_offsets[k] || q_offsets[k + 1] < q_offsets[k])
            fail(DOM_AGG_EINVAL, "offsets decrease at instance %lld", (long long)k);
    const int64_t nD = d_offsets[n_inst], nQ = q_offsets[n_inst];
    if (nD > 0 && !d_coords) fail(DOM_AGG_EINVAL, "d_coords is NULL with %lld data points", (long long)nD);
    if (nQ > 0 && !q_coords) fail(DOM_AGG_EINVAL, "q_coords is NULL with %lld queries", (long long)nQ);
    if (nD + nQ > 0x7fffffffll) fail(DOM_AGG_ETOOBIG, "|D| + |Q| must be below 2^31");
}

void check_forward_args(dom_agg_op op, dom_agg_dtype weight_dtype, const void *weights, const void *out, int64_t nD,
                        int64_t nQ) {
    if (op != DOM_AGG_SUM && op != DOM_AGG_MAX && op != DOM_AGG_COUNT) fail(DOM_AGG_EINVAL, "unknown op %d", (int)op);
    if (op != DOM_AGG_COUNT && (weight_dtype < DOM_AGG_I32 || weight_dtype > DOM_AGG_F64))
        fail(DOM_AGG_EINVAL, "unknown weight dtype %d", (int)weight_dtype);
    if (op != DOM_AGG_COUNT && nD > 0 && !weights) fail(DOM_AGG_EINVAL, "weights are NULL");
    if (nQ > 0 && !out) fail(DOM_AGG_EINVAL, "out is NULL");
}

size_t value_bytes(dom_agg_op op, dom_agg_dtype wdt) {
    const bool wide = op == DOM_AGG_COUNT || (op == DOM_AGG_SUM && wdt != DOM_AGG_F32) || wdt == DOM_AGG_I64 ||
                      wdt == DOM_AGG_F64;
    return wide ? 8 : 4;
}

// Builds a plan (validated arguments).  With inline_req, the records carry
// the weights w (4-byte dtype, or none for COUNT) when the key leaves room
// for the query flag.
std::unique_ptr<Plan> make_plan(int m, dom_agg_dtype coord_dtype, const void *d_coords, const void *q_coords,
                                int64_t n_inst, const int64_t *d_offsets, const int64_t *q_offsets, uint32_t flags,
                                hipStream_t s, const void *w, dom_agg_dtype wdt, bool inline_req) {
    const int64_t nD = d_offsets[n_inst], nQ = q_offsets[n_inst];
    int dev;
    require_gfx950(&dev);
    auto P = std::make_unique<Plan>();
    P->device = dev;
    P->m = m;
    P->flags = flags;
    P->le_mask = (flags >> 8) & 0xfu;
    P->basic = (flags & DOM_AGG_BASIC) != 0;
    P->nax = P->basic ? m : m - 1;  // (after basic is known)
    P->n_inst = n_inst;
    P->nD = nD;
    P->nQ = nQ;
    P->n = nD + nQ;
    P->batched = n_inst > 1;
    P->inst_bits = P->batched ? bits_for((uint64_t)n_inst) : 0;
    P->tune = default_tune();
    P->inline_req = inline_req;
    P->w_src = w;
    P->w_dt = wdt;
    if (P->n > 0) {
        HostStage hs;
        DevBuf sig_keys, sig_slots;
        if (coord_dtype == DOM_AGG_F32) {
            if (P->batched)
                build_points<float, uint64_t>(P.get(), (const float *)d_coords, (const float *)q_coords,
                                              d_offsets, q_offsets, s, hs, sig_keys, sig_slots);
            else
                build_points<float, uint32_t>(P.get(), (const float *)d_coords, (const float *)q_coords,
                                              d_offsets, q_offsets, s, hs, sig_keys, sig_slots);
        } else {
            if (P->batched)
                build_points<int32_t, uint64_t>(P.get(), (const int32_t *)d_coords, (const int32_t *)q_coords,
                                                d_offsets, q_offsets, s, hs, sig_keys, sig_slots);
            else
                build_points<int32_t, uint32_t>(P.get(), (const int32_t *)d_coords,
                                                (const int32_t *)q_coords, d_offsets, q_offsets, s, hs,
                                                sig_keys, sig_slots);
        }
        sig_keys.reset();
        sig_slots.reset();
        if (P->nax > 0 && !P->use_slots) build_compact_state(P.get(), s);
        const uint64_t tiles = ceil_div((uint64_t)std::max<int64_t>(P->E, 1), kBlock * 8);
        P->scan_words = tiles * 4;
        P->scan_status.alloc(P->scan_words * 8, s);
        P->scan_ticket.alloc(16, s);
        if (P->E > 0) {
            const bool tuned = !(flags & DOM_AGG_NO_TUNE) && tune_lookup(P.get());
            if (const int fdb = forced_digit_bits()) {
                if (fdb != P->rbits) {
                    if (!class_layout(P.get(), fdb))
                        fail(DOM_AGG_EINVAL, "the record key (%d bits) needs more than %d passes of %d-bit digits",
                             P->key_bits, kMaxPasses, fdb);
                    P->rbits = fdb;
                }
            }
            DevBuf k, v;
            if (P->key64) build_records<uint64_t>(P.get(), s, &hs, true, k, v);
            else build_records<uint32_t>(P.get(), s, &hs, true, k, v);
            P->rkeys = std::move(k);
            P->rvals = std::move(v);
            if (!(flags & DOM_AGG_NO_TUNE) && !tuned) tune_plan(P.get(), s);
            if (flags & DOM_AGG_RECOMPUTE) {
                P->rkeys.reset();
                P->rvals.reset();
            } else {
                // the last-axis-ordered state is only needed to rebuild the records
                P->rs.reset();
                P->pay.reset();
                P->inst_s.reset();
                P->off.reset();
                P->rw.reset();
                P->wv.reset();
                P->cdf_d.reset();
                P->cdf_q.reset();
            }
        }
        HIPCHK(hipStreamSynchronize(s));
    }
    return P;
}

void check_run_args(int m, dom_agg_dtype coord_dtype, const void *d_coords, const void *q_coords,
                    int64_t n_inst, const int64_t *d_offsets, const int64_t *q_offsets, dom_agg_op op,
                    dom_agg_dtype weight_dtype, const void *weights, const void *out, uint32_t flags) {
    check_plan_args(m, coord_dtype, d_coords, q_coords, n_inst, d_offsets, q_offsets);
    if (flags & ~(uint32_t)(DOM_AGG_NO_TUNE | DOM_AGG_BASIC | le_flags(m)))
        fail(DOM_AGG_EINVAL, "unknown flags 0x%x", flags);
    check_basic(m, flags);
    check_forward_args(op, weight_dtype, weights, out, d_offsets[n_inst], q_offsets[n_inst]);
}

// Plan + forward with records that carry the weights (dom_agg_run).
void run_oneshot(int m, dom_agg_dtype coord_dtype, const void *d_coords, const void *q_coords, int64_t n_inst,
                 const int64_t *d_offsets, const int64_t *q_offsets, dom_agg_op op, dom_agg_dtype weight_dtype,
                 const void *weights, void *out, uint32_t flags, void *stream) {
    check_run_args(m, coord_dtype, d_coords, q_coords, n_inst, d_offsets, q_offsets, op, weight_dtype, weights,
                   out, flags);
    if (q_offsets[n_inst] == 0) return;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // 4-byte weights (and no weights) travel inside the records
    const bool inl = op == DOM_AGG_COUNT || weight_dtype == DOM_AGG_I32 || weight_dtype == DOM_AGG_F32;
    auto P = make_plan(m, coord_dtype, d_coords, q_coords, n_inst, d_offsets, q_offsets, flags, s,
                       op == DOM_AGG_COUNT ? nullptr : weights, weight_dtype, inl);
    ensure_part(P.get(), value_bytes(op, weight_dtype), s);
    const void *kp = P->rkeys.p;
    const uint32_t *vp = P->rvals.as<uint32_t>();
    if (P->key64) forward_dispatch<uint64_t>(P.get(), op, weight_dtype, kp, vp, weights, out, s);
    else forward_dispatch<uint32_t>(P.get(), op, weight_dtype, kp, vp, weights, out, s);
    // the plan's buffers go back stream-ordered (or through hipFree, which waits)
}

}  // namespace

// ===========================================================================
// Exported entry points.

extern "C" {

const char *dom_agg_status_string(dom_agg_status st) {
    switch (st) {
        case DOM_AGG_OK: return "ok";
        case DOM_AGG_EINVAL: return "invalid argument";
        case DOM_AGG_ENAN: return "NaN coordinate";
        case DOM_AGG_ENOMEM: return "out of device memory";
        case DOM_AGG_ETOOBIG: return "problem too large";
        case DOM_AGG_EUNSUPPORTED: return "unsupported op or dtype";
        case DOM_AGG_ENODEV: return "no gfx950 device";
        case DOM_AGG_EHIP: return "HIP runtime error";
    }
    return "unknown status";
}

const char *dom_agg_last_error(void) { return t_last_error.c_str(); }

dom_agg_status dom_agg_set_allocator(dom_agg_alloc_fn alloc, dom_agg_release_fn release, void *ctx) {
    return guarded([&] {
        if ((alloc == nullptr) != (release == nullptr))
            fail(DOM_AGG_EINVAL, "alloc and release must both be set or both be NULL");
        g_alloc = alloc;
        g_release = release;
        g_alloc_ctx = ctx;
    });
}

dom_agg_status dom_agg_plan(dom_agg_plan_t *plan, int m, dom_agg_dtype coord_dtype, const void *d_coords,
                            const void *q_coords, int64_t n_inst, const int64_t *d_offsets,
                            const int64_t *q_offsets, uint32_t flags, void *stream) {
    return guarded([&] {
        if (!plan) fail(DOM_AGG_EINVAL, "plan is NULL");
        check_plan_args(m, coord_dtype, d_coords, q_coords, n_inst, d_offsets, q_offsets);
        if (flags & ~(uint32_t)(DOM_AGG_RECOMPUTE | DOM_AGG_GRAPH | DOM_AGG_NO_TUNE | DOM_AGG_BASIC | le_flags(m)))
            fail(DOM_AGG_EINVAL, "unknown flags 0x%x", flags);
        check_basic(m, flags);
        auto P = make_plan(m, coord_dtype, d_coords, q_coords, n_inst, d_offsets, q_offsets, flags,
                           static_cast<hipStream_t>(stream), nullptr, DOM_AGG_F32, false);
        *plan = P.release();
    });
}

dom_agg_status dom_agg_run(int m, dom_agg_dtype coord_dtype, const void *d_coords, const void *q_coords,
                           int64_t n_inst, const int64_t *d_offsets, const int64_t *q_offsets, dom_agg_op op,
                           dom_agg_dtype weight_dtype, const void *weights, void *out, uint32_t flags,
                           void *stream) {
    return guarded([&] {
        run_oneshot(m, coord_dtype, d_coords, q_coords, n_inst, d_offsets, q_offsets, op, weight_dtype, weights,
                    out, flags, stream);
    });
}

dom_agg_status dom_agg_run_static(int m, dom_agg_dtype coord_dtype, const void *d_coords, const void *q_coords,
                                  int64_t n_inst, const int64_t *d_offsets, const int64_t *q_offsets,
                                  dom_agg_op op, dom_agg_dtype weight_dtype, const void *weights, void *out,
                                  uint32_t flags, void *stream) {
    return guarded([&] {
        check_run_args(m, coord_dtype, d_coords, q_coords, n_inst, d_offsets, q_offsets, op, weight_dtype,
                       weights, out, flags);
        if (q_offsets[n_inst] == 0) return;
        int dev;
        require_gfx950(&dev);
        Arena arena{static_scratch(dev), kStaticScratchBytes, 0};
        ArenaScope scope(&arena);
        // (the tuner times candidates in buffers of their own: off here)
        run_oneshot(m, coord_dtype, d_coords, q_coords, n_inst, d_offsets, q_offsets, op, weight_dtype, weights,
                    out, flags | DOM_AGG_NO_TUNE, stream);
    });
}

dom_agg_status dom_agg_forward(dom_agg_plan_t plan, dom_agg_op op, dom_agg_dtype weight_dtype,
                               const void *weights, void *out, void *stream) {
    return guarded([&] {
        if (!plan) fail(DOM_AGG_EINVAL, "plan is NULL");
        check_forward_args(op, weight_dtype, weights, out, plan->nD, plan->nQ);
        if (plan->nQ == 0) return;
        int dev;
        require_gfx950(&dev);
        if (dev != plan->device) fail(DOM_AGG_EINVAL, "plan belongs to device %d, current is %d", plan->device, dev);
        hipStream_t s = static_cast<hipStream_t>(stream);
        ensure_part(plan, value_bytes(op, weight_dtype), s);
        const std::vector<uintptr_t> key{1, (uintptr_t)op, (uintptr_t)weight_dtype, (uintptr_t)weights,
                                         (uintptr_t)out};
        maybe_graph(plan, key, s, [&](hipStream_t cs) {
            DevBuf k, v;
            const void *kp = nullptr;
            const uint32_t *vp = nullptr;
            if (plan->E > 0) records_for_call(plan, cs, k, v, &kp, &vp);
            if (plan->key64) forward_dispatch<uint64_t>(plan, op, weight_dtype, kp, vp, weights, out, cs);
            else forward_dispatch<uint32_t>(plan, op, weight_dtype, kp, vp, weights, out, cs);
        });
    });
}

dom_agg_status dom_agg_forward_records(dom_agg_plan_t plan, dom_agg_op op, dom_agg_dtype weight_dtype,
                                       const void *weights, int64_t *ids, void *vals, void *stream) {
    return guarded([&] {
        if (!plan) fail(DOM_AGG_EINVAL, "plan is NULL");
        check_forward_args(op, weight_dtype, weights, vals, plan->nD, plan->E);
        if (plan->E > 0 && !ids) fail(DOM_AGG_EINVAL, "ids is NULL");
        if (plan->E == 0) return;
        int dev;
        require_gfx950(&dev);
        if (dev != plan->device) fail(DOM_AGG_EINVAL, "plan belongs to device %d, current is %d", plan->device, dev);
        hipStream_t s = static_cast<hipStream_t>(stream);
        DevBuf k, v;
        const void *kp = nullptr;
        const uint32_t *vp = nullptr;
        records_for_call(plan, s, k, v, &kp, &vp);
        if (plan->key64) records_dispatch<uint64_t>(plan, op, weight_dtype, kp, vp, weights, ids, vals, s);
        else records_dispatch<uint32_t>(plan, op, weight_dtype, kp, vp, weights, ids, vals, s);
    });
}

dom_agg_status dom_agg_backward(dom_agg_plan_t plan, dom_agg_dtype grad_dtype, const void *grad_out,
                                void *grad_weights, void *stream) {
    return guarded([&] {
        if (!plan) fail(DOM_AGG_EINVAL, "plan is NULL");
        if (grad_dtype == DOM_AGG_I32 || grad_dtype == DOM_AGG_I64)
            fail(DOM_AGG_EUNSUPPORTED, "the gradient is provided for float32 and float64 only");
        if (grad_dtype != DOM_AGG_F32 && grad_dtype != DOM_AGG_F64)
            fail(DOM_AGG_EINVAL, "unknown gradient dtype %d", (int)grad_dtype);
        if (plan->nQ > 0 && !grad_out) fail(DOM_AGG_EINVAL, "grad_out is NULL");
        if (plan->nD > 0 && !grad_weights) fail(DOM_AGG_EINVAL, "grad_weights is NULL");
        if (plan->nD == 0) return;
        int dev;
        require_gfx950(&dev);
        if (dev != plan->device) fail(DOM_AGG_EINVAL, "plan belongs to device %d, current is %d", plan->device, dev);
        hipStream_t s = static_cast<hipStream_t>(stream);
        ensure_part(plan, grad_dtype == DOM_AGG_F64 ? 8 : 4, s);
        const std::vector<uintptr_t> key{2, (uintptr_t)grad_dtype, (uintptr_t)grad_out, (uintptr_t)grad_weights};
        maybe_graph(plan, key, s, [&](hipStream_t cs) {
            DevBuf k, v;
            const void *kp = nullptr;
            const uint32_t *vp = nullptr;
            if (plan->E > 0) records_for_call(plan, cs, k, v, &kp, &vp);
            if (grad_dtype == DOM_AGG_F32) {
                if (plan->key64) backward_typed<uint64_t, float>(plan, kp, vp, grad_out, grad_weights, cs);
                else backward_typed<uint32_t, float>(plan, kp, vp, grad_out, grad_weights, cs);
            } else {
                if (plan->key64) backward_typed<uint64_t, double>(plan, kp, vp, grad_out, grad_weights, cs);
                else backward_typed<uint32_t, double>(plan, kp, vp, grad_out, grad_weights, cs);
            }
        });
    });
}

dom_agg_status dom_agg_plan_get_info(dom_agg_plan_t plan, dom_agg_plan_info *info) {
    return guarded([&] {
        if (!plan || !info) fail(DOM_AGG_EINVAL, "NULL argument");
        std::memset(info, 0, sizeof *info);
        info->n_inst = plan->n_inst;
        info->n_data = plan->nD;
        info->n_query = plan->nQ;
        info->records = plan->E;
        info->data_records = plan->E_D;
        info->m = plan->m;
        info->key_bits = plan->key_bits;
        for (int a = 0; a < 3; ++a) info->L[a] = plan->Lmax[a];  // (nax <= 3 axes)
        info->sort_passes = (int32_t)plan->rec_shifts.size();
        info->digit_bits = plan->rbits;
        info->sort_tile = plan->tune.record_sort_tile;
        info->scan_tile = kBlock * ((plan->tune.scan_items == 8 || plan->key64) ? 8 : 16);
        info->regroup_slots = plan->use_slots ? (int32_t)plan->n_slots : 0;
        info->sort_classes = plan->ncls;
        if (plan->ncls > 1)
            for (int q = 0; q < plan->ncls; ++q) info->sort_class_records[q] = (int64_t)plan->cls_tot[q];
        else
            info->sort_class_records[0] = plan->E;
        info->workspace_bytes = plan->workspace();
        info->le_mask = plan->le_mask;
        info->graph_captures = plan->graph_captures;
        info->record_bytes = plan->packed ? 8 : (plan->key64 ? 8 : 4) + 4;
        info->basic = plan->basic ? 1 : 0;
    });
}

void dom_agg_plan_destroy(dom_agg_plan_t plan) {
    if (!plan) return;
    for (auto &g : plan->graphs) (void)hipGraphExecDestroy(g.second);
    if (plan->cap_stream) (void)hipStreamDestroy(plan->cap_stream);
    delete plan;
}

dom_agg_status dom_agg_timing_enable(int enable) {
    return guarded([&] {
        std::lock_guard<std::mutex> lk(g_tmu);
        g_timing = enable != 0;
        for (auto &t : g_pending) {
            (void)hipEventSynchronize(t.b);
            g_event_pool.push_back(t.a);
            g_event_pool.push_back(t.b);
        }
        g_pending.clear();
        g_totals.clear();
    });
}

int dom_agg_timing_read(const char **names, double *total_ms, int64_t *launches, int cap) {
    std::lock_guard<std::mutex> lk(g_tmu);
    for (auto &t : g_pending) {
        if (hipEventSynchronize(t.b) != hipSuccess) return -1;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t.a, t.b) != hipSuccess) return -1;
        auto it = std::find_if(g_totals.begin(), g_totals.end(),
                               [&](const KernelTotal &k) { return std::strcmp(k.name, t.name) == 0; });
        if (it == g_totals.end()) g_totals.push_back({t.name, (double)ms, 1});
        else {
            it->ms += ms;
            it->launches += 1;
        }
        g_event_pool.push_back(t.a);
        g_event_pool.push_back(t.b);
    }
    g_pending.clear();
    const int k = (int)g_totals.size();
    for (int i = 0; i < k && i < cap; ++i) {
        if (names) names[i] = g_totals[i].name;
        if (total_ms) total_ms[i] = g_totals[i].ms;
        if (launches) launches[i] = g_totals[i].launches;
    }
    return k;
}

}  // extern "C"
