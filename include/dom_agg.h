/*
 * dom_agg — aggregation over dominated points on one AMD Instinct MI355X
 * (gfx950), computed by sorting, flat maps, segmented scans and zips as in
 * Sroka & Tyszkiewicz, "Aggregating over Dominated Points by Sorting,
 * Scanning, Zip and Flat Maps" (arXiv 2305.16751).
 *
 * The operation (Sec. 1.2 of the paper): data points D and queries Q in R^m,
 * weights w on D, and an associative, commutative F with unit e.  For every
 * query q the result is F over w(d) for all d in D with d < q in EVERY
 * coordinate (strict dominance), or e when there is none.
 *
 * The computation (Sec. 4 with the improvement of Sec. 5):
 *   plan     — coordinates only: per-axis dense ranks of axes 1..m-1 over D
 *              and Q jointly, the order of all points along axis m (queries
 *              before data on equal coordinates), the flat map of every point
 *              into the prefix sets of its binary ranks (Lemma 2), and one
 *              stable radix sort of the expanded records by bitstring tuple;
 *   forward  — the segmented scan of the weights over the sorted records and
 *              the regrouping of the partial aggregates by query;
 *   backward — for F = sum only: the transposed dominance sum
 *              grad_w[d] = sum of grad_out[q] over all q with d < q, as a
 *              reverse segmented scan over the same sorted records.
 *
 * Conventions shared by every entry point:
 *   - Device pointers: all coordinate, weight, output and gradient buffers
 *     live in device memory of the current HIP device and are owned by the
 *     caller.  Host pointers are marked (host) below.
 *   - Streams: every call is ordered on the given hipStream_t (passed as
 *     void*; NULL = the null stream).  dom_agg_plan blocks the host for a few
 *     small device-to-host reads (sizes); forward and backward do not block
 *     and allocate nothing, so they can be captured in a HIP graph.
 *   - Errors: every call returns a status; nothing throws across the
 *     boundary.  Arguments are validated before any HIP call is made.
 *     dom_agg_last_error() returns a message for the last failure on the
 *     calling thread.  A device fault is reported as DOM_AGG_EHIP by the
 *     first call that observes it.
 *   - Thread safety: a plan may be used by one thread at a time; distinct
 *     plans are independent.
 */
#ifndef DOM_AGG_H
#define DOM_AGG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DOM_AGG_OK = 0,
    DOM_AGG_EINVAL = 1,       /* an argument is invalid */
    DOM_AGG_ENAN = 2,         /* a coordinate is NaN (strict order undefined) */
    DOM_AGG_ENOMEM = 3,       /* a workspace allocation failed */
    DOM_AGG_ETOOBIG = 4,      /* > 2^32-1 expanded records, or sort keys wider than 64 bits */
    DOM_AGG_EUNSUPPORTED = 5, /* op / dtype combination not provided */
    DOM_AGG_ENODEV = 6,       /* no gfx950 device is current */
    DOM_AGG_EHIP = 7          /* a HIP runtime call failed */
} dom_agg_status;

typedef enum {
    DOM_AGG_SUM = 0,   /* e = 0 */
    DOM_AGG_MAX = 1,   /* e = the weight dtype's minimum (-inf for floats) */
    DOM_AGG_COUNT = 2  /* sum of unit weights; weights ignored (may be NULL) */
} dom_agg_op;

typedef enum {
    DOM_AGG_I32 = 0,
    DOM_AGG_I64 = 1,
    DOM_AGG_F32 = 2,
    DOM_AGG_F64 = 3
} dom_agg_dtype;

/* Plan flags. */
enum {
    /* Keep the sorted expanded records in the plan (default): forward and
     * backward only scan them. */
    DOM_AGG_KEEP = 0,
    /* Keep only the per-point state (ranks, point order, record offsets);
     * every forward/backward call rebuilds and re-sorts the expanded records
     * in a temporary workspace and frees it afterwards.  For when memory is
     * short.  Forward/backward then allocate, so they cannot be captured. */
    DOM_AGG_RECOMPUTE = 2,
    /* Capture forward/backward launches in a HIP graph on first use and
     * replay it on later calls with the same arguments (one graph is kept
     * per distinct call: kind, op, dtypes and buffers; up to 8 per plan). */
    DOM_AGG_GRAPH = 4,
    /* Skip the autotuner and use the built-in tile and digit widths. */
    DOM_AGG_NO_TUNE = 8,
    /* The basic variant of Sec. 4 instead of the Sec. 5 improvement: every
     * axis is replaced by binary ranks and expanded (n log^m n records), and
     * inside a run of equal tuples data precede queries.  Same results; a
     * second, independent GPU path.  m <= 3. */
    DOM_AGG_BASIC = 16
};

/* Non-strict dominance on chosen axes: with DOM_AGG_LE(a) in the flags of
 * dom_agg_plan or dom_agg_run, axis a (0-based, a < m) compares d_a <= q_a
 * instead of d_a < q_a (e.g. all axes for the multivariate empirical CDF,
 * the statistics use named in Sec. 1.2).  On an expanded axis the queries'
 * dense ranks move up by one, so that the strict comparison of Lemma 1
 * applies to (rank of d, rank of q + 1) with ceil(log2(K + 1)) digits; on the
 * last axis (Sec. 5) data precede queries on equal coordinates.  The
 * backward is then the transpose of that relation. */
#define DOM_AGG_LE(axis) (0x100u << (axis))

typedef struct dom_agg_plan_s *dom_agg_plan_t;

typedef struct {
    int64_t n_inst;        /* instances in the batch (1 for a plain call) */
    int64_t n_data;        /* |D| over all instances */
    int64_t n_query;       /* |Q| over all instances */
    int64_t records;       /* E: expanded records (Sec. 5 flat map) */
    int64_t data_records;  /* records that came from data points */
    int32_t m;             /* dimension */
    int32_t key_bits;      /* width of the record sort key */
    int32_t L[4];          /* max over instances of ceil(log2 K_i), axes 1..m-1 */
    int32_t sort_passes;   /* radix passes run by the record sort (its longest class) */
    int32_t digit_bits;    /* radix digit width chosen for the record sort */
    int32_t sort_tile;     /* records per workgroup tile in the record sort */
    int32_t scan_tile;     /* records per workgroup tile in the segmented scans */
    int32_t regroup_slots; /* level-tuple slots of the regrouping table; 0 = the
                              compact table (one place per record) */
    int32_t sort_classes;  /* key-length classes the record sort is split into (1 = none) */
    int64_t sort_class_records[4]; /* records per class (class c is sorted with
                                      sort_passes - sort_classes + 1 + c passes) */
    size_t workspace_bytes;/* device memory held by the plan */
    uint32_t le_mask;      /* bit a: <= on axis a (DOM_AGG_LE) */
    int32_t basic;         /* 1: the basic variant (DOM_AGG_BASIC), L has m entries */
    int64_t graph_captures;/* DOM_AGG_GRAPH: graphs captured so far (a call whose
                              arguments match a cached graph replays it) */
    int32_t record_bytes;  /* bytes per sorted record: 8 when key and payload are
                              packed into one 64-bit word, else key + 4 */
} dom_agg_plan_info;

/*
 * Device memory hook.  When set, every workspace allocation goes through
 * alloc(bytes, stream, ctx) and is returned with release(ptr, stream, ctx)
 * (e.g. PyTorch's caching allocator).  When unset, hipMalloc/hipFree are used.
 * alloc returns NULL on failure (reported as DOM_AGG_ENOMEM).  Process-wide;
 * pass NULLs to restore the default.  Not to be changed while plans exist.
 */
typedef void *(*dom_agg_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*dom_agg_release_fn)(void *ptr, void *stream, void *ctx);
dom_agg_status dom_agg_set_allocator(dom_agg_alloc_fn alloc, dom_agg_release_fn release,
                                     void *ctx);

/*
 * Build a plan from the coordinates (Sec. 4: union, ranks, binary ranks,
 * flat map, sort; Sec. 5: the last axis stays real and orders each segment).
 *
 *   plan        (host) receives the new plan; unchanged on failure.
 *   m           dimension, 1 <= m <= 4.
 *   coord_dtype DOM_AGG_F32 or DOM_AGG_I32.  -0.0 and +0.0 are equal; NaN is
 *               rejected with DOM_AGG_ENAN; +-inf order normally.
 *   d_coords    device, [n_data, m] row-major, n_data = d_offsets[n_inst].
 *   q_coords    device, [n_query, m] row-major, n_query = q_offsets[n_inst].
 *               Either may be NULL when its count is 0.  Read only during
 *               this call.
 *   n_inst      number of independent instances, >= 1.
 *   d_offsets   (host) [n_inst + 1] nondecreasing, d_offsets[0] = 0: instance
 *               k owns data rows d_offsets[k] .. d_offsets[k+1]-1.
 *   q_offsets   (host) likewise for queries.  Points of different instances
 *               never interact.
 *   flags       DOM_AGG_KEEP / DOM_AGG_RECOMPUTE | DOM_AGG_GRAPH | DOM_AGG_NO_TUNE
 *               | DOM_AGG_BASIC | DOM_AGG_LE(a) for any axes a < m.
 *   stream      hipStream_t.
 *
 * Errors: EINVAL (m, counts, offsets, NULL pointers with nonzero counts,
 * unknown flags or dtype), EUNSUPPORTED (DOM_AGG_BASIC with m = 4), ENAN,
 * ETOOBIG, ENOMEM, ENODEV, EHIP.
 */
dom_agg_status dom_agg_plan(dom_agg_plan_t *plan, int m, dom_agg_dtype coord_dtype,
                            const void *d_coords, const void *q_coords, int64_t n_inst,
                            const int64_t *d_offsets, const int64_t *q_offsets,
                            uint32_t flags, void *stream);

/*
 * Forward (Sec. 4: segmented scan of the weights over the sorted records,
 * then the regrouping by query ID).
 *
 *   op / weight_dtype   supported pairs and the output dtype:
 *       SUM   I32 -> I64, I64 -> I64, F32 -> F32 (fp32 accumulation),
 *             F64 -> F64
 *       MAX   I32 -> I32, I64 -> I64, F32 -> F32, F64 -> F64
 *       COUNT (weight_dtype ignored) -> I64
 *   weights  device, [n_data] of weight_dtype in data-row order (NULL for COUNT).
 *   out      device, [n_query] of the output dtype, fully overwritten.
 *
 * Integer results and MAX are exact.  fp32/fp64 sums are exact up to
 * rounding order, and that order is fixed for a plan (every fold, the
 * regrouping included, runs in an order set by the records alone), so
 * results repeat bit for bit; fp32 sums accumulate in a compensated pair of
 * floats, so long runs keep their error to a few units in the last place.
 */
dom_agg_status dom_agg_forward(dom_agg_plan_t plan, dom_agg_op op, dom_agg_dtype weight_dtype,
                               const void *weights, void *out, void *stream);

/*
 * The forward with the final list of Sec. 4 (instructions 6m+6 .. 6m+9:
 * sort by ID, shift, neutral_if_eq, segmented scan by ID) as its output:
 * every expanded record once, in nondecreasing ID order, each carrying the
 * total of its ID.  IDs follow the union of Sec. 4: data row i has ID i,
 * query row j has ID n_data + j (rows of the whole batch).  A query's total
 * is its result (dom_agg_forward); a data point's total is F over the
 * partial aggregates the scan leaves at its own records (F over the data of
 * each of its tuples up to it on the last axis), which the construction
 * carries along.  Each ID appears once per record of its point (zero times
 * when its prefix sets are empty).
 *
 *   op / weight_dtype / weights  as for dom_agg_forward.
 *   ids    device, [E] int64 (E = dom_agg_plan_info.records), overwritten.
 *   vals   device, [E] of the forward's output dtype, overwritten.
 *
 * Allocates its working buffers (not capturable).  Same numerics as the
 * forward (integer and max exact; fp32 sums compensated).
 */
dom_agg_status dom_agg_forward_records(dom_agg_plan_t plan, dom_agg_op op, dom_agg_dtype weight_dtype,
                                       const void *weights, int64_t *ids, void *vals, void *stream);

/*
 * Backward of the SUM forward with respect to the weights: the transposed
 * dominance sum grad_weights[d] = sum of grad_out[q] over all q with d < q.
 * It reuses the plan's sorted records (or rebuilds them under
 * DOM_AGG_RECOMPUTE) and scans them in reverse.
 *
 *   grad_dtype    DOM_AGG_F32 or DOM_AGG_F64 (of both buffers).
 *   grad_out      device, [n_query].
 *   grad_weights  device, [n_data], fully overwritten.
 */
dom_agg_status dom_agg_backward(dom_agg_plan_t plan, dom_agg_dtype grad_dtype,
                                const void *grad_out, void *grad_weights, void *stream);

/*
 * One-shot forward: dom_agg_plan + dom_agg_forward in one call, for callers
 * that need no plan afterwards (no backward, no second forward).  The
 * records of the flat map carry the weights themselves, as the expanded list
 * of the construction does (Sec. 4: each element of the union carries its
 * weight; Sec. 5), so the segmented scan reads them in sequence instead of
 * gathering them; query records are told apart by a flag bit above every key
 * digit the sort reads.  This holds for weight dtypes of 4 bytes (I32, F32)
 * and for COUNT, when m >= 2 and the record key leaves room for the flag;
 * otherwise the call runs a plan + forward internally.  Same results as
 * plan + forward (integer results and MAX exact, fp sums to rounding order).
 *
 *   m, coord_dtype, d_coords, q_coords, n_inst, d_offsets, q_offsets: as
 *       for dom_agg_plan;
 *   op, weight_dtype, weights, out: as for dom_agg_forward;
 *   flags    0 or DOM_AGG_NO_TUNE, | DOM_AGG_BASIC, | DOM_AGG_LE(a) for any
 *            axes a < m.
 *   stream   hipStream_t; the call synchronises with it while it sizes the
 *            flat map, and returns with the scan and the regrouping enqueued.
 *
 * Errors: those of dom_agg_plan and dom_agg_forward.
 */
dom_agg_status dom_agg_run(int m, dom_agg_dtype coord_dtype, const void *d_coords,
                           const void *q_coords, int64_t n_inst, const int64_t *d_offsets,
                           const int64_t *q_offsets, dom_agg_op op, dom_agg_dtype weight_dtype,
                           const void *weights, void *out, uint32_t flags, void *stream);

/*
 * dom_agg_run for callers that cannot allocate device memory: code being
 * captured into a HIP graph, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, validation and results as dom_agg_run (flags
 * as there; the autotuner is always off, as with DOM_AGG_NO_TUNE, so that
 * results equal dom_agg_run's with that flag bit for bit).  Every workspace
 * buffer of the call comes from one static device array of 256 MiB that the
 * library holds on each GPU it runs on until the process ends; no hipMalloc,
 * hipFree, pinned host allocation or allocator hook is called.  Problems whose
 * workspace does not fit return DOM_AGG_ETOOBIG before writing out (roughly:
 * m = 2 with |D| + |Q| up to about 2^20 uniform points; the size of the flat
 * map decides).  Every call on one GPU uses the same array, which keeps the
 * last call's contents: calls that overlap on one GPU (different streams or
 * threads) race and must not be issued.  The call synchronises with the
 * stream while it sizes the flat map, like dom_agg_run.
 */
dom_agg_status dom_agg_run_static(int m, dom_agg_dtype coord_dtype, const void *d_coords,
                                  const void *q_coords, int64_t n_inst, const int64_t *d_offsets,
                                  const int64_t *q_offsets, dom_agg_op op,
                                  dom_agg_dtype weight_dtype, const void *weights, void *out,
                                  uint32_t flags, void *stream);

/* Sizes of a plan.  info (host) is filled on success. */
dom_agg_status dom_agg_plan_get_info(dom_agg_plan_t plan, dom_agg_plan_info *info);

/* Releases the plan's device memory (stream-ordered on the plan's last
 * stream) and the plan.  NULL is ignored. */
void dom_agg_plan_destroy(dom_agg_plan_t plan);

/* Static text for a status code. */
const char *dom_agg_status_string(dom_agg_status status);

/* Message for the last failing call on this thread ("" if none). */
const char *dom_agg_last_error(void);

/*
 * Per-kernel timing, for measurement.  While enabled (process-wide), every
 * kernel the library launches is bracketed by a pair of HIP events recorded
 * on the stream it runs on.  dom_agg_timing_read waits for the recorded
 * events and writes, for up to `cap` distinct kernels, the kernel's name
 * (host, static string), the summed milliseconds and the number of launches
 * since the last dom_agg_timing_enable call; it returns the number of
 * distinct kernels (or -1 on a HIP error).  Enabling resets the totals.
 */
dom_agg_status dom_agg_timing_enable(int enable);
int dom_agg_timing_read(const char **names, double *total_ms, int64_t *launches, int cap);

#ifdef __cplusplus
}
#endif
#endif /* DOM_AGG_H */
