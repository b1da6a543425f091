/*
 * CPU oracle for aggregation over dominated points.  TEST INFRASTRUCTURE ONLY:
 * called by the tests, the smoke check and the benchmark's CPU-baseline leg,
 * never by the product library.  Plain, sequential, single-threaded C.
 *
 * Two independent computations live here:
 *   - the plain definition (Sec. 1.2), a double loop over D x Q;
 *   - the paper's construction (Sec. 4, with the Sec. 5 improvement, and the
 *     basic Sec. 4 variant), each step materialising its list the way the
 *     paper describes it: rank, expand by the prefix sets of Lemma 2, sort,
 *     segmented scan, sort by ID, segmented scan by ID.
 * The construction is checked against the definition (and against the
 * worked examples of Sec. 2.2 and Sec. 3, closed forms and invariants) by the
 * tests.
 *
 * Non-strict dominance (an extension for the ECDF use the paper names in
 * Sec. 1.2): bit a of le_mask asks for d_a <= q_a instead of d_a < q_a on
 * axis a.  On an expanded axis this is the strict comparison of the data
 * point's rank with the query's rank plus one (there are then K + 1 possible
 * ranks, written with ceil(log2(K + 1)) bits); on the last axis of Sec. 5 it
 * is the opposite tie rule, data before queries on equal coordinates.
 *
 * Readings taken where the paper leaves room (each is also listed in the
 * design notes):
 *   - the union of D and Q is their concatenation; |D| != |Q| is allowed;
 *   - ranks are computed jointly over D and Q and carried back to each
 *     point's ID before the per-point zip;
 *   - ranks are 0-based (1-based rank minus one) written with ceil(log2 K)
 *     bits, 0 bits when K <= 1 (then nothing can be strictly smaller);
 *   - a point whose prefix set is empty produces no record; outputs start at e;
 *   - only the aggregates at query records are regrouped; data-record
 *     partial aggregates are discarded.
 */
#define _GNU_SOURCE
#include "dom_agg_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* The monoid (F, e).                                                        */

typedef union {
    double f;
    int64_t i;
} val_t;

typedef struct {
    int is_float;
    int op; /* ORACLE_SUM or ORACLE_MAX; COUNT arrives as SUM with w = 1 */
    val_t e;
} monoid_t;

static val_t F(const monoid_t *M, val_t a, val_t b) {
    val_t r;
    if (M->is_float) {
        if (M->op == ORACLE_MAX)
            r.f = (b.f > a.f) ? b.f : a.f;
        else
            r.f = a.f + b.f;
    } else {
        if (M->op == ORACLE_MAX)
            r.i = (b.i > a.i) ? b.i : a.i;
        else
            r.i = a.i + b.i;
    }
    return r;
}

/* ------------------------------------------------------------------------ */
/* Plain definition.                                                         */

static int dominated(int m, const double *d, const double *q, int le_mask) {
    for (int k = 0; k < m; k++) {
        if ((le_mask >> k) & 1) {
            if (!(d[k] <= q[k])) return 0;
        } else if (!(d[k] < q[k])) {
            return 0;
        }
    }
    return 1;
}

static int has_nan(int64_t n, const double *x) {
    for (int64_t i = 0; i < n; i++)
        if (isnan(x[i])) return 1;
    return 0;
}

static int brute(int m, int64_t nD, const double *D, int64_t nQ,
                 const double *Q, const val_t *w, const monoid_t *M,
                 int le_mask, val_t *out) {
    for (int64_t j = 0; j < nQ; j++) {
        val_t acc = M->e;
        for (int64_t i = 0; i < nD; i++)
            if (dominated(m, D + i * m, Q + j * m, le_mask)) acc = F(M, acc, w[i]);
        out[j] = acc;
    }
    return 0;
}

static int check_common(int m, int64_t nD, const double *D, int64_t nQ,
                        const double *Q, int op) {
    if (m < 1 || m > ORACLE_MAX_DIM || nD < 0 || nQ < 0) return -1;
    if ((nD > 0 && !D) || (nQ > 0 && !Q)) return -1;
    if (op != ORACLE_SUM && op != ORACLE_MAX && op != ORACLE_COUNT) return -1;
    if (has_nan(nD * m, D) || has_nan(nQ * m, Q)) return -2;
    return 0;
}

int oracle_brute_le_f64(int m, int64_t nD, const double *D, int64_t nQ,
                        const double *Q, const double *w, int op, double e,
                        int le_mask, double *out) {
    int rc = check_common(m, nD, D, nQ, Q, op);
    if (rc) return rc;
    if (op == ORACLE_COUNT || (nD > 0 && !w) || (nQ > 0 && !out)) return -1;
    monoid_t M = {1, op, {.f = e}};
    /* double and val_t share size and representation of the float member */
    return brute(m, nD, D, nQ, Q, (const val_t *)w, &M, le_mask, (val_t *)out);
}

int oracle_brute_f64(int m, int64_t nD, const double *D, int64_t nQ,
                     const double *Q, const double *w, int op, double e,
                     double *out) {
    return oracle_brute_le_f64(m, nD, D, nQ, Q, w, op, e, 0, out);
}

int oracle_brute_i64(int m, int64_t nD, const double *D, int64_t nQ,
                     const double *Q, const int64_t *w, int op, int64_t e,
                     int64_t *out) {
    return oracle_brute_le_i64(m, nD, D, nQ, Q, w, op, e, 0, out);
}

int oracle_brute_le_i64(int m, int64_t nD, const double *D, int64_t nQ,
                        const double *Q, const int64_t *w, int op, int64_t e,
                        int le_mask, int64_t *out) {
    int rc = check_common(m, nD, D, nQ, Q, op);
    if (rc) return rc;
    if (nQ > 0 && !out) return -1;
    monoid_t M = {0, op == ORACLE_COUNT ? ORACLE_SUM : op, {.i = e}};
    val_t *ww = (val_t *)malloc(sizeof(val_t) * (size_t)(nD > 0 ? nD : 1));
    if (!ww) return -3;
    for (int64_t i = 0; i < nD; i++) {
        if (op == ORACLE_COUNT)
            ww[i].i = 1;
        else {
            if (!w) { free(ww); return -1; }
            ww[i].i = w[i];
        }
    }
    rc = brute(m, nD, D, nQ, Q, ww, &M, le_mask, (val_t *)out);
    free(ww);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Primitives of Sec. 2.2 and Sec. 3.                                        */

int oracle_sscan_f64(int64_t n, const double *a, const int64_t *t, int op,
                     double *out) {
    if (n < 0 || (n > 0 && (!a || !t || !out))) return -1;
    if (op != ORACLE_SUM && op != ORACLE_MAX) return -1;
    monoid_t M = {1, op, {.f = op == ORACLE_MAX ? -INFINITY : 0.0}};
    val_t acc = M.e;
    for (int64_t k = 0; k < n; k++) {
        if (k == 0 || t[k] != t[k - 1]) acc = M.e; /* a new maximal run */
        val_t x = {.f = a[k]};
        acc = F(&M, acc, x);
        out[k] = acc.f;
    }
    return 0;
}

int oracle_prefix_set(uint64_t x, int L, int bit, int *lens, uint64_t *vals) {
    if (L < 0 || L > 62 || (bit != 0 && bit != 1)) return -1;
    int c = 0;
    for (int j = 0; j < L; j++) {
        /* bit j of x counted from the most significant of its L digits */
        int b = (int)((x >> (L - 1 - j)) & 1u);
        if (b == bit) {
            lens[c] = j;
            vals[c] = j ? (x >> (L - j)) : 0; /* the first j digits */
            c++;
        }
    }
    return c;
}

int oracle_bits_for(int64_t K) {
    int L = 0;
    while (L < 62 && ((int64_t)1 << L) < K) L++;
    return L;
}

typedef struct {
    double x;
    int64_t id;
} xid_t;

static int xid_cmp(const void *pa, const void *pb) {
    const xid_t *a = (const xid_t *)pa, *b = (const xid_t *)pb;
    if (a->x < b->x) return -1;
    if (b->x < a->x) return 1;
    return (a->id > b->id) - (a->id < b->id);
}

int oracle_dense_rank(int64_t n, const double *v, int64_t *rank, int64_t *K) {
    if (n < 0 || (n > 0 && (!v || !rank)) || !K) return -1;
    if (has_nan(n, v)) return -2;
    xid_t *s = (xid_t *)malloc(sizeof(xid_t) * (size_t)(n > 0 ? n : 1));
    if (!s) return -3;
    for (int64_t i = 0; i < n; i++) {
        s[i].x = v[i];
        s[i].id = i;
    }
    /* sort the coordinate list, carrying the ID of each value */
    qsort(s, (size_t)n, sizeof(xid_t), xid_cmp);
    /* 1 where a value differs from its predecessor (the first value is
     * compared with -inf), summed by a prefix scan: the 1-based rank */
    int64_t R = 0;
    for (int64_t k = 0; k < n; k++) {
        if (k == 0 || s[k - 1].x < s[k].x) R++;
        rank[s[k].id] = R - 1;
    }
    *K = R; /* the broadcast maximum: number of distinct values */
    free(s);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The construction.                                                         */

/* A bitstring of length len <= 62 stored as its value; packed as
 * (len << 58) | value is not needed: two fields keep it readable. */
typedef struct {
    uint64_t v;
    int32_t len;
} bits_t;

/* Lexicographic order of bitstrings: compare the common prefix digit by
 * digit; when one is a prefix of the other, the shorter comes first. */
static int bits_cmp(bits_t a, bits_t b) {
    int c = a.len < b.len ? a.len : b.len;
    uint64_t pa = c ? (a.v >> (a.len - c)) : 0;
    uint64_t pb = c ? (b.v >> (b.len - c)) : 0;
    if (pa != pb) return pa < pb ? -1 : 1;
    if (a.len != b.len) return a.len < b.len ? -1 : 1;
    return 0;
}

typedef struct {
    bits_t t[ORACLE_MAX_DIM]; /* the tuple of bitstrings */
    double xm;                /* last coordinate, kept real (Sec. 5) */
    int64_t id;
    val_t w;                  /* weight; e for queries */
    int32_t is_query;
} rec_t;

typedef struct {
    int nt;      /* tuple length */
    int sec5;    /* 1: order (tuple, x_m, queries first, ID); 0: (tuple, data first, ID) */
    int last_le; /* Sec. 5 with <= on the last axis: data before queries on equal x_m */
} order_t;

static int rec_cmp(const void *pa, const void *pb, void *pctx) {
    const rec_t *a = (const rec_t *)pa, *b = (const rec_t *)pb;
    const order_t *o = (const order_t *)pctx;
    for (int i = 0; i < o->nt; i++) {
        int r = bits_cmp(a->t[i], b->t[i]);
        if (r) return r;
    }
    if (o->sec5) {
        if (a->xm < b->xm) return -1;
        if (b->xm < a->xm) return 1;
        if (a->is_query != b->is_query) return (a->is_query != o->last_le) ? -1 : 1;
    } else {
        if (a->is_query != b->is_query) return a->is_query ? 1 : -1;
    }
    return (a->id > b->id) - (a->id < b->id);
}

typedef struct {
    int64_t id;
    int64_t pos; /* position in the sorted expanded list, for a total order */
    val_t a;
} idval_t;

/* the order >=_ID (nonincreasing ID); equal IDs keep list order */
static int idval_cmp(const void *pa, const void *pb) {
    const idval_t *a = (const idval_t *)pa, *b = (const idval_t *)pb;
    if (a->id != b->id) return a->id > b->id ? -1 : 1;
    return (a->pos > b->pos) - (a->pos < b->pos);
}

/* Optional outputs of the construction beyond the per-query results. */
typedef struct {
    int le_mask;       /* bit a: <= on axis a (see the header comment) */
    /* The final list of Sec. 4 (instructions 6m+6 .. 6m+9): E entries in
     * nondecreasing ID order, each carrying the total of its ID.  NULL: not
     * built.  shortcut: build it instead by the segmented broadcast of the
     * maximum described before those instructions (valid when F(a, b) >= a). */
    int64_t *agg_ids;
    val_t *agg_vals;
    int64_t agg_cap;
    int shortcut;
} extras_t;

/*
 * The construction on n = nD + nQ points.  `nt` axes (the first nt of m) are
 * replaced by binary ranks and expanded; with sec5 the last axis stays real.
 */
static int construct(int m, int64_t nD, const double *D, int64_t nQ,
                     const double *Q, const val_t *wD, const monoid_t *M,
                     int sec5, val_t *out, int64_t *E_out, int *L_out,
                     const extras_t *X) {
    const int le_mask = X ? X->le_mask : 0;
    const int64_t n = nD + nQ;
    const int nt = sec5 ? m - 1 : m;
    int rc = 0;
    int64_t *rank = NULL;
    rec_t *ed = NULL;
    idval_t *a2 = NULL;
    val_t *a1 = NULL;
    double *col = NULL;
    int L[ORACLE_MAX_DIM] = {0};

    /* Union: DQ lists D then Q; the ID of D[i] is i, of Q[j] is nD + j. */
#define COORD(id, k) ((id) < nD ? D[(id) * m + (k)] : Q[((id) - nD) * m + (k)])

    /* Ranks of the expanded axes, computed over DQ jointly. */
    rank = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n * (nt > 0 ? nt : 1) + 1));
    col = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!rank || !col) { rc = -3; goto done; }
    for (int k = 0; k < nt; k++) {
        int64_t K = 0;
        for (int64_t id = 0; id < n; id++) col[id] = COORD(id, k);
        rc = oracle_dense_rank(n, col, rank + k * n, &K);
        if (rc) goto done;
        /* bin(rank, K): ceil(log2 K) digits; with <= on this axis the
         * queries' ranks move up by one, so K + 1 values occur */
        L[k] = oracle_bits_for(K + ((le_mask >> k) & 1));
        if ((le_mask >> k) & 1)
            for (int64_t id = nD; id < n; id++) rank[k * n + id] += 1;
        if (L_out) L_out[k] = L[k];
    }

    /* Flat map: a data point yields P0 of its binary rank tuple, a query P1
     * (the Cartesian product of the per-axis prefix sets, Lemma 2).  Count
     * first, then materialise. */
    int64_t E = 0;
    {
        int lens[64];
        uint64_t vals[64];
        for (int64_t id = 0; id < n; id++) {
            int64_t c = 1;
            for (int k = 0; k < nt; k++)
                c *= oracle_prefix_set((uint64_t)rank[k * n + id], L[k],
                                       id >= nD, lens, vals);
            E += c;
        }
    }
    if (E_out) *E_out = E;
    ed = (rec_t *)malloc(sizeof(rec_t) * (size_t)(E > 0 ? E : 1));
    if (!ed) { rc = -3; goto done; }
    {
        int64_t pos = 0;
        int cnt[ORACLE_MAX_DIM];
        int lens[ORACLE_MAX_DIM][64];
        uint64_t vals[ORACLE_MAX_DIM][64];
        for (int64_t id = 0; id < n; id++) {
            const int isq = id >= nD;
            int empty = 0;
            for (int k = 0; k < nt; k++) {
                cnt[k] = oracle_prefix_set((uint64_t)rank[k * n + id], L[k],
                                           isq, lens[k], vals[k]);
                if (cnt[k] == 0) empty = 1;
            }
            if (empty) continue;
            /* enumerate the product with a mixed-radix counter */
            int idx[ORACLE_MAX_DIM] = {0};
            for (;;) {
                rec_t *r = &ed[pos++];
                memset(r, 0, sizeof(*r));
                for (int k = 0; k < nt; k++) {
                    r->t[k].len = lens[k][idx[k]];
                    r->t[k].v = vals[k][idx[k]];
                }
                r->xm = sec5 ? COORD(id, m - 1) : 0.0;
                r->id = id;
                r->is_query = isq;
                r->w = isq ? M->e : wD[id];
                int k = nt - 1;
                while (k >= 0 && ++idx[k] == cnt[k]) idx[k--] = 0;
                if (k < 0) break;
            }
        }
        if (pos != E) { rc = -1; goto done; }
    }

    /* Sort in doubly lexicographic order (Sec. 5: then by the real last
     * coordinate, queries before data on equality; basic: data first). */
    {
        order_t o = {nt, sec5, sec5 ? (le_mask >> (m - 1)) & 1 : 0};
        qsort_r(ed, (size_t)E, sizeof(rec_t), rec_cmp, &o);
    }

    /* Segmented scan of the weights, tagged by the bitstring tuple. */
    a1 = (val_t *)malloc(sizeof(val_t) * (size_t)(E > 0 ? E : 1));
    if (!a1) { rc = -3; goto done; }
    {
        val_t acc = M->e;
        for (int64_t k = 0; k < E; k++) {
            int same = k > 0;
            for (int i = 0; same && i < nt; i++)
                same = bits_cmp(ed[k].t[i], ed[k - 1].t[i]) == 0;
            if (!same) acc = M->e;
            acc = F(M, acc, ed[k].w);
            a1[k] = acc;
        }
    }

    /* Sort the partial aggregates by ID (nonincreasing) and scan them with
     * the ID as the segment tag; the last entry of each ID run holds that
     * point's total.  Only query IDs are read out. */
    a2 = (idval_t *)malloc(sizeof(idval_t) * (size_t)(E > 0 ? E : 1));
    if (!a2) { rc = -3; goto done; }
    for (int64_t k = 0; k < E; k++) {
        a2[k].id = ed[k].id;
        a2[k].pos = k;
        a2[k].a = a1[k];
    }
    qsort(a2, (size_t)E, sizeof(idval_t), idval_cmp);
    for (int64_t j = 0; j < nQ; j++) out[j] = M->e;
    {
        val_t acc = M->e;
        for (int64_t k = 0; k < E; k++) {
            if (k == 0 || a2[k].id != a2[k - 1].id) acc = M->e;
            acc = F(M, acc, a2[k].a);
            a2[k].a = acc; /* A3: the scan tagged by ID */
            const int last = (k == E - 1) || a2[k + 1].id != a2[k].id;
            if (last && a2[k].id >= nD) out[a2[k].id - nD] = acc;
        }
    }
    if (X && X->agg_ids) {
        if (X->agg_cap < E) { rc = -4; goto done; }
        if (!X->shortcut) {
            /* A4: the reverse of A3, so IDs are nondecreasing and each ID's
             * complete aggregate comes first in its run; H: the IDs shifted
             * right by one (-inf first); A5: e wherever the ID equals its
             * predecessor; then the segmented scan of A5 tagged by ID. */
            val_t acc = M->e;
            for (int64_t k = 0; k < E; k++) {
                const idval_t *a4 = &a2[E - 1 - k];
                const int has_h = k > 0;
                const int64_t h = has_h ? a2[E - k].id : 0;
                const val_t a5 = (has_h && h == a4->id) ? M->e : a4->a;
                if (!has_h || h != a4->id) acc = M->e; /* a new run of equal IDs */
                acc = F(M, acc, a5);
                X->agg_ids[k] = a4->id;
                X->agg_vals[k] = acc;
            }
        } else {
            /* the segmented broadcast of the maximum over each ID run of A3
             * (its last entry, when F(a, b) >= a), listed in the same
             * nondecreasing ID order as the general tail */
            int64_t k = 0;
            while (k < E) {
                int64_t r = k;
                val_t mx = a2[k].a;
                while (r + 1 < E && a2[r + 1].id == a2[k].id) {
                    r++;
                    const int gt = M->is_float ? a2[r].a.f > mx.f : a2[r].a.i > mx.i;
                    if (gt) mx = a2[r].a;
                }
                for (int64_t t = k; t <= r; t++) {
                    X->agg_ids[E - 1 - t] = a2[k].id;
                    X->agg_vals[E - 1 - t] = mx;
                }
                k = r + 1;
            }
        }
    }
#undef COORD
done:
    free(rank);
    free(col);
    free(ed);
    free(a1);
    free(a2);
    return rc;
}

static int run_f64(int m, int64_t nD, const double *D, int64_t nQ,
                   const double *Q, const double *w, int op, double e,
                   double *out, int sec5, int64_t *E_out, int *L_out,
                   const extras_t *X) {
    int rc = check_common(m, nD, D, nQ, Q, op);
    if (rc) return rc;
    if (op == ORACLE_COUNT || (nD > 0 && !w) || (nQ > 0 && !out)) return -1;
    monoid_t M = {1, op, {.f = e}};
    return construct(m, nD, D, nQ, Q, (const val_t *)w, &M, sec5,
                     (val_t *)out, E_out, L_out, X);
}

static int run_i64(int m, int64_t nD, const double *D, int64_t nQ,
                   const double *Q, const int64_t *w, int op, int64_t e,
                   int64_t *out, int sec5, int64_t *E_out, int *L_out,
                   const extras_t *X) {
    int rc = check_common(m, nD, D, nQ, Q, op);
    if (rc) return rc;
    if ((nD > 0 && op != ORACLE_COUNT && !w) || (nQ > 0 && !out)) return -1;
    monoid_t M = {0, op == ORACLE_COUNT ? ORACLE_SUM : op, {.i = e}};
    val_t *ww = (val_t *)malloc(sizeof(val_t) * (size_t)(nD > 0 ? nD : 1));
    if (!ww) return -3;
    for (int64_t i = 0; i < nD; i++) ww[i].i = (op == ORACLE_COUNT) ? 1 : w[i];
    rc = construct(m, nD, D, nQ, Q, ww, &M, sec5, (val_t *)out, E_out, L_out, X);
    free(ww);
    return rc;
}

int oracle_dom_agg_f64(int m, int64_t nD, const double *D, int64_t nQ,
                       const double *Q, const double *w, int op, double e,
                       double *out, int64_t *E_out, int *L_out) {
    return run_f64(m, nD, D, nQ, Q, w, op, e, out, 1, E_out, L_out, NULL);
}

int oracle_dom_agg_i64(int m, int64_t nD, const double *D, int64_t nQ,
                       const double *Q, const int64_t *w, int op, int64_t e,
                       int64_t *out, int64_t *E_out, int *L_out) {
    return run_i64(m, nD, D, nQ, Q, w, op, e, out, 1, E_out, L_out, NULL);
}

int oracle_dom_agg_basic_f64(int m, int64_t nD, const double *D, int64_t nQ,
                             const double *Q, const double *w, int op,
                             double e, double *out, int64_t *E_out) {
    return run_f64(m, nD, D, nQ, Q, w, op, e, out, 0, E_out, NULL, NULL);
}

int oracle_dom_agg_basic_i64(int m, int64_t nD, const double *D, int64_t nQ,
                             const double *Q, const int64_t *w, int op,
                             int64_t e, int64_t *out, int64_t *E_out) {
    return run_i64(m, nD, D, nQ, Q, w, op, e, out, 0, E_out, NULL, NULL);
}

int oracle_dom_agg_ex_f64(int m, int64_t nD, const double *D, int64_t nQ,
                          const double *Q, const double *w, int op, double e,
                          int sec5, int le_mask, double *out, int64_t *E_out,
                          int *L_out, int64_t *agg_ids, double *agg_vals,
                          int64_t agg_cap, int shortcut) {
    extras_t X = {le_mask, agg_ids, (val_t *)agg_vals, agg_cap, shortcut};
    if (agg_ids && !agg_vals) return -1;
    return run_f64(m, nD, D, nQ, Q, w, op, e, out, sec5, E_out, L_out, &X);
}

int oracle_dom_agg_ex_i64(int m, int64_t nD, const double *D, int64_t nQ,
                          const double *Q, const int64_t *w, int op, int64_t e,
                          int sec5, int le_mask, int64_t *out, int64_t *E_out,
                          int *L_out, int64_t *agg_ids, int64_t *agg_vals,
                          int64_t agg_cap, int shortcut) {
    extras_t X = {le_mask, agg_ids, (val_t *)agg_vals, agg_cap, shortcut};
    if (agg_ids && !agg_vals) return -1;
    return run_i64(m, nD, D, nQ, Q, w, op, e, out, sec5, E_out, L_out, &X);
}

int oracle_transposed_sum_f64(int m, int64_t nD, const double *D, int64_t nQ,
                              const double *Q, const double *g, double *grad) {
    return oracle_transposed_sum_le_f64(m, nD, D, nQ, Q, g, 0, grad);
}

int oracle_transposed_sum_le_f64(int m, int64_t nD, const double *D,
                                 int64_t nQ, const double *Q, const double *g,
                                 int le_mask, double *grad) {
    int rc = check_common(m, nD, D, nQ, Q, ORACLE_SUM);
    if (rc) return rc;
    if ((nQ > 0 && !g) || (nD > 0 && !grad)) return -1;
    double *nd = (double *)malloc(sizeof(double) * (size_t)(nQ * m + 1));
    double *nq = (double *)malloc(sizeof(double) * (size_t)(nD * m + 1));
    if (!nd || !nq) { free(nd); free(nq); return -3; }
    /* the roles swap: queries become data (weights g), data become queries */
    for (int64_t i = 0; i < nQ * m; i++) nd[i] = -Q[i];
    for (int64_t i = 0; i < nD * m; i++) nq[i] = -D[i];
    /* d <= q on an axis  <=>  -q <= -d: the same le_mask applies */
    rc = oracle_dom_agg_ex_f64(m, nQ, nd, nD, nq, g, ORACLE_SUM, 0.0, 1, le_mask,
                               grad, NULL, NULL, NULL, NULL, 0, 0);
    free(nd);
    free(nq);
    return rc;
}
