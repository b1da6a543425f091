/*
 * Textbook sweep for two-dimensional dominance aggregation, used ONLY to pin
 * the oracle at sizes where the double loop of the definition is too slow.
 * TEST INFRASTRUCTURE ONLY.  It shares no code with the construction in
 * dom_agg_oracle.c: it is the classical sequential method (sweep along the
 * first axis, a Fenwick tree over ranks of the second axis), not the paper's.
 *
 * out[j] = F over w[i] with D[i].x < Q[j].x and D[i].y < Q[j].y, e if none.
 * Points are swept by ascending x; at equal x all queries are answered before
 * any data point is inserted, which makes the x comparison strict; the tree
 * is asked for the prefix of y-ranks strictly below the query's y-rank.
 * SUM and MAX (insert-only prefix maximum) are supported; COUNT is SUM with
 * unit weights supplied by the caller.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef struct {
    double x, y;
    int64_t idx;   /* index into D (kind 1) or Q (kind 0) */
    int kind;      /* 0 query, 1 data: queries sort first at equal x */
} sweep_pt;

static int sweep_cmp(const void *pa, const void *pb) {
    const sweep_pt *a = (const sweep_pt *)pa, *b = (const sweep_pt *)pb;
    if (a->x < b->x) return -1;
    if (b->x < a->x) return 1;
    if (a->kind != b->kind) return a->kind - b->kind;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

static int dbl_cmp(const void *pa, const void *pb) {
    double a = *(const double *)pa, b = *(const double *)pb;
    return (a > b) - (a < b);
}

/* number of distinct values strictly below v in the sorted distinct array u */
static int64_t below(const double *u, int64_t k, double v) {
    int64_t lo = 0, hi = k;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (u[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

static int prepare(int64_t nD, const double *D, int64_t nQ, const double *Q,
                   sweep_pt **pts_out, double **u_out, int64_t *k_out) {
    int64_t n = nD + nQ;
    sweep_pt *p = (sweep_pt *)malloc(sizeof(sweep_pt) * (size_t)(n + 1));
    double *u = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    if (!p || !u) { free(p); free(u); return -3; }
    for (int64_t i = 0; i < nD; i++) {
        if (isnan(D[2 * i]) || isnan(D[2 * i + 1])) { free(p); free(u); return -2; }
        p[i] = (sweep_pt){D[2 * i], D[2 * i + 1], i, 1};
        u[i] = D[2 * i + 1] == 0.0 ? 0.0 : D[2 * i + 1];
    }
    for (int64_t j = 0; j < nQ; j++) {
        if (isnan(Q[2 * j]) || isnan(Q[2 * j + 1])) { free(p); free(u); return -2; }
        p[nD + j] = (sweep_pt){Q[2 * j], Q[2 * j + 1], j, 0};
        u[nD + j] = Q[2 * j + 1] == 0.0 ? 0.0 : Q[2 * j + 1];
    }
    qsort(p, (size_t)n, sizeof(sweep_pt), sweep_cmp);
    qsort(u, (size_t)n, sizeof(double), dbl_cmp);
    int64_t k = 0;
    for (int64_t i = 0; i < n; i++)
        if (k == 0 || u[k - 1] < u[i]) u[k++] = u[i];
    *pts_out = p;
    *u_out = u;
    *k_out = k;
    return 0;
}

int pin_fenwick2_f64(int64_t nD, const double *D, int64_t nQ, const double *Q,
                     const double *w, int is_max, double e, double *out) {
    sweep_pt *p; double *u; int64_t k;
    int rc = prepare(nD, D, nQ, Q, &p, &u, &k);
    if (rc) return rc;
    double *tree = (double *)malloc(sizeof(double) * (size_t)(k + 1));
    if (!tree) { free(p); free(u); return -3; }
    for (int64_t i = 0; i <= k; i++) tree[i] = e;
    for (int64_t s = 0; s < nD + nQ; s++) {
        int64_t r = below(u, k, p[s].y); /* 0-based y-rank */
        if (p[s].kind == 0) {
            double acc = e;
            for (int64_t i = r; i > 0; i -= i & (-i))   /* ranks 0..r-1 */
                acc = is_max ? (tree[i] > acc ? tree[i] : acc) : acc + tree[i];
            out[p[s].idx] = acc;
        } else {
            double v = w[p[s].idx];
            for (int64_t i = r + 1; i <= k; i += i & (-i))
                tree[i] = is_max ? (v > tree[i] ? v : tree[i]) : tree[i] + v;
        }
    }
    free(tree); free(p); free(u);
    return 0;
}

int pin_fenwick2_i64(int64_t nD, const double *D, int64_t nQ, const double *Q,
                     const int64_t *w, int is_max, int64_t e, int64_t *out) {
    sweep_pt *p; double *u; int64_t k;
    int rc = prepare(nD, D, nQ, Q, &p, &u, &k);
    if (rc) return rc;
    int64_t *tree = (int64_t *)malloc(sizeof(int64_t) * (size_t)(k + 1));
    if (!tree) { free(p); free(u); return -3; }
    for (int64_t i = 0; i <= k; i++) tree[i] = e;
    for (int64_t s = 0; s < nD + nQ; s++) {
        int64_t r = below(u, k, p[s].y);
        if (p[s].kind == 0) {
            int64_t acc = e;
            for (int64_t i = r; i > 0; i -= i & (-i))
                acc = is_max ? (tree[i] > acc ? tree[i] : acc) : acc + tree[i];
            out[p[s].idx] = acc;
        } else {
            int64_t v = w[p[s].idx];
            for (int64_t i = r + 1; i <= k; i += i & (-i))
                tree[i] = is_max ? (v > tree[i] ? v : tree[i]) : tree[i] + v;
        }
    }
    free(tree); free(p); free(u);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The same sweep for several weight columns at once (sums only), sorting
 * with a radix sort instead of qsort, for pins at tens of millions of
 * points.  W and out are column-major: W[c * nD + i], out[c * nQ + j].
 * le_mask bit 0 / bit 1: <= instead of < on the first / second axis (the
 * order of equal first coordinates, and the tree prefix that is asked for).
 * is_int: W and out hold int64 instead of double. */

static uint64_t sortable(double v) {
    if (v == 0.0) v = 0.0; /* -0 and +0 are the same number */
    uint64_t u;
    memcpy(&u, &v, 8);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

/* stable LSD radix sort of (key, idx) by key, 8-bit digits; digits that are
 * the same for every key are skipped.  Returns the sorted arrays (one of the
 * two buffers of each kind). */
static void radix_sort_u64(uint64_t **key, uint32_t **idx, uint64_t **key2, uint32_t **idx2, int64_t n) {
    size_t cnt[256];
    for (int pass = 0; pass < 8; pass++) {
        const int sh = 8 * pass;
        memset(cnt, 0, sizeof cnt);
        for (int64_t i = 0; i < n; i++) cnt[((*key)[i] >> sh) & 255]++;
        int trivial = 0;
        for (int d = 0; d < 256; d++)
            if (cnt[d] == (size_t)n) trivial = 1;
        if (trivial) continue;
        size_t sum = 0;
        for (int d = 0; d < 256; d++) {
            const size_t c = cnt[d];
            cnt[d] = sum;
            sum += c;
        }
        for (int64_t i = 0; i < n; i++) {
            const size_t at = cnt[((*key)[i] >> sh) & 255]++;
            (*key2)[at] = (*key)[i];
            (*idx2)[at] = (*idx)[i];
        }
        uint64_t *tk = *key; *key = *key2; *key2 = tk;
        uint32_t *ti = *idx; *idx = *idx2; *idx2 = ti;
    }
}

int pin_fenwick2_multi(int64_t nD, const double *D, int64_t nQ, const double *Q, int nw, const void *W,
                       int is_int, int le_mask, void *out) {
    const int64_t n = nD + nQ;
    if (nD < 0 || nQ < 0 || nw < 1 || n >= (int64_t)1 << 32) return -1;
    for (int64_t i = 0; i < 2 * nD; i++)
        if (isnan(D[i])) return -2;
    for (int64_t j = 0; j < 2 * nQ; j++)
        if (isnan(Q[j])) return -2;
    const int le_x = le_mask & 1, le_y = (le_mask >> 1) & 1;
    uint64_t *k1 = malloc(sizeof(uint64_t) * (size_t)(n + 1)), *k2 = malloc(sizeof(uint64_t) * (size_t)(n + 1));
    uint32_t *i1 = malloc(sizeof(uint32_t) * (size_t)(n + 1)), *i2 = malloc(sizeof(uint32_t) * (size_t)(n + 1));
    uint32_t *yr = malloc(sizeof(uint32_t) * (size_t)(n + 1));
    if (!k1 || !k2 || !i1 || !i2 || !yr) {
        free(k1); free(k2); free(i1); free(i2); free(yr);
        return -3;
    }
    /* point p < nD is data row p, else query row p - nD */
    /* dense ranks of the second coordinate */
    for (int64_t p = 0; p < n; p++) {
        k1[p] = sortable(p < nD ? D[2 * p + 1] : Q[2 * (p - nD) + 1]);
        i1[p] = (uint32_t)p;
    }
    radix_sort_u64(&k1, &i1, &k2, &i2, n);
    int64_t K = 0;
    for (int64_t s = 0; s < n; s++) {
        if (s == 0 || k1[s] != k1[s - 1]) K++;
        yr[i1[s]] = (uint32_t)(K - 1);
    }
    /* sweep order: first coordinate ascending; on ties, queries first for <
     * (the input order of a stable sort), data first for <= */
    for (int64_t s = 0; s < n; s++) {
        int64_t p;
        if (le_x) p = s;                               /* data rows, then queries */
        else p = s < nQ ? nD + s : s - nQ;             /* queries, then data rows */
        k1[s] = sortable(p < nD ? D[2 * p] : Q[2 * (p - nD)]);
        i1[s] = (uint32_t)p;
    }
    radix_sort_u64(&k1, &i1, &k2, &i2, n);
    const size_t tsz = (size_t)(K + 1) * (size_t)nw;
    double *tf = is_int ? NULL : calloc(tsz, sizeof(double));
    int64_t *ti = is_int ? calloc(tsz, sizeof(int64_t)) : NULL;
    if ((is_int && !ti) || (!is_int && !tf)) {
        free(k1); free(k2); free(i1); free(i2); free(yr);
        return -3;
    }
    const double *Wf = (const double *)W;
    const int64_t *Wi = (const int64_t *)W;
    double *of = (double *)out;
    int64_t *oi = (int64_t *)out;
    for (int64_t s = 0; s < n; s++) {
        const int64_t p = i1[s];
        const int64_t r = yr[p];
        if (p >= nD) {
            const int64_t j = p - nD;
            /* ranks strictly below r (<), or up to r (<=) */
            for (int c = 0; c < nw; c++) {
                if (is_int) {
                    int64_t acc = 0;
                    for (int64_t i = r + le_y; i > 0; i -= i & (-i)) acc += ti[(size_t)i * nw + c];
                    oi[(size_t)c * nQ + j] = acc;
                } else {
                    double acc = 0.0;
                    for (int64_t i = r + le_y; i > 0; i -= i & (-i)) acc += tf[(size_t)i * nw + c];
                    of[(size_t)c * nQ + j] = acc;
                }
            }
        } else {
            for (int64_t i = r + 1; i <= K; i += i & (-i))
                for (int c = 0; c < nw; c++) {
                    if (is_int) ti[(size_t)i * nw + c] += Wi[(size_t)c * nD + p];
                    else tf[(size_t)i * nw + c] += Wf[(size_t)c * nD + p];
                }
        }
    }
    free(tf); free(ti); free(k1); free(k2); free(i1); free(i2); free(yr);
    return 0;
}
