/*
 * Textbook offline divide and conquer for three-dimensional dominance
 * aggregation, used ONLY to pin the GPU path at sizes where the double loop
 * of the definition is too slow.  TEST INFRASTRUCTURE ONLY.  It shares no
 * code with the construction in dom_agg_oracle.c: it is the classical
 * sequential method (sort by the first axis; recursively split the sorted
 * list in halves; every pair of a data point in the left half and a query in
 * the right half is settled when the halves are merged in order of the
 * second axis, with a Fenwick tree over ranks of the third axis), not the
 * paper's construction.
 *
 * out[j] = F over w[i] with D[i] before Q[j] on every axis, e if none, where
 * "before" on axis a is < (strict dominance), or <= when bit a of le_mask is
 * set.  On the first two axes the comparison is made exact by the order of
 * equal coordinates (queries before data for <, data before queries for <=);
 * on the third, by the prefix of ranks the tree is asked for.  SUM and MAX
 * (prefix maximum, undone after each merge) are supported; COUNT is SUM with
 * unit weights supplied by the caller.  Arithmetic: fp64 or int64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double x, y;
    int64_t zr;   /* 0-based dense rank of the third coordinate */
    int64_t idx;  /* index into D (data) or Q (query) */
    int kind;     /* ordering key of the kind on axes 1 and 2 (see below) */
    int isq;
} cdq_pt;

typedef union {
    double f;
    int64_t i;
} cval;

typedef struct {
    int is_float, is_max;
    cval e;
    const cval *w;
    cval *out;
    cval *tree;
    int64_t k;       /* distinct third coordinates */
    int le_x, le_y, le_z;
    cdq_pt *tmp;
} cdq_ctx;

/* kind = 0 sorts first on equal coordinates: queries for <, data for <= */
static int x_cmp(const void *pa, const void *pb) {
    const cdq_pt *a = (const cdq_pt *)pa, *b = (const cdq_pt *)pb;
    if (a->x < b->x) return -1;
    if (b->x < a->x) return 1;
    if (a->kind != b->kind) return a->kind - b->kind;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

static cval cv_comb(const cdq_ctx *c, cval a, cval b) {
    cval r;
    if (c->is_float) r.f = c->is_max ? (b.f > a.f ? b.f : a.f) : a.f + b.f;
    else r.i = c->is_max ? (b.i > a.i ? b.i : a.i) : a.i + b.i;
    return r;
}

static void bit_add(cdq_ctx *c, int64_t r, cval v) {
    for (int64_t i = r + 1; i <= c->k; i += i & (-i)) c->tree[i] = cv_comb(c, c->tree[i], v);
}

static void bit_reset(cdq_ctx *c, int64_t r) {
    for (int64_t i = r + 1; i <= c->k; i += i & (-i)) c->tree[i] = c->e;
}

/* F over tree positions of ranks 0 .. cnt-1 */
static cval bit_prefix(const cdq_ctx *c, int64_t cnt) {
    cval acc = c->e;
    for (int64_t i = cnt; i > 0; i -= i & (-i)) acc = cv_comb(c, acc, c->tree[i]);
    return acc;
}

/* y-order of a merge: y ascending, then the kind order of the second axis */
static int y_before(const cdq_ctx *c, const cdq_pt *a, const cdq_pt *b) {
    if (a->y < b->y) return 1;
    if (b->y < a->y) return 0;
    const int ka = c->le_y ? a->isq : !a->isq, kb = c->le_y ? b->isq : !b->isq;
    return ka <= kb;
}

/* p[lo, hi) is in first-axis order on entry and in second-axis order on exit */
static void solve(cdq_ctx *c, cdq_pt *p, int64_t lo, int64_t hi) {
    if (hi - lo <= 1) return;
    const int64_t mid = lo + (hi - lo) / 2;
    solve(c, p, lo, mid);
    solve(c, p, mid, hi);
    /* merge by the second axis; left data enter the tree, right queries ask */
    int64_t i = lo, j = mid, o = 0;
    while (i < mid || j < hi) {
        const int take_left = j >= hi || (i < mid && y_before(c, &p[i], &p[j]));
        cdq_pt *s = take_left ? &p[i++] : &p[j++];
        if (take_left && !s->isq) bit_add(c, s->zr, c->w[s->idx]);
        if (!take_left && s->isq)
            c->out[s->idx] = cv_comb(c, c->out[s->idx], bit_prefix(c, s->zr + (c->le_z ? 1 : 0)));
        c->tmp[o++] = *s;
    }
    for (int64_t t = lo; t < mid; t++)
        if (!p[t].isq) bit_reset(c, p[t].zr);
    memcpy(p + lo, c->tmp, sizeof(cdq_pt) * (size_t)(hi - lo));
}

static int dbl_cmp(const void *pa, const void *pb) {
    const double a = *(const double *)pa, b = *(const double *)pb;
    return (a > b) - (a < b);
}

static int64_t rank_of(const double *u, int64_t k, double v) {
    int64_t lo = 0, hi = k;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (u[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

static int run(int64_t nD, const double *D, int64_t nQ, const double *Q, const cval *w, int is_float,
               int is_max, cval e, int le_mask, cval *out) {
    const int64_t n = nD + nQ;
    if (nD < 0 || nQ < 0 || (nD && (!D || !w)) || (nQ && (!Q || !out))) return -1;
    for (int64_t i = 0; i < 3 * nD; i++)
        if (isnan(D[i])) return -2;
    for (int64_t i = 0; i < 3 * nQ; i++)
        if (isnan(Q[i])) return -2;
    cdq_ctx c;
    memset(&c, 0, sizeof c);
    c.is_float = is_float;
    c.is_max = is_max;
    c.e = e;
    c.w = w;
    c.out = out;
    c.le_x = le_mask & 1;
    c.le_y = (le_mask >> 1) & 1;
    c.le_z = (le_mask >> 2) & 1;
    cdq_pt *p = (cdq_pt *)malloc(sizeof(cdq_pt) * (size_t)(n + 1));
    double *u = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    c.tmp = (cdq_pt *)malloc(sizeof(cdq_pt) * (size_t)(n + 1));
    if (!p || !u || !c.tmp) {
        free(p); free(u); free(c.tmp);
        return -3;
    }
    for (int64_t i = 0; i < n; i++) {
        const double *x = i < nD ? D + 3 * i : Q + 3 * (i - nD);
        u[i] = x[2] == 0.0 ? 0.0 : x[2];
    }
    qsort(u, (size_t)n, sizeof(double), dbl_cmp);
    int64_t k = 0;
    for (int64_t i = 0; i < n; i++)
        if (k == 0 || u[k - 1] < u[i]) u[k++] = u[i];
    c.k = k;
    for (int64_t i = 0; i < n; i++) {
        const int isq = i >= nD;
        const double *x = isq ? Q + 3 * (i - nD) : D + 3 * i;
        p[i].x = x[0];
        p[i].y = x[1];
        p[i].zr = rank_of(u, k, x[2] == 0.0 ? 0.0 : x[2]);
        p[i].idx = isq ? i - nD : i;
        p[i].isq = isq;
        p[i].kind = c.le_x ? isq : !isq;
    }
    c.tree = (cval *)malloc(sizeof(cval) * (size_t)(k + 1));
    if (!c.tree) {
        free(p); free(u); free(c.tmp);
        return -3;
    }
    for (int64_t i = 0; i <= k; i++) c.tree[i] = e;
    for (int64_t j = 0; j < nQ; j++) out[j] = e;
    qsort(p, (size_t)n, sizeof(cdq_pt), x_cmp);
    solve(&c, p, 0, n);
    free(c.tree); free(p); free(u); free(c.tmp);
    return 0;
}

int pin_cdq3_f64(int64_t nD, const double *D, int64_t nQ, const double *Q, const double *w, int is_max,
                 double e, int le_mask, double *out) {
    cval ev;
    ev.f = e;
    return run(nD, D, nQ, Q, (const cval *)w, 1, is_max, ev, le_mask, (cval *)out);
}

int pin_cdq3_i64(int64_t nD, const double *D, int64_t nQ, const double *Q, const int64_t *w, int is_max,
                 int64_t e, int le_mask, int64_t *out) {
    cval ev;
    ev.i = e;
    return run(nD, D, nQ, Q, (const cval *)w, 0, is_max, ev, le_mask, (cval *)out);
}
