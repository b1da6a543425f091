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
