/*
 * CPU oracle for aggregation over dominated points (Sroka & Tyszkiewicz,
 * "Aggregating over Dominated Points by Sorting, Scanning, Zip and Flat Maps").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this code; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no header, helper, table or constant with the
 * GPU path.
 *
 * All arithmetic is fp64 (float weights) or int64 (integer weights).
 * Coordinates are taken as fp64: int32 and fp32 inputs convert exactly.
 *
 * Conventions (the paper's data model, Sec. 2.1): data points carry IDs
 * 0..nD-1 in input order, queries nD..nD+nQ-1.  Queries carry the unit e as
 * their weight.  Dominance is strict in every coordinate (Sec. 1.2).
 *
 * Return codes: 0 ok, -1 bad argument, -2 NaN coordinate, -3 out of memory,
 * -4 output list too short.
 */
#ifndef DOM_AGG_ORACLE_H
#define DOM_AGG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_SUM = 0, ORACLE_MAX = 1, ORACLE_COUNT = 2 };
enum { ORACLE_MAX_DIM = 4 };  /* m <= 4 */

/* Plain definition (Sec. 1.2): out[j] = F over w[i] for all i with
 * D[i] < Q[j] in every coordinate; e when there is none.  O(nD*nQ*m).
 * D is [nD, m] row-major, Q is [nQ, m].  For COUNT, w is ignored and the
 * result counts the dominated points (int64 path only). */
int oracle_brute_f64(int m, int64_t nD, const double *D, int64_t nQ,
                     const double *Q, const double *w, int op, double e,
                     double *out);
int oracle_brute_i64(int m, int64_t nD, const double *D, int64_t nQ,
                     const double *Q, const int64_t *w, int op, int64_t e,
                     int64_t *out);

/* The paper's construction, improved variant of Sec. 5 (the hot path), with
 * the steps of Sec. 4 in their order: union of D and Q; per-axis dense ranks
 * of axes 1..m-1; fixed-width binary ranks; flat map over the prefix sets of
 * Lemma 2 with the last axis kept real; sort in doubly lexicographic order
 * with queries before data on full ties (Sec. 5); segmented scan of the
 * weights tagged by the bitstring tuple; sort by ID and segmented scan by ID.
 * E_out (may be NULL) receives the number of expanded records; L_out (may be
 * NULL, else [m-1]) the bit width of each expanded axis. */
int oracle_dom_agg_f64(int m, int64_t nD, const double *D, int64_t nQ,
                       const double *Q, const double *w, int op, double e,
                       double *out, int64_t *E_out, int *L_out);
int oracle_dom_agg_i64(int m, int64_t nD, const double *D, int64_t nQ,
                       const double *Q, const int64_t *w, int op, int64_t e,
                       int64_t *out, int64_t *E_out, int *L_out);

/* Basic variant of Sec. 4: every axis expanded (n log^m n records), data
 * before queries on ties of the whole tuple.  Used to cross-check. */
int oracle_dom_agg_basic_f64(int m, int64_t nD, const double *D, int64_t nQ,
                             const double *Q, const double *w, int op,
                             double e, double *out, int64_t *E_out);
int oracle_dom_agg_basic_i64(int m, int64_t nD, const double *D, int64_t nQ,
                             const double *Q, const int64_t *w, int op,
                             int64_t e, int64_t *out, int64_t *E_out);

/* Transposed sum (the adjoint of the forward sum with respect to w):
 * grad[i] = sum of g[j] over all j with D[i] < Q[j].  Computed as the
 * Sec. 5 construction on D' = -Q (weights g) and Q' = -D, since
 * d < q  <=>  -q < -d coordinate-wise. */
int oracle_transposed_sum_f64(int m, int64_t nD, const double *D, int64_t nQ,
                              const double *Q, const double *g, double *grad);

/* Non-strict dominance and the final list of Sec. 4.
 *
 * le_mask: bit a asks for D[i][a] <= Q[j][a] instead of < on axis a
 * (0 = strict dominance everywhere, as above).
 *
 * oracle_dom_agg_ex_*: the construction (sec5 = 1: Sec. 5, sec5 = 0: basic
 * Sec. 4) with le_mask; when agg_ids is not NULL it also writes the list the
 * last instructions of Sec. 4 build (6m+6 .. 6m+9: sort by ID, shift,
 * neutral_if_eq, segmented scan by ID): E entries in nondecreasing ID order
 * (data IDs 0..nD-1, then queries nD..nD+nQ-1), each ID repeated once per
 * record of its point, each entry the total of its ID.  shortcut = 1 builds
 * the same list with the segmented broadcast of the maximum that Sec. 4
 * offers when F(a, b) >= a.  agg_cap < E returns -4. */
int oracle_brute_le_f64(int m, int64_t nD, const double *D, int64_t nQ,
                        const double *Q, const double *w, int op, double e,
                        int le_mask, double *out);
int oracle_brute_le_i64(int m, int64_t nD, const double *D, int64_t nQ,
                        const double *Q, const int64_t *w, int op, int64_t e,
                        int le_mask, int64_t *out);
int oracle_dom_agg_ex_f64(int m, int64_t nD, const double *D, int64_t nQ,
                          const double *Q, const double *w, int op, double e,
                          int sec5, int le_mask, double *out, int64_t *E_out,
                          int *L_out, int64_t *agg_ids, double *agg_vals,
                          int64_t agg_cap, int shortcut);
int oracle_dom_agg_ex_i64(int m, int64_t nD, const double *D, int64_t nQ,
                          const double *Q, const int64_t *w, int op, int64_t e,
                          int sec5, int le_mask, int64_t *out, int64_t *E_out,
                          int *L_out, int64_t *agg_ids, int64_t *agg_vals,
                          int64_t agg_cap, int shortcut);
int oracle_transposed_sum_le_f64(int m, int64_t nD, const double *D,
                                 int64_t nQ, const double *Q, const double *g,
                                 int le_mask, double *grad);

/* Primitives, exposed so they can be checked against the paper's examples. */

/* Segmented scan (Def. of sscan, Sec. 2.2): out[k] = F of a[i] over i <= k
 * with t[i] == t[k] inside the maximal run of equal tags containing k. */
int oracle_sscan_f64(int64_t n, const double *a, const int64_t *t, int op,
                     double *out);

/* P0 (bit=0) or P1 (bit=1) of an L-bit string x (Sec. 3): every prefix v
 * such that v followed by `bit` is a prefix of x.  Writes the prefixes as
 * (length, value) pairs, shortest first; returns how many. */
int oracle_prefix_set(uint64_t x, int L, int bit, int *lens, uint64_t *vals);

/* Dense 0-based ranks of v[0..n-1] (ties share a rank) and the number K of
 * distinct values (Sec. 4, rank steps: the 1-based rank minus one). */
int oracle_dense_rank(int64_t n, const double *v, int64_t *rank, int64_t *K);

/* Number of binary digits used for ranks 0..K-1: ceil(log2 K), 0 for K <= 1. */
int oracle_bits_for(int64_t K);

#ifdef __cplusplus
}
#endif
#endif
