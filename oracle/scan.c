/*
 * CPU oracle -- plain C scans over all m*n transport variables.
 *
 * TEST INFRASTRUCTURE ONLY.  This file belongs to the reference oracle that the
 * tests, the smoke check and the benchmark's CPU baseline compare the HIP
 * library against.  It shares no code with the library and the library never
 * calls it.
 *
 * Everything here is a direct, unblocked loop over the variables in the
 * paper's vec order (variable index idx = i + j*m, i the source, j the target;
 * Section 2.1 and the index map of Section 3.4, read 0-based).  Costs are
 * norms of the integer offset (d0, d1) between pixel coordinates (Section 5.1
 * uses the 1-, 2- and inf-norm; the squared 2-norm is this project's default
 * workload), by `kind`:
 *   0  d0^2 + d1^2            (exact in 64-bit integers, then double)
 *   1  |d0| + |d1|            (exact)
 *   2  sqrt(d0^2 + d1^2)      (IEEE square root, correctly rounded, of the
 *                              exact integer)
 *   3  max(|d0|, |d1|)        (exact)
 *
 * The reduced cost of variable (i, j) is evaluated as ((double)c_ij - y_i) - z_j,
 * i.e. c - A^T y with the two dual blocks subtracted in that order
 * (Section 3.4).  Build with -O2 -ffp-contract=off and no fast-math so that
 * this is exactly two IEEE-754 double subtractions.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline int64_t iabs64(int64_t v) { return v < 0 ? -v : v; }

/* The integer that orders the costs of a kind: the cost itself for kinds 0,
 * 1 and 3, the squared norm for kind 2 (the square root is increasing).  The
 * initial support's thresholds and cheapest entries are taken on it. */
static inline int64_t cost_key(const int32_t *xs, const int32_t *xt, int64_t i, int64_t j,
                               int kind)
{
    int64_t d0 = (int64_t)xs[2 * i] - (int64_t)xt[2 * j];
    int64_t d1 = (int64_t)xs[2 * i + 1] - (int64_t)xt[2 * j + 1];
    if (kind == 1) return iabs64(d0) + iabs64(d1);
    if (kind == 3) return iabs64(d0) > iabs64(d1) ? iabs64(d0) : iabs64(d1);
    return d0 * d0 + d1 * d1;
}

/* The cost C_ij as a double. */
static inline double cost_d(const int32_t *xs, const int32_t *xt, int64_t i, int64_t j, int kind)
{
    int64_t q = cost_key(xs, xt, i, j, kind);
    return kind == 2 ? sqrt((double)q) : (double)q;
}

/* ---- bounded max-heap keyed by (r, idx), keeps the kmax smallest keys ---- */
typedef struct { double r; int64_t idx; } key_t_;

static inline int key_less(key_t_ a, key_t_ b)
{
    return (a.r < b.r) || (a.r == b.r && a.idx < b.idx);
}

static void heap_sift_down(key_t_ *h, int64_t n, int64_t k)
{
    for (;;) {
        int64_t l = 2 * k + 1, r = l + 1, big = k;
        if (l < n && key_less(h[big], h[l])) big = l;
        if (r < n && key_less(h[big], h[r])) big = r;
        if (big == k) return;
        key_t_ t = h[k]; h[k] = h[big]; h[big] = t;
        k = big;
    }
}

static void heap_sift_up(key_t_ *h, int64_t k)
{
    while (k > 0) {
        int64_t p = (k - 1) / 2;
        if (!key_less(h[p], h[k])) return;
        key_t_ t = h[k]; h[k] = h[p]; h[p] = t;
        k = p;
    }
}

static int cmp_key(const void *a, const void *b)
{
    key_t_ x = *(const key_t_ *)a, y = *(const key_t_ *)b;
    if (key_less(x, y)) return -1;
    if (key_less(y, x)) return 1;
    return 0;
}

/*
 * Pricing (Section 3.2, update phase; Section 3.4): among all variables not in
 * the support whose reduced cost is strictly negative, return the kmax with
 * the most negative reduced cost, ordered by (r, idx) ascending.
 *
 * sup     : the support, variable indices sorted ascending (psi entries).
 * out_idx, out_r : at least kmax entries.
 * n_neg   : number of strictly negative reduced costs outside the support.
 * key_limit : > 0 restricts the scan to the heuristic subset of Section 3.4,
 *           J = {(i, j) : cost key < key_limit} (the cost itself, the squared
 *           norm for the 2-norm); <= 0 scans every variable.
 * returns the number of entries written (<= kmax), or -1 on allocation error.
 */
int64_t orc_price(int64_t m, int64_t n, const int32_t *xs, const int32_t *xt,
                  const double *y, const double *z, const int64_t *sup, int64_t psi,
                  int64_t kmax, int64_t *out_idx, double *out_r, int64_t *n_neg, int kind,
                  int64_t key_limit)
{
    key_t_ *h = NULL;
    int64_t hn = 0, neg = 0, sp = 0;
    if (kmax > 0) {
        h = (key_t_ *)malloc(sizeof(key_t_) * (size_t)kmax);
        if (!h) return -1;
    }
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) {
            int64_t idx = i + j * m;
            while (sp < psi && sup[sp] < idx) ++sp;
            if (sp < psi && sup[sp] == idx) continue;
            if (key_limit > 0 && cost_key(xs, xt, i, j, kind) >= key_limit) continue;
            double c = cost_d(xs, xt, i, j, kind);
            double r = (c - y[i]) - z[j];
            if (!(r < 0.0)) continue;
            ++neg;
            if (kmax <= 0) continue;
            key_t_ k = { r, idx };
            if (hn < kmax) {
                h[hn] = k;
                heap_sift_up(h, hn);
                ++hn;
            } else if (key_less(k, h[0])) {
                h[0] = k;
                heap_sift_down(h, hn, 0);
            }
        }
    }
    if (hn > 1) qsort(h, (size_t)hn, sizeof(key_t_), cmp_key);
    for (int64_t t = 0; t < hn; ++t) { out_idx[t] = h[t].idx; out_r[t] = h[t].r; }
    if (n_neg) *n_neg = neg;
    free(h);
    return hn;
}

/*
 * Smallest reduced cost over ALL m*n variables (support included), with the
 * first index attaining it.  Used for the a-posteriori dual certificate
 * s_hat = c - A^T y_hat (Section 3.3).
 */
double orc_rmin(int64_t m, int64_t n, const int32_t *xs, const int32_t *xt,
                const double *y, const double *z, int64_t *argmin, int kind)
{
    double best = 0.0;
    int64_t arg = -1;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) {
            double r = (cost_d(xs, xt, i, j, kind) - y[i]) - z[j];
            if (arg < 0 || r < best) { best = r; arg = i + j * m; }
        }
    if (argmin) *argmin = arg;
    return best;
}

/* Histogram of the integer cost keys <= cmax over all variables. */
void orc_cost_hist(int64_t m, int64_t n, const int32_t *xs, const int32_t *xt,
                   int64_t cmax, int64_t *hist, int kind)
{
    memset(hist, 0, sizeof(int64_t) * (size_t)(cmax + 1));
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) {
            int64_t c = cost_key(xs, xt, i, j, kind);
            if (c <= cmax) hist[c]++;
        }
}

/* All variable indices with cost key <= T, ascending; returns the count (capped). */
int64_t orc_collect_le(int64_t m, int64_t n, const int32_t *xs, const int32_t *xt,
                       int64_t T, int64_t *out_idx, int64_t cap, int kind)
{
    int64_t k = 0;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i)
            if (cost_key(xs, xt, i, j, kind) <= T) {
                if (k < cap) out_idx[k] = i + j * m;
                ++k;
            }
    return k;
}

/* For every source i the target of least cost (ties: smallest j), and for
 * every target j the source of least cost (ties: smallest i). */
void orc_row_col_argmin(int64_t m, int64_t n, const int32_t *xs, const int32_t *xt,
                        int64_t *row_arg, int64_t *col_arg, int kind)
{
    for (int64_t i = 0; i < m; ++i) {
        int64_t best = -1, arg = -1;
        for (int64_t j = 0; j < n; ++j) {
            int64_t c = cost_key(xs, xt, i, j, kind);
            if (arg < 0 || c < best) { best = c; arg = j; }
        }
        row_arg[i] = arg;
    }
    for (int64_t j = 0; j < n; ++j) {
        int64_t best = -1, arg = -1;
        for (int64_t i = 0; i < m; ++i) {
            int64_t c = cost_key(xs, xt, i, j, kind);
            if (arg < 0 || c < best) { best = c; arg = i; }
        }
        col_arg[j] = arg;
    }
}
