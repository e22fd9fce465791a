/*
 * CPU oracle -- L D L^T of a sparse symmetric matrix with the infinite-pivot
 * rule.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle/__init__.py); shares no code with the
 * HIP library.
 *
 * Section 4.2: after the switch the Schur complement (symmetric, singular by
 * one per connected component of the support, weakly diagonally dominant) is
 * factorised exactly as L D L^T, after a fill-reducing ordering chosen by the
 * caller.  The paper's remark on the vanishing pivot allows replacing it by an
 * infinitely large value.  Reading used here: a pivot d_k that is not above
 * pivtol * a_kk (a_kk the diagonal entry of the input) or not positive becomes
 * +inf.  Its column of L is then zero (the multipliers divide by +inf), it
 * contributes nothing to later columns, and the solve returns 0 for that
 * unknown.
 *
 * The factor is computed column by column straight from its definition,
 *     d_k  = a_kk - sum_{j<k} l_kj^2 d_j,
 *     l_ik = (a_ik - sum_{j<k} l_ij l_kj d_j) / d_k,   i > k,
 * i.e. column k of the lower triangle of A is gathered into a dense work
 * vector w, every earlier column j whose entry l_kj is structurally nonzero
 * subtracts (l_kj d_j) L(k:n, j) from it, then d_k = w_k and L(k+1:n, k) =
 * w(k+1:n) / d_k.  The earlier columns that reach row k are kept in one list
 * per row: a finished column waits in the list of the row of its first entry,
 * and after it has been used for row r it moves to the list of its next row.
 * The structure of a column is the union of the structures that reach it, so
 * the entries counted are those of the symbolic factorisation (an infinite
 * pivot's column keeps its structure, with zero values).
 *
 * Input: the LOWER triangle (rows i >= k) of the already permuted matrix in
 * compressed-column form, 0-based int32 indices; entries above the diagonal
 * are ignored.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t n, ninf;
    int64_t nnz, cap;
    int64_t *colp;  /* n + 1: start of each column of L (strictly lower part) */
    int32_t *row;   /* row index of each stored entry, increasing in a column */
    double *val;    /* its value l_ik */
    double *d;      /* n pivots (+inf for an infinite pivot) */
} orc_ldl;

static int cmp_i32(const void *a, const void *b)
{
    const int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

void orc_ldl_free(orc_ldl *F)
{
    if (!F) return;
    free(F->colp);
    free(F->row);
    free(F->val);
    free(F->d);
    free(F);
}

static int grow(orc_ldl *F, int64_t need)
{
    if (need <= F->cap) return 1;
    int64_t c = F->cap ? F->cap : 1024;
    while (c < need) c *= 2;
    int32_t *r = (int32_t *)realloc(F->row, sizeof(int32_t) * (size_t)c);
    if (!r) return 0;
    F->row = r;
    double *v = (double *)realloc(F->val, sizeof(double) * (size_t)c);
    if (!v) return 0;
    F->val = v;
    F->cap = c;
    return 1;
}

/* factorise; returns NULL when memory runs out */
orc_ldl *orc_ldl_factor(int32_t n, const int32_t *Ap, const int32_t *Ai, const double *Ax,
                        double pivtol)
{
    orc_ldl *F = (orc_ldl *)calloc(1, sizeof(orc_ldl));
    double *w = (double *)calloc((size_t)n + 1, sizeof(double));
    int32_t *seen = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *pat = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *head = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *link = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int64_t *next_pos = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (F) {
        F->n = n;
        F->colp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
        F->d = (double *)calloc((size_t)n + 1, sizeof(double));
    }
    if (!F || !w || !seen || !pat || !head || !link || !next_pos || !F->colp || !F->d) {
        orc_ldl_free(F);
        F = NULL;
        goto done;
    }
    for (int32_t i = 0; i < n; ++i) {
        seen[i] = -1;
        head[i] = -1;
    }
    for (int32_t k = 0; k < n; ++k) {
        int32_t np = 0;
        double akk = 0.0;
        /* column k of A, rows >= k */
        seen[k] = k;
        w[k] = 0.0;
        for (int32_t q = Ap[k]; q < Ap[k + 1]; ++q) {
            const int32_t i = Ai[q];
            if (i < k) continue;
            if (seen[i] != k) {
                seen[i] = k;
                w[i] = 0.0;
                pat[np++] = i;
            }
            w[i] += Ax[q];
            if (i == k) akk += Ax[q];
        }
        /* the earlier columns with an entry in row k */
        int32_t j = head[k];
        head[k] = -1;
        while (j >= 0) {
            const int32_t after = link[j];
            const int64_t p0 = next_pos[j]; /* F->row[p0] == k */
            const int finite = isfinite(F->d[j]);
            const double c = finite ? F->val[p0] * F->d[j] : 0.0;
            for (int64_t q = p0; q < F->colp[j + 1]; ++q) {
                const int32_t i = F->row[q];
                if (seen[i] != k) {
                    seen[i] = k;
                    w[i] = 0.0;
                    pat[np++] = i;
                }
                if (finite) w[i] -= F->val[q] * c;
            }
            if (p0 + 1 < F->colp[j + 1]) {
                const int32_t r = F->row[p0 + 1];
                next_pos[j] = p0 + 1;
                link[j] = head[r];
                head[r] = j;
            }
            j = after;
        }
        /* pivot and column k of L */
        double dk = w[k];
        if (!(dk > pivtol * akk) || !(dk > 0.0)) {
            dk = INFINITY;
            F->ninf++;
        }
        F->d[k] = dk;
        /* pat holds the rows > k reached (k itself was marked before) */
        int32_t m = 0;
        for (int32_t t = 0; t < np; ++t)
            if (pat[t] > k) pat[m++] = pat[t];
        qsort(pat, (size_t)m, sizeof(int32_t), cmp_i32);
        if (!grow(F, F->nnz + m)) {
            orc_ldl_free(F);
            F = NULL;
            goto done;
        }
        F->colp[k] = F->nnz;
        for (int32_t t = 0; t < m; ++t) {
            F->row[F->nnz] = pat[t];
            F->val[F->nnz] = isinf(dk) ? 0.0 : w[pat[t]] / dk;
            F->nnz++;
        }
        F->colp[k + 1] = F->nnz;
        if (m > 0) {
            const int32_t r = pat[0];
            next_pos[k] = F->colp[k];
            link[k] = head[r];
            head[r] = k;
        }
    }
done:
    free(w);
    free(seen);
    free(pat);
    free(head);
    free(link);
    free(next_pos);
    return F;
}

int64_t orc_ldl_nnz(const orc_ldl *F) { return F->nnz; }
int32_t orc_ldl_ninf(const orc_ldl *F) { return F->ninf; }

/* x <- (L D L^T)^{-1} x: forward with L, scale by D (an infinite pivot gives
 * 0), backward with L^T */
void orc_ldl_solve(const orc_ldl *F, double *x)
{
    const int32_t n = F->n;
    for (int32_t j = 0; j < n; ++j) {
        const double xj = x[j];
        for (int64_t q = F->colp[j]; q < F->colp[j + 1]; ++q) x[F->row[q]] -= F->val[q] * xj;
    }
    for (int32_t j = 0; j < n; ++j) x[j] = isinf(F->d[j]) ? 0.0 : x[j] / F->d[j];
    for (int32_t j = n - 1; j >= 0; --j) {
        double s = x[j];
        for (int64_t q = F->colp[j]; q < F->colp[j + 1]; ++q) s -= F->val[q] * x[F->row[q]];
        x[j] = s;
    }
}

/* copy the factor out: colp (n + 1), row and val (nnz), d (n) */
void orc_ldl_export(const orc_ldl *F, int64_t *colp, int32_t *row, double *val, double *d)
{
    memcpy(colp, F->colp, sizeof(int64_t) * ((size_t)F->n + 1));
    if (F->nnz) {
        memcpy(row, F->row, sizeof(int32_t) * (size_t)F->nnz);
        memcpy(val, F->val, sizeof(double) * (size_t)F->nnz);
    }
    memcpy(d, F->d, sizeof(double) * (size_t)F->n);
}
