/*
 * CPU oracle -- sparse LDL^T factorisation with the "infinite pivot" rule.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle/__init__.py); shares no code with the
 * HIP library.
 *
 * Section 4.2: once the method switches to a direct solver, the Schur
 * complement (symmetric, singular, weakly diagonally dominant) is factorised
 * exactly as L D L^T after a fill-reducing ordering.  One pivot is expected to
 * vanish; the paper notes that a modified factorisation replacing small pivots
 * by an infinitely large value handles it.  Here a pivot d_k <= pivtol * a_kk
 * (a_kk the original diagonal entry) is set to +inf: the multipliers in its
 * column become 0 and the solve returns 0 for that unknown, which grounds one
 * node of every (numerically) disconnected component.
 *
 * Algorithm: the up-looking row-by-row factorisation (elimination tree,
 * nonzero pattern of row k of L from the tree reach of column k of A), as
 * described in T. Davis, "Direct Methods for Sparse Linear Systems", SIAM 2006,
 * chapter 4.  Input: the UPPER triangle of the (already permuted) matrix in
 * compressed-column form (rows i <= k in column k).  0-based int32 indices.
 */
#include <math.h>
#include <stdint.h>

/* elimination tree and column counts of L */
void orc_ldl_symbolic(int32_t n, const int32_t *Ap, const int32_t *Ai,
                      int32_t *Lp, int32_t *Parent, int32_t *Lnz, int32_t *Flag)
{
    for (int32_t k = 0; k < n; ++k) {
        Parent[k] = -1;
        Flag[k] = k;
        Lnz[k] = 0;
        for (int32_t p = Ap[k]; p < Ap[k + 1]; ++p) {
            int32_t i = Ai[p];
            if (i >= k) continue;
            for (; Flag[i] != k; i = Parent[i]) {
                if (Parent[i] == -1) Parent[i] = k;
                Lnz[i]++;
                Flag[i] = k;
            }
        }
    }
    Lp[0] = 0;
    for (int32_t k = 0; k < n; ++k) Lp[k + 1] = Lp[k] + Lnz[k];
}

/* numeric factorisation; returns the number of infinite pivots */
int32_t orc_ldl_numeric(int32_t n, const int32_t *Ap, const int32_t *Ai, const double *Ax,
                        const int32_t *Lp, const int32_t *Parent, int32_t *Lnz,
                        int32_t *Li, double *Lx, double *D, double *Y,
                        int32_t *Pattern, int32_t *Flag, double pivtol)
{
    int32_t ninf = 0;
    for (int32_t k = 0; k < n; ++k) {
        double akk = 0.0;
        Y[k] = 0.0;
        int32_t top = n;
        Flag[k] = k;
        Lnz[k] = 0;
        for (int32_t p = Ap[k]; p < Ap[k + 1]; ++p) {
            int32_t i = Ai[p];
            if (i > k) continue;
            Y[i] += Ax[p];
            if (i == k) akk += Ax[p];
            int32_t len = 0;
            for (; Flag[i] != k; i = Parent[i]) {
                Pattern[len++] = i;
                Flag[i] = k;
            }
            while (len > 0) Pattern[--top] = Pattern[--len];
        }
        D[k] = Y[k];
        Y[k] = 0.0;
        for (; top < n; ++top) {
            int32_t i = Pattern[top];
            double yi = Y[i];
            Y[i] = 0.0;
            int32_t p2 = Lp[i] + Lnz[i];
            for (int32_t p = Lp[i]; p < p2; ++p) Y[Li[p]] -= Lx[p] * yi;
            double lki = isinf(D[i]) ? 0.0 : yi / D[i];
            D[k] -= lki * yi;
            Li[p2] = k;
            Lx[p2] = lki;
            Lnz[i]++;
        }
        if (!(D[k] > pivtol * akk) || !(D[k] > 0.0)) {
            D[k] = INFINITY;
            ++ninf;
        }
    }
    return ninf;
}

/* solve L D L^T x = b in place */
void orc_ldl_solve(int32_t n, double *x, const int32_t *Lp, const int32_t *Li,
                   const double *Lx, const double *D)
{
    for (int32_t j = 0; j < n; ++j)
        for (int32_t p = Lp[j]; p < Lp[j + 1]; ++p) x[Li[p]] -= Lx[p] * x[j];
    for (int32_t j = 0; j < n; ++j) x[j] = isinf(D[j]) ? 0.0 : x[j] / D[j];
    for (int32_t j = n - 1; j >= 0; --j)
        for (int32_t p = Lp[j]; p < Lp[j + 1]; ++p) x[j] -= Lx[p] * x[Li[p]];
}
