/*
 * otip -- interior-point-inspired column generation for the Kantorovich
 * optimal-transport LP on AMD Instinct MI355X (gfx950).
 *
 * Method: Zanetti & Gondzio, "An Interior-Point-Inspired algorithm for Linear
 * Programs arising in Discrete Optimal Transport" (arXiv 2206.11009).
 *
 * Problem (Section 2, eqs. feasible_region, OT_problem, kantorovichlp): given
 * masses a in R^m_+, b in R^n_+ with sum(a) = sum(b) and a cost C, find the
 * plan P in R^{m x n}_+ with row sums a and column sums b minimising
 * sum_ij C_ij P_ij.  Here C_ij is the integer squared Euclidean distance between
 * integer points xs[i] and xt[j] (the paper's pixel-offset costs of Section 5.1,
 * in the squared 2-norm), generated on the fly and never stored.
 *
 * Variable order is the paper's vec order: variable idx = i + j*m (0-based),
 * i the source (row of P), j the target (column of P).
 *
 * Conventions of every call below
 *   - "device" pointers live on the context's device (any allocator, e.g.
 *     torch); "host" pointers are ordinary CPU memory.
 *   - The caller owns every buffer it passes; nothing is retained after the
 *     call returns.  The library owns contexts and result objects.
 *   - All device work is enqueued on the context's stream; a call that returns
 *     host values synchronises that stream before returning.
 *   - Calls return OTIP_OK or an error code; otip_last_error() gives the
 *     message.  No exception crosses this boundary.
 *   - A context is not thread-safe; use one context per host thread.
 */
#ifndef OTIP_H
#define OTIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OTIP_ABI_VERSION 4

enum otip_status {
    OTIP_OK = 0,
    OTIP_EINVAL = 1,      /* bad argument: sizes, null pointers, masses (negative, non-finite,
                             unbalanced, all zero), coordinates out of range */
    OTIP_ENOMEM = 2,      /* device allocation failed */
    OTIP_EHIP = 3,        /* HIP runtime error */
    OTIP_EMAXITER = 4,    /* iteration limit: result valid but not certified to tol */
    OTIP_ENUMERIC = 5,    /* NaN or breakdown */
    OTIP_EUNSUPPORTED = 6 /* request outside what this build supports */
};

enum otip_linear_solver { OTIP_LS_AUTO = 0, OTIP_LS_PCG = 1, OTIP_LS_DIRECT = 2 };
enum otip_precision { OTIP_FP64 = 0, OTIP_MIXED = 1 };

/* Cost C_ij between integer pixel coordinates, from the offset d = x_i - x'_j
 * (Section 5.1 compares the 1-, 2- and inf-norms; the squared 2-norm is the
 * default).  Every cost is evaluated exactly, except the 2-norm, which is the
 * correctly rounded square root of the exact integer d0^2 + d1^2. */
enum otip_cost {
    OTIP_COST_SQEUCLID = 0, /* d0^2 + d1^2 */
    OTIP_COST_L1 = 1,       /* |d0| + |d1| */
    OTIP_COST_L2 = 2,       /* sqrt(d0^2 + d1^2) */
    OTIP_COST_LINF = 3      /* max(|d0|, |d1|) */
};

/*
 * Solver parameters.  Defaults (otip_params_default) are the paper's values
 * where it states them (Section 5.2: tol 1e-6, CG tolerance 1e-6 for
 * predictors and 1e-3 for correctors, 200 iterations, 1000 CG iterations per
 * call, 3 correctors; Section 3.3: step 0.995 of the step to the boundary;
 * Section 4.3: window of 5 iterations for the switch) and otherwise readings of
 * points it leaves open.
 */
typedef struct otip_params {
    double tol;              /* stop test tolerance (Section 3.2) */
    double cg_tol_pred;      /* CG relative tolerance, predictor/Mehrotra solves */
    double cg_tol_corr;      /* CG relative tolerance, centrality correctors */
    int32_t max_iter;        /* outer iterations */
    int32_t cg_max_iter;     /* CG iterations per solve */
    int32_t max_corr;        /* centrality correctors per iteration */
    double step_scale;       /* fraction of the step to the boundary */
    double kappa;            /* initial support ~ kappa*(m+n-1) cheapest variables */
    int32_t switch_window;   /* psi history window for the CG -> direct switch */
    double switch_drop;      /* relative psi drop over the window that switches */
    double mcc_beta_min;     /* centrality target box [beta_min, beta_max]*sigma*mu */
    double mcc_beta_max;
    double mcc_delta;        /* trial step increase for a corrector */
    double mcc_accept;       /* minimum step gain to accept a corrector */
    double remove_gate;      /* remove only when max(rel r1, rel r2) <= gate */
    double remove_rel;       /* remove p_ij < remove_rel*min(a_i, b_j) */
    double pivot_tol;        /* LDL^T pivot d_k <= pivot_tol*S_kk becomes +inf */
    double cert_rel;         /* a-posteriori pricing: significant if sum(a)|r| > cert_rel*max(1,|obj|) */
    double polish_tol;       /* final primal projection target ||Ap-f||_1/||f||_1 */
    int32_t polish_steps;
    double drop_rel;         /* purified flows below drop_rel*min(a_i,b_j) are zero */
    double cg_eta;           /* CG residual must also be <= cg_eta*max(||r1||, cg_floor*(1+||f||)) */
    double cg_floor;
    int32_t linear_solver;   /* otip_linear_solver */
    int32_t precision;       /* otip_precision */
    int32_t dense_max_n;     /* largest Schur order factorised by the dense LDL^T (65536);
                                the factorisation also needs about 26 n^2 bytes of free
                                device memory (112 GB at 65536), else CG continues */
    int32_t force_switch_at; /* >= 0: switch to the direct solver at this iteration */
    int32_t enter_cap;       /* max entering columns per iteration; <= 0 means m */
    int32_t scale;           /* power-of-two scaling of masses and costs (1 = on) */
    int32_t verbose;         /* 1: one line per iteration on stderr */
    int32_t profile;         /* 1: time every SpMV and pricing launch with HIP events */
    int32_t switch_cost;     /* 1: also switch once a dense factorisation is estimated (fixed
                                cost model) to cost less than the last iteration's CG */
    int32_t batch_workers;   /* otip_solve_batch: host workers, each with its own HIP stream
                                and solver state (0: min(8, count)) */
    int32_t price_tile;      /* targets per pricing-scan block, a power of two in [16, 256];
                                0: chosen from m and n */
    double ws_kappa;         /* warm start: initial support ~ ws_kappa*(m+n-1) smallest
                                reduced costs under the given duals (0: use kappa) */
    double heur_radius;      /* Section 3.4 heuristic pricing: > 0 prices only
                                J = {(i,j): distance < heur_radius * D} (D the largest
                                distance of the points' bounding box in the cost's norm;
                                integer key bound ceil(r^2 Dsq) for the squared and 2-norm
                                costs, ceil(r D) for the 1- and inf-norm) in heur_run
                                consecutive iterations out of every heur_run + 1; the
                                stop test and certificate always scan all m n.  0: off */
    int32_t heur_run;        /* consecutive heuristic iterations before a full scan (3) */
    double switch_back_grow; /* Section 4.3 remark: after the switch, return to CG when
                                psi has grown by this fraction over the switch window
                                (and the switch was made by the support-drop rule);
                                0: never */
    int32_t force_switch_back_at; /* >= 0: return to CG at this iteration if the direct
                                     solver is in use (host-forced test hook) */
    int32_t schur_reuse;     /* 1: keep the Schur pattern across support updates that
                                only remove entries (a superset of the new one; its
                                extra entries get the value 0) */
    int32_t ws_union;        /* warm start: 1 (default) starts from the union of the
                                predicted support and the plain rule's (end of
                                Section 3.2); 0 from the predicted support alone */
} otip_params;

/* Problem description.  All arrays are DEVICE pointers.
 *   a  : m doubles, >= 0         b : n doubles, >= 0, |sum a - sum b| <= 1e-12 sum a,
 *        sums > 0.  Rows and columns of zero mass are dropped before solving and
 *        returned with zero flow and c-transform duals (every reduced cost of
 *        theirs >= 0), so the certificate covers the whole problem.
 *   xs : m x 2 int32, row-major   xt: n x 2 int32, row-major, coordinates in
 *        [-2^14, 2^14] so that every cost fits in 31 bits.
 *   y0, z0: optional predicted duals (m and n doubles, cost units) or both NULL.
 *        When given, the initial support is built from them instead of from
 *        the costs alone (a warm start); the method and its certificate are
 *        unchanged.  Non-finite values fall back to the plain initial support.
 *   cost_kind: otip_cost (0, the squared 2-norm, in a zero-initialised struct). */
typedef struct otip_problem {
    int32_t m;
    int32_t n;
    const double *a;
    const double *b;
    const int32_t *xs;
    const int32_t *xt;
    const double *y0;
    const double *z0;
    int32_t cost_kind; /* otip_cost; any other value is OTIP_EINVAL */
} otip_problem;

/* Summary of a solve (Section 5.3 reports iterations, time, CG iterations,
 * fill and iterative/direct iteration counts; Table 3). */
typedef struct otip_info {
    int32_t status;            /* OTIP_OK (certified), OTIP_EMAXITER or OTIP_ENUMERIC */
    int32_t iterations;        /* outer iterations */
    int32_t cg_iterations;     /* total CG iterations */
    int32_t direct_iterations; /* iterations solved by the direct factorisation */
    int64_t nnz;               /* nonzeros of the returned plan (<= m+n-1) */
    int64_t psi_max;           /* largest support size seen */
    double objective;          /* sum_ij C_ij P_ij of the returned plan */
    double dual_bound;         /* a.y + b.z + sum(a)*min(0, r_min): a certified lower bound */
    double rel_gap;            /* (objective - dual_bound) / max(1, |objective|) */
    double marginal_residual;  /* ||P e - a||_1 + ||P^T e - b||_1 over ||a||_1 + ||b||_1 */
    double r_min;              /* min over all (i,j) of C_ij - y_i - z_j */
    double max_fill_pct;       /* largest factor density, 100*nnz(L)/n^2 */
    double seconds_total;
    double seconds_pricing;    /* full m*n scans (pricing, certification) */
    double seconds_newton;     /* Schur assembly, solves, step computation */
    double seconds_direct;     /* dense factorisations (part of seconds_newton) */
    double seconds_update;     /* support update and rebuild */
    double seconds_setup;      /* initial support, starting point */
    double seconds_final;      /* polish, purification, certificate */
    int64_t pricing_scans;     /* full m*n passes of the pricing and certificate scans */
    /* with params.profile: event-timed launches of the hot kernels, sampled so
       that the events do not slow the solve */
    int64_t spmv_launches;     /* CG iteration launches (Schur SpMV with the vector updates
                                  and the dot products, one per iteration), those of the
                                  first of every 8 CG solves */
    double spmv_ms;            /* their summed durations */
    double spmv_bytes;         /* their algorithmic bytes: 12 nnz + 100 n per launch (FP64;
                                  8 nnz + 52 n for the FP32 inner solves); a Schur matrix
                                  beyond 96 MB takes two launches per iteration, of which
                                  the SpMV is timed: 12 nnz + 36 n (8 nnz + 20 n) */
    int64_t price_launches;    /* pricing-pass launches of the first of every 8 pricing
                                  calls */
    double price_ms;
    double price_elems;        /* reduced costs evaluated: m*n per launch */
    int64_t diag_launches;     /* diagonal-block factor launches of the dense LDL^T (those of
                                  the first of every 8 factorisations: events at every dispatch
                                  of the dependent chain would slow it) */
    double diag_ms;
    double diag_flops;         /* 2 b^3 / 3 per launch of a b x b block (factor and inverse of
                                  its unit lower factor, b^3 / 3 each) */
    int64_t update_launches;   /* trailing-update launches of the dense LDL^T (same sample) */
    double update_ms;
    double update_flops;       /* r^2 b per launch: the lower triangle of an r x r trailing
                                  matrix less a rank-b product (b = 64 or, two block columns
                                  at once, 128); 2b (c(r-c) + c(c+1)/2) for a launch that
                                  updates only the next c-wide block column */
    int64_t heuristic_scans;   /* pricing calls on the heuristic subset (Section 3.4) */
    int64_t switches_back;     /* returns from the direct solver to CG (Section 4.3) */
    int64_t patterns_kept;     /* support updates that kept the Schur pattern (schur_reuse) */
} otip_info;

typedef struct otip_ctx otip_ctx;
typedef struct otip_result otip_result;

/* ABI version of the loaded library (OTIP_ABI_VERSION). */
int otip_version(void);

/* Identity of the sources the library was built from: a 16-hex-digit hash of
 * the library's source files and this header, fixed at build time.  Static
 * string, never NULL; "unknown" for a build that did not set it. */
const char *otip_source_id(void);

/* Fill *p with the defaults described above. */
void otip_params_default(otip_params *p);

/* Create a context on HIP device `device`; `hip_stream` is a hipStream_t to
 * run on (NULL: the default stream).  On success *ctx owns device scratch
 * memory that otip_destroy frees.  Errors: OTIP_EINVAL, OTIP_EHIP. */
int otip_create(otip_ctx **ctx, int device, void *hip_stream);
void otip_destroy(otip_ctx *ctx);

/* Message of the last error on this context (never NULL). */
const char *otip_last_error(const otip_ctx *ctx);

/*
 * Solve one problem (the whole method of Sections 3-4: initial support,
 * Newton steps on the restricted problem, pricing and support updates, the
 * CG -> LDL^T switch; then a final primal projection, purification to a basic
 * plan and the dual certificate).  params may be NULL (defaults).
 * OTIP_OK means certified: the plan meets the marginals to 1e-9 (relative, 1-norm)
 * and its gap to the certified dual bound is at most params->tol.  On OTIP_OK,
 * OTIP_EMAXITER (limits reached before that) or OTIP_ENUMERIC (the iterate
 * became non-finite) *out holds a result to query and free; only OTIP_OK's is
 * certified.
 */
int otip_solve(otip_ctx *ctx, const otip_problem *pr, const otip_params *params,
               otip_result **out);

/*
 * Solve `count` independent problems; outs[k] receives each result.  The
 * problems are taken largest first (by m*n) by params->batch_workers host
 * workers, each owning a non-blocking HIP stream (default priority) and a
 * solver whose device buffers persist across problems and calls, so that the
 * many small launches of different instances overlap on the device.  Input
 * arrays must be ready on the context's stream, which is synchronised first.
 * Returns OTIP_OK if every instance is certified, else OTIP_EMAXITER or
 * OTIP_ENUMERIC (the worse of the instances' statuses); every outs[k] is valid
 * then and its info.status tells its own.  On any other error no result is returned
 * (every outs[k] is NULL) and otip_last_error names the failing instance.
 * The context must not be used by another thread during the call.
 */
int otip_solve_batch(otip_ctx *ctx, const otip_problem *prs, int32_t count,
                     const otip_params *params, otip_result **outs);

int otip_result_info(const otip_result *r, otip_info *info);
/* Copy the plan (COO, sorted by variable index i + j*m, nnz entries) and the
 * duals, gauge-normalised so that z[n-1] = 0, into HOST buffers.  Any pointer
 * may be NULL to skip that output. */
int otip_result_copy(const otip_result *r, int32_t *rows, int32_t *cols, double *vals,
                     double *y, double *z);
void otip_result_free(otip_result *r);

/*
 * Pricing scan (Sections 3.2 and 3.4): over all variables NOT in the support,
 * the reduced costs r_ij = (C_ij - y_i) - z_j (two IEEE double subtractions in
 * this order, C_ij the double of otip_cost cost_kind); the at most kmax
 * strictly negative ones, ordered by (r, i + j*m) ascending, are returned.
 *   xs, xt, y (m), z (n): DEVICE.  support_bitmap: DEVICE, ceil(m*n/32) words,
 *   bit (idx & 31) of word idx >> 5 set for variables in the support; NULL for
 *   an empty support.  out_i, out_j (int32), out_r (double): DEVICE, kmax
 *   entries.  out_count (selected) and out_nneg (all negative reduced costs
 *   outside the support): HOST.
 *   precision: OTIP_FP64, or OTIP_MIXED (FP32 scan with an FP64 re-check of
 *   every candidate within a proven margin; same result).  The FP32 scan is
 *   written for the squared cost: the other kinds take the FP64 scan.
 *   tile: targets per workgroup (as otip_params.price_tile; 0 = by size).
 */
int otip_price(otip_ctx *ctx, int32_t m, int32_t n, const int32_t *xs, const int32_t *xt,
               const double *y, const double *z, const uint32_t *support_bitmap, int64_t kmax,
               int32_t precision, int32_t tile, int32_t cost_kind, int32_t *out_i,
               int32_t *out_j, double *out_r, int64_t *out_count, int64_t *out_nneg);

/*
 * Heuristic pricing (Section 3.4): otip_price restricted to the subset
 * J = {(i, j) : integer cost key < key_limit} fixed before the iteration (the
 * key is the cost itself, the squared norm for the 2-norm; otip_params
 * heur_radius describes how the solver chooses key_limit).  Same arguments,
 * ordering and exactness as otip_price in FP64; the selected columns, the
 * count out_nneg and the values are those of the variables of J only.  The
 * subset is built on the device for each call (per-source target lists,
 * 4 bytes per member of J plus 8 bytes per source, held by the context).
 *   key_limit: >= 1.  out_subset_size: HOST, optional, |J|.
 */
int otip_price_subset(otip_ctx *ctx, int32_t m, int32_t n, const int32_t *xs, const int32_t *xt,
                      const double *y, const double *z, const uint32_t *support_bitmap,
                      int64_t kmax, int32_t cost_kind, int64_t key_limit, int32_t *out_i,
                      int32_t *out_j, double *out_r, int64_t *out_count, int64_t *out_nneg,
                      int64_t *out_subset_size);

/* min over ALL (i, j) of (C_ij - y_i) - z_j (C_ij of otip_cost cost_kind) and
 * the first variable index attaining it (Section 3.3: s_hat = c - A^T y_hat).
 * Outputs are HOST. */
int otip_rmin(otip_ctx *ctx, int32_t m, int32_t n, const int32_t *xs, const int32_t *xt,
              const double *y, const double *z, int32_t cost_kind, double *out_rmin,
              int64_t *out_arg);

/*
 * Matrix-free Kronecker products of Section 2.1 on a dense m x n array X
 * stored column-major (x = vec(X)), all DEVICE:
 *   otip_kron_apply : rowsum = A_1 x = X e_n (m), colsum = A_2 x = X^T e_m (n)
 *   otip_kron_apply_t: X = vec^{-1}(A_1^T y + A_2^T z), X_ij = y_i + z_j
 */
int otip_kron_apply(otip_ctx *ctx, int32_t m, int32_t n, const double *X, double *rowsum,
                    double *colsum);
int otip_kron_apply_t(otip_ctx *ctx, int32_t m, int32_t n, const double *y, const double *z,
                      double *X);

/*
 * otip_kron_apply without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, kernels and results (bit for bit)
 * as otip_kron_apply; X, rowsum and colsum are caller-owned DEVICE arrays.
 * The partial sums live in a static array of 64 MiB per GPU (held from library
 * load to process end), so m and n are limited to
 *   ceil(n / 64) m + ceil(m / 1024) n <= 8,388,608   (m n up to about 4.9e8);
 * larger sizes return OTIP_EINVAL with a message and launch nothing.  Every
 * call on one GPU shares that GPU's array: calls that overlap in time on one
 * GPU (several contexts or streams) race and must be serialised by the caller.
 * Errors: OTIP_EINVAL (bad arguments, too large), OTIP_EHIP.
 */
int otip_kron_apply_noalloc(otip_ctx *ctx, int32_t m, int32_t n, const double *X,
                            double *rowsum, double *colsum);

/*
 * Normal-equation blocks on a support (Sections 3.5 and 4).  idx: DEVICE, psi
 * variable indices sorted ascending, no duplicates, every row and column of
 * the plan covered; theta: DEVICE, psi positive values (theta = p/s).
 * Computes M = row sums, N = column sums of V (vec(V) = theta on the support)
 * and the Schur complement S_M = N - V^T M^-1 V in CSR form (n x n, column
 * indices sorted).  Two calls: with rowptr == NULL only *out_nnz (HOST) is
 * set; then pass rowptr (n+1 int32), colidx (nnz int32), vals (nnz double),
 * M (m), N (n), all DEVICE.  The diagonal is formed as minus the sum of the
 * off-diagonal entries of its row, which eq. diagdom shows equal to
 * N_jj - (V^T M^-1 V)_jj without the cancellation of the latter.
 */
int otip_schur(otip_ctx *ctx, int32_t m, int32_t n, int64_t psi, const int64_t *idx,
               const double *theta, int64_t *out_nnz, int32_t *rowptr, int32_t *colidx,
               double *vals, double *M, double *N);

/*
 * Preconditioned conjugate gradients of the Newton step (Section 4, eq. for
 * the Schur complement; tolerances of Section 5.2), on a caller's matrix:
 * solves S x = b for a symmetric positive (semi)definite n x n CSR matrix with
 * the Jacobi preconditioner, stopping when ||b - S x||_2 <= rtol ||b||_2 (as
 * the iteration's recurrence tracks it) or after maxit iterations, as inside
 * otip_solve: one launch per iteration (the single-reduction form of CG:
 * SpMV, vector updates and the three dot products together), or two for a
 * matrix that streams from HBM (below).
 *   rowptr (n+1 int32), colidx (nnz int32, in [0, n)), vals (nnz), b (n):
 *   DEVICE, read only (copied; rowptr is validated on the host, colidx on the
 *   device).  x (n): DEVICE, output (the iteration starts from 0).  A row
 *   whose diagonal is absent or not positive gets preconditioner 0.  For a
 *   singular S (as the Schur complement, whose rows sum to 0) b must lie in
 *   its range.
 *   precision: OTIP_FP64, or OTIP_MIXED (FP32 CG inside FP64 iterative
 *   refinement on the FP64 residual).
 *   iterations, res_norm: HOST, optional.  spmv_stats: HOST, optional, 3
 *   values: iteration launches that did work, their mean duration in seconds
 *   (events recorded at the dispatches' own start and end), and their
 *   algorithmic bytes per launch ((w + 4) nnz + (4 + 12 w) n, w = 8 in FP64
 *   and 4 in the FP32 inner solves).  A matrix whose values and columns
 *   exceed 96 MB streams from HBM at every iteration: it takes two launches
 *   per iteration (an SpMV with the direction update, timed here at
 *   (w + 4) nnz + (4 + 4 w) n bytes, and a vector update).
 * Returns OTIP_OK when converged, OTIP_EMAXITER when maxit was reached,
 * OTIP_ENUMERIC on a breakdown (p'Sp <= 0).
 */
int otip_pcg(otip_ctx *ctx, int32_t n, int64_t nnz, const int32_t *rowptr, const int32_t *colidx,
             const double *vals, const double *b, double *x, double rtol, int32_t maxit,
             int32_t precision, int32_t *iterations, double *res_norm, double *spmv_stats);

/*
 * Direct solve of the Newton step after the switch (Section 4.2): the
 * library's FP64 L D L^T of a caller's symmetric n x n CSR matrix with the
 * infinite-pivot rule (a pivot d_k <= pivot_tol * A_kk or d_k <= 0 becomes
 * +inf: that unknown is 0 in the solution, grounding one node of each
 * connected component of a singular Schur complement), then x = (L D L^T)^+ b
 * through the explicit inverse of L as inside otip_solve.
 *   rowptr (n+1), colidx (nnz, in [0, n), both triangles), vals, b (n):
 *   DEVICE, read only.  x (n): DEVICE, output.  flags: bit 0 solves by
 *   substitution on L and L^T instead of the explicit inverse (the path taken
 *   when the inverse is not finite).  out_ninf (infinite pivots) and
 *   out_nnz_L (nonzeros of L counted as written, plus n): HOST, optional.
 * Memory: about 3.25 * 8 n^2 bytes of device scratch for the call.
 * Errors: OTIP_EINVAL, OTIP_ENOMEM, OTIP_EHIP.
 */
int otip_ldl_solve(otip_ctx *ctx, int32_t n, int64_t nnz, const int32_t *rowptr,
                   const int32_t *colidx, const double *vals, double pivot_tol, int32_t flags,
                   const double *b, double *x, int32_t *out_ninf, int64_t *out_nnz_L);

/*
 * Checkpoint and resume (the paper has none; these serve long solves and the
 * replay of an iteration).  Every otip_solve records, in host memory, the
 * state at which it stopped iterating, before its certificate and
 * purification: the support, the iterate (p, s, y, z), the iteration count
 * and the loop's own state (solver mode, support-size history, the last CG
 * work, the stop tolerance in force).
 *   otip_state_save: writes that record of the context's latest otip_solve to
 *     buf (HOST, cap bytes) and its length to *size (HOST); with buf NULL only
 *     the length.  OTIP_EINVAL before any solve or when cap is too small.
 *   otip_state_load: reads a record (HOST bytes) and makes the context's next
 *     otip_solve continue from it instead of building an initial support;
 *     that solve must be of the same problem (m, n, the cost kind and the
 *     bytes of a, b, xs, xt, compared through a 64-bit hash), else it fails
 *     with OTIP_EINVAL.
 *     The record is checked (sizes, increasing support indices below m*n, an
 *     interior iterate) before it reaches the device.  y0/z0 are ignored by a
 *     resumed solve.
 * A solve stopped by max_iter and resumed with a larger max_iter and
 * otherwise equal parameters takes the same steps as one solve with the larger
 * max_iter.  The layout is the library's own (host byte order), versioned.
 * otip_solve_batch neither records nor resumes.
 */
int otip_state_save(otip_ctx *ctx, void *buf, int64_t cap, int64_t *size);
int otip_state_load(otip_ctx *ctx, const void *buf, int64_t size);

/* ------------------------------------------------------------------------
 * Learned warm start.  A small convolutional network maps the two marginals of
 * a side x side grid problem (pixel i at coordinates (i / side, i % side)) to
 * predicted duals; passing them as otip_problem.y0/z0 replaces the initial
 * support rule of Section 3.2 (end) by the c-transform of the prediction and
 * its smallest reduced costs.  The solve, its pricing and its certificate are
 * those of the plain method, so a poor prediction costs time, not accuracy.
 *
 * Network (FP32): four 3x3 convolutions, 2 -> 32 -> 32 -> 32 -> 2 channels,
 * dilations 1, 2, 4, 8, zero padding equal to the dilation, ReLU after the
 * first three.  Parameters: one flat FP32 array of otip_ws_param_count()
 * values, per layer W[out][in][3][3] then b[out].  Input x: N x 2 x H x W
 * (NCHW, the marginals as densities: mass * side^2 per pixel); output: N x 2 x
 * H x W (duals in normalised coordinates: pixel cost units / side^2, any
 * gauge).  All pointers are DEVICE pointers except `loss`.
 * ------------------------------------------------------------------------ */
int64_t otip_ws_param_count(void);

/* out = net(in).  batch <= 65535, H*W <= 2^24. */
int otip_ws_forward(otip_ctx *ctx, const float *weights, int32_t batch, int32_t h, int32_t w,
                    const float *in, float *out);

/* Gradient of the mean squared error mean((net(in) - target)^2) with respect
 * to the parameters into grad (otip_ws_param_count() floats); the loss into
 * *loss (host, may be NULL).  Weight-gradient sums are accumulated in FP64. */
int otip_ws_grad(otip_ctx *ctx, const float *weights, int32_t batch, int32_t h, int32_t w,
                 const float *in, const float *target, float *grad, double *loss);

/* One Adam step (Kingma & Ba) with bias correction for step >= 1; weights,
 * first and second moments m, v are updated in place (FP32).  The
 * hyperparameters are doubles so that 1 - beta is formed exactly. */
int otip_ws_adam(otip_ctx *ctx, float *weights, float *m, float *v, const float *grad,
                 int32_t step, double lr, double beta1, double beta2, double eps);

/* Predicted duals of a side x side grid problem with marginals a, b (m = n =
 * side^2 doubles): the marginals are averaged over a 32 x 32 partition of the
 * square (exact area weights), the network runs at 32 x 32, and its output is
 * interpolated bilinearly at the pixel centres (clamped at the border) and
 * scaled by side^2 into y0, z0 (pixel cost units). */
int otip_ws_predict(otip_ctx *ctx, const float *weights, int32_t side, const double *a,
                    const double *b, double *y0, double *z0);

#ifdef __cplusplus
}
#endif
#endif /* OTIP_H */
