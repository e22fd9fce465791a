// Internal interfaces between the otip sources (not part of the ABI).
#pragma once

#include <algorithm>
#include <cmath>

#include "../../include/otip.h"
#include "common.h"

namespace otip {

// ------------------------------------------------------------ sort / scan (rocPRIM)
void sort_pairs_u64(hipStream_t st, const uint64_t *kin, const uint64_t *vin, uint64_t *kout,
                    uint64_t *vout, int64_t n, int begin_bit, int end_bit, DBuf<char> &tmp);
void sort_pairs_u64_f64x2(hipStream_t st, const uint64_t *kin, const double *v1in,
                          const double *v2in, uint64_t *kout, double *v1out, double *v2out,
                          int64_t n, int end_bit, DBuf<char> &tmp, DBuf<int32_t> &perm_a,
                          DBuf<int32_t> &perm_b);
void sort_pairs_u32_i32(hipStream_t st, const uint32_t *kin, const int32_t *vin, uint32_t *kout,
                        int32_t *vout, int64_t n, int end_bit, DBuf<char> &tmp);
void sort_keys_u64(hipStream_t st, const uint64_t *kin, uint64_t *kout, int64_t n,
                   DBuf<char> &tmp);
int64_t unique_u64(hipStream_t st, const uint64_t *in, uint64_t *out, int64_t n, DBuf<char> &tmp,
                   DBuf<unsigned long long> &cnt);
void exclusive_scan_i64(hipStream_t st, const int64_t *in, int64_t *out, int64_t n,
                        DBuf<char> &tmp);

// ------------------------------------------------------------------- full scans
// targets per scan block: `tile` if it is a power of two in [16, 256], else a
// size-based choice
int pick_tj(int m, int n, int tile);

struct PriceResult {
    int64_t count;  // selected
    int64_t nneg;   // negative reduced costs outside the support
    int passes;     // full m*n passes used
};

class Scanner {
  public:
    LaunchTimer *timer = nullptr;  // pricing-pass launches (optional)
    int64_t scans = 0;             // full m*n passes so far
    int tile = 0;                  // targets per scan block (0: chosen from m, n)
    int kind = 0;                  // otip_cost of every scan
    // <= kmax most negative reduced costs outside the support, ordered by
    // (r, idx); outputs may be null.
    PriceResult price(hipStream_t st, int m, int n, const int32_t *xs, const int32_t *xt,
                      const double *y, const double *z, const uint32_t *bitmap, int64_t kmax,
                      int32_t *oi, int32_t *oj, double *orr, uint64_t *oidx);
    // FP32 scan with an FP64 re-check of every candidate within the margin
    PriceResult price_mixed(hipStream_t st, int m, int n, const int32_t *xs, const int32_t *xt,
                            const double *y, const double *z, const uint32_t *bitmap,
                            int64_t kmax, int32_t *oi, int32_t *oj, double *orr,
                            uint64_t *oidx);
    void rmin(hipStream_t st, int m, int n, const int32_t *xs, const int32_t *xt,
              const double *y, const double *z, double *out, int64_t *arg);
    int64_t initial_support(hipStream_t st, int m, int n, const int32_t *xs, const int32_t *xt,
                            double kappa, int64_t cmax, DBuf<uint64_t> &out, int64_t *T);
    // c-transforms: y_i = min_j (C_ij - z_j), z_j = min_i (C_ij - y_i) (an entry
    // of -inf in the given duals excludes its row or column)
    void ctransform_rows(hipStream_t st, int m, int n, const int32_t *xs, const int32_t *xt,
                         const double *z, double *y);
    void ctransform_cols(hipStream_t st, int m, int n, const int32_t *xs, const int32_t *xt,
                         const double *y, double *z);
    // initial support from predicted duals (c-transform, smallest reduced
    // costs, row and column covers); -1 if the duals are unusable
    int64_t warm_support(hipStream_t st, int m, int n, const int32_t *xs, const int32_t *xt,
                         const double *y0, const double *z0, double kappa,
                         DBuf<uint64_t> &out, DBuf<double> &yw, DBuf<double> &zw);
    // heuristic subset J = {(i, j) : integer cost key < key_limit} of
    // Section 3.4, kept as per-source target lists; returns |J|.  While
    // use_subset is set, price() scans J only (in FP64, also for price_mixed).
    int64_t set_subset(hipStream_t st, int m, int n, const int32_t *xs, const int32_t *xt,
                       int64_t key_limit);
    bool use_subset = false;
    int64_t subset_size() const { return subset_nnz_; }
    // forget the cutoff guessed from the previous pricing call (a new problem)
    void reset_guess() {
        guess_key_ = 0;
        guess_f_ = 0.5;
    }

  private:
    void prepare(hipStream_t st, int m, int n, const int32_t *xt, const double *z);
    DBuf<char> jt_;
    DBuf<unsigned long long> hist_, cnt_;
    DBuf<uint64_t> ck_, ci_, ck2_, ci2_, u64a_, u64b_;
    DBuf<int64_t> i64a_, i64b_;
    DBuf<double> bmin_;
    DBuf<uint64_t> barg_;
    DBuf<char> tmp_;
    DBuf<float> f32a_;
    DBuf<int> flag_;
    DBuf<int64_t> sptr_, scnt_;
    DBuf<int32_t> scol_;
    int subset_m_ = -1;
    int64_t subset_nnz_ = 0;
    uint64_t guess_key_ = 0;  // cutoff key for the first pass's compaction (0: none)
    double guess_f_ = 0.5;    // with fewer than 4 kmax candidates kept: the next cutoff as a
                              // fraction of the last candidate's value
};

// ---------------------------------------------------------- fixed-order reductions
// Sums (or minima) of up to 8 per-element quantities in a fixed, input-size
// determined order: results are bitwise reproducible.
class Reducer {
  public:
    static constexpr int kBlocks = 256;
    static constexpr int kThreads = 256;
    double *partial(int k) { return part_.need((size_t)kBlocks * 8) + (size_t)k * kBlocks; }
    double *base() { return part_.need((size_t)kBlocks * 8); }
    // fetch K totals of the partial sums written by a reduce kernel
    void fetch_sum(hipStream_t st, int K, int nblocks, double *out);
    void fetch_min(hipStream_t st, int K, int nblocks, double *out);

  private:
    DBuf<double> part_;
    DBuf<double> out_;
    std::vector<double> host_;
};

// ---------------------------------------------------------------- Schur / PCG
struct SchurCSR {
    int n = 0;
    int64_t nnz = 0;
    DBuf<int32_t> rowptr, col, row, diag;
    DBuf<double> val, dinv;
};

struct CGStats {
    int iterations = 0;
    bool converged = false;
    double res_norm = 0.0;
};

struct CGScal;  // device-side CG scalars (schur.hip)

// CG on a Schur matrix of nnz values of w bytes: beyond 96 MB of values and
// columns the matrix streams from HBM at every iteration and the two-launch
// form runs (an SpMV launch with the direction, an update launch); below, one
// launch per iteration.  Algorithmic bytes of the timed launch of each form:
// values and columns, row pointers, and the vectors read and written once.
inline bool cg_streams(double w, int64_t nnz) { return (w + 4.0) * (double)nnz > 96.0 * (1 << 20); }
inline double cg_launch_bytes(double w, int64_t nnz, int n) {
    return (w + 4.0) * (double)nnz + (cg_streams(w, nnz) ? 4.0 + 4.0 * w : 4.0 + 12.0 * w) * n;
}

class SchurSolver {
  public:
    LaunchTimer *timer = nullptr;  // SpMV launches inside CG (optional)
    // pattern of S_M = N - V^T M^-1 V for the support (CSC arrays by column)
    void symbolic(hipStream_t st, int m, int n, int64_t psi, const int32_t *col_ptr,
                  const int32_t *si, const int32_t *row_ptr, const int32_t *csr_pos,
                  const int32_t *sj);
    // keep the pattern of the last symbolic() for a support that only lost
    // entries (it is a superset of the new pattern; the extra entries get the
    // value 0): repacks the per-source target lists of the new support
    void keep_pattern(hipStream_t st, int64_t psi, const int32_t *csr_pos, const int32_t *sj);
    // values: S_jk = -sum_{i in col j and col k} theta_ij theta_ik / M_i (j != k),
    // S_jj = -sum_{k != j} S_jk; also the Jacobi inverse diagonal
    void numeric(hipStream_t st, int m, int n, const int32_t *col_ptr, const int32_t *si,
                 const int32_t *row_ptr, const int32_t *csr_pos, const int32_t *sj,
                 const double *theta, const double *invM);
    // S from a caller's CSR matrix (device arrays, copied; row pointers and
    // column indices validated) with its Jacobi inverse diagonal
    void load_csr(hipStream_t st, int n, int64_t nnz, const int32_t *rowptr, const int32_t *col,
                  const double *val);
    // y = S x
    void spmv(hipStream_t st, const double *x, double *y);
    // Jacobi-preconditioned CG on S x = b (b projected on e-perp by the caller)
    CGStats pcg(hipStream_t st, const double *b, double *x, double rtol, double atol, int maxit);
    // the same in FP32 inside FP64 iterative refinement
    CGStats pcg_mixed(hipStream_t st, const double *b, double *x, double rtol, double atol,
                      int maxit);
    SchurCSR S;

  private:
    template <typename T>
    CGStats pcg_impl(hipStream_t st, const T *val, const T *dinv, const T *b, T *x, double rtol,
                     double atol, int maxit, DBuf<T> &p, DBuf<T> &g);
    template <typename T>
    CGStats pcg_stream(hipStream_t st, const T *val, const T *dinv, const T *b, T *x,
                       double rtol, double atol, int maxit, T *r, T *g, double *part,
                       CGScal *sc, int *done);
    DBuf<int32_t> cnt_, rk_;
    DBuf<double> rth_;
    int64_t psi_ = 0;  // support size of the last symbolic()
    int32_t span_ = 0;  // largest kmax - kmin + 1 over the rows of S
    DBuf<char> tmp_;
    DBuf<int64_t> off64_, cnt64_;
    DBuf<double> p_, g_, part_, scal_, rd_, sx_, rpart_;
    DBuf<float> val32_, dinv32_, rf_, df_, pf_, gf_;
    DBuf<int> flag_;
};

// From this order on, the dense inverse X = L^-1 omits its top doubling level
// and the solves apply the factor's off-diagonal block between the two halves.
constexpr int kDenseSplitMinN = 2048;
// Largest order whose starting point (Theta = I, a well-conditioned system)
// is solved by the dense factorisation rather than by CG.
constexpr int kDenseStartMaxN = 16384;
// Panels (64-column blocks of L) the dense factorisation's trailing update
// applies per pass over the trailing matrix.
constexpr int kDenseUpdPanels = 4;

// Dense LDL^T (FP64) of a Schur complement with the infinite-pivot rule.
class DenseLDL {
  public:
    // factor the CSR matrix; returns number of infinite pivots
    int factor(hipStream_t st, const SchurCSR &S, double pivtol);
    void solve(hipStream_t st, const double *b, double *x);
    int64_t nnz_L() const { return nnzL_; }
    // device bytes a factorisation of order n needs, and what this object holds
    static size_t bytes_for(int n) {
        const size_t nn = (size_t)n * (size_t)n;
        return 8 * (3 * nn + nn / 4 + (size_t)kDenseUpdPanels * 64 * n + (size_t)64 * (n + 63) +
                    8 * (size_t)n);
    }
    size_t held_bytes() const {
        return 8 * (A_.cap + X_.cap + XT_.cap + T_.cap + W_.cap + linv_.cap + d_.cap + orig_.cap +
                    v_.cap + t_.cap);
    }
    const double *pivots() const { return d_.get(); }
    int n = 0;
    // optional timers of the diagonal-factor and trailing-update launches;
    // they time the first of every timer_stride factorisations (events at
    // every dispatch of a dependent chain slow it down)
    LaunchTimer *diag_timer = nullptr, *update_timer = nullptr;
    int timer_stride = 8;
    // solve by substitution on L even when the explicit inverse is finite
    // (the path otherwise taken only when the inverse overflows)
    bool force_substitution = false;
    void restart_sampling() { factorisations_ = 0; }

  private:
    DBuf<double> A_, X_, XT_, T_, d_, orig_, W_, v_, linv_, t_;
    DBuf<int> ninf_, bad_, hrow_;
    DBuf<unsigned long long> cnt_;
    int64_t nnzL_ = 0;
    int64_t factorisations_ = 0;
    bool inverse_ok_ = true;
    int split_ = 0;  // X holds the diagonal inverses of [0, split_) and [split_, n)
};

// Warm-start network (cnn.hip): 4 dilated 3x3 convolution layers, 32 channels,
// FP32.  Buffers for activations and gradients are owned here.
class WarmNet {
  public:
    static int64_t param_count();
    // out = net(x), x: N x 2 x H x W, out: N x 2 x H x W (NCHW)
    void forward(hipStream_t st, const float *theta, int N, int H, int W, const float *x,
                 float *out);
    // mean-squared-error loss of net(x) against target; its gradient into g
    double grad(hipStream_t st, const float *theta, int N, int H, int W, const float *x,
                const float *target, float *g);
    void adam(hipStream_t st, float *theta, float *m, float *v, const float *g, int step,
              double lr, double b1, double b2, double eps);
    // predicted duals of a side x side grid pair (pixel cost units)
    void predict(hipStream_t st, const float *theta, int side, const double *a, const double *b,
                 double *y0, double *z0);

  private:
    DBuf<float> a_[3], out_, ga_, gb_, in_;
    DBuf<double> part_;
};

// dense Kronecker products (kron.hip)
void kron_apply(hipStream_t st, int m, int n, const double *X, double *rowsum, double *colsum,
                DBuf<double> &prow, DBuf<double> &pcol);
void kron_apply_t(hipStream_t st, int m, int n, const double *y, const double *z, double *X);
// the same A x with its partial sums in a static per-GPU array (no allocation):
// kKronScratchDoubles doubles (64 MiB), enough for m n up to about 4.9e8
constexpr int64_t kKronScratchDoubles = (int64_t)8 << 20;
void kron_scratch_init(int device);  // once per device, that device current
int64_t kron_scratch_need(int m, int n);
void kron_apply_noalloc(hipStream_t st, int device, int m, int n, const double *X,
                        double *rowsum, double *colsum);

}  // namespace otip
