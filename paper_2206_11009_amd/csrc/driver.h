// Solver state of one problem (internal).
#pragma once

#include <cstdarg>
#include <memory>

#include "../../include/otip.h"
#include "internal.h"

namespace otip {

struct Result {
    otip_info info{};
    std::vector<int32_t> rows, cols;
    std::vector<double> vals, y, z;
};

// Host-side purification of a plan to an acyclic support (purify.cpp).
void purify_plan(int m, int n, const std::vector<int32_t> &rows, const std::vector<int32_t> &cols,
                 const std::vector<double> &flows, const std::vector<double> &costs,
                 const std::vector<double> &a, const std::vector<double> &b, double drop_rel,
                 std::vector<int32_t> &orows, std::vector<int32_t> &ocols,
                 std::vector<double> &oflows);

enum class Mode { PCG, Direct };

// Where a solve stopped iterating (before its certificate and purification):
// the iterate and the loop's own state, enough to continue the iteration
// exactly as if it had not stopped.  Host memory.
struct Checkpoint {
    int32_t m = 0, n = 0;
    uint64_t fingerprint = 0;  // of m, n, the cost kind and the bytes of a, b, xs, xt
    int32_t it = 0, mode = 0, cg_its_last = 0, solves_last = 2, cg_failed = 0, warm_used = 0;
    int32_t direct_its = 0;
    int32_t forced_switch_done = 0, forced_back_done = 0, switched_by_drop = 0,
            switches_back = 0;
    int64_t psi = 0, psi_max = 0, cg_total = 0;
    double tol_int = 0.0, max_fill = 0.0;
    std::vector<int64_t> psi_hist;
    std::vector<uint64_t> idx;
    std::vector<double> p, s, y, z;
};

struct Dir {
    DBuf<double> dp, ds, dy, dz;
};

class Solver {
  public:
    explicit Solver(hipStream_t s) : st(s) {}
    int run(const otip_problem &pr, const otip_params &prm, Result &res);
    // normal-equation blocks and S_M for a given support and theta (parity checks)
    int64_t schur_export(int m, int n, int64_t psi, const uint64_t *idx, const double *theta,
                         int32_t *rowptr, int32_t *colidx, double *vals, double *Mout,
                         double *Nout);
    // the state at which the latest run stopped iterating (null before any)
    const Checkpoint *last_state() const { return have_last_ ? &last_ : nullptr; }
    // a state for the next run to continue from (it must be the same problem)
    void set_resume(std::unique_ptr<Checkpoint> c) { pending_ = std::move(c); }

  private:
    void rebuild_views();
    void alloc_support(int64_t cap);
    void rowsum(const double *v, const double *base, double *out, double sign);
    void colsum(const double *v, const double *base, double *out, double sign);
    void newton(const double *r1a, const double *r1b, const double *r2, const double *r3,
                double rtol, double atol, Dir &out);
    void max_steps(const Dir &d, double &ap, double &ad);
    void assemble();
    void residuals(double &rel1, double &rel2, double &mu, double &primal, double &r1n);
    int64_t price(int64_t kmax, uint64_t *out_idx, double *out_r, int64_t *nneg,
                  bool heuristic = false);
    void update_support(const uint64_t *add_idx, int64_t nadd, double pin, const uint8_t *removed,
                        int64_t nrem);
    int64_t select_removals(uint8_t *removed);
    void starting_point();
    // the dense direct solver is allowed (dense_max_n) and its buffers fit in
    // the device memory still free
    bool direct_available();
    void finalize(Result &res);
    void reset_state();
    void snapshot(int it, double tol_int, const std::vector<int64_t> &hist);
    void resume_from(const Checkpoint &c);
    int run_without_zeros(const otip_problem &pr, const otip_params &prm, Result &res);
    static double now();
    void log(const char *fmt, ...);
    // debug aid (OTIP_TRACE in the environment): FNV-1a hash of a device
    // buffer, printed with the problem's fingerprint, a tag and the iteration
    void trace(const char *tag, int it, const void *dev, size_t bytes);
    void trace_val(const char *tag, int it, double v);

    hipStream_t st;
    otip_params P{};
    Scanner scan;
    Reducer red;
    SchurSolver schur;
    DenseLDL ldl;
    DBuf<char> tmp;
    LaunchTimer t_spmv, t_price, t_diag, t_upd;

    int m = 0, n = 0;
    const int32_t *xs = nullptr, *xt = nullptr;
    int kind = 0;      // otip_cost
    int64_t cmax = 0;  // largest cost key (the squared norm for the 2-norm)
    double omega = 1.0, zeta = 1.0, fnorm = 0.0;
    const double *a_in = nullptr, *b_in = nullptr;

    int64_t psi_ = 0, psi_max = 0;
    DBuf<uint64_t> idx;
    DBuf<int32_t> si, sj, col_ptr, row_ptr, csr_pos;
    DBuf<double> p, s, c, theta, r2, r3, w;
    DBuf<uint8_t> prot;
    DBuf<uint32_t> bitmap;
    DBuf<double> a, b, y, z, M, invM, N, r1a, r1b, beta1, beta2, rhs, tmpn, tmpn2, zm, zn, zpsi;
    DBuf<double> yun, zun;
    Dir D[3];
    DBuf<uint64_t> tmp_u64a, tmp_u64b, tmp_u64c, tmp_u64d;
    DBuf<double> tmp_f64a, tmp_f64b, tmp_f64c, tmp_f64d;
    DBuf<int32_t> tmp_i32a, tmp_i32b;
    DBuf<uint32_t> tmp_u32a;
    DBuf<uint64_t> init_, init2_, sel_idx_;
    DBuf<unsigned long long> ucnt_;
    DBuf<double> sel_r_;
    DBuf<uint8_t> removed_;
    DBuf<int32_t> zc_;
    DBuf<double> yws_, zws_, zmass_, zdual_;
    DBuf<int32_t> zcoord_;
    bool warm_used = false;
    bool schur_valid = false;
    uint64_t fp_ = 0;
    Checkpoint last_;
    bool have_last_ = false;
    std::unique_ptr<Checkpoint> pending_;

    Mode mode = Mode::PCG;
    bool cg_failed = false;
    bool heur_on = false;        // heuristic pricing subset built for this solve
    int64_t heur_scans = 0;      // pricing calls on the subset
    bool forced_switch_done = false, forced_back_done = false;
    bool switched_by_drop = false;  // the last switch to Direct came from the psi-drop rule
    int switches_back = 0;
    bool pattern_kept = false;   // the last support update kept the Schur pattern
    int64_t patterns_kept = 0;
    int cg_its_iter = 0, max_cg_solve = 0;
    int64_t cg_total = 0;
    int direct_its = 0, iterations = 0;
    int64_t pricing_passes = 0;
    double max_fill = 0.0;
    int cg_its_last = 0;
    int solves_last = 2;
    double t_pricing = 0, t_newton = 0, t_direct = 0, t_update = 0, t_setup = 0, t_final = 0;
};

}  // namespace otip
