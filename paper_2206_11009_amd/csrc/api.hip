// C-ABI entry points (include/otip.h).  Every call catches the library's
// exceptions and returns a status code; the message is kept on the context.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <memory>
#include <mutex>
#include <numeric>
#include <thread>

#include "driver.h"

// One worker of otip_solve_batch: a non-blocking stream (default priority) and
// a solver whose device buffers are kept from one problem to the next.
struct BatchWorker {
    hipStream_t st = nullptr;
    std::unique_ptr<otip::Solver> solver;
    ~BatchWorker() {
        solver.reset();
        if (st) (void)hipStreamDestroy(st);
    }
};

struct otip_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    std::unique_ptr<otip::Solver> solver;  // otip_solve's, on `stream`
    std::vector<std::unique_ptr<BatchWorker>> workers;
    otip::Scanner scan;
    otip::SchurSolver schur;
    otip::WarmNet net;
    otip::DBuf<double> buf_a, buf_b, buf_c;
    otip::DBuf<uint64_t> buf_u;
    otip::DBuf<int32_t> buf_i;
    otip::DBuf<char> tmp;
};

struct otip_result {
    otip::Result r;
};

namespace {

template <class F>
int guarded(otip_ctx *ctx, F &&f) {
    if (!ctx) return OTIP_EINVAL;
    try {
        OTIP_HIP(hipSetDevice(ctx->device));
        f();
        ctx->err.clear();
        return OTIP_OK;
    } catch (const otip::Error &e) {
        ctx->err = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        ctx->err = "host allocation failed";
        return OTIP_ENOMEM;
    } catch (const std::exception &e) {
        ctx->err = e.what();
        return OTIP_EHIP;
    }
}

// Checkpoint byte layout (host byte order): "OTIPCKP1", u32 version (2), i32
// m, n, u64 fingerprint, i32 it, mode, cg_its_last, solves_last, cg_failed,
// warm_used, direct_its, forced_switch_done, forced_back_done,
// switched_by_drop, switches_back, i64 psi, psi_max, cg_total, f64 tol_int, max_fill,
// i64 hist_len, then i64 psi_hist[hist_len], u64 idx[psi], f64 p[psi],
// s[psi], y[m], z[n].
constexpr char kCkMagic[8] = {'O', 'T', 'I', 'P', 'C', 'K', 'P', '1'};
constexpr uint32_t kCkVersion = 2;

template <class T>
void put(std::vector<unsigned char> &o, const T *v, size_t count) {
    const unsigned char *c = (const unsigned char *)v;
    o.insert(o.end(), c, c + sizeof(T) * count);
}
template <class T>
void put1(std::vector<unsigned char> &o, T v) {
    put(o, &v, 1);
}

std::vector<unsigned char> serialize(const otip::Checkpoint &c) {
    std::vector<unsigned char> o;
    put(o, kCkMagic, 8);
    put1(o, kCkVersion);
    put1(o, c.m);
    put1(o, c.n);
    put1(o, c.fingerprint);
    for (int32_t v : {c.it, c.mode, c.cg_its_last, c.solves_last, c.cg_failed, c.warm_used,
                      c.direct_its, c.forced_switch_done, c.forced_back_done, c.switched_by_drop,
                      c.switches_back})
        put1(o, v);
    put1(o, c.psi);
    put1(o, c.psi_max);
    put1(o, c.cg_total);
    put1(o, c.tol_int);
    put1(o, c.max_fill);
    put1(o, (int64_t)c.psi_hist.size());
    put(o, c.psi_hist.data(), c.psi_hist.size());
    put(o, c.idx.data(), c.idx.size());
    put(o, c.p.data(), c.p.size());
    put(o, c.s.data(), c.s.size());
    put(o, c.y.data(), c.y.size());
    put(o, c.z.data(), c.z.size());
    return o;
}

struct ByteReader {
    const unsigned char *p;
    size_t left;
    template <class T>
    void get(T *v, size_t count) {
        const size_t len = sizeof(T) * count;
        OTIP_CHECK(len <= left, OTIP_EINVAL, "checkpoint: truncated");
        std::memcpy(v, p, len);
        p += len;
        left -= len;
    }
    template <class T>
    T get1() {
        T v;
        get(&v, 1);
        return v;
    }
};

std::unique_ptr<otip::Checkpoint> deserialize(const void *buf, size_t size) {
    ByteReader r{(const unsigned char *)buf, size};
    char magic[8];
    r.get(magic, 8);
    OTIP_CHECK(std::memcmp(magic, kCkMagic, 8) == 0 && r.get1<uint32_t>() == kCkVersion,
               OTIP_EINVAL, "not a checkpoint of this library version");
    auto c = std::make_unique<otip::Checkpoint>();
    c->m = r.get1<int32_t>();
    c->n = r.get1<int32_t>();
    c->fingerprint = r.get1<uint64_t>();
    for (int32_t *v : {&c->it, &c->mode, &c->cg_its_last, &c->solves_last, &c->cg_failed,
                       &c->warm_used, &c->direct_its, &c->forced_switch_done,
                       &c->forced_back_done, &c->switched_by_drop, &c->switches_back})
        *v = r.get1<int32_t>();
    c->psi = r.get1<int64_t>();
    c->psi_max = r.get1<int64_t>();
    c->cg_total = r.get1<int64_t>();
    c->tol_int = r.get1<double>();
    c->max_fill = r.get1<double>();
    const int64_t nh = r.get1<int64_t>();
    OTIP_CHECK(c->m >= 1 && c->n >= 1 && c->psi >= 1 && nh >= 0, OTIP_EINVAL,
               "checkpoint: bad sizes");
    // every array must fit in what is left (no allocation beyond the input)
    const double need = 8.0 * ((double)nh + 3.0 * (double)c->psi + (double)c->m + (double)c->n);
    OTIP_CHECK(need == (double)r.left, OTIP_EINVAL, "checkpoint: size does not match its header");
    c->psi_hist.resize(nh);
    c->idx.resize(c->psi);
    c->p.resize(c->psi);
    c->s.resize(c->psi);
    c->y.resize(c->m);
    c->z.resize(c->n);
    r.get(c->psi_hist.data(), nh);
    r.get(c->idx.data(), c->psi);
    r.get(c->p.data(), c->psi);
    r.get(c->s.data(), c->psi);
    r.get(c->y.data(), c->m);
    r.get(c->z.data(), c->n);
    return c;
}

}  // namespace

extern "C" {

int otip_version(void) { return OTIP_ABI_VERSION; }

#ifndef OTIP_SOURCE_ID
#define OTIP_SOURCE_ID "unknown"
#endif
const char *otip_source_id(void) { return OTIP_SOURCE_ID; }

void otip_params_default(otip_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->tol = 1e-6;
    p->cg_tol_pred = 1e-6;
    p->cg_tol_corr = 1e-3;
    p->max_iter = 200;
    p->cg_max_iter = 1000;
    p->max_corr = 3;
    p->step_scale = 0.995;
    p->kappa = 5.0;
    p->switch_window = 5;
    p->switch_drop = 0.1;
    p->mcc_beta_min = 0.1;
    p->mcc_beta_max = 10.0;
    p->mcc_delta = 0.1;
    p->mcc_accept = 0.01;
    p->remove_gate = 1e-3;
    p->remove_rel = 1e-6;
    p->pivot_tol = 1e-12;
    p->cert_rel = 1e-7;
    p->polish_tol = 1e-12;
    p->polish_steps = 4;
    p->drop_rel = 1e-7;
    p->cg_eta = 0.1;
    p->cg_floor = 1e-9;
    p->linear_solver = OTIP_LS_AUTO;
    p->precision = OTIP_FP64;
    p->dense_max_n = 65536;
    p->force_switch_at = -1;
    p->enter_cap = 0;
    p->scale = 1;
    p->verbose = 0;
    p->profile = 0;
    p->switch_cost = 1;
    p->batch_workers = 0;
    p->price_tile = 0;
    p->ws_kappa = 0.0;
    p->heur_radius = 0.0;
    p->heur_run = 3;
    p->switch_back_grow = 0.0;
    p->force_switch_back_at = -1;
    p->schur_reuse = 1;
    p->ws_union = 1;
}

int otip_create(otip_ctx **ctx, int device, void *hip_stream) {
    if (!ctx) return OTIP_EINVAL;
    *ctx = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return OTIP_EINVAL;
    auto c = std::make_unique<otip_ctx>();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    // the device address of this GPU's static scratch (otip_kron_apply_noalloc)
    const int rc = guarded(c.get(), [&] { otip::kron_scratch_init(device); });
    if (rc != OTIP_OK) return rc;
    *ctx = c.release();
    return OTIP_OK;
}

void otip_destroy(otip_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    delete ctx;
}

const char *otip_last_error(const otip_ctx *ctx) {
    if (!ctx) return "null context";
    return ctx->err.c_str();
}

int otip_solve(otip_ctx *ctx, const otip_problem *pr, const otip_params *params,
               otip_result **out) {
    if (!ctx || !pr || !out) return OTIP_EINVAL;
    *out = nullptr;
    int status = OTIP_OK;
    auto res = std::make_unique<otip_result>();
    int rc = guarded(ctx, [&] {
        otip_params P;
        if (params)
            P = *params;
        else
            otip_params_default(&P);
        if (!ctx->solver) ctx->solver = std::make_unique<otip::Solver>(ctx->stream);
        status = ctx->solver->run(*pr, P, res->r);
        OTIP_HIP(hipStreamSynchronize(ctx->stream));
    });
    if (rc != OTIP_OK) return rc;
    *out = res.release();
    return status;
}

int otip_solve_batch(otip_ctx *ctx, const otip_problem *prs, int32_t count,
                     const otip_params *params, otip_result **outs) {
    if (!ctx || count < 0 || (count > 0 && (!prs || !outs))) return OTIP_EINVAL;
    for (int32_t k = 0; k < count; ++k) outs[k] = nullptr;
    if (count == 0) return OTIP_OK;
    otip_params P;
    if (params)
        P = *params;
    else
        otip_params_default(&P);
    const int nw = std::max(1, std::min<int>(P.batch_workers > 0 ? P.batch_workers : 8, count));
    int rc = guarded(ctx, [&] {
        OTIP_CHECK(nw <= 64, OTIP_EINVAL, "batch_workers must be <= 64");
        // the caller's stream produced the inputs
        OTIP_HIP(hipStreamSynchronize(ctx->stream));
        while ((int)ctx->workers.size() < nw) {
            auto w = std::make_unique<BatchWorker>();
            OTIP_HIP(hipStreamCreateWithFlags(&w->st, hipStreamNonBlocking));
            w->solver = std::make_unique<otip::Solver>(w->st);
            ctx->workers.push_back(std::move(w));
        }
    });
    if (rc != OTIP_OK) return rc;
    // largest first, so that a worker's buffers grow on its first problems only
    std::vector<int32_t> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t u, int32_t v) {
        return (int64_t)prs[u].m * prs[u].n > (int64_t)prs[v].m * prs[v].n;
    });
    std::atomic<int32_t> next{0};
    std::atomic<bool> abort{false};
    std::vector<int> codes(count, OTIP_OK);
    std::mutex mu;
    int first_code = OTIP_OK;
    std::string first_msg;
    auto fail = [&](int32_t k, int code, const char *msg) {
        std::lock_guard<std::mutex> g(mu);
        if (first_code == OTIP_OK) {
            first_code = code;
            first_msg = "instance " + std::to_string(k) + ": " + msg;
        }
        abort = true;
    };
    auto work = [&](int w) {
        BatchWorker &W = *ctx->workers[w];
        if (hipSetDevice(ctx->device) != hipSuccess) {
            fail(-1, OTIP_EHIP, "hipSetDevice failed in a batch worker");
            return;
        }
        for (;;) {
            if (abort.load()) return;
            const int32_t q = next.fetch_add(1);
            if (q >= count) return;
            const int32_t k = order[q];
            try {
                auto res = std::make_unique<otip_result>();
                codes[k] = W.solver->run(prs[k], P, res->r);
                OTIP_HIP(hipStreamSynchronize(W.st));
                outs[k] = res.release();
            } catch (const otip::Error &e) {
                (void)hipStreamSynchronize(W.st);
                fail(k, e.code, e.what());
            } catch (const std::bad_alloc &) {
                fail(k, OTIP_ENOMEM, "host allocation failed");
            } catch (const std::exception &e) {
                (void)hipStreamSynchronize(W.st);
                fail(k, OTIP_EHIP, e.what());
            }
        }
    };
    std::vector<std::thread> threads;
    threads.reserve(nw - 1);
    try {
        for (int w = 1; w < nw; ++w) threads.emplace_back(work, w);
    } catch (const std::exception &) {
        fail(-1, OTIP_EHIP, "could not start batch worker threads");
    }
    work(0);
    for (auto &t : threads) t.join();
    if (first_code != OTIP_OK) {
        for (int32_t k = 0; k < count; ++k) {
            otip_result_free(outs[k]);
            outs[k] = nullptr;
        }
        ctx->err = first_msg;
        return first_code;
    }
    ctx->err.clear();
    int worst = OTIP_OK;
    for (int32_t k = 0; k < count; ++k) {
        if (codes[k] == OTIP_ENUMERIC) worst = OTIP_ENUMERIC;
        if (codes[k] == OTIP_EMAXITER && worst == OTIP_OK) worst = OTIP_EMAXITER;
    }
    return worst;
}

int otip_result_info(const otip_result *r, otip_info *info) {
    if (!r || !info) return OTIP_EINVAL;
    *info = r->r.info;
    return OTIP_OK;
}

int otip_result_copy(const otip_result *r, int32_t *rows, int32_t *cols, double *vals, double *y,
                     double *z) {
    if (!r) return OTIP_EINVAL;
    const auto &R = r->r;
    if (rows) std::memcpy(rows, R.rows.data(), R.rows.size() * sizeof(int32_t));
    if (cols) std::memcpy(cols, R.cols.data(), R.cols.size() * sizeof(int32_t));
    if (vals) std::memcpy(vals, R.vals.data(), R.vals.size() * sizeof(double));
    if (y) std::memcpy(y, R.y.data(), R.y.size() * sizeof(double));
    if (z) std::memcpy(z, R.z.data(), R.z.size() * sizeof(double));
    return OTIP_OK;
}

void otip_result_free(otip_result *r) { delete r; }

int otip_price(otip_ctx *ctx, int32_t m, int32_t n, const int32_t *xs, const int32_t *xt,
               const double *y, const double *z, const uint32_t *support_bitmap, int64_t kmax,
               int32_t precision, int32_t tile, int32_t cost_kind, int32_t *out_i,
               int32_t *out_j, double *out_r, int64_t *out_count, int64_t *out_nneg) {
    return guarded(ctx, [&] {
        ctx->scan.tile = tile;
        OTIP_CHECK(m >= 1 && n >= 1 && xs && xt && y && z && kmax >= 0, OTIP_EINVAL,
                   "otip_price: bad arguments");
        OTIP_CHECK(cost_kind >= OTIP_COST_SQEUCLID && cost_kind <= OTIP_COST_LINF, OTIP_EINVAL,
                   "otip_price: unknown cost kind");
        ctx->scan.kind = cost_kind;
        OTIP_CHECK(kmax == 0 || (out_i && out_j && out_r), OTIP_EINVAL,
                   "otip_price: null outputs");
        otip::PriceResult pr;
        if (precision == OTIP_MIXED)
            pr = ctx->scan.price_mixed(ctx->stream, m, n, xs, xt, y, z, support_bitmap, kmax,
                                       out_i, out_j, out_r, nullptr);
        else
            pr = ctx->scan.price(ctx->stream, m, n, xs, xt, y, z, support_bitmap, kmax, out_i,
                                 out_j, out_r, nullptr);
        OTIP_HIP(hipStreamSynchronize(ctx->stream));
        if (out_count) *out_count = pr.count;
        if (out_nneg) *out_nneg = pr.nneg;
    });
}

int otip_price_subset(otip_ctx *ctx, int32_t m, int32_t n, const int32_t *xs, const int32_t *xt,
                      const double *y, const double *z, const uint32_t *support_bitmap,
                      int64_t kmax, int32_t cost_kind, int64_t key_limit, int32_t *out_i,
                      int32_t *out_j, double *out_r, int64_t *out_count, int64_t *out_nneg,
                      int64_t *out_subset_size) {
    return guarded(ctx, [&] {
        OTIP_CHECK(m >= 1 && n >= 1 && xs && xt && y && z && kmax >= 0 && key_limit >= 1,
                   OTIP_EINVAL, "otip_price_subset: bad arguments");
        OTIP_CHECK(cost_kind >= OTIP_COST_SQEUCLID && cost_kind <= OTIP_COST_LINF, OTIP_EINVAL,
                   "otip_price_subset: unknown cost kind");
        OTIP_CHECK(kmax == 0 || (out_i && out_j && out_r), OTIP_EINVAL,
                   "otip_price_subset: null outputs");
        ctx->scan.tile = 0;
        ctx->scan.kind = cost_kind;
        const int64_t size = ctx->scan.set_subset(ctx->stream, m, n, xs, xt, key_limit);
        otip::PriceResult pr{0, 0, 0};
        if (size > 0) {
            ctx->scan.use_subset = true;
            try {
                pr = ctx->scan.price(ctx->stream, m, n, xs, xt, y, z, support_bitmap, kmax, out_i,
                                     out_j, out_r, nullptr);
            } catch (...) {
                ctx->scan.use_subset = false;
                throw;
            }
            ctx->scan.use_subset = false;
        }
        OTIP_HIP(hipStreamSynchronize(ctx->stream));
        if (out_count) *out_count = pr.count;
        if (out_nneg) *out_nneg = pr.nneg;
        if (out_subset_size) *out_subset_size = size;
    });
}

int otip_rmin(otip_ctx *ctx, int32_t m, int32_t n, const int32_t *xs, const int32_t *xt,
              const double *y, const double *z, int32_t cost_kind, double *out_rmin,
              int64_t *out_arg) {
    return guarded(ctx, [&] {
        OTIP_CHECK(m >= 1 && n >= 1 && xs && xt && y && z && out_rmin, OTIP_EINVAL,
                   "otip_rmin: bad arguments");
        OTIP_CHECK(cost_kind >= OTIP_COST_SQEUCLID && cost_kind <= OTIP_COST_LINF, OTIP_EINVAL,
                   "otip_rmin: unknown cost kind");
        ctx->scan.kind = cost_kind;
        ctx->scan.rmin(ctx->stream, m, n, xs, xt, y, z, out_rmin, out_arg);
    });
}

int otip_kron_apply(otip_ctx *ctx, int32_t m, int32_t n, const double *X, double *rowsum,
                    double *colsum) {
    return guarded(ctx, [&] {
        OTIP_CHECK(m >= 1 && n >= 1 && X && rowsum && colsum, OTIP_EINVAL,
                   "otip_kron_apply: bad arguments");
        otip::kron_apply(ctx->stream, m, n, X, rowsum, colsum, ctx->buf_a, ctx->buf_b);
        OTIP_HIP(hipStreamSynchronize(ctx->stream));
    });
}

int otip_kron_apply_noalloc(otip_ctx *ctx, int32_t m, int32_t n, const double *X,
                            double *rowsum, double *colsum) {
    return guarded(ctx, [&] {
        OTIP_CHECK(m >= 1 && n >= 1 && X && rowsum && colsum, OTIP_EINVAL,
                   "otip_kron_apply_noalloc: bad arguments");
        otip::kron_apply_noalloc(ctx->stream, ctx->device, m, n, X, rowsum, colsum);
        OTIP_HIP(hipStreamSynchronize(ctx->stream));
    });
}

int otip_kron_apply_t(otip_ctx *ctx, int32_t m, int32_t n, const double *y, const double *z,
                      double *X) {
    return guarded(ctx, [&] {
        OTIP_CHECK(m >= 1 && n >= 1 && X && y && z, OTIP_EINVAL,
                   "otip_kron_apply_t: bad arguments");
        otip::kron_apply_t(ctx->stream, m, n, y, z, X);
        OTIP_HIP(hipStreamSynchronize(ctx->stream));
    });
}

int otip_schur(otip_ctx *ctx, int32_t m, int32_t n, int64_t psi, const int64_t *idx,
               const double *theta, int64_t *out_nnz, int32_t *rowptr, int32_t *colidx,
               double *vals, double *M, double *N) {
    return guarded(ctx, [&] {
        OTIP_CHECK(m >= 1 && n >= 1 && psi >= 1 && idx && theta && out_nnz, OTIP_EINVAL,
                   "otip_schur: bad arguments");
        OTIP_CHECK(!rowptr || (colidx && vals), OTIP_EINVAL, "otip_schur: null outputs");
        otip::Solver s(ctx->stream);
        *out_nnz = s.schur_export(m, n, psi, (const uint64_t *)idx, theta, rowptr, colidx, vals,
                                  M, N);
    });
}

int otip_pcg(otip_ctx *ctx, int32_t n, int64_t nnz, const int32_t *rowptr, const int32_t *colidx,
             const double *vals, const double *b, double *x, double rtol, int32_t maxit,
             int32_t precision, int32_t *iterations, double *res_norm, double *spmv_stats) {
    otip::CGStats cs;
    int rc = guarded(ctx, [&] {
        OTIP_CHECK(n >= 1 && nnz >= 0 && nnz <= 0x7fffffff && rowptr && b && x &&
                       (nnz == 0 || (colidx && vals)) && rtol > 0.0 && maxit >= 1 &&
                       (precision == OTIP_FP64 || precision == OTIP_MIXED),
                   OTIP_EINVAL, "otip_pcg: bad arguments");
        otip::SchurSolver s;
        otip::LaunchTimer t;
        t.on = spmv_stats != nullptr;
        s.timer = &t;
        s.load_csr(ctx->stream, n, nnz, rowptr, colidx, vals);
        cs = precision == OTIP_MIXED ? s.pcg_mixed(ctx->stream, b, x, rtol, INFINITY, maxit)
                                     : s.pcg(ctx->stream, b, x, rtol, INFINITY, maxit);
        OTIP_HIP(hipStreamSynchronize(ctx->stream));
        if (iterations) *iterations = cs.iterations;
        if (res_norm) *res_norm = cs.res_norm;
        if (spmv_stats) {
            const double w = precision == OTIP_MIXED ? 4.0 : 8.0;
            spmv_stats[0] = (double)t.launches;
            spmv_stats[1] = t.launches ? t.ms * 1e-3 / (double)t.launches : 0.0;
            spmv_stats[2] = otip::cg_launch_bytes(w, nnz, n);
        }
    });
    if (rc != OTIP_OK) return rc;
    if (cs.converged) return OTIP_OK;
    return cs.iterations >= maxit ? OTIP_EMAXITER : OTIP_ENUMERIC;
}

int otip_ldl_solve(otip_ctx *ctx, int32_t n, int64_t nnz, const int32_t *rowptr,
                   const int32_t *colidx, const double *vals, double pivot_tol, int32_t flags,
                   const double *b, double *x, int32_t *out_ninf, int64_t *out_nnz_L) {
    return guarded(ctx, [&] {
        OTIP_CHECK(n >= 1 && nnz >= 1 && nnz <= 0x7fffffff && rowptr && colidx && vals && b && x &&
                       pivot_tol >= 0.0 && (flags & ~1) == 0,
                   OTIP_EINVAL, "otip_ldl_solve: bad arguments");
        otip::SchurSolver s;
        s.load_csr(ctx->stream, n, nnz, rowptr, colidx, vals);
        otip::DenseLDL ldl;
        ldl.force_substitution = (flags & 1) != 0;
        const int ninf = ldl.factor(ctx->stream, s.S, pivot_tol);
        ldl.solve(ctx->stream, b, x);
        OTIP_HIP(hipStreamSynchronize(ctx->stream));
        if (out_ninf) *out_ninf = ninf;
        if (out_nnz_L) *out_nnz_L = ldl.nnz_L();
    });
}

int otip_state_save(otip_ctx *ctx, void *buf, int64_t cap, int64_t *size) {
    return guarded(ctx, [&] {
        OTIP_CHECK(size, OTIP_EINVAL, "otip_state_save: null size");
        const otip::Checkpoint *c = ctx->solver ? ctx->solver->last_state() : nullptr;
        OTIP_CHECK(c, OTIP_EINVAL, "otip_state_save: no solve on this context yet");
        const std::vector<unsigned char> bytes = serialize(*c);
        *size = (int64_t)bytes.size();
        if (buf) {
            OTIP_CHECK(cap >= (int64_t)bytes.size(), OTIP_EINVAL, "otip_state_save: buffer too small");
            std::memcpy(buf, bytes.data(), bytes.size());
        }
    });
}

int otip_state_load(otip_ctx *ctx, const void *buf, int64_t size) {
    return guarded(ctx, [&] {
        OTIP_CHECK(buf && size > 0, OTIP_EINVAL, "otip_state_load: bad arguments");
        std::unique_ptr<otip::Checkpoint> c = deserialize(buf, (size_t)size);
        if (!ctx->solver) ctx->solver = std::make_unique<otip::Solver>(ctx->stream);
        ctx->solver->set_resume(std::move(c));
    });
}

int64_t otip_ws_param_count(void) { return otip::WarmNet::param_count(); }

int otip_ws_forward(otip_ctx *ctx, const float *weights, int32_t batch, int32_t h, int32_t w,
                    const float *in, float *out) {
    return guarded(ctx, [&] {
        OTIP_CHECK(weights && in && out && batch >= 1 && batch <= 65535 && h >= 1 && w >= 1 &&
                       (int64_t)h * w <= (1 << 24),
                   OTIP_EINVAL, "otip_ws_forward: bad arguments");
        ctx->net.forward(ctx->stream, weights, batch, h, w, in, out);
        OTIP_HIP(hipStreamSynchronize(ctx->stream));
    });
}

int otip_ws_grad(otip_ctx *ctx, const float *weights, int32_t batch, int32_t h, int32_t w,
                 const float *in, const float *target, float *grad, double *loss) {
    return guarded(ctx, [&] {
        OTIP_CHECK(weights && in && target && grad && batch >= 1 && batch <= 65535 && h >= 1 &&
                       w >= 1 && (int64_t)h * w <= (1 << 24),
                   OTIP_EINVAL, "otip_ws_grad: bad arguments");
        const double l = ctx->net.grad(ctx->stream, weights, batch, h, w, in, target, grad);
        if (loss) *loss = l;
    });
}

int otip_ws_adam(otip_ctx *ctx, float *weights, float *m, float *v, const float *grad,
                 int32_t step, double lr, double beta1, double beta2, double eps) {
    return guarded(ctx, [&] {
        OTIP_CHECK(weights && m && v && grad && step >= 1 && beta1 >= 0.0 && beta1 < 1.0 &&
                       beta2 >= 0.0 && beta2 < 1.0 && eps >= 0.0,
                   OTIP_EINVAL, "otip_ws_adam: bad arguments");
        ctx->net.adam(ctx->stream, weights, m, v, grad, step, lr, beta1, beta2, eps);
        OTIP_HIP(hipStreamSynchronize(ctx->stream));
    });
}

int otip_ws_predict(otip_ctx *ctx, const float *weights, int32_t side, const double *a,
                    const double *b, double *y0, double *z0) {
    return guarded(ctx, [&] {
        OTIP_CHECK(weights && a && b && y0 && z0 && side >= 1 && side <= 32768, OTIP_EINVAL,
                   "otip_ws_predict: bad arguments");
        ctx->net.predict(ctx->stream, weights, side, a, b, y0, z0);
        OTIP_HIP(hipStreamSynchronize(ctx->stream));
    });
}

}  // extern "C"
