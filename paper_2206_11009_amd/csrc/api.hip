// C-ABI entry points (include/otip.h).  Every call catches the library's
// exceptions and returns a status code; the message is kept on the context.
#include <cstring>
#include <memory>

#include "driver.h"

struct otip_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    otip::Scanner scan;
    otip::SchurSolver schur;
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

}  // namespace

extern "C" {

int otip_version(void) { return OTIP_ABI_VERSION; }

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
    p->dense_max_n = 16384;
    p->force_switch_at = -1;
    p->enter_cap = 0;
    p->scale = 1;
    p->verbose = 0;
    p->profile = 0;
    p->switch_cost = 1;
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
        otip::Solver s(ctx->stream);
        status = s.run(*pr, P, res->r);
        OTIP_HIP(hipStreamSynchronize(ctx->stream));
    });
    if (rc != OTIP_OK) return rc;
    *out = res.release();
    return status;
}

int otip_solve_batch(otip_ctx *ctx, const otip_problem *prs, int32_t count,
                     const otip_params *params, otip_result **outs) {
    if (!ctx || !prs || !outs || count < 0) return OTIP_EINVAL;
    int worst = OTIP_OK;
    for (int32_t k = 0; k < count; ++k) {
        int rc = otip_solve(ctx, &prs[k], params, &outs[k]);
        if (rc != OTIP_OK && rc != OTIP_EMAXITER) {
            for (int32_t q = 0; q < k; ++q) {
                otip_result_free(outs[q]);
                outs[q] = nullptr;
            }
            return rc;
        }
        if (rc == OTIP_EMAXITER) worst = rc;
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
               int32_t precision, int32_t *out_i, int32_t *out_j, double *out_r,
               int64_t *out_count, int64_t *out_nneg) {
    return guarded(ctx, [&] {
        OTIP_CHECK(m >= 1 && n >= 1 && xs && xt && y && z && kmax >= 0, OTIP_EINVAL,
                   "otip_price: bad arguments");
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

int otip_rmin(otip_ctx *ctx, int32_t m, int32_t n, const int32_t *xs, const int32_t *xt,
              const double *y, const double *z, double *out_rmin, int64_t *out_arg) {
    return guarded(ctx, [&] {
        OTIP_CHECK(m >= 1 && n >= 1 && xs && xt && y && z && out_rmin, OTIP_EINVAL,
                   "otip_rmin: bad arguments");
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

}  // extern "C"
