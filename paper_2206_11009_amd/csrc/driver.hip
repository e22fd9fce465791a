// The method's outer loop (Sections 3.1-3.4, 4.2-4.3) on one GPU.
//
// Device state: the support ("index", Section 3.2) as variable indices sorted
// ascending -- i.e. grouped by target j, a compressed-column view of the plan --
// with p, s, costs and (i, j); a compressed-row view through a permutation; a
// bit per variable for the pricing scan; the duals y (m) and z (n).  All
// per-element work runs in the kernels below and in scan/schur/dense; the host
// only takes the scalar decisions (stop test, step lengths, corrector
// acceptance, switch), each after one small device-to-host copy.
#include <chrono>
#include <cstring>

#include "driver.h"

namespace otip {

// ============================================================== reductions
template <int K, class F>
__global__ __launch_bounds__(Reducer::kThreads) void rsum_k(int64_t N, F f, double *part) {
    __shared__ double lds[16];
    double acc[K];
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N;
         t += (int64_t)gridDim.x * blockDim.x)
        f(t, acc);
#pragma unroll
    for (int q = 0; q < K; ++q) {
        double v = block_sum(acc[q], lds);
        if (threadIdx.x == 0) part[q * Reducer::kBlocks + blockIdx.x] = v;
    }
}

template <int K, class F>
__global__ __launch_bounds__(Reducer::kThreads) void rmin_k(int64_t N, F f, double *part) {
    __shared__ double lds[16];
    double acc[K];
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] = INFINITY;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N;
         t += (int64_t)gridDim.x * blockDim.x)
        f(t, acc);
#pragma unroll
    for (int q = 0; q < K; ++q) {
        double v = wave_min(acc[q]);
        __syncthreads();
        if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            double b = lds[0];
            for (int w = 1; w < (int)(blockDim.x >> 6); ++w) b = fmin(b, lds[w]);
            part[q * Reducer::kBlocks + blockIdx.x] = b;
        }
    }
}

void Reducer::fetch_sum(hipStream_t st, int K, int nb, double *out) {
    host_.resize((size_t)K * kBlocks);
    OTIP_HIP(hipMemcpyAsync(host_.data(), part_.get(), sizeof(double) * K * kBlocks,
                            hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipStreamSynchronize(st));
    for (int q = 0; q < K; ++q) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += host_[(size_t)q * kBlocks + b];
        out[q] = s;
    }
}

void Reducer::fetch_min(hipStream_t st, int K, int nb, double *out) {
    host_.resize((size_t)K * kBlocks);
    OTIP_HIP(hipMemcpyAsync(host_.data(), part_.get(), sizeof(double) * K * kBlocks,
                            hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipStreamSynchronize(st));
    for (int q = 0; q < K; ++q) {
        double s = INFINITY;
        for (int b = 0; b < nb; ++b) s = std::min(s, host_[(size_t)q * kBlocks + b]);
        out[q] = s;
    }
}

static int red_blocks(int64_t N) {
    return (int)std::min<int64_t>(Reducer::kBlocks, std::max<int64_t>(1, (N + 255) / 256));
}

template <int K, class F>
static void reduce_sum(hipStream_t st, Reducer &R, int64_t N, F f, double *out) {
    const int nb = red_blocks(N);
    hipLaunchKernelGGL((rsum_k<K, F>), dim3(nb), dim3(Reducer::kThreads), 0, st, N, f, R.base());
    OTIP_HIP(hipGetLastError());
    R.fetch_sum(st, K, nb, out);
}

template <int K, class F>
static void reduce_min(hipStream_t st, Reducer &R, int64_t N, F f, double *out) {
    const int nb = red_blocks(N);
    hipLaunchKernelGGL((rmin_k<K, F>), dim3(nb), dim3(Reducer::kThreads), 0, st, N, f, R.base());
    OTIP_HIP(hipGetLastError());
    R.fetch_min(st, K, nb, out);
}

// launch an element-wise functor over [0, N)
template <class F>
__global__ void foreach_k(int64_t N, F f) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N;
         t += (int64_t)gridDim.x * blockDim.x)
        f(t);
}
template <class F>
static void foreach(hipStream_t st, int64_t N, F f) {
    if (N <= 0) return;
    const unsigned g = (unsigned)std::min<int64_t>(4096, (N + 255) / 256);
    hipLaunchKernelGGL((foreach_k<F>), dim3(g), dim3(256), 0, st, N, f);
    OTIP_HIP(hipGetLastError());
}

// =============================================================== support views
// C_ij of a cost kind (Section 5.1) from the integer offset d = x_i - x_j
// (|d| <= 2^15: every integer here is an exact double; the 2-norm is the
// correctly rounded square root of the exact d0^2 + d1^2)
__host__ __device__ inline double pair_cost(const int32_t *xs, const int32_t *xt, int i, int j,
                                            int kind) {
    const int64_t d0 = (int64_t)xs[2 * i] - xt[2 * j], d1 = (int64_t)xs[2 * i + 1] - xt[2 * j + 1];
    const int64_t a0 = d0 < 0 ? -d0 : d0, a1 = d1 < 0 ? -d1 : d1;
    if (kind == OTIP_COST_L1) return (double)(a0 + a1);
    if (kind == OTIP_COST_LINF) return (double)(a0 > a1 ? a0 : a1);
    const double q = (double)(d0 * d0 + d1 * d1);
    return kind == OTIP_COST_L2 ? std::sqrt(q) : q;
}

// idx sorted ascending -> (i, j), scaled costs
struct FDerive {
    const uint64_t *idx;
    int32_t *si, *sj;
    double *c;
    const int32_t *xs, *xt;
    int m, kind;
    double zeta;
    __device__ void operator()(int64_t k) const {
        const uint64_t v = idx[k];
        const int i = (int)(v % (uint64_t)m), j = (int)(v / (uint64_t)m);
        si[k] = i;
        sj[k] = j;
        c[k] = pair_cost(xs, xt, i, j, kind) * zeta;
    }
};

// ptr[t] = first position whose key >= t (keys sorted ascending)
struct FLowerBound {
    const int32_t *key;
    int64_t len;
    int32_t *ptr;
    __device__ void operator()(int64_t t) const {
        int64_t lo = 0, hi = len;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (key[mid] < (int32_t)t)
                lo = mid + 1;
            else
                hi = mid;
        }
        ptr[t] = (int32_t)lo;
    }
};

struct FIota {
    int32_t *v;
    __device__ void operator()(int64_t t) const { v[t] = (int32_t)t; }
};

struct FBits {
    const uint64_t *idx;
    uint32_t *bm;
    bool set;
    __device__ void operator()(int64_t k) const {
        const uint64_t v = idx[k];
        if (v == ~0ull) return;
        if (set)
            atomicOr(&bm[v >> 5], 1u << (v & 31u));
        else
            atomicAnd(&bm[v >> 5], ~(1u << (v & 31u)));
    }
};

void Solver::rebuild_views() {
    const int64_t psi = psi_;
    foreach(st, psi, FDerive{idx.get(), si.get(), sj.get(), c.get(), xs, xt, m, kind, zeta});
    col_ptr.need((size_t)n + 1);
    foreach(st, (int64_t)n + 1, FLowerBound{sj.get(), psi, col_ptr.get()});
    // compressed-row view: stable sort of positions by source
    tmp_i32a.need(psi);
    tmp_u32a.need(psi);
    foreach(st, psi, FIota{tmp_i32a.get()});
    csr_pos.need(psi);
    int bits = 1;
    while ((1ll << bits) < m) ++bits;
    sort_pairs_u32_i32(st, (const uint32_t *)si.get(), tmp_i32a.get(), tmp_u32a.get(),
                       csr_pos.get(), psi, bits, tmp);
    row_ptr.need((size_t)m + 1);
    foreach(st, (int64_t)m + 1, FLowerBound{(const int32_t *)tmp_u32a.get(), psi, row_ptr.get()});
    schur_valid = false;
}

void Solver::alloc_support(int64_t cap) {
    idx.need(cap);
    si.need(cap);
    sj.need(cap);
    p.need(cap);
    s.need(cap);
    c.need(cap);
    theta.need(cap);
    r2.need(cap);
    r3.need(cap);
    w.need(cap);
    for (auto *d : {&D[0], &D[1], &D[2]}) {
        d->dp.need(cap);
        d->ds.need(cap);
        d->dy.need(m);
        d->dz.need(n);
    }
    prot.need(cap);
}

// ============================================================ segmented sums
// G lanes per segment (row of the compressed-row view or column of the
// compressed-column view), fixed-order shuffle reduction: deterministic.
template <int G, class F>
__global__ __launch_bounds__(256) void segsum_k(int64_t rows, F f) {
    constexpr int groups = 256 / G;
    const int g = threadIdx.x / G, l = threadIdx.x % G;
    for (int64_t r = (int64_t)blockIdx.x * groups + g; r < rows;
         r += (int64_t)gridDim.x * groups) {
        const int b = f.begin(r), e = f.end(r);
        double acc = 0.0;
        for (int k = b + l; k < e; k += G) acc += f.val(r, k);
        for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
        if (l == 0) f.finish(r, acc);
    }
}
// lanes per segment: the segments are short (tens of entries) and their
// entries are reached through dependent gathers, so more lanes per segment
// put more of them in flight at once
constexpr int kSegLanes = 32;
template <class F>
static void segsum(hipStream_t st, int64_t rows, F f) {
    if (rows <= 0) return;
    constexpr int per_block = 256 / kSegLanes;
    const unsigned g = (unsigned)std::min<int64_t>(4096, (rows + per_block - 1) / per_block);
    hipLaunchKernelGGL((segsum_k<kSegLanes, F>), dim3(g), dim3(256), 0, st, rows, f);
    OTIP_HIP(hipGetLastError());
}

// out[i] = base[i] + sign * sum over row i of v (compressed-row view)
struct FRowSum {
    const int32_t *row_ptr, *csr_pos;
    const double *v, *base;
    double *out;
    double sign;
    __device__ int begin(int64_t i) const { return row_ptr[i]; }
    __device__ int end(int64_t i) const { return row_ptr[i + 1]; }
    __device__ double val(int64_t, int k) const { return v[csr_pos[k]]; }
    __device__ void finish(int64_t i, double s) const { out[i] = (base ? base[i] : 0.0) + sign * s; }
};
struct FColSum {
    const int32_t *col_ptr;
    const double *v, *base;
    double *out;
    double sign;
    __device__ int begin(int64_t j) const { return col_ptr[j]; }
    __device__ int end(int64_t j) const { return col_ptr[j + 1]; }
    __device__ double val(int64_t, int k) const { return v[k]; }
    __device__ void finish(int64_t j, double s) const { out[j] = (base ? base[j] : 0.0) + sign * s; }
};

void Solver::rowsum(const double *v, const double *base, double *out, double sign) {
    segsum(st, m, FRowSum{row_ptr.get(), csr_pos.get(), v, base, out, sign});
}
void Solver::colsum(const double *v, const double *base, double *out, double sign) {
    segsum(st, n, FColSum{col_ptr.get(), v, base, out, sign});
}

// ============================================================ Newton pieces
struct FTheta {
    const double *p, *s;
    double *th;
    __device__ void operator()(int64_t k) const { th[k] = p[k] / s[k]; }
};
struct FInv {
    const double *v;
    double *o;
    __device__ void operator()(int64_t k) const { o[k] = 1.0 / v[k]; }
};
// w = theta (r2 - r3 / p)
struct FW {
    const double *th, *r2, *r3, *p;
    double *w;
    __device__ void operator()(int64_t k) const {
        // r3 null: zero (the projection of the final polish, where p may be 0)
        w[k] = th[k] * ((r2 ? r2[k] : 0.0) - (r3 ? r3[k] / p[k] : 0.0));
    }
};
// rhs_j = beta2_j - sum_{i in col j} theta_ij beta1_i / M_i
struct FRhs {
    const int32_t *col_ptr, *si;
    const double *th, *beta1, *invM, *beta2;
    double *rhs;
    __device__ int begin(int64_t j) const { return col_ptr[j]; }
    __device__ int end(int64_t j) const { return col_ptr[j + 1]; }
    __device__ double val(int64_t, int e) const { return th[e] * (beta1[si[e]] * invM[si[e]]); }
    __device__ void finish(int64_t j, double s) const { rhs[j] = beta2[j] - s; }
};
// dy_i = (beta1_i - sum_{j in row i} theta_ij dz_j) / M_i
struct FDy {
    const int32_t *row_ptr, *csr_pos, *sj;
    const double *th, *beta1, *invM, *dz;
    double *dy;
    __device__ int begin(int64_t i) const { return row_ptr[i]; }
    __device__ int end(int64_t i) const { return row_ptr[i + 1]; }
    __device__ double val(int64_t, int e) const {
        const int k = csr_pos[e];
        return th[k] * dz[sj[k]];
    }
    __device__ void finish(int64_t i, double s) const { dy[i] = (beta1[i] - s) * invM[i]; }
};
// ds = r2 - (dy_i + dz_j); dp = (r3 - p ds) / s
struct FDsDp {
    const int32_t *si, *sj;
    const double *r2, *r3, *p, *s, *dy, *dz, *th;
    double *ds, *dp;
    __device__ void operator()(int64_t k) const {
        const double d = (r2 ? r2[k] : 0.0) - (dy[si[k]] + dz[sj[k]]);
        ds[k] = d;
        // r3 null: dp = -Theta ds with the assembled Theta
        dp[k] = r3 ? (r3[k] - p[k] * d) / s[k] : -th[k] * d;
    }
};
struct FSub {
    double *v;
    double c;
    __device__ void operator()(int64_t k) const { v[k] -= c; }
};

void Solver::newton(const double *r1a_, const double *r1b_, const double *r2_, const double *r3_,
                    double rtol, double atol, Dir &out) {
    foreach(st, psi_, FW{theta.get(), r2_, r3_, p.get(), w.get()});
    rowsum(w.get(), r1a_, beta1.get(), 1.0);
    colsum(w.get(), r1b_, beta2.get(), 1.0);
    segsum(st, n, FRhs{col_ptr.get(), si.get(), theta.get(), beta1.get(), invM.get(),
                       beta2.get(), rhs.get()});
    bool use_cg = mode != Mode::Direct;
    if (!use_cg) {
        ldl.solve(st, rhs.get(), out.dz.get());
        // one step of iterative refinement against S
        schur.spmv(st, out.dz.get(), tmpn.get());
        double *res = tmpn2.need(n);
        double *rhsp = rhs.get();
        double *tn = tmpn.get();
        foreach(st, n, [=] __device__(int64_t j) { res[j] = rhsp[j] - tn[j]; });
        ldl.solve(st, res, tmpn.get());
        double *dz = out.dz.get();
        foreach(st, n, [=] __device__(int64_t j) { dz[j] += tn[j]; });
        // a factorisation of a nearly singular S can lose all accuracy (huge
        // multipliers); CG on the same system degrades gracefully instead
        double bad = 0.0;
        reduce_sum<1>(st, red, n,
                      [=] __device__(int64_t j, double *acc) { acc[0] += isfinite(dz[j]) ? 0.0 : 1.0; },
                      &bad);
        if (bad != 0.0) {
            log("otip: direct solve not finite; this solve by CG\n");
            use_cg = true;
        }
    }
    if (use_cg) {
        // project on the range of S (orthogonal to e: the null vector of a
        // connected support, Section 4)
        double mean = 0.0;
        const double *rp = rhs.get();
        reduce_sum<1>(st, red, n, [=] __device__(int64_t j, double *acc) { acc[0] += rp[j]; },
                      &mean);
        foreach(st, n, FSub{rhs.get(), mean / n});
        t_spmv.begin_call();
        CGStats cs = (P.precision == OTIP_MIXED)
                         ? schur.pcg_mixed(st, rhs.get(), out.dz.get(), rtol, atol, P.cg_max_iter)
                         : schur.pcg(st, rhs.get(), out.dz.get(), rtol, atol, P.cg_max_iter);
        cg_its_iter += cs.iterations;
        max_cg_solve = std::max(max_cg_solve, cs.iterations);
        if (!cs.converged) cg_failed = true;
    }
    segsum(st, m, FDy{row_ptr.get(), csr_pos.get(), sj.get(), theta.get(), beta1.get(),
                      invM.get(), out.dz.get(), out.dy.get()});
    foreach(st, psi_, FDsDp{si.get(), sj.get(), r2_, r3_, p.get(), s.get(), out.dy.get(),
                            out.dz.get(), theta.get(), out.ds.get(), out.dp.get()});
}

// max step to the boundary for p and s
void Solver::max_steps(const Dir &d, double &ap, double &ad) {
    const double *pp = p.get(), *ss = s.get(), *dp = d.dp.get(), *ds = d.ds.get();
    double r[2];
    reduce_min<2>(st, red, psi_,
                  [=] __device__(int64_t k, double *acc) {
                      if (dp[k] < 0.0) acc[0] = fmin(acc[0], -pp[k] / dp[k]);
                      if (ds[k] < 0.0) acc[1] = fmin(acc[1], -ss[k] / ds[k]);
                  },
                  r);
    ap = r[0];
    ad = r[1];
}

void Solver::assemble() {
    foreach(st, psi_, FTheta{p.get(), s.get(), theta.get()});
    rowsum(theta.get(), nullptr, M.get(), 1.0);
    colsum(theta.get(), nullptr, N.get(), 1.0);
    foreach(st, m, FInv{M.get(), invM.get()});
    if (!schur_valid) {
        schur.symbolic(st, m, n, psi_, col_ptr.get(), si.get(), row_ptr.get(), csr_pos.get(),
                       sj.get());
        schur_valid = true;
    }
    schur.numeric(st, m, n, col_ptr.get(), si.get(), row_ptr.get(), csr_pos.get(), sj.get(),
                  theta.get(), invM.get());
}

// ============================================================ scaffolding
double Solver::now() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

static bool trace_on() {
    static const bool on = std::getenv("OTIP_TRACE") != nullptr;
    return on;
}

void Solver::trace(const char *tag, int it, const void *dev, size_t bytes) {
    if (!trace_on()) return;
    std::vector<unsigned char> h(bytes);
    if (bytes) {
        OTIP_HIP(hipMemcpyAsync(h.data(), dev, bytes, hipMemcpyDeviceToHost, st));
        OTIP_HIP(hipStreamSynchronize(st));
    }
    uint64_t f = 14695981039346656037ull;
    for (unsigned char c : h) f = (f ^ c) * 1099511628211ull;
    fprintf(stderr, "TRACE %016llx %d %s %016llx %zu\n", (unsigned long long)fp_, it, tag,
            (unsigned long long)f, bytes);
}

void Solver::trace_val(const char *tag, int it, double v) {
    if (!trace_on()) return;
    fprintf(stderr, "TRACE %016llx %d %s %a\n", (unsigned long long)fp_, it, tag, v);
}

void Solver::log(const char *fmt, ...) {
    if (!P.verbose) return;
    va_list ap;
    va_start(ap, fmt);
    vfprintf(stderr, fmt, ap);
    va_end(ap);
}

// ------------------------------------------------------------------ residuals
void Solver::residuals(double &rel1, double &rel2, double &mu, double &primal, double &r1n) {
    rowsum(p.get(), a.get(), r1a.get(), -1.0);
    colsum(p.get(), b.get(), r1b.get(), -1.0);
    const double *cc = c.get(), *pp = p.get(), *ss = s.get(), *yy = y.get(), *zz = z.get();
    const int32_t *ii = si.get(), *jj = sj.get();
    double *rr2 = r2.get();
    double v[4];
    reduce_sum<4>(st, red, psi_,
                  [=] __device__(int64_t k, double *acc) {
                      const double r = cc[k] - (yy[ii[k]] + zz[jj[k]]) - ss[k];
                      rr2[k] = r;
                      acc[0] = fma(r, r, acc[0]);
                      acc[1] = fma(cc[k], cc[k], acc[1]);
                      acc[2] = fma(pp[k], ss[k], acc[2]);
                      acc[3] = fma(cc[k], pp[k], acc[3]);
                  },
                  v);
    const double *ra = r1a.get(), *rb = r1b.get();
    const int mm = m;
    double q;
    reduce_sum<1>(st, red, (int64_t)m + n,
                  [=] __device__(int64_t t, double *acc) {
                      const double r = t < mm ? ra[t] : rb[t - mm];
                      acc[0] = fma(r, r, acc[0]);
                  },
                  &q);
    r1n = std::sqrt(q);
    rel1 = r1n / (1.0 + fnorm);
    rel2 = std::sqrt(v[0]) / (1.0 + std::sqrt(v[1]));
    mu = v[2] / (double)psi_;
    primal = v[3];
}

// ------------------------------------------------------------------ pricing
int64_t Solver::price(int64_t kmax, uint64_t *out_idx, double *out_r, int64_t *nneg,
                      bool heuristic) {
    double t0 = now();
    // pricing runs on the unscaled costs: duals divided by the power-of-two cost scale
    double *yu = yun.need(m), *zu = zun.need(n);
    const double *yy = y.get(), *zz = z.get();
    const double iz = 1.0 / zeta;
    foreach(st, m, [=] __device__(int64_t i) { yu[i] = yy[i] * iz; });
    foreach(st, n, [=] __device__(int64_t j) { zu[j] = zz[j] * iz; });
    PriceResult pr;
    t_price.begin_call();
    scan.use_subset = heuristic && heur_on;
    if (P.precision == OTIP_MIXED)
        pr = scan.price_mixed(st, m, n, xs, xt, yu, zu, bitmap.get(), kmax, nullptr, nullptr,
                              out_r, out_idx);
    else
        pr = scan.price(st, m, n, xs, xt, yu, zu, bitmap.get(), kmax, nullptr, nullptr, out_r,
                        out_idx);
    scan.use_subset = false;
    if (nneg) *nneg = pr.nneg;
    pricing_passes += pr.passes;
    OTIP_HIP(hipStreamSynchronize(st));
    t_pricing += now() - t0;
    return pr.count;
}

// --------------------------------------------------------- support update
// New support = kept old entries plus entering ones (p = s = sqrt(mu)),
// re-sorted by variable index; removed entries get the key ~0 and sort last.
void Solver::update_support(const uint64_t *add_idx, int64_t nadd, double pin,
                            const uint8_t *removed, int64_t nrem) {
    const int64_t psi_new = psi_ - nrem + nadd;
    const int64_t tot = psi_ + nadd;
    uint64_t *kin = tmp_u64a.need(tot);
    double *pin_ = tmp_f64a.need(tot), *sin_ = tmp_f64b.need(tot);
    const uint64_t *id = idx.get();
    const double *pp = p.get(), *ss = s.get();
    const int64_t psi = psi_;
    foreach(st, psi, [=] __device__(int64_t k) {
        kin[k] = (removed && removed[k]) ? ~0ull : id[k];
        pin_[k] = pp[k];
        sin_[k] = ss[k];
    });
    if (nadd > 0) {
        foreach(st, nadd, [=] __device__(int64_t k) {
            kin[psi + k] = add_idx[k];
            pin_[psi + k] = pin;
            sin_[psi + k] = pin;
        });
        foreach(st, nadd, FBits{add_idx, bitmap.get(), true});
    }
    if (removed && nrem > 0) {
        const uint8_t *rm = removed;
        uint32_t *bm = bitmap.get();
        foreach(st, psi, [=] __device__(int64_t k) {
            if (rm[k]) {
                const uint64_t v = id[k];
                atomicAnd(&bm[v >> 5], ~(1u << (v & 31u)));
            }
        });
    }
    uint64_t *kout = tmp_u64b.need(tot);
    double *pout = tmp_f64c.need(tot), *sout = tmp_f64d.need(tot);
    // variable indices are below m n; removed entries carry ~0, whose low
    // `bits` bits (all ones) still order after every index
    int bits = 2;
    while (bits < 64 && (((uint64_t)1 << (bits - 1)) < (uint64_t)m * (uint64_t)n)) ++bits;
    sort_pairs_u64_f64x2(st, kin, pin_, sin_, kout, pout, sout, tot, bits, tmp, tmp_i32a,
                         tmp_i32b);
    psi_ = psi_new;
    if ((size_t)psi_new > idx.cap) alloc_support(psi_new * 2);
    OTIP_HIP(hipMemcpyAsync(idx.get(), kout, sizeof(uint64_t) * psi_new, hipMemcpyDeviceToDevice, st));
    OTIP_HIP(hipMemcpyAsync(p.get(), pout, sizeof(double) * psi_new, hipMemcpyDeviceToDevice, st));
    OTIP_HIP(hipMemcpyAsync(s.get(), sout, sizeof(double) * psi_new, hipMemcpyDeviceToDevice, st));
    // a support that only lost entries keeps its Schur pattern (Section 4.2
    // remark on updating the symbolic structure instead of rebuilding it)
    const bool keep = P.schur_reuse && schur_valid && nadd == 0 && nrem > 0;
    rebuild_views();
    if (keep) {
        schur.keep_pattern(st, psi_, csr_pos.get(), sj.get());
        schur_valid = true;
    }
    pattern_kept = keep;
    patterns_kept += keep ? 1 : 0;
    psi_max = std::max(psi_max, psi_);
}

// removal (Section 3.2): small p leave once near convergence; the largest p of
// every row and column stays so that no row or column is left uncovered.
// G lanes per segment (a row of the compressed-row view, through its
// positions, or a column of the compressed-column view): marks the entry of
// largest p, ties to the smaller variable index.  That order is total, so the
// marked entry does not depend on how the lanes split the segment.
template <int G, bool ROWS>
__global__ __launch_bounds__(256) void protect_max_k(int64_t segs, const int32_t *__restrict__ ptr,
                                                     const int32_t *__restrict__ pos,
                                                     const double *__restrict__ p,
                                                     const uint64_t *__restrict__ id,
                                                     uint8_t *__restrict__ prot) {
    constexpr int groups = 256 / G;
    const int g = threadIdx.x / G, l = threadIdx.x % G;
    for (int64_t sg = (int64_t)blockIdx.x * groups + g; sg < segs;
         sg += (int64_t)gridDim.x * groups) {
        const int b = ptr[sg], e = ptr[sg + 1];
        int best = -1;
        double bp = 0.0;
        unsigned long long bi = 0ull;
        for (int q = b + l; q < e; q += G) {
            const int k = ROWS ? pos[q] : q;
            const double pk = p[k];
            const unsigned long long ik = id[k];
            if (best < 0 || pk > bp || (pk == bp && ik < bi)) {
                best = k;
                bp = pk;
                bi = ik;
            }
        }
        for (int o = G / 2; o > 0; o >>= 1) {
            const int ob = __shfl_xor(best, o, G);
            const double op = __shfl_xor(bp, o, G);
            const unsigned long long oi = __shfl_xor(bi, o, G);
            if (ob >= 0 && (best < 0 || op > bp || (op == bp && oi < bi))) {
                best = ob;
                bp = op;
                bi = oi;
            }
        }
        if (l == 0 && best >= 0) prot[best] = 1;
    }
}

int64_t Solver::select_removals(uint8_t *removed) {
    const int64_t psi = psi_;
    uint8_t *pr = prot.get();
    OTIP_HIP(hipMemsetAsync(pr, 0, psi, st));
    OTIP_HIP(hipMemsetAsync(removed, 0, psi, st));
    const double *pp = p.get();
    const uint64_t *id = idx.get();
    const int32_t *rp = row_ptr.get(), *cp = csr_pos.get(), *cptr = col_ptr.get();
    // the largest entry of every row and every column stays (no row or
    // column of the plan may lose its last entry)
    hipLaunchKernelGGL((protect_max_k<16, true>), dim3(std::min<int64_t>(4096, (m + 15) / 16)),
                       dim3(256), 0, st, (int64_t)m, rp, cp, pp, id, pr);
    hipLaunchKernelGGL((protect_max_k<16, false>), dim3(std::min<int64_t>(4096, (n + 15) / 16)),
                       dim3(256), 0, st, (int64_t)n, cptr, (const int32_t *)nullptr, pp, id, pr);
    OTIP_HIP(hipGetLastError());
    const double *aa = a.get(), *bb = b.get();
    const int32_t *ii = si.get(), *jj = sj.get();
    const double rel = P.remove_rel;
    double cnt;
    reduce_sum<1>(st, red, psi,
                  [=] __device__(int64_t k, double *acc) {
                      const double thr = rel * fmin(aa[ii[k]], bb[jj[k]]);
                      if (!pr[k] && pp[k] < thr) acc[0] += 1.0;
                  },
                  &cnt);
    const int64_t ncand = (int64_t)cnt;
    if (ncand == 0) return 0;
    if (ncand <= m) {
        foreach(st, psi, [=] __device__(int64_t k) {
            const double thr = rel * fmin(aa[ii[k]], bb[jj[k]]);
            removed[k] = (!pr[k] && pp[k] < thr) ? 1 : 0;
        });
        return ncand;
    }
    // more than m candidates: the m smallest by (p, idx)
    uint64_t *keys = tmp_u64a.need(psi), *vals = tmp_u64c.need(psi);
    foreach(st, psi, [=] __device__(int64_t k) {
        const double thr = rel * fmin(aa[ii[k]], bb[jj[k]]);
        const bool c = !pr[k] && pp[k] < thr;
        keys[k] = c ? dkey(pp[k]) : ~0ull;
        vals[k] = (uint64_t)k;  // position order == variable order
    });
    uint64_t *ko = tmp_u64b.need(psi), *vo = tmp_u64d.need(psi);
    sort_pairs_u64(st, keys, vals, ko, vo, psi, 0, 64, tmp);  // stable: ties keep index order
    const int64_t take = m;
    foreach(st, take, [=] __device__(int64_t t) { removed[vo[t]] = 1; });
    return take;
}

// ================================================================ the solve
struct FScaleIn {
    const double *src;
    double *dst;
    double f;
    __device__ void operator()(int64_t k) const { dst[k] = src[k] * f; }
};

// Zero masses (the marginals lie in R+): the rows and columns with zero mass
// carry no flow, so they are dropped, the problem without them is solved, and
// they come back with zero flow and c-transform duals (y_i = min_j C_ij - z_j
// over the kept targets, then z_j = min_i C_ij - y_i over all sources), which
// keep every reduced cost of the added rows and columns >= 0: the certificate
// of the smaller problem holds for the whole one.
int Solver::run_without_zeros(const otip_problem &pr, const otip_params &prm, Result &res) {
    const int M = pr.m, Nn = pr.n;
    std::vector<double> ha(M), hb(Nn);
    std::vector<int32_t> hxs((size_t)2 * M), hxt((size_t)2 * Nn);
    std::vector<double> hy0, hz0;
    OTIP_HIP(hipMemcpyAsync(ha.data(), pr.a, sizeof(double) * M, hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipMemcpyAsync(hb.data(), pr.b, sizeof(double) * Nn, hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipMemcpyAsync(hxs.data(), pr.xs, sizeof(int32_t) * 2 * M, hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipMemcpyAsync(hxt.data(), pr.xt, sizeof(int32_t) * 2 * Nn, hipMemcpyDeviceToHost, st));
    if (pr.y0 && pr.z0) {
        hy0.resize(M);
        hz0.resize(Nn);
        OTIP_HIP(hipMemcpyAsync(hy0.data(), pr.y0, sizeof(double) * M, hipMemcpyDeviceToHost, st));
        OTIP_HIP(hipMemcpyAsync(hz0.data(), pr.z0, sizeof(double) * Nn, hipMemcpyDeviceToHost, st));
    }
    OTIP_HIP(hipStreamSynchronize(st));
    std::vector<int32_t> ki, kj;
    for (int i = 0; i < M; ++i)
        if (ha[i] > 0.0) ki.push_back(i);
    for (int j = 0; j < Nn; ++j)
        if (hb[j] > 0.0) kj.push_back(j);
    const int mk = (int)ki.size(), nk = (int)kj.size();
    std::vector<double> cm((size_t)mk + nk), cy((size_t)mk + nk);
    std::vector<int32_t> cx((size_t)2 * (mk + nk));
    for (int q = 0; q < mk; ++q) {
        cm[q] = ha[ki[q]];
        cx[2 * q] = hxs[2 * ki[q]];
        cx[2 * q + 1] = hxs[2 * ki[q] + 1];
        if (!hy0.empty()) cy[q] = hy0[ki[q]];
    }
    for (int q = 0; q < nk; ++q) {
        cm[mk + q] = hb[kj[q]];
        cx[2 * (mk + q)] = hxt[2 * kj[q]];
        cx[2 * (mk + q) + 1] = hxt[2 * kj[q] + 1];
        if (!hz0.empty()) cy[mk + q] = hz0[kj[q]];
    }
    double *dm = zmass_.need(cm.size()), *dy = zdual_.need(cy.size());
    int32_t *dx = zcoord_.need(cx.size());
    OTIP_HIP(hipMemcpyAsync(dm, cm.data(), sizeof(double) * cm.size(), hipMemcpyHostToDevice, st));
    OTIP_HIP(hipMemcpyAsync(dy, cy.data(), sizeof(double) * cy.size(), hipMemcpyHostToDevice, st));
    OTIP_HIP(hipMemcpyAsync(dx, cx.data(), sizeof(int32_t) * cx.size(), hipMemcpyHostToDevice, st));
    otip_problem sub{mk, nk, dm, dm + mk, dx, dx + 2 * (size_t)mk,
                     hy0.empty() ? nullptr : dy, hz0.empty() ? nullptr : dy + mk, pr.cost_kind};
    Result r;
    const int status = run(sub, prm, r);  // no zero masses left: no further recursion
    res.info = r.info;
    res.rows.resize(r.rows.size());
    res.cols.resize(r.cols.size());
    for (size_t k = 0; k < r.rows.size(); ++k) {
        res.rows[k] = ki[r.rows[k]];
        res.cols[k] = kj[r.cols[k]];
    }
    res.vals = r.vals;
    // order of the expanded plan: by variable index i + j*M
    {
        std::vector<size_t> ord(res.vals.size());
        for (size_t k = 0; k < ord.size(); ++k) ord[k] = k;
        std::sort(ord.begin(), ord.end(), [&](size_t u, size_t v) {
            const int64_t iu = res.rows[u] + (int64_t)res.cols[u] * M;
            const int64_t iv = res.rows[v] + (int64_t)res.cols[v] * M;
            return iu < iv;
        });
        std::vector<int32_t> rr(ord.size()), cc(ord.size());
        std::vector<double> vv(ord.size());
        for (size_t k = 0; k < ord.size(); ++k) {
            rr[k] = res.rows[ord[k]];
            cc[k] = res.cols[ord[k]];
            vv[k] = res.vals[ord[k]];
        }
        res.rows.swap(rr);
        res.cols.swap(cc);
        res.vals.swap(vv);
    }
    std::vector<double> yf(M, 0.0), zf(Nn, -INFINITY);
    for (int q = 0; q < mk; ++q) yf[ki[q]] = r.y[q];
    for (int q = 0; q < nk; ++q) zf[kj[q]] = r.z[q];
    double *gy = zdual_.need((size_t)2 * (M + Nn));
    double *gz = gy + M, *ty = gz + Nn, *tz = ty + M;
    OTIP_HIP(hipMemcpyAsync(gz, zf.data(), sizeof(double) * Nn, hipMemcpyHostToDevice, st));
    if (mk < M) {
        std::vector<double> h(M);
        scan.ctransform_rows(st, M, Nn, pr.xs, pr.xt, gz, ty);
        OTIP_HIP(hipMemcpyAsync(h.data(), ty, sizeof(double) * M, hipMemcpyDeviceToHost, st));
        OTIP_HIP(hipStreamSynchronize(st));
        for (int i = 0; i < M; ++i)
            if (!(ha[i] > 0.0)) yf[i] = h[i];
    }
    if (nk < Nn) {
        std::vector<double> h(Nn);
        OTIP_HIP(hipMemcpyAsync(gy, yf.data(), sizeof(double) * M, hipMemcpyHostToDevice, st));
        scan.ctransform_cols(st, M, Nn, pr.xs, pr.xt, gy, tz);
        OTIP_HIP(hipMemcpyAsync(h.data(), tz, sizeof(double) * Nn, hipMemcpyDeviceToHost, st));
        OTIP_HIP(hipStreamSynchronize(st));
        for (int j = 0; j < Nn; ++j)
            if (!(hb[j] > 0.0)) zf[j] = h[j];
    }
    const double g = zf[Nn - 1];  // gauge z_{n-1} = 0
    for (auto &v : yf) v += g;
    for (auto &v : zf) v -= g;
    res.y.swap(yf);
    res.z.swap(zf);
    res.info.nnz = (int64_t)res.vals.size();
    return status;
}

void Solver::snapshot(int it, double tol_int, const std::vector<int64_t> &hist) {
    Checkpoint &c = last_;
    c.m = m;
    c.n = n;
    c.fingerprint = fp_;
    c.it = it;
    c.mode = mode == Mode::Direct ? 1 : 0;
    c.cg_its_last = cg_its_last;
    c.solves_last = solves_last;
    c.cg_failed = cg_failed ? 1 : 0;
    c.warm_used = warm_used ? 1 : 0;
    c.direct_its = direct_its;
    c.forced_switch_done = forced_switch_done ? 1 : 0;
    c.forced_back_done = forced_back_done ? 1 : 0;
    c.switched_by_drop = switched_by_drop ? 1 : 0;
    c.switches_back = switches_back;
    c.psi = psi_;
    c.psi_max = psi_max;
    c.cg_total = cg_total;
    c.tol_int = tol_int;
    c.max_fill = max_fill;
    // one entry per iteration started before `it` (a break inside iteration
    // `it` has already recorded it)
    c.psi_hist.assign(hist.begin(), hist.begin() + std::min<size_t>(hist.size(), (size_t)it));
    c.idx.resize(psi_);
    c.p.resize(psi_);
    c.s.resize(psi_);
    c.y.resize(m);
    c.z.resize(n);
    OTIP_HIP(hipMemcpyAsync(c.idx.data(), idx.get(), sizeof(uint64_t) * psi_, hipMemcpyDeviceToHost,
                            st));
    OTIP_HIP(hipMemcpyAsync(c.p.data(), p.get(), sizeof(double) * psi_, hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipMemcpyAsync(c.s.data(), s.get(), sizeof(double) * psi_, hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipMemcpyAsync(c.y.data(), y.get(), sizeof(double) * m, hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipMemcpyAsync(c.z.data(), z.get(), sizeof(double) * n, hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipStreamSynchronize(st));
    have_last_ = true;
}

// The support, iterate and loop state of a checkpoint of this same problem,
// checked on the host before anything reaches the device.
void Solver::resume_from(const Checkpoint &c) {
    OTIP_CHECK(c.m == m && c.n == n && c.fingerprint == fp_, OTIP_EINVAL,
               "checkpoint belongs to another problem");
    const uint64_t mn = (uint64_t)m * (uint64_t)n;
    OTIP_CHECK(c.psi >= 1 && (uint64_t)c.psi <= mn && (int64_t)c.idx.size() == c.psi &&
                   (int64_t)c.p.size() == c.psi && (int64_t)c.s.size() == c.psi &&
                   (int64_t)c.y.size() == m && (int64_t)c.z.size() == n,
               OTIP_EINVAL, "checkpoint: inconsistent sizes");
    for (int64_t k = 0; k < c.psi; ++k) {
        OTIP_CHECK(c.idx[k] < mn && (k == 0 || c.idx[k] > c.idx[k - 1]), OTIP_EINVAL,
                   "checkpoint: support indices out of range or not increasing");
        OTIP_CHECK(std::isfinite(c.p[k]) && std::isfinite(c.s[k]) && c.p[k] > 0.0 && c.s[k] > 0.0,
                   OTIP_EINVAL, "checkpoint: iterate not interior");
    }
    for (double v : c.y) OTIP_CHECK(std::isfinite(v), OTIP_EINVAL, "checkpoint: non-finite y");
    for (double v : c.z) OTIP_CHECK(std::isfinite(v), OTIP_EINVAL, "checkpoint: non-finite z");
    OTIP_CHECK(c.mode == 0 || (c.mode == 1 && n <= P.dense_max_n), OTIP_EINVAL,
               "checkpoint: solver mode not available");
    OTIP_CHECK(c.it >= 0 && c.tol_int > 0.0 && c.psi_max >= c.psi, OTIP_EINVAL,
               "checkpoint: bad loop state");
    alloc_support(std::max<int64_t>(c.psi * 2, c.psi + 4 * (int64_t)std::max(m, n)));
    OTIP_HIP(hipMemcpyAsync(idx.get(), c.idx.data(), sizeof(uint64_t) * c.psi,
                            hipMemcpyHostToDevice, st));
    OTIP_HIP(hipMemcpyAsync(p.get(), c.p.data(), sizeof(double) * c.psi, hipMemcpyHostToDevice, st));
    OTIP_HIP(hipMemcpyAsync(s.get(), c.s.data(), sizeof(double) * c.psi, hipMemcpyHostToDevice, st));
    OTIP_HIP(hipMemcpyAsync(y.get(), c.y.data(), sizeof(double) * m, hipMemcpyHostToDevice, st));
    OTIP_HIP(hipMemcpyAsync(z.get(), c.z.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
    psi_ = c.psi;
    psi_max = c.psi_max;
    rebuild_views();
    foreach(st, psi_, FBits{idx.get(), bitmap.get(), true});
    mode = c.mode == 1 ? Mode::Direct : Mode::PCG;
    cg_its_last = c.cg_its_last;
    solves_last = c.solves_last;
    warm_used = c.warm_used != 0;
    direct_its = c.direct_its;
    forced_switch_done = c.forced_switch_done != 0;
    forced_back_done = c.forced_back_done != 0;
    switched_by_drop = c.switched_by_drop != 0;
    switches_back = c.switches_back;
    cg_total = c.cg_total;
    max_fill = c.max_fill;
    OTIP_HIP(hipStreamSynchronize(st));
    log("otip: m=%d n=%d resumed at iteration %d with psi=%lld\n", m, n, c.it, (long long)c.psi);
}

// Per-solve scalars back to their initial values; device buffers are kept so
// that a solver reused for a stream of problems allocates (and frees) nothing
// once it has seen the largest one.
void Solver::reset_state() {
    if (poison_allocations()) ++poison_epoch();
    psi_ = psi_max = 0;
    schur_valid = false;
    mode = Mode::PCG;
    cg_failed = false;
    cg_its_iter = max_cg_solve = 0;
    cg_total = 0;
    direct_its = iterations = 0;
    pricing_passes = 0;
    max_fill = 0.0;
    cg_its_last = 0;
    solves_last = 2;
    heur_on = false;
    heur_scans = 0;
    forced_switch_done = forced_back_done = switched_by_drop = false;
    switches_back = 0;
    pattern_kept = false;
    patterns_kept = 0;
    t_pricing = t_newton = t_direct = t_update = t_setup = t_final = 0.0;
    t_spmv.reset();
    t_price.reset();
    t_diag.reset();
    t_upd.reset();
    ldl.restart_sampling();
    scan.scans = 0;
    scan.reset_guess();
    warm_used = false;
}

int Solver::run(const otip_problem &pr, const otip_params &prm, Result &res) {
    const double T0 = now();
    reset_state();
    P = prm;
    t_spmv.on = t_price.on = t_diag.on = t_upd.on = P.profile != 0;
    // events on every SpMV and pricing launch slow the solve by a few per
    // cent; the first of every 8 CG solves and pricing calls is timed
    t_spmv.stride = t_price.stride = 8;
    schur.timer = &t_spmv;
    scan.timer = &t_price;
    ldl.diag_timer = &t_diag;
    ldl.update_timer = &t_upd;
    scan.tile = P.price_tile;
    m = pr.m;
    n = pr.n;
    xs = pr.xs;
    xt = pr.xt;
    a_in = pr.a;
    b_in = pr.b;
    OTIP_CHECK(m >= 1 && n >= 1, OTIP_EINVAL, "m and n must be >= 1");
    OTIP_CHECK(pr.a && pr.b && pr.xs && pr.xt, OTIP_EINVAL, "null problem array");
    OTIP_CHECK(pr.cost_kind >= OTIP_COST_SQEUCLID && pr.cost_kind <= OTIP_COST_LINF, OTIP_EINVAL,
               "unknown cost kind");
    kind = pr.cost_kind;
    scan.kind = kind;
    // ---- validation on the device data (masses > 0, balanced)
    double sa, sb, bad, zeros;
    {
        const double *A = pr.a, *B = pr.b;
        const int mm = m;
        double v[4];
        reduce_sum<4>(st, red, (int64_t)m + n,
                      [=] __device__(int64_t t, double *acc) {
                          const double x = t < mm ? A[t] : B[t - mm];
                          if (t < mm)
                              acc[0] += x;
                          else
                              acc[1] += x;
                          if (!(x >= 0.0) || isinf(x)) acc[2] += 1.0;
                          if (x == 0.0) acc[3] += 1.0;
                      },
                      v);
        sa = v[0];
        sb = v[1];
        bad = v[2];
        zeros = v[3];
    }
    OTIP_CHECK(bad == 0.0, OTIP_EINVAL, "masses must be finite and nonnegative");
    OTIP_CHECK(sa > 0.0 && sb > 0.0, OTIP_EINVAL, "total mass must be positive");
    OTIP_CHECK(std::fabs(sa - sb) <= 1e-12 * sa, OTIP_EINVAL, "sum(a) != sum(b)");
    if (zeros > 0.0) return run_without_zeros(pr, prm, res);
    {
        // coordinate range -> largest cost (for scaling and the initial support)
        std::vector<int32_t> hx((size_t)2 * m), ht((size_t)2 * n);
        std::vector<double> ha(m), hb(n);
        OTIP_HIP(hipMemcpyAsync(hx.data(), xs, sizeof(int32_t) * 2 * m, hipMemcpyDeviceToHost, st));
        OTIP_HIP(hipMemcpyAsync(ht.data(), xt, sizeof(int32_t) * 2 * n, hipMemcpyDeviceToHost, st));
        OTIP_HIP(hipMemcpyAsync(ha.data(), pr.a, sizeof(double) * m, hipMemcpyDeviceToHost, st));
        OTIP_HIP(hipMemcpyAsync(hb.data(), pr.b, sizeof(double) * n, hipMemcpyDeviceToHost, st));
        OTIP_HIP(hipStreamSynchronize(st));
        // identity of the problem, for checkpoints (FNV-1a over its bytes)
        fp_ = 14695981039346656037ull;
        auto mix = [&](const void *q, size_t len) {
            const unsigned char *c = (const unsigned char *)q;
            for (size_t k = 0; k < len; ++k) fp_ = (fp_ ^ c[k]) * 1099511628211ull;
        };
        mix(&m, sizeof m);
        mix(&n, sizeof n);
        mix(&kind, sizeof kind);
        mix(ha.data(), sizeof(double) * m);
        mix(hb.data(), sizeof(double) * n);
        mix(hx.data(), sizeof(int32_t) * 2 * m);
        mix(ht.data(), sizeof(int32_t) * 2 * n);
        int64_t lo[2] = {INT64_MAX, INT64_MAX}, hi[2] = {INT64_MIN, INT64_MIN};
        for (int q = 0; q < m; ++q)
            for (int d = 0; d < 2; ++d) {
                lo[d] = std::min<int64_t>(lo[d], hx[2 * q + d]);
                hi[d] = std::max<int64_t>(hi[d], hx[2 * q + d]);
            }
        for (int q = 0; q < n; ++q)
            for (int d = 0; d < 2; ++d) {
                lo[d] = std::min<int64_t>(lo[d], ht[2 * q + d]);
                hi[d] = std::max<int64_t>(hi[d], ht[2 * q + d]);
            }
        for (int d = 0; d < 2; ++d)
            OTIP_CHECK(lo[d] >= -(1 << 14) && hi[d] <= (1 << 14), OTIP_EINVAL,
                       "coordinates must lie in [-2^14, 2^14]");
        const int64_t w0 = hi[0] - lo[0], w1 = hi[1] - lo[1];
        cmax = kind == OTIP_COST_L1     ? w0 + w1
               : kind == OTIP_COST_LINF ? std::max(w0, w1)
                                        : w0 * w0 + w1 * w1;
    }
    omega = 1.0;
    zeta = 1.0;
    if (P.scale) {
        // the largest cost bounds the scale: for the 2-norm the root of its key
        double cm = (double)std::max<int64_t>(1, cmax);
        if (kind == OTIP_COST_L2) cm = std::sqrt(cm);
        omega = std::ldexp(1.0, (int)std::lround(std::log2((double)m / sa)));
        zeta = std::ldexp(1.0, -(int)std::ceil(std::log2(cm)));
    }
    a.need(m);
    b.need(n);
    foreach(st, m, FScaleIn{pr.a, a.get(), omega});
    foreach(st, n, FScaleIn{pr.b, b.get(), omega});
    {
        const double *A = a.get(), *B = b.get();
        const int mm = m;
        double q;
        reduce_sum<1>(st, red, (int64_t)m + n,
                      [=] __device__(int64_t t, double *acc) {
                          const double x = t < mm ? A[t] : B[t - mm];
                          acc[0] = fma(x, x, acc[0]);
                      },
                      &q);
        fnorm = std::sqrt(q);
    }
    // heuristic pricing subset (Section 3.4): pairs closer than heur_radius
    // times the largest distance, as an integer bound on the cost key
    if (P.heur_radius > 0.0 && P.heur_run >= 1) {
        const double lim = (kind == OTIP_COST_L1 || kind == OTIP_COST_LINF)
                               ? std::ceil(P.heur_radius * (double)cmax)
                               : std::ceil(P.heur_radius * P.heur_radius * (double)cmax);
        OTIP_CHECK(std::isfinite(lim) && lim < 9.0e18, OTIP_EINVAL, "heur_radius too large");
        const int64_t L = std::max<int64_t>(1, (int64_t)lim);
        heur_on = scan.set_subset(st, m, n, xs, xt, L) > 0;
    }
    y.need(m);
    z.need(n);
    M.need(m);
    invM.need(m);
    N.need(n);
    r1a.need(m);
    r1b.need(n);
    beta1.need(m);
    beta2.need(n);
    rhs.need(n);
    tmpn.need(n);
    tmpn2.need(n);
    OTIP_HIP(hipMemsetAsync(zm.need(m), 0, sizeof(double) * m, st));
    OTIP_HIP(hipMemsetAsync(zn.need(n), 0, sizeof(double) * n, st));
    const size_t words = ((size_t)m * (size_t)n + 31) / 32;
    bitmap.need(words);
    OTIP_HIP(hipMemsetAsync(bitmap.get(), 0, words * sizeof(uint32_t), st));

    // ---- initial support (Section 3.2, end), or a checkpoint's state
    double ts = now();
    int64_t T = 0;
    DBuf<uint64_t> &init = init_;
    OTIP_CHECK((pr.y0 == nullptr) == (pr.z0 == nullptr), OTIP_EINVAL,
               "warm start needs both y0 and z0");
    const std::unique_ptr<Checkpoint> resume = std::move(pending_);
    if (resume) {
        resume_from(*resume);
    } else {
        int64_t psi0 = -1;
        if (pr.y0) {
            psi0 = scan.warm_support(st, m, n, xs, xt, pr.y0, pr.z0,
                                     P.ws_kappa > 0 ? P.ws_kappa : P.kappa, init, yws_, zws_);
            warm_used = psi0 >= 0;
            if (warm_used && P.ws_union) {
                // the plain rule's support joined to the predicted one: a poor
                // prediction then adds columns without taking the cheap ones away
                const int64_t psi_p =
                    scan.initial_support(st, m, n, xs, xt, P.kappa, cmax, init2_, &T);
                const int64_t tot = psi0 + psi_p;
                uint64_t *cat = tmp_u64a.need(tot), *srt = tmp_u64b.need(tot);
                OTIP_HIP(hipMemcpyAsync(cat, init.get(), sizeof(uint64_t) * psi0,
                                        hipMemcpyDeviceToDevice, st));
                OTIP_HIP(hipMemcpyAsync(cat + psi0, init2_.get(), sizeof(uint64_t) * psi_p,
                                        hipMemcpyDeviceToDevice, st));
                sort_keys_u64(st, cat, srt, tot, tmp);
                init.need(tot);
                psi0 = unique_u64(st, srt, init.get(), tot, tmp, ucnt_);
            }
        }
        if (psi0 < 0) psi0 = scan.initial_support(st, m, n, xs, xt, P.kappa, cmax, init, &T);
        alloc_support(std::max<int64_t>(psi0 * 2, psi0 + 4 * (int64_t)std::max(m, n)));
        OTIP_HIP(hipMemcpyAsync(idx.get(), init.get(), sizeof(uint64_t) * psi0,
                                hipMemcpyDeviceToDevice, st));
        psi_ = psi0;
        psi_max = psi0;
        rebuild_views();
        foreach(st, psi_, FBits{idx.get(), bitmap.get(), true});
        log("otip: m=%d n=%d psi0=%lld T=%lld omega=%g zeta=%g\n", m, n, (long long)psi0,
            (long long)T, omega, zeta);
        starting_point();
        trace("p0", -1, p.get(), sizeof(double) * psi_);
        trace("s0", -1, s.get(), sizeof(double) * psi_);
        trace("y0", -1, y.get(), sizeof(double) * m);
        trace("z0", -1, z.get(), sizeof(double) * n);
        mode = (P.linear_solver == OTIP_LS_DIRECT) ? Mode::Direct : Mode::PCG;
    }
    t_setup += now() - ts;

    if (mode == Mode::Direct)
        OTIP_CHECK(direct_available(), OTIP_EUNSUPPORTED,
                   "direct solver: n exceeds dense_max_n or its buffers do not fit");
    std::vector<int64_t> psi_hist;
    if (resume) psi_hist = resume->psi_hist;
    const int64_t kcap = P.enter_cap > 0 ? P.enter_cap : m;
    DBuf<uint64_t> &sel_idx = sel_idx_;
    DBuf<double> &sel_r = sel_r_;
    sel_idx.need(kcap);
    sel_r.need(kcap);
    DBuf<uint8_t> &removed = removed_;
    int status = OTIP_EMAXITER;
    int it = resume ? resume->it : 0;
    cg_failed = resume ? resume->cg_failed != 0 : false;
    double tol_int = resume ? resume->tol_int : P.tol;
    for (int round = 0;; ++round) {
    status = OTIP_EMAXITER;
    for (; it < P.max_iter; ++it) {
        double tn = now();
        double rel1, rel2, mu, primal, r1n;
        residuals(rel1, rel2, mu, primal, r1n);
        trace("idx", it, idx.get(), sizeof(uint64_t) * psi_);
        trace("p", it, p.get(), sizeof(double) * psi_);
        trace("s", it, s.get(), sizeof(double) * psi_);
        trace("y", it, y.get(), sizeof(double) * m);
        trace("z", it, z.get(), sizeof(double) * n);
        trace("r2", it, r2.get(), sizeof(double) * psi_);
        trace_val("mu", it, mu);
        if (!std::isfinite(rel1) || !std::isfinite(rel2) || !std::isfinite(mu)) {
            log("otip: it %d non-finite iterate\n", it);
            status = OTIP_ENUMERIC;
            break;
        }
        const double relmu = (double)psi_ * mu / std::max(1.0, std::fabs(primal));
        psi_hist.push_back(psi_);
        if (std::max(std::max(rel1, rel2), relmu) < tol_int) {
            t_newton += now() - tn;
            std::vector<double> hr(1);
            int64_t k = price(kcap, sel_idx.get(), sel_r.get(), nullptr);
            int64_t nbig = 0;
            if (k > 0) {
                std::vector<double> rs(k);
                OTIP_HIP(hipMemcpyAsync(rs.data(), sel_r.get(), sizeof(double) * k,
                                        hipMemcpyDeviceToHost, st));
                OTIP_HIP(hipStreamSynchronize(st));
                const double thr = P.cert_rel * std::max(1.0, std::fabs(primal));
                for (int64_t q = 0; q < k; ++q)
                    if (std::fabs(rs[q] * zeta) * (sa * omega) > thr) ++nbig;  // ordered by r
            }
            if (nbig == 0) {
                status = OTIP_OK;
                break;
            }
            double tu = now();
            update_support(sel_idx.get(), nbig, std::sqrt(mu), nullptr, 0);
            t_update += now() - tu;
            log("otip: it %d certification re-entered %lld columns\n", it, (long long)nbig);
            continue;
        }
        // ---- switch back to CG (remark of Section 4.3: the support grows again
        // after a switch made by the support-drop rule), or a forced one
        bool just_back = false;
        if (mode == Mode::Direct && P.linear_solver == OTIP_LS_AUTO) {
            const int wdw = P.switch_window;
            const char *why = nullptr;
            if (P.force_switch_back_at >= 0 && it >= P.force_switch_back_at && !forced_back_done) {
                forced_back_done = true;
                why = "forced";
            } else if (P.switch_back_grow > 0.0 && switched_by_drop &&
                       (int)psi_hist.size() > wdw) {
                const double old = (double)psi_hist[psi_hist.size() - 1 - wdw];
                if (((double)psi_ - old) / old >= P.switch_back_grow) why = "support growing";
            }
            if (why) {
                mode = Mode::PCG;
                switched_by_drop = false;
                cg_failed = false;
                ++switches_back;
                just_back = true;
                log("otip: it %d switch back to CG (%s)\n", it, why);
            }
        }
        // ---- switch test (Section 4.3)
        if (mode == Mode::PCG && !just_back && P.linear_solver == OTIP_LS_AUTO &&
            direct_available()) {
            const int wdw = P.switch_window;
            // fill "allows" a factorisation once it is cheaper than the CG it
            // replaces.  A fixed cost model (not wall time, so the switch point
            // is reproducible): CG iteration = SpMV bytes at 3 TB/s + three
            // launches of 6 us; dense = factor and inverse (2 n^3/3 flops at
            // 30 TF/s, the rate measured for both at n = 16384) + their
            // dependent launches (3 per 64-column block, 2 per doubling level,
            // 20 us each) + per solve two products over n^2/2 entries each at
            // 2 TB/s and two launches of 6 us.  From kDenseSplitMinN the
            // inverse's top level is not formed: n^3/12 flops for the inverse,
            // one level fewer, six launches per solve.
            const double nb = (double)((n + 63) / 64);
            const bool split = n >= kDenseSplitMinN;
            const double levels =
                std::ceil(std::log2(std::max(1.0, nb))) - (split ? 1.0 : 0.0);
            const double t_cg = cg_its_last * ((12.0 * (double)schur.S.nnz + 20.0 * n) / 3e12 +
                                               3 * 6e-6);
            const double t_dense = (split ? 5.0 / 12.0 : 2.0 / 3.0) * (double)n * n * n / 30e12 +
                                   (3.0 * nb + 2.0 * levels) * 20e-6 +
                                   solves_last * (8.0 * (double)n * n / 2e12 +
                                                  (split ? 6 : 2) * 6e-6);
            const bool cheaper = P.switch_cost && it >= 1 && t_dense < t_cg;
            const bool forced =
                P.force_switch_at >= 0 && it >= P.force_switch_at && !forced_switch_done;
            const bool force = forced || cg_failed || cheaper;
            bool drop = false;
            if ((int)psi_hist.size() > wdw) {
                const double old = (double)psi_hist[psi_hist.size() - 1 - wdw];
                drop = (old - (double)psi_) / old >= P.switch_drop;
            }
            if (force || drop) {
                mode = Mode::Direct;
                if (forced) forced_switch_done = true;
                switched_by_drop = !force && drop;
                log("otip: it %d switch to the direct solver (%s)\n", it,
                    cheaper ? "factorisation cheaper than CG"
                            : (force ? "forced/CG failure" : "support shrinking"));
            }
        }
        // ---- Newton direction
        assemble();
        trace("theta", it, theta.get(), sizeof(double) * psi_);
        trace("Sval", it, schur.S.val.get(), sizeof(double) * schur.S.nnz);
        trace("Scol", it, schur.S.col.get(), sizeof(int32_t) * schur.S.nnz);
        trace_val("mode", it, mode == Mode::Direct ? 1.0 : 0.0);
        double td = now();
        if (mode == Mode::Direct) {
            ldl.factor(st, schur.S, P.pivot_tol);
            trace("piv", it, ldl.pivots(), sizeof(double) * n);
            max_fill = std::max(max_fill, 100.0 * (double)ldl.nnz_L() / ((double)n * n));
            direct_its++;
        }
        t_direct += (mode == Mode::Direct) ? now() - td : 0.0;
        cg_its_iter = 0;
        max_cg_solve = 0;
        cg_failed = false;
        const double atol = P.cg_eta * std::max(r1n, P.cg_floor * (1.0 + fnorm));
        int nsolves = 2;
        // predictor (sigma = 0)
        double *rr3 = r3.get();
        const double *pp = p.get(), *ss = s.get();
        foreach(st, psi_, [=] __device__(int64_t k) { rr3[k] = -pp[k] * ss[k]; });
        Dir &Da = D[0];
        newton(r1a.get(), r1b.get(), r2.get(), r3.get(), P.cg_tol_pred, atol, Da);
        trace("rhs_a", it, rhs.get(), sizeof(double) * n);
        trace("dz_a", it, Da.dz.get(), sizeof(double) * n);
        trace("dp_a", it, Da.dp.get(), sizeof(double) * psi_);
        double apa, ada;
        max_steps(Da, apa, ada);
        apa = std::min(1.0, apa);
        ada = std::min(1.0, ada);
        double mu_aff;
        {
            const double *dp = Da.dp.get(), *ds = Da.ds.get();
            const double ap_ = apa, ad_ = ada;
            reduce_sum<1>(st, red, psi_,
                          [=] __device__(int64_t k, double *acc) {
                              acc[0] = fma(pp[k] + ap_ * dp[k], ss[k] + ad_ * ds[k], acc[0]);
                          },
                          &mu_aff);
            mu_aff /= (double)psi_;
        }
        const double sigma = mu > 0.0 ? std::pow(mu_aff / mu, 3.0) : 0.0;
        // Mehrotra corrector
        {
            const double *dp = Da.dp.get(), *ds = Da.ds.get();
            const double sm = sigma * mu;
            foreach(st, psi_, [=] __device__(int64_t k) {
                rr3[k] = sm - pp[k] * ss[k] - dp[k] * ds[k];
            });
        }
        int cur = 1;
        newton(r1a.get(), r1b.get(), r2.get(), r3.get(), P.cg_tol_pred, atol, D[cur]);
        trace("dz_c", it, D[cur].dz.get(), sizeof(double) * n);
        double ap, ad;
        max_steps(D[cur], ap, ad);
        ap = std::min(1.0, P.step_scale * ap);
        ad = std::min(1.0, P.step_scale * ad);
        // Gondzio centrality correctors
        int ncorr = 0;
        while (ncorr < P.max_corr && std::min(ap, ad) < 1.0) {
            const double atp = std::min(1.0, ap + P.mcc_delta), atd = std::min(1.0, ad + P.mcc_delta);
            const double lo = P.mcc_beta_min * sigma * mu, hi = P.mcc_beta_max * sigma * mu;
            {
                const double *dp = D[cur].dp.get(), *ds = D[cur].ds.get();
                foreach(st, psi_, [=] __device__(int64_t k) {
                    const double v = (pp[k] + atp * dp[k]) * (ss[k] + atd * ds[k]);
                    double rc = fmin(fmax(v, lo), hi) - v;
                    rr3[k] = fmax(rc, -hi);
                });
            }
            const int tri = 3 - cur;  // the other of D[1], D[2]
            newton(zm.get(), zn.get(), nullptr, r3.get(), P.cg_tol_corr, atol, D[tri]);
            ++nsolves;
            {
                const double *dp = D[cur].dp.get(), *ds = D[cur].ds.get();
                const double *dy = D[cur].dy.get(), *dz = D[cur].dz.get();
                double *tp = D[tri].dp.get(), *ts_ = D[tri].ds.get();
                double *ty = D[tri].dy.get(), *tz = D[tri].dz.get();
                foreach(st, psi_, [=] __device__(int64_t k) {
                    tp[k] += dp[k];
                    ts_[k] += ds[k];
                });
                foreach(st, m, [=] __device__(int64_t i) { ty[i] += dy[i]; });
                foreach(st, n, [=] __device__(int64_t j) { tz[j] += dz[j]; });
            }
            double nap, nad;
            max_steps(D[tri], nap, nad);
            nap = std::min(1.0, P.step_scale * nap);
            nad = std::min(1.0, P.step_scale * nad);
            if (std::min(nap, nad) >= std::min(ap, ad) + P.mcc_accept) {
                cur = tri;
                ap = nap;
                ad = nad;
                ++ncorr;
            } else {
                break;
            }
        }
        cg_total += cg_its_iter;
        if (mode == Mode::PCG) cg_its_last = cg_its_iter;
        solves_last = nsolves;
        const bool failed_now = cg_failed;
        // ---- update
        {
            Dir &d = D[cur];
            const double *dp = d.dp.get(), *ds = d.ds.get(), *dy = d.dy.get(), *dz = d.dz.get();
            double *pw = p.get(), *sw = s.get(), *yw = y.get(), *zw = z.get();
            const double ap_ = ap, ad_ = ad;
            foreach(st, psi_, [=] __device__(int64_t k) {
                pw[k] += ap_ * dp[k];
                sw[k] += ad_ * ds[k];
            });
            foreach(st, m, [=] __device__(int64_t i) { yw[i] += ad_ * dy[i]; });
            foreach(st, n, [=] __device__(int64_t j) { zw[j] += ad_ * dz[j]; });
        }
        double mu_new;
        {
            const double *pw = p.get(), *sw = s.get();
            reduce_sum<1>(st, red, psi_,
                          [=] __device__(int64_t k, double *acc) { acc[0] = fma(pw[k], sw[k], acc[0]); },
                          &mu_new);
            mu_new /= (double)psi_;
        }
        t_newton += now() - tn;
        // ---- pricing and support update
        int64_t nneg = 0;
        // heuristic pricing (Section 3.4): heur_run iterations on the subset J,
        // then one full scan
        const bool heur = heur_on && it % (P.heur_run + 1) < P.heur_run;
        const int64_t k = price(kcap, sel_idx.get(), sel_r.get(), &nneg, heur);
        if (heur) ++heur_scans;
        trace_val("ap", it, ap);
        trace_val("ad", it, ad);
        trace_val("ncorr", it, ncorr);
        trace_val("cg", it, cg_its_iter);
        trace_val("nneg", it, (double)nneg);
        trace("sel", it, sel_idx.get(), sizeof(uint64_t) * k);
        double tu = now();
        int64_t nrem = 0;
        removed.need(psi_);
        if (std::max(rel1, rel2) <= P.remove_gate) nrem = select_removals(removed.get());
        if (k > 0 || nrem > 0)
            update_support(sel_idx.get(), k, std::sqrt(mu_new), nrem ? removed.get() : nullptr, nrem);
        t_update += now() - tu;
        if (failed_now && mode == Mode::PCG) cg_failed = true;
        log("otip: it %3d psi=%lld r1=%.2e r2=%.2e mu=%.2e ap=%.3f ad=%.3f sig=%.2e corr=%d cg=%d %s "
            "add=%lld rem=%lld\n",
            it, (long long)psi_hist.back(), rel1, rel2, relmu, ap, ad, sigma, ncorr, cg_its_iter,
            mode == Mode::Direct ? "dir" : "pcg", (long long)k, (long long)nrem);
    }
    snapshot(it, tol_int, psi_hist);
    if (status == OTIP_OK) ++it;
    double tf = now();
    finalize(res);
    t_final += now() - tf;
    // the certificate decides: a feasible plan (marginals to 1e-9) whose gap to
    // the certified bound is within the tolerance; a negative gap beyond it
    // means an infeasible plan.  Otherwise tighten the internal tolerance and
    // resume.
    const bool certified = std::isfinite(res.info.rel_gap) && res.info.rel_gap <= P.tol &&
                           res.info.rel_gap >= -P.tol && res.info.marginal_residual <= 1e-9;
    if (certified || status == OTIP_ENUMERIC || it >= P.max_iter || tol_int <= 1e-13) {
        if (!certified && status != OTIP_ENUMERIC) status = OTIP_EMAXITER;
        break;
    }
    tol_int = std::max(tol_int * 0.1, 1e-13);
    log("otip: certified gap %.3e above tolerance; resuming with stop tolerance %.1e\n",
        res.info.rel_gap, tol_int);
    }
    iterations = it;
    res.info.status = status;
    res.info.iterations = iterations;
    res.info.cg_iterations = (int32_t)cg_total;
    res.info.direct_iterations = direct_its;
    res.info.psi_max = psi_max;
    res.info.max_fill_pct = max_fill;
    res.info.seconds_total = now() - T0;
    res.info.seconds_pricing = t_pricing;
    res.info.seconds_newton = t_newton;
    res.info.seconds_direct = t_direct;
    res.info.seconds_update = t_update;
    res.info.seconds_setup = t_setup;
    res.info.seconds_final = t_final;
    res.info.pricing_scans = scan.scans;
    res.info.heuristic_scans = heur_scans;
    res.info.switches_back = switches_back;
    res.info.patterns_kept = patterns_kept;
    res.info.spmv_launches = t_spmv.launches;
    res.info.spmv_ms = t_spmv.ms;
    res.info.spmv_bytes = t_spmv.work;
    res.info.price_launches = t_price.launches;
    res.info.price_ms = t_price.ms;
    res.info.price_elems = t_price.work;
    res.info.diag_launches = t_diag.launches;
    res.info.diag_ms = t_diag.ms;
    res.info.diag_flops = t_diag.work;
    res.info.update_launches = t_upd.launches;
    res.info.update_ms = t_upd.ms;
    res.info.update_flops = t_upd.work;
    return status;
}

bool Solver::direct_available() {
    if (n > P.dense_max_n) return false;
    const size_t need = DenseLDL::bytes_for(n), held = ldl.held_bytes();
    if (need <= held) return true;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return false;
    // keep a margin for the Schur matrix and the support's arrays
    return need - held + ((size_t)1 << 30) <= free_b;
}

// Mehrotra's starting-point heuristic on the restricted LP (Theta = I); the
// paper leaves the starting point open.
void Solver::starting_point() {
    const int64_t psi = psi_;
    double *pp = p.get(), *ss = s.get();
    foreach(st, psi, [=] __device__(int64_t k) {
        pp[k] = 1.0;
        ss[k] = 1.0;
    });
    assemble();
    // with Theta = I the system is well conditioned: CG serves large orders
    const bool direct = n <= kDenseStartMaxN && direct_available();
    if (direct) ldl.factor(st, schur.S, P.pivot_tol);
    auto normal_solve = [&](const double *b1, const double *b2, double *dy, double *dz) {
        segsum(st, n, FRhs{col_ptr.get(), si.get(), theta.get(), b1, invM.get(), b2, rhs.get()});
        if (direct) {
            ldl.solve(st, rhs.get(), dz);
        } else {
            double mean = 0.0;
            const double *rp = rhs.get();
            reduce_sum<1>(st, red, n, [=] __device__(int64_t j, double *acc) { acc[0] += rp[j]; },
                          &mean);
            foreach(st, n, FSub{rhs.get(), mean / n});
            t_spmv.begin_call();
            schur.pcg(st, rhs.get(), dz, 1e-12, 0.0 + 1e300, std::max(P.cg_max_iter, 5000));
        }
        segsum(st, m, FDy{row_ptr.get(), csr_pos.get(), sj.get(), theta.get(), b1, invM.get(),
                          dz, dy});
    };
    // least-norm p~ = A^T (A A^T)^-1 f
    double *wy = D[0].dy.get(), *wz = D[0].dz.get();
    normal_solve(a.get(), b.get(), wy, wz);
    const int32_t *ii = si.get(), *jj = sj.get();
    foreach(st, psi, [=] __device__(int64_t k) { pp[k] = wy[ii[k]] + wz[jj[k]]; });
    // least-squares duals for c, s~ = c - A^T lambda
    rowsum(c.get(), nullptr, beta1.get(), 1.0);
    colsum(c.get(), nullptr, beta2.get(), 1.0);
    double *ly = y.get(), *lz = z.get();
    normal_solve(beta1.get(), beta2.get(), ly, lz);
    const double *cc = c.get();
    foreach(st, psi, [=] __device__(int64_t k) { ss[k] = cc[k] - (ly[ii[k]] + lz[jj[k]]); });
    double mins[2];
    reduce_min<2>(st, red, psi,
                  [=] __device__(int64_t k, double *acc) {
                      acc[0] = fmin(acc[0], pp[k]);
                      acc[1] = fmin(acc[1], ss[k]);
                  },
                  mins);
    const double dp = std::max(-1.5 * mins[0], 0.0), dsv = std::max(-1.5 * mins[1], 0.0);
    double sums[3];
    reduce_sum<3>(st, red, psi,
                  [=] __device__(int64_t k, double *acc) {
                      const double ph = pp[k] + dp, sh = ss[k] + dsv;
                      acc[0] = fma(ph, sh, acc[0]);
                      acc[1] += ph;
                      acc[2] += sh;
                  },
                  sums);
    const double dph = sums[2] > 0 ? 0.5 * sums[0] / sums[2] : 0.0;
    const double dsh = sums[1] > 0 ? 0.5 * sums[0] / sums[1] : 0.0;
    foreach(st, psi, [=] __device__(int64_t k) {
        pp[k] = pp[k] + dp + dph;
        ss[k] = ss[k] + dsv + dsh;
    });
    reduce_min<2>(st, red, psi,
                  [=] __device__(int64_t k, double *acc) {
                      acc[0] = fmin(acc[0], pp[k]);
                      acc[1] = fmin(acc[1], ss[k]);
                  },
                  mins);
    if (!(mins[0] > 0.0 && mins[1] > 0.0)) {
        foreach(st, psi, [=] __device__(int64_t k) {
            pp[k] = fmax(pp[k], 1e-8);
            ss[k] = fmax(ss[k], 1e-8);
        });
    }
}

// ------------------------------------------------------------------ final
// Primal projection onto A p = f on the support (dp = Theta A^T (A Theta A^T)^-1 r1,
// the Newton step with r2 = r3 = 0), purification to a basic plan, dual
// certificate from one full reduced-cost scan (Section 3.3: s_hat = c - A^T y_hat).
void Solver::finalize(Result &res) {
    // the projection below moves p off the interior; keep the interior
    // iterate for a resumed iteration
    double *pkeep = zpsi.need(psi_);
    OTIP_HIP(hipMemcpyAsync(pkeep, p.get(), sizeof(double) * psi_, hipMemcpyDeviceToDevice, st));
    bool assembled = false;
    for (int q = 0; q < P.polish_steps; ++q) {
        rowsum(p.get(), a.get(), r1a.get(), -1.0);
        colsum(p.get(), b.get(), r1b.get(), -1.0);
        const double *ra = r1a.get(), *rb = r1b.get(), *A = a.get(), *B = b.get();
        const int mm = m;
        double v[2];
        reduce_sum<2>(st, red, (int64_t)m + n,
                      [=] __device__(int64_t t, double *acc) {
                          acc[0] += fabs(t < mm ? ra[t] : rb[t - mm]);
                          acc[1] += fabs(t < mm ? A[t] : B[t - mm]);
                      },
                      v);
        if (v[0] / v[1] <= P.polish_tol) break;
        // Theta of the interior iterate, assembled and factorised once
        const bool direct = direct_available();
        if (!assembled) {
            assemble();
            if (direct) ldl.factor(st, schur.S, P.pivot_tol);
            assembled = true;
        }
        Mode keep = mode;
        mode = direct ? Mode::Direct : Mode::PCG;
        newton(r1a.get(), r1b.get(), nullptr, nullptr, 1e-14, 0.0, D[0]);
        mode = keep;
        double *pw = p.get();
        const double *dp = D[0].dp.get();
        double bad = 0.0;
        reduce_sum<1>(st, red, psi_,
                      [=] __device__(int64_t k, double *acc) { acc[0] += isfinite(dp[k]) ? 0.0 : 1.0; },
                      &bad);
        if (bad != 0.0) {
            log("otip: polish step %d not finite; plan kept as it was\n", q);
            break;
        }
        foreach(st, psi_, [=] __device__(int64_t k) { pw[k] = fmax(pw[k] + dp[k], 0.0); });
    }
    // to the host, unscaled
    const int64_t psi = psi_;
    std::vector<uint64_t> hidx(psi);
    std::vector<double> hp(psi), hy(m), hz(n), ha(m), hb(n);
    std::vector<int32_t> hxs((size_t)2 * m), hxt((size_t)2 * n);
    OTIP_HIP(hipMemcpyAsync(hidx.data(), idx.get(), sizeof(uint64_t) * psi, hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipMemcpyAsync(hp.data(), p.get(), sizeof(double) * psi, hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipMemcpyAsync(hy.data(), y.get(), sizeof(double) * m, hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipMemcpyAsync(hz.data(), z.get(), sizeof(double) * n, hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipMemcpyAsync(ha.data(), a_in, sizeof(double) * m, hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipMemcpyAsync(hb.data(), b_in, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipMemcpyAsync(hxs.data(), xs, sizeof(int32_t) * 2 * m, hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipMemcpyAsync(hxt.data(), xt, sizeof(int32_t) * 2 * n, hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipStreamSynchronize(st));
    OTIP_HIP(hipMemcpyAsync(p.get(), pkeep, sizeof(double) * psi_, hipMemcpyDeviceToDevice, st));
    std::vector<int32_t> rows(psi), cols(psi);
    std::vector<double> flows(psi);
    std::vector<double> costs(psi);
    auto icost = [&](int i, int j) { return pair_cost(hxs.data(), hxt.data(), i, j, kind); };
    for (int64_t k = 0; k < psi; ++k) {
        rows[k] = (int32_t)(hidx[k] % (uint64_t)m);
        cols[k] = (int32_t)(hidx[k] / (uint64_t)m);
        flows[k] = hp[k] / omega;
        costs[k] = icost(rows[k], cols[k]);
    }
    if (trace_on()) {
        uint64_t f = 14695981039346656037ull;
        for (double v : hp) {
            const unsigned char *c = (const unsigned char *)&v;
            for (int q = 0; q < 8; ++q) f = (f ^ c[q]) * 1099511628211ull;
        }
        fprintf(stderr, "TRACE %016llx -1 polished %016llx %lld\n", (unsigned long long)fp_,
                (unsigned long long)f, (long long)psi);
    }
    purify_plan(m, n, rows, cols, flows, costs, ha, hb, P.drop_rel, res.rows, res.cols, res.vals);
    // gauge z_{n-1} = 0 on the unscaled duals
    const double g = hz[n - 1] / zeta;
    res.y.resize(m);
    res.z.resize(n);
    for (int i = 0; i < m; ++i) res.y[i] = hy[i] / zeta + g;
    for (int j = 0; j < n; ++j) res.z[j] = hz[j] / zeta - g;
    // compensated sums on the host
    auto ksum = [](const std::vector<double> &v) {
        double s = 0.0, c = 0.0;
        for (double x : v) {
            const double t = s + x;
            c += (std::fabs(s) >= std::fabs(x)) ? (s - t) + x : (x - t) + s;
            s = t;
        }
        return s + c;
    };
    std::vector<double> terms;
    terms.reserve(res.vals.size());
    for (size_t k = 0; k < res.vals.size(); ++k)
        terms.push_back(icost(res.rows[k], res.cols[k]) * res.vals[k]);
    const double obj = ksum(terms);
    const double suma = ksum(ha);
    double *yu = yun.need(m), *zu = zun.need(n);
    // certified bound a.y + b.z + sum(a) min(0, min_ij r_ij) of a dual pair
    auto bound = [&](const std::vector<double> &yy, const std::vector<double> &zz, double &rmin) {
        OTIP_HIP(hipMemcpyAsync(yu, yy.data(), sizeof(double) * m, hipMemcpyHostToDevice, st));
        OTIP_HIP(hipMemcpyAsync(zu, zz.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
        double t0 = now();
        int64_t arg = 0;
        scan.rmin(st, m, n, xs, xt, yu, zu, &rmin, &arg);
        t_pricing += now() - t0;
        std::vector<double> dt;
        dt.reserve((size_t)m + n);
        for (int i = 0; i < m; ++i) dt.push_back(ha[i] * yy[i]);
        for (int j = 0; j < n; ++j) dt.push_back(hb[j] * zz[j]);
        return ksum(dt) + suma * std::min(0.0, rmin);
    };
    double rmin = 0.0;
    double dual = bound(res.y, res.z, rmin);
    // duals of the basic plan: y_i + z_j = C_ij on its (forest) edges, each
    // tree anchored at the interior-point dual of its smallest node; kept when
    // their certificate is the stronger one
    {
        std::vector<std::vector<std::pair<int, int>>> adj((size_t)m + n);
        for (size_t k = 0; k < res.vals.size(); ++k) {
            adj[res.rows[k]].push_back({m + res.cols[k], (int)k});
            adj[m + res.cols[k]].push_back({res.rows[k], (int)k});
        }
        std::vector<double> pot((size_t)m + n, 0.0);
        std::vector<char> seen((size_t)m + n, 0);
        for (int r = 0; r < m + n; ++r) {
            if (seen[r]) continue;
            seen[r] = 1;
            pot[r] = r < m ? res.y[r] : res.z[r - m];
            std::vector<int> stack{r};
            while (!stack.empty()) {
                const int u = stack.back();
                stack.pop_back();
                for (auto [v, k] : adj[u])
                    if (!seen[v]) {
                        seen[v] = 1;
                        pot[v] = icost(res.rows[k], res.cols[k]) - pot[u];
                        stack.push_back(v);
                    }
            }
        }
        const double g2 = pot[m + n - 1];
        std::vector<double> yb(m), zb(n);
        for (int i = 0; i < m; ++i) yb[i] = pot[i] + g2;
        for (int j = 0; j < n; ++j) zb[j] = pot[m + j] - g2;
        double rmin_b = 0.0;
        const double dual_b = bound(yb, zb, rmin_b);
        if (dual_b > dual) {
            dual = dual_b;
            rmin = rmin_b;
            res.y.swap(yb);
            res.z.swap(zb);
        }
    }
    std::vector<double> rs(m, 0.0), cs(n, 0.0);
    for (size_t k = 0; k < res.vals.size(); ++k) {
        rs[res.rows[k]] += res.vals[k];
        cs[res.cols[k]] += res.vals[k];
    }
    double num = 0.0, den = 0.0;
    for (int i = 0; i < m; ++i) {
        num += std::fabs(rs[i] - ha[i]);
        den += std::fabs(ha[i]);
    }
    for (int j = 0; j < n; ++j) {
        num += std::fabs(cs[j] - hb[j]);
        den += std::fabs(hb[j]);
    }
    res.info.nnz = (int64_t)res.vals.size();
    res.info.objective = obj;
    res.info.dual_bound = dual;
    res.info.rel_gap = (obj - dual) / std::max(1.0, std::fabs(obj));
    res.info.marginal_residual = num / den;
    res.info.r_min = rmin;
}


int64_t Solver::schur_export(int m_, int n_, int64_t psi, const uint64_t *idx_in,
                             const double *theta_in, int32_t *rowptr, int32_t *colidx,
                             double *vals, double *Mout, double *Nout) {
    m = m_;
    n = n_;
    OTIP_CHECK(m >= 1 && n >= 1 && psi >= 1, OTIP_EINVAL, "schur: bad sizes");
    // the views need coordinates only for costs; use a zero coordinate table
    DBuf<int32_t> &zc = zc_;
    const int mx = std::max(m, n);
    OTIP_HIP(hipMemsetAsync(zc.need((size_t)2 * mx), 0, sizeof(int32_t) * 2 * mx, st));
    xs = zc.get();
    xt = zc.get();
    zeta = 1.0;
    {
        // the support must be sorted, duplicate-free and cover every row and column
        std::vector<uint64_t> h(psi);
        OTIP_HIP(hipMemcpyAsync(h.data(), idx_in, sizeof(uint64_t) * psi, hipMemcpyDeviceToHost, st));
        OTIP_HIP(hipStreamSynchronize(st));
        std::vector<char> rc((size_t)m, 0), cc((size_t)n, 0);
        for (int64_t k = 0; k < psi; ++k) {
            OTIP_CHECK(h[k] < (uint64_t)m * (uint64_t)n && (k == 0 || h[k] > h[k - 1]), OTIP_EINVAL,
                       "schur: support must be sorted, unique and in range");
            rc[h[k] % (uint64_t)m] = 1;
            cc[h[k] / (uint64_t)m] = 1;
        }
        for (int i = 0; i < m; ++i) OTIP_CHECK(rc[i], OTIP_EINVAL, "schur: a row is not covered");
        for (int j = 0; j < n; ++j) OTIP_CHECK(cc[j], OTIP_EINVAL, "schur: a column is not covered");
    }
    alloc_support(psi);
    OTIP_HIP(hipMemcpyAsync(idx.get(), idx_in, sizeof(uint64_t) * psi, hipMemcpyDeviceToDevice, st));
    psi_ = psi;
    rebuild_views();
    OTIP_HIP(hipMemcpyAsync(theta.get(), theta_in, sizeof(double) * psi, hipMemcpyDeviceToDevice, st));
    M.need(m);
    invM.need(m);
    N.need(n);
    rowsum(theta.get(), nullptr, M.get(), 1.0);
    colsum(theta.get(), nullptr, N.get(), 1.0);
    foreach(st, m, FInv{M.get(), invM.get()});
    schur.symbolic(st, m, n, psi_, col_ptr.get(), si.get(), row_ptr.get(), csr_pos.get(), sj.get());
    schur.numeric(st, m, n, col_ptr.get(), si.get(), row_ptr.get(), csr_pos.get(), sj.get(),
                  theta.get(), invM.get());
    const int64_t nnz = schur.S.nnz;
    if (rowptr) {
        OTIP_HIP(hipMemcpyAsync(rowptr, schur.S.rowptr.get(), sizeof(int32_t) * (n + 1),
                                hipMemcpyDeviceToDevice, st));
        OTIP_HIP(hipMemcpyAsync(colidx, schur.S.col.get(), sizeof(int32_t) * nnz,
                                hipMemcpyDeviceToDevice, st));
        OTIP_HIP(hipMemcpyAsync(vals, schur.S.val.get(), sizeof(double) * nnz,
                                hipMemcpyDeviceToDevice, st));
        if (Mout) OTIP_HIP(hipMemcpyAsync(Mout, M.get(), sizeof(double) * m, hipMemcpyDeviceToDevice, st));
        if (Nout) OTIP_HIP(hipMemcpyAsync(Nout, N.get(), sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    }
    OTIP_HIP(hipStreamSynchronize(st));
    return nnz;
}

}  // namespace otip
