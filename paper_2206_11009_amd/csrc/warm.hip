// Initial support from predicted duals (a warm start of the initial support
// rule of Section 3.2, end).  Given dual estimates y0, z0 (cost units):
//   1. c-transform: z_j = min_i (C_ij - y0_i), then y_i = min_j (C_ij - z_j).
//      The pair is dual feasible (every reduced cost >= 0 up to rounding) and
//      every row and column has a zero reduced cost.
//   2. take the variables whose reduced cost r_ij = (C_ij - y_i) - z_j lies
//      below the smallest 2-digit (24-bit) key-prefix boundary that holds at
//      least kappa*(m+n-1) of them, plus the reduced-cost argmin of every row
//      and column (so that every row and column is covered).
// The result is a sorted, duplicate-free list of variable indices i + j*m.
#include "internal.h"

namespace otip {

namespace {

constexpr int kWB = 256;
constexpr int kWBins = 4096;

// C_ij of a cost kind (Section 5.1) from the integer offset d = x_i - x_j:
// |d| <= 2^15, so d0^2 + d1^2 <= 2^31 and every integer here is an exact
// double; the 2-norm is its correctly rounded square root.
__device__ __forceinline__ double wcost(const int32_t *__restrict__ xs,
                                        const int32_t *__restrict__ xt, int i, int j, int kind) {
    const int64_t d0 = (int64_t)xs[2 * i] - xt[2 * j];
    const int64_t d1 = (int64_t)xs[2 * i + 1] - xt[2 * j + 1];
    const int64_t a0 = d0 < 0 ? -d0 : d0, a1 = d1 < 0 ? -d1 : d1;
    if (kind == OTIP_COST_L1) return (double)(a0 + a1);
    if (kind == OTIP_COST_LINF) return (double)max(a0, a1);
    const double q = (double)(d0 * d0 + d1 * d1);
    return kind == OTIP_COST_L2 ? __builtin_sqrt(q) : q;
}

// one block per column: z_j = min_i (C_ij - y_i)
__global__ __launch_bounds__(kWB) void ctrans_col(int m, int n, int kind, const int32_t *xs,
                                                  const int32_t *xt, const double *y,
                                                  double *z) {
    __shared__ double lds[kWB / 64];
    const int j = blockIdx.x;
    double best = INFINITY;
    for (int i = threadIdx.x; i < m; i += kWB) best = fmin(best, wcost(xs, xt, i, j, kind) - y[i]);
    best = wave_min(best);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kWB / 64; ++w) best = fmin(best, lds[w]);
        z[j] = best;
    }
}

// one block per row: y_i = min_j (C_ij - z_j) and its argmin (smallest j on ties)
__global__ __launch_bounds__(kWB) void ctrans_row(int m, int n, int kind, const int32_t *xs,
                                                  const int32_t *xt, const double *z, double *y,
                                                  uint64_t *cover) {
    __shared__ double sv[kWB];
    __shared__ int sa[kWB];
    const int i = blockIdx.x;
    double best = INFINITY;
    int arg = n;
    for (int j = threadIdx.x; j < n; j += kWB) {
        const double v = wcost(xs, xt, i, j, kind) - z[j];
        if (v < best) {
            best = v;
            arg = j;
        }
    }
    sv[threadIdx.x] = best;
    sa[threadIdx.x] = arg;
    __syncthreads();
    for (int h = kWB / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            const double v = sv[threadIdx.x + h];
            const int a2 = sa[threadIdx.x + h];
            if (v < sv[threadIdx.x] || (v == sv[threadIdx.x] && a2 < sa[threadIdx.x])) {
                sv[threadIdx.x] = v;
                sa[threadIdx.x] = a2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        y[i] = sv[0];
        if (cover) cover[i] = (uint64_t)i + (uint64_t)min(sa[0], n - 1) * (uint64_t)m;
    }
}

// one block per column: argmin_i r_ij (smallest i on ties)
__global__ __launch_bounds__(kWB) void rc_col_argmin(int m, int n, int kind, const int32_t *xs,
                                                     const int32_t *xt, const double *y,
                                                     const double *z, uint64_t *cover) {
    __shared__ double sv[kWB];
    __shared__ int sa[kWB];
    const int j = blockIdx.x;
    const double zj = z[j];
    double best = INFINITY;
    int arg = m;
    for (int i = threadIdx.x; i < m; i += kWB) {
        const double v = (wcost(xs, xt, i, j, kind) - y[i]) - zj;
        if (v < best) {
            best = v;
            arg = i;
        }
    }
    sv[threadIdx.x] = best;
    sa[threadIdx.x] = arg;
    __syncthreads();
    for (int h = kWB / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            const double v = sv[threadIdx.x + h];
            const int a2 = sa[threadIdx.x + h];
            if (v < sv[threadIdx.x] || (v == sv[threadIdx.x] && a2 < sa[threadIdx.x])) {
                sv[threadIdx.x] = v;
                sa[threadIdx.x] = a2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) cover[j] = (uint64_t)min(sa[0], m - 1) + (uint64_t)j * (uint64_t)m;
}

// histogram of 12-bit digit (key >> shift) of r's ordered key over the keys
// whose bits above shift+12 equal prefix; grid (row blocks, column tiles)
__global__ __launch_bounds__(kWB) void rc_hist(int m, int n, int kind, int tj, const int32_t *xs,
                                               const int32_t *xt, const double *y,
                                               const double *z, int shift, uint64_t prefix,
                                               unsigned long long *hist) {
    __shared__ unsigned int lh[kWBins];
    for (int t = threadIdx.x; t < kWBins; t += kWB) lh[t] = 0u;
    __syncthreads();
    const int i = blockIdx.x * kWB + threadIdx.x;
    const int j0 = blockIdx.y * tj, j1 = min(n, j0 + tj);
    const int pshift = shift + 12;
    if (i < m) {
        const double yi = y[i];
        for (int j = j0; j < j1; ++j) {
            const uint64_t key = dkey((wcost(xs, xt, i, j, kind) - yi) - z[j]);
            if (pshift >= 64 || (key >> pshift) == prefix)
                atomicAdd(&lh[(key >> shift) & 4095u], 1u);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kWBins; t += kWB)
        if (lh[t]) atomicAdd(&hist[t], (unsigned long long)lh[t]);
}

// per column: number of keys <= key_max
__global__ __launch_bounds__(kWB) void rc_count_col(int m, int n, int kind, const int32_t *xs,
                                                    const int32_t *xt, const double *y,
                                                    const double *z, uint64_t key_max,
                                                    int64_t *cnt) {
    __shared__ double lds[16];
    const int j = blockIdx.x;
    const double zj = z[j];
    int c = 0;
    for (int i = threadIdx.x; i < m; i += kWB)
        c += dkey((wcost(xs, xt, i, j, kind) - y[i]) - zj) <= key_max;
    const double t = block_sum((double)c, lds);
    if (threadIdx.x == 0) cnt[j] = (int64_t)t;
}

// per column: the variable indices with key <= key_max, increasing i
__global__ __launch_bounds__(kWB) void rc_collect_col(int m, int n, int kind, const int32_t *xs,
                                                      const int32_t *xt, const double *y,
                                                      const double *z, uint64_t key_max,
                                                      const int64_t *off, uint64_t *out) {
    __shared__ int wcount[kWB / 64];
    const int j = blockIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const double zj = z[j];
    int64_t base = off[j];
    for (int i0 = 0; i0 < m; i0 += kWB) {
        const int i = i0 + threadIdx.x;
        const bool take = i < m && dkey((wcost(xs, xt, i, j, kind) - y[i]) - zj) <= key_max;
        const uint64_t mask = __ballot(take);
        if (lane == 0) wcount[w] = __popcll(mask);
        __syncthreads();
        int before = 0, total = 0;
        for (int k = 0; k < kWB / 64; ++k) {
            if (k < w) before += wcount[k];
            total += wcount[k];
        }
        if (take)
            out[base + before + __popcll(mask & ((1ull << lane) - 1ull))] =
                (uint64_t)i + (uint64_t)j * (uint64_t)m;
        base += total;
        __syncthreads();
    }
}

// 1 if any entry is not finite
__global__ void nonfinite_flag(int64_t len, const double *v, int *flag) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < len && !isfinite(v[t])) atomicOr(flag, 1);
}

}  // namespace

void Scanner::ctransform_rows(hipStream_t st, int m, int n, const int32_t *xs, const int32_t *xt,
                              const double *z, double *y) {
    hipLaunchKernelGGL(ctrans_row, dim3(m), dim3(kWB), 0, st, m, n, kind, xs, xt, z, y,
                       (uint64_t *)nullptr);
    OTIP_HIP(hipGetLastError());
}

void Scanner::ctransform_cols(hipStream_t st, int m, int n, const int32_t *xs, const int32_t *xt,
                              const double *y, double *z) {
    hipLaunchKernelGGL(ctrans_col, dim3(n), dim3(kWB), 0, st, m, n, kind, xs, xt, y, z);
    OTIP_HIP(hipGetLastError());
}

int64_t Scanner::warm_support(hipStream_t st, int m, int n, const int32_t *xs, const int32_t *xt,
                              const double *y0, const double *z0, double kappa,
                              DBuf<uint64_t> &out, DBuf<double> &yw, DBuf<double> &zw) {
    // non-finite predictions: the caller falls back to the plain rule
    flag_.need(1);
    OTIP_HIP(hipMemsetAsync(flag_.get(), 0, sizeof(int), st));
    hipLaunchKernelGGL(nonfinite_flag, dim3(grid_for(m, 256)), dim3(256), 0, st, (int64_t)m, y0,
                       flag_.get());
    hipLaunchKernelGGL(nonfinite_flag, dim3(grid_for(n, 256)), dim3(256), 0, st, (int64_t)n, z0,
                       flag_.get());
    int bad = 0;
    OTIP_HIP(hipMemcpyAsync(&bad, flag_.get(), sizeof(int), hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipStreamSynchronize(st));
    if (bad) return -1;

    double *y = yw.need(m), *z = zw.need(n);
    DBuf<uint64_t> &cover = u64b_;
    cover.need((size_t)m + n);
    hipLaunchKernelGGL(ctrans_col, dim3(n), dim3(kWB), 0, st, m, n, kind, xs, xt, y0, z);
    hipLaunchKernelGGL(ctrans_row, dim3(m), dim3(kWB), 0, st, m, n, kind, xs, xt, z, y, cover.get());
    hipLaunchKernelGGL(rc_col_argmin, dim3(n), dim3(kWB), 0, st, m, n, kind, xs, xt, y, z,
                       cover.get() + m);
    OTIP_HIP(hipGetLastError());

    // threshold: two 12-bit digits of the ordered key
    const int64_t target = std::min<int64_t>((int64_t)std::ceil(kappa * (double)(m + n - 1)),
                                             (int64_t)m * (int64_t)n);
    const int tj = pick_tj(m, n, tile);
    dim3 grid(grid_for(m, kWB), grid_for(n, tj));
    hist_.need(kWBins);
    std::vector<unsigned long long> h(kWBins);
    uint64_t prefix = 0;
    int64_t cum = 0;
    for (int level = 0; level < 2; ++level) {
        const int shift = level == 0 ? 52 : 40;
        OTIP_HIP(hipMemsetAsync(hist_.get(), 0, kWBins * sizeof(unsigned long long), st));
        hipLaunchKernelGGL(rc_hist, grid, dim3(kWB), 0, st, m, n, kind, tj, xs, xt, y, z, shift, prefix,
                           hist_.get());
        OTIP_HIP(hipGetLastError());
        OTIP_HIP(hipMemcpyAsync(h.data(), hist_.get(), kWBins * sizeof(unsigned long long),
                                hipMemcpyDeviceToHost, st));
        OTIP_HIP(hipStreamSynchronize(st));
        scans++;
        int b = 0;
        for (; b < kWBins - 1; ++b) {
            if (cum + (int64_t)h[b] >= target) break;
            cum += (int64_t)h[b];
        }
        prefix = (prefix << 12) | (uint64_t)b;
    }
    const uint64_t key_max = (prefix << 40) | ((1ull << 40) - 1ull);

    DBuf<int64_t> &cnt = i64a_;
    DBuf<int64_t> &off = i64b_;
    cnt.need((size_t)n);
    off.need((size_t)n + 1);
    hipLaunchKernelGGL(rc_count_col, dim3(n), dim3(kWB), 0, st, m, n, kind, xs, xt, y, z, key_max,
                       cnt.get());
    OTIP_HIP(hipGetLastError());
    exclusive_scan_i64(st, cnt.get(), off.get(), n, tmp_);
    int64_t last_off = 0, last_cnt = 0;
    OTIP_HIP(hipMemcpyAsync(&last_off, off.get() + (n - 1), sizeof(int64_t),
                            hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipMemcpyAsync(&last_cnt, cnt.get() + (n - 1), sizeof(int64_t),
                            hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipStreamSynchronize(st));
    const int64_t nle = last_off + last_cnt;
    // massive ties at the cut (e.g. constant predictions): use the plain rule
    if (nle > 16 * target + m + n) return -1;
    const int64_t tot = nle + m + n;
    DBuf<uint64_t> &tmpk = u64a_;
    tmpk.need((size_t)tot);
    hipLaunchKernelGGL(rc_collect_col, dim3(n), dim3(kWB), 0, st, m, n, kind, xs, xt, y, z, key_max,
                       off.get(), tmpk.get());
    OTIP_HIP(hipGetLastError());
    OTIP_HIP(hipMemcpyAsync(tmpk.get() + nle, cover.get(), sizeof(uint64_t) * (m + n),
                            hipMemcpyDeviceToDevice, st));
    DBuf<uint64_t> &sorted = ck_;
    sorted.need((size_t)tot);
    sort_keys_u64(st, tmpk.get(), sorted.get(), tot, tmp_);
    out.need((size_t)tot);
    return unique_u64(st, sorted.get(), out.get(), tot, tmp_, cnt_);
}

}  // namespace otip
