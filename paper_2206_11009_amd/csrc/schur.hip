// Schur complement of the normal equations restricted to the support and its
// preconditioned CG solve (Sections 3.5, 4 and 4.2).
//
// With vec(V) = theta on the support, M and N the row and column sums of V,
// S_M = N - V^T M^-1 V is n x n and has entry (j, k), j != k, equal to
// -sum over sources i adjacent to both j and k of theta_ij theta_ik / M_i.
// Its diagonal equals minus the sum of the off-diagonal entries of its row
// (eq. diagdom: the row sums of S_M vanish), which is how it is formed here:
// the direct form N_jj - sum_i theta_ij^2 / M_i cancels catastrophically when
// one entry dominates its row of V, as happens near optimality.
#include "internal.h"

namespace otip {

// ---------------------------------------------------------------- symbolic
// Row-ordered copies of the support's targets and weights: rk[t] =
// sj[csr_pos[t]] and rth[t] = theta[csr_pos[t]], so that the targets of a
// source (sorted) are read contiguously, without the permutation.
__global__ void pack_rows(int64_t psi, const int32_t *__restrict__ csr_pos,
                          const int32_t *__restrict__ sj, const double *__restrict__ theta,
                          int32_t *__restrict__ rk, double *__restrict__ rth) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < psi;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int q = csr_pos[t];
        if (rk) rk[t] = sj[q];
        if (rth) rth[t] = theta[q];
    }
}

__device__ __forceinline__ int wave_min_i(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double rdlane_d(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ void lds_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wave per S row j.  The union of the targets of all sources adjacent to j
// is marked in a per-wave LDS bitmap over [kmin, kmax]; the marked bits, read in
// order, are the sorted column indices of row j.  The sources of column j are
// read one per lane; their target lists kSrcGroup at a time, all loads in flight.
// sources whose target lists are requested together before any is applied
// (their loads overlap; the order of application is unchanged)
constexpr int kSrcGroup = 16;

template <bool FILL>
__global__ __launch_bounds__(64) void schur_pattern(int n, const int32_t *__restrict__ col_ptr,
                                                    const int32_t *__restrict__ si,
                                                    const int32_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ rk,
                                                    int32_t *__restrict__ cnt,
                                                    const int32_t *__restrict__ rowptr,
                                                    int32_t *__restrict__ col,
                                                    int32_t *__restrict__ row,
                                                    int32_t *__restrict__ diag) {
    extern __shared__ uint32_t bits[];
    const int j = blockIdx.x;
    const int lane = threadIdx.x;
    const int c0 = col_ptr[j], c1 = col_ptr[j + 1];
    int kmin = n, kmax = -1;
    for (int e = c0 + lane; e < c1; e += 64) {
        const int i = si[e];
        const int r0 = row_ptr[i], r1 = row_ptr[i + 1];
        kmin = min(kmin, rk[r0]);
        kmax = max(kmax, rk[r1 - 1]);
    }
    kmin = wave_min_i(kmin);
    kmax = wave_max_i(kmax);
    const int w0 = kmin >> 5, w1 = kmax >> 5;
    for (int w = w0 + lane; w <= w1; w += 64) bits[w - w0] = 0u;
    __syncthreads();
    for (int e0 = c0; e0 < c1; e0 += 64) {
        int r0l = 0, r1l = 0;
        if (e0 + lane < c1) {
            const int i = si[e0 + lane];
            r0l = row_ptr[i];
            r1l = row_ptr[i + 1];
        }
        const int ns = min(64, c1 - e0);
        for (int s0 = 0; s0 < ns; s0 += kSrcGroup) {
            int k[kSrcGroup];
#pragma unroll
            for (int u = 0; u < kSrcGroup; ++u) {
                const int sl = min(s0 + u, ns - 1);
                const int r = __builtin_amdgcn_readlane(r0l, sl) + lane;
                k[u] = (s0 + u < ns && r < __builtin_amdgcn_readlane(r1l, sl)) ? rk[r] : -1;
            }
#pragma unroll
            for (int u = 0; u < kSrcGroup; ++u) {
                if (k[u] >= 0) atomicOr(&bits[(k[u] >> 5) - w0], 1u << (k[u] & 31));
                if (s0 + u < ns) {  // sources with more than 64 targets
                    const int r1 = __builtin_amdgcn_readlane(r1l, s0 + u);
                    for (int r = __builtin_amdgcn_readlane(r0l, s0 + u) + 64 + lane; r < r1;
                         r += 64)
                        atomicOr(&bits[(rk[r] >> 5) - w0], 1u << (rk[r] & 31));
                }
            }
        }
    }
    __syncthreads();
    if (!FILL) {
        int c = 0;
        for (int w = w0 + lane; w <= w1; w += 64) c += __popc(bits[w - w0]);
        c = wave_sum_i(c);
        if (lane == 0) {
            cnt[j] = c;
            atomicMax(&cnt[n], kmax - kmin + 1);  // the widest row's column span
        }
        return;
    }
    int base = rowptr[j];
    for (int wb = w0; wb <= w1; wb += 64) {
        const int w = wb + lane;
        uint32_t word = (w <= w1) ? bits[w - w0] : 0u;
        int pc = __popc(word);
        // inclusive prefix over the wave
        int incl = pc;
        for (int o = 1; o < 64; o <<= 1) {
            int t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        int pos = base + incl - pc;
        while (word) {
            const int b = __ffs(word) - 1;
            word &= word - 1u;
            const int k = (w << 5) + b;
            col[pos] = k;
            row[pos] = j;
            if (k == j) diag[j] = pos;
            ++pos;
        }
        base += __shfl(incl, 63, 64);
    }
}

__global__ void counts_to_i64(int n, const int32_t *c, int64_t *o) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) o[t] = c[t];
}
__global__ void i64_to_rowptr(int n, const int64_t *off, const int32_t *c, int32_t *rowptr) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) rowptr[t] = (int32_t)off[t];
    if (t == n - 1) rowptr[n] = (int32_t)(off[t] + c[t]);
}

void SchurSolver::symbolic(hipStream_t st, int m, int n, int64_t psi, const int32_t *col_ptr,
                           const int32_t *si, const int32_t *row_ptr, const int32_t *csr_pos,
                           const int32_t *sj) {
    const int words = (n + 31) / 32 + 1;
    OTIP_CHECK(words * 4 <= 64 * 1024, 6, "Schur pattern: n too large for the LDS bitmap");
    S.n = n;
    cnt_.need((size_t)n + 1);
    OTIP_HIP(hipMemsetAsync(cnt_.get() + n, 0, sizeof(int32_t), st));
    rk_.need((size_t)std::max<int64_t>(psi, 1));
    hipLaunchKernelGGL(pack_rows, dim3(std::min<unsigned>(4096, grid_for(psi, 256))), dim3(256), 0,
                       st, psi, csr_pos, sj, nullptr, rk_.get(), nullptr);
    hipLaunchKernelGGL(schur_pattern<false>, dim3(n), dim3(64), words * 4, st, n, col_ptr, si,
                       row_ptr, rk_.get(), cnt_.get(), nullptr, nullptr, nullptr, nullptr);
    OTIP_HIP(hipGetLastError());
    cnt64_.need((size_t)n);
    off64_.need((size_t)n);
    hipLaunchKernelGGL(counts_to_i64, dim3(grid_for(n, 256)), dim3(256), 0, st, n, cnt_.get(),
                       cnt64_.get());
    exclusive_scan_i64(st, cnt64_.get(), off64_.get(), n, tmp_);
    S.rowptr.need((size_t)n + 1);
    hipLaunchKernelGGL(i64_to_rowptr, dim3(grid_for(n, 256)), dim3(256), 0, st, n, off64_.get(),
                       cnt_.get(), S.rowptr.get());
    int32_t nnz = 0;
    OTIP_HIP(hipMemcpyAsync(&nnz, S.rowptr.get() + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipMemcpyAsync(&span_, cnt_.get() + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipStreamSynchronize(st));
    OTIP_CHECK(span_ >= 1 && span_ <= n, 5, "Schur pattern: bad column span");
    OTIP_CHECK(nnz >= n, 5, "Schur pattern: missing diagonal");
    S.nnz = nnz;
    S.col.need((size_t)nnz);
    S.row.need((size_t)nnz);
    S.diag.need((size_t)n);
    S.val.need((size_t)nnz);
    S.dinv.need((size_t)n);
    hipLaunchKernelGGL(schur_pattern<true>, dim3(n), dim3(64), words * 4, st, n, col_ptr, si,
                       row_ptr, rk_.get(), nullptr, S.rowptr.get(), S.col.get(), S.row.get(),
                       S.diag.get());
    psi_ = psi;
    OTIP_HIP(hipGetLastError());
}

void SchurSolver::keep_pattern(hipStream_t st, int64_t psi, const int32_t *csr_pos,
                               const int32_t *sj) {
    OTIP_CHECK(psi >= 1 && psi <= psi_, OTIP_EINVAL, "Schur pattern reuse: support grew");
    hipLaunchKernelGGL(pack_rows, dim3(std::min<unsigned>(4096, grid_for(psi, 256))), dim3(256), 0,
                       st, psi, csr_pos, sj, nullptr, rk_.get(), nullptr);
    OTIP_HIP(hipGetLastError());
    psi_ = psi;
}

// ---------------------------------------------------------------- numeric
// Off-diagonal entries by intersecting the (i-sorted) source lists of targets j
// and k.  The product theta_ij * theta_ik is commutative, so S is exactly
// symmetric; each entry is summed in increasing i (deterministic).
__global__ void schur_offdiag(int64_t nnz, const int32_t *__restrict__ srow,
                              const int32_t *__restrict__ scol,
                              const int32_t *__restrict__ col_ptr, const int32_t *__restrict__ si,
                              const double *__restrict__ theta, const double *__restrict__ invM,
                              double *__restrict__ val) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    const int j = srow[e], k = scol[e];
    if (j == k) {
        val[e] = 0.0;
        return;
    }
    int a = col_ptr[j], ae = col_ptr[j + 1];
    int b = col_ptr[k], be = col_ptr[k + 1];
    double acc = 0.0;
    while (a < ae && b < be) {
        const int ia = si[a], ib = si[b];
        if (ia == ib) {
            acc = fma(theta[a] * theta[b], invM[ia], acc);
            ++a;
            ++b;
        } else if (ia < ib) {
            ++a;
        } else {
            ++b;
        }
    }
    val[e] = -acc;
}

// Off-diagonal values by rows, for n <= kRowAccMax: one wavefront per row j of
// S accumulates sum_i theta_ij theta_ik / M_i into a dense LDS row (over the
// widest column span of any row, so that many rows fit a compute unit) over the
// sources i of column j in increasing i (each source's targets k are distinct,
// and successive sources are ordered by the wave's program order), then
// gathers the row's pattern.  Same products and summation order as
// schur_offdiag, so the values are identical; the work is
// sum_j sum_{i in col j} deg(i) instead of a merge per nonzero.  The sources'
// data are read one per lane and their row-ordered targets and weights (rk,
// rth) kSrcGroup sources at a time, before they are accumulated in order.
constexpr int kRowAccMax = 8192;

__global__ __launch_bounds__(64) void schur_offdiag_rows(
    int n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ scol,
    const int32_t *__restrict__ col_ptr, const int32_t *__restrict__ si,
    const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ rk,
    const double *__restrict__ rth, const double *__restrict__ theta,
    const double *__restrict__ invM, double *__restrict__ val) {
    extern __shared__ double acc[];
    const int j = blockIdx.x, l = threadIdx.x;
    const int e0 = rowptr[j], e1 = rowptr[j + 1];
    // the row's columns are sorted and span at most the LDS row: k at k - kb
    const int kb = scol[e0];
    for (int e = e0 + l; e < e1; e += 64) acc[scol[e] - kb] = 0.0;
    __syncthreads();
    const int c0 = col_ptr[j], c1 = col_ptr[j + 1];
    for (int a0 = c0; a0 < c1; a0 += 64) {
        int r0l = 0, r1l = 0;
        double tml = 0.0, iml = 0.0;
        if (a0 + l < c1) {
            const int i = si[a0 + l];
            r0l = row_ptr[i];
            r1l = row_ptr[i + 1];
            tml = theta[a0 + l];
            iml = invM[i];
        }
        const int ns = min(64, c1 - a0);
        for (int s0 = 0; s0 < ns; s0 += kSrcGroup) {
            int k[kSrcGroup];
            double th[kSrcGroup];
#pragma unroll
            for (int u = 0; u < kSrcGroup; ++u) {
                const int sl = min(s0 + u, ns - 1);
                const int r = __builtin_amdgcn_readlane(r0l, sl) + l;
                const bool ok = s0 + u < ns && r < __builtin_amdgcn_readlane(r1l, sl);
                k[u] = ok ? rk[r] : -1;
                th[u] = ok ? rth[r] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kSrcGroup; ++u) {
                if (s0 + u >= ns) break;
                const int sl = s0 + u;
                const double ta = rdlane_d(tml, sl), im = rdlane_d(iml, sl);
                if (k[u] >= 0) acc[k[u] - kb] = fma(ta * th[u], im, acc[k[u] - kb]);
                // sources with more than 64 targets: the rest, still before the
                // next source
                const int r1 = __builtin_amdgcn_readlane(r1l, sl);
                for (int r = __builtin_amdgcn_readlane(r0l, sl) + 64 + l; r < r1; r += 64)
                    acc[rk[r] - kb] = fma(ta * rth[r], im, acc[rk[r] - kb]);
                lds_wave_sync();
            }
        }
    }
    __syncthreads();
    for (int e = e0 + l; e < e1; e += 64) {
        const int k = scol[e];
        val[e] = (k == j) ? 0.0 : -acc[k - kb];
    }
}

// one wave per row: S_jj = -(sum of the row's off-diagonal entries)
__global__ __launch_bounds__(256) void schur_diag(int n, const int32_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ diag,
                                                  double *__restrict__ val,
                                                  double *__restrict__ dinv) {
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int l = threadIdx.x & 63;
    if (j >= n) return;
    const int d = diag[j];
    double s = 0.0;
    for (int e = rowptr[j] + l; e < rowptr[j + 1]; e += 64)
        if (e != d) s += val[e];
    s = wave_sum(s);
    if (l == 0) {
        val[d] = -s;
        dinv[j] = (-s > 0.0) ? 1.0 / (-s) : 0.0;
    }
}

void SchurSolver::numeric(hipStream_t st, int m, int n, const int32_t *col_ptr,
                          const int32_t *si, const int32_t *row_ptr, const int32_t *csr_pos,
                          const int32_t *sj, const double *theta, const double *invM) {
    if (n <= kRowAccMax) {
        // the targets rk of this support were packed by symbolic()
        rth_.need((size_t)std::max<int64_t>(psi_, 1));
        hipLaunchKernelGGL(pack_rows, dim3(std::min<unsigned>(4096, grid_for(psi_, 256))),
                           dim3(256), 0, st, psi_, csr_pos, sj, theta, nullptr, rth_.get());
        hipLaunchKernelGGL(schur_offdiag_rows, dim3(n), dim3(64), sizeof(double) * span_, st, n,
                           S.rowptr.get(), S.col.get(), col_ptr, si, row_ptr, rk_.get(),
                           rth_.get(), theta, invM, S.val.get());
    } else
        hipLaunchKernelGGL(schur_offdiag, dim3(grid_for(S.nnz, 256)), dim3(256), 0, st, S.nnz,
                           S.row.get(), S.col.get(), col_ptr, si, theta, invM, S.val.get());
    hipLaunchKernelGGL(schur_diag, dim3(grid_for(n, 4)), dim3(256), 0, st, n, S.rowptr.get(),
                       S.diag.get(), S.val.get(), S.dinv.get());
    OTIP_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- SpMV + CG
constexpr int kCGBlocks = 256;
constexpr int kCGThreads = 256;
constexpr int kSpmvMaxBlocks = 4096;
constexpr int kSpmvDirBlocks = 768;

// G lanes per row; rows distributed round-robin over a fixed grid.  If
// partial, partial[block] = sum over the block's rows of x_j * y_j (in FP64).
// T is the storage type of the values and vectors (double, or float for the
// inner solves of the mixed-precision mode).
template <int G, typename T>
__global__ __launch_bounds__(256) void spmv_rows(int n, const int32_t *__restrict__ rowptr,
                                                 const int32_t *__restrict__ col,
                                                 const T *__restrict__ val,
                                                 const T *__restrict__ x, T *__restrict__ y,
                                                 double *partial) {
    __shared__ double lds[16];
    const int groups = 256 / G;
    const int g = threadIdx.x / G, l = threadIdx.x % G;
    double dot = 0.0;
    for (int r = blockIdx.x * groups + g; r < n; r += gridDim.x * groups) {
        T acc = (T)0;
        const int e1 = rowptr[r + 1];
        int e = rowptr[r] + l;
        for (; e + 3 * G < e1; e += 4 * G) {
            const int c0 = col[e], c1 = col[e + G], c2 = col[e + 2 * G], c3 = col[e + 3 * G];
            const T v0 = val[e], v1 = val[e + G], v2 = val[e + 2 * G], v3 = val[e + 3 * G];
            const T x0 = x[c0], x1 = x[c1], x2 = x[c2], x3 = x[c3];
            acc = fma(v0, x0, acc);
            acc = fma(v1, x1, acc);
            acc = fma(v2, x2, acc);
            acc = fma(v3, x3, acc);
        }
        for (; e < e1; e += G) acc = fma(val[e], x[col[e]], acc);
        for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
        if (l == 0) {
            y[r] = acc;
            dot = fma((double)x[r], (double)acc, dot);
        }
    }
    if (partial) {
        double t = block_sum(dot, lds);
        if (threadIdx.x == 0) partial[blockIdx.x] = t;
    }
}

// Jacobi-preconditioned CG in the single-reduction form of Chronopoulos and
// Gear (mathematically the same iterates as CG), one launch per iteration.
// With u = D^-1 r and w = S u:
//   gamma_i = r_i.u_i, delta_i = w_i.u_i, beta_i = gamma_i / gamma_{i-1},
//   alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_{i-1})  (beta_0 = 0),
//   p_i = u_i + beta_i p_{i-1}, s_i = w_i + beta_i s_{i-1}  (s_i = S p_i),
//   x_{i+1} = x_i + alpha_i p_i, r_{i+1} = r_i - alpha_i s_i.
// All three dot products of an iteration come from one reduction, so the
// launch that forms w_{i+1} = S u_{i+1} also applies the updates: every
// workgroup sums the previous launch's partials in the same order (the same
// alpha_i and beta_i everywhere), and u_{i+1} of a neighbour row is formed
// where the SpMV gathers that row's (r_i, w_i, s_{i-1}, d).

// Device-side CG scalars.  gamma and alpha (single-reduction form) and rho
// (two-launch form) are double-buffered by launch parity: a launch reads its
// predecessor's at [par ^ 1] in every workgroup, and workgroup 0 writes its
// own at [par].
struct CGScal {
    double gam[2], alpha[2], rho[2], rr, target, its;
};

// fixed-order sum of nb per-block partials, computed by wave 0 and broadcast
__device__ __forceinline__ double sum_partials(const double *p, int nb, double *lds) {
    if (threadIdx.x < 64) {
        double s = 0.0;
        for (int k = threadIdx.x; k < nb; k += 64) s += p[k];
        s = wave_sum(s);
        if (threadIdx.x == 0) lds[0] = s;
    }
    __syncthreads();
    const double v = lds[0];
    __syncthreads();
    return v;
}

// The device flag *f as one value for the whole workgroup.  Workgroup 0 of
// the same launch may set it while other workgroups read it; read once and
// broadcast, every wave of a workgroup takes the same branch, so none leaves
// while the others wait at a barrier or read its partial sum.
__device__ __forceinline__ int block_flag(const int *f, double *lds) {
    if (threadIdx.x == 0) lds[15] = (double)*f;
    __syncthreads();
    const int v = (int)lds[15];
    __syncthreads();
    return v;
}

// the three partial sums of a launch (gamma, delta, r.r: kSpmvMaxBlocks slots
// apart), one per wavefront in parallel, each in the fixed order of
// sum_partials; broadcast to the workgroup
// (and the device flag *f, read once by the fourth wave and returned to all)
__device__ __forceinline__ int sum_partials3(const double *p, int nb, double *lds,
                                             double (&out)[3], const int *f) {
    const int wv = threadIdx.x >> 6;
    if (wv < 3) {
        const double *q = p + wv * kSpmvMaxBlocks;
        double s = 0.0;
        for (int k = threadIdx.x & 63; k < nb; k += 64) s += q[k];
        s = wave_sum(s);
        if ((threadIdx.x & 63) == 0) lds[wv] = s;
    } else if (threadIdx.x == 192) {
        lds[3] = (double)*f;
    }
    __syncthreads();
    out[0] = lds[0];
    out[1] = lds[1];
    out[2] = lds[2];
    const int flag = (int)lds[3];
    __syncthreads();
    return flag;
}

// One row's state as the next launch gathers it: r_i, w_i, s_{i-1} and the
// Jacobi inverse d, double-buffered by launch parity.
template <typename T>
struct __attribute__((aligned(4 * sizeof(T)))) RWS {
    T r, w, s, d;
};

// s_i = w_i + beta s_{i-1} and r_{i+1} = r_i - alpha s_i of one row, in the one
// order used both by the row's owner and where its u_{i+1} = d r_{i+1} is
// gathered
template <typename T>
__device__ __forceinline__ T next_r(const RWS<T> &q, T alpha, T beta, T &s) {
    s = fma(beta, q.s, q.w);
    return fma(-alpha, s, q.r);
}

// partial-sum slots of one launch: gamma, delta, r.r, kSpmvMaxBlocks each
constexpr int kCGPart = 3 * kSpmvMaxBlocks;

// the state the first launch gathers: r = b, w = s = 0, d = D^-1
template <typename T>
__global__ __launch_bounds__(kCGThreads) void cg_init(int n, const T *__restrict__ b,
                                                      const T *__restrict__ dinv,
                                                      RWS<T> *__restrict__ g) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x)
        g[j] = RWS<T>{b[j], (T)0, (T)0, dinv[j]};
}

// after the first launch: the target from |b| and the done flag
__global__ __launch_bounds__(64) void cg_init_finish(int nb, const double *part, double rtol,
                                                     double atol, CGScal *sc, int *done) {
    __shared__ double lds[2];
    const double rr = sum_partials(part + 2 * kSpmvMaxBlocks, nb, lds);
    if (threadIdx.x == 0) {
        const double target = fmin(rtol * sqrt(rr), atol);
        sc->rr = rr;
        sc->target = target;
        sc->its = 0.0;
        *done = (sqrt(rr) <= target || rr == 0.0) ? 1 : 0;
    }
}

// Entries e, e + G, ..., e + (kSpmvU - 1) G of a row ending at e1 (those past
// the end get column -1): columns and values, then the gathered row states.
// Four at a time: a gathered state is four values, and eight kept the kernel
// at over 200 VGPRs (two waves per SIMD).
constexpr int kSpmvU = 4;
template <int G, bool NT, typename T>
__device__ __forceinline__ void load_chunk(int e, int e1, const int32_t *__restrict__ col,
                                           const T *__restrict__ val,
                                           const RWS<T> *__restrict__ gold, int (&c)[kSpmvU],
                                           T (&v)[kSpmvU], RWS<T> (&w)[kSpmvU]) {
#pragma unroll
    for (int k = 0; k < kSpmvU; ++k) {
        const int ek = e + k * G;
        if (ek < e1) {
            c[k] = NT ? __builtin_nontemporal_load(col + ek) : col[ek];
            v[k] = NT ? __builtin_nontemporal_load(val + ek) : val[ek];
        } else {
            c[k] = -1;
            v[k] = (T)0;
        }
    }
#pragma unroll
    for (int k = 0; k < kSpmvU; ++k)
        w[k] = c[k] >= 0 ? gold[c[k]] : RWS<T>{(T)0, (T)0, (T)0, (T)0};
}

// One launch of the iteration.  mode 0: the start (alpha = beta = 0: x = 0,
// r_0 = b, w_0 = S u_0 and its partials); mode 1: the first iteration
// (beta = 0); mode 2: the others.  From the predecessor's partials pin:
// gamma_i, delta_i and r_i.r_i (the convergence test), then alpha_i and beta_i.
// G lanes per row; each lane takes its entries e, e + G, ... kSpmvU at a
// time, all their loads in flight together (the summation order is that of
// one entry at a time).  The first chunk is requested before the partials
// are summed, and each row's first chunk and the next row's pointers before
// the previous row's lane reduction.  NT: the matrix streams past the caches
// (nontemporal loads); the launcher takes this form for cache-resident
// matrices only (NT false), larger ones take the two-launch form below.
template <int G, bool NT, typename T>
__global__ __launch_bounds__(256) void cg_step(int n, const int32_t *__restrict__ rowptr,
                                               const int32_t *__restrict__ col,
                                               const T *__restrict__ val,
                                               const RWS<T> *__restrict__ gold,
                                               RWS<T> *__restrict__ gnew, T *__restrict__ x,
                                               T *__restrict__ p, int nbp,
                                               const double *__restrict__ pin,
                                               double *__restrict__ pout, CGScal *sc, int *done,
                                               int mode, int par) {
    __shared__ double lds[16];
    const int groups = 256 / G;
    const int g = threadIdx.x / G, l = threadIdx.x % G;
    const int stride = gridDim.x * groups;
    int r = blockIdx.x * groups + g;
    int e = 0, e1 = 0, en = 0, en1 = 0;
    if (r < n) {
        e = rowptr[r] + l;
        e1 = rowptr[r + 1];
    }
    if (r + stride < n) {
        en = rowptr[r + stride] + l;
        en1 = rowptr[r + stride + 1];
    }
    int c[kSpmvU];
    T v[kSpmvU];
    RWS<T> w[kSpmvU];
    load_chunk<G, NT>(e, e1, col, val, gold, c, v, w);
    T alpha = (T)0, beta = (T)0;
    // the row's own state, x and p, requested with its first chunk
    RWS<T> own{};
    T xo = (T)0, po = (T)0;
    if (l == 0 && r < n) {
        own = gold[r];
        if (mode != 0) {
            xo = x[r];
            po = p[r];
        }
    }
    if (mode != 0) {
        double sums[3];
        if (sum_partials3(pin, nbp, lds, sums, done)) return;
        const double gam = sums[0], del = sums[1], rr = sums[2];
        const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
        if (sqrt(rr) <= sc->target || rr == 0.0) {
            if (lead) {
                sc->rr = rr;
                *done = 1;
            }
            return;
        }
        const double b64 = mode == 1 ? 0.0 : gam / sc->gam[par ^ 1];
        const double den = mode == 1 ? del : del - b64 * gam / sc->alpha[par ^ 1];
        if (!(den > 0.0)) {  // breakdown (S is positive semidefinite)
            if (lead) {
                sc->rr = rr;
                *done = 2;
            }
            return;
        }
        const double a64 = gam / den;
        alpha = (T)a64;
        beta = (T)b64;
        if (lead) {
            sc->gam[par] = gam;
            sc->alpha[par] = a64;
            sc->rr = rr;
            sc->its += 1.0;
        }
    }
    double dg = 0.0, dd = 0.0, dr = 0.0;
    while (r < n) {
        T acc = (T)0;
        for (;;) {
#pragma unroll
            for (int k = 0; k < kSpmvU; ++k) {
                T sk;
                const T uk = w[k].d * next_r(w[k], alpha, beta, sk);
                if (c[k] >= 0) acc = fma(v[k], uk, acc);
            }
            e += kSpmvU * G;
            if (e >= e1) break;
            load_chunk<G, NT>(e, e1, col, val, gold, c, v, w);
        }
        const int rc = r;
        const RWS<T> cur = own;
        const T xc = xo, pc = po;
        r += stride;
        e = en;
        e1 = en1;
        if (r < n) {
            load_chunk<G, NT>(e, e1, col, val, gold, c, v, w);
            if (l == 0) {
                own = gold[r];
                if (mode != 0) {
                    xo = x[r];
                    po = p[r];
                }
            }
            if (r + stride < n) {
                en = rowptr[r + stride] + l;
                en1 = rowptr[r + stride + 1];
            }
        }
        for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
        if (l == 0) {
            // p_i = u_i + beta p_{i-1} (the start leaves p = u_0; x = 0)
            const T pj = fma(beta, pc, cur.d * cur.r);
            T sj;
            const T rn = next_r(cur, alpha, beta, sj);
            const T un = cur.d * rn;
            x[rc] = mode == 0 ? (T)0 : fma(alpha, pj, xc);
            p[rc] = pj;
            gnew[rc] = RWS<T>{rn, acc, sj, cur.d};
            dg = fma((double)rn, (double)un, dg);
            dd = fma((double)acc, (double)un, dd);
            dr = fma((double)rn, (double)rn, dr);
        }
    }
    // the three block sums (wave sums, then the waves in order) behind one barrier
    dg = wave_sum(dg);
    dd = wave_sum(dd);
    dr = wave_sum(dr);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) {
        lds[wv] = dg;
        lds[4 + wv] = dd;
        lds[8 + wv] = dr;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double t = 0.0;
        for (int k = 0; k < nw; ++k) t += lds[4 * threadIdx.x + k];
        pout[threadIdx.x * kSpmvMaxBlocks + blockIdx.x] = t;
    }
}

// convergence test on the last launch's partials (end of a chunk of
// iterations, so that a converged last iteration is reported as such)
__global__ __launch_bounds__(64) void cg_check(int nb, const double *part, CGScal *sc,
                                               int *done) {
    __shared__ double lds[2];
    if (*done) return;
    const double rr = sum_partials(part + 2 * kSpmvMaxBlocks, nb, lds);
    if (threadIdx.x == 0) {
        sc->rr = rr;
        if (sqrt(rr) <= sc->target || rr == 0.0) *done = 1;
    }
}

// ---- The two-launch form, for matrices that stream from HBM.  There the
// iteration is bound by the matrix stream and the gathers, and the single-
// reduction form's four-value row states halve the loads in flight per lane
// (628 against 438 us per iteration at n = 65536).  Standard CG: an SpMV
// launch that also forms the direction, and an update launch.

// The preconditioned residual z and the search direction p of one iteration
// parity, interleaved so that the SpMV gathers both with one load per nonzero.
template <typename T>
struct __attribute__((aligned(2 * sizeof(T)))) ZP {
    T z, p;
};

template <typename T>
__global__ __launch_bounds__(kCGThreads) void cg2_init(int n, const T *__restrict__ b,
                                                      const T *__restrict__ dinv, T *x, T *r,
                                                      ZP<T> *w, double *part) {
    __shared__ double lds[16];
    double rz = 0.0, rr = 0.0;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
        const T bj = b[j];
        const T zj = dinv[j] * bj;
        x[j] = (T)0;
        r[j] = bj;
        w[j] = ZP<T>{zj, (T)0};  // the first direction is z itself (beta = 0)
        rz = fma((double)bj, (double)zj, rz);
        rr = fma((double)bj, (double)bj, rr);
    }
    double t1 = block_sum(rz, lds);
    double t2 = block_sum(rr, lds);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = t1;
        part[kCGBlocks + blockIdx.x] = t2;
    }
}

__global__ __launch_bounds__(64) void cg2_init_finish(int nb, const double *part, double rtol,
                                                     double atol, CGScal *sc, int *done) {
    __shared__ double lds[2];
    const double rz = sum_partials(part, nb, lds);
    const double rr = sum_partials(part + kCGBlocks, nb, lds);
    if (threadIdx.x == 0) {
        const double target = fmin(rtol * sqrt(rr), atol);
        sc->rho[0] = 0.0;
        sc->rho[1] = 1.0;  // previous rho of the first iteration (its beta is 0)
        sc->rr = rr;
        sc->target = target;
        sc->its = 0.0;
        *done = (sqrt(rr) <= target || rr == 0.0) ? 1 : 0;
    }
}

// Entries e, e + G, ..., e + (kSpmvU2 - 1) G of a row ending at e1 (those past
// the end get column -1): columns and values, then the gathered (z, p) pairs
// (eight at a time: the pairs are half the size of the row states above).
constexpr int kSpmvU2 = 8;
template <int G, bool NT, typename T>
__device__ __forceinline__ void load_chunk2(int e, int e1, const int32_t *__restrict__ col,
                                           const T *__restrict__ val,
                                           const ZP<T> *__restrict__ wold, int (&c)[kSpmvU2],
                                           T (&v)[kSpmvU2], ZP<T> (&w)[kSpmvU2]) {
#pragma unroll
    for (int k = 0; k < kSpmvU2; ++k) {
        const int ek = e + k * G;
        if (ek < e1) {
            c[k] = NT ? __builtin_nontemporal_load(col + ek) : col[ek];
            v[k] = NT ? __builtin_nontemporal_load(val + ek) : val[ek];
        } else {
            c[k] = -1;
            v[k] = (T)0;
        }
    }
#pragma unroll
    for (int k = 0; k < kSpmvU2; ++k) w[k] = c[k] >= 0 ? wold[c[k]] : ZP<T>{(T)0, (T)0};
}

// One CG iteration's first half.  From the previous update's partials:
// rho = r.z and r.r (convergence test); beta = rho / rho_prev (0 on the first
// iteration); the new direction p_new = z + beta p_old is formed where the
// SpMV gathers it (from the pairs wold = (z, p_old)), q = S p_new, p_new goes
// to wnew[r].p and the rows' p_new . q to partial.  rho is double-buffered by
// parity: every workgroup reads rho[par ^ 1] (the previous one) and workgroup
// 0 writes rho[par].
//
// G lanes per row; each lane takes its entries e, e + G, ... kSpmvU2 at a
// time, all their loads in flight together (the summation order is that of
// one entry at a time).  Nothing loaded depends on beta, so the first chunk
// is requested before the partials are summed, and each row's first chunk and
// the next row's pointers before the previous row's lane reduction.  NT: the
// matrix streams past the caches (nontemporal loads), for matrices too large
// to stay cache-resident between iterations, so that the gathered pairs stay.
template <int G, bool NT, typename T>
__global__ __launch_bounds__(256) void spmv_dir(int n, const int32_t *__restrict__ rowptr,
                                                const int32_t *__restrict__ col,
                                                const T *__restrict__ val,
                                                const ZP<T> *__restrict__ wold,
                                                ZP<T> *__restrict__ wnew, T *__restrict__ q,
                                                int nb2, const double *part2, double *partial,
                                                CGScal *sc, int *done, int first, int par) {
    __shared__ double lds[16];
    const int groups = 256 / G;
    const int g = threadIdx.x / G, l = threadIdx.x % G;
    const int stride = gridDim.x * groups;
    int r = blockIdx.x * groups + g;
    int e = 0, e1 = 0, en = 0, en1 = 0;
    if (r < n) {
        e = rowptr[r] + l;
        e1 = rowptr[r + 1];
    }
    if (r + stride < n) {
        en = rowptr[r + stride] + l;
        en1 = rowptr[r + stride + 1];
    }
    int c[kSpmvU2];
    T v[kSpmvU2];
    ZP<T> w[kSpmvU2];
    load_chunk2<G, NT>(e, e1, col, val, wold, c, v, w);
    if (block_flag(done, lds)) return;
    const double rz = sum_partials(part2, nb2, lds);
    const double rr = sum_partials(part2 + kCGBlocks, nb2, lds);
    if (sqrt(rr) <= sc->target || rr == 0.0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->rr = rr;
            *done = 1;
        }
        return;
    }
    const T beta = first ? (T)0 : (T)(rz / sc->rho[par ^ 1]);
    double dot = 0.0;
    while (r < n) {
        T acc = (T)0;
        for (;;) {
#pragma unroll
            for (int k = 0; k < kSpmvU2; ++k)
                if (c[k] >= 0) acc = fma(v[k], fma(beta, w[k].p, w[k].z), acc);
            e += kSpmvU2 * G;
            if (e >= e1) break;
            load_chunk2<G, NT>(e, e1, col, val, wold, c, v, w);
        }
        const int rc = r;
        const ZP<T> wr = wold[rc];
        r += stride;
        e = en;
        e1 = en1;
        if (r < n) {
            load_chunk2<G, NT>(e, e1, col, val, wold, c, v, w);
            if (r + stride < n) {
                en = rowptr[r + stride] + l;
                en1 = rowptr[r + stride + 1];
            }
        }
        for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
        if (l == 0) {
            const T pr = fma(beta, wr.p, wr.z);
            wnew[rc].p = pr;
            q[rc] = acc;
            dot = fma((double)pr, (double)acc, dot);
        }
    }
    const double t = block_sum(dot, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->rho[par] = rz;
        sc->rr = rr;
    }
}

// alpha = rho / (p.q); x += alpha p; r -= alpha q; z = D^-1 r into w[j].z;
// partials r.z, r.r
template <typename T>
__global__ __launch_bounds__(kCGThreads) void cg_update(int n, int nb1, const double *part1,
                                                        ZP<T> *w, const T *__restrict__ q,
                                                        const T *__restrict__ dinv, T *x, T *r,
                                                        double *part2, CGScal *sc, int *done,
                                                        int par) {
    __shared__ double lds[16];
    // the first element's operands are requested before the partials are summed
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    T pj = (T)0, qj = (T)0, rj = (T)0, xj = (T)0, dj = (T)0;
    if (j < n) {
        pj = w[j].p;
        qj = q[j];
        rj = r[j];
        xj = x[j];
        dj = dinv[j];
    }
    if (block_flag(done, lds)) return;
    const double pq = sum_partials(part1, nb1, lds);
    if (!(pq > 0.0)) {  // breakdown (S is positive semidefinite)
        if (blockIdx.x == 0 && threadIdx.x == 0) *done = 2;
        return;
    }
    const T alpha = (T)(sc->rho[par] / pq);
    double rz = 0.0, rr = 0.0;
    for (bool head = true; j < n; j += gridDim.x * blockDim.x, head = false) {
        if (!head) {
            pj = w[j].p;
            qj = q[j];
            rj = r[j];
            xj = x[j];
            dj = dinv[j];
        }
        x[j] = fma(alpha, pj, xj);
        rj = fma(-alpha, qj, rj);
        r[j] = rj;
        const T zj = dj * rj;
        w[j].z = zj;
        rz = fma((double)rj, (double)zj, rz);
        rr = fma((double)rj, (double)rj, rr);
    }
    double t1 = block_sum(rz, lds);
    double t2 = block_sum(rr, lds);
    if (threadIdx.x == 0) {
        part2[blockIdx.x] = t1;
        part2[kCGBlocks + blockIdx.x] = t2;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->its += 1.0;
}

// convergence test on the last update's partials (end of a chunk of
// iterations, so that a converged last iteration is reported as such)
__global__ __launch_bounds__(64) void cg2_check(int nb2, const double *part2, CGScal *sc,
                                               int *done) {
    __shared__ double lds[2];
    if (*done) return;
    const double rr = sum_partials(part2 + kCGBlocks, nb2, lds);
    if (threadIdx.x == 0) {
        sc->rr = rr;
        if (sqrt(rr) <= sc->target || rr == 0.0) *done = 1;
    }
}

// lanes per row: at least four nonzeros per lane on average, 8 to 64 lanes
static int lanes_per_row(const SchurCSR &S) {
    const double avg = (double)S.nnz / std::max(1, S.n);
    return avg >= 256.0 ? 64 : avg >= 128.0 ? 32 : avg >= 64.0 ? 16 : 8;
}

template <typename T>
static void launch_spmv(hipStream_t st, const SchurCSR &S, const T *val, const T *x, T *y,
                        double *partial, unsigned &nb_out) {
    const int n = S.n;
    const int G = lanes_per_row(S) >= 64 ? 64 : 16;
    const unsigned nb = std::min<unsigned>(kSpmvMaxBlocks, grid_for(n, 256 / G));
    nb_out = nb;
    if (G == 64)
        hipLaunchKernelGGL((spmv_rows<64, T>), dim3(nb), dim3(256), 0, st, n, S.rowptr.get(),
                           S.col.get(), val, x, y, partial);
    else
        hipLaunchKernelGGL((spmv_rows<16, T>), dim3(nb), dim3(256), 0, st, n, S.rowptr.get(),
                           S.col.get(), val, x, y, partial);
}

// e0, e1: events recorded at the dispatch's own start and end (may be null)
template <typename T>
static void launch_cg_step(hipStream_t st, const SchurCSR &S, const T *val, const RWS<T> *gold,
                           RWS<T> *gnew, T *x, T *p, int nbp, const double *pin, double *pout,
                           CGScal *sc, int *done, int mode, int par, unsigned nb, hipEvent_t e0,
                           hipEvent_t e1) {
    // only cache-resident matrices take this form (no nontemporal loads)
    const int n = S.n;
    const int G = lanes_per_row(S);
    const int32_t *rp = S.rowptr.get(), *cl = S.col.get();
#define OTIP_CG_STEP(GG)                                                                        \
    hipExtLaunchKernelGGL(cg_step<GG, false, T>, dim3(nb), dim3(256), 0, st, e0, e1, 0, n, rp,  \
                          cl, val, gold, gnew, x, p, nbp, pin, pout, sc, done, mode, par)
    switch (G) {
        case 64: OTIP_CG_STEP(64); break;
        case 32: OTIP_CG_STEP(32); break;
        case 16: OTIP_CG_STEP(16); break;
        default: OTIP_CG_STEP(8); break;
    }
#undef OTIP_CG_STEP
}

// e0, e1: events recorded at the dispatch's own start and end (may be null)
template <typename T>
static void launch_spmv_dir(hipStream_t st, const SchurCSR &S, const T *val, const ZP<T> *wold,
                            ZP<T> *wnew, T *q, int nb2, const double *part2, double *partial,
                            CGScal *sc, int *done, int first, int par, unsigned &nb_out,
                            hipEvent_t e0, hipEvent_t e1) {
    const int n = S.n;
    const int G = lanes_per_row(S);
    // about as many workgroups as stay resident at once (three per compute
    // unit at this kernel's register use): each lane group then walks several
    // rows with the next row's loads in flight
    const unsigned nb = std::min<unsigned>(kSpmvDirBlocks, grid_for(n, 256 / G));
    nb_out = nb;
    const int32_t *rp = S.rowptr.get(), *cl = S.col.get();
    // matrices beyond this size do not stay cache-resident between iterations
    const bool nt = ((double)sizeof(T) + 4.0) * (double)S.nnz > 96.0 * (1 << 20);
#define OTIP_SPMV_DIR(GG, NT)                                                                  \
    hipExtLaunchKernelGGL(spmv_dir<GG, NT, T>, dim3(nb), dim3(256), 0, st, e0, e1, 0, n, rp,   \
                          cl, val, wold, wnew, q, nb2, part2, partial, sc, done, first, par)
    if (nt) {
        switch (G) {
            case 64: OTIP_SPMV_DIR(64, true); break;
            case 32: OTIP_SPMV_DIR(32, true); break;
            case 16: OTIP_SPMV_DIR(16, true); break;
            default: OTIP_SPMV_DIR(8, true); break;
        }
    } else {
        switch (G) {
            case 64: OTIP_SPMV_DIR(64, false); break;
            case 32: OTIP_SPMV_DIR(32, false); break;
            case 16: OTIP_SPMV_DIR(16, false); break;
            default: OTIP_SPMV_DIR(8, false); break;
        }
    }
#undef OTIP_SPMV_DIR
}

// Jacobi inverse diagonal of a caller's CSR matrix, by the rule of schur_diag
// (0 where the diagonal is absent or not positive), and a flag for column
// indices outside [0, n).  The row pointers were checked on the host.
__global__ void csr_jacobi(int n, const int32_t *__restrict__ rowptr,
                           const int32_t *__restrict__ col, const double *__restrict__ val,
                           double *__restrict__ dinv, int *bad) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double d = 0.0;
    int flag = 0;
    for (int e = rowptr[r]; e < rowptr[r + 1]; ++e) {
        const int c = col[e];
        if (c < 0 || c >= n)
            flag = 1;
        else if (c == r)
            d += val[e];
    }
    dinv[r] = d > 0.0 ? 1.0 / d : 0.0;
    if (flag) atomicOr(bad, 1);
}

void SchurSolver::load_csr(hipStream_t st, int n, int64_t nnz, const int32_t *rowptr,
                           const int32_t *col, const double *val) {
    std::vector<int32_t> rp((size_t)n + 1);
    OTIP_HIP(hipMemcpyAsync(rp.data(), rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost,
                            st));
    OTIP_HIP(hipStreamSynchronize(st));
    OTIP_CHECK(rp[0] == 0 && (int64_t)rp[n] == nnz, 1, "CSR: rowptr[0] != 0 or rowptr[n] != nnz");
    for (int r = 0; r < n; ++r)
        OTIP_CHECK(rp[r + 1] >= rp[r], 1, "CSR: row pointers decrease at row " + std::to_string(r));
    S.n = n;
    S.nnz = nnz;
    S.rowptr.need((size_t)n + 1);
    S.col.need((size_t)std::max<int64_t>(nnz, 1));
    S.val.need((size_t)std::max<int64_t>(nnz, 1));
    S.dinv.need((size_t)n);
    OTIP_HIP(hipMemcpyAsync(S.rowptr.get(), rowptr, sizeof(int32_t) * (n + 1),
                            hipMemcpyDeviceToDevice, st));
    if (nnz > 0) {
        OTIP_HIP(hipMemcpyAsync(S.col.get(), col, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice,
                                st));
        OTIP_HIP(hipMemcpyAsync(S.val.get(), val, sizeof(double) * nnz, hipMemcpyDeviceToDevice,
                                st));
    }
    flag_.need(1);
    OTIP_HIP(hipMemsetAsync(flag_.get(), 0, sizeof(int), st));
    hipLaunchKernelGGL(csr_jacobi, dim3(grid_for(n, 256)), dim3(256), 0, st, n, S.rowptr.get(),
                       S.col.get(), S.val.get(), S.dinv.get(), flag_.get());
    OTIP_HIP(hipGetLastError());
    int bad = 0;
    OTIP_HIP(hipMemcpyAsync(&bad, flag_.get(), sizeof(int), hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipStreamSynchronize(st));
    OTIP_CHECK(!bad, 1, "CSR: column index outside [0, n)");
}

void SchurSolver::spmv(hipStream_t st, const double *x, double *y) {
    unsigned nb;
    launch_spmv<double>(st, S, S.val.get(), x, y, nullptr, nb);
    OTIP_HIP(hipGetLastError());
}

// The two-launch form's iteration loop (matrices that stream from HBM); r is
// n values of scratch, g 8 n (two (z, p) pair arrays and q), part the partial
// sums, sc and done the device scalars.
template <typename T>
CGStats SchurSolver::pcg_stream(hipStream_t st, const T *val, const T *dinv, const T *b, T *x,
                                double rtol, double atol, int maxit, T *r, T *g, double *part,
                                CGScal *sc, int *done) {
    const int n = S.n;
    CGStats out;
    double *part1 = part;
    double *part2 = part + kSpmvMaxBlocks;
    ZP<T> *W[2] = {(ZP<T> *)g, (ZP<T> *)(g + 2 * (size_t)n)};
    T *q = g + 4 * (size_t)n;
    const unsigned nbv = std::min<unsigned>(kCGBlocks, grid_for(n, kCGThreads));
    hipLaunchKernelGGL((cg2_init<T>), dim3(nbv), dim3(kCGThreads), 0, st, n, b, dinv, x, r, W[1],
                       part2);
    hipLaunchKernelGGL(cg2_init_finish, dim3(1), dim3(64), 0, st, (int)nbv, part2, rtol, atol, sc,
                       done);
    OTIP_HIP(hipGetLastError());
    int chunk = std::min(4, std::max(1, maxit));
    int launched = 0;
    CGScal hs{};
    int hdone = 0;
    double its_prev = 0.0, rr_prev = -1.0;  // at the previous check
    // algorithmic bytes of one SpMV launch: values and columns, row pointers,
    // the two gathered vectors read once, the new direction and q written
    const double bytes = cg_launch_bytes((double)sizeof(T), S.nnz, n);
    while (true) {
        for (int c = 0; c < chunk; ++c) {
            const int par = launched & 1;
            unsigned nbs;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (timer) timer->arm(bytes, &e0, &e1);
            launch_spmv_dir<T>(st, S, val, W[par ^ 1], W[par], q, (int)nbv, part2, part1, sc, done,
                               launched == 0 ? 1 : 0, par, nbs, e0, e1);
            hipLaunchKernelGGL((cg_update<T>), dim3(nbv), dim3(kCGThreads), 0, st, n, (int)nbs,
                               part1, W[par], q, dinv, x, r, part2, sc, done, par);
            ++launched;
        }
        hipLaunchKernelGGL(cg2_check, dim3(1), dim3(64), 0, st, (int)nbv, part2, sc, done);
        OTIP_HIP(hipGetLastError());
        OTIP_HIP(hipMemcpyAsync(&hs, sc, sizeof(CGScal), hipMemcpyDeviceToHost, st));
        OTIP_HIP(hipMemcpyAsync(&hdone, done, sizeof(int), hipMemcpyDeviceToHost, st));
        OTIP_HIP(hipStreamSynchronize(st));
        // launches past the last executed iteration found the work done
        if (timer) timer->collect((size_t)std::max(0.0, hs.its - its_prev));
        if (hdone || launched >= maxit) break;
        int next = std::min(chunk * 2, 64);
        const double ran = hs.its - its_prev;
        if (rr_prev > 0.0 && hs.rr > 0.0 && hs.rr < rr_prev && ran > 0.0) {
            const double rate = std::log(hs.rr / rr_prev) / ran;
            const double need = std::log(hs.target * hs.target / hs.rr) / rate;
            if (std::isfinite(need))
                next = (int)std::min(64.0, std::max(4.0, std::ceil(1.1 * need) + 1.0));
        }
        rr_prev = hs.rr;
        its_prev = hs.its;
        chunk = std::min(next, maxit - launched);
        if (chunk <= 0) break;
    }
    out.iterations = (int)hs.its;
    out.res_norm = std::sqrt(std::max(0.0, hs.rr));
    out.converged = (hdone == 1);
    return out;
}

// Jacobi-preconditioned CG in storage type T on S x = b: one launch per
// iteration (the single-reduction form) while the matrix stays cache-resident,
// the two-launch form beyond.
template <typename T>
CGStats SchurSolver::pcg_impl(hipStream_t st, const T *val, const T *dinv, const T *b, T *x,
                              double rtol, double atol, int maxit, DBuf<T> &p_, DBuf<T> &g_) {
    const int n = S.n;
    CGStats out;
    T *p = p_.need(n);
    g_.need(8 * (size_t)n);  // two row-state arrays, alternating by launch parity
    part_.need(2 * (size_t)kCGPart);
    scal_.need(sizeof(CGScal) / sizeof(double));
    flag_.need(1);
    double *part[2] = {part_.get(), part_.get() + kCGPart};
    CGScal *sc = (CGScal *)scal_.get();
    int *done = flag_.get();
    if (cg_streams((double)sizeof(T), S.nnz))
        return pcg_stream<T>(st, val, dinv, b, x, rtol, atol, maxit, p, g_.get(), part[0], sc,
                             done);
    RWS<T> *G[2] = {(RWS<T> *)g_.get(), (RWS<T> *)(g_.get() + 4 * (size_t)n)};
    // about as many workgroups as stay resident at once: each lane group then
    // walks several rows with the next row's loads in flight
    const unsigned nb =
        std::min<unsigned>(kSpmvDirBlocks, grid_for(n, 256 / lanes_per_row(S)));
    const unsigned nbv = std::min<unsigned>(kCGBlocks, grid_for(n, kCGThreads));
    hipLaunchKernelGGL((cg_init<T>), dim3(nbv), dim3(kCGThreads), 0, st, n, b, dinv, G[1]);
    launch_cg_step<T>(st, S, val, G[1], G[0], x, p, (int)nb, part[1], part[0], sc, done, 0, 0,
                      nb, nullptr, nullptr);
    hipLaunchKernelGGL(cg_init_finish, dim3(1), dim3(64), 0, st, (int)nb, part[0], rtol, atol, sc,
                       done);
    OTIP_HIP(hipGetLastError());
    int chunk = std::min(4, std::max(1, maxit));
    int launched = 1;  // launch 0 was the start
    CGScal hs{};
    int hdone = 0;
    double its_prev = 0.0, rr_prev = -1.0;  // at the previous check
    // algorithmic bytes of one launch: values and columns, row pointers, each
    // row's state read once (gathered and by its owner) and written, x and p
    // read and written
    const double bytes = cg_launch_bytes((double)sizeof(T), S.nnz, n);
    while (true) {
        for (int c = 0; c < chunk; ++c) {
            const int par = launched & 1;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (timer) timer->arm(bytes, &e0, &e1);
            launch_cg_step<T>(st, S, val, G[par ^ 1], G[par], x, p, (int)nb, part[par ^ 1],
                              part[par], sc, done, launched == 1 ? 1 : 2, par, nb, e0, e1);
            ++launched;
        }
        hipLaunchKernelGGL(cg_check, dim3(1), dim3(64), 0, st, (int)nb, part[(launched - 1) & 1],
                           sc, done);
        OTIP_HIP(hipGetLastError());
        OTIP_HIP(hipMemcpyAsync(&hs, sc, sizeof(CGScal), hipMemcpyDeviceToHost, st));
        OTIP_HIP(hipMemcpyAsync(&hdone, done, sizeof(int), hipMemcpyDeviceToHost, st));
        OTIP_HIP(hipStreamSynchronize(st));
        // launches past the last executed iteration found the work done
        if (timer) timer->collect((size_t)std::max(0.0, hs.its - its_prev));
        if (hdone || launched - 1 >= maxit) break;
        // next chunk: the iterations still needed at the rate the residual
        // fell over the last chunk (plus a tenth), else twice the last chunk;
        // launches past convergence return at once but still cost a dispatch
        int next = std::min(chunk * 2, 64);
        const double ran = hs.its - its_prev;
        if (rr_prev > 0.0 && hs.rr > 0.0 && hs.rr < rr_prev && ran > 0.0) {
            const double rate = std::log(hs.rr / rr_prev) / ran;
            const double need = std::log(hs.target * hs.target / hs.rr) / rate;
            if (std::isfinite(need))
                next = (int)std::min(64.0, std::max(4.0, std::ceil(1.1 * need) + 1.0));
        }
        rr_prev = hs.rr;
        its_prev = hs.its;
        chunk = std::min(next, maxit - (launched - 1));
        if (chunk <= 0) break;
    }
    out.iterations = (int)hs.its;
    out.res_norm = std::sqrt(std::max(0.0, hs.rr));
    out.converged = (hdone == 1);
    return out;
}

CGStats SchurSolver::pcg(hipStream_t st, const double *b, double *x, double rtol, double atol,
                         int maxit) {
    return pcg_impl<double>(st, S.val.get(), S.dinv.get(), b, x, rtol, atol, maxit, p_, g_);
}

__global__ void to_f32(int64_t n, const double *__restrict__ a, float *__restrict__ b) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        b[t] = (float)a[t];
}
__global__ void resid64(int n, const double *__restrict__ b, const double *__restrict__ Sx,
                        double *__restrict__ r, float *__restrict__ r32, double *part) {
    __shared__ double lds[16];
    double s = 0.0;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
        const double v = b[j] - Sx[j];
        r[j] = v;
        r32[j] = (float)v;
        s = fma(v, v, s);
    }
    const double t = block_sum(s, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}
__global__ void add_f32(int n, const float *__restrict__ d, double *__restrict__ x) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x)
        x[j] += (double)d[j];
}

// Mixed precision: FP64 iterative refinement around FP32 Jacobi-CG.  Each
// outer step forms the FP64 residual r = b - S x and solves S d = r in FP32 to
// a relative 1e-4 (or the remaining target); x += d.  Stops on the FP64
// residual, so the accuracy is that of an FP64 solve.
CGStats SchurSolver::pcg_mixed(hipStream_t st, const double *b, double *x, double rtol,
                               double atol, int maxit) {
    const int n = S.n;
    CGStats out;
    val32_.need((size_t)S.nnz);
    dinv32_.need(n);
    hipLaunchKernelGGL(to_f32, dim3(std::min<unsigned>(4096, grid_for(S.nnz, 256))), dim3(256), 0,
                       st, S.nnz, S.val.get(), val32_.get());
    hipLaunchKernelGGL(to_f32, dim3(grid_for(n, 256)), dim3(256), 0, st, (int64_t)n,
                       S.dinv.get(), dinv32_.get());
    double *r = rd_.need(n), *Sx = sx_.need(n);
    float *r32 = rf_.need(n), *d32 = df_.need(n);
    double *part = rpart_.need(256);
    OTIP_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, st));
    const unsigned nbv = std::min<unsigned>(256, grid_for(n, 256));
    double target = -1.0;
    std::vector<double> hp(nbv);
    for (int outer = 0; outer < 12; ++outer) {
        spmv(st, x, Sx);
        hipLaunchKernelGGL(resid64, dim3(nbv), dim3(256), 0, st, n, b, Sx, r, r32, part);
        OTIP_HIP(hipMemcpyAsync(hp.data(), part, sizeof(double) * nbv, hipMemcpyDeviceToHost, st));
        OTIP_HIP(hipStreamSynchronize(st));
        double rr = 0.0;
        for (double v : hp) rr += v;
        const double rn = std::sqrt(rr);
        if (target < 0.0) target = std::min(rtol * rn, atol);
        out.res_norm = rn;
        if (rn <= target || rn == 0.0) {
            out.converged = true;
            break;
        }
        if (out.iterations >= maxit) break;
        const double inner = std::max(1e-4, 0.5 * target / rn);
        CGStats cs = pcg_impl<float>(st, val32_.get(), dinv32_.get(), r32, d32, inner, 1e300,
                                     maxit - out.iterations, pf_, gf_);
        out.iterations += std::max(cs.iterations, 1);
        hipLaunchKernelGGL(add_f32, dim3(nbv), dim3(256), 0, st, n, d32, x);
    }
    return out;
}

}  // namespace otip
