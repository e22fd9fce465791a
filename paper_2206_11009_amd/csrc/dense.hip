// Dense LDL^T of the Schur complement with the infinite-pivot rule
// (Section 4.2: after the switch the Schur complement is factorised exactly;
// its zero pivot is replaced by an infinitely large value).
//
// Right-looking blocked factorisation of the lower triangle of a column-major
// n x n array, block width 64:
//   1. the 64 x 64 diagonal block is factorised in LDS by one workgroup;
//   2. every row below solves w_i L11^T = a_i (w = L21 D1) and l_i = w_i D1^-1;
//   3. the trailing lower triangle is updated, A22 -= L21 W21^T, in 64 x 64
//      tiles staged through LDS.
// A pivot d_k <= pivtol * S_kk (original diagonal) or d_k <= 0 becomes +inf:
// its column of L is zero and the solve returns 0 for that unknown.
#include "internal.h"

namespace otip {

constexpr int NB = 64;

__global__ void dense_fill(int n, const int32_t *__restrict__ rowptr,
                           const int32_t *__restrict__ col, const double *__restrict__ val,
                           double *__restrict__ A, double *__restrict__ orig) {
    const int j = blockIdx.x;  // row j of S -> column j of the symmetric array
    for (int e = rowptr[j] + threadIdx.x; e < rowptr[j + 1]; e += blockDim.x) {
        const int k = col[e];
        A[(size_t)k + (size_t)j * n] = val[e];  // A(k, j) = S(j, k) = S(k, j)
        if (k == j) orig[j] = val[e];
    }
}

__global__ void dense_zero(size_t total, double *A) {
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (size_t)gridDim.x * blockDim.x)
        A[t] = 0.0;
}

// Factor the diagonal block [kb, kb+nb): thread (i, q) keeps row i, columns
// 16q..16q+15 of the block (t) and of its running inverse (x) in registers;
// each step broadcasts the pivot, column k of L and row k of the inverse
// through LDS.  L11 = prod_k (I + l_k e_k^T), so applying the row operations
// X <- (I - l_k e_k^T) X to X = I in the same order leaves X = L11^-1, which
// is written to Linv (nb x nb, column-major) for the panel product.
__global__ __launch_bounds__(256) void ldl_diag(int n, int kb, int nb, double *A,
                                                const double *orig, double *d, double pivtol,
                                                int *ninf, double *Linv) {
    __shared__ double colk[NB];
    __shared__ double xrow[NB];
    __shared__ double dk;
    const int i = threadIdx.x & 63, q = threadIdx.x >> 6;
    double t[16], x[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        const int j = 16 * q + c;
        t[c] = (i < nb && j < nb && i >= j) ? A[(size_t)(kb + i) + (size_t)(kb + j) * n] : 0.0;
        x[c] = (i == j) ? 1.0 : 0.0;
    }
    for (int k = 0; k < nb; ++k) {
        const int kq = k >> 4, kc = k & 15;
        if (q == kq && i == k) {
            double v = 0.0;
#pragma unroll
            for (int c = 0; c < 16; ++c)
                if (c == kc) v = t[c];
            const double o = orig[kb + k];
            if (!(v > pivtol * o) || !(v > 0.0)) {
                v = INFINITY;
                atomicAdd(ninf, 1);
            }
            dk = v;
            d[kb + k] = v;
        }
        if (i == k) {
#pragma unroll
            for (int c = 0; c < 16; ++c) xrow[16 * q + c] = x[c];
        }
        __syncthreads();
        const double dd = dk;
        if (q == kq) {
            // column k of L (rows below k)
            double l = 0.0;
#pragma unroll
            for (int c = 0; c < 16; ++c)
                if (c == kc) l = t[c];
            l = (i > k && !isinf(dd)) ? l / dd : 0.0;
            colk[i] = l;
#pragma unroll
            for (int c = 0; c < 16; ++c)
                if (c == kc && i > k) t[c] = l;
        }
        __syncthreads();
        const double lik = colk[i];
        if (!isinf(dd)) {
            const double li = lik * dd;
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const int j = 16 * q + c;
                if (j > k && i >= j) t[c] = fma(-li, colk[j], t[c]);
            }
        }
        // inverse: rows below k lose l_ik times row k
#pragma unroll
        for (int c = 0; c < 16; ++c) x[c] = fma(-lik, xrow[16 * q + c], x[c]);
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        const int j = 16 * q + c;
        if (i < nb && j < nb && i > j) A[(size_t)(kb + i) + (size_t)(kb + j) * n] = t[c];
        Linv[(size_t)i + (size_t)j * NB] = (i < nb && j < nb) ? x[c] : (i == j ? 1.0 : 0.0);
    }
}

// Rows below the diagonal block: W21 = A21 L11^-T (so W21 = L21 D1) and
// L21 = W21 D1^-1.  A 64-row tile of A21 and Linv are staged in LDS; each
// thread forms 16 entries of W as dot products with rows of Linv.
__global__ __launch_bounds__(256) void ldl_panel(int n, int kb, int nb, double *A,
                                                 const double *d, double *W,
                                                 const double *Linv) {
    __shared__ double As[NB][NB + 1];
    __shared__ double Li[NB][NB + 1];
    const int r0 = kb + nb + blockIdx.x * NB;
    const int rows = n - kb - nb;
    for (int t = threadIdx.x; t < NB * NB; t += 256) {
        const int a = t % NB, k = t / NB;
        As[a][k] = (r0 + a < n && k < nb) ? A[(size_t)(r0 + a) + (size_t)(kb + k) * n] : 0.0;
        Li[a][k] = Linv[(size_t)a + (size_t)k * NB];  // Linv(a, k)
    }
    __syncthreads();
    const int a = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int i = r0 + a;
    // W(i, k) = sum_t A(i, t) * Linv(k, t), t <= k
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        const int k = 16 * q + c;
        double v = 0.0;
        for (int tt = 0; tt <= k && tt < nb; ++tt) v = fma(As[a][tt], Li[k][tt], v);
        if (i < n && k < nb) {
            const double dd = d[kb + k];
            const bool inf = isinf(dd);
            const double wk = inf ? 0.0 : v;
            W[(size_t)(i - kb - nb) + (size_t)k * rows] = wk;
            A[(size_t)i + (size_t)(kb + k) * n] = inf ? 0.0 : wk / dd;
        }
    }
}

// A22 -= L21 W21^T on lower-triangular 64x64 tiles
__global__ __launch_bounds__(256) void ldl_update(int n, int kb, int nb, double *A,
                                                  const double *W) {
    const int r0 = kb + nb;
    const int rows = n - r0;
    const int ti = blockIdx.x, tj = blockIdx.y;
    if (tj > ti) return;
    __shared__ double Ls[NB][NB + 1];
    __shared__ double Ws[NB][NB + 1];
    const int i0 = ti * NB, j0 = tj * NB;
    for (int t = threadIdx.x; t < NB * NB; t += blockDim.x) {
        const int a = t % NB, k = t / NB;
        const int ii = i0 + a, jj = j0 + a;
        Ls[a][k] = (ii < rows && k < nb) ? A[(size_t)(r0 + ii) + (size_t)(kb + k) * n] : 0.0;
        Ws[a][k] = (jj < rows && k < nb) ? W[(size_t)jj + (size_t)k * rows] : 0.0;
    }
    __syncthreads();
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (int k = 0; k < nb; ++k) {
        double lv[4], wv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) lv[a] = Ls[tx + 16 * a][k];
#pragma unroll
        for (int b = 0; b < 4; ++b) wv[b] = Ws[ty + 16 * b][k];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = fma(lv[a], wv[b], acc[a][b]);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int ii = i0 + tx + 16 * a, jj = j0 + ty + 16 * b;
            if (ii < rows && jj < rows && ii >= jj) {
                double *p = &A[(size_t)(r0 + ii) + (size_t)(r0 + jj) * n];
                *p -= acc[a][b];
            }
        }
}

// Triangular solves, one launch per 64-wide block column.  Every workgroup
// re-solves the 64 x 64 diagonal block in one wave (register shuffles) from
// the final right-hand side entries of that block, then applies the block's
// columns to its own rows of the remaining right-hand side; workgroup 0 stores
// the solved block.  Right-hand side (w) and solution (x) are separate arrays,
// so no workgroup reads an entry another one writes in the same launch.
//
// forward:  L y = b, unit lower, L column-major           (rows below the block)
// backward: L^T x = y' (y' = D^-1 y) with U = L^T stored column-major (rows above)
__device__ __forceinline__ double diag_solve_wave(int n, const double *__restrict__ T, int kb,
                                                  int nb, double wt, bool lower) {
    const int t = threadIdx.x & 63;
    double row[NB];
    // lane t's row of the 64 x 64 diagonal block, loaded before the recurrence
#pragma unroll
    for (int k = 0; k < NB; ++k)
        row[k] = (t < nb && k < nb) ? T[(size_t)(kb + t) + (size_t)(kb + k) * n] : 0.0;
    double x = wt;
    if (lower) {
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            const double xk = __shfl(x, k, 64);
            if (t > k && t < nb) x = fma(-row[k], xk, x);
        }
    } else {
#pragma unroll
        for (int k = NB - 1; k >= 0; --k) {
            const double xk = __shfl(x, k, 64);
            if (t < k && k < nb) x = fma(-row[k], xk, x);
        }
    }
    return x;
}

__global__ __launch_bounds__(256) void trsv_step(int n, int kb, int nb, const double *__restrict__ T,
                                                 const double *__restrict__ d, double *w, double *x,
                                                 int lower) {
    __shared__ double xb[64];
    if (threadIdx.x < 64) {
        const int t = threadIdx.x;
        const double wt = (t < nb) ? w[kb + t] : 0.0;
        const double v = diag_solve_wave(n, T, kb, nb, wt, lower != 0);
        if (t < nb) {
            xb[t] = v;
            if (blockIdx.x == 0) x[kb + t] = v;
        }
    }
    __syncthreads();
    // remaining rows: below the block (forward) or above it (backward)
    const int r0 = lower ? kb + nb : 0;
    const int r1 = lower ? n : kb;
    const int i = r0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= r1) return;
    double v = w[i];
    for (int k = 0; k < nb; ++k) v = fma(-T[(size_t)i + (size_t)(kb + k) * n], xb[k], v);
    w[i] = v;
}

// y = D^-1 y (an infinite pivot gives 0)
__global__ void scale_by_pivots(int n, const double *__restrict__ d, double *y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = isinf(d[i]) ? 0.0 : y[i] / d[i];
}

// U = L^T (64 x 64 tiles through LDS), unit diagonal implied
__global__ __launch_bounds__(256) void transpose_lower(int n, const double *__restrict__ L,
                                                       double *__restrict__ U) {
    __shared__ double tile[64][65];
    const int bi = blockIdx.x * 64, bj = blockIdx.y * 64;  // tile of L: rows bi.., cols bj..
    if (blockIdx.y > blockIdx.x) return;
    for (int t = threadIdx.x; t < 64 * 64; t += 256) {
        const int r = t % 64, c = t / 64;
        const int i = bi + r, j = bj + c;
        tile[r][c] = (i < n && j < n && i > j) ? L[(size_t)i + (size_t)j * n] : 0.0;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 64 * 64; t += 256) {
        const int r = t % 64, c = t / 64;  // U(bj + r, bi + c) = L(bi + c, bj + r)
        const int i = bj + r, j = bi + c;
        if (i < n && j < n) U[(size_t)i + (size_t)j * n] = tile[c][r];
    }
}

__global__ void count_nonzero_lower(int n, const double *A, unsigned long long *cnt) {
    unsigned long long c = 0;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < (size_t)n * n;
         t += (size_t)gridDim.x * blockDim.x) {
        const size_t i = t % n, j = t / n;
        if (i > j && A[t] != 0.0) ++c;
    }
    if (c) atomicAdd(cnt, c);
}

int DenseLDL::factor(hipStream_t st, const SchurCSR &S, double pivtol) {
    n = S.n;
    const size_t total = (size_t)n * n;
    double *A = A_.need(total);
    d_.need(n);
    orig_.need(n);
    W_.need((size_t)n * NB);
    linv_.need((size_t)NB * NB);
    ninf_.need(1);
    hipLaunchKernelGGL(dense_zero, dim3(2048), dim3(256), 0, st, total, A);
    hipLaunchKernelGGL(dense_fill, dim3(n), dim3(64), 0, st, n, S.rowptr.get(), S.col.get(),
                       S.val.get(), A, orig_.get());
    OTIP_HIP(hipMemsetAsync(ninf_.get(), 0, sizeof(int), st));
    for (int kb = 0; kb < n; kb += NB) {
        const int nb = std::min(NB, n - kb);
        hipLaunchKernelGGL(ldl_diag, dim3(1), dim3(256), 0, st, n, kb, nb, A, orig_.get(),
                           d_.get(), pivtol, ninf_.get(), linv_.get());
        const int rows = n - kb - nb;
        if (rows > 0) {
            hipLaunchKernelGGL(ldl_panel, dim3(grid_for(rows, NB)), dim3(256), 0, st, n, kb, nb,
                               A, d_.get(), W_.get(), linv_.get());
            const unsigned tiles = grid_for(rows, NB);
            hipLaunchKernelGGL(ldl_update, dim3(tiles, tiles), dim3(256), 0, st, n, kb, nb, A,
                               W_.get());
        }
    }
    OTIP_HIP(hipGetLastError());
    U_.need(total);
    const unsigned tl = grid_for(n, 64);
    hipLaunchKernelGGL(transpose_lower, dim3(tl, tl), dim3(256), 0, st, n, A, U_.get());
    DBuf<unsigned long long> c;
    c.need(1);
    OTIP_HIP(hipMemsetAsync(c.get(), 0, sizeof(unsigned long long), st));
    hipLaunchKernelGGL(count_nonzero_lower, dim3(1024), dim3(256), 0, st, n, A, c.get());
    int hn = 0;
    unsigned long long hc = 0;
    OTIP_HIP(hipMemcpyAsync(&hn, ninf_.get(), sizeof(int), hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipMemcpyAsync(&hc, c.get(), sizeof(hc), hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipStreamSynchronize(st));
    nnzL_ = (int64_t)hc + n;
    return hn;
}

void DenseLDL::solve(hipStream_t st, const double *b, double *x) {
    double *w = v_.need(n);
    double *yv = W_.get();  // n doubles of the panel buffer (free after factor)
    OTIP_HIP(hipMemcpyAsync(w, b, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    for (int kb = 0; kb < n; kb += NB) {
        const int nb = std::min(NB, n - kb);
        const int rows = n - kb - nb;
        hipLaunchKernelGGL(trsv_step, dim3(std::max(1u, grid_for(rows, 256))), dim3(256), 0, st,
                           n, kb, nb, A_.get(), d_.get(), w, yv, 1);
    }
    // yv = D^-1 L^-1 b; then backward on U = L^T
    hipLaunchKernelGGL(scale_by_pivots, dim3(grid_for(n, 256)), dim3(256), 0, st, n, d_.get(), yv);
    for (int kb = ((n - 1) / NB) * NB; kb >= 0; kb -= NB) {
        const int nb = std::min(NB, n - kb);
        hipLaunchKernelGGL(trsv_step, dim3(std::max(1u, grid_for(kb, 256))), dim3(256), 0, st, n,
                           kb, nb, U_.get(), d_.get(), yv, x, 0);
    }
    OTIP_HIP(hipGetLastError());
}

}  // namespace otip
