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

// factor the diagonal block [kb, kb+nb) in LDS
__global__ __launch_bounds__(256) void ldl_diag(int n, int kb, int nb, double *A,
                                                const double *orig, double *d, double pivtol,
                                                int *ninf) {
    __shared__ double T[NB][NB + 1];
    __shared__ double dk;
    for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) {
        const int i = t % nb, j = t / nb;
        T[i][j] = (i >= j) ? A[(size_t)(kb + i) + (size_t)(kb + j) * n] : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < nb; ++k) {
        if (threadIdx.x == 0) {
            double v = T[k][k];
            const double o = orig[kb + k];
            if (!(v > pivtol * o) || !(v > 0.0)) {
                v = INFINITY;
                atomicAdd(ninf, 1);
            }
            dk = v;
            d[kb + k] = v;
        }
        __syncthreads();
        const double dd = dk;
        // column k of L
        for (int i = k + 1 + threadIdx.x; i < nb; i += blockDim.x)
            T[i][k] = isinf(dd) ? 0.0 : T[i][k] / dd;
        __syncthreads();
        // rank-1 update of the remaining lower triangle: A_ij -= l_ik d_k l_jk
        if (!isinf(dd)) {
            const int rem = nb - k - 1;
            for (int t = threadIdx.x; t < rem * rem; t += blockDim.x) {
                const int i = k + 1 + t % rem, j = k + 1 + t / rem;
                if (i >= j) T[i][j] = fma(-T[i][k] * dd, T[j][k], T[i][j]);
            }
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) {
        const int i = t % nb, j = t / nb;
        if (i > j) A[(size_t)(kb + i) + (size_t)(kb + j) * n] = T[i][j];
    }
}

// rows below the diagonal block: w_i solves w L11^T = a_i; l_i = w D^-1
__global__ __launch_bounds__(256) void ldl_panel(int n, int kb, int nb, double *A,
                                                 const double *d, double *W) {
    __shared__ double L11[NB][NB + 1];
    __shared__ double dd[NB];
    for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) {
        const int i = t % nb, j = t / nb;
        L11[i][j] = (i > j) ? A[(size_t)(kb + i) + (size_t)(kb + j) * n] : 0.0;
    }
    for (int t = threadIdx.x; t < nb; t += blockDim.x) dd[t] = d[kb + t];
    __syncthreads();
    const int i = kb + nb + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double w[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        if (k < nb) {
            double v = A[(size_t)i + (size_t)(kb + k) * n];
            for (int t = 0; t < k; ++t) v = fma(-w[t], L11[k][t], v);
            w[k] = v;
        }
    }
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        if (k < nb) {
            const bool inf = isinf(dd[k]);
            const double wk = inf ? 0.0 : w[k];
            W[(size_t)(i - kb - nb) + (size_t)k * (n - kb - nb)] = wk;
            A[(size_t)i + (size_t)(kb + k) * n] = inf ? 0.0 : wk / dd[k];
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

// single-workgroup triangular solves with the factor
__global__ __launch_bounds__(1024) void ldl_solve_k(int n, const double *__restrict__ A,
                                                   const double *__restrict__ d, double *x) {
    // forward: L y = b (unit lower)
    for (int kb = 0; kb < n; kb += NB) {
        const int nb = min(NB, n - kb);
        for (int k = 0; k < nb; ++k) {
            __syncthreads();
            const double xk = x[kb + k];
            for (int i = kb + k + 1 + threadIdx.x; i < kb + nb; i += blockDim.x)
                x[i] = fma(-A[(size_t)i + (size_t)(kb + k) * n], xk, x[i]);
        }
        __syncthreads();
        for (int i = kb + nb + threadIdx.x; i < n; i += blockDim.x) {
            double v = x[i];
            for (int k = 0; k < nb; ++k) v = fma(-A[(size_t)i + (size_t)(kb + k) * n], x[kb + k], v);
            x[i] = v;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = isinf(d[i]) ? 0.0 : x[i] / d[i];
    // backward: L^T x = y
    for (int kb = ((n - 1) / NB) * NB; kb >= 0; kb -= NB) {
        const int nb = min(NB, n - kb);
        __syncthreads();
        // x[kb..kb+nb) -= sum_{i >= kb+nb} L(i, k) x[i]
        for (int k = threadIdx.x; k < nb; k += blockDim.x) {
            double v = x[kb + k];
            for (int i = kb + nb; i < n; ++i) v = fma(-A[(size_t)i + (size_t)(kb + k) * n], x[i], v);
            x[kb + k] = v;
        }
        __syncthreads();
        for (int k = nb - 1; k >= 0; --k) {
            __syncthreads();
            if (threadIdx.x == 0) {
                double v = x[kb + k];
                for (int i = kb + k + 1; i < kb + nb; ++i)
                    v = fma(-A[(size_t)i + (size_t)(kb + k) * n], x[i], v);
                x[kb + k] = v;
            }
        }
        __syncthreads();
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
    ninf_.need(1);
    hipLaunchKernelGGL(dense_zero, dim3(2048), dim3(256), 0, st, total, A);
    hipLaunchKernelGGL(dense_fill, dim3(n), dim3(64), 0, st, n, S.rowptr.get(), S.col.get(),
                       S.val.get(), A, orig_.get());
    OTIP_HIP(hipMemsetAsync(ninf_.get(), 0, sizeof(int), st));
    for (int kb = 0; kb < n; kb += NB) {
        const int nb = std::min(NB, n - kb);
        hipLaunchKernelGGL(ldl_diag, dim3(1), dim3(256), 0, st, n, kb, nb, A, orig_.get(),
                           d_.get(), pivtol, ninf_.get());
        const int rows = n - kb - nb;
        if (rows > 0) {
            hipLaunchKernelGGL(ldl_panel, dim3(grid_for(rows, 256)), dim3(256), 0, st, n, kb, nb,
                               A, d_.get(), W_.get());
            const unsigned tiles = grid_for(rows, NB);
            hipLaunchKernelGGL(ldl_update, dim3(tiles, tiles), dim3(256), 0, st, n, kb, nb, A,
                               W_.get());
        }
    }
    OTIP_HIP(hipGetLastError());
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
    if (x != b) OTIP_HIP(hipMemcpyAsync(x, b, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(ldl_solve_k, dim3(1), dim3(1024), 0, st, n, A_.get(), d_.get(), x);
    OTIP_HIP(hipGetLastError());
}

}  // namespace otip
