// Matrix-free Kronecker-structured products of Section 2.1 on a dense m x n
// array X stored column-major (x = vec(X)):
//   A_1 x = X e_n (row sums), A_2 x = X^T e_m (column sums)     -> kron_apply
//   A_1^T y + A_2^T z = vec(y e_n^T + e_m z^T)                  -> kron_apply_t
// Both stream X once through HBM; every other access stays on chip.
//
// kron_apply: a 256-thread block owns a tile of 1024 rows x 64 columns; each
// thread reads 4 rows of each column (coalesced along the column), keeps its 4
// running row sums in registers and reduces each column over the block.
// Partial sums per tile go to small side arrays that a second, fixed-order
// pass adds up, so the result is bitwise reproducible.
#include "internal.h"

namespace otip {

constexpr int KR_ROWS = 1024;  // rows per tile (4 per thread)
constexpr int KR_COLS = 64;    // columns per tile

__global__ __launch_bounds__(256) void kron_tile(int m, int n, const double *__restrict__ X,
                                                 double *__restrict__ prow,
                                                 double *__restrict__ pcol) {
    __shared__ double cs[4][KR_COLS];
    const int rt = blockIdx.x, ct = blockIdx.y;
    const int i0 = rt * KR_ROWS + threadIdx.x;
    const int j0 = ct * KR_COLS;
    const int jn = min(KR_COLS, n - j0);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double rs[4] = {0.0, 0.0, 0.0, 0.0};
    const bool full = (rt + 1) * KR_ROWS <= m;
    for (int c = 0; c < jn; ++c) {
        const double *col = X + (size_t)(j0 + c) * (size_t)m;
        double v[4];
        if (full) {
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = __builtin_nontemporal_load(&col[i0 + 256 * q]);
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = i0 + 256 * q;
                v[q] = i < m ? __builtin_nontemporal_load(&col[i]) : 0.0;
            }
        }
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            rs[q] += v[q];
            t += v[q];
        }
        t = wave_sum(t);
        if (lane == 0) cs[w][c] = t;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < jn; c += 256)
        pcol[(size_t)rt * n + j0 + c] = ((cs[0][c] + cs[1][c]) + cs[2][c]) + cs[3][c];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = i0 + 256 * q;
        if (i < m) prow[(size_t)ct * m + i] = rs[q];
    }
}

__global__ void kron_finish(int len, int parts, const double *__restrict__ part,
                            double *__restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= len) return;
    double s = 0.0;
    for (int q = 0; q < parts; ++q) s += part[(size_t)q * len + t];
    out[t] = s;
}

void kron_apply(hipStream_t st, int m, int n, const double *X, double *rowsum, double *colsum,
                DBuf<double> &prow, DBuf<double> &pcol) {
    const int rtiles = (m + KR_ROWS - 1) / KR_ROWS, ctiles = (n + KR_COLS - 1) / KR_COLS;
    prow.need((size_t)ctiles * m);
    pcol.need((size_t)rtiles * n);
    hipLaunchKernelGGL(kron_tile, dim3(rtiles, ctiles), dim3(256), 0, st, m, n, X, prow.get(),
                       pcol.get());
    hipLaunchKernelGGL(kron_finish, dim3(grid_for(m, 256)), dim3(256), 0, st, m, ctiles,
                       prow.get(), rowsum);
    hipLaunchKernelGGL(kron_finish, dim3(grid_for(n, 256)), dim3(256), 0, st, n, rtiles,
                       pcol.get(), colsum);
    OTIP_HIP(hipGetLastError());
}

// X_ij = y_i + z_j: each block writes a 1024 x 64 tile, rows along the lanes
__global__ __launch_bounds__(256) void kron_t_tile(int m, int n, const double *__restrict__ y,
                                                   const double *__restrict__ z,
                                                   double *__restrict__ X) {
    const int i0 = blockIdx.x * KR_ROWS + threadIdx.x;
    const int j0 = blockIdx.y * KR_COLS;
    const int jn = min(KR_COLS, n - j0);
    double yv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = i0 + 256 * q;
        yv[q] = i < m ? y[i] : 0.0;
    }
    for (int c = 0; c < jn; ++c) {
        const double zj = z[j0 + c];
        double *col = X + (size_t)(j0 + c) * (size_t)m;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = i0 + 256 * q;
            if (i < m) __builtin_nontemporal_store(yv[q] + zj, &col[i]);
        }
    }
}

void kron_apply_t(hipStream_t st, int m, int n, const double *y, const double *z, double *X) {
    const int rtiles = (m + KR_ROWS - 1) / KR_ROWS, ctiles = (n + KR_COLS - 1) / KR_COLS;
    hipLaunchKernelGGL(kron_t_tile, dim3(rtiles, ctiles), dim3(256), 0, st, m, n, y, z, X);
    OTIP_HIP(hipGetLastError());
}

}  // namespace otip
