// Matrix-free Kronecker-structured products of Section 2.1 on a dense m x n
// array X stored column-major (x = vec(X)):
//   A_1 x = X e_n (row sums), A_2 x = X^T e_m (column sums)     -> kron_apply
//   A_1^T y + A_2^T z = vec(y e_n^T + e_m z^T)                  -> kron_apply_t
// Both stream X once through HBM; every other access stays on chip.
//
// kron_apply: a 256-thread block owns a tile of 1024 rows x 64 columns; each
// thread reads 2 x 2 adjacent rows of each column with 16-byte loads (a wave
// covers 1 KB contiguous per load), keeps its 4 running row sums in registers
// and reduces each column over the block.
// Partial sums per tile go to small side arrays that a second, fixed-order
// pass adds up, so the result is bitwise reproducible.
#include <mutex>

#include "internal.h"

namespace otip {

constexpr int KR_ROWS = 1024;  // rows per tile (4 per thread)
typedef double dv2 __attribute__((ext_vector_type(2)));
constexpr int KR_COLS = 64;    // columns per tile

__global__ __launch_bounds__(256) void kron_tile(int m, int n, const double *__restrict__ X,
                                                 double *__restrict__ prow,
                                                 double *__restrict__ pcol) {
    __shared__ double cs[4][KR_COLS];
    const int rt = blockIdx.x, ct = blockIdx.y;
    const int r0 = rt * KR_ROWS;
    const int j0 = ct * KR_COLS;
    const int jn = min(KR_COLS, n - j0);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // rows of this thread: r0 + 2t, r0 + 2t + 1 and the same 512 rows further
    const int ia = r0 + 2 * threadIdx.x, ib = ia + 512;
    double rs[4] = {0.0, 0.0, 0.0, 0.0};
    // 16-byte loads when every column of the tile starts 16-byte aligned (X
    // aligned, m even) and the tile has all its rows
    const bool wide = (m % 2 == 0) && r0 + KR_ROWS <= m && ((uintptr_t)X % 16 == 0);
    for (int c = 0; c < jn; ++c) {
        const double *col = X + (size_t)(j0 + c) * (size_t)m;
        double v[4];
        if (wide) {
            const dv2 va = __builtin_nontemporal_load((const dv2 *)(col + ia));
            const dv2 vb = __builtin_nontemporal_load((const dv2 *)(col + ib));
            v[0] = va.x;
            v[1] = va.y;
            v[2] = vb.x;
            v[3] = vb.y;
        } else {
            v[0] = ia < m ? col[ia] : 0.0;
            v[1] = ia + 1 < m ? col[ia + 1] : 0.0;
            v[2] = ib < m ? col[ib] : 0.0;
            v[3] = ib + 1 < m ? col[ib + 1] : 0.0;
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
    const int rows[4] = {ia, ia + 1, ib, ib + 1};
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (rows[q] < m) prow[(size_t)ct * m + rows[q]] = rs[q];
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

// X_ij = y_i + z_j: each block writes a 1024 x 64 tile, 16 bytes per lane and
// store when the columns are 16-byte aligned (m even) and the tile is full
__global__ __launch_bounds__(256) void kron_t_tile(int m, int n, const double *__restrict__ y,
                                                   const double *__restrict__ z,
                                                   double *__restrict__ X) {
    const int r0 = blockIdx.x * KR_ROWS;
    const int ia = r0 + 2 * threadIdx.x, ib = ia + 512;
    const int j0 = blockIdx.y * KR_COLS;
    const int jn = min(KR_COLS, n - j0);
    const int rows[4] = {ia, ia + 1, ib, ib + 1};
    double yv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) yv[q] = rows[q] < m ? y[rows[q]] : 0.0;
    const bool wide = (m % 2 == 0) && r0 + KR_ROWS <= m && ((uintptr_t)X % 16 == 0);
    for (int c = 0; c < jn; ++c) {
        const double zj = z[j0 + c];
        double *col = X + (size_t)(j0 + c) * (size_t)m;
        if (wide) {
            *(dv2 *)(col + ia) = dv2{yv[0] + zj, yv[1] + zj};
            *(dv2 *)(col + ib) = dv2{yv[2] + zj, yv[3] + zj};
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (rows[q] < m) col[rows[q]] = yv[q] + zj;
        }
    }
}

// ------------------------------------------------------- allocation-free variant
// The partial sums of kron_apply live in one file-scope device array per GPU
// instead of context buffers.  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol): the device
// address of each GPU's copy is resolved once per device by
// kron_scratch_init and used from then on.
static __device__ __align__(256) double scratch[kKronScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
double *scratch_ptr[kMaxDevices] = {};
}  // namespace

void kron_scratch_init(int device) {
    OTIP_CHECK(device >= 0 && device < kMaxDevices, OTIP_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> g(scratch_mu);
    if (scratch_ptr[device]) return;
    void *p = nullptr;
    OTIP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    OTIP_CHECK(p != nullptr, OTIP_EHIP, "scratch array has no device address");
    scratch_ptr[device] = (double *)p;
}

int64_t kron_scratch_need(int m, int n) {
    const int64_t rtiles = (m + KR_ROWS - 1) / KR_ROWS, ctiles = (n + KR_COLS - 1) / KR_COLS;
    return ctiles * (int64_t)m + rtiles * (int64_t)n;
}

void kron_apply_noalloc(hipStream_t st, int device, int m, int n, const double *X,
                        double *rowsum, double *colsum) {
    OTIP_CHECK(device >= 0 && device < kMaxDevices, OTIP_EINVAL, "device index out of range");
    double *base;
    {
        std::lock_guard<std::mutex> g(scratch_mu);
        base = scratch_ptr[device];
    }
    OTIP_CHECK(base != nullptr, OTIP_EHIP, "scratch not set up on this device");
    const int64_t need = kron_scratch_need(m, n);
    OTIP_CHECK(need <= kKronScratchDoubles, OTIP_EINVAL,
               "otip_kron_apply_noalloc: m x n needs " + std::to_string(need) +
                   " partial sums, more than the " + std::to_string(kKronScratchDoubles) +
                   " of the static scratch");
    const int rtiles = (m + KR_ROWS - 1) / KR_ROWS, ctiles = (n + KR_COLS - 1) / KR_COLS;
    double *prow = base, *pcol = base + (size_t)ctiles * m;
    // every partial read by kron_finish is written by kron_tile: nothing to clear
    hipLaunchKernelGGL(kron_tile, dim3(rtiles, ctiles), dim3(256), 0, st, m, n, X, prow, pcol);
    hipLaunchKernelGGL(kron_finish, dim3(grid_for(m, 256)), dim3(256), 0, st, m, ctiles,
                       (const double *)prow, rowsum);
    hipLaunchKernelGGL(kron_finish, dim3(grid_for(n, 256)), dim3(256), 0, st, n, rtiles,
                       (const double *)pcol, colsum);
    OTIP_HIP(hipGetLastError());
}

void kron_apply_t(hipStream_t st, int m, int n, const double *y, const double *z, double *X) {
    const int rtiles = (m + KR_ROWS - 1) / KR_ROWS, ctiles = (n + KR_COLS - 1) / KR_COLS;
    hipLaunchKernelGGL(kron_t_tile, dim3(rtiles, ctiles), dim3(256), 0, st, m, n, y, z, X);
    OTIP_HIP(hipGetLastError());
}

}  // namespace otip
