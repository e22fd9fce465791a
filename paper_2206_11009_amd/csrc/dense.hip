// Dense LDL^T of the Schur complement with the infinite-pivot rule
// (Section 4.2: after the switch the Schur complement is factorised exactly;
// its zero pivot is replaced by an infinitely large value).
//
// Right-looking blocked factorisation of the lower triangle of a column-major
// n x n array, block width 64:
//   1. the 64 x 64 diagonal block is factorised by one wavefront while a
//      second inverts its unit lower factor, column by column behind it;
//   2. the rows below form W21 = A21 L11^-T (= L21 D1) and L21 = W21 D1^-1;
//   3. the trailing lower triangle is updated, A22 -= L21 W21^T, in 128 x 64
//      tiles once per group of four block steps (16-row tiles where only the
//      next block column is updated, inside a group).
// Steps 2 and 3 run on the FP64 matrix cores with operands loaded straight
// into registers.
// A pivot d_k <= pivtol * S_kk (original diagonal) or d_k <= 0 becomes +inf:
// its column of L is zero and the solve returns 0 for that unknown.
// After the factorisation X = L^-1 is formed (recursive doubling with tiled
// products), so that each solve x = X^T D^-1 X b is two matrix-vector
// products instead of a chain of dependent triangular steps; for large n
// without its top level, the solves then applying L21 between the halves.
#include "internal.h"

namespace otip {

constexpr int NB = 64;

// FP64 matrix core: D(16x16) += A(16x4) B(4x16).  Lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; it receives D[mfma_row(l, q)][l % 16] in register q.
typedef double d4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ int mfma_row(int lane, int q) { return (lane >> 4) + 4 * q; }
__device__ __forceinline__ d4 mfma4(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

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

// Factor the diagonal block [kb, kb+nb) and invert its unit lower factor, four
// wavefronts.  Wave q keeps, for lane i, columns [16q, 16q+16) of row i of the
// block and rows [16q, 16q+16) of column i of L11^-1, in registers.  Pivot k
// (right-looking) takes one workgroup barrier: the wave that holds column k
// reads the pivot from lane k (v_readlane), forms every row's l = u_k / d_k
// and writes it to row k of Lt (Lt[k][r] = L(r, k): column k of L,
// contiguous); after the barrier each wave reads its 16 entries of that column
// as LDS broadcasts (all lanes read one address) and applies the rank-one
// update to its columns of every row, and step k of the inverse (L11 x = e_c,
// x_r -= L(r, k) x_k) to its rows of every column.  x_k is published in Xs by
// the wave that holds row k once step k - 1 is applied.  Entries that a step
// does not change (columns and rows at or left of k, where column k of L is
// zero) take an exact no-op, and waves whose 16 columns and rows are all
// finished skip the step.  The pivot chain is the kernel's bound: one wave
// does all of a pivot's dependent work (pivot test, division, publication),
// while the rank-one work is spread over four SIMDs.
constexpr int kDiagWaves = 4;
constexpr int kDiagCols = NB / kDiagWaves;  // columns (and inverse rows) per wave

// s_waitcnt operand (GFX9 encoding) that waits for every vector memory load of
// the wave: vmcnt 0, expcnt and lgkmcnt at their maxima (no wait)
constexpr int kWaitVmcnt0 = 0x0F70;

__device__ __forceinline__ int wave_max_i(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ double rdlane(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

__global__ __launch_bounds__(64 * kDiagWaves) void ldl_diag(int n, int kb, int nb, double *A,
                                                            const double *orig, double *d,
                                                            double pivtol, int *ninf,
                                                            double *Linv) {
    __shared__ __align__(16) double Lt[NB][NB];  // Lt[k][r] = L(r, k)
    __shared__ double Xs[NB][NB];                // Xs[s][c] = L11^-1 (s, c), final
    __shared__ double Ls[NB][NB + 1];            // L11^-1, transposed for the store
    __shared__ double pm[NB];                    // d_k, or 0 where pivot k is dropped
    const int i = threadIdx.x & 63;
    const int q0 = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) * kDiagCols;
    double u[kDiagCols], x[kDiagCols];  // row i: columns q0 + m; L11^-1 column i: rows q0 + m
#pragma unroll
    for (int m = 0; m < kDiagCols; ++m) {
        const int c = q0 + m;
        u[m] = (i < nb && c < nb && c <= i) ? A[(size_t)(kb + i) + (size_t)(kb + c) * n] : 0.0;
        x[m] = (c == i) ? 1.0 : 0.0;
    }
    const double oi = (i < nb) ? orig[kb + i] : 1.0;
    int ninf_local = 0;
    if (q0 == 0) Xs[0][i] = x[0];
    for (int kq = 0; kq < kDiagWaves; ++kq) {
        const int owner = kq * kDiagCols;
#pragma unroll
        for (int m = 0; m < kDiagCols; ++m) {
            const int k = owner + m;
            if (q0 == owner) {
                const bool act = k < nb;
                double piv = rdlane(u[m], k);
                const bool bad = !(piv > pivtol * rdlane(oi, k)) || !(piv > 0.0);
                piv = bad ? INFINITY : piv;
                const bool fin = act && !bad;
                ninf_local += (act && bad) ? 1 : 0;
                Lt[k][i] = (fin && i > k && i < nb) ? u[m] / piv : 0.0;
                if (i == 0) {
                    pm[k] = fin ? piv : 0.0;
                    if (act) d[kb + k] = piv;
                }
            }
            __syncthreads();
            if (q0 >= owner) {
                const double ld = Lt[k][i] * pm[k];  // l_i d_k, 0 for a dropped pivot
                const double xk = Xs[k][i];
#pragma unroll
                for (int m2 = 0; m2 < kDiagCols; ++m2) {
                    const double lj = Lt[k][q0 + m2];
                    u[m2] = fma(-ld, lj, u[m2]);
                    x[m2] = fma(-lj, xk, x[m2]);
                }
                const int m1 = (m + 1) % kDiagCols;
                const int next = (m + 1 == kDiagCols) ? owner + kDiagCols : owner;
                if (k + 1 < NB && q0 == next) Xs[k + 1][i] = x[m1];
            }
        }
    }
#pragma unroll
    for (int m = 0; m < kDiagCols; ++m) Ls[q0 + m][i] = x[m];
    if (i == 0 && ninf_local) atomicAdd(ninf, ninf_local);
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kDiagCols; ++m) {
        const int c = q0 + m;
        if (i < nb && c < i) A[(size_t)(kb + i) + (size_t)(kb + c) * n] = Lt[c][i];
        Linv[(size_t)i + (size_t)c * NB] = Ls[i][c];
    }
}

// Rows below the diagonal block: W21 = A21 L11^-T (so W21 = L21 D1) and
// L21 = W21 D1^-1.  One workgroup per TR-row tile forms W = A21 Linv^T on the
// FP64 matrix cores (Linv is zero above its diagonal); its four waves split
// the TR x 64 tile into blocks of 16 x 16, with their operands loaded straight
// from global memory into the registers of the matrix-core layout (no LDS;
// one barrier before the in-place store of L21).  Small tiles (TR = 16) give
// the early block steps enough workgroups and each wave a short chain of
// products.
template <int TR>
__global__ __launch_bounds__(256) void ldl_panel(int n, int kb, int nb, double *A,
                                                 const double *d, double *W,
                                                 const double *Linv,
                                                 unsigned long long *nnz, int *hrow) {
    // the four waves split the TR x 64 tile into WC column groups of 64 / WC
    // columns and 4 / WC row groups: UR 16-row and VC 16-column blocks each
    constexpr int WC = TR >= 32 ? 2 : 4;
    constexpr int UR = TR / (4 / WC) / 16, VC = 64 / WC / 16;
    int nz = 0;     // nonzeros of L21 written here (the fill statistic)
    int last = -1;  // the last row with a nonzero entry of L21 or W21 written here
    const int r0 = kb + nb + blockIdx.x * TR;
    const int rows = n - kb - nb;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = (wave / WC) * (16 * UR), wc = (wave % WC) * (16 * VC);
    const int li = lane & 15, lk = lane >> 4;
    // operands: A(r0 + wr + 16u + li, kb + c) and Linv(wc + 16v + li, c), c = 4t + lk
    double av[UR][16], bv[VC][16];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int c = 4 * t + lk;
#pragma unroll
        for (int u = 0; u < UR; ++u) {
            const int ii = r0 + wr + 16 * u + li;
            av[u][t] = (ii < n && c < nb) ? A[(size_t)ii + (size_t)(kb + c) * n] : 0.0;
        }
#pragma unroll
        for (int v = 0; v < VC; ++v) bv[v][t] = Linv[(size_t)(wc + 16 * v + li) + (size_t)c * NB];
    }
    d4 acc[UR][VC];
#pragma unroll
    for (int u = 0; u < UR; ++u)
#pragma unroll
        for (int v = 0; v < VC; ++v) acc[u][v] = d4{0.0, 0.0, 0.0, 0.0};
    // W(a, k) = sum_c A(a, c) Linv(k, c)
#pragma unroll
    for (int t = 0; t < 16; ++t)
#pragma unroll
        for (int u = 0; u < UR; ++u)
#pragma unroll
            for (int v = 0; v < VC; ++v) acc[u][v] = mfma4(av[u][t], bv[v][t], acc[u][v]);
    // L21 overwrites A21 in place, and the waves that share a row block each
    // store a different column slice of it after reading the whole row: every
    // wave's loads have returned (vmcnt 0; the barrier alone lets the compiler
    // leave some in flight across it) before any wave of the workgroup stores.
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < UR; ++u)
#pragma unroll
        for (int v = 0; v < VC; ++v)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = r0 + wr + 16 * u + mfma_row(lane, q);
                const int k = wc + 16 * v + li;
                if (i < n && k < nb) {
                    const double dd = d[kb + k];
                    const bool inf = isinf(dd);
                    const double wk = inf ? 0.0 : acc[u][v][q];
                    const double lv = inf ? 0.0 : wk / dd;
                    W[(size_t)(i - kb - nb) + (size_t)k * rows] = wk;
                    A[(size_t)i + (size_t)(kb + k) * n] = lv;
                    nz += lv != 0.0;
                    if (wk != 0.0 || lv != 0.0) last = max(last, i);
                }
            }
    nz = wave_sum_i(nz);
    if ((threadIdx.x & 63) == 0 && nz) atomicAdd(nnz, (unsigned long long)nz);
    last = wave_max_i(last);
    if ((threadIdx.x & 63) == 0 && last >= 0) atomicMax(hrow + kb / NB, last);
}

// rows per panel workgroup
constexpr int kPanelRows = 16;

// A22 -= sum over panels of L21 W21^T on the lower triangle of the trailing
// matrix that starts at row and column r0, in TR x 64 tiles, one workgroup per
// tile that reaches the triangle (1D grid, tiles in row-major order from the
// block index); each of the four waves forms a (TR / 2) x 32 part of the tile
// as blocks of 16x16 matrix-core products, with its operands loaded straight
// from global memory into the registers of the matrix-core layout (no LDS, no
// barrier; entries above the diagonal are computed and not stored).  Panel p
// holds the 64 columns [kcol, kcol + 64) of L (in A) and its W with row r0 + j
// at wrow0 + j (leading dimension wld); a panel always has 64 columns, since
// only a block with rows below it forms one.  Up to kDenseUpdPanels panels per
// launch: the trailing matrix is read and written once per group of block
// steps.  first_col restricts the launch to the first tile column (the next
// diagonal block and the rows below it).
//
// Rows past the trailing matrix (in the last tile row or column when its order
// is not a multiple of 64) are clamped to its last row: they read valid memory
// and feed only outputs that are not stored, so no load is conditional.  Every
// address is a wave-uniform base plus a 32-bit lane offset fixed for the whole
// tile, so the loads of a k step need no per-lane address arithmetic.
struct UpdPanel {
    const double *W;
    int kcol, wrow0, wld;
};
struct UpdArgs {
    int n, r0, first_col;
    // hrow[q]: the last row with a nonzero entry in block q's L21 or W21 (-1:
    // none).  Rows and columns of the trailing matrix beyond the group's last
    // such row take exactly zero from its panels, so their tiles are skipped:
    // the factors of these Schur complements are banded (a few percent of n^2).
    const int *hrow;
    UpdPanel p[kDenseUpdPanels];
};
__device__ __forceinline__ double ld_at(const double *base, uint32_t byte_off) {
    return *(const double *)((const char *)base + byte_off);
}
// TR: rows per workgroup tile.  The triangle takes TR = kUpdRows (128); a
// first-column launch uses TR = 16 (one workgroup per 16 rows of the 64-wide
// block column, four waves of 16 x 16 across its columns), which fills the
// chip in the early block steps and shortens each wave's chain.
template <int NP, int TR>
__global__ __launch_bounds__(256) void ldl_update(double *A, UpdArgs a) {
    constexpr int WC = TR >= 32 ? 2 : 4;
    constexpr int UR = TR / (4 / WC) / 16, VC = 64 / WC / 16;
    const int n = a.n, r0 = a.r0;
    const int rows = n - r0, last = rows - 1;
    const int blk = blockIdx.x;
    // rows (relative to r0) that the group's panels reach
    int reach = -1;
#pragma unroll
    for (int pi = 0; pi < NP; ++pi) reach = max(reach, a.hrow[a.p[pi].kcol / NB]);
    const int live = min(rows, reach - r0 + 1);
    int i0, j0;
    if (a.first_col) {
        i0 = blk * TR;
        j0 = 0;
        if (i0 >= live) return;  // (no barrier follows)
    } else {
        // TR x 64 tiles of the triangle: tile row a (rows TR a..) holds the
        // (TR / 64)(a + 1) column tiles that reach its diagonal
        constexpr int H = TR >= NB ? TR / NB : 1;  // (the 16-row form is first-column only)
        // tile row a starts at block H a (a + 1) / 2
        int ta = (int)((sqrt(8.0 * blk / H + 1.0) - 1.0) * 0.5);
        while (H * (ta + 1) * (ta + 2) / 2 <= blk) ++ta;
        while (H * ta * (ta + 1) / 2 > blk) --ta;
        const int tb = blk - H * ta * (ta + 1) / 2;
        i0 = ta * TR;
        j0 = tb * NB;
        // outside the triangle or beyond the panels' reach (no barrier follows)
        if (i0 >= live || j0 >= live || j0 >= i0 + TR) return;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = (wave / WC) * (16 * UR), wc = (wave % WC) * (16 * VC);
    const int li = lane & 15, lk = lane >> 4;
    // the tile: base at (r0, r0 + j0), lane offsets of its entries (clamped)
    double *C = A + (size_t)(r0 + j0) * n + r0;
    uint32_t coff[UR][VC][4];
    double cur[UR][VC][4];
#pragma unroll
    for (int u = 0; u < UR; ++u)
#pragma unroll
        for (int v = 0; v < VC; ++v)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int ii = min(i0 + wr + 16 * u + mfma_row(lane, q), last);
                const int jj = min(j0 + wc + 16 * v + li, last) - j0;
                coff[u][v][q] = 8u * ((uint32_t)ii + (uint32_t)jj * (uint32_t)n);
                // requested with the operands, so that the latency is hidden
                cur[u][v][q] = ld_at(C, coff[u][v][q]);
            }
    // operand rows of this lane (clamped), relative to r0
    int ar[UR], br[VC];
#pragma unroll
    for (int u = 0; u < UR; ++u) ar[u] = min(i0 + wr + 16 * u + li, last);
#pragma unroll
    for (int v = 0; v < VC; ++v) br[v] = min(j0 + wc + 16 * v + li, last);
    d4 acc[UR][VC];
#pragma unroll
    for (int u = 0; u < UR; ++u)
#pragma unroll
        for (int v = 0; v < VC; ++v) acc[u][v] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int pi = 0; pi < NP; ++pi) {
        const UpdPanel P = a.p[pi];
        // operands: L(r0 + ar[u], kcol + k) and W(wrow0 + br[v], k), k = 4t + lk
        const double *Lb = A + (size_t)P.kcol * n + r0;
        const double *Wb = P.W + P.wrow0;
        uint32_t ao[UR], bo[VC];
#pragma unroll
        for (int u = 0; u < UR; ++u) ao[u] = 8u * ((uint32_t)ar[u] + (uint32_t)lk * (uint32_t)n);
#pragma unroll
        for (int v = 0; v < VC; ++v)
            bo[v] = 8u * ((uint32_t)br[v] + (uint32_t)lk * (uint32_t)P.wld);
        double av[UR][16], bv[VC][16];
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const double *Lt = Lb + (size_t)(4 * t) * n;
            const double *Wt = Wb + (size_t)(4 * t) * P.wld;
#pragma unroll
            for (int u = 0; u < UR; ++u) av[u][t] = ld_at(Lt, ao[u]);
#pragma unroll
            for (int v = 0; v < VC; ++v) bv[v][t] = ld_at(Wt, bo[v]);
        }
#pragma unroll
        for (int t = 0; t < 16; ++t)
#pragma unroll
            for (int u = 0; u < UR; ++u)
#pragma unroll
                for (int v = 0; v < VC; ++v) acc[u][v] = mfma4(av[u][t], bv[v][t], acc[u][v]);
    }
#pragma unroll
    for (int u = 0; u < UR; ++u)
#pragma unroll
        for (int v = 0; v < VC; ++v)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int ii = i0 + wr + 16 * u + mfma_row(lane, q);
                const int jj = j0 + wc + 16 * v + li;
                if (ii < rows && jj < rows && ii >= jj)
                    *(double *)((char *)C + coff[u][v][q]) = cur[u][v][q] - acc[u][v][q];
            }
}

// rows per workgroup of a first-column update, and of a trailing-update tile
// (128 x 64: each wave forms 64 x 32, 4 x 2 blocks of 16 x 16, so that six
// operand loads feed eight matrix-core products instead of four feeding four;
// 413 -> 383 ms of updates per 128 x 128 LP against 64 x 64 tiles)
constexpr int kFirstColRows = 16;
constexpr int kUpdRows = 128;

// X = L^-1 by recursive doubling.  The 64 x 64 diagonal blocks of X are the
// block inverses from ldl_diag.  At level b (b = 64, 128, ...) every pair of
// consecutive diagonal blocks [c1, c1+b), [r2, r2+b') (r2 = c1 + b) whose
// inverses are known gives the off-diagonal block of the inverse of the pair:
//   X(r2.., c1..) = -X22 L21 X11,
// computed as T = L21 X11 (mode 0), then X21 = -X22 T (mode 1).  Both are
// 64 x 64-tiled products that skip the zero tiles of the triangular factors.
__global__ void inv_init(int n, const double *__restrict__ linv, double *__restrict__ X) {
    const int blk = blockIdx.x, kb = blk * NB;
    for (int t = threadIdx.x; t < NB * NB; t += blockDim.x) {
        const int r = t % NB, c = t / NB;
        if (kb + r < n && kb + c < n)
            X[(size_t)(kb + r) + (size_t)(kb + c) * n] = linv[(size_t)blk * NB * NB + t];
    }
}

// Reduction chunk of inv_mul: 32 columns of the left operand and 32 rows of
// the right one per LDS stage (33 KB of LDS per workgroup instead of 66 KB
// with 64-wide chunks, so four workgroups fit a compute unit's 160 KB).  The
// mode is a template parameter, each thread's chunk elements keep one row and
// step in columns, and rows outside the matrix are clamped with their values
// replaced by 0 (no branches); held to 128 VGPRs, four waves per SIMD.
constexpr int kInvKC = 32;
template <int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void inv_mul(
    int n, int b, const double *__restrict__ L,
                                               double *__restrict__ X, double *__restrict__ T) {
    const int p = blockIdx.z;
    const int c1 = 2 * p * b, r2 = c1 + b;
    const int rows2 = min(b, n - r2);
    // a tile's work grows with b/64 - tj (MODE 0) or with ti (MODE 1); the
    // slower-varying grid index walks it from the heaviest tiles down, so the
    // launch ends on light tiles
    const int ti = MODE == 0 ? blockIdx.x : (int)gridDim.y - 1 - (int)blockIdx.y;
    const int tj = MODE == 0 ? blockIdx.y : blockIdx.x;
    if (ti * NB >= rows2) return;
    __shared__ double As[NB][kInvKC + 1];
    __shared__ double Bs[kInvKC][NB + 1];
    double *Tp = T + (size_t)p * b * b;  // b x b column-major, rows < rows2 used
    // MODE 0: A(r, k) = L(r2 + r, c1 + k), B(k, c) = X(c1 + k, c1 + c), zero for k < c
    // MODE 1: A(r, k) = X(r2 + r, r2 + k), zero for k > r; B(k, c) = T(k, c)
    // (chunk indices: kInvKC columns of A and rows of B each)
    constexpr int per64 = NB / kInvKC;
    const int kt0 = MODE == 0 ? tj * per64 : 0;
    const int kt1 = MODE == 0 ? (b / NB) * per64 : (ti + 1) * per64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    d4 acc[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc[u][v] = d4{0.0, 0.0, 0.0, 0.0};
    // Thread tid moves A chunk elements (q, k) = (tid % 64, tid / 64 + 4e) and
    // B chunk elements (k2, c) = (tid % 32, tid / 32 + 8e), e < kE: the row in
    // memory is fixed per thread, the column steps by 4 (A) or 8 (B).
    constexpr int kE = NB * kInvKC / 256;
    const int q = threadIdx.x % NB, k0 = threadIdx.x / NB;
    const int k2 = threadIdx.x % kInvKC, cb0 = threadIdx.x / kInvKC;
    const int ar = ti * NB + q;
    const bool a_in = ar < rows2;
    const int arc = min(ar, rows2 - 1);
    // column-major operands: A base at (row base, column base), B likewise
    const double *Abase = MODE == 0 ? L + (size_t)(c1)*n + r2 : X + (size_t)r2 * n + r2;
    const int lda = n;
    const double *Bbase = MODE == 0 ? X + (size_t)(c1 + tj * NB) * n + c1 : Tp + (size_t)(tj * NB) * b;
    const int ldb = MODE == 0 ? n : b;
    double pa[kE], pb[kE];
    auto fetch = [&](int kt) {
        const int kc = kt * kInvKC;  // first reduction index of the chunk
        const double *Ak = Abase + (size_t)kc * lda;
        // B row of this thread, clamped (MODE 1 reads T rows below rows2 as 0)
        const int bk = kc + k2;
        const bool b_in = MODE == 0 || bk < rows2;
        const int bkc = MODE == 0 ? bk : min(bk, rows2 - 1);
#pragma unroll
        for (int e = 0; e < kE; ++e) {
            const int k = k0 + 4 * e;
            double av, bv;
            if (MODE == 0) {
                av = Ak[(size_t)arc + (size_t)k * lda];
                av = a_in ? av : 0.0;
            } else {
                const int ak = kc + k;
                const int akc = min(ak, rows2 - 1);
                av = Abase[(size_t)arc + (size_t)akc * lda];
                av = (a_in && ak < rows2) ? av : 0.0;
            }
            bv = Bbase[(size_t)bkc + (size_t)(cb0 + 8 * e) * ldb];
            pa[e] = av;
            pb[e] = b_in ? bv : 0.0;
        }
    };
    if (kt0 < kt1) fetch(kt0);
    for (int kt = kt0; kt < kt1; ++kt) {
#pragma unroll
        for (int e = 0; e < kE; ++e) {
            As[q][k0 + 4 * e] = pa[e];
            Bs[k2][cb0 + 8 * e] = pb[e];
        }
        __syncthreads();
        if (kt + 1 < kt1) fetch(kt + 1);
#pragma unroll
        for (int k = 0; k < kInvKC; k += 4) {
            const double a0 = As[wr + li][k + lk], a1 = As[wr + 16 + li][k + lk];
            const double b0 = Bs[k + lk][wc + li], b1 = Bs[k + lk][wc + 16 + li];
            acc[0][0] = mfma4(a0, b0, acc[0][0]);
            acc[0][1] = mfma4(a0, b1, acc[0][1]);
            acc[1][0] = mfma4(a1, b0, acc[1][0]);
            acc[1][1] = mfma4(a1, b1, acc[1][1]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
                const int r = ti * NB + wr + 16 * u + mfma_row(lane, qq);
                const int c = tj * NB + wc + 16 * v + li;
                if (r >= rows2) continue;
                if (MODE == 0)
                    Tp[(size_t)r + (size_t)c * b] = acc[u][v][qq];
                else
                    X[(size_t)(r2 + r) + (size_t)(c1 + c) * n] = -acc[u][v][qq];
            }
}

// Solve L D L^T x = b with X = L^-1 (unit lower, column-major) and XT, the
// strict upper part of X^T, by products with one wavefront per entry.  Without
// a split: forward y_i = (b_i + sum_{j<i} X(i, j) b_j) / d_i (infinite pivot:
// 0), backward x_j = y_j + sum_{i>j} X(i, j) y_i.  With a split at h (the top
// doubling level not formed, X holding only the diagonal inverses X11 and
// X22), the factor's own block L21 sits between them:
//   z1 = X11 b1,  z2 = X22 (b2 - L21 z1),  y = D^-1 z,
//   x2 = X22^T y2,  x1 = X11^T (y1 - L21^T x2).
// One lane's share of a wavefront's dot product: sum of a[k] v[k] for k = k0,
// k0 + 64, ... below k1, in four independent chains so that four loads of
// each operand are in flight.
__device__ __forceinline__ double dot4(const double *__restrict__ a,
                                       const double *__restrict__ v, int k0, int k1) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int k = k0;
    for (; k + 192 < k1; k += 256) {
        s0 = fma(a[k], v[k], s0);
        s1 = fma(a[k + 64], v[k + 64], s1);
        s2 = fma(a[k + 128], v[k + 128], s2);
        s3 = fma(a[k + 192], v[k + 192], s3);
    }
    for (; k < k1; k += 64) s0 = fma(a[k], v[k], s0);
    return (s0 + s1) + (s2 + s3);
}

// Rows: out_i = base_i + sgn sum_{j0 <= j < min(i, j1)} M(i, j) v_j for i in
// [i0, i1), with M(i, j) read as MT(j, i) (column i of MT is row i of M), and
// y_i = out_i / d_i when y is given.
__global__ __launch_bounds__(256) void x_rows(int n, int i0, int i1, int j0, int j1,
                                              const double *__restrict__ MT,
                                              const double *__restrict__ v,
                                              const double *__restrict__ base, double sgn,
                                              const double *__restrict__ d,
                                              double *__restrict__ out, double *__restrict__ y) {
    const int i = i0 + blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (i >= i1) return;
    const double *col = MT + (size_t)i * n;
    const double acc = wave_sum(dot4(col, v, j0 + lane, min(i, j1)));
    if (lane == 0) {
        const double val = base[i] + sgn * acc;
        if (out) out[i] = val;
        if (y) y[i] = isinf(d[i]) ? 0.0 : val / d[i];
    }
}

// Columns: out_j = base_j + sgn sum_{max(j+1, i0) <= i < i1} M(i, j) v_i for j
// in [j0, j1) (column j of M is contiguous).
__global__ __launch_bounds__(256) void x_cols(int n, int j0, int j1, int i0, int i1,
                                              const double *__restrict__ M,
                                              const double *__restrict__ v,
                                              const double *__restrict__ base, double sgn,
                                              double *__restrict__ out) {
    const int j = j0 + blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (j >= j1) return;
    const double *col = M + (size_t)j * n;
    const double acc = wave_sum(dot4(col, v, max(j + 1, i0) + lane, i1));
    if (lane == 0) out[j] = base[j] + sgn * acc;
}

// Substitution solves, one launch per 64-wide block column (used for a
// factorisation whose explicit inverse is not finite).  Every workgroup
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
// Nonzeros of the strict lower part of every 64 x 64 diagonal block of L (one
// workgroup per block), for the fill statistic; the panels count the rest.
__global__ __launch_bounds__(256) void count_diag_blocks(int n, const double *__restrict__ A,
                                                         unsigned long long *nnz) {
    const int kb = blockIdx.x * NB, nb = min(NB, n - kb);
    int c = 0;
    for (int t = threadIdx.x; t < NB * NB; t += 256) {
        const int r = t % NB, q = t / NB;
        c += (r < nb && q < r) && A[(size_t)(kb + r) + (size_t)(kb + q) * n] != 0.0;
    }
    c = wave_sum_i(c);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(nnz, (unsigned long long)c);
}

// (and, with a flag, sets it when an entry of the strict lower part is not
// finite).  With L2, the block of rows >= h and columns < h comes from L2.
__global__ __launch_bounds__(256) void transpose_lower(int n, const double *__restrict__ L1,
                                                       double *__restrict__ U, int *flag,
                                                       const double *__restrict__ L2, int h) {
    __shared__ double tile[64][65];
    const int bi = blockIdx.x * 64, bj = blockIdx.y * 64;  // tile of L: rows bi.., cols bj..
    if (blockIdx.y > blockIdx.x) return;
    const double *L = (L2 && bi >= h && bj < h) ? L2 : L1;
    bool bad = false;
    for (int t = threadIdx.x; t < 64 * 64; t += 256) {
        const int r = t % 64, c = t / 64;
        const int i = bi + r, j = bj + c;
        const double v = (i < n && j < n && i > j) ? L[(size_t)i + (size_t)j * n] : 0.0;
        bad |= !isfinite(v);
        tile[r][c] = v;
    }
    if (flag && __ballot(bad) != 0ull && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
    __syncthreads();
    for (int t = threadIdx.x; t < 64 * 64; t += 256) {
        const int r = t % 64, c = t / 64;  // U(bj + r, bi + c) = L(bi + c, bj + r)
        const int i = bj + r, j = bi + c;
        if (i < n && j < n) U[(size_t)i + (size_t)j * n] = tile[c][r];
    }
}

static_assert(kDenseUpdPanels == 4, "launch_update instantiates one to four panels");
template <int TR>
static void launch_update(int np, unsigned blocks, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
                          double *A, const UpdArgs &u) {
    switch (np) {
    case 1:
        hipExtLaunchKernelGGL((ldl_update<1, TR>), dim3(blocks), dim3(256), 0, st, e0, e1, 0, A, u);
        break;
    case 2:
        hipExtLaunchKernelGGL((ldl_update<2, TR>), dim3(blocks), dim3(256), 0, st, e0, e1, 0, A, u);
        break;
    case 3:
        hipExtLaunchKernelGGL((ldl_update<3, TR>), dim3(blocks), dim3(256), 0, st, e0, e1, 0, A, u);
        break;
    default:
        hipExtLaunchKernelGGL((ldl_update<4, TR>), dim3(blocks), dim3(256), 0, st, e0, e1, 0, A, u);
        break;
    }
}

int DenseLDL::factor(hipStream_t st, const SchurCSR &S, double pivtol) {
    n = S.n;
    const size_t total = (size_t)n * n;
    const int nblk = (n + NB - 1) / NB;
    double *A = A_.need(total);
    d_.need(n);
    orig_.need(n);
    double *W = W_.need((size_t)kDenseUpdPanels * n * NB);
    double *linv = linv_.need((size_t)nblk * NB * NB);
    ninf_.need(1);
    hipLaunchKernelGGL(dense_zero, dim3(2048), dim3(256), 0, st, total, A);
    hipLaunchKernelGGL(dense_fill, dim3(n), dim3(64), 0, st, n, S.rowptr.get(), S.col.get(),
                       S.val.get(), A, orig_.get());
    OTIP_HIP(hipMemsetAsync(ninf_.get(), 0, sizeof(int), st));
    unsigned long long *nzL = cnt_.need(1);  // nonzeros of L, counted where they are written
    OTIP_HIP(hipMemsetAsync(nzL, 0, sizeof(unsigned long long), st));
    int *hrow = hrow_.need(nblk);  // last nonzero row of each block's panel
    OTIP_HIP(hipMemsetAsync(hrow, 0xff, sizeof(int) * nblk, st));
    const bool timed = factorisations_++ % std::max(1, timer_stride) == 0;
    LaunchTimer *tdiag = timed ? diag_timer : nullptr, *tupd = timed ? update_timer : nullptr;
    auto diag = [&](int kb, int nb) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (tdiag) tdiag->arm(2.0 * nb * nb * nb / 3.0, &e0, &e1);
        hipExtLaunchKernelGGL(ldl_diag, dim3(1), dim3(64 * kDiagWaves), 0, st, e0, e1, 0, n, kb, nb, A,
                              (const double *)orig_.get(), d_.get(), pivtol, ninf_.get(),
                              linv + (size_t)(kb / NB) * NB * NB);
    };
    auto panel = [&](int kb, int nb, double *W) {
        hipLaunchKernelGGL(ldl_panel<kPanelRows>, dim3(grid_for(n - kb - nb, kPanelRows)), dim3(256), 0, st, n, kb,
                           nb, A, d_.get(), W, (const double *)(linv + (size_t)(kb / NB) * NB * NB),
                           nzL, hrow);
    };
    // the timed update launches, whose algorithmic flops (over the rows the
    // panels reach) are known once the factorisation has run
    struct UpdRec {
        int first_col, r0, np, kcol[kDenseUpdPanels];
    };
    std::vector<UpdRec> recs;
    auto update = [&](int np, const UpdArgs &u, unsigned blocks, double flops) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (tupd) {
            tupd->arm(flops, &e0, &e1);
            UpdRec r{u.first_col, u.r0, np, {}};
            for (int p = 0; p < np; ++p) r.kcol[p] = u.p[p].kcol;
            recs.push_back(r);
        }
        if (u.first_col)
            launch_update<kFirstColRows>(np, blocks, st, e0, e1, A, u);
        else
            launch_update<kUpdRows>(np, blocks, st, e0, e1, A, u);
    };
    // Block steps in groups of up to kDenseUpdPanels: each block of a group
    // first takes the group's earlier panels on its own block column (a
    // first-column launch), is factorised and forms its panel; the rest of the
    // trailing matrix then takes all of the group's panels in one pass.  A
    // group closes early when the next block is the last one.  Every block
    // that forms a panel has 64 columns (only the last block can be narrower,
    // and it has no rows below it).
    for (int kb = 0; kb < n;) {
        UpdArgs u{n, 0, 0, hrow, {}};
        int g = 0, kq = kb;
        for (;;) {
            const int nbq = std::min(NB, n - kq);
            if (g > 0) {
                u.r0 = kq;
                u.first_col = 1;
                for (int p = 0; p < g; ++p) u.p[p].wrow0 = kq - u.p[p].kcol - NB;
                const double rq = n - kq;
                update(g, u, grid_for(n - kq, kFirstColRows),
                       2.0 * g * NB * (nbq * (rq - nbq) + nbq * (nbq + 1) / 2.0));
            }
            diag(kq, nbq);
            const int below = n - kq - nbq;
            if (below == 0) {  // the last block (g == 0 here: see the loop's exit test)
                kq = n;
                break;
            }
            double *Wq = W + (size_t)g * n * NB;
            panel(kq, nbq, Wq);
            u.p[g] = UpdPanel{Wq, kq, 0, below};
            ++g;
            kq += nbq;
            if (g == kDenseUpdPanels || n - kq <= NB) break;
        }
        if (kq >= n) break;
        u.r0 = kq;
        u.first_col = 0;
        for (int p = 0; p < g; ++p) u.p[p].wrow0 = kq - u.p[p].kcol - NB;
        const unsigned th = grid_for(n - kq, kUpdRows);
        constexpr unsigned H = kUpdRows / NB;
        update(g, u, H * th * (th + 1) / 2, (double)(n - kq) * (n - kq) * g * NB);
        kb = kq;
    }
    // X = L^-1 (unit lower; the strict lower part of A holds L)
    double *X = X_.need(total);
    hipLaunchKernelGGL(dense_zero, dim3(2048), dim3(256), 0, st, total, X);
    hipLaunchKernelGGL(inv_init, dim3(nblk), dim3(256), 0, st, n, linv, X);
    // From kDenseSplitMinN on, the top level (one pair, [0, h) and [h, n), three
    // quarters of the doubling's flops) is not formed: the solves apply
    // between the two diagonal inverses instead, a bandwidth-bound product
    // much cheaper than the two matrix products it replaces.
    int top = NB;
    while (2 * top < n) top *= 2;
    split_ = (n > NB && n >= kDenseSplitMinN) ? top : n;
    const int bend = split_ < n ? split_ : n;
    if (n > NB) {
        size_t tmax = 0;
        for (int b = NB; b < bend; b *= 2) {
            const int pairs = (n - b + 2 * b - 1) / (2 * b);
            tmax = std::max(tmax, (size_t)pairs * b * b);
        }
        double *T = tmax ? T_.need(tmax) : nullptr;
        for (int b = NB; b < bend; b *= 2) {
            const int pairs = (n - b + 2 * b - 1) / (2 * b);
            dim3 grid(b / NB, b / NB, pairs);
            hipLaunchKernelGGL(inv_mul<0>, grid, dim3(256), 0, st, n, b, A, X, T);
            hipLaunchKernelGGL(inv_mul<1>, grid, dim3(256), 0, st, n, b, A, X, T);
        }
    }
    OTIP_HIP(hipGetLastError());
    XT_.need(total);
    const unsigned tl = grid_for(n, 64);
    // an explicit inverse can overflow where the factor itself is finite
    // (products of large multipliers): then solve by substitution.  The
    // transpose reads all of X's strict lower part (its diagonal is 1, its
    // upper part 0) and flags a non-finite entry.
    hipLaunchKernelGGL(count_diag_blocks, dim3(nblk), dim3(256), 0, st, n, (const double *)A, nzL);
    OTIP_HIP(hipMemsetAsync(bad_.need(1), 0, sizeof(int), st));
    hipLaunchKernelGGL(transpose_lower, dim3(tl, tl), dim3(256), 0, st, n, X, XT_.get(),
                       bad_.get(), split_ < n ? (const double *)A : nullptr, split_);
    int hn = 0, hbad = 0;
    unsigned long long hc = 0;
    OTIP_HIP(hipMemcpyAsync(&hn, ninf_.get(), sizeof(int), hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipMemcpyAsync(&hc, nzL, sizeof(hc), hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipMemcpyAsync(&hbad, bad_.get(), sizeof(int), hipMemcpyDeviceToHost, st));
    std::vector<int> hh(tupd ? nblk : 0);
    if (tupd)
        OTIP_HIP(hipMemcpyAsync(hh.data(), hrow, sizeof(int) * nblk, hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipStreamSynchronize(st));
    if (tdiag) tdiag->collect();
    if (tupd) {
        // algorithmic flops of each timed update: over the rows its panels reach
        for (size_t k = 0; k < recs.size(); ++k) {
            const UpdRec &r = recs[k];
            int reach = -1;
            for (int p = 0; p < r.np; ++p) reach = std::max(reach, hh[r.kcol[p] / NB]);
            const double live = std::max(0, std::min(n - r.r0, reach - r.r0 + 1));
            double entries;  // lower-triangle entries of the launch's region
            if (r.first_col) {
                const double w = std::min(NB, n - r.r0);
                entries = live >= w ? w * (w + 1) / 2.0 + (live - w) * w : live * (live + 1) / 2.0;
            } else {
                entries = live * live / 2.0;
            }
            tupd->set_pending(k, 2.0 * NB * r.np * entries);
        }
        tupd->collect();
    }
    nnzL_ = (int64_t)hc + n;
    inverse_ok_ = hbad == 0 && !force_substitution;
    if (!inverse_ok_)  // U = L^T for the backward substitution
        hipLaunchKernelGGL(transpose_lower, dim3(tl, tl), dim3(256), 0, st, n, A, XT_.get(),
                           (int *)nullptr, (const double *)nullptr, n);
    return hn;
}

void DenseLDL::solve(hipStream_t st, const double *b, double *x) {
    double *y = v_.need(n);
    if (inverse_ok_) {
        const double *X = X_.get(), *XT = XT_.get(), *d = d_.get();
        const int h = split_;
        if (h >= n) {
            const unsigned g = grid_for(n, 4);
            hipLaunchKernelGGL(x_rows, dim3(g), dim3(256), 0, st, n, 0, n, 0, n, XT, b, b, 1.0, d,
                               (double *)nullptr, y);
            hipLaunchKernelGGL(x_cols, dim3(g), dim3(256), 0, st, n, 0, n, 0, n, X, y, y, 1.0, x);
        } else {
            // z (rows < h) and w = b2 - L21 z1 (rows >= h) in separate halves of t
            double *t = t_.need(2 * (size_t)n), *z = t, *w = t + n;
            const unsigned g1 = grid_for(h, 4), g2 = grid_for(n - h, 4);
            hipLaunchKernelGGL(x_rows, dim3(g1), dim3(256), 0, st, n, 0, h, 0, h, XT, b, b, 1.0, d,
                               z, y);
            hipLaunchKernelGGL(x_rows, dim3(g2), dim3(256), 0, st, n, h, n, 0, h, XT,
                               (const double *)z, b, -1.0, d, w, (double *)nullptr);
            hipLaunchKernelGGL(x_rows, dim3(g2), dim3(256), 0, st, n, h, n, h, n, XT,
                               (const double *)w, (const double *)w, 1.0, d, (double *)nullptr, y);
            // x2 = X22^T y2; z1 = y1 - L21^T x2 (L21 from the factor); x1 = X11^T z1
            hipLaunchKernelGGL(x_cols, dim3(g2), dim3(256), 0, st, n, h, n, 0, n, X, y, y, 1.0, x);
            hipLaunchKernelGGL(x_cols, dim3(g1), dim3(256), 0, st, n, 0, h, h, n,
                               (const double *)A_.get(), (const double *)x, (const double *)y,
                               -1.0, z);
            hipLaunchKernelGGL(x_cols, dim3(g1), dim3(256), 0, st, n, 0, h, 0, h, X,
                               (const double *)z, (const double *)z, 1.0, x);
        }
        OTIP_HIP(hipGetLastError());
        return;
    }
    // substitution on L (in A_) and U = L^T (in XT_)
    double *w = X_.get();  // n doubles of scratch: X is not used on this path
    double *yv = y;
    OTIP_HIP(hipMemcpyAsync(w, b, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    for (int kb = 0; kb < n; kb += NB) {
        const int nb = std::min(NB, n - kb);
        const int rows = n - kb - nb;
        hipLaunchKernelGGL(trsv_step, dim3(std::max(1u, grid_for(rows, 256))), dim3(256), 0, st,
                           n, kb, nb, A_.get(), d_.get(), w, yv, 1);
    }
    hipLaunchKernelGGL(scale_by_pivots, dim3(grid_for(n, 256)), dim3(256), 0, st, n, d_.get(), yv);
    for (int kb = ((n - 1) / NB) * NB; kb >= 0; kb -= NB) {
        const int nb = std::min(NB, n - kb);
        hipLaunchKernelGGL(trsv_step, dim3(std::max(1u, grid_for(kb, 256))), dim3(256), 0, st, n,
                           kb, nb, XT_.get(), d_.get(), yv, x, 0);
    }
    OTIP_HIP(hipGetLastError());
}

}  // namespace otip
