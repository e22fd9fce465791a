// Index bookkeeping primitives: stable LSD radix sort, exclusive prefix sums
// and deduplication of sorted keys.  They serve the integer side of the
// method: ordering selected columns, rebuilding the support's row/column views
// and deduplicating index sets.
//
// Radix sort: 8-bit digits from the lowest requested bit up, one pass per
// digit.  A pass is three launches over tiles of kTile keys: (1) per-tile
// digit counts, stored digit-major (counts[d][tile]); (2) an exclusive scan of
// those counts, which gives every (digit, tile) its first output position;
// (3) the scatter, in which each tile ranks its keys among equal digits in
// input order -- lanes of a wavefront by ballots on the digit's bits, then
// wavefronts of a round in order, then rounds in order -- so the pass, and the
// sort, are stable and deterministic.
#include "internal.h"

namespace otip {

namespace {

constexpr int kThreads = 256;
constexpr int kRounds = 8;
constexpr int kTile = kThreads * kRounds;  // keys per tile
constexpr int kBins = 256;

__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename K>
__device__ __forceinline__ int digit_of(K k, int shift, int bits) {
    return (int)((k >> shift) & (K)((1u << bits) - 1u));
}

template <typename K>
__global__ __launch_bounds__(kThreads) void rs_count(const K *__restrict__ keys, int64_t n,
                                                     int shift, int bits, int tiles,
                                                     uint32_t *__restrict__ counts) {
    __shared__ uint32_t h[kBins];
    h[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kTile;
    for (int r = 0; r < kRounds; ++r) {
        const int64_t i = t0 + (int64_t)r * kThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[digit_of(keys[i], shift, bits)], 1u);
    }
    __syncthreads();
    counts[(size_t)threadIdx.x * tiles + blockIdx.x] = h[threadIdx.x];
}

// V = void-like marker when there is no payload
struct NoVal {};

template <typename K, typename V>
__global__ __launch_bounds__(kThreads) void rs_scatter(const K *__restrict__ kin,
                                                       const V *__restrict__ vin, int64_t n,
                                                       int shift, int bits, int tiles,
                                                       const uint32_t *__restrict__ offsets,
                                                       K *__restrict__ kout, V *__restrict__ vout) {
    __shared__ uint32_t base[kBins];
    __shared__ uint32_t wcnt[kThreads / 64][kBins];
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    base[t] = offsets[(size_t)t * tiles + blockIdx.x];
    const uint64_t lt = (1ull << lane) - 1ull;
    const int64_t t0 = (int64_t)blockIdx.x * kTile;
    for (int r = 0; r < kRounds; ++r) {
        const int64_t i = t0 + (int64_t)r * kThreads + t;
        const bool valid = i < n;
        const K k = valid ? kin[i] : (K)0;
        const int d = valid ? digit_of(k, shift, bits) : 0;
        // lanes of this wavefront with the same digit (and validity)
        uint64_t peers = __ballot(valid);
        if (!valid) peers = ~peers;
        for (int b = 0; b < bits; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
#pragma unroll
        for (int q = 0; q < kBins / 64; ++q) wcnt[w][lane * (kBins / 64) + q] = 0u;
        wave_fence();
        const bool leader = (peers & lt) == 0ull;
        if (valid && leader) wcnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = base[d] + (uint32_t)__popcll(peers & lt);
            for (int u = 0; u < w; ++u) pos += wcnt[u][d];
            kout[pos] = k;
            if (vout) vout[pos] = vin[i];
        }
        __syncthreads();
        uint32_t add = 0u;
#pragma unroll
        for (int u = 0; u < kThreads / 64; ++u) add += wcnt[u][t];
        base[t] += add;
        __syncthreads();
    }
}

// ---------------------------------------------------------- exclusive scan
// out[i] = sum of in[j] for j < i.  Three launches: each block scans kTile
// consecutive entries (kRounds contiguous per thread) and leaves its total;
// one block scans the totals; each block adds its offset.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int lane = threadIdx.x & 63;
    for (int o = 1; o < 64; o <<= 1) {
        const T u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

// exclusive scan of one value per thread over the block; the block total in
// *total
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T *lds /* kThreads / 64 */, T *total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const T incl = wave_incl_scan(v);
    if (lane == 63) lds[w] = incl;
    __syncthreads();
    T before = (T)0, all = (T)0;
    for (int u = 0; u < kThreads / 64; ++u) {
        if (u < w) before += lds[u];
        all += lds[u];
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

template <typename T, typename S>
__global__ __launch_bounds__(kThreads) void scan_tiles(const T *__restrict__ in, S *__restrict__ out,
                                                       int64_t n, S *__restrict__ sums) {
    __shared__ S lds[kThreads / 64];
    const int64_t t0 = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kRounds;
    S v[kRounds];
    S s = (S)0;
#pragma unroll
    for (int q = 0; q < kRounds; ++q) {
        v[q] = (t0 + q < n) ? (S)in[t0 + q] : (S)0;
        s += v[q];
    }
    S total;
    S run = block_excl_scan(s, lds, &total);
#pragma unroll
    for (int q = 0; q < kRounds; ++q) {
        if (t0 + q < n) out[t0 + q] = run;
        run += v[q];
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// exclusive scan of the tile totals in place, by one block
template <typename S>
__global__ __launch_bounds__(kThreads) void scan_sums(S *sums, int nb) {
    __shared__ S lds[kThreads / 64];
    S carry = (S)0;
    for (int b0 = 0; b0 < nb; b0 += kThreads) {
        const int b = b0 + threadIdx.x;
        const S v = b < nb ? sums[b] : (S)0;
        S total;
        const S ex = block_excl_scan(v, lds, &total);
        if (b < nb) sums[b] = carry + ex;
        carry += total;
    }
}

template <typename S>
__global__ __launch_bounds__(kThreads) void scan_add(S *__restrict__ out, int64_t n,
                                                     const S *__restrict__ sums) {
    const int64_t t0 = (int64_t)blockIdx.x * kTile;
    const S add = sums[blockIdx.x];
    for (int r = 0; r < kRounds; ++r) {
        const int64_t i = t0 + (int64_t)r * kThreads + threadIdx.x;
        if (i < n) out[i] += add;
    }
}

int tiles_of(int64_t n) { return (int)std::max<int64_t>(1, (n + kTile - 1) / kTile); }

// bytes of scratch used by a scan of n entries of type S
template <typename S>
size_t scan_scratch(int64_t n) {
    return sizeof(S) * ((size_t)tiles_of(n) + 64);
}

template <typename T, typename S>
void scan_excl(hipStream_t st, const T *in, S *out, int64_t n, S *sums) {
    const int nb = tiles_of(n);
    hipLaunchKernelGGL((scan_tiles<T, S>), dim3(nb), dim3(kThreads), 0, st, in, out, n, sums);
    hipLaunchKernelGGL((scan_sums<S>), dim3(1), dim3(kThreads), 0, st, sums, nb);
    hipLaunchKernelGGL((scan_add<S>), dim3(nb), dim3(kThreads), 0, st, out, n,
                       (const S *)sums);
    OTIP_HIP(hipGetLastError());
}

// Stable sort of n keys (bits [begin_bit, end_bit)) with an optional payload.
// Scratch from tmp: two key/value ping-pong arrays, the digit counts and the
// scan's tile sums.
template <typename K, typename V>
void radix_sort(hipStream_t st, const K *kin, const V *vin, K *kout, V *vout, int64_t n,
                int begin_bit, int end_bit, DBuf<char> &tmp) {
    if (n <= 0) return;
    OTIP_CHECK(n < ((int64_t)1 << 32), OTIP_EINVAL, "radix sort: more than 2^32 keys");
    const int tiles = tiles_of(n);
    const int passes = std::max(0, (end_bit - begin_bit + 7) / 8);
    const size_t cnt_n = (size_t)kBins * tiles;
    auto align = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t kb = align(sizeof(K) * (size_t)n), vb = vout ? align(sizeof(V) * (size_t)n) : 0;
    const size_t cb = align(sizeof(uint32_t) * cnt_n), sb = align(scan_scratch<uint32_t>(cnt_n));
    char *base = tmp.need(kb + vb + cb + sb);
    K *kt = (K *)base;
    V *vt = vout ? (V *)(base + kb) : nullptr;
    uint32_t *counts = (uint32_t *)(base + kb + vb);
    uint32_t *sums = (uint32_t *)(base + kb + vb + cb);
    if (passes == 0) {
        OTIP_HIP(hipMemcpyAsync(kout, kin, sizeof(K) * n, hipMemcpyDeviceToDevice, st));
        if (vout) OTIP_HIP(hipMemcpyAsync(vout, vin, sizeof(V) * n, hipMemcpyDeviceToDevice, st));
        return;
    }
    const K *ks = kin;
    const V *vs = vin;
    for (int p = 0; p < passes; ++p) {
        const int shift = begin_bit + 8 * p;
        const int bits = std::min(8, end_bit - shift);
        // the last pass lands in the output arrays
        const bool to_out = ((passes - 1 - p) % 2) == 0;
        K *kd = to_out ? kout : kt;
        V *vd = vout ? (to_out ? vout : vt) : nullptr;
        hipLaunchKernelGGL((rs_count<K>), dim3(tiles), dim3(kThreads), 0, st, ks, n, shift, bits,
                           tiles, counts);
        scan_excl<uint32_t, uint32_t>(st, counts, counts, (int64_t)cnt_n, sums);
        hipLaunchKernelGGL((rs_scatter<K, V>), dim3(tiles), dim3(kThreads), 0, st, ks, vs, n,
                           shift, bits, tiles, (const uint32_t *)counts, kd, vd);
        OTIP_HIP(hipGetLastError());
        ks = kd;
        vs = vd;
    }
}

__global__ void iota_i32(int64_t n, int32_t *v) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) v[t] = (int32_t)t;
}

__global__ void gather2(int64_t n, const int32_t *perm, const double *a, const double *b,
                        double *oa, double *ob) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) {
        oa[t] = a[perm[t]];
        ob[t] = b[perm[t]];
    }
}

// 1 where a sorted key differs from its predecessor
__global__ void first_flags(int64_t n, const uint64_t *__restrict__ in, uint32_t *__restrict__ f) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) f[t] = (t == 0 || in[t] != in[t - 1]) ? 1u : 0u;
}

__global__ void scatter_firsts(int64_t n, const uint64_t *__restrict__ in,
                               const uint32_t *__restrict__ f, const uint32_t *__restrict__ pos,
                               uint64_t *__restrict__ out, unsigned long long *count) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    if (f[t]) out[pos[t]] = in[t];
    if (t == n - 1) *count = (unsigned long long)pos[t] + f[t];
}

}  // namespace

void sort_pairs_u64(hipStream_t st, const uint64_t *kin, const uint64_t *vin, uint64_t *kout,
                    uint64_t *vout, int64_t n, int begin_bit, int end_bit, DBuf<char> &tmp) {
    radix_sort<uint64_t, uint64_t>(st, kin, vin, kout, vout, n, begin_bit, end_bit, tmp);
}

void sort_pairs_u32_i32(hipStream_t st, const uint32_t *kin, const int32_t *vin, uint32_t *kout,
                        int32_t *vout, int64_t n, int end_bit, DBuf<char> &tmp) {
    radix_sort<uint32_t, int32_t>(st, kin, vin, kout, vout, n, 0, end_bit, tmp);
}

void sort_keys_u64(hipStream_t st, const uint64_t *kin, uint64_t *kout, int64_t n,
                   DBuf<char> &tmp) {
    radix_sort<uint64_t, uint64_t>(st, kin, (const uint64_t *)nullptr, kout, (uint64_t *)nullptr,
                                   n, 0, 64, tmp);
}

void sort_pairs_u64_f64x2(hipStream_t st, const uint64_t *kin, const double *v1in,
                          const double *v2in, uint64_t *kout, double *v1out, double *v2out,
                          int64_t n, int end_bit, DBuf<char> &tmp, DBuf<int32_t> &perm_a,
                          DBuf<int32_t> &perm_b) {
    if (n <= 0) return;
    int32_t *pa = perm_a.need((size_t)n);
    int32_t *pb = perm_b.need((size_t)n);
    hipLaunchKernelGGL(iota_i32, dim3(grid_for(n, 256)), dim3(256), 0, st, n, pa);
    radix_sort<uint64_t, int32_t>(st, kin, (const int32_t *)pa, kout, pb, n, 0, end_bit, tmp);
    hipLaunchKernelGGL(gather2, dim3(grid_for(n, 256)), dim3(256), 0, st, n, (const int32_t *)pb,
                       v1in, v2in, v1out, v2out);
    OTIP_HIP(hipGetLastError());
}

int64_t unique_u64(hipStream_t st, const uint64_t *in, uint64_t *out, int64_t n, DBuf<char> &tmp,
                   DBuf<unsigned long long> &cnt) {
    if (n <= 0) return 0;
    OTIP_CHECK(n < ((int64_t)1 << 32), OTIP_EINVAL, "unique: more than 2^32 keys");
    unsigned long long *c = cnt.need(1);
    auto align = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t fb = align(sizeof(uint32_t) * (size_t)n);
    char *base = tmp.need(2 * fb + align(scan_scratch<uint32_t>(n)));
    uint32_t *f = (uint32_t *)base, *pos = (uint32_t *)(base + fb);
    uint32_t *sums = (uint32_t *)(base + 2 * fb);
    hipLaunchKernelGGL(first_flags, dim3(grid_for(n, 256)), dim3(256), 0, st, n, in, f);
    scan_excl<uint32_t, uint32_t>(st, f, pos, n, sums);
    hipLaunchKernelGGL(scatter_firsts, dim3(grid_for(n, 256)), dim3(256), 0, st, n, in,
                       (const uint32_t *)f, (const uint32_t *)pos, out, c);
    OTIP_HIP(hipGetLastError());
    unsigned long long h = 0;
    OTIP_HIP(hipMemcpyAsync(&h, c, sizeof(h), hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipStreamSynchronize(st));
    return (int64_t)h;
}

void exclusive_scan_i64(hipStream_t st, const int64_t *in, int64_t *out, int64_t n,
                        DBuf<char> &tmp) {
    if (n <= 0) return;
    int64_t *sums = (int64_t *)tmp.need(scan_scratch<int64_t>(n));
    scan_excl<int64_t, int64_t>(st, in, out, n, sums);
}

}  // namespace otip
