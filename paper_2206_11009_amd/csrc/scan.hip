// Full m x n scans: pricing (Sections 3.2 and 3.4), the reduced-cost minimum
// of the dual certificate (Section 3.3), and the cheap-variable scans of the
// initial support (Section 3.2, end).  Costs are generated on the fly from
// integer coordinates and never stored.
//
// Thread mapping of every scan: a 256-thread block covers 256 consecutive
// sources i (lanes along i, so the variable index i + j*m is contiguous across
// a wave) and a run of TJ consecutive targets j.  Per-target data is
// wave-uniform and is read through the scalar cache from a small table built
// per call.
#include "common.h"
#include <cstring>

#include "internal.h"

namespace otip {

// Per-target table, all exact doubles.  Squared cost: B_j = |x_j|^2, a2 =
// -2 x_j0, b2 = -2 x_j1; the norm costs: B_j = x_j0, a2 = x_j1 (b2 unused).
// Then z_j.
struct __align__(32) JEntry {
    double B, a2, b2, z;
};

// The per-target tables are read-only during a scan and every lane of a wave
// reads the same entry: reading them through the constant address space lets
// the compiler use scalar loads even in kernels that also store to memory.
typedef const __attribute__((address_space(4))) double *cdptr;
typedef const __attribute__((address_space(4))) float *cfptr;
__device__ __forceinline__ JEntry ldj(const JEntry *p, int j) {
    const cdptr q = (cdptr)(p + j);
    JEntry e;
    e.B = q[0];
    e.a2 = q[1];
    e.b2 = q[2];
    e.z = q[3];
    return e;
}

__global__ void build_jtab(int n, int kind, const int32_t *__restrict__ xt,
                           const double *__restrict__ z, JEntry *__restrict__ jt) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double a = (double)xt[2 * j], b = (double)xt[2 * j + 1];
    JEntry e;
    if (kind == OTIP_COST_SQEUCLID) {
        e.B = a * a + b * b;
        e.a2 = -2.0 * a;
        e.b2 = -2.0 * b;
    } else {
        e.B = a;
        e.a2 = b;
        e.b2 = 0.0;
    }
    e.z = z ? z[j] : 0.0;
    jt[j] = e;
}

// Per-source data: A_i = |x_i|^2, x_i0, x_i1, y_i.  Rows past m get y = -inf so
// that every reduced cost they produce is +inf (never selected).
struct RowData {
    double A, al, be, y;
};

__device__ __forceinline__ RowData load_row(int i, int m, const int32_t *__restrict__ xs,
                                            const double *__restrict__ y) {
    RowData d;
    if (i < m) {
        d.al = (double)xs[2 * i];
        d.be = (double)xs[2 * i + 1];
        d.A = d.al * d.al + d.be * d.be;
        d.y = y ? y[i] : 0.0;
    } else {
        d.al = d.be = d.A = 0.0;
        d.y = -INFINITY;
    }
    return d;
}

// C_ij of a cost kind (Section 5.1).  Squared: |x_i|^2 + |x_j|^2 - 2 x_i.x_j;
// every intermediate is an integer below 2^53, so the two fused multiply-adds
// are exact.  Norms of the offset d = x_i - x_j (|d| <= 2^15): the 1- and
// inf-norms are exact; for the 2-norm d0^2 + d1^2 <= 2^31 is formed exactly
// by the fused multiply-add and its IEEE square root is correctly rounded.
template <int K>
__device__ __forceinline__ double cost_of(const RowData &r, const JEntry &t) {
    if (K == OTIP_COST_SQEUCLID) return fma(r.be, t.b2, fma(r.al, t.a2, r.A + t.B));
    const double d0 = r.al - t.B, d1 = r.be - t.a2;
    if (K == OTIP_COST_L1) return fabs(d0) + fabs(d1);
    if (K == OTIP_COST_L2) return __builtin_sqrt(fma(d0, d0, d1 * d1));
    return fmax(fabs(d0), fabs(d1));
}

__device__ __forceinline__ bool in_support(const uint32_t *__restrict__ bm, uint64_t idx) {
    return bm && ((bm[idx >> 5] >> (idx & 31u)) & 1u);
}

constexpr int kScanBlock = 256;
constexpr int kHistBins = 4096;

// Compaction output of one wave, staged in LDS: the output space is reserved
// with one global atomic per kStage candidates instead of one per ballot.  The
// most negative reduced costs cluster in few waves, whose many atomics on the
// one counter would otherwise serialise.  W words per candidate: (key, idx) or
// idx alone.  Every lane of the wave calls push and flush.
constexpr int kStage = 256;
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
template <int W>
struct WaveStage {
    uint64_t *buf;  // this wave's kStage * W words of LDS
    int cnt;        // staged candidates (the same in every lane)
    unsigned long long *count;
    uint64_t *out_key, *out_idx;
    uint64_t cap;

    __device__ void flush() {
        if (cnt == 0) return;
        const int lane = threadIdx.x & 63;
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(count, (unsigned long long)cnt);
        base = __shfl(base, 0, 64);
        wave_sync();
        for (int k = lane; k < cnt; k += 64) {
            const uint64_t pos = base + (uint64_t)k;
            if (pos < cap) {
                if (W == 2) {
                    out_key[pos] = buf[2 * k];
                    out_idx[pos] = buf[2 * k + 1];
                } else {
                    out_idx[pos] = buf[k];
                }
            }
        }
        wave_sync();
        cnt = 0;
    }
    __device__ void push(bool take, uint64_t key, uint64_t idx) {
        const uint64_t mask = __ballot(take);
        if (mask == 0ull) return;
        const int nw = __popcll(mask);
        if (cnt + nw > kStage) flush();
        if (take) {
            const int lane = threadIdx.x & 63;
            const int pos = cnt + __popcll(mask & ((1ull << lane) - 1ull));
            if (W == 2) {
                buf[2 * pos] = key;
                buf[2 * pos + 1] = idx;
            } else {
                buf[pos] = idx;
            }
        }
        cnt += nw;
    }
};

struct PriceArgs {
    int m, n, tj;
    const int32_t *xs;
    const double *y;
    const JEntry *jt;
    const uint32_t *bitmap;
    // histogram mode: digit = (key >> shift) & 4095 over keys whose bits above
    // shift+12 equal `prefix` (no filter when shift + 12 >= 64)
    int shift;
    uint64_t prefix;
    unsigned long long *hist;
    // compaction mode: every key <= key_max; rkey is the double whose key is
    // key_max (a group whose smallest r is above it has no candidate)
    uint64_t key_max;
    double rkey;
    // no key of interest belongs to an r above rcut (the double whose key is
    // the largest one of interest, or +inf): groups with no r <= rcut skip
    double rcut;
    unsigned long long *count;
    uint64_t *out_key, *out_idx;
    uint64_t cap;
};

// the per-variable part of a pricing pass (all lanes of the wave call it)
template <int MODE>
__device__ __forceinline__ void price_one(const PriceArgs &a, int i, int j, double r,
                                          unsigned int *lh, WaveStage<2> &stg,
                                          bool group_cand = true) {
    {
        const int pshift = a.shift + 12;
        const bool neg = r < 0.0 && r <= a.rcut;
        if (__ballot(neg) == 0ull) return;
        const uint64_t idx = (uint64_t)i + (uint64_t)j * (uint64_t)a.m;
        bool take = neg && !in_support(a.bitmap, idx);
        const uint64_t key = dkey(r);
        if (MODE != 1) {
            if (take && (pshift >= 64 || (key >> pshift) == a.prefix))
                atomicAdd(&lh[(key >> a.shift) & 4095u], 1u);
        }
        // group_cand is wave-uniform: no lane's group of four has an r <= rkey
        if (MODE != 0 && group_cand) stg.push(take && key <= a.key_max, key, idx);
    }
}

// Pricing pass.  MODE 0: histogram of one 12-bit digit of the ordered key of
// every strictly negative reduced cost outside the support.  MODE 1: append
// (key, idx) of those with key <= key_max.  MODE 2: both in one pass (the
// first pass of a call: the top digit's histogram, and the candidates below
// a cutoff guessed from the previous call).
template <int MODE, int K>
__global__ __launch_bounds__(kScanBlock) void price_pass(PriceArgs a) {
    __shared__ unsigned int lh[MODE != 1 ? kHistBins : 1];
    __shared__ uint64_t sbuf[MODE != 0 ? (kScanBlock / 64) * kStage * 2 : 1];
    WaveStage<2> stg{sbuf + (MODE != 0 ? (threadIdx.x >> 6) * kStage * 2 : 0), 0, a.count,
                     a.out_key, a.out_idx, a.cap};
    const int i = blockIdx.x * kScanBlock + threadIdx.x;
    const int j0 = blockIdx.y * a.tj;
    const int j1 = min(a.n, j0 + a.tj);
    if (MODE != 1) {
        for (int t = threadIdx.x; t < kHistBins; t += kScanBlock) lh[t] = 0u;
        __syncthreads();
    }
    const RowData rd = load_row(i, a.m, a.xs, a.y);
    const JEntry *jt = a.jt;
    int j = j0;
    // four targets at a time: table loads issued together, and a whole group
    // without a negative reduced cost costs one ballot
    for (; j + 4 <= j1; j += 4) {
        const JEntry t0 = ldj(jt, j), t1 = ldj(jt, j + 1), t2 = ldj(jt, j + 2),
                     t3 = ldj(jt, j + 3);
        const double r0 = (cost_of<K>(rd, t0) - rd.y) - t0.z;
        const double r1 = (cost_of<K>(rd, t1) - rd.y) - t1.z;
        const double r2 = (cost_of<K>(rd, t2) - rd.y) - t2.z;
        const double r3 = (cost_of<K>(rd, t3) - rd.y) - t3.z;
        const double lo = fmin(fmin(r0, r1), fmin(r2, r3));
        if (__ballot(lo < 0.0 && lo <= a.rcut) == 0ull) continue;
        // the first pass histograms every negative; its candidate compaction
        // only matters where some r is at most the guessed cutoff
        const bool cand = MODE != 2 || __ballot(lo <= a.rkey) != 0ull;
        price_one<MODE>(a, i, j, r0, lh, stg, cand);
        price_one<MODE>(a, i, j + 1, r1, lh, stg, cand);
        price_one<MODE>(a, i, j + 2, r2, lh, stg, cand);
        price_one<MODE>(a, i, j + 3, r3, lh, stg, cand);
    }
    for (; j < j1; ++j) {
        const JEntry t = ldj(jt, j);
        const double r = (cost_of<K>(rd, t) - rd.y) - t.z;
        price_one<MODE>(a, i, j, r, lh, stg);
    }
    if (MODE != 0) stg.flush();
    if (MODE != 1) {
        __syncthreads();
        for (int t = threadIdx.x; t < kHistBins; t += kScanBlock)
            if (lh[t]) atomicAdd(&a.hist[t], (unsigned long long)lh[t]);
    }
}

// Pricing pass over the heuristic subset J of Section 3.4, stored as
// per-source target lists (jptr: m + 1 offsets, jcol: targets in increasing
// j).  One wavefront per source at a time: the source's data is uniform
// across the wave, each lane takes one target of the list and gathers its
// table entry; the reduced cost is formed exactly as by price_pass, so the
// values (and the selection) are those of the full scan restricted to J.
// Lanes past the end of a list carry r = +inf so that every lane of the wave
// takes part in the ballots.
template <int MODE, int K>
__global__ __launch_bounds__(kScanBlock) void price_list_pass(PriceArgs a,
                                                              const int64_t *__restrict__ jptr,
                                                              const int32_t *__restrict__ jcol) {
    __shared__ unsigned int lh[MODE != 1 ? kHistBins : 1];
    __shared__ uint64_t sbuf[MODE != 0 ? (kScanBlock / 64) * kStage * 2 : 1];
    WaveStage<2> stg{sbuf + (MODE != 0 ? (threadIdx.x >> 6) * kStage * 2 : 0), 0, a.count,
                     a.out_key, a.out_idx, a.cap};
    if (MODE != 1) {
        for (int t = threadIdx.x; t < kHistBins; t += kScanBlock) lh[t] = 0u;
        __syncthreads();
    }
    const int lane = threadIdx.x & 63;
    const int waves = gridDim.x * (kScanBlock / 64);
    for (int i = blockIdx.x * (kScanBlock / 64) + (threadIdx.x >> 6); i < a.m; i += waves) {
        const RowData rd = load_row(i, a.m, a.xs, a.y);
        const int64_t e0 = jptr[i], e1 = jptr[i + 1];
        for (int64_t base = e0; base < e1; base += 64) {
            const int64_t e = base + lane;
            int j = 0;
            double r = INFINITY;
            if (e < e1) {
                j = jcol[e];
                const JEntry t = a.jt[j];
                r = (cost_of<K>(rd, t) - rd.y) - t.z;
            }
            price_one<MODE>(a, i, j, r, lh, stg);
        }
    }
    if (MODE != 0) stg.flush();
    if (MODE != 1) {
        __syncthreads();
        for (int t = threadIdx.x; t < kHistBins; t += kScanBlock)
            if (lh[t]) atomicAdd(&a.hist[t], (unsigned long long)lh[t]);
    }
}

// Heuristic subset J = {(i, j) : cost key < L} (Section 3.4) as per-source
// target lists: one wavefront per source counts (pass 0) or writes, in
// increasing j (pass 1), the targets whose integer cost key is below L.
template <int PASS>
__global__ __launch_bounds__(kScanBlock) void subset_lists(int m, int n, int kind,
                                                           const int32_t *__restrict__ xs,
                                                           const int32_t *__restrict__ xt,
                                                           int64_t L, int64_t *cnt,
                                                           const int64_t *__restrict__ off,
                                                           int32_t *__restrict__ col);

// Decode the selected (key, idx) into (i, j, r).
__global__ void decode_selection(int64_t k, int m, const uint64_t *__restrict__ key,
                                 const uint64_t *__restrict__ idx, int32_t *oi, int32_t *oj,
                                 double *orr, uint64_t *oidx) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= k) return;
    uint64_t v = idx[t];
    if (oi) oi[t] = (int32_t)(v % (uint64_t)m);
    if (oj) oj[t] = (int32_t)(v / (uint64_t)m);
    if (orr) orr[t] = dkey_inv(key[t]);
    if (oidx) oidx[t] = v;
}

// targets per block: enough blocks to fill 256 CUs several times over, but
// enough work per block to amortise the histogram's LDS setup
// the double with ordered key k (host side), or +inf where k is not a number's key
static double rcut_of_key(uint64_t k) {
    const uint64_t u = (k & 0x8000000000000000ull) ? (k & 0x7fffffffffffffffull) : ~k;
    double d;
    std::memcpy(&d, &u, sizeof d);
    return std::isnan(d) ? INFINITY : d;
}

// the ordered key of a double (host side; no NaNs)
static uint64_t host_dkey(double r) {
    uint64_t u;
    std::memcpy(&u, &r, sizeof u);
    return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}

// the instance of a kernel templated on the cost kind
template <typename Fn>
static Fn by_kind(int kind, Fn k0, Fn k1, Fn k2, Fn k3) {
    return kind == OTIP_COST_L1 ? k1 : kind == OTIP_COST_L2 ? k2 : kind == OTIP_COST_LINF ? k3 : k0;
}

int pick_tj(int m, int n, int tile) {
    if (tile >= 16 && tile <= 256 && (tile & (tile - 1)) == 0) return tile;
    const int64_t rb = (m + 255) / 256;
    int tj = 256;
    while (tj > 16 && rb * ((n + tj - 1) / tj) < 2048) tj >>= 1;
    return tj;
}

void Scanner::prepare(hipStream_t st, int m, int n, const int32_t *xt, const double *z) {
    jt_.need((size_t)n * sizeof(JEntry));
    hipLaunchKernelGGL(build_jtab, dim3(grid_for(n, 256)), dim3(256), 0, st, n, kind, xt, z,
                       (JEntry *)jt_.get());
    OTIP_HIP(hipGetLastError());
}

int64_t Scanner::set_subset(hipStream_t st, int m, int n, const int32_t *xs, const int32_t *xt,
                            int64_t key_limit) {
    OTIP_CHECK(m >= 1 && n >= 1 && key_limit >= 1, OTIP_EINVAL, "subset: bad arguments");
    scnt_.need((size_t)m);
    sptr_.need((size_t)m + 1);
    const unsigned blocks = grid_for(m, kScanBlock / 64);
    hipLaunchKernelGGL(subset_lists<0>, dim3(blocks), dim3(kScanBlock), 0, st, m, n, kind, xs, xt,
                       key_limit, scnt_.get(), (const int64_t *)nullptr, (int32_t *)nullptr);
    OTIP_HIP(hipGetLastError());
    exclusive_scan_i64(st, scnt_.get(), sptr_.get(), m, tmp_);
    int64_t last_off = 0, last_cnt = 0;
    OTIP_HIP(hipMemcpyAsync(&last_off, sptr_.get() + (m - 1), sizeof(int64_t),
                            hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipMemcpyAsync(&last_cnt, scnt_.get() + (m - 1), sizeof(int64_t),
                            hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipStreamSynchronize(st));
    const int64_t total = last_off + last_cnt;
    OTIP_HIP(hipMemcpyAsync(sptr_.get() + m, &total, sizeof(int64_t), hipMemcpyHostToDevice, st));
    scol_.need((size_t)std::max<int64_t>(total, 1));
    hipLaunchKernelGGL(subset_lists<1>, dim3(blocks), dim3(kScanBlock), 0, st, m, n, kind, xs, xt,
                       key_limit, (int64_t *)nullptr, (const int64_t *)sptr_.get(), scol_.get());
    OTIP_HIP(hipGetLastError());
    OTIP_HIP(hipStreamSynchronize(st));  // the host value `total` above is on the stack
    subset_m_ = m;
    subset_nnz_ = total;
    return total;
}

PriceResult Scanner::price(hipStream_t st, int m, int n, const int32_t *xs, const int32_t *xt,
                           const double *y, const double *z, const uint32_t *bitmap,
                           int64_t kmax, int32_t *oi, int32_t *oj, double *orr,
                           uint64_t *oidx) {
    PriceResult res{0, 0, 0};
    if (m <= 0 || n <= 0) return res;
    prepare(st, m, n, xt, z);
    const bool sub = use_subset;
    OTIP_CHECK(!sub || subset_m_ == m, OTIP_EINVAL, "pricing: no subset built for this problem");
    const int tj = pick_tj(m, n, tile);
    dim3 grid(grid_for(m, kScanBlock), grid_for(n, tj));
    const dim3 lgrid(grid_for(m, kScanBlock / 64));
    const double units = sub ? (double)subset_nnz_ : (double)m * (double)n;
    // one pass of the given mode over all variables or over the subset
    auto launch = [&](int mode, const PriceArgs &pa, hipEvent_t e0_, hipEvent_t e1_) {
        if (sub) {
            auto kfn = mode == 0   ? by_kind(kind, price_list_pass<0, 0>, price_list_pass<0, 1>,
                                             price_list_pass<0, 2>, price_list_pass<0, 3>)
                       : mode == 1 ? by_kind(kind, price_list_pass<1, 0>, price_list_pass<1, 1>,
                                             price_list_pass<1, 2>, price_list_pass<1, 3>)
                                   : by_kind(kind, price_list_pass<2, 0>, price_list_pass<2, 1>,
                                             price_list_pass<2, 2>, price_list_pass<2, 3>);
            hipExtLaunchKernelGGL(kfn, lgrid, dim3(kScanBlock), 0, st, e0_, e1_, 0, pa,
                                  (const int64_t *)sptr_.get(), (const int32_t *)scol_.get());
        } else {
            auto kfn = mode == 0   ? by_kind(kind, price_pass<0, 0>, price_pass<0, 1>,
                                             price_pass<0, 2>, price_pass<0, 3>)
                       : mode == 1 ? by_kind(kind, price_pass<1, 0>, price_pass<1, 1>,
                                             price_pass<1, 2>, price_pass<1, 3>)
                                   : by_kind(kind, price_pass<2, 0>, price_pass<2, 1>,
                                             price_pass<2, 2>, price_pass<2, 3>);
            hipExtLaunchKernelGGL(kfn, grid, dim3(kScanBlock), 0, st, e0_, e1_, 0, pa);
        }
        OTIP_HIP(hipGetLastError());
    };
    hist_.need(kHistBins);
    cnt_.need(1);
    PriceArgs a{};
    a.m = m;
    a.n = n;
    a.tj = tj;
    a.xs = xs;
    a.y = y;
    a.jt = (const JEntry *)jt_.get();
    a.bitmap = bitmap;
    a.hist = hist_.get();
    std::vector<unsigned long long> h(kHistBins);

    auto histogram = [&](int shift, uint64_t prefix) {
        OTIP_HIP(hipMemsetAsync(hist_.get(), 0, kHistBins * sizeof(unsigned long long), st));
        a.shift = shift;
        a.prefix = prefix;
        a.rcut = (shift + 12 >= 64) ? INFINITY
                                    : rcut_of_key(((prefix + 1) << (shift + 12)) - 1);
        hipEvent_t e0_, e1_;
        if (timer) timer->arm(units, &e0_, &e1_);
        else e0_ = e1_ = nullptr;
        launch(0, a, e0_, e1_);
        OTIP_HIP(hipMemcpyAsync(h.data(), hist_.get(), kHistBins * sizeof(unsigned long long),
                                hipMemcpyDeviceToHost, st));
        OTIP_HIP(hipStreamSynchronize(st));
        if (timer) timer->collect();
        res.passes++;
        scans++;
    };

    // First pass: the histogram of the top 12 key bits of every negative
    // reduced cost outside the support (their count is the top digit's total)
    // and, in the same pass, the candidates whose key is at most a cutoff
    // guessed from the previous call's k-th selected value.  When those
    // include the k smallest keys (at least kmax of them, or all negatives),
    // the selection needs no further pass over m n.
    const bool guessing = guess_key_ != 0 && kmax > 0;
    const uint64_t gcap =
        guessing ? (uint64_t)std::max<int64_t>(4 * kmax, (int64_t)1 << 20) : 0;
    ck_.need(std::max<uint64_t>(gcap, 1));
    ci_.need(std::max<uint64_t>(gcap, 1));
    OTIP_HIP(hipMemsetAsync(hist_.get(), 0, kHistBins * sizeof(unsigned long long), st));
    OTIP_HIP(hipMemsetAsync(cnt_.get(), 0, sizeof(unsigned long long), st));
    a.shift = 52;
    a.prefix = 0;
    a.rcut = INFINITY;
    a.key_max = guessing ? guess_key_ : 0;
    a.rkey = guessing ? rcut_of_key(guess_key_) : -INFINITY;
    a.count = cnt_.get();
    a.out_key = ck_.get();
    a.out_idx = ci_.get();
    a.cap = gcap;
    unsigned long long emitted = 0;
    {
        hipEvent_t e0_, e1_;
        if (timer) timer->arm(units, &e0_, &e1_);
        else e0_ = e1_ = nullptr;
        launch(2, a, e0_, e1_);
        OTIP_HIP(hipMemcpyAsync(h.data(), hist_.get(), kHistBins * sizeof(unsigned long long),
                                hipMemcpyDeviceToHost, st));
        OTIP_HIP(hipMemcpyAsync(&emitted, cnt_.get(), sizeof(emitted), hipMemcpyDeviceToHost, st));
        OTIP_HIP(hipStreamSynchronize(st));
        if (timer) timer->collect();
        res.passes++;
        scans++;
    }
    uint64_t total = 0;
    for (auto v : h) total += v;
    res.nneg = (int64_t)total;
    if (kmax <= 0 || total == 0) return res;

    uint64_t cap = 0;
    if (guessing && emitted <= gcap &&
        ((total <= (uint64_t)kmax && emitted == total) ||
         (total > (uint64_t)kmax && emitted >= (uint64_t)kmax))) {
        cap = emitted;  // the guess held
    } else {
        // adapt the guess: too many candidates -> a cutoff further from 0
        if (guessing && emitted > gcap) guess_f_ = std::min(0.95, 0.5 * (guess_f_ + 1.0));
        if (guessing && emitted <= gcap) guess_f_ = std::max(0.05, 0.5 * guess_f_);
        // radix select of the kmax smallest keys, 12 bits per level from the
        // top, continuing from the first pass's histogram
        uint64_t key_max;
        uint64_t emit_bound;
        if (total <= (uint64_t)kmax) {
            key_max = ~0ull;
            emit_bound = total;
        } else {
            uint64_t need = (uint64_t)kmax, less = 0, prefix = 0;
            int shift = 52;
            const uint64_t slack = (uint64_t)std::max<int64_t>(kmax, 1 << 16);
            for (;;) {
                uint64_t cum = 0;
                int b = 0;
                for (; b < kHistBins; ++b) {
                    if (cum + h[b] >= need) break;
                    cum += h[b];
                }
                OTIP_CHECK(b < kHistBins, 5, "pricing: histogram inconsistent");
                less += cum;
                need -= cum;
                prefix = (prefix << 12) | (uint64_t)b;
                const uint64_t bucket = h[b];
                if (bucket <= slack || shift == 4) {
                    // every key whose top (64 - shift) bits are <= prefix
                    key_max = (shift == 0) ? prefix : (((prefix + 1) << shift) - 1);
                    if (shift == 4) key_max = ((prefix + 1) << 4) - 1;
                    emit_bound = less + bucket;
                    break;
                }
                shift = (shift >= 16) ? shift - 12 : 4;
                // the last level covers the remaining low bits in one digit
                histogram(shift, prefix);
            }
        }
        // compaction
        cap = emit_bound;
        ck_.need(cap);
        ci_.need(cap);
        OTIP_HIP(hipMemsetAsync(cnt_.get(), 0, sizeof(unsigned long long), st));
        a.key_max = key_max;
        a.rcut = key_max == ~0ull ? INFINITY : rcut_of_key(key_max);
        a.rkey = a.rcut;
        a.count = cnt_.get();
        a.out_key = ck_.get();
        a.out_idx = ci_.get();
        a.cap = cap;
        hipEvent_t e0_, e1_;
        if (timer) timer->arm(units, &e0_, &e1_);
        else e0_ = e1_ = nullptr;
        launch(1, a, e0_, e1_);
        OTIP_HIP(hipMemcpyAsync(&emitted, cnt_.get(), sizeof(emitted), hipMemcpyDeviceToHost, st));
        OTIP_HIP(hipStreamSynchronize(st));
        if (timer) timer->collect();
        res.passes++;
        scans++;
        OTIP_CHECK(emitted == cap, 5,
                   "pricing: compaction count " + std::to_string(emitted) +
                       " != histogram count " + std::to_string(cap));
    }
    // order by (key, idx): sort by idx, then stably by key (keys of negative
    // values are below 2^63)
    int ibits = 1;
    while (ibits < 64 && (((uint64_t)1 << ibits) < (uint64_t)m * (uint64_t)n)) ++ibits;
    ck2_.need(cap);
    ci2_.need(cap);
    sort_pairs_u64(st, ci_.get(), ck_.get(), ci2_.get(), ck2_.get(), (int64_t)cap, 0, ibits, tmp_);
    sort_pairs_u64(st, ck2_.get(), ci2_.get(), ck_.get(), ci_.get(), (int64_t)cap, 0, 63, tmp_);
    const int64_t k = std::min<int64_t>(kmax, (int64_t)cap);
    hipLaunchKernelGGL(decode_selection, dim3(grid_for(k, 256)), dim3(256), 0, st, k, m,
                       ck_.get(), ci_.get(), oi, oj, orr, oidx);
    OTIP_HIP(hipGetLastError());
    // next call's cutoff: the key that admits about 4 kmax of this call's
    // candidates (the first pass keeps up to 16 kmax, so the next iterate's
    // distribution may move either way); with fewer candidates than that, a
    // fraction guess_f_ of the last one's value (nearer to 0: more of them)
    const int64_t want = std::min<int64_t>(4 * (int64_t)kmax, (int64_t)cap);
    uint64_t gk = 0;
    OTIP_HIP(hipMemcpyAsync(&gk, ck_.get() + (want - 1), sizeof(gk), hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipStreamSynchronize(st));
    double rg = rcut_of_key(gk);
    if (want < 4 * (int64_t)kmax) rg *= guess_f_;
    guess_key_ = (std::isfinite(rg) && rg < 0.0) ? host_dkey(rg) : 0;
    res.count = k;
    return res;
}

// ----------------------------------------------------------------- minimum scan
struct MinArgs {
    int m, n, tj;
    const int32_t *xs;
    const double *y;
    const JEntry *jt;
    double *bmin;
    uint64_t *barg;
};

template <int K>
__global__ __launch_bounds__(kScanBlock) void rmin_pass(MinArgs a) {
    __shared__ double sv[kScanBlock / 64];
    __shared__ uint64_t si[kScanBlock / 64];
    const int i = blockIdx.x * kScanBlock + threadIdx.x;
    const int j0 = blockIdx.y * a.tj, j1 = min(a.n, j0 + a.tj);
    const RowData rd = load_row(i, a.m, a.xs, a.y);
    double best = INFINITY;
    uint64_t arg = ~0ull;
    for (int j = j0; j < j1; ++j) {
        const JEntry t = ldj(a.jt, j);
        const double r = (cost_of<K>(rd, t) - rd.y) - t.z;
        if (r < best) {  // first j attaining the minimum for this row
            best = r;
            arg = (uint64_t)i + (uint64_t)j * (uint64_t)a.m;
        }
    }
    // (value, index) lexicographic minimum over the block
    for (int o = 32; o > 0; o >>= 1) {
        double ov = __shfl_xor(best, o, 64);
        uint64_t oa = __shfl_xor(arg, o, 64);
        if (ov < best || (ov == best && oa < arg)) {
            best = ov;
            arg = oa;
        }
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sv[w] = best;
        si[w] = arg;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kScanBlock / 64; ++k)
            if (sv[k] < best || (sv[k] == best && si[k] < arg)) {
                best = sv[k];
                arg = si[k];
            }
        const size_t b = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
        a.bmin[b] = best;
        a.barg[b] = arg;
    }
}

void Scanner::rmin(hipStream_t st, int m, int n, const int32_t *xs, const int32_t *xt,
                   const double *y, const double *z, double *out, int64_t *arg) {
    prepare(st, m, n, xt, z);
    const int tj = pick_tj(m, n, tile);
    dim3 grid(grid_for(m, kScanBlock), grid_for(n, tj));
    const size_t nb = (size_t)grid.x * grid.y;
    bmin_.need(nb);
    barg_.need(nb);
    MinArgs a{m, n, tj, xs, y, (const JEntry *)jt_.get(), bmin_.get(), barg_.get()};
    hipLaunchKernelGGL(by_kind(kind, rmin_pass<0>, rmin_pass<1>, rmin_pass<2>, rmin_pass<3>),
                       grid, dim3(kScanBlock), 0, st, a);
    OTIP_HIP(hipGetLastError());
    scans++;
    std::vector<double> v(nb);
    std::vector<uint64_t> ai(nb);
    OTIP_HIP(hipMemcpyAsync(v.data(), bmin_.get(), nb * sizeof(double), hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipMemcpyAsync(ai.data(), barg_.get(), nb * sizeof(uint64_t), hipMemcpyDeviceToHost,
                            st));
    OTIP_HIP(hipStreamSynchronize(st));
    double best = INFINITY;
    uint64_t ba = ~0ull;
    for (size_t b = 0; b < nb; ++b)
        if (v[b] < best || (v[b] == best && ai[b] < ba)) {
            best = v[b];
            ba = ai[b];
        }
    *out = best;
    if (arg) *arg = (int64_t)ba;
}

// ------------------------------------------------------- initial support scans
// The integer that orders the costs of a kind: the cost itself for the
// squared, 1- and inf-norm costs, the squared norm for the 2-norm (its square
// root is increasing, so thresholds and argmins on it select the same sets).
__device__ __forceinline__ int64_t int_cost(const int32_t *xs, const int32_t *xt, int i, int j,
                                            int kind) {
    int64_t d0 = (int64_t)xs[2 * i] - xt[2 * j];
    int64_t d1 = (int64_t)xs[2 * i + 1] - xt[2 * j + 1];
    if (kind == OTIP_COST_L1) return (d0 < 0 ? -d0 : d0) + (d1 < 0 ? -d1 : d1);
    if (kind == OTIP_COST_LINF) return max(d0 < 0 ? -d0 : d0, d1 < 0 ? -d1 : d1);
    return d0 * d0 + d1 * d1;
}

template <int PASS>
__global__ __launch_bounds__(kScanBlock) void subset_lists(int m, int n, int kind,
                                                           const int32_t *__restrict__ xs,
                                                           const int32_t *__restrict__ xt,
                                                           int64_t L, int64_t *cnt,
                                                           const int64_t *__restrict__ off,
                                                           int32_t *__restrict__ col) {
    const int lane = threadIdx.x & 63;
    const int waves = gridDim.x * (kScanBlock / 64);
    for (int i = blockIdx.x * (kScanBlock / 64) + (threadIdx.x >> 6); i < m; i += waves) {
        int64_t pos = PASS == 1 ? off[i] : 0;
        int c = 0;
        for (int j0 = 0; j0 < n; j0 += 64) {
            const int j = j0 + lane;
            const bool take = j < n && int_cost(xs, xt, i, j, kind) < L;
            const uint64_t mask = __ballot(take);
            if (PASS == 0) {
                c += __popcll(mask);
            } else {
                if (take) col[pos + __popcll(mask & ((1ull << lane) - 1ull))] = j;
                pos += __popcll(mask);
            }
        }
        if (PASS == 0 && lane == 0) cnt[i] = c;
    }
}

// histogram of (c - lo) >> shift for lo <= c <= hi; count of c < lo
__global__ __launch_bounds__(kScanBlock) void cost_hist(int m, int n, int tj, int kind, const int32_t *xs,
                                                        const int32_t *xt, int64_t lo, int64_t hi,
                                                        int shift, unsigned long long *hist,
                                                        unsigned long long *below) {
    __shared__ unsigned int lh[kHistBins];
    __shared__ unsigned int lbelow;
    for (int t = threadIdx.x; t < kHistBins; t += kScanBlock) lh[t] = 0u;
    if (threadIdx.x == 0) lbelow = 0u;
    __syncthreads();
    const int i = blockIdx.x * kScanBlock + threadIdx.x;
    const int j0 = blockIdx.y * tj, j1 = min(n, j0 + tj);
    if (i < m) {
        unsigned int nb = 0;
        for (int j = j0; j < j1; ++j) {
            int64_t c = int_cost(xs, xt, i, j, kind);
            if (c < lo)
                ++nb;
            else if (c <= hi)
                atomicAdd(&lh[(c - lo) >> shift], 1u);
        }
        if (nb) atomicAdd(&lbelow, nb);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kHistBins; t += kScanBlock)
        if (lh[t]) atomicAdd(&hist[t], (unsigned long long)lh[t]);
    if (threadIdx.x == 0 && lbelow) atomicAdd(below, (unsigned long long)lbelow);
}

// number of c_ij <= T in each column j (one block per column)
__global__ __launch_bounds__(kScanBlock) void count_le_col(int m, int n, int kind, const int32_t *xs,
                                                           const int32_t *xt, int64_t T,
                                                           int64_t *cnt) {
    __shared__ double lds[16];
    const int j = blockIdx.x;
    int c = 0;
    for (int i = threadIdx.x; i < m; i += kScanBlock) c += int_cost(xs, xt, i, j, kind) <= T;
    double t = block_sum((double)c, lds);
    if (threadIdx.x == 0) cnt[j] = (int64_t)t;
}

// write the variable indices with c_ij <= T of column j in increasing i
__global__ __launch_bounds__(kScanBlock) void collect_le_col(int m, int n, int kind, const int32_t *xs,
                                                             const int32_t *xt, int64_t T,
                                                             const int64_t *off,
                                                             uint64_t *out) {
    __shared__ int wcount[kScanBlock / 64];
    const int j = blockIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t base = off[j];
    for (int i0 = 0; i0 < m; i0 += kScanBlock) {
        const int i = i0 + threadIdx.x;
        const bool take = i < m && int_cost(xs, xt, i, j, kind) <= T;
        const uint64_t mask = __ballot(take);
        if (lane == 0) wcount[w] = __popcll(mask);
        __syncthreads();
        int before = 0, total = 0;
        for (int k = 0; k < kScanBlock / 64; ++k) {
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

// cheapest target of each source (ties: smallest j) -> variable index
__global__ __launch_bounds__(kScanBlock) void row_argmin(int m, int n, int kind, const int32_t *xs,
                                                         const int32_t *xt, uint64_t *out) {
    __shared__ int64_t sc[kScanBlock];
    __shared__ int sj[kScanBlock];
    const int i = blockIdx.x;
    int64_t best = INT64_MAX;
    int arg = n;
    for (int j = threadIdx.x; j < n; j += kScanBlock) {
        int64_t c = int_cost(xs, xt, i, j, kind);
        if (c < best) {
            best = c;
            arg = j;
        }
    }
    sc[threadIdx.x] = best;
    sj[threadIdx.x] = arg;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int t = 1; t < kScanBlock; ++t)
            if (sc[t] < best || (sc[t] == best && sj[t] < arg)) {
                best = sc[t];
                arg = sj[t];
            }
        out[i] = (uint64_t)i + (uint64_t)arg * (uint64_t)m;
    }
}

// cheapest source of each target (ties: smallest i) -> variable index
__global__ __launch_bounds__(kScanBlock) void col_argmin(int m, int n, int kind, const int32_t *xs,
                                                         const int32_t *xt, uint64_t *out) {
    __shared__ int64_t sc[kScanBlock];
    __shared__ int si[kScanBlock];
    const int j = blockIdx.x;
    int64_t best = INT64_MAX;
    int arg = m;
    for (int i = threadIdx.x; i < m; i += kScanBlock) {
        int64_t c = int_cost(xs, xt, i, j, kind);
        if (c < best) {
            best = c;
            arg = i;
        }
    }
    sc[threadIdx.x] = best;
    si[threadIdx.x] = arg;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int t = 1; t < kScanBlock; ++t)
            if (sc[t] < best || (sc[t] == best && si[t] < arg)) {
                best = sc[t];
                arg = si[t];
            }
        out[j] = (uint64_t)arg + (uint64_t)j * (uint64_t)m;
    }
}

int64_t Scanner::initial_support(hipStream_t st, int m, int n, const int32_t *xs,
                                 const int32_t *xt, double kappa, int64_t cmax,
                                 DBuf<uint64_t> &out, int64_t *T_out) {
    const int64_t target = std::min<int64_t>((int64_t)std::ceil(kappa * (double)(m + n - 1)),
                                             (int64_t)m * (int64_t)n);
    const int tj = pick_tj(m, n, tile);
    dim3 grid(grid_for(m, kScanBlock), grid_for(n, tj));
    hist_.need(kHistBins);
    cnt_.need(1);
    std::vector<unsigned long long> h(kHistBins);
    int64_t lo = 0, hi = cmax, below_total = 0, T = cmax;
    for (;;) {
        int shift = 0;
        while (((hi - lo) >> shift) >= kHistBins) ++shift;
        OTIP_HIP(hipMemsetAsync(hist_.get(), 0, kHistBins * sizeof(unsigned long long), st));
        OTIP_HIP(hipMemsetAsync(cnt_.get(), 0, sizeof(unsigned long long), st));
        hipLaunchKernelGGL(cost_hist, grid, dim3(kScanBlock), 0, st, m, n, tj, kind, xs, xt, lo, hi,
                           shift, hist_.get(), cnt_.get());
        OTIP_HIP(hipGetLastError());
        unsigned long long below = 0;
        OTIP_HIP(hipMemcpyAsync(h.data(), hist_.get(), kHistBins * sizeof(unsigned long long),
                                hipMemcpyDeviceToHost, st));
        OTIP_HIP(hipMemcpyAsync(&below, cnt_.get(), sizeof(below), hipMemcpyDeviceToHost, st));
        OTIP_HIP(hipStreamSynchronize(st));
        below_total = (int64_t)below;
        int64_t cum = below_total;
        int b = 0;
        for (; b < kHistBins; ++b) {
            if (cum + (int64_t)h[b] >= target) break;
            cum += (int64_t)h[b];
        }
        if (b >= kHistBins) {
            T = hi;
            break;
        }
        const int64_t nlo = lo + ((int64_t)b << shift);
        const int64_t nhi = std::min(hi, lo + (((int64_t)b + 1) << shift) - 1);
        if (shift == 0) {
            T = nlo;
            break;
        }
        lo = nlo;
        hi = nhi;
    }
    *T_out = T;
    // collect {c <= T} in variable order
    DBuf<int64_t> &cnt = i64a_;
    DBuf<int64_t> &off = i64b_;
    cnt.need((size_t)n);
    off.need((size_t)n + 1);
    hipLaunchKernelGGL(count_le_col, dim3(n), dim3(kScanBlock), 0, st, m, n, kind, xs, xt, T, cnt.get());
    OTIP_HIP(hipGetLastError());
    exclusive_scan_i64(st, cnt.get(), off.get(), n, tmp_);
    int64_t last_off = 0, last_cnt = 0;
    OTIP_HIP(hipMemcpyAsync(&last_off, off.get() + (n - 1), sizeof(int64_t), hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipMemcpyAsync(&last_cnt, cnt.get() + (n - 1), sizeof(int64_t), hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipStreamSynchronize(st));
    const int64_t nle = last_off + last_cnt;
    const int64_t tot = nle + m + n;
    DBuf<uint64_t> &tmpk = u64a_;
    tmpk.need((size_t)tot);
    hipLaunchKernelGGL(collect_le_col, dim3(n), dim3(kScanBlock), 0, st, m, n, kind, xs, xt, T, off.get(),
                       tmpk.get());
    hipLaunchKernelGGL(row_argmin, dim3(m), dim3(kScanBlock), 0, st, m, n, kind, xs, xt,
                       tmpk.get() + nle);
    hipLaunchKernelGGL(col_argmin, dim3(n), dim3(kScanBlock), 0, st, m, n, kind, xs, xt,
                       tmpk.get() + nle + m);
    OTIP_HIP(hipGetLastError());
    // union: sort and drop duplicates
    DBuf<uint64_t> &sorted = u64b_;
    sorted.need((size_t)tot);
    sort_keys_u64(st, tmpk.get(), sorted.get(), tot, tmp_);
    out.need((size_t)tot);
    int64_t nu = unique_u64(st, sorted.get(), out.get(), tot, tmp_, cnt_);
    return nu;
}

}  // namespace otip

namespace otip {

// ------------------------------------------------------------ mixed precision
// FP32 pricing with an FP64 re-check.  The FP32 pass need not round like the
// FP64 one, only stay within a proven distance of the exact reduced cost, so
// it uses the separable form r = (|x_i|^2 - y_i) + (|x_j|^2 - z_j)
// - 2 x_i.x_j: u_i = fl32(fl64(|x_i|^2 - y_i)) per source, v_j likewise per
// target, then r32 = fl(b_i (-2 b_j) + fl(a_i (-2 a_j) + fl(u_i + v_j))) with
// two fused multiply-adds (coordinates and their doubles are exact in FP32):
// three operations per reduced cost against five in the exact FP64 form.
// With K = 2 (X + X')^2 + Y + Z (X, X' the largest source and target
// coordinate magnitudes, Y, Z the largest |y|, |z|), every intermediate is at
// most K in magnitude and each of the five roundings (two in u and v, three in
// the sum and the two fused operations) errs by at most u32 K (u32 = 2^-24),
// up to second-order terms: |r32 - r| <= 4 (u32 + u64) K, while the FP64 scan's
// value errs by at most 2 u64 K.  margin = 9 u32 K exceeds twice their sum.
// Hence
//   r32 < -margin  =>  r64 < 0 (certainly negative);
//   an entry of the FP64 top-k has r32 <= tau32 + 2 margin, tau32 the k-th
//   smallest FP32 value among r32 < margin.
// Every candidate with r32 <= min(margin, tau32 + 2 margin), and every entry of
// the band -margin <= r32 < margin (for the exact negative count), is
// re-evaluated in FP64 exactly as the FP64 scan does; the selection is then
// identical to the FP64 one.  (The FP32 form is used only while 2 (X + X')^2
// < 2^24, which keeps the band narrow for duals on the scale of the costs.)
struct __align__(16) JEntry32 {
    float v, a2, b2, pad;
};

__device__ __forceinline__ JEntry32 ldj32(const JEntry32 *p, int j) {
    const cfptr q = (cfptr)(p + j);
    JEntry32 e;
    e.v = q[0];
    e.a2 = q[1];
    e.b2 = q[2];
    e.pad = 0.f;
    return e;
}

// four consecutive entries (j a multiple of 4; the table is 256-byte aligned)
// with one 64-byte scalar load
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef const __attribute__((address_space(4))) f32x16 *cf16ptr;
__device__ __forceinline__ void ldj32x4(const JEntry32 *p, int j, JEntry32 (&t)[4]) {
    const f32x16 q = *(cf16ptr)(p + j);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        t[k].v = q[4 * k];
        t[k].a2 = q[4 * k + 1];
        t[k].b2 = q[4 * k + 2];
        t[k].pad = 0.f;
    }
}

__global__ void build_jtab32(int n, const int32_t *__restrict__ xt, const double *__restrict__ z,
                             JEntry32 *__restrict__ jt) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double a = (double)xt[2 * j], b = (double)xt[2 * j + 1];
    JEntry32 e;
    e.v = (float)((a * a + b * b) - z[j]);
    e.a2 = (float)(-2.0 * a);
    e.b2 = (float)(-2.0 * b);
    e.pad = 0.f;
    jt[j] = e;
}

__device__ __forceinline__ uint32_t fkey(float r) {
    uint32_t u = __float_as_uint(r);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

struct Price32Args {
    int m, n, tj;
    const int32_t *xs;
    const double *y;
    const JEntry32 *jt;
    const uint32_t *bitmap;
    float margin;
    int shift;          // histogram digit (key >> shift) & 4095, keys r32 < margin
    uint32_t prefix;    // bits above shift + 12 (no filter when shift + 12 >= 32)
    unsigned long long *hist, *certain, *band;
    float t32;          // compaction: r32 <= t32, or -margin <= r32 < margin
    float rcut;         // no value of interest lies above rcut (+inf: no bound)
    unsigned long long *count;
    uint64_t *out_idx;
    uint64_t cap;
};

// the per-variable part of an FP32 pass (all lanes of the wave call it)
template <int MODE>
__device__ __forceinline__ void price32_one(const Price32Args &a, int i, int j, float r,
                                            unsigned int *lh, unsigned int &ncert,
                                            unsigned int &nband, WaveStage<1> &stg) {
    const float mg = a.margin;
    const bool lo = MODE == 0 ? (r < mg && r <= a.rcut) : (r < mg && (r <= a.t32 || r >= -mg));
    if (__ballot(lo) == 0ull) return;
    const uint64_t idx = (uint64_t)i + (uint64_t)j * (uint64_t)a.m;
    bool take = lo && !in_support(a.bitmap, idx);
    if (MODE == 0) {
        if (take) {
            const int pshift = a.shift + 12;
            if (pshift >= 32) {  // first level: the certain and uncertain counts
                if (r < -mg)
                    ++ncert;
                else
                    ++nband;
            }
            const uint32_t key = fkey(r);
            if (pshift >= 32 || (key >> pshift) == a.prefix)
                atomicAdd(&lh[(key >> a.shift) & 4095u], 1u);
        }
    } else {
        stg.push(take, 0ull, idx);
    }
}

// FP32 pass.  MODE 0: histogram of one 12-bit digit of the FP32 key of every
// r32 < margin outside the support (and, on the first level, the counts of
// the certain negatives r32 < -margin and of the band); MODE 1: append the
// variable index of every candidate.  Four targets at a time: a group with no
// value of interest costs one ballot.
template <int MODE>
__global__ __launch_bounds__(kScanBlock) void price32_pass(Price32Args a) {
    __shared__ unsigned int lh[MODE == 0 ? kHistBins : 1];
    __shared__ unsigned int lc[2];
    __shared__ uint64_t sbuf[MODE == 1 ? (kScanBlock / 64) * kStage : 1];
    WaveStage<1> stg{sbuf + (MODE == 1 ? (threadIdx.x >> 6) * kStage : 0), 0, a.count, nullptr,
                     a.out_idx, a.cap};
    const int i = blockIdx.x * kScanBlock + threadIdx.x;
    const int j0 = blockIdx.y * a.tj, j1 = min(a.n, j0 + a.tj);
    if (MODE == 0) {
        for (int t = threadIdx.x; t < kHistBins; t += kScanBlock) lh[t] = 0u;
        if (threadIdx.x < 2) lc[threadIdx.x] = 0u;
        __syncthreads();
    }
    // rows past m get u = +inf: every value they produce is +inf
    float al = 0.f, be = 0.f, u = INFINITY;
    if (i < a.m) {
        const double ad = (double)a.xs[2 * i], bd = (double)a.xs[2 * i + 1];
        al = (float)ad;
        be = (float)bd;
        u = (float)((ad * ad + bd * bd) - a.y[i]);
    }
    const float lim = fminf(a.margin, a.rcut);
    unsigned int ncert = 0, nband = 0;
    int j = j0;
    for (; j + 4 <= j1; j += 4) {
        JEntry32 t[4];
        ldj32x4(a.jt, j, t);
        const float r0 = fmaf(be, t[0].b2, fmaf(al, t[0].a2, u + t[0].v));
        const float r1 = fmaf(be, t[1].b2, fmaf(al, t[1].a2, u + t[1].v));
        const float r2 = fmaf(be, t[2].b2, fmaf(al, t[2].a2, u + t[2].v));
        const float r3 = fmaf(be, t[3].b2, fmaf(al, t[3].a2, u + t[3].v));
        const float lo = fminf(fminf(r0, r1), fminf(r2, r3));
        bool any;
        if (MODE == 0) {
            any = lo < a.margin && lo <= lim;
        } else {  // candidates r32 <= t32 (< margin), or the band |r32| < margin
            const float la = fminf(fminf(fabsf(r0), fabsf(r1)), fminf(fabsf(r2), fabsf(r3)));
            any = lo <= a.t32 || la < a.margin;
        }
        if (__ballot(any) == 0ull) continue;
        price32_one<MODE>(a, i, j, r0, lh, ncert, nband, stg);
        price32_one<MODE>(a, i, j + 1, r1, lh, ncert, nband, stg);
        price32_one<MODE>(a, i, j + 2, r2, lh, ncert, nband, stg);
        price32_one<MODE>(a, i, j + 3, r3, lh, ncert, nband, stg);
    }
    for (; j < j1; ++j) {
        const JEntry32 t = ldj32(a.jt, j);
        const float r = fmaf(be, t.b2, fmaf(al, t.a2, u + t.v));
        price32_one<MODE>(a, i, j, r, lh, ncert, nband, stg);
    }
    if (MODE == 1) stg.flush();
    if (MODE == 0) {
        if (ncert) atomicAdd(&lc[0], ncert);
        if (nband) atomicAdd(&lc[1], nband);
        __syncthreads();
        for (int t = threadIdx.x; t < kHistBins; t += kScanBlock)
            if (lh[t]) atomicAdd(&a.hist[t], (unsigned long long)lh[t]);
        if (threadIdx.x == 0) {
            if (lc[0]) atomicAdd(a.certain, (unsigned long long)lc[0]);
            if (lc[1]) atomicAdd(a.band, (unsigned long long)lc[1]);
        }
    }
}

// FP64 re-evaluation of the compacted candidates, exactly as the FP64 scan;
// negative ones get their ordered key, others the key ~0 (sorted last).
__global__ void recheck64(int64_t k, int m, const uint64_t *__restrict__ idx,
                          const int32_t *__restrict__ xs, const int32_t *__restrict__ xt,
                          const double *__restrict__ y, const double *__restrict__ z,
                          float margin, uint64_t *__restrict__ key,
                          unsigned long long *band_neg) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= k) return;
    const uint64_t v = idx[t];
    const int i = (int)(v % (uint64_t)m), j = (int)(v / (uint64_t)m);
    const double al = (double)xs[2 * i], be = (double)xs[2 * i + 1];
    const double aj = (double)xt[2 * j], bj = (double)xt[2 * j + 1];
    const double c = fma(be, -2.0 * bj, fma(al, -2.0 * aj, (al * al + be * be) + (aj * aj + bj * bj)));
    const double r = (c - y[i]) - z[j];
    key[t] = r < 0.0 ? dkey(r) : ~0ull;
    // the same FP32 value as the scan, to recognise the band
    const float u = (float)((al * al + be * be) - y[i]);
    const float w = (float)((aj * aj + bj * bj) - z[j]);
    const float r32 = fmaf((float)be, (float)(-2.0 * bj), fmaf((float)al, (float)(-2.0 * aj), u + w));
    if (r32 >= -margin && r32 < margin && r < 0.0) atomicAdd(band_neg, 1ull);
}

// out[0..3] = max |xs|, max |xt|, max |y|, max |z| over a grid of blocks; out
// is zeroed first.  The maxima are non-negative, so their IEEE bit patterns
// order like the values and an integer atomic maximum combines the blocks.
__global__ void maxabs4(int m, int n, const int32_t *xs, const int32_t *xt, const double *y,
                        const double *z, unsigned long long *out) {
    __shared__ double sm[4][16];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const int stride = gridDim.x * blockDim.x;
    const int t0 = blockIdx.x * blockDim.x + threadIdx.x;
    for (int t = t0; t < 2 * m; t += stride) v[0] = fmax(v[0], fabs((double)xs[t]));
    for (int t = t0; t < 2 * n; t += stride) v[1] = fmax(v[1], fabs((double)xt[t]));
    for (int t = t0; t < m; t += stride) v[2] = fmax(v[2], fabs(y[t]));
    for (int t = t0; t < n; t += stride) v[3] = fmax(v[3], fabs(z[t]));
    for (int q = 0; q < 4; ++q) {
        double w = v[q];
        for (int o = 32; o > 0; o >>= 1) w = fmax(w, __shfl_xor(w, o, 64));
        if ((threadIdx.x & 63) == 0) sm[q][threadIdx.x >> 6] = w;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double w = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) w = fmax(w, sm[threadIdx.x][k]);
        atomicMax(&out[threadIdx.x], (unsigned long long)__double_as_longlong(w));
    }
}

// the float with ordered FP32 key k (host side), or +inf where k is no number's key
static float rcut32_of_key(uint32_t k) {
    const uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    float f;
    std::memcpy(&f, &u, sizeof f);
    return std::isnan(f) ? INFINITY : f;
}

PriceResult Scanner::price_mixed(hipStream_t st, int m, int n, const int32_t *xs,
                                 const int32_t *xt, const double *y, const double *z,
                                 const uint32_t *bitmap, int64_t kmax, int32_t *oi, int32_t *oj,
                                 double *orr, uint64_t *oidx) {
    // the heuristic subset is scanned in FP64 (a small fraction of m n)
    if (use_subset)
        return price(st, m, n, xs, xt, y, z, bitmap, kmax, oi, oj, orr, oidx);
    PriceResult res{0, 0, 0};
    if (m <= 0 || n <= 0) return res;
    // the FP32 scan is written for the squared cost; the norm costs take the
    // FP64 scan (same result)
    if (kind != OTIP_COST_SQEUCLID)
        return price(st, m, n, xs, xt, y, z, bitmap, kmax, oi, oj, orr, oidx);
    // bounds for the margin and the exactness of FP32 costs
    DBuf<double> &mx = bmin_;
    mx.need(4);
    OTIP_HIP(hipMemsetAsync(mx.get(), 0, 4 * sizeof(double), st));
    const unsigned nbm = std::min<unsigned>(256, grid_for(2 * (int64_t)std::max(m, n), 256));
    hipLaunchKernelGGL(maxabs4, dim3(nbm), dim3(256), 0, st, m, n, xs, xt, y, z,
                       (unsigned long long *)mx.get());
    double h4[4];
    OTIP_HIP(hipMemcpyAsync(h4, mx.get(), sizeof(h4), hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipStreamSynchronize(st));
    const double X = h4[0], Xt = h4[1];
    const double Cbound = 2.0 * (X + Xt) * (X + Xt);
    const double inter = 2.0 * X * X + 2.0 * Xt * Xt + 4.0 * X * Xt;
    if (!(inter < 16777216.0))  // a wide band: the FP64 scan (same result)
        return price(st, m, n, xs, xt, y, z, bitmap, kmax, oi, oj, orr, oidx);
    const double margin = 9.0 * std::ldexp(1.0, -24) * (Cbound + h4[2] + h4[3]);
    const float mg = (float)margin;

    jt_.need((size_t)n * sizeof(JEntry32));
    hipLaunchKernelGGL(build_jtab32, dim3(grid_for(n, 256)), dim3(256), 0, st, n, xt, z,
                       (JEntry32 *)jt_.get());
    const int tj = pick_tj(m, n, tile);
    dim3 grid(grid_for(m, kScanBlock), grid_for(n, tj));
    hist_.need(kHistBins + 3);
    cnt_.need(2);
    Price32Args a{};
    a.m = m;
    a.n = n;
    a.tj = tj;
    a.xs = xs;
    a.y = y;
    a.jt = (const JEntry32 *)jt_.get();
    a.bitmap = bitmap;
    a.margin = mg;
    a.hist = hist_.get();
    a.certain = hist_.get() + kHistBins;
    a.band = hist_.get() + kHistBins + 1;
    std::vector<unsigned long long> h(kHistBins + 2);
    auto histogram = [&](int shift, uint32_t prefix) {
        OTIP_HIP(hipMemsetAsync(hist_.get(), 0, (kHistBins + 2) * sizeof(unsigned long long), st));
        a.shift = shift;
        a.prefix = prefix;
        a.rcut = (shift + 12 >= 32) ? INFINITY : rcut32_of_key(((prefix + 1u) << (shift + 12)) - 1u);
        hipEvent_t e0_, e1_;
        if (timer) timer->arm((double)m * (double)n, &e0_, &e1_);
        else e0_ = e1_ = nullptr;
        hipExtLaunchKernelGGL(price32_pass<0>, grid, dim3(kScanBlock), 0, st, e0_, e1_, 0, a);
        OTIP_HIP(hipGetLastError());
        OTIP_HIP(hipMemcpyAsync(h.data(), hist_.get(), (kHistBins + 2) * sizeof(unsigned long long),
                                hipMemcpyDeviceToHost, st));
        OTIP_HIP(hipStreamSynchronize(st));
        if (timer) timer->collect();
        res.passes++;
        scans++;
    };
    histogram(20, 0);
    const uint64_t certain = h[kHistBins], band = h[kHistBins + 1];
    const uint64_t total32 = certain + band;
    // threshold of the FP64 candidates
    float t32 = mg;
    if (kmax > 0 && total32 > (uint64_t)kmax) {
        // two 12-bit levels resolve the top 24 key bits; tau32 is taken as the
        // largest value of the selected bucket (an upper bound: a larger
        // threshold only adds candidates to the FP64 re-check)
        uint64_t need = (uint64_t)kmax;
        uint32_t prefix = 0;
        int shift = 20;
        for (;;) {
            uint64_t cum = 0;
            int b = 0;
            for (; b < kHistBins; ++b) {
                if (cum + h[b] >= need) break;
                cum += h[b];
            }
            OTIP_CHECK(b < kHistBins, 5, "mixed pricing: histogram inconsistent");
            need -= cum;
            prefix = (prefix << 12) | (uint32_t)b;
            if (shift == 8 || h[b] <= 1) {
                const uint32_t kmaxkey = ((prefix + 1u) << shift) - 1u;
                const uint32_t u = (kmaxkey & 0x80000000u) ? (kmaxkey & 0x7fffffffu) : ~kmaxkey;
                const float tau = __builtin_bit_cast(float, u);
                t32 = std::min(mg, (float)((double)tau + 2.0 * margin));
                break;
            }
            shift = 8;
            histogram(shift, prefix);
        }
    }
    // compaction of the candidates and of the uncertain band
    uint64_t cap = std::max<uint64_t>((uint64_t)std::max<int64_t>(kmax, 0) + band + 1024, 1 << 16);
    OTIP_HIP(hipMemsetAsync(cnt_.get(), 0, sizeof(unsigned long long), st));
    unsigned long long emitted = 0;
    for (int attempt = 0; attempt < 2; ++attempt) {
        ci_.need(cap);
        OTIP_HIP(hipMemsetAsync(cnt_.get(), 0, sizeof(unsigned long long), st));
        a.t32 = t32;
        a.rcut = INFINITY;
        a.count = cnt_.get();
        a.out_idx = ci_.get();
        a.cap = cap;
        hipEvent_t e0_, e1_;
        if (timer) timer->arm((double)m * (double)n, &e0_, &e1_);
        else e0_ = e1_ = nullptr;
        hipExtLaunchKernelGGL(price32_pass<1>, grid, dim3(kScanBlock), 0, st, e0_, e1_, 0, a);
        OTIP_HIP(hipGetLastError());
        OTIP_HIP(hipMemcpyAsync(&emitted, cnt_.get(), sizeof(emitted), hipMemcpyDeviceToHost, st));
        OTIP_HIP(hipStreamSynchronize(st));
        if (timer) timer->collect();
        res.passes++;
        scans++;
        if (emitted <= cap) break;
        cap = emitted + 1024;
    }
    OTIP_CHECK(emitted <= cap, 5, "mixed pricing: compaction overflow");
    const int64_t E = (int64_t)emitted;
    ck_.need(std::max<int64_t>(E, 1));
    unsigned long long *bneg = cnt_.get() + 1;
    OTIP_HIP(hipMemsetAsync(bneg, 0, sizeof(unsigned long long), st));
    if (E > 0)
        hipLaunchKernelGGL(recheck64, dim3(grid_for(E, 256)), dim3(256), 0, st, E, m, ci_.get(), xs,
                           xt, y, z, mg, ck_.get(), bneg);
    unsigned long long hb = 0;
    OTIP_HIP(hipMemcpyAsync(&hb, bneg, sizeof(hb), hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipStreamSynchronize(st));
    res.nneg = (int64_t)(certain + hb);
    if (kmax <= 0 || E == 0) return res;
    ck2_.need(E);
    ci2_.need(E);
    sort_pairs_u64(st, ci_.get(), ck_.get(), ci2_.get(), ck2_.get(), E, 0, 64, tmp_);
    sort_pairs_u64(st, ck2_.get(), ci2_.get(), ck_.get(), ci_.get(), E, 0, 64, tmp_);
    const int64_t k = std::min<int64_t>(kmax, res.nneg);
    hipLaunchKernelGGL(decode_selection, dim3(grid_for(std::max<int64_t>(k, 1), 256)), dim3(256), 0,
                       st, k, m, ck_.get(), ci_.get(), oi, oj, orr, oidx);
    OTIP_HIP(hipGetLastError());
    res.count = k;
    return res;
}

}  // namespace otip
