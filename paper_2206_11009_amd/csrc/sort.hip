// Index bookkeeping primitives (sorting, unique, prefix sums) on rocPRIM.
// They serve the integer side of the method: ordering selected columns,
// rebuilding the support's row/column views and deduplicating index sets.
#include <cstring>

#include <rocprim/rocprim.hpp>

#include "internal.h"

namespace otip {

#define OTIP_PRIM(call_with_temp)                                                  \
    do {                                                                           \
        size_t bytes_ = 0;                                                         \
        {                                                                          \
            void *t_ = nullptr;                                                    \
            size_t &sz_ = bytes_;                                                  \
            (void)t_;                                                              \
            OTIP_HIP(call_with_temp(nullptr, sz_));                                \
        }                                                                          \
        void *tp_ = tmp.need(bytes_ + 256);                                        \
        OTIP_HIP(call_with_temp(tp_, bytes_));                                     \
    } while (0)

void sort_pairs_u64(hipStream_t st, const uint64_t *kin, const uint64_t *vin, uint64_t *kout,
                    uint64_t *vout, int64_t n, int begin_bit, int end_bit, DBuf<char> &tmp) {
    if (n <= 0) return;
    auto call = [&](void *t, size_t &sz) {
        return rocprim::radix_sort_pairs(t, sz, kin, kout, vin, vout, (size_t)n,
                                         (unsigned)begin_bit, (unsigned)end_bit, st);
    };
    OTIP_PRIM(call);
}

void sort_pairs_u32_i32(hipStream_t st, const uint32_t *kin, const int32_t *vin, uint32_t *kout,
                        int32_t *vout, int64_t n, int end_bit, DBuf<char> &tmp) {
    if (n <= 0) return;
    auto call = [&](void *t, size_t &sz) {
        return rocprim::radix_sort_pairs(t, sz, kin, kout, vin, vout, (size_t)n, 0u,
                                         (unsigned)end_bit, st);
    };
    OTIP_PRIM(call);
}

void sort_keys_u64(hipStream_t st, const uint64_t *kin, uint64_t *kout, int64_t n,
                   DBuf<char> &tmp) {
    if (n <= 0) return;
    auto call = [&](void *t, size_t &sz) {
        return rocprim::radix_sort_keys(t, sz, kin, kout, (size_t)n, 0u, 64u, st);
    };
    OTIP_PRIM(call);
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

void sort_pairs_u64_f64x2(hipStream_t st, const uint64_t *kin, const double *v1in,
                          const double *v2in, uint64_t *kout, double *v1out, double *v2out,
                          int64_t n, int end_bit, DBuf<char> &tmp, DBuf<int32_t> &perm_a,
                          DBuf<int32_t> &perm_b) {
    if (n <= 0) return;
    int32_t *pa = perm_a.need((size_t)n);
    int32_t *pb = perm_b.need((size_t)n);
    hipLaunchKernelGGL(iota_i32, dim3(grid_for(n, 256)), dim3(256), 0, st, n, pa);
    auto call = [&](void *t, size_t &sz) {
        return rocprim::radix_sort_pairs(t, sz, kin, kout, (const int32_t *)pa, pb, (size_t)n, 0u,
                                         (unsigned)end_bit, st);
    };
    OTIP_PRIM(call);
    hipLaunchKernelGGL(gather2, dim3(grid_for(n, 256)), dim3(256), 0, st, n, (const int32_t *)pb,
                       v1in, v2in, v1out, v2out);
    OTIP_HIP(hipGetLastError());
}

int64_t unique_u64(hipStream_t st, const uint64_t *in, uint64_t *out, int64_t n, DBuf<char> &tmp,
                   DBuf<unsigned long long> &cnt) {
    if (n <= 0) return 0;
    unsigned long long *c = cnt.need(1);
    auto call = [&](void *t, size_t &sz) {
        return rocprim::unique(t, sz, in, out, c, (size_t)n, rocprim::equal_to<uint64_t>(), st);
    };
    OTIP_PRIM(call);
    unsigned long long h = 0;
    OTIP_HIP(hipMemcpyAsync(&h, c, sizeof(h), hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipStreamSynchronize(st));
    return (int64_t)h;
}

void exclusive_scan_i64(hipStream_t st, const int64_t *in, int64_t *out, int64_t n,
                        DBuf<char> &tmp) {
    if (n <= 0) return;
    auto call = [&](void *t, size_t &sz) {
        return rocprim::exclusive_scan(t, sz, in, out, (int64_t)0, (size_t)n,
                                       rocprim::plus<int64_t>(), st);
    };
    OTIP_PRIM(call);
}

}  // namespace otip
