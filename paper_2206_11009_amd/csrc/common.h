// Internal declarations shared by the otip HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <stdexcept>
#include <string>
#include <vector>

namespace otip {

// Thrown inside the library, turned into a status code at the C boundary.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &msg) : std::runtime_error(msg), code(c) {}
};

#define OTIP_HIP(call)                                                                        \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            throw ::otip::Error(3, std::string(#call) + ": " + hipGetErrorString(e_) + " (" + \
                                     __FILE__ + ":" + std::to_string(__LINE__) + ")");        \
    } while (0)

#define OTIP_CHECK(cond, code, msg)                          \
    do {                                                     \
        if (!(cond)) throw ::otip::Error((code), (msg));     \
    } while (0)

// Debug aid: with OTIP_POISON set in the environment every buffer is filled
// with 0xFF bytes (NaN doubles, -1 integers) when it is allocated and again at
// its first use in each solve (a new poison epoch per solve and host thread),
// so that a read of memory the current problem never wrote gives the same
// result on every machine and in every schedule.
inline bool poison_allocations() {
    static const bool on = std::getenv("OTIP_POISON") != nullptr;
    return on;
}
inline uint64_t &poison_epoch() {
    static thread_local uint64_t e = 1;
    return e;
}

// Growable device allocation owned by a context.  Contents are not preserved
// across growth.
template <typename T>
struct DBuf {
    T *ptr = nullptr;
    size_t cap = 0;
    uint64_t epoch_ = 0;  // poison epoch of the last fill (debug aid)
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    ~DBuf() { release(); }
    void release() {
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        cap = 0;
    }
    T *need(size_t n) {
        if (n == 0) n = 1;
        if (n > cap) {
            release();
            size_t c = n + n / 4;
            hipError_t e = hipMalloc(&ptr, c * sizeof(T));
            if (e != hipSuccess) {
                ptr = nullptr;
                throw Error(2, "device allocation of " + std::to_string(c * sizeof(T)) +
                                   " bytes failed: " + hipGetErrorString(e));
            }
            cap = c;
            epoch_ = 0;
        }
        if (poison_allocations() && epoch_ != poison_epoch()) {
            if (hipDeviceSynchronize() != hipSuccess || hipMemset(ptr, 0xFF, cap * sizeof(T)) != hipSuccess ||
                hipDeviceSynchronize() != hipSuccess)
                throw Error(3, "poisoning a buffer failed");
            epoch_ = poison_epoch();
        }
        return ptr;
    }
    T *get() const { return ptr; }
};

// Event timing of individual kernel launches on their stream (opt-in).  A
// caller that makes many calls (CG solves, pricing calls) may sample them: it
// opens each call with begin_call(), and only the first of every `stride`
// calls since the last reset() records events.
struct LaunchTimer {
    bool on = false;
    bool active = true;
    int stride = 1;
    int64_t calls = 0;
    int64_t launches = 0;
    double ms = 0.0, work = 0.0;
    std::vector<hipEvent_t> ev;
    std::vector<double> pending_work;
    size_t used = 0;
    ~LaunchTimer() {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
    void begin_call() { active = calls++ % std::max(1, stride) == 0; }
    // record the start event of a launch carrying `w` units of work
    void start(hipStream_t st, double w) {
        if (!on || !active) return;
        if (used + 2 > ev.size()) {
            for (int k = 0; k < 64; ++k) {
                hipEvent_t e;
                if (hipEventCreate(&e) != hipSuccess) throw Error(3, "hipEventCreate failed");
                ev.push_back(e);
            }
        }
        (void)hipEventRecord(ev[used], st);
        pending_work.push_back(w);
    }
    void stop(hipStream_t st) {
        if (!on || !active) return;
        (void)hipEventRecord(ev[used + 1], st);
        used += 2;
    }
    // events for one launch of `w` units made with hipExtLaunchKernelGGL, which
    // records them at the dispatch's own start and end; null when timing is off
    void arm(double w, hipEvent_t *a, hipEvent_t *b) {
        *a = *b = nullptr;
        if (!on || !active) return;
        if (used + 2 > ev.size()) {
            for (int k = 0; k < 64; ++k) {
                hipEvent_t e;
                if (hipEventCreate(&e) != hipSuccess) throw Error(3, "hipEventCreate failed");
                ev.push_back(e);
            }
        }
        *a = ev[used];
        *b = ev[used + 1];
        used += 2;
        pending_work.push_back(w);
    }
    // replace the units of work of the k-th launch armed since the last
    // collect (work known only once the launch has run)
    void set_pending(size_t k, double w) {
        if (k < pending_work.size()) pending_work[k] = w;
    }
    void reset() {
        active = true;
        calls = 0;
        launches = 0;
        ms = work = 0.0;
        used = 0;
        pending_work.clear();
    }
    // after the stream has been synchronised; only the first `keep` launches
    // armed since the last collect count (launches that found their work
    // already done are dropped from both the time and the work)
    void collect(size_t keep = SIZE_MAX) {
        if (!on) return;
        const size_t lim = keep >= used / 2 ? used : 2 * keep;
        for (size_t k = 0; k + 1 < lim; k += 2) {
            float t = 0.0f;
            if (hipEventElapsedTime(&t, ev[k], ev[k + 1]) == hipSuccess) {
                ms += t;
                work += pending_work[k / 2];
                ++launches;
            }
        }
        used = 0;
        pending_work.clear();
    }
};

inline unsigned grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 0x7fffffff) g = 0x7fffffff;
    return (unsigned)g;
}

constexpr int kWave = 64;

// ---------------------------------------------------------------- device helpers
__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_sum_i(int v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block-wide fixed-order sum of one double per thread (blockDim.x multiple of
// 64, <= 1024).  Result valid in every thread.
__device__ __forceinline__ double block_sum(double v, double *lds /* >= 16 */) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < nw; ++k) t += lds[k];
    return t;
}

// Ordered 64-bit key of a double: key(a) < key(b)  <=>  a < b (no NaNs).
__device__ __forceinline__ uint64_t dkey(double r) {
    uint64_t u = (uint64_t)__double_as_longlong(r);
    return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double dkey_inv(uint64_t k) {
    uint64_t u = (k & 0x8000000000000000ull) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)u);
}

}  // namespace otip
