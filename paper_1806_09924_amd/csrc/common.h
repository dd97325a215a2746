// Shared host/device helpers of the fracture library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/fracture.h"

namespace fr {

constexpr int kWave = 64;

// Error carried from internal code to the ABI boundary.
struct Error : std::runtime_error {
    fr_status status;
    Error(fr_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

[[noreturn]] inline void fail(fr_status s, const std::string& m) { throw Error(s, m); }

// The worse of two statuses (what a call over several instances or steps returns):
// FR_OK < FR_ENOCONV < FR_ECYCLE < FR_EBREAKDOWN < FR_ENAN < every argument / device error.
inline int status_rank(fr_status s) {
    switch (s) {
        case FR_OK: return 0;
        case FR_ENOCONV: return 1;
        case FR_ECYCLE: return 2;
        case FR_EBREAKDOWN: return 3;
        case FR_ENAN: return 4;
        default: return 5;
    }
}
inline fr_status worse_status(fr_status a, fr_status b) { return status_rank(b) > status_rank(a) ? b : a; }

#define FR_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            ::fr::fail(e_ == hipErrorOutOfMemory ? FR_ENOMEM : FR_EDEVICE,             \
                       std::string(#call) + ": " + hipGetErrorString(e_));             \
    } while (0)

#define FR_LAUNCH_CHECK() FR_HIP(hipGetLastError())

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Device memory of the current device, stream ordered: a block freed on stream s is reused
// by later allocations on s.  trim_pool hands every cached block and the pool's unused
// memory back to the driver (synchronises the device); forget_stream does so for the
// blocks cached for s (synchronises s), before s is destroyed.
void* dev_alloc(size_t bytes, hipStream_t s);
void dev_free(void* p, hipStream_t s);
void trim_pool();
void forget_stream(hipStream_t s);
// Installs the caller's allocator (both NULL: the library's pool again).
void set_allocator(fr_alloc_fn alloc, fr_free_fn dealloc, void* ctx);

// Stream-ordered device buffer.  Released on the stream it was allocated on.
template <typename T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    hipStream_t s = nullptr;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    DBuf(DBuf&& o) noexcept : p(o.p), n(o.n), s(o.s) { o.p = nullptr; o.n = 0; }
    DBuf& operator=(DBuf&& o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; s = o.s; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DBuf() { release(); }
    void alloc(size_t count, hipStream_t stream) {
        release();
        s = stream;
        n = count;
        if (count) p = static_cast<T*>(dev_alloc(count * sizeof(T), stream));
    }
    // Grows (never shrinks); contents are not preserved.
    void reserve(size_t count, hipStream_t stream) {
        if (count > n || p == nullptr) alloc(count, stream);
    }
    void release() {
        if (p) { dev_free(p, s); p = nullptr; n = 0; }
    }
    void upload(const T* h, size_t count, hipStream_t stream) {
        if (count) FR_HIP(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, stream));
    }
    void upload(const std::vector<T>& v, hipStream_t stream) {
        alloc(v.size(), stream);
        upload(v.data(), v.size(), stream);
    }
    void zero(hipStream_t stream) {
        if (n) FR_HIP(hipMemsetAsync(p, 0, n * sizeof(T), stream));
    }
};

// Waits until everything enqueued on s so far has finished, by polling an event: the setup
// reads many small results back (sizes, counts), and a blocking synchronise can take tens of
// microseconds to wake the host after the device is done.
void stream_wait(hipStream_t s);

template <typename T>
std::vector<T> download(const T* d, size_t n, hipStream_t s) {
    std::vector<T> h(n);
    if (n) {
        FR_HIP(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, s));
        stream_wait(s);
    }
    return h;
}

template <typename T>
T download1(const T* d, hipStream_t s) {
    T v{};
    FR_HIP(hipMemcpyAsync(&v, d, sizeof(T), hipMemcpyDeviceToHost, s));
    stream_wait(s);
    return v;
}

// ---- device helpers -------------------------------------------------------------------

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ inline float wave_sum(float v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

__device__ inline double wave_min(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}

__device__ inline int wave_sum_int(int v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Block-wide sum in a fixed order (deterministic).  blockDim.x multiple of 64, <= 1024.
__device__ inline double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
    if (l == 0) sh[w] = v;
    __syncthreads();
    const int nw = blockDim.x / kWave;
    double t = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < nw; ++i) t += sh[i];
        sh[0] = t;
    }
    __syncthreads();
    t = sh[0];
    __syncthreads();
    return t;
}

// 32-bit integer hash (a published finaliser: the "lowbias32" mix by C. Wellons).
__host__ __device__ inline uint32_t hash32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

}  // namespace fr
