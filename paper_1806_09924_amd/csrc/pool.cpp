// Device memory for the library.
//
// Blocks come from a library-owned stream-ordered pool per device whose release threshold
// is unbounded, and a freed block goes to a cache keyed by (device, stream, size) from
// which a later allocation on the same stream takes it back without any runtime call.  In
// a steady state (every Newton call of a loading step allocates the same sizes) setup and
// solve then make no allocation calls at all; the runtime's own free path can stall the
// host for a whole device drain.  Reuse on the stream of the free is safe by stream order,
// the same contract as the stream-ordered allocator's.
#include <map>
#include <mutex>
#include <unordered_map>
#include <utility>

#include "common.h"

namespace fr {
namespace {

constexpr int kMaxDevices = 64;

struct Cache {
    std::mutex mu;
    hipMemPool_t pool[kMaxDevices] = {};
    // (device, stream) -> size -> cached blocks
    std::map<std::pair<int, hipStream_t>, std::multimap<size_t, void*>> free_blocks;
    std::unordered_map<void*, std::pair<size_t, int>> size_of;   // every block we made: bytes, device
};

Cache& cache() {
    static Cache* c = new Cache;   // process lifetime: no destruction-order hazards at exit
    return *c;
}

int current_device() {
    int dev = 0;
    FR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) fail(FR_EDEVICE, "memory pool: device ordinal out of range");
    return dev;
}

// 512 B granularity below 1 MiB, 1 MiB above
size_t round_bytes(size_t b) {
    if (b < (size_t(1) << 20)) return (std::max<size_t>(b, 1) + 511) & ~size_t(511);
    return (b + (size_t(1) << 20) - 1) & ~((size_t(1) << 20) - 1);
}

hipMemPool_t pool_locked(Cache& c, int dev) {
    if (!c.pool[dev]) {
        hipMemPoolProps props{};
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = dev;
        hipMemPool_t p = nullptr;
        FR_HIP(hipMemPoolCreate(&p, &props));
        uint64_t keep = ~uint64_t(0);
        FR_HIP(hipMemPoolSetAttribute(p, hipMemPoolAttrReleaseThreshold, &keep));
        c.pool[dev] = p;
    }
    return c.pool[dev];
}

// Frees every cached block of device `dev` and, with `s_only`, only those cached for
// stream s.  The blocks' last users must have finished (the caller synchronised).
void release_locked(Cache& c, int dev, bool s_only, hipStream_t s) {
    for (auto it = c.free_blocks.begin(); it != c.free_blocks.end();) {
        if (it->first.first != dev || (s_only && it->first.second != s)) {
            ++it;
            continue;
        }
        for (auto& kv : it->second) {
            (void)hipFreeAsync(kv.second, nullptr);
            c.size_of.erase(kv.second);
        }
        it = c.free_blocks.erase(it);
    }
}

}  // namespace

void* dev_alloc(size_t bytes, hipStream_t s) {
    Cache& c = cache();
    const int dev = current_device();
    const size_t rb = round_bytes(bytes);
    hipMemPool_t pool = nullptr;
    {
        std::lock_guard<std::mutex> lk(c.mu);
        auto fb = c.free_blocks.find({dev, s});
        if (fb != c.free_blocks.end()) {
            auto b = fb->second.lower_bound(rb);
            if (b != fb->second.end() && b->first <= rb + rb / 8) {
                void* p = b->second;
                fb->second.erase(b);
                return p;
            }
        }
        pool = pool_locked(c, dev);
    }
    void* p = nullptr;
    hipError_t e = hipMallocFromPoolAsync(&p, rb, pool, s);
    if (e == hipErrorOutOfMemory) {
        // hand the cached blocks of this device back and try once more
        (void)hipGetLastError();
        FR_HIP(hipDeviceSynchronize());
        {
            std::lock_guard<std::mutex> lk(c.mu);
            release_locked(c, dev, false, nullptr);
        }
        FR_HIP(hipDeviceSynchronize());
        FR_HIP(hipMemPoolTrimTo(pool, 0));
        e = hipMallocFromPoolAsync(&p, rb, pool, s);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(e == hipErrorOutOfMemory ? FR_ENOMEM : FR_EDEVICE,
             std::string("device allocation of ") + std::to_string(rb) + " bytes: " + hipGetErrorString(e));
    }
    std::lock_guard<std::mutex> lk(c.mu);
    c.size_of[p] = {rb, dev};
    return p;
}

void dev_free(void* p, hipStream_t s) {
    if (!p) return;
    Cache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.size_of.find(p);
    if (it == c.size_of.end()) {
        (void)hipFreeAsync(p, s);
        return;
    }
    c.free_blocks[{it->second.second, s}].insert({it->second.first, p});
}

void forget_stream(hipStream_t s) {
    Cache& c = cache();
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return;
    (void)hipStreamSynchronize(s);
    {
        std::lock_guard<std::mutex> lk(c.mu);
        release_locked(c, dev, true, s);
    }
    (void)hipDeviceSynchronize();
}

void trim_pool() {
    Cache& c = cache();
    const int dev = current_device();
    FR_HIP(hipDeviceSynchronize());
    hipMemPool_t pool = nullptr;
    {
        std::lock_guard<std::mutex> lk(c.mu);
        release_locked(c, dev, false, nullptr);
        pool = c.pool[dev];
    }
    FR_HIP(hipDeviceSynchronize());
    if (pool) FR_HIP(hipMemPoolTrimTo(pool, 0));
}

}  // namespace fr
