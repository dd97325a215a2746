// Device memory for the library.
//
// By default blocks come from a library-owned stream-ordered pool per device whose release threshold
// is unbounded, and a freed block goes to a cache keyed by (device, stream, size) from
// which a later allocation on the same stream takes it back without any runtime call.  In
// a steady state (every Newton call of a loading step allocates the same sizes) setup and
// solve then make no allocation calls at all; the runtime's own free path can stall the
// host for a whole device drain.  Reuse on the stream of the free is safe by stream order,
// the same contract as the stream-ordered allocator's.
//
// A caller may install an allocator of its own (fracture_set_allocator, e.g. PyTorch's caching
// allocator): new blocks then come from it and go back to it when freed, with the stream of
// the free; the library keeps no cache of them.  Every block remembers the allocator that made
// it, so changing the allocator while objects are alive is safe.
#include <map>
#include <mutex>
#include <unordered_map>
#include <utility>

#include "common.h"

namespace fr {
namespace {

constexpr int kMaxDevices = 64;

struct Hook {
    fr_alloc_fn alloc = nullptr;
    fr_free_fn dealloc = nullptr;
    void* ctx = nullptr;
};

struct Block {
    size_t bytes = 0;
    int dev = 0;
    Hook hook;                 // the caller's allocator that made it (alloc == nullptr: the pool)
};

struct Cache {
    std::mutex mu;
    hipMemPool_t pool[kMaxDevices] = {};
    Hook hook;                 // installed allocator (alloc == nullptr: the library's pool)
    // (device, stream) -> size -> cached blocks (pool blocks only)
    std::map<std::pair<int, hipStream_t>, std::multimap<size_t, void*>> free_blocks;
    std::unordered_map<void*, Block> blocks;   // every block handed out
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
            c.blocks.erase(kv.second);
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
    Hook hook;
    {
        std::lock_guard<std::mutex> lk(c.mu);
        hook = c.hook;
    }
    if (hook.alloc) {
        // the caller's allocator, called without the lock held
        void* p = hook.alloc(rb, dev, reinterpret_cast<void*>(s), hook.ctx);
        if (!p) fail(FR_ENOMEM, std::string("installed allocator returned NULL for ") + std::to_string(rb) + " bytes");
        std::lock_guard<std::mutex> lk(c.mu);
        c.blocks[p] = Block{rb, dev, hook};
        return p;
    }
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
    c.blocks[p] = Block{rb, dev, Hook{}};
    return p;
}

void dev_free(void* p, hipStream_t s) {
    if (!p) return;
    Cache& c = cache();
    Block b;
    {
        std::lock_guard<std::mutex> lk(c.mu);
        auto it = c.blocks.find(p);
        if (it == c.blocks.end()) {
            (void)hipFreeAsync(p, s);
            return;
        }
        if (!it->second.hook.alloc) {
            c.free_blocks[{it->second.dev, s}].insert({it->second.bytes, p});
            return;
        }
        b = it->second;
        c.blocks.erase(it);
    }
    b.hook.dealloc(p, b.bytes, b.dev, reinterpret_cast<void*>(s), b.hook.ctx);
}

void set_allocator(fr_alloc_fn alloc, fr_free_fn dealloc, void* ctx) {
    Cache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    c.hook = Hook{alloc, dealloc, ctx};
}

namespace {
// one event per host thread (the phase-field setup runs in a thread of its own)
struct WaitEvent {
    hipEvent_t e = nullptr;
    ~WaitEvent() {
        if (e) (void)hipEventDestroy(e);
    }
};
}  // namespace

void stream_wait(hipStream_t s) {
    thread_local WaitEvent w;
    if (!w.e) FR_HIP(hipEventCreateWithFlags(&w.e, hipEventDisableTiming));
    FR_HIP(hipEventRecord(w.e, s));
    for (;;) {
        const hipError_t q = hipEventQuery(w.e);
        if (q == hipSuccess) break;
        if (q != hipErrorNotReady) FR_HIP(q);
    }
    // the not-ready answers must not linger as the thread's last error (launch checks read it)
    (void)hipGetLastError();
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
