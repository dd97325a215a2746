// Library-owned stream-ordered memory pool, one per device.  Its release threshold is
// unbounded: memory returned by hipFreeAsync stays mapped for the next allocation instead of
// going back to the driver at every synchronisation (re-mapping gigabytes of HBM per Newton
// iteration costs more than the iteration).  fracture_trim_pool hands the unused part back.
#include <mutex>

#include "common.h"

namespace fr {
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_pool_mu;
hipMemPool_t g_pool[kMaxDevices] = {};
}  // namespace

hipMemPool_t device_pool() {
    int dev = 0;
    FR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) fail(FR_EDEVICE, "memory pool: device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (!g_pool[dev]) {
        hipMemPoolProps props{};
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = dev;
        hipMemPool_t p = nullptr;
        FR_HIP(hipMemPoolCreate(&p, &props));
        uint64_t keep = ~uint64_t(0);
        FR_HIP(hipMemPoolSetAttribute(p, hipMemPoolAttrReleaseThreshold, &keep));
        g_pool[dev] = p;
    }
    return g_pool[dev];
}

void trim_pool() {
    int dev = 0;
    FR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return;
    hipMemPool_t p = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        p = g_pool[dev];
    }
    if (!p) return;
    FR_HIP(hipDeviceSynchronize());
    FR_HIP(hipMemPoolTrimTo(p, 0));
}

}  // namespace fr
