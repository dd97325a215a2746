// Optional per-kernel timing with HIP events recorded on the launch stream, plus the
// algorithmic bytes each launch must move (for the roofline).  Off unless enabled.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace fr {

bool prof_enabled();
void prof_enable(bool on);
// Records an event pair around the launches issued while the scope is alive.
struct ProfScope {
    int idx = -1;
    hipStream_t s = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(const char* name, hipStream_t stream, double bytes);
    ~ProfScope();
};
int prof_count();
// Sums the recorded intervals of entry i (synchronises their events).
bool prof_read(int i, const char** name, int64_t* launches, double* ms, double* bytes);

}  // namespace fr
