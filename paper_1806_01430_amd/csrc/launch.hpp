// Kernel launch helper: plain launch, or -- when the executor has armed a
// pair of timing events for the next launch -- a launch whose dispatch packet
// itself records the start and stop timestamps (hipExtLaunchKernel), so the
// measured interval is the kernel alone, without marker-packet overhead.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

namespace ofl {
namespace k {

struct ArmedEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};

inline ArmedEvents &armed_events() {
    thread_local ArmedEvents ev;
    return ev;
}

// Arm the events for the next launch on this thread (consumed by it).
inline void arm_launch_events(hipEvent_t start, hipEvent_t stop) {
    armed_events().start = start;
    armed_events().stop = stop;
}

template <typename F, typename... Args>
hipError_t launch(F kernel, const dim3 &grid, const dim3 &block, uint32_t shmem, hipStream_t s, Args... args) {
    ArmedEvents &ev = armed_events();
    if (ev.start || ev.stop) {
        hipEvent_t a = ev.start, b = ev.stop;
        ev.start = ev.stop = nullptr;
        hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, a, b, 0, args...);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
    }
    return hipGetLastError();
}

}  // namespace k
}  // namespace ofl
