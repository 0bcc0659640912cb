// axpic_timing.hpp -- optional per-kernel timing shared by the library's
// translation units.  While timing is enabled (axpic_timing_enable), LAUNCH
// brackets the kernel twice: hipExtLaunchKernel attaches a start and a stop
// event to the dispatch itself, and two stream markers are recorded just
// before and after it.  axpic_timing_read takes, per launch, the smaller of
// the two intervals (the markers' contains the kernel, so it bounds the
// dispatch events' from above when those are late to start) and accumulates
// them per kernel name.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

namespace axpic_timing {
// true when timing is on: ev[0], ev[1] are events to attach to the next launch,
// ev[2], ev[3] markers to record around it, all registered under `name`
bool begin(const char* name, hipEvent_t ev[4]);
}  // namespace axpic_timing

#define LAUNCH(NAME, KERNEL, GRID, BLOCK, SHM, STREAM, ...)                                       \
    do {                                                                                           \
        hipEvent_t ev_[4] = {nullptr, nullptr, nullptr, nullptr};                                  \
        if (axpic_timing::begin(NAME, ev_)) {                                                      \
            (void)hipEventRecord(ev_[2], STREAM);                                                  \
            hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, SHM, STREAM, ev_[0], ev_[1], 0, __VA_ARGS__); \
            (void)hipEventRecord(ev_[3], STREAM);                                                  \
        } else {                                                                                   \
            hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHM, STREAM, __VA_ARGS__);                     \
        }                                                                                          \
    } while (0)
