// axpic_timing.hpp -- optional per-kernel timing shared by the library's
// translation units.  While timing is enabled (axpic_timing_enable), LAUNCH
// attaches a start and a stop event to the kernel dispatch
// (hipExtLaunchKernel records them when the dispatch begins and ends on the
// launch stream, so the interval is the kernel's own duration);
// axpic_timing_read accumulates them per kernel name.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

namespace axpic_timing {
// true when timing is on: *a and *b are events to attach to the next launch,
// already registered under `name`
bool begin(const char* name, hipEvent_t* a, hipEvent_t* b);
}  // namespace axpic_timing

#define LAUNCH(NAME, KERNEL, GRID, BLOCK, SHM, STREAM, ...)                                       \
    do {                                                                                           \
        hipEvent_t ta_ = nullptr, tb_ = nullptr;                                                   \
        if (axpic_timing::begin(NAME, &ta_, &tb_))                                                 \
            hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, SHM, STREAM, ta_, tb_, 0, __VA_ARGS__);     \
        else                                                                                       \
            hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHM, STREAM, __VA_ARGS__);                     \
    } while (0)
