// Kernel launch that honours the calling thread's DispatchClock (device
// sources only: it expands to a HIP launch).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "wmd_internal.h"

namespace wmd {

template <typename... P, typename... A>
inline hipError_t launch_kernel(void (*kernel)(P...), dim3 grid, dim3 block, uint32_t lds, hipStream_t s,
                                A... args) {
    DispatchClock& c = dispatch_clock();
    if (c.stop) {
        hipExtLaunchKernelGGL(kernel, grid, block, lds, s, c.start, c.stop, 0u, args...);
        c.start = nullptr;
    } else {
        hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
    }
    return hipGetLastError();
}

}  // namespace wmd
