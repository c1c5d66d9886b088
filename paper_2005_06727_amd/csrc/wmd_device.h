// Device-side helpers shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace wmd {

// Global memory reached through a pointer that was itself loaded from device
// memory (the per-query record): the compiler cannot prove its address space
// and would emit generic (flat) accesses, whose completion it cannot track
// against the other loads, so it would wait for every load in flight before
// each use.  Accesses through gmem() are plain global loads and stores.
#define WMD_GLOBAL __attribute__((address_space(1)))

template <typename T>
__device__ __forceinline__ WMD_GLOBAL T* gmem(T* p) {
    return (WMD_GLOBAL T*)p;
}

typedef float gv4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float4 ld4(WMD_GLOBAL const float* p) {
    const gv4f v = *(WMD_GLOBAL const gv4f*)p;
    return make_float4(v.x, v.y, v.z, v.w);
}

}  // namespace wmd
