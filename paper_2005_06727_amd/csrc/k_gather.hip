// Row gather used at corpus creation, and the parameter upload of a query
// call (small parameter blocks travel as kernel arguments, so a call needs no
// host-to-device copy and no pinned staging buffer).
#include <algorithm>
#include <cstring>

#include "wmd_internal.h"

namespace wmd {

namespace {

__global__ void k_gather_rows(const float* __restrict__ vecs, const int32_t* __restrict__ ids,
                              float* __restrict__ out, int64_t nrows, int ldv) {
    const int64_t total = nrows * (ldv / 4);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / (ldv / 4);
        const int c = (int)(e % (ldv / 4));
        reinterpret_cast<float4*>(out + r * ldv)[c] =
            reinterpret_cast<const float4*>(vecs + (int64_t)ids[r] * ldv)[c];
    }
}

constexpr int kBlobWords = kUploadChunkBytes / 4;

struct Blob {
    uint32_t w[kBlobWords];
};

__global__ __launch_bounds__(256) void k_upload(Blob b, uint32_t* __restrict__ dst, int nwords) {
    for (int i = threadIdx.x; i < nwords; i += blockDim.x) dst[i] = b.w[i];
}

}  // namespace

hipError_t launch_gather_rows(const float* vecs, const int32_t* ids, float* out, int64_t nrows, int ldv,
                              hipStream_t s) {
    if (nrows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_rows, dim3(2048), dim3(256), 0, s, vecs, ids, out, nrows, ldv);
    return hipGetLastError();
}

hipError_t launch_upload(const void* src, size_t bytes, void* dst, hipStream_t s) {
    if (bytes % 4 != 0 || bytes > (size_t)kUploadMaxBytes) return hipErrorInvalidValue;
    const char* p = static_cast<const char*>(src);
    char* d = static_cast<char*>(dst);
    for (size_t off = 0; off < bytes; off += kUploadChunkBytes) {
        const size_t n = std::min<size_t>(kUploadChunkBytes, bytes - off);
        Blob b;
        std::memcpy(b.w, p + off, n);
        hipLaunchKernelGGL(k_upload, dim3(1), dim3(256), 0, s, b, reinterpret_cast<uint32_t*>(d + off),
                           (int)(n / 4));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace wmd
