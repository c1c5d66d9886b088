// Row gather used at corpus creation: act[i, :] = vecs[act_word[i], :].
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

}  // namespace

hipError_t launch_gather_rows(const float* vecs, const int32_t* ids, float* out, int64_t nrows, int ldv,
                              hipStream_t s) {
    if (nrows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_rows, dim3(2048), dim3(256), 0, s, vecs, ids, out, nrows, ldv);
    return hipGetLastError();
}

}  // namespace wmd
