// Corpus preparation kernels: row norms, BF16 copies, per-document
// normalisation of the histogram weights (columns of c sum to one, Sec. 4).
#include "wmd_internal.h"

namespace wmd {

namespace {

// |row|^2 in FP32, sequential over the padded row (padding is zero).
__global__ void k_row_norms(const float* __restrict__ rows, int64_t nrows, int ldv,
                            float* __restrict__ norms) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    const float4* p = reinterpret_cast<const float4*>(rows + i * ldv);
    float s = 0.f;
    for (int k = 0; k < ldv / 4; ++k) {
        float4 v = p[k];
        s = fmaf(v.x, v.x, s);
        s = fmaf(v.y, v.y, s);
        s = fmaf(v.z, v.z, s);
        s = fmaf(v.w, v.w, s);
    }
    norms[i] = s;
}

// Round-to-nearest-even FP32 -> BF16 (finite inputs).
__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t h) {
    return __uint_as_float((uint32_t)h << 16);
}

// BF16 copy of each row plus |bf16 row|^2 (so the GEMM expansion is
// consistent with the rounded operands).
__global__ void k_rows_bf16(const float* __restrict__ src, uint16_t* __restrict__ dst,
                            float* __restrict__ norms, int64_t nrows, int ldv) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    const float* p = src + i * ldv;
    uint16_t* q = dst + i * ldv;
    float s = 0.f;
    for (int k = 0; k < ldv; ++k) {
        uint16_t h = to_bf16(p[k]);
        q[k] = h;
        float f = from_bf16(h);
        s = fmaf(f, f, s);
    }
    norms[i] = s;
}

// c_ij = w_ij / sum_i w_ij, the sum in FP64, the quotient rounded once to FP32.
// May run in place (cw == w): each entry is read before it is overwritten.
__global__ void k_doc_normalise(const int32_t* __restrict__ ptr, const float* w, float* cw, int64_t N) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    int b = ptr[j], e = ptr[j + 1];
    double s = 0.0;
    for (int p = b; p < e; ++p) s += (double)w[p];
    for (int p = b; p < e; ++p) cw[p] = (float)((double)w[p] / s);
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_prep_norms(const float* rows, int64_t nrows, int ldv, float* norms, hipStream_t s) {
    if (nrows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_row_norms, dim3(blocks_for(nrows, 256)), dim3(256), 0, s, rows, nrows, ldv,
                       norms);
    return hipGetLastError();
}

hipError_t launch_prep_bf16(const float* src, uint16_t* dst, float* norms, int64_t nrows, int ldv,
                            hipStream_t s) {
    if (nrows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rows_bf16, dim3(blocks_for(nrows, 256)), dim3(256), 0, s, src, dst, norms,
                       nrows, ldv);
    return hipGetLastError();
}

hipError_t launch_prep_docs(const int32_t* ptr, const float* w, float* cw, int64_t N, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_doc_normalise, dim3(blocks_for(N, 256)), dim3(256), 0, s, ptr, w, cw, N);
    return hipGetLastError();
}

}  // namespace wmd
