// k nearest documents of a query (retrieval with WMD, Sec. 3: the query's
// distances to all N documents, then the k smallest).
//
// Keys are (distance, document index) pairs in lexicographic order, so ties
// are broken by the smaller index and the result is unique.  A distance is
// non-negative, so its IEEE bit pattern orders like its value (-0 is folded
// into +0; a NaN sorts after +inf).  Pass 1 sorts tiles of 4096 keys in LDS
// (bitonic network) and keeps each tile's first k; the survivors are tiled
// again until one tile holds them all, whose first k are the answer.
#include <cstdint>

#include "wmd_internal.h"

namespace wmd {

namespace {

constexpr int kTile = 4096;
constexpr int kThreads = 512;

__device__ __forceinline__ bool key_less(uint64_t ka, uint32_t ia, uint64_t kb, uint32_t ib) {
    return ka < kb || (ka == kb && ia < ib);
}

__device__ __forceinline__ uint64_t dist_key(double d) {
    return (uint64_t)__double_as_longlong(d + 0.0);   // -0 -> +0
}

// in: either distances (keys made from dist, index = position) or (key, index)
// pairs from a previous pass; out: the first k of every tile, as pairs, or as
// (index, distance) for the last pass.
__global__ __launch_bounds__(kThreads) void k_topk_tiles(const double* __restrict__ dist,
                                                         const uint64_t* __restrict__ in_key,
                                                         const uint32_t* __restrict__ in_idx, int64_t n, int k,
                                                         uint64_t* __restrict__ out_key,
                                                         uint32_t* __restrict__ out_idx, int32_t* __restrict__ res_idx,
                                                         double* __restrict__ res_dist) {
    __shared__ uint64_t sk[kTile];
    __shared__ uint32_t si[kTile];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int i = threadIdx.x; i < kTile; i += kThreads) {
        const int64_t g = base + i;
        if (g < n) {
            if (dist) {
                sk[i] = dist_key(dist[g]);
                si[i] = (uint32_t)g;
            } else {
                sk[i] = in_key[g];
                si[i] = in_idx[g];
            }
        } else {
            sk[i] = UINT64_MAX;
            si[i] = UINT32_MAX;
        }
    }
    __syncthreads();
    // bitonic sort, ascending
    for (int size = 2; size <= kTile; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < kTile / 2; t += kThreads) {
                const int lo = 2 * t - (t & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const uint64_t ka = sk[lo], kb = sk[hi];
                const uint32_t ia = si[lo], ib = si[hi];
                if (key_less(kb, ib, ka, ia) == up) {
                    sk[lo] = kb;
                    sk[hi] = ka;
                    si[lo] = ib;
                    si[hi] = ia;
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < k; i += kThreads) {
        if (res_idx) {
            res_idx[i] = (int32_t)si[i];
            res_dist[i] = __longlong_as_double((long long)sk[i]);
        } else {
            out_key[(int64_t)blockIdx.x * k + i] = sk[i];
            out_idx[(int64_t)blockIdx.x * k + i] = si[i];
        }
    }
}

}  // namespace

size_t topk_scratch_bytes(int64_t n, int k) {
    const int64_t tiles = (n + kTile - 1) / kTile;
    const int64_t cand = tiles * k;
    return 2 * (size_t)cand * (sizeof(uint64_t) + sizeof(uint32_t)) + 256;
}

hipError_t launch_topk(const double* dist, int64_t n, int k, void* scratch, size_t scratch_bytes, int32_t* res_idx,
                       double* res_dist, hipStream_t s) {
    if (n <= 0 || k < 1 || k > kMaxTopK || k > n) return hipErrorInvalidValue;
    if (scratch_bytes < topk_scratch_bytes(n, k)) return hipErrorInvalidValue;
    const int64_t tiles0 = (n + kTile - 1) / kTile;
    const int64_t cap = tiles0 * k;
    uint64_t* key[2] = {static_cast<uint64_t*>(scratch), static_cast<uint64_t*>(scratch) + cap};
    uint32_t* idx[2] = {reinterpret_cast<uint32_t*>(key[1] + cap), reinterpret_cast<uint32_t*>(key[1] + cap) + cap};
    int64_t cur = n;
    int side = -1;   // -1: the distances themselves
    for (;;) {
        const int64_t tiles = (cur + kTile - 1) / kTile;
        const bool last = tiles == 1;
        const double* d = side < 0 ? dist : nullptr;
        const uint64_t* ik = side < 0 ? nullptr : key[side];
        const uint32_t* ii = side < 0 ? nullptr : idx[side];
        const int o = side < 0 ? 0 : side ^ 1;
        hipLaunchKernelGGL(k_topk_tiles, dim3((unsigned)tiles), dim3(kThreads), 0, s, d, ik, ii, cur, k,
                           last ? nullptr : key[o], last ? nullptr : idx[o], last ? res_idx : nullptr,
                           last ? res_dist : nullptr);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || last) return e;
        cur = tiles * k;   // k <= kTile / 2, so every pass at least halves the count
        side = o;
    }
}

}  // namespace wmd
