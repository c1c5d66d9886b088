// k nearest documents of a query (retrieval with WMD, Sec. 3: the query's
// distances to all N documents, then the k smallest).
//
// Keys are (distance, document index) pairs in lexicographic order, so ties
// are broken by the smaller index and the result is unique.  A distance is
// non-negative, so its IEEE bit pattern orders like its value (-0 is folded
// into +0; a NaN sorts after +inf).
//
// Each workgroup takes a tile of 8192 keys into LDS and selects its first k:
// eight 8-bit radix passes (most significant first) find the k-th smallest
// key T and how many of the keys equal to T belong to the answer; one more
// pass gathers every key below T and, in index order, that many keys equal
// to T; a bitonic sort of those k pairs orders them.  The tiles' survivors
// are tiled again until one tile holds them all, whose first k are the
// answer.
#include <cstdint>

#include "wmd_internal.h"

namespace wmd {

namespace {


__device__ __forceinline__ bool key_less(uint64_t ka, uint32_t ia, uint64_t kb, uint32_t ib) {
    return ka < kb || (ka == kb && ia < ib);
}

__device__ __forceinline__ uint64_t dist_key(double d) {
    return (uint64_t)__double_as_longlong(d + 0.0);   // -0 -> +0
}

constexpr int kSelThreads = 1024;
constexpr int kTile = 8192;    // keys per workgroup (in LDS)

// inclusive prefix sum over the 64 lanes of a wave
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}

// The first k (by key, then index) of tile blockIdx.x of the input: keys
// [kTile * b, kTile * b + kTile) of either the distances (index = position)
// or the (key, index) pairs of a previous pass.  Output: the k pairs in order,
// to res (the last pass: index and distance) or to out at [k * b, k * b + k);
// a tile with fewer than k keys is padded with (UINT64_MAX, UINT32_MAX).
// Among equal keys, position order is index order here: every pass's tiles
// cover consecutive input, and every tile's output is sorted.
__global__ __launch_bounds__(kSelThreads) void k_topk_select(const double* __restrict__ dist,
                                                             const uint64_t* __restrict__ in_key,
                                                             const uint32_t* __restrict__ in_idx, int64_t n, int k,
                                                             uint64_t* __restrict__ out_key,
                                                             uint32_t* __restrict__ out_idx,
                                                             int32_t* __restrict__ res_idx,
                                                             double* __restrict__ res_dist) {
    __shared__ uint64_t lk[kTile];
    __shared__ uint32_t li[kTile];
    __shared__ uint32_t hist[256];
    __shared__ uint64_t ck[kMaxTopK];      // the selected pairs, then sorted
    __shared__ uint32_t ci[kMaxTopK];
    __shared__ uint32_t s_digit, s_before, s_inbin, s_nless, s_wave[kSelThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    const int tn = (int)(n - base < kTile ? n - base : kTile);   // keys in this tile
    for (int i = tid; i < tn; i += kSelThreads) {
        if (dist) {
            lk[i] = dist_key(dist[base + i]);
            li[i] = (uint32_t)(base + i);
        } else {
            lk[i] = in_key[base + i];
            li[i] = in_idx[base + i];
        }
    }
    const int kk = k < tn ? k : tn;                                 // keys this tile selects
    // radix passes: the rank-th smallest key (1-based) among those matching prefix
    uint64_t prefix = 0, mask = 0;
    uint32_t rank = (uint32_t)kk, inbin = 0;
    for (int shift = 56; shift >= 0; shift -= 8) {
        for (int b = tid; b < 256; b += kSelThreads) hist[b] = 0;
        __syncthreads();
        for (int i = tid; i < tn; i += kSelThreads) {
            const uint64_t key = lk[i];
            if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (wave == 0) {
            const uint32_t c[4] = {hist[4 * lane], hist[4 * lane + 1], hist[4 * lane + 2], hist[4 * lane + 3]};
            const uint32_t sum = c[0] + c[1] + c[2] + c[3];
            uint32_t before = wave_incl_scan(sum) - sum;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (before < rank && rank <= before + c[j]) {   // exactly one bin holds the rank-th key
                    s_digit = 4 * lane + j;
                    s_before = before;
                    s_inbin = c[j];
                }
                before += c[j];
            }
        }
        __syncthreads();
        prefix |= (uint64_t)s_digit << shift;
        mask |= (uint64_t)255 << shift;
        rank -= s_before;
        inbin = s_inbin;
        __syncthreads();
    }
    // T = prefix: the keys below T are in the answer, and the first `rank` keys
    // equal to T (of `inbin`) in position order
    const uint64_t T = prefix;
    const uint32_t need_eq = rank, nless = (uint32_t)kk - need_eq;
    const bool all_eq = inbin == need_eq;   // every key equal to T is in the answer (no tie at the boundary)
    if (tid == 0) s_nless = 0;
    __syncthreads();
    for (int i = tid; i < tn; i += kSelThreads) {
        const uint64_t key = lk[i];
        if (key < T || (all_eq && key == T)) {   // exactly kk keys when all_eq, else nless
            const uint32_t slot = atomicAdd(&s_nless, 1u);
            if (slot < (uint32_t)kk) {   // always true by the counts; keeps the LDS writes in bounds
                ck[slot] = key;
                ci[slot] = li[i];
            }
        }
    }
    __syncthreads();
    if (!all_eq) {
        // keys equal to T: the first need_eq in position order, by a block-wide
        // count (the loop condition is the same in every thread)
        uint32_t taken = 0;
        for (int c0 = 0; c0 < tn && taken < need_eq; c0 += kSelThreads) {
            const int i = c0 + tid;
            const bool eq = i < tn && lk[i] == T;
            const uint64_t bal = __ballot(eq);
            const uint32_t below = (uint32_t)__popcll(bal & ((uint64_t(1) << lane) - 1));
            if (lane == 0) s_wave[wave] = (uint32_t)__popcll(bal);
            __syncthreads();
            uint32_t off = 0, tot = 0;
            for (int w = 0; w < kSelThreads / 64; ++w) {
                if (w < wave) off += s_wave[w];
                tot += s_wave[w];
            }
            const uint32_t r = taken + off + below;
            if (eq && r < need_eq) {
                ck[nless + r] = T;
                ci[nless + r] = li[i];
            }
            taken += tot;
            __syncthreads();
        }
    }
    // bitonic sort of the pairs by (key, index), padded to a power of two >= k
    int P = 1;
    while (P < k) P <<= 1;
    for (int i = kk + tid; i < P; i += kSelThreads) {
        ck[i] = UINT64_MAX;
        ci[i] = UINT32_MAX;
    }
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = tid; t < P / 2; t += kSelThreads) {
                const int lo = 2 * t - (t & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const uint64_t ka = ck[lo], kb = ck[hi];
                const uint32_t ia = ci[lo], ib = ci[hi];
                if (key_less(kb, ib, ka, ia) == up) {
                    ck[lo] = kb;
                    ck[hi] = ka;
                    ci[lo] = ib;
                    ci[hi] = ia;
                }
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < k; i += kSelThreads) {
        if (res_idx) {
            res_idx[i] = (int32_t)ci[i];
            res_dist[i] = __longlong_as_double((long long)ck[i]);
        } else {
            out_key[(int64_t)blockIdx.x * k + i] = ck[i];
            out_idx[(int64_t)blockIdx.x * k + i] = ci[i];
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
        hipLaunchKernelGGL(k_topk_select, dim3((unsigned)tiles), dim3(kSelThreads), 0, s, d, ik, ii, cur, k,
                           last ? nullptr : key[o], last ? nullptr : idx[o], last ? res_idx : nullptr,
                           last ? res_dist : nullptr);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || last) return e;
        cur = tiles * k;   // k <= kTile / 4, so every pass shrinks the count at least fourfold
        side = o;
    }
}

}  // namespace wmd
