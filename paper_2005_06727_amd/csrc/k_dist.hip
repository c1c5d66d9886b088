// Distance GEMM with the kernel-matrix epilogue (the lazily computed M of
// Algorithm 1's first step, restricted to the query rows, Sec. 4; done as a
// matrix product as Sec. 6 proposes, here on the CDNA4 matrix cores).
//
// For one query q (blockIdx.y) and 64 corpus words i (blockIdx.x):
//   G[i, k]  = <E[word(i)], E[qid[k]]>                 MFMA, FP32 or BF16 operands
//   d2       = |E[word(i)]|^2 + |E[qid[k]]|^2 - 2 G     (FP32)
//   d        = 0 when word(i) == qid[k];
//              sqrt(sum_d (E[word(i), d] - E[qid[k], d])^2) in FP32 when d2 < tau^2
//              (the expansion cancels there); sqrt(max(d2, 0)) otherwise
//   n_i      = min_k d[i, k] when the log-domain shift is on, else 0
//   Kt[i, k] = exp(-lambda (d - n_i)),  KMt[i, k] = Kt[i, k] * d
// Columns m <= k < ldk are written as zeros.
#include "wmd_internal.h"

namespace wmd {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int BM = 64;   // corpus rows per workgroup (4 waves x 16)
constexpr int BN = 64;   // query columns per chunk (4 MFMA column blocks of 16)

// Operand staging geometry per precision.
template <bool BF16> struct Tile;
template <> struct Tile<false> {
    typedef float T;
    static constexpr int BK = 32;          // k per stage
    static constexpr int LD = BK + 4;      // LDS row stride (elements)
};
template <> struct Tile<true> {
    typedef uint16_t T;
    static constexpr int BK = 64;
    static constexpr int LD = BK + 8;
};

struct DistArgs {
    const float* act;        // U x ldv FP32
    const uint16_t* act16;   // U x ldv BF16 (BF16 path)
    const float* norm;       // U: |row|^2 matching the operand precision
    const int32_t* act_word; // U
    const float* vecs;       // V x ldv FP32 (query rows)
    const QueryDev* qd;
    int64_t U;
    int32_t ldv;
};

__device__ __forceinline__ uint16_t bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_val(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Direct FP32 sum of squared differences over a padded row.
__device__ float direct_d2(const float* __restrict__ a, const float* __restrict__ b, int ldv) {
    const float4* pa = reinterpret_cast<const float4*>(a);
    const float4* pb = reinterpret_cast<const float4*>(b);
    float s = 0.f;
    for (int k = 0; k < ldv / 4; ++k) {
        float4 x = pa[k], y = pb[k];
        float t0 = x.x - y.x, t1 = x.y - y.y, t2 = x.z - y.z, t3 = x.w - y.w;
        s = fmaf(t0, t0, s);
        s = fmaf(t1, t1, s);
        s = fmaf(t2, t2, s);
        s = fmaf(t3, t3, s);
    }
    return s;
}

// min over the 16 lanes of a DPP row (lane % 16 varies the column).
__device__ __forceinline__ float row16_min(float v) {
    v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false)));
    v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false)));
    v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false)));
    v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false)));
    return v;
}

template <bool BF16>
__global__ __launch_bounds__(256) void k_dist(DistArgs a) {
    typedef Tile<BF16> TL;
    typedef typename TL::T T;
    constexpr int BK = TL::BK, LD = TL::LD;
    __shared__ __attribute__((aligned(16))) T As[BM * LD];
    __shared__ __attribute__((aligned(16))) T Qs[BN * LD];
    __shared__ int32_t s_qid[BN];
    __shared__ float s_qn[BN];

    const QueryDev q = a.qd[blockIdx.y];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * BM;
    const int m = q.m, ldk = q.ldk, ldv = a.ldv;
    const float lam = q.lambda;

    float rmin[4] = {INFINITY, INFINITY, INFINITY, INFINITY};

    for (int chunk0 = 0; chunk0 < ldk; chunk0 += BN) {
        const int nb_act = min(4, (ldk - chunk0 + 15) / 16);   // column blocks in use
        if (tid < BN) {
            int j = chunk0 + tid;
            s_qid[tid] = (j < m) ? q.qid[j] : -1;
        }
        __syncthreads();
        v4f acc[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) acc[nb] = v4f{0.f, 0.f, 0.f, 0.f};
        float qn = 0.f;

        for (int k0 = 0; k0 < ldv; k0 += BK) {
            // stage the 64 x BK corpus tile and the 64 x BK query tile
            if constexpr (!BF16) {
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    int idx = tid + 256 * e;
                    int r = idx >> 3, c4 = (idx & 7) * 4;
                    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (row0 + r < a.U)
                        v = *reinterpret_cast<const float4*>(a.act + (row0 + r) * ldv + k0 + c4);
                    *reinterpret_cast<float4*>(&As[r * LD + c4]) = v;
                    float4 w = make_float4(0.f, 0.f, 0.f, 0.f);
                    int qi = s_qid[r];
                    if (qi >= 0)
                        w = *reinterpret_cast<const float4*>(a.vecs + (int64_t)qi * ldv + k0 + c4);
                    *reinterpret_cast<float4*>(&Qs[r * LD + c4]) = w;
                }
            } else {
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    int idx = tid + 256 * e;
                    int r = idx >> 3, c8 = (idx & 7) * 8;
                    uint4 v = make_uint4(0u, 0u, 0u, 0u);
                    if (row0 + r < a.U)
                        v = *reinterpret_cast<const uint4*>(a.act16 + (row0 + r) * ldv + k0 + c8);
                    *reinterpret_cast<uint4*>(&As[r * LD + c8]) = v;
                    uint16_t h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                    int qi = s_qid[r];
                    if (qi >= 0) {
                        const float4* src = reinterpret_cast<const float4*>(a.vecs + (int64_t)qi * ldv + k0 + c8);
                        float4 f0 = src[0], f1 = src[1];
                        h[0] = bf16_rne(f0.x); h[1] = bf16_rne(f0.y); h[2] = bf16_rne(f0.z); h[3] = bf16_rne(f0.w);
                        h[4] = bf16_rne(f1.x); h[5] = bf16_rne(f1.y); h[6] = bf16_rne(f1.z); h[7] = bf16_rne(f1.w);
                    }
                    uint4 w;
                    w.x = h[0] | ((uint32_t)h[1] << 16);
                    w.y = h[2] | ((uint32_t)h[3] << 16);
                    w.z = h[4] | ((uint32_t)h[5] << 16);
                    w.w = h[6] | ((uint32_t)h[7] << 16);
                    *reinterpret_cast<uint4*>(&Qs[r * LD + c8]) = w;
                }
            }
            __syncthreads();
            if (tid < BN) {
                // query norms from the staged operand values
#pragma unroll 8
                for (int k = 0; k < BK; ++k) {
                    float f;
                    if constexpr (BF16) f = bf16_val(Qs[tid * LD + k]);
                    else f = Qs[tid * LD + k];
                    qn = fmaf(f, f, qn);
                }
            }
            const int ar = wave * 16 + (lane & 15);
            const int kg = lane >> 4;
            if constexpr (!BF16) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    float4 av = *reinterpret_cast<const float4*>(&As[ar * LD + h * 16 + kg * 4]);
#pragma unroll
                    for (int nb = 0; nb < 4; ++nb) {
                        if (nb < nb_act) {
                            float4 bv = *reinterpret_cast<const float4*>(&Qs[(nb * 16 + (lane & 15)) * LD + h * 16 + kg * 4]);
                            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv.x, acc[nb], 0, 0, 0);
                            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bv.y, acc[nb], 0, 0, 0);
                            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, bv.z, acc[nb], 0, 0, 0);
                            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, bv.w, acc[nb], 0, 0, 0);
                        }
                    }
                }
            } else {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    v8bf av = *reinterpret_cast<const v8bf*>(&As[ar * LD + h * 32 + kg * 8]);
#pragma unroll
                    for (int nb = 0; nb < 4; ++nb) {
                        if (nb < nb_act) {
                            v8bf bv = *reinterpret_cast<const v8bf*>(&Qs[(nb * 16 + (lane & 15)) * LD + h * 32 + kg * 8]);
                            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[nb], 0, 0, 0);
                        }
                    }
                }
            }
            __syncthreads();
        }
        if (tid < BN) s_qn[tid] = qn;
        __syncthreads();

        // epilogue: lane holds G[row 4*(lane/16)+r][col lane%16] of each column block
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            if (nb >= nb_act) continue;
            const int jl = nb * 16 + (lane & 15);
            const int gj = chunk0 + jl;
            const int qi = s_qid[jl];
            const float qnj = s_qn[jl];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = row0 + wave * 16 + 4 * (lane >> 4) + r;
                if (gi >= a.U || gj >= ldk) continue;
                float* kt = q.Kt + gi * ldk + gj;
                float* km = q.KMt + gi * ldk + gj;
                if (gj >= m) { *kt = 0.f; *km = 0.f; continue; }
                float d;
                if (a.act_word[gi] == qi) {
                    d = 0.f;
                } else {
                    float d2 = a.norm[gi] + qnj - 2.f * acc[nb][r];
                    if (d2 < q.tau2)
                        d2 = direct_d2(a.act + gi * ldv, a.vecs + (int64_t)qi * ldv, ldv);
                    d = sqrtf(fmaxf(d2, 0.f));
                }
                if (q.shift) {
                    *kt = d;
                    rmin[r] = fminf(rmin[r], d);
                } else {
                    float kv = expf(-lam * d);
                    *kt = kv;
                    *km = kv * d;
                }
            }
        }
        __syncthreads();
    }

    if (q.shift) {
        // n_i = min_k d[i, k]: over this lane's columns (done), then the 16 lanes of the row
#pragma unroll
        for (int r = 0; r < 4; ++r) rmin[r] = row16_min(rmin[r]);
        for (int chunk0 = 0; chunk0 < ldk; chunk0 += BN) {
            const int nb_act = min(4, (ldk - chunk0 + 15) / 16);
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
                if (nb >= nb_act) continue;
                const int gj = chunk0 + nb * 16 + (lane & 15);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t gi = row0 + wave * 16 + 4 * (lane >> 4) + r;
                    if (gi >= a.U || gj >= m) continue;
                    float* kt = q.Kt + gi * ldk + gj;
                    float d = *kt;                     // written by this same lane above
                    float kv = expf(-lam * (d - rmin[r]));
                    *kt = kv;
                    q.KMt[gi * ldk + gj] = kv * d;
                }
            }
        }
    }
}

}  // namespace

hipError_t launch_dist(const DevCorpus& c, const QueryDev* qd, int B, int max_m, int bf16,
                       hipStream_t s) {
    (void)max_m;
    if (B <= 0 || c.U <= 0) return hipSuccess;
    DistArgs a;
    a.act = c.act;
    a.act16 = c.act_bf16;
    a.norm = bf16 ? c.act_norm_bf16 : c.act_norm;
    a.act_word = c.act_word;
    a.vecs = c.vecs;
    a.qd = qd;
    a.U = c.U;
    a.ldv = c.ldv;
    dim3 grid((unsigned)((c.U + BM - 1) / BM), (unsigned)B);
    if (bf16)
        hipLaunchKernelGGL(k_dist<true>, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_dist<false>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace wmd
