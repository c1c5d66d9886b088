// Distance GEMM with the kernel-matrix epilogue (the lazily computed M of
// Algorithm 1's first step, restricted to the query rows, Sec. 4; done as a
// matrix product as Sec. 6 proposes, here on the CDNA4 matrix cores).
//
// For a group of queries (blockIdx.y) and a tile of corpus words i (blockIdx.x):
//   G[i, k]  = <E[word(i)], E[qid[k]]>                 MFMA, FP32 or BF16 operands
//   d2       = |E[word(i)]|^2 + |E[qid[k]]|^2 - 2 G     (FP32)
//   d        = 0 when word(i) == qid[k];
//              sqrt(sum_d (E[word(i), d] - E[qid[k], d])^2) in FP32 when d2 < tau^2
//              (the expansion cancels there); sqrt(max(d2, 0)) otherwise
//   n_i      = min_k d[i, k] over the query's words when the log-domain shift
//              is on, else 0
//   Kt[i, k] = exp(-lambda (d - n_i)),  KMt[i, k] = Kt[i, k] * d
// Columns m <= k < ldk are written as zeros.
//
// Split-K: the 4 waves of a block share the tile's corpus rows and each takes
// a slice of the embedding dimension (FP32: 32 rows, 4 slices; BF16: 2 x 32
// rows, 2 slices); each wave computes two 16-row groups so that every query
// fragment it loads serves 32 corpus rows.  A wave loads its slice of the corpus rows into
// registers once (every load in flight together) and keeps it for every query
// column chunk of the group; the query fragments come straight from global
// memory (they are few and cache-resident).  The slices' partial products are
// summed through LDS in a fixed order, so results do not depend on timing.
#include <algorithm>
#include <type_traits>

#include "wmd_internal.h"

namespace wmd {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int BN = 32;     // query columns per chunk (2 MFMA column blocks)
constexpr int KB = 64;     // embedding elements per fragment step of the whole block
constexpr int NFMAX = 16;  // fragments per wave per register-resident chunk (ldv <= 1024)

template <bool BF16> struct Op;
template <> struct Op<false> {   // v_mfma_f32_16x16x4_f32: float4 fragment = 4 MFMAs, 16 k
    typedef float4 Frag;
    static constexpr int RGW = 1;   // waves along rows per block
    static constexpr int KSPL = 4;  // k slices per block
    static constexpr int KF = 16;   // k per fragment (4 lane groups x 4)
};
template <> struct Op<true> {    // v_mfma_f32_16x16x32_bf16: 8 bf16 per lane, 32 k
    typedef uint4 Frag;
    static constexpr int RGW = 2;
    static constexpr int KSPL = 2;
    static constexpr int KF = 32;
};
constexpr int RT = 2;   // 16-row groups per wave: each query fragment load serves 32 corpus rows

struct DistArgs {
    const float* act;        // U x ldv FP32
    const uint16_t* act16;   // U x ldv BF16 (BF16 path)
    const float* norm;       // U: |row|^2 matching the operand precision
    const int32_t* act_word; // U
    const float* vecs;       // V x ldv FP32 (query rows)
    const QueryDev* qd;
    const int32_t* qgroup;   // G+1: queries [qgroup[g], qgroup[g+1]) form group g
    int64_t U;
    int32_t ldv;
};

__device__ __forceinline__ uint16_t bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

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

template <int CTRL>
__device__ __forceinline__ float dppf(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// min over 32 consecutive lanes
__device__ __forceinline__ float min32(float v) {
    v = fminf(v, dppf<0xB1>(v));     // lane ^ 1
    v = fminf(v, dppf<0x4E>(v));     // lane ^ 2
    v = fminf(v, dppf<0x141>(v));    // other quad of the 8 (quads uniform)
    v = fminf(v, dppf<0x140>(v));    // other half of the row (halves uniform)
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return fminf(__uint_as_float(r[0]), __uint_as_float(r[1]));   // rows 2j, 2j+1
}

// sum over the 4 lane groups (lanes l, l^16, l^32, l^48)
__device__ __forceinline__ float sum_lane_groups(float v) {
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    auto t = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(t[0]) + __uint_as_float(t[1]);
}

// NF: fragments per wave per chunk; one chunk covers KSPL*NF*KF embedding
// elements (the launcher picks NF = ldv / 64 when ldv <= 1024).
template <bool BF16, int NF>
__global__ __launch_bounds__(256) void k_dist(DistArgs a) {
    typedef Op<BF16> O;
    typedef typename O::Frag Frag;
    constexpr int RGW = O::RGW, KSPL = O::KSPL, KF = O::KF;
    constexpr int TR = 16 * RT * RGW;        // rows per tile
    constexpr int KCH = KSPL * NF * KF;      // embedding elements per chunk
    __shared__ float red[KSPL][TR][BN + 1];  // partial products of the k slices
    __shared__ float qnp[KSPL][BN];          // partial query norms
    __shared__ int32_t s_qid[BN];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int rw = wave / KSPL, ks = wave % KSPL;   // row wave, k slice of this wave
    const int lr = lane & 15;                       // operand row / result column
    const int lg = lane >> 4;                       // lane group
    const int64_t row0 = (int64_t)blockIdx.x * TR;
    // row group t of this wave: rows row0 + (rw * RT + t) * 16 + 0..15
    const int ldv = a.ldv;
    const int nkc = (ldv + KCH - 1) / KCH;
    const int q_begin = a.qgroup[blockIdx.y], q_end = a.qgroup[blockIdx.y + 1];

    // fragment f of this wave covers k = kc*KCH + (ks*NF + f)*KF + lg*(KF/4) .. + KF/4 - 1
    auto kof = [&](int kc, int f) { return kc * KCH + (ks * NF + f) * KF + lg * (KF / 4); };
    // epilogue ownership: thread t handles (row t/32 + 8j, column t%32), j < TR/8;
    // its rows' vocabulary ids and norms are fetched before the operand stream
    constexpr int EJ = TR / 8;
    const int ec = tid & 31, er = tid >> 5;
    int e_word[EJ];
    float e_norm[EJ];
#pragma unroll
    for (int j = 0; j < EJ; ++j) {
        const int64_t gi = row0 + er + 8 * j;
        e_word[j] = (gi < a.U) ? a.act_word[gi] : -2;
        e_norm[j] = (gi < a.U) ? a.norm[gi] : 0.f;
    }

    Frag A[RT][NF];
    auto load_a = [&](int kc) {
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            const int64_t arow = row0 + (rw * RT + t) * 16 + lr;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const int k = kof(kc, f);
                Frag z;
                if constexpr (BF16) z = make_uint4(0u, 0u, 0u, 0u);
                else z = make_float4(0.f, 0.f, 0.f, 0.f);
                if (arow < a.U && k < ldv) {
                    if constexpr (BF16) z = *reinterpret_cast<const uint4*>(a.act16 + arow * ldv + k);
                    else z = *reinterpret_cast<const float4*>(a.act + arow * ldv + k);
                }
                A[t][f] = z;
            }
        }
    };
    bool a_loaded = false;   // one chunk: A is loaded once, after the first query fragments

    for (int qi = q_begin; qi < q_end; ++qi) {
        const QueryDev q = a.qd[qi];
        const int m = q.m, ldk = q.ldk;
        const float lam = q.lambda;
        float rmin[EJ];
#pragma unroll
        for (int j = 0; j < EJ; ++j) rmin[j] = INFINITY;

        for (int col0 = 0; col0 < ldk; col0 += BN) {
            const int nb_act = min(2, (ldk - col0 + 15) / 16);
            int w[2];
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                const int c = col0 + nb * 16 + lr;
                w[nb] = (c < m) ? q.qid[c] : -1;
            }
            v4f acc[RT][2];
#pragma unroll
            for (int t = 0; t < RT; ++t) acc[t][0] = acc[t][1] = v4f{0.f, 0.f, 0.f, 0.f};
            float qn[2] = {0.f, 0.f};
            for (int kc = 0; kc < nkc; ++kc) {
                // query fragments of this wave's slice for both column blocks (issued
                // before the corpus rows so the MFMAs can start while those stream in)
                Frag B[2][NF];
#pragma unroll
                for (int nb = 0; nb < 2; ++nb) {
#pragma unroll
                    for (int f = 0; f < NF; ++f) {
                        const int k = kof(kc, f);
                        Frag z;
                        if constexpr (BF16) z = make_uint4(0u, 0u, 0u, 0u);
                        else z = make_float4(0.f, 0.f, 0.f, 0.f);
                        if (nb < nb_act && w[nb] >= 0 && k < ldv) {
                            const float* src = a.vecs + (int64_t)w[nb] * ldv + k;
                            if constexpr (!BF16) {
                                z = *reinterpret_cast<const float4*>(src);
                            } else {
                                const float4 f0 = reinterpret_cast<const float4*>(src)[0];
                                const float4 f1 = reinterpret_cast<const float4*>(src)[1];
                                z.x = bf16_rne(f0.x) | ((uint32_t)bf16_rne(f0.y) << 16);
                                z.y = bf16_rne(f0.z) | ((uint32_t)bf16_rne(f0.w) << 16);
                                z.z = bf16_rne(f1.x) | ((uint32_t)bf16_rne(f1.y) << 16);
                                z.w = bf16_rne(f1.z) | ((uint32_t)bf16_rne(f1.w) << 16);
                            }
                        }
                        B[nb][f] = z;
                    }
                }
                if (nkc > 1) {
                    load_a(kc);
                } else if (!a_loaded) {
                    load_a(0);
                    a_loaded = true;
                }
                // |q|^2 of the operand values (partial over this lane's k)
#pragma unroll
                for (int nb = 0; nb < 2; ++nb) {
#pragma unroll
                    for (int f = 0; f < NF; ++f) {
                        if constexpr (!BF16) {
                            const float4 b = B[nb][f];
                            qn[nb] = fmaf(b.x, b.x, qn[nb]);
                            qn[nb] = fmaf(b.y, b.y, qn[nb]);
                            qn[nb] = fmaf(b.z, b.z, qn[nb]);
                            qn[nb] = fmaf(b.w, b.w, qn[nb]);
                        } else {
                            const uint4 b = B[nb][f];
                            const uint32_t ws[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const float lo = bf16_lo(ws[e]), hi = bf16_hi(ws[e]);
                                qn[nb] = fmaf(lo, lo, qn[nb]);
                                qn[nb] = fmaf(hi, hi, qn[nb]);
                            }
                        }
                    }
                }
                auto mma = [&](auto nbc) {
                    constexpr int NB = decltype(nbc)::value;
#pragma unroll
                    for (int f = 0; f < NF; ++f) {
#pragma unroll
                        for (int t = 0; t < RT; ++t) {
#pragma unroll
                            for (int nb = 0; nb < NB; ++nb) {
                                v4f& c = acc[t][nb];
                                if constexpr (!BF16) {
                                    const float4 av = A[t][f], bv = B[nb][f];
                                    c = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv.x, c, 0, 0, 0);
                                    c = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bv.y, c, 0, 0, 0);
                                    c = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, bv.z, c, 0, 0, 0);
                                    c = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, bv.w, c, 0, 0, 0);
                                } else {
                                    const uint4 ai = A[t][f], bi = B[nb][f];
                                    const v8bf av = *reinterpret_cast<const v8bf*>(&ai);
                                    const v8bf bv = *reinterpret_cast<const v8bf*>(&bi);
                                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
                                }
                            }
                        }
                    }
                };
                if (nb_act == 2) mma(std::integral_constant<int, 2>());
                else mma(std::integral_constant<int, 1>());
            }
            // partial results of this slice -> LDS: lane holds G[4*lg + r][16*nb + lr]
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
#pragma unroll
                for (int t = 0; t < RT; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        red[ks][(rw * RT + t) * 16 + 4 * lg + r][nb * 16 + lr] = acc[t][nb][r];
                const float qs = sum_lane_groups(qn[nb]);
                if (rw == 0 && lg == 0) qnp[ks][nb * 16 + lr] = qs;
            }
            if (tid < BN) s_qid[tid] = (col0 + tid < m) ? q.qid[col0 + tid] : -1;
            __syncthreads();

            // epilogue: sum the slices in order, then distance, K and K .* M
            const int gj = col0 + ec;
            const int qw = s_qid[ec];
            float qnj = 0.f;
#pragma unroll
            for (int s2 = 0; s2 < KSPL; ++s2) qnj += qnp[s2][ec];
#pragma unroll
            for (int j = 0; j < EJ; ++j) {
                const int rr = er + 8 * j;
                const int64_t gi = row0 + rr;
                if (gi >= a.U || gj >= ldk) continue;
                float* kt = q.Kt + gi * ldk + gj;
                float* km = q.KMt + gi * ldk + gj;
                if (gj >= m) {
                    *kt = 0.f;
                    if (!q.km_from_k) *km = 0.f;
                    continue;
                }
                float g = 0.f;
#pragma unroll
                for (int s2 = 0; s2 < KSPL; ++s2) g += red[s2][rr][ec];
                float d;
                if (e_word[j] == qw) {
                    d = 0.f;
                } else {
                    float d2 = e_norm[j] + qnj - 2.f * g;
                    if (d2 < q.tau2) d2 = direct_d2(a.act + gi * ldv, a.vecs + (int64_t)qw * ldv, ldv);
                    d = sqrtf(fmaxf(d2, 0.f));
                }
                if (q.shift) {
                    *kt = d;
                    rmin[j] = fminf(rmin[j], d);
                } else {
                    const float kv = expf(-lam * d);
                    *kt = kv;
                    if (!q.km_from_k) *km = kv * d;
                }
            }
            __syncthreads();   // red, qnp, s_qid are reused by the next chunk
        }

        if (q.shift) {
            // n_i = min_k d[i, k]: this thread's columns (done), then the 32 threads of the row
#pragma unroll
            for (int j = 0; j < EJ; ++j) {
                rmin[j] = min32(rmin[j]);
                const int64_t gi = row0 + er + 8 * j;
                if (ec == 0 && gi < a.U) q.nrow[gi] = rmin[j];
            }
            for (int col0 = 0; col0 < ldk; col0 += BN) {
                const int gj = col0 + ec;
#pragma unroll
                for (int j = 0; j < EJ; ++j) {
                    const int64_t gi = row0 + er + 8 * j;
                    if (gi >= a.U || gj >= m) continue;
                    float* kt = q.Kt + gi * ldk + gj;
                    const float d = *kt;                   // written by this same thread above
                    const float kv = expf(-lam * (d - rmin[j]));
                    *kt = kv;
                    if (!q.km_from_k) q.KMt[gi * ldk + gj] = kv * d;
                }
            }
        }
    }
}

}  // namespace

hipError_t launch_dist(const DevCorpus& c, const QueryDev* qd, const int32_t* qgroup, int groups, int bf16,
                       hipStream_t s) {
    if (groups <= 0 || c.U <= 0) return hipSuccess;
    DistArgs a;
    a.act = c.act;
    a.act16 = c.act_bf16;
    a.norm = bf16 ? c.act_norm_bf16 : c.act_norm;
    a.act_word = c.act_word;
    a.vecs = c.vecs;
    a.qd = qd;
    a.qgroup = qgroup;
    a.U = c.U;
    a.ldv = c.ldv;
    const int tr = bf16 ? 64 : 32;   // 16 * RT * RGW
    dim3 grid((unsigned)((c.U + tr - 1) / tr), (unsigned)groups);
    // fragments per wave: ldv / 64 (one chunk) up to 1024 elements, chunks of 16 beyond
    const int nf = std::min(NFMAX, (c.ldv + KB - 1) / KB);
#define WMD_DIST_CASE(K)                                                              \
    case K:                                                                           \
        if (bf16) hipLaunchKernelGGL((k_dist<true, K>), grid, dim3(256), 0, s, a);    \
        else hipLaunchKernelGGL((k_dist<false, K>), grid, dim3(256), 0, s, a);        \
        break;
    switch (nf) {
        WMD_DIST_CASE(1) WMD_DIST_CASE(2) WMD_DIST_CASE(3) WMD_DIST_CASE(4)
        WMD_DIST_CASE(5) WMD_DIST_CASE(6) WMD_DIST_CASE(7) WMD_DIST_CASE(8)
        WMD_DIST_CASE(9) WMD_DIST_CASE(10) WMD_DIST_CASE(11) WMD_DIST_CASE(12)
        WMD_DIST_CASE(13) WMD_DIST_CASE(14) WMD_DIST_CASE(15) WMD_DIST_CASE(16)
        default: return hipErrorInvalidValue;
    }
#undef WMD_DIST_CASE
    return hipGetLastError();
}

}  // namespace wmd
