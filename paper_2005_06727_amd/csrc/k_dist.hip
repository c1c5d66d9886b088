// Distance GEMM with the kernel-matrix epilogue (the lazily computed M of
// Algorithm 1's first step, restricted to the query rows, Sec. 4; done as a
// matrix product as Sec. 6 proposes, here on the CDNA4 matrix cores).
//
// The query words of every query of a call form the columns of one GEMM
// (query b owns global columns [kofs[b], kofs[b] + ldk_b)).  For a tile of 64
// corpus words i and TC columns c (query b, local column k):
//   G[i, c]  = <E[word(i)], E[qid_b[k]]>               MFMA, FP32 or BF16 operands
//   d2       = |E[word(i)]|^2 + |E[qid_b[k]]|^2 - 2 G   (FP32, norms of the operand values)
//   d        = 0 when word(i) == qid_b[k];
//              sqrt(sum_d (E[word(i), d] - E[qid_b[k], d])^2) in FP32 when d2 < tau^2
//              (the expansion cancels there); sqrt(max(d2, 0)) otherwise
//   Kt_b[i, k] = exp(-lambda d), KMt_b[i, k] = Kt_b[i, k] * d (small lambda only);
//   with the log-domain shift the tile writes d and folds it into
//   n_i = min_k d[i, k] (an atomic minimum), and k_shift_exp then writes
//   Kt_b[i, k] = exp(-lambda (d - n_i)).
// Columns m_b <= k < ldk_b are written as zeros.
//
// Each block streams its 64 corpus rows through LDS in chunks of the embedding
// dimension (128 or 256 bytes per row and chunk), double buffered: the global loads
// of chunk c + 1 are in flight while the matrix cores work on chunk c.  The
// query columns are staged the same way.  Tiles are ordered so that the
// column tiles of one row tile run on the same XCD and share its L2.
#include <algorithm>
#include <cstring>

#include "wmd_device.h"
#include "launch.h"
#include "wmd_internal.h"

namespace wmd {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int TR = 64;        // corpus rows per tile

struct DistArgs {
    const float* act;         // U x ldv FP32
    const uint16_t* act16;    // U x ldv BF16 (BF16 path)
    const float* norm;        // U: |row|^2 matching the operand precision
    const int32_t* act_word;  // U
    const float* vecs;        // V x ldv FP32 (query rows)
    const QueryDev* qd;       // B queries
    const int32_t* kofs;      // B + 1: first global column of each query
    int64_t U;
    int32_t ldv;
    int32_t B;
    int32_t ncols;            // kofs[B]
    int32_t tiles_c;
    int32_t nblocks;
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

// sum over the 4 lane groups (lanes l, l^16, l^32, l^48)
__device__ __forceinline__ float sum_lane_groups(float v) {
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    auto t = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(t[0]) + __uint_as_float(t[1]);
}

// query of a global column: the largest b with kofs[b] <= c
__device__ __forceinline__ int query_of(const int32_t* kofs, int B, int c) {
    int lo = 0, hi = B - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (kofs[mid] <= c) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Epilogue of a wave's sub-tile: lane (lr, lg) holds G[row 16 t + 4 lg + r]
// [column 16 nb + lr] of the rows from rbase and columns from cbase.  With the
// column shift, Kt receives d and the row minima go to each query's nrow by
// atomics; when the wave's 32 columns belong to one query (always in a
// one-query call, and for most columns of a batch), the minimum over them is
// taken in the wave first and one lane per row does the atomic.
template <int RT>
__device__ __forceinline__ void epilogue(const DistArgs& a, const v4f (&acc)[RT][2], const float (&qn)[2],
                                         const int (&e_word)[RT][4], const float (&e_norm)[RT][4],
                                         const int64_t rbase, const int cbase, const int lr, const int lg) {
    const int ldv = a.ldv;
    const int clast = min(cbase + 31, a.ncols - 1);
    const int b0 = query_of(a.kofs, a.B, cbase);
    const bool one_query = b0 == query_of(a.kofs, a.B, clast);
    const bool shift = a.qd[b0].shift != 0;   // one option for every query of a call
    float dmin[RT][4];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) dmin[t][r] = INFINITY;
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
        const float qnj = sum_lane_groups(qn[nb]);
        const int c = cbase + 16 * nb + lr;
        if (c >= a.ncols) continue;
        const int b = query_of(a.kofs, a.B, c);
        const int k = c - a.kofs[b];
        const QueryDev* q = a.qd + b;
        const int m = q->m, ldk = q->ldk;
        const int qw = (k < m) ? q->qid[k] : -1;
        const float lam = q->lambda, tau2 = q->tau2;
        const bool km = !q->km_from_k;
        // squared distances (0 for a word the query shares); the FP32
        // recompute below tau is rare, so it runs behind one wave-wide test
        float d2v[RT][4];
        bool need = false;
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const bool same = e_word[t][r] == qw;
                d2v[t][r] = same ? 0.f : e_norm[t][r] + qnj - 2.f * acc[t][nb][r];
                need |= k < m && !same && d2v[t][r] < tau2 && rbase + 16 * t + 4 * lg + r < a.U;
            }
        if (__builtin_amdgcn_ballot_w64(need)) {
#pragma unroll
            for (int t = 0; t < RT; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t gi = rbase + 16 * t + 4 * lg + r;
                    if (k < m && e_word[t][r] != qw && d2v[t][r] < tau2 && gi < a.U)
                        d2v[t][r] = direct_d2(a.act + gi * ldv, a.vecs + (int64_t)qw * ldv, ldv);
                }
        }
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = rbase + 16 * t + 4 * lg + r;
                if (gi >= a.U) continue;
                float* kt = q->Kt + gi * ldk + k;
                if (k >= m) {
                    *kt = 0.f;
                    if (km) q->KMt[gi * ldk + k] = 0.f;
                    continue;
                }
                const float d = sqrtf(fmaxf(d2v[t][r], 0.f));
                if (shift) {
                    *kt = d;
                    // d >= 0, so the bit patterns order like the values
                    if (one_query) dmin[t][r] = fminf(dmin[t][r], d);
                    else atomicMin(reinterpret_cast<unsigned int*>(q->nrow + gi), __float_as_uint(d));
                } else {
                    const float kv = expf(-lam * d);
                    *kt = kv;
                    if (km) q->KMt[gi * ldk + k] = kv * d;
                }
            }
    }
    if (shift && one_query) {
        float* nrow = a.qd[b0].nrow;
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float v = dmin[t][r];
#pragma unroll
                for (int o = 1; o < 16; o <<= 1) v = fminf(v, __shfl_xor(v, o, 64));
                const int64_t gi = rbase + 16 * t + 4 * lg + r;
                if (lr == 0 && gi < a.U && v < INFINITY)
                    atomicMin(reinterpret_cast<unsigned int*>(nrow + gi), __float_as_uint(v));
            }
    }
}

// TC: query columns per tile (32: 4 waves of 16 rows x 32 columns; 64: 2 x 2
// waves of 32 x 32).  CHB: bytes per row and chunk; the narrow tile (one short
// query, bound by HBM) streams bigger chunks to keep more bytes in flight.
template <bool BF16, int TC, int CHB>
__global__ __launch_bounds__(256) void k_dist(DistArgs a) {
    constexpr int SB = CHB + 16;                // LDS row stride: 8 lanes on distinct banks
    constexpr int RT = (TC == 64) ? 2 : 1;      // 16-row groups per wave
    constexpr int NB = 2;                       // 16-column groups per wave
    constexpr int AP = TR * (CHB / 16) / 256;   // A staging pieces per thread
    constexpr int BP = TC * (CHB / 16) / 256;   // B staging pieces per thread
    constexpr int SEG = CHB / 16;               // 16-byte segments per row and chunk
    constexpr int KS = CHB / 128;               // 128-byte sub-chunks per chunk
    __shared__ __attribute__((aligned(16))) char As[2][TR * SB];
    __shared__ __attribute__((aligned(16))) char Bs[2][TC * SB];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const int wr = (TC == 64) ? (wave >> 1) : wave;
    const int wc = (TC == 64) ? (wave & 1) : 0;

    // XCD-aware tile order: blocks b and b + 8 share an XCD, so consecutive
    // logical tiles (the column tiles of one row tile) go to the same XCD
    int L = blockIdx.x;
    const int nb8 = a.nblocks / 8 * 8;
    if (L < nb8) L = (L % 8) * (a.nblocks / 8) + L / 8;
    const int64_t row0 = (int64_t)(L / a.tiles_c) * TR;
    const int col0 = (L % a.tiles_c) * TC;
    const int ldv = a.ldv;
    const int nchunks = ldv * (BF16 ? 2 : 4) / CHB;

    // ---- staging sources: A pieces (row, 16-byte segment), B pieces (column, segment)
    const char* asrc[AP];
#pragma unroll
    for (int j = 0; j < AP; ++j) {
        const int p = tid + 256 * j;
        const int64_t row = row0 + p / SEG;
        asrc[j] = nullptr;
        if (row < a.U) {
            if constexpr (BF16) asrc[j] = reinterpret_cast<const char*>(a.act16 + row * ldv) + (p % SEG) * 16;
            else asrc[j] = reinterpret_cast<const char*>(a.act + row * ldv) + (p % SEG) * 16;
        }
    }
    const float* bsrc[BP];
#pragma unroll
    for (int j = 0; j < BP; ++j) {
        const int p = tid + 256 * j;
        const int c = col0 + p / SEG;
        bsrc[j] = nullptr;
        if (c < a.ncols) {
            const int b = query_of(a.kofs, a.B, c);
            const int k = c - a.kofs[b];
            const QueryDev* q = a.qd + b;
            // FP32: 4 floats per segment; BF16: 8 floats rounded to 8 bf16
            if (k < q->m) bsrc[j] = a.vecs + (int64_t)q->qid[k] * ldv + (p % SEG) * (BF16 ? 8 : 4);
        }
    }
    uint4 ra[AP], rb[BP];
    auto load_chunk = [&](int ch) {
#pragma unroll
        for (int j = 0; j < AP; ++j)
            ra[j] = asrc[j] ? *reinterpret_cast<const uint4*>(asrc[j] + ch * CHB) : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
        for (int j = 0; j < BP; ++j) {
            if constexpr (BF16) {
                if (bsrc[j]) {
                    const float4 f0 = reinterpret_cast<const float4*>(bsrc[j] + ch * (CHB / 2))[0];
                    const float4 f1 = reinterpret_cast<const float4*>(bsrc[j] + ch * (CHB / 2))[1];
                    rb[j].x = bf16_rne(f0.x) | ((uint32_t)bf16_rne(f0.y) << 16);
                    rb[j].y = bf16_rne(f0.z) | ((uint32_t)bf16_rne(f0.w) << 16);
                    rb[j].z = bf16_rne(f1.x) | ((uint32_t)bf16_rne(f1.y) << 16);
                    rb[j].w = bf16_rne(f1.z) | ((uint32_t)bf16_rne(f1.w) << 16);
                } else {
                    rb[j] = make_uint4(0u, 0u, 0u, 0u);
                }
            } else {
                rb[j] = bsrc[j] ? *reinterpret_cast<const uint4*>(bsrc[j] + ch * (CHB / 4)) : make_uint4(0u, 0u, 0u, 0u);
            }
        }
    };
    auto store_chunk = [&](int buf) {
#pragma unroll
        for (int j = 0; j < AP; ++j) {
            const int p = tid + 256 * j;
            *reinterpret_cast<uint4*>(&As[buf][(p / SEG) * SB + (p % SEG) * 16]) = ra[j];
        }
#pragma unroll
        for (int j = 0; j < BP; ++j) {
            const int p = tid + 256 * j;
            *reinterpret_cast<uint4*>(&Bs[buf][(p / SEG) * SB + (p % SEG) * 16]) = rb[j];
        }
    };

    // ---- epilogue metadata, fetched before the operand stream
    int e_word[RT][4];
    float e_norm[RT][4];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t gi = row0 + wr * 16 * RT + 16 * t + 4 * lg + r;
            e_word[t][r] = (gi < a.U) ? a.act_word[gi] : -2;
            e_norm[t][r] = (gi < a.U) ? a.norm[gi] : 0.f;
        }

    load_chunk(0);
    store_chunk(0);
    __syncthreads();

    v4f acc[RT][NB];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[t][nb] = v4f{0.f, 0.f, 0.f, 0.f};
    float qn[NB] = {0.f, 0.f};

    for (int ch = 0; ch < nchunks; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nchunks) load_chunk(ch + 1);
        // lane (lr, lg) takes bytes [32 lg, 32 lg + 32) of every 128-byte piece of
        // a row, in the same order as k_dist_narrow (results do not depend on
        // which kernel ran)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            uint4 fa[RT][2], fb[NB][2];
#pragma unroll
            for (int t = 0; t < RT; ++t)
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    fa[t][h] = *reinterpret_cast<const uint4*>(
                        &As[buf][(wr * 16 * RT + 16 * t + lr) * SB + ks * 128 + lg * 32 + 16 * h]);
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    fb[nb][h] = *reinterpret_cast<const uint4*>(
                        &Bs[buf][(wc * 32 + 16 * nb + lr) * SB + ks * 128 + lg * 32 + 16 * h]);
            // |q|^2 of the operand values (partial over this lane's k)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const uint32_t w4[4] = {fb[nb][h].x, fb[nb][h].y, fb[nb][h].z, fb[nb][h].w};
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        if constexpr (BF16) {
                            const float lo = bf16_lo(w4[e]), hi = bf16_hi(w4[e]);
                            qn[nb] = fmaf(lo, lo, qn[nb]);
                            qn[nb] = fmaf(hi, hi, qn[nb]);
                        } else {
                            const float f = __uint_as_float(w4[e]);
                            qn[nb] = fmaf(f, f, qn[nb]);
                        }
                    }
                }
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int t = 0; t < RT; ++t)
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) {
                        v4f& c = acc[t][nb];
                        const uint4 av = fa[t][h], bv = fb[nb][h];
                        if constexpr (BF16) {
                            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(*reinterpret_cast<const v8bf*>(&av),
                                                                        *reinterpret_cast<const v8bf*>(&bv), c, 0, 0, 0);
                        } else {
                            c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(av.x), __uint_as_float(bv.x), c, 0, 0, 0);
                            c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(av.y), __uint_as_float(bv.y), c, 0, 0, 0);
                            c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(av.z), __uint_as_float(bv.z), c, 0, 0, 0);
                            c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(av.w), __uint_as_float(bv.w), c, 0, 0, 0);
                        }
                    }
        }
        if (ch + 1 < nchunks) store_chunk(buf ^ 1);
        __syncthreads();
    }

    epilogue<RT>(a, acc, qn, e_word, e_norm, row0 + wr * 16 * RT, col0 + wc * 32, lr, lg);
}

// One short query (at most 64 columns), bound by reading the corpus rows.
// The query travels in the kernel arguments (its fields, and the whole
// parameter block, which block 0 stores to device memory for the Sinkhorn
// kernel), so no upload launch and no dependent metadata loads precede the
// stream.  The block first stages the query columns in LDS, then each wave
// issues the loads of its 16 corpus rows (the whole embedding dimension) into
// registers at once and the MFMAs consume them as they arrive.  Lane (lr, lg)
// loads row lr, bytes [128 c + 32 lg, +32) of every 128-byte chunk c, so four
// lanes read one full cache line; the general kernel uses the same k order,
// so results do not depend on which kernel ran.  A query of 33..64 columns
// takes NP = 2 passes over the rows held in registers, the second with the
// next 32 columns staged in the same LDS (their loads in flight during the
// first pass), so the rows are read once.
struct NarrowArgs {
    const float* act;
    const uint16_t* act16;
    const float* norm;
    const int32_t* act_word;
    const float* vecs;
    int64_t U;
    int32_t ldv;
    float* Kt;
    float* KMt;
    float* nrow;
    float lambda, tau2;
    int32_t m, ldk, shift, km;   // km: K1 also writes KMt
    int32_t qid_word;            // word index of the query ids in blob
    int32_t pwords;              // parameter block words
    uint32_t* params;            // device parameter block
    const float* zpad;           // the corpus's zero block (1, then zeros)
    uint32_t blob[kUploadChunkBytes / 4];
};

template <bool BF16, int NC, int NP>
__global__ __launch_bounds__(256) void k_dist_narrow(NarrowArgs a) {
    constexpr int SBB = NC * 128 + 16;   // LDS column stride (bytes): 8 lanes on distinct banks
    static_assert(4 + 64 * NC <= kZpadFloats, "padded loads stay inside the zero block");
    __shared__ __attribute__((aligned(16))) char Bs[32 * SBB];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const int64_t rbase = (int64_t)blockIdx.x * TR + 16 * wave;
    const int ldv = a.ldv, m = a.m;

    if (blockIdx.x == 0)
        for (int i = tid; i < a.pwords; i += 256) a.params[i] = a.blob[i];

    // Every load of the first pass is issued before the first wait, in three
    // dependent rounds: the query ids (kernel arguments), then the query
    // column pieces and the corpus rows.  Rows beyond U read the zero block
    // and columns beyond m the first query word's row (the address is chosen,
    // not the value, so nothing is selected later).  Query columns -> LDS:
    // 16-byte pieces, 32 columns x 8 NC pieces, NC per thread.
    const auto zero = gmem(a.zpad) + 4;
    uint4 v[NC];
    const auto vecs = gmem(a.vecs);
    auto load_cols = [&](int ps) {
        int qrow[NC];
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            const int cl = 32 * ps + (tid + 256 * j) / (8 * NC);
            qrow[j] = (int32_t)a.blob[a.qid_word + (cl < m ? cl : 0)];
        }
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            const int p = tid + 256 * j;
            const int seg = p % (8 * NC);
            // a column beyond m reads the first query word's row (qrow holds
            // its id there): its products are never used (the epilogue
            // writes 0 there), and the load needs no branch
            const auto src = vecs + (int64_t)qrow[j] * ldv;
            if constexpr (BF16) {
                const float4 f0 = ld4(src + seg * 8);
                const float4 f1 = ld4(src + seg * 8 + 4);
                v[j].x = bf16_rne(f0.x) | ((uint32_t)bf16_rne(f0.y) << 16);
                v[j].y = bf16_rne(f0.z) | ((uint32_t)bf16_rne(f0.w) << 16);
                v[j].z = bf16_rne(f1.x) | ((uint32_t)bf16_rne(f1.y) << 16);
                v[j].w = bf16_rne(f1.z) | ((uint32_t)bf16_rne(f1.w) << 16);
            } else {
                const float4 f = ld4(src + seg * 4);
                v[j] = make_uint4(__float_as_uint(f.x), __float_as_uint(f.y), __float_as_uint(f.z),
                                  __float_as_uint(f.w));
            }
        }
    };
    auto store_cols = [&](void) {
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            const int p = tid + 256 * j;
            *reinterpret_cast<uint4*>(&Bs[(p / (8 * NC)) * SBB + (p % (8 * NC)) * 16]) = v[j];
        }
    };
    load_cols(0);
    // the rows' epilogue metadata, loaded before the rows themselves: the
    // barrier below waits for these loads (and, loads completing in order,
    // for every load issued before them), not for the row stream
    int e_word[4];
    float e_norm[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t gi = rbase + 4 * lg + r;
        const int64_t gc = (gi < a.U) ? gi : 0;
        const int w = a.act_word[gc];
        const float nv = a.norm[gc];
        e_word[r] = (gi < a.U) ? w : -2;
        e_norm[r] = (gi < a.U) ? nv : 0.f;
    }
    uint4 fa[NC][2];
    {
        const int64_t row = rbase + lr;
        const char* src = (row >= a.U) ? reinterpret_cast<const char*>(a.zpad + 4)
                          : BF16       ? reinterpret_cast<const char*>(a.act16 + row * ldv)
                                       : reinterpret_cast<const char*>(a.act + row * ldv);
        const auto gs = gmem(src);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const float4 f0 = ld4(reinterpret_cast<WMD_GLOBAL const float*>(gs + c * 128 + lg * 32));
            const float4 f1 = ld4(reinterpret_cast<WMD_GLOBAL const float*>(gs + c * 128 + lg * 32 + 16));
            fa[c][0] = make_uint4(__float_as_uint(f0.x), __float_as_uint(f0.y), __float_as_uint(f0.z), __float_as_uint(f0.w));
            fa[c][1] = make_uint4(__float_as_uint(f1.x), __float_as_uint(f1.y), __float_as_uint(f1.z), __float_as_uint(f1.w));
        }
    }
    store_cols();
    int qw[NP][2];
#pragma unroll
    for (int ps = 0; ps < NP; ++ps)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            const int k = 32 * ps + 16 * nb + lr;
            qw[ps][nb] = (k < m) ? (int32_t)a.blob[a.qid_word + k] : -1;
        }
    __syncthreads();
    if constexpr (NP > 1) load_cols(1);   // in flight during the first pass

    v4f acc[NP][2];
    float qn[NP][2];
#pragma unroll
    for (int ps = 0; ps < NP; ++ps) {
        if (ps > 0) {
            __syncthreads();   // every wave is done with the previous columns
            store_cols();
            __syncthreads();
        }
        acc[ps][0] = acc[ps][1] = v4f{0.f, 0.f, 0.f, 0.f};
        qn[ps][0] = qn[ps][1] = 0.f;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            uint4 fb[2][2];
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    fb[nb][h] = *reinterpret_cast<const uint4*>(&Bs[(16 * nb + lr) * SBB + c * 128 + lg * 32 + 16 * h]);
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const uint32_t w4[4] = {fb[nb][h].x, fb[nb][h].y, fb[nb][h].z, fb[nb][h].w};
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        if constexpr (BF16) {
                            const float lo = bf16_lo(w4[e]), hi = bf16_hi(w4[e]);
                            qn[ps][nb] = fmaf(lo, lo, qn[ps][nb]);
                            qn[ps][nb] = fmaf(hi, hi, qn[ps][nb]);
                        } else {
                            const float f = __uint_as_float(w4[e]);
                            qn[ps][nb] = fmaf(f, f, qn[ps][nb]);
                        }
                    }
                }
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int nb = 0; nb < 2; ++nb) {
                    v4f& cc = acc[ps][nb];
                    const uint4 av = fa[c][h], bv = fb[nb][h];
                    if constexpr (BF16) {
                        cc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(*reinterpret_cast<const v8bf*>(&av),
                                                                     *reinterpret_cast<const v8bf*>(&bv), cc, 0, 0, 0);
                    } else {
                        cc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(av.x), __uint_as_float(bv.x), cc, 0, 0, 0);
                        cc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(av.y), __uint_as_float(bv.y), cc, 0, 0, 0);
                        cc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(av.z), __uint_as_float(bv.z), cc, 0, 0, 0);
                        cc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(av.w), __uint_as_float(bv.w), cc, 0, 0, 0);
                    }
                }
        }
    }

    // epilogue (the same arithmetic as the general kernel's).  Lane (lr, lg)
    // holds rows 4 lg + r of columns 32 ps + 16 nb + lr: the wave has every
    // column of its 16 rows, so the column shift's row minimum is a reduction
    // over the 16 lanes of a row group, and K is written once (the general
    // kernel needs atomics and a second pass, as a query's columns may span
    // several blocks).
    float dv[NP][2][4];
    bool live[NP][2][4];
    float dmin[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
    // squared distances (0 for a word the query shares); the FP32 recompute
    // below tau is rare, so it runs behind one wave-wide test
    bool need = false;
#pragma unroll
    for (int ps = 0; ps < NP; ++ps)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            const float qnj = sum_lane_groups(qn[ps][nb]);
            const int k = 32 * ps + 16 * nb + lr;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = rbase + 4 * lg + r;
                live[ps][nb][r] = k < m && gi < a.U;
                const bool same = e_word[r] == qw[ps][nb];
                dv[ps][nb][r] = same ? 0.f : e_norm[r] + qnj - 2.f * acc[ps][nb][r];
                need |= live[ps][nb][r] && !same && dv[ps][nb][r] < a.tau2;
            }
        }
    if (__builtin_amdgcn_ballot_w64(need)) {
#pragma unroll
        for (int ps = 0; ps < NP; ++ps)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t gi = rbase + 4 * lg + r;
                    if (live[ps][nb][r] && e_word[r] != qw[ps][nb] && dv[ps][nb][r] < a.tau2)
                        dv[ps][nb][r] = direct_d2(a.act + gi * ldv, a.vecs + (int64_t)qw[ps][nb] * ldv, ldv);
                }
    }
#pragma unroll
    for (int ps = 0; ps < NP; ++ps)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float d = live[ps][nb][r] ? sqrtf(fmaxf(dv[ps][nb][r], 0.f)) : INFINITY;
                dv[ps][nb][r] = d;
                dmin[r] = fminf(dmin[r], d);
            }
    if (a.shift) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float t = dmin[r];
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) t = fminf(t, __shfl_xor(t, o, 64));
            dmin[r] = t;
            const int64_t gi = rbase + 4 * lg + r;
            if (lr == 0 && gi < a.U) a.nrow[gi] = t;
        }
    }
#pragma unroll
    for (int ps = 0; ps < NP; ++ps)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            const int k = 32 * ps + 16 * nb + lr;
            if (k >= a.ldk) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = rbase + 4 * lg + r;
                if (gi >= a.U) continue;
                float* kt = a.Kt + gi * a.ldk + k;
                if (!live[ps][nb][r]) {
                    *kt = 0.f;
                    if (a.km) a.KMt[gi * a.ldk + k] = 0.f;
                    continue;
                }
                const float d = dv[ps][nb][r];
                const float kv = a.shift ? expf(-a.lambda * (d - dmin[r])) : expf(-a.lambda * d);
                *kt = kv;
                if (a.km) a.KMt[gi * a.ldk + k] = kv * d;
            }
        }
}

// Log-domain shift, second pass: Kt holds d, nrow holds n_i = min_k d.
__global__ __launch_bounds__(256) void k_shift_exp(const QueryDev* qd, int64_t U) {
    const QueryDev q = qd[blockIdx.y];
    const int64_t total = U * q.ldk;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(e % q.ldk);
        if (k >= q.m) continue;
        const int64_t i = e / q.ldk;
        const float d = q.Kt[e];
        const float kv = expf(-q.lambda * (d - q.nrow[i]));
        q.Kt[e] = kv;
        if (!q.km_from_k) q.KMt[e] = kv * d;
    }
}

// The row-minimum arrays of B queries (wherever each lies) set to +inf, query
// b in grid row b.
__global__ __launch_bounds__(256) void k_fill_nrow_inf(const QueryDev* qd, int64_t U) {
    float* p = qd[blockIdx.y].nrow;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < U; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = INFINITY;
}

}  // namespace

hipError_t launch_dist(const DevCorpus& c, const QueryDev* qd, const int32_t* kofs, int B, int ncols, int bf16,
                       int shift, hipStream_t s) {
    if (B <= 0 || c.U <= 0 || ncols <= 0) return hipSuccess;
    if (c.ldv % 64 != 0) return hipErrorInvalidValue;   // whole chunks
    hipError_t e;
    if (shift && (e = launch_kernel(k_fill_nrow_inf, dim3((unsigned)std::min<int64_t>((c.U + 255) / 256, 1024),
                                                          (unsigned)B),
                                    dim3(256), 0, s, qd, c.U)) != hipSuccess)
        return e;
    DistArgs a;
    a.act = c.act;
    a.act16 = c.act_bf16;
    a.norm = bf16 ? c.act_norm_bf16 : c.act_norm;
    a.act_word = c.act_word;
    a.vecs = c.vecs;
    a.qd = qd;
    a.kofs = kofs;
    a.U = c.U;
    a.ldv = c.ldv;
    a.B = B;
    a.ncols = ncols;
    const int tc = ncols <= 32 ? 32 : 64;
    const int64_t tiles_r = (c.U + TR - 1) / TR;
    a.tiles_c = (ncols + tc - 1) / tc;
    const int64_t nblocks = tiles_r * a.tiles_c;
    if (nblocks > INT32_MAX) return hipErrorInvalidValue;
    a.nblocks = (int32_t)nblocks;
    // FP32 rows are 4 * ldv bytes (a multiple of 256), BF16 rows 2 * ldv (of 128)
    auto kern = tc == 32 ? (bf16 ? k_dist<true, 32, 128> : k_dist<false, 32, 256>)
                         : (bf16 ? k_dist<true, 64, 128> : k_dist<false, 64, 128>);
    if ((e = launch_kernel(kern, dim3((unsigned)nblocks), dim3(256), 0, s, a)) != hipSuccess || !shift) return e;
    const int64_t per_q = (c.U * 64 + 255) / 256;
    return launch_kernel(k_shift_exp, dim3((unsigned)std::min<int64_t>(per_q, 2048), (unsigned)B), dim3(256), 0, s,
                         qd, c.U);
}

bool dist_narrow_fits(const DevCorpus& c, int bf16, int B, int ncols, size_t pbytes) {
    (void)bf16;   // FP32 rows are ldv / 32 chunks of 128 bytes (even), BF16 rows ldv / 64: at most 12 and 6
    return B == 1 && ncols <= 64 && c.ldv >= 64 && c.ldv <= 384 && c.ldv % 64 == 0 &&
           pbytes <= (size_t)kUploadChunkBytes && pbytes % 4 == 0 && (c.U + TR - 1) / TR <= INT32_MAX;
}

hipError_t launch_dist_narrow(const DevCorpus& c, const QueryDev& hq, const void* blob,
                              size_t pbytes, size_t off_id, void* params_dev, int bf16, hipStream_t s) {
    NarrowArgs a;
    a.act = c.act;
    a.act16 = c.act_bf16;
    a.norm = bf16 ? c.act_norm_bf16 : c.act_norm;
    a.act_word = c.act_word;
    a.vecs = c.vecs;
    a.U = c.U;
    a.ldv = c.ldv;
    a.Kt = hq.Kt;
    a.KMt = hq.KMt;
    a.nrow = hq.nrow;
    a.lambda = hq.lambda;
    a.tau2 = hq.tau2;
    a.m = hq.m;
    a.ldk = hq.ldk;
    a.shift = hq.shift;
    a.km = hq.km_from_k ? 0 : 1;
    a.qid_word = (int32_t)(off_id / 4);
    a.pwords = (int32_t)(pbytes / 4);
    a.params = static_cast<uint32_t*>(params_dev);
    a.zpad = c.zpad;
    std::memset(a.blob, 0, sizeof a.blob);
    std::memcpy(a.blob, blob, pbytes);
    hipError_t e;
    const int nc = c.ldv * (bf16 ? 2 : 4) / 128;
    const unsigned blocks = (unsigned)((c.U + TR - 1) / TR);
    const bool two = hq.ldk > 32;   // a second pass over the next 32 columns
#define WMD_NARROW(B16, K)                                                                            \
    case K:                                                                                           \
        e = launch_kernel(two ? k_dist_narrow<B16, K, 2> : k_dist_narrow<B16, K, 1>, dim3(blocks), dim3(256), \
                          0, s, a);                                                                   \
        break;
    if (bf16) {
        switch (nc) {
            WMD_NARROW(true, 1) WMD_NARROW(true, 2) WMD_NARROW(true, 3) WMD_NARROW(true, 4) WMD_NARROW(true, 5)
            WMD_NARROW(true, 6)
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (nc) {
            WMD_NARROW(false, 2) WMD_NARROW(false, 4) WMD_NARROW(false, 6) WMD_NARROW(false, 8)
            WMD_NARROW(false, 10) WMD_NARROW(false, 12)
            default: return hipErrorInvalidValue;
        }
    }
#undef WMD_NARROW
    return e;
}

}  // namespace wmd
