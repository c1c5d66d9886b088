// The Sinkhorn iteration of Algorithm 1 carried in the log domain, for lambda
// beyond the range of K = exp(-lambda M) (FP32: lambda M > ~87, FP64: > ~745).
//
// With lu = log u, lv = log v and log K = -lambda M, the iteration of the
// sparse form (Sec. 4) becomes, per document:
//   lv_i = log c_i - LSE_k(lu_k - lambda M[k, i])         (SDDMM at the nonzeros)
//   lu_k = log r_k - LSE_i(lv_i - lambda M[k, i])         (SpMM, then u = 1/x)
// with LSE_j(a_j) = max_j a + log sum_j exp(a_j - max_j a), and x = 1/v_r at
// the start (lu = log v_r).  The final step needs no large exponent at all:
// with w_ik = exp(lu_k - lambda M[k, i] - max_k(...)) the document's share of
// row i is v_i sum_k u_k K_ki M_ki = c_i (sum_k w_ik M_ki) / (sum_k w_ik).
//
// Precision: the distances are FP64 (direct differences of the FP32 rows, as
// the definition writes them), the potentials lu, lv, the exponent arguments
// and the maxima are FP64; only exp(a - max) (a non-positive argument, so the
// terms that matter have small magnitude) and the sums of those terms are
// FP32.  FP32 distances would not do: lambda times their rounding error is
// already ~1e-4 at lambda = 1000.
#include "wmd_device.h"
#include "launch.h"
#include "wmd_internal.h"

namespace wmd {

namespace {

constexpr int kRows = 256;     // corpus rows per distance block (one per thread)
constexpr int kCols = 32;      // query columns per distance block (all in each thread)
constexpr double kLog2e = 1.4426950408889634;

struct LseDistArgs {
    const float* act;          // U x ldv FP32 corpus rows (zero padded)
    const float* vecs;         // V x ldv FP32 vocabulary rows (zero padded)
    const QueryDev* qd;        // B queries; Kt of each holds U x ldk doubles here
    const int32_t* kofs;       // B + 1: first global column of each query
    int64_t U;
    int32_t ldv;
    int32_t B;
    int32_t ncols;             // kofs[B]
};

// the query of global column c: the largest b with kofs[b] <= c
__device__ int query_of_col(const int32_t* kofs, int B, int c) {
    int lo = 0, hi = B - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (kofs[mid] <= c) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// d[i, c] = sqrt(sum_d (E[word(i), d] - E[qid(c), d])^2) in FP64 for kRows
// corpus rows x kCols global query columns per block: thread t takes corpus
// row t (streamed from memory, its own row per lane) against all kCols
// columns, whose query rows are staged in LDS (FP32, row stride ldv + 4) and
// read as broadcasts.  Columns m_b <= k < ldk_b are written as zeros.  32
// columns per block (one whole query of up to 32 words) read each corpus row
// once per query where 8 read it four times (20000 documents of 10-60 words,
// lambda 1000: 4.8e8 -> 6.3e8 doc*iters/s).
__global__ __launch_bounds__(kRows) void k_dist_lse(LseDistArgs a) {
    extern __shared__ float4 qsh4[];
    float* qsh = reinterpret_cast<float*>(qsh4);
    __shared__ int64_t qrow[kCols];     // vocabulary row of each column, -1 for padding
    __shared__ int qb[kCols], qk[kCols];
    const int tid = threadIdx.x;
    const int c0 = blockIdx.y * kCols;
    const int stride = a.ldv + 4;
    if (tid < kCols) {
        const int c = c0 + tid;
        int64_t row = -1;
        int b = 0, k = 0;
        if (c < a.ncols) {
            b = query_of_col(a.kofs, a.B, c);
            k = c - a.kofs[b];
            if (k < a.qd[b].m) row = a.qd[b].qid[k];
        }
        qrow[tid] = row;
        qb[tid] = b;
        qk[tid] = k;
    }
    __syncthreads();
    const int q4 = a.ldv / 4;
    for (int p = tid; p < kCols * q4; p += kRows) {
        const int cc = p / q4, e = p % q4;
        const int64_t row = qrow[cc];
        const float4 v = row >= 0 ? ld4(gmem(a.vecs) + row * a.ldv + 4 * e) : make_float4(0.f, 0.f, 0.f, 0.f);
        *reinterpret_cast<float4*>(qsh + cc * stride + 4 * e) = v;
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kRows + tid;
    const auto arow = gmem(a.act) + (i < a.U ? i : 0) * a.ldv;   // rows beyond U read row 0, not stored
    double acc[kCols];
#pragma unroll
    for (int j = 0; j < kCols; ++j) acc[j] = 0.0;
    for (int e = 0; e < q4; ++e) {
        const float4 x = ld4(arow + 4 * e);
#pragma unroll
        for (int j = 0; j < kCols; ++j) {
            const float4 y = *reinterpret_cast<const float4*>(qsh + j * stride + 4 * e);
            const double d0 = (double)x.x - (double)y.x, d1 = (double)x.y - (double)y.y;
            const double d2 = (double)x.z - (double)y.z, d3 = (double)x.w - (double)y.w;
            acc[j] = fma(d0, d0, acc[j]);
            acc[j] = fma(d1, d1, acc[j]);
            acc[j] = fma(d2, d2, acc[j]);
            acc[j] = fma(d3, d3, acc[j]);
        }
    }
    if (i < a.U) {
#pragma unroll
        for (int j = 0; j < kCols; ++j) {
            if (c0 + j < a.ncols) {
                const QueryDev& q = a.qd[qb[j]];
                double* D = reinterpret_cast<double*>(q.Kt);
                gmem(D)[i * q.ldk + qk[j]] = qrow[j] >= 0 ? sqrt(acc[j]) : 0.0;
            }
        }
    }
}

// independent chains per pass of a log-sum-exp
constexpr int kLseChains = 8;

// Two-pass log-sum-exp in base 2 of a_j = base(j) - lam2 dist(j), j < len,
// shared by a group of G consecutive lanes (G a power of two): lane j0 of the
// group takes j = j0, j0 + G, ...  Returns the maximum and the FP32 sum of
// 2^(a_j - max) (with want_sd also the FP64 sum of those terms times
// dist(j)), combined over the group with xor shuffles so every lane of the
// group holds the same values.  kLseChains independent chains per pass keep
// the loop from waiting on each maximum or sum.  Every lane of the wave must call
// it (the shuffles).
template <typename Base, typename Dist>
__device__ __forceinline__ double lse2(int len, int j0, int G, double lam2, Base base, Dist dist, float& s_out,
                                       bool want_sd, double& sd_out) {
    constexpr int NCH = kLseChains;
    double mc[NCH];
#pragma unroll
    for (int h = 0; h < NCH; ++h) mc[h] = -INFINITY;
    int j = j0;
    for (; j + (NCH - 1) * G < len; j += NCH * G) {
#pragma unroll
        for (int h = 0; h < NCH; ++h) mc[h] = fmax(mc[h], fma(-lam2, dist(j + h * G), base(j + h * G)));
    }
    for (; j < len; j += G) mc[0] = fmax(mc[0], fma(-lam2, dist(j), base(j)));
#pragma unroll
    for (int w = NCH / 2; w >= 1; w /= 2) {
#pragma unroll
        for (int h = 0; h < w; ++h) mc[h] = fmax(mc[h], mc[h + w]);
    }
    double mx = mc[0];
    for (int o = 1; o < G; o <<= 1) mx = fmax(mx, __shfl_xor(mx, o));
    float s[NCH];
    double sd[NCH];
#pragma unroll
    for (int h = 0; h < NCH; ++h) {
        s[h] = 0.f;
        sd[h] = 0.0;
    }
    j = j0;
    for (; j + (NCH - 1) * G < len; j += NCH * G) {
#pragma unroll
        for (int h = 0; h < NCH; ++h) {
            const double dj = dist(j + h * G);
            const float w = __builtin_amdgcn_exp2f((float)(fma(-lam2, dj, base(j + h * G)) - mx));
            s[h] += w;
            if (want_sd) sd[h] = fma((double)w, dj, sd[h]);
        }
    }
    for (; j < len; j += G) {
        const double dj = dist(j);
        const float w = __builtin_amdgcn_exp2f((float)(fma(-lam2, dj, base(j)) - mx));
        s[0] += w;
        if (want_sd) sd[0] = fma((double)w, dj, sd[0]);
    }
#pragma unroll
    for (int w = NCH / 2; w >= 1; w /= 2) {
#pragma unroll
        for (int h = 0; h < w; ++h) {
            s[h] += s[h + w];
            sd[h] += sd[h + w];
        }
    }
    float st = s[0];
    double sdt = sd[0];
    for (int o = 1; o < G; o <<= 1) {
        st += __shfl_xor(st, o);
        if (want_sd) sdt += __shfl_xor(sdt, o);
    }
    s_out = st;
    sd_out = sdt;
    return mx;
}

// lanes per log-sum-exp for `items` of them in a wave: 64 over the items
// rounded up to a power of two, at most 8
__device__ __forceinline__ int lse_group(int items) {
    int p = 1;
    while (p < items) p <<= 1;
    const int g = 64 / p;
    return g < 1 ? 1 : (g > 8 ? 8 : g);
}

// LDS of one (query, document) pair: lu[m], lr[m] = log r, lv[n], lc[n] =
// log c (doubles), then col[n] (ints); with STAGED also the document's
// distance block, column-major with an odd stride (both phases read it
// without bank conflicts).
__host__ __device__ inline int lse_stride(int n) { return n | 1; }

__host__ __device__ inline size_t lse_lds_doubles(int m, int n, bool staged) {
    return 2 * (size_t)m + 2 * (size_t)n + (n + 1) / 2 + (staged ? (size_t)m * lse_stride(n) : 0);
}

// One wave per (query, document).  Each lane owns a whole row in the row
// phase and a whole column in the column phase, so no cross-lane reduction
// is needed; each log-sum-exp takes two passes (the maximum, then the sum of
// FP32 exponentials below it).
template <bool STAGED>
__global__ __launch_bounds__(64) void k_sink_lse(SinkArgs g) {
    extern __shared__ double sm[];
    const int lane = threadIdx.x;
    const int64_t item = blockIdx.x;
    const int nd = g.d_end - g.d_begin;
    const int qidx = g.qlist[item / nd];
    const int d = g.d_begin + (int)(item % nd);
    const QueryDev* qp = g.qd + qidx;
    const int m = qp->m, ldk = qp->ldk;
    const double lam = qp->lambda;
    const auto D = gmem(reinterpret_cast<const double*>(qp->Kt));
    const int rs = g.sptr[d], n = g.sptr[d + 1] - rs;
    const int S = lse_stride(n);
    // the potentials are kept in base 2: lu = log2 u, lv = log2 v, and
    // lam2 = lambda log2(e), so every exponential is a plain 2^x
    const double lam2 = lam * kLog2e;
    double* lu = sm;
    double* lr = lu + m;
    double* lv = lr + m;
    double* lc = lv + n;
    int* col = reinterpret_cast<int*>(lc + n);
    double* Ds = reinterpret_cast<double*>(col) + (n + 1) / 2;   // STAGED: Ds[k * S + i]
    const auto rq = gmem(qp->r);
    for (int k = lane; k < m; k += 64) {
        lr[k] = log2((double)rq[k]);
        lu[k] = log2((double)m);          // x = 1/v_r, u = 1/x
    }
    for (int i = lane; i < n; i += 64) {
        lc[i] = log2((double)g.scw[rs + i]);
        col[i] = g.scol[rs + i];
    }
    __syncthreads();
    if constexpr (STAGED) {
        for (int p = lane; p < n * m; p += 64) {
            const int i = p / m, k = p % m;
            Ds[k * S + i] = D[(int64_t)col[i] * ldk + k];
        }
        __syncthreads();
    }
    auto dist = [&](int i, int k) -> double {
        if constexpr (STAGED) return Ds[k * S + i];
        else return D[(int64_t)col[i] * ldk + k];
    };

    // row i: lv_i = log2 c_i - LSE2_k(lu_k - lam2 d_ik); on the final pass
    // c_i (sum_k w_ik d_ik) / (sum_k w_ik) instead, summed over the lane's rows.
    // Gr lanes per row (Gc per column below), so short documents and queries
    // still keep most of the wave busy.
    const int Gr = lse_group(n), Gc = lse_group(m);
    auto rows = [&](bool final) -> double {
        double wsum = 0.0;
        for (int i0 = 0; i0 < n; i0 += 64 / Gr) {
            const int i = i0 + lane / Gr;
            const bool ok = i < n;
            const int ic = ok ? i : 0;
            float s;
            double sd;
            const double mx = lse2(m, lane % Gr, Gr, lam2, [&](int k) { return lu[k]; },
                                   [&](int k) { return dist(ic, k); }, s, final, sd);
            if (ok && lane % Gr == 0) {
                if (final) wsum += (double)g.scw[rs + i] * sd / (double)s;
                else lv[i] = lc[i] - (mx + log2((double)s));
            }
        }
        return wsum;
    };
    // column k: lu_k = log2 r_k - LSE2_i(lv_i - lam2 d_ik); with resid,
    // sum_k |P1_k - r_k| where P1_k = 2^(lu_k + LSE2_i(...))
    auto cols = [&](bool resid) -> double {
        double rsum = 0.0;
        for (int k0 = 0; k0 < m; k0 += 64 / Gc) {
            const int k = k0 + lane / Gc;
            const bool ok = k < m;
            const int kc = ok ? k : 0;
            float s;
            double sd;
            const double mx = lse2(n, lane % Gc, Gc, lam2, [&](int i) { return lv[i]; },
                                   [&](int i) { return dist(i, kc); }, s, false, sd);
            const double l = mx + log2((double)s);
            if (ok && lane % Gc == 0) {
                if (resid) rsum += fabs(exp2(lu[k] + l) - (double)rq[k]);
                else lu[k] = lr[k] - l;
            }
        }
        return rsum;
    };

    for (int it = 0; it < qp->iters; ++it) {
        rows(false);
        __syncthreads();
        cols(false);
        __syncthreads();
    }
    if (qp->resid) {      // the final v, for the residual's column sums
        rows(false);
        __syncthreads();
    }
    double wsum = rows(true);
    double rsum = qp->resid ? cols(true) : 0.0;
    for (int o = 32; o >= 1; o >>= 1) {
        wsum += __shfl_xor(wsum, o);
        rsum += __shfl_xor(rsum, o);
    }
    if (lane == 0) {
        const int doc = g.sdoc[d];
        gmem(qp->out)[doc] = wsum;
        if (qp->resid) gmem(qp->resid)[doc] = rsum;
        if (qp->it_out) gmem(qp->it_out)[doc] = qp->iters;
    }
}

// Register tiles: one wave per (query, document) with the document's whole
// block of scaled distances L[i][k] = lambda log2(e) d(i, k) in registers
// (FP64), read from memory once.  Lane (a, b) of the R x C wave holds rows
// i = a + R p (p < P) and columns k = Q b + q (q < Q); the potentials of its
// rows (lv) and columns (lu) are kept by every lane that needs them.  A row's
// log-sum-exp is formed over its Q columns in each lane and combined over
// the C lanes of the row group (lane bits 0 .. log2 C - 1) with xor
// shuffles, a column's over its P rows and the R row lanes (the remaining
// lane bits), so both partners of every step get the same bits and the
// copies agree.  Rows and columns beyond the block hold a large finite L
// (their terms underflow to 0 and 0 * L stays 0), and their potentials are
// kept at 0.  The arithmetic is the stream kernel's: FP64 exponent
// arguments and maxima, FP32 2^(a - max) and sums; log2 of the sums in FP32
// (an error below 4e-7 in a potential).
constexpr double kPadL = 1e300;

// One butterfly step over lane bit log2(O): each lane combines its value with
// that of lane ^ O (DPP moves within a 16-lane row for O <= 8, the gfx950
// permlane swaps for 16 and 32), so both partners get the same bits.
template <int O>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v) {
    static_assert(O == 1 || O == 2 || O == 4 || O == 8, "DPP offsets");
    const int i = (int)v;
    if constexpr (O == 1) return (uint32_t)__builtin_amdgcn_update_dpp(i, i, 0xB1, 0xF, 0xF, false);
    else if constexpr (O == 2) return (uint32_t)__builtin_amdgcn_update_dpp(i, i, 0x4E, 0xF, 0xF, false);
    else if constexpr (O == 8) return (uint32_t)__builtin_amdgcn_update_dpp(i, i, 0x128, 0xF, 0xF, false);
    else {
        // banks 0 and 2 (lanes 0-3, 8-11 of a row) read lane + 4, banks 1 and 3 lane - 4
        int t = __builtin_amdgcn_update_dpp(i, i, 0x104, 0xF, 0x5, false);
        t = __builtin_amdgcn_update_dpp(t, i, 0x114, 0xF, 0xA, false);
        return (uint32_t)t;
    }
}

template <int O, bool MAX>
__device__ __forceinline__ double xstep(double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)u, hi = (uint32_t)(u >> 32);
    double x, y;
    if constexpr (O <= 8) {
        x = v;
        y = __longlong_as_double((long long)(((uint64_t)xor_lane<O>(hi) << 32) | xor_lane<O>(lo)));
    } else {
        auto rl = (O == 16) ? __builtin_amdgcn_permlane16_swap(lo, lo, false, false)
                            : __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        auto rh = (O == 16) ? __builtin_amdgcn_permlane16_swap(hi, hi, false, false)
                            : __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        x = __longlong_as_double((long long)(((uint64_t)rh[0] << 32) | rl[0]));
        y = __longlong_as_double((long long)(((uint64_t)rh[1] << 32) | rl[1]));
    }
    return MAX ? fmax(x, y) : x + y;
}

template <int O, bool MAX>
__device__ __forceinline__ float xstep(float v) {
    const uint32_t u = __float_as_uint(v);
    float x, y;
    if constexpr (O <= 8) {
        x = v;
        y = __uint_as_float(xor_lane<O>(u));
    } else {
        auto r = (O == 16) ? __builtin_amdgcn_permlane16_swap(u, u, false, false)
                           : __builtin_amdgcn_permlane32_swap(u, u, false, false);
        x = __uint_as_float(r[0]);
        y = __uint_as_float(r[1]);
    }
    return MAX ? fmaxf(x, y) : x + y;
}

// all-reduce over the G lanes at stride LO (lane bits log2 LO .. log2 LO G - 1)
template <int G, int LO, bool MAX, typename T>
__device__ __forceinline__ T xred(T v) {
    if constexpr (G > 1) {
        v = xstep<LO, MAX>(v);
        return xred<G / 2, LO * 2, MAX>(v);
    } else {
        return v;
    }
}

// One document with PN rows per lane (PN = ceil(n / R), chosen per wave: a
// wave holds one document, so rows beyond it cost nothing).
template <int R, int C, int PN, int Q>
__device__ __forceinline__ void lse_tile_doc(const SinkArgs& g, const QueryDev* qp, const int d, const int rs,
                                             const int n, const int lane) {
    const int a = lane / C, b = lane % C;
    const int m = qp->m, ldk = qp->ldk;
    const double lam2 = (double)qp->lambda * kLog2e;
    const auto D = gmem(reinterpret_cast<const double*>(qp->Kt));
    const int kb = Q * b;

    double L[PN][Q];
    double lv[PN], lc[PN];
    float cw[PN];
    bool rv[PN];
#pragma unroll
    for (int p = 0; p < PN; ++p) {
        const int i = a + R * p;
        rv[p] = i < n;
        const int e = rs + (rv[p] ? i : 0);
        const int col = g.scol[e];
        cw[p] = rv[p] ? g.scw[e] : 0.f;
        const auto row = D + (int64_t)col * ldk;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int k = kb + q;
            const double dv = row[k < m ? k : 0];
            L[p][q] = (rv[p] && k < m) ? lam2 * dv : kPadL;
        }
    }
    const auto rq = gmem(qp->r);
    double lu[Q], lr[Q];
    bool cv[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int k = kb + q;
        cv[q] = k < m;
        const float r = rq[cv[q] ? k : 0];
        lr[q] = cv[q] ? log2((double)r) : 0.0;
        lu[q] = cv[q] ? log2((double)m) : 0.0;   // x = 1/v_r, u = 1/x
    }
#pragma unroll
    for (int p = 0; p < PN; ++p) {
        lc[p] = rv[p] ? log2((double)cw[p]) : 0.0;
        lv[p] = 0.0;
    }

    // rows: lv_i = log2 c_i - LSE2_k(lu_k - L_ik); final: c_i (sum_k w_ik d_ik) / (sum_k w_ik)
    auto rows = [&](bool final) -> double {
        double wsum = 0.0;
#pragma unroll
        for (int p = 0; p < PN; ++p) {
            double mx = -INFINITY;
#pragma unroll
            for (int q = 0; q < Q; ++q) mx = fmax(mx, lu[q] - L[p][q]);
            mx = xred<C, 1, true>(mx);
            float sv = 0.f;
            double sd = 0.0;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const float w = __builtin_amdgcn_exp2f((float)((lu[q] - L[p][q]) - mx));
                sv += w;
                if (final) sd = fma((double)w, L[p][q], sd);
            }
            sv = xred<C, 1, false>(sv);
            if (final) {
                sd = xred<C, 1, false>(sd);
                if (rv[p] && b == 0) wsum += (double)cw[p] * (sd / lam2) / (double)sv;
            } else {
                lv[p] = rv[p] ? lc[p] - (mx + (double)__log2f(sv)) : 0.0;
            }
        }
        return wsum;
    };
    // columns: lu_k = log2 r_k - LSE2_i(lv_i - L_ik); with resid,
    // sum_k |P1_k - r_k| where P1_k = 2^(lu_k + LSE2_i(...))
    auto cols = [&](bool resid) -> double {
        double rsum = 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            double mx = -INFINITY;
#pragma unroll
            for (int p = 0; p < PN; ++p) mx = fmax(mx, lv[p] - L[p][q]);
            mx = xred<R, C, true>(mx);
            float sv = 0.f;
#pragma unroll
            for (int p = 0; p < PN; ++p) sv += __builtin_amdgcn_exp2f((float)((lv[p] - L[p][q]) - mx));
            sv = xred<R, C, false>(sv);
            const double l = mx + (double)__log2f(sv);
            if (resid) {
                if (cv[q] && a == 0) rsum += fabs(exp2(lu[q] + l) - (double)rq[kb + q]);
            } else {
                lu[q] = cv[q] ? lr[q] - l : 0.0;
            }
        }
        return rsum;
    };

    for (int it = 0; it < qp->iters; ++it) {
        rows(false);
        cols(false);
    }
    if (qp->resid) rows(false);   // the final v, for the residual's column sums
    double wsum = rows(true);
    double rsum = qp->resid ? cols(true) : 0.0;
    wsum = xred<64, 1, false>(wsum);
    rsum = xred<64, 1, false>(rsum);
    if (lane == 0) {
        const int doc = g.sdoc[d];
        gmem(qp->out)[doc] = wsum;
        if (qp->resid) gmem(qp->resid)[doc] = rsum;
        if (qp->it_out) gmem(qp->it_out)[doc] = qp->iters;
    }
}

template <int R, int C, int P, int Q, int PN>
__device__ __forceinline__ void lse_tile_dispatch(int pr, const SinkArgs& g, const QueryDev* qp, int d, int rs,
                                                  int n, int lane) {
    if constexpr (PN >= P) {
        lse_tile_doc<R, C, P, Q>(g, qp, d, rs, n, lane);
    } else {
        if (pr <= PN) lse_tile_doc<R, C, PN, Q>(g, qp, d, rs, n, lane);
        else lse_tile_dispatch<R, C, P, Q, PN + 1>(pr, g, qp, d, rs, n, lane);
    }
}

template <int R, int C, int P, int Q>
__global__ __launch_bounds__(64) void k_sink_lse_tile(SinkArgs g) {
    static_assert(R * C == 64, "one wave per document");
    const int lane = threadIdx.x;
    const int64_t item = blockIdx.x;
    const int nd = g.d_end - g.d_begin;
    const int qidx = g.single ? 0 : g.qlist[item / nd];
    const int d = g.d_begin + (int)(item % nd);
    const QueryDev* qp = g.qd + qidx;
    const int rs = g.sptr[d], n = g.sptr[d + 1] - rs;
    // the wave's document is uniform: rows per lane as an SGPR
    const int pr = __builtin_amdgcn_readfirstlane((n + R - 1) / R);
    lse_tile_dispatch<R, C, P, Q, 1>(pr, g, qp, d, rs, n, lane);
}

}  // namespace

hipError_t launch_sinkhorn_lse_tile(const SinkArgs& a, hipStream_t s) {
    const int64_t nitems = (int64_t)a.nq * (a.d_end - a.d_begin);
    if (nitems <= 0) return hipSuccess;
    return launch_kernel(k_sink_lse_tile<8, 8, 8, 5>, dim3((unsigned)nitems), dim3(64), 0, s, a);
}

size_t lse_dist_lds_bytes(int ldv) { return sizeof(float) * (size_t)kCols * (ldv + 4); }

// the documents' distance blocks are staged in LDS when every pair of the
// launch fits in this much
constexpr size_t kStageLds = 48 * 1024;

size_t lse_sink_lds_bytes(int max_m, int max_n) {
    const size_t staged = sizeof(double) * lse_lds_doubles(max_m, max_n, true);
    return staged <= kStageLds ? staged : sizeof(double) * lse_lds_doubles(max_m, max_n, false);
}

hipError_t launch_dist_lse(const DevCorpus& c, const QueryDev* qd, const int32_t* kofs, int B, int ncols,
                           hipStream_t s) {
    LseDistArgs a;
    a.act = c.act;
    a.vecs = c.vecs;
    a.qd = qd;
    a.kofs = kofs;
    a.U = c.U;
    a.ldv = c.ldv;
    a.B = B;
    a.ncols = ncols;
    const size_t lds = lse_dist_lds_bytes(c.ldv);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)k_dist_lse, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const dim3 grid((unsigned)((c.U + kRows - 1) / kRows), (unsigned)((ncols + kCols - 1) / kCols));
    return launch_kernel(k_dist_lse, grid, dim3(kRows), (uint32_t)lds, s, a);
}

hipError_t launch_sinkhorn_lse(const SinkArgs& a, int max_m, int max_n, hipStream_t s) {
    const int64_t nitems = (int64_t)a.nq * (a.d_end - a.d_begin);
    if (nitems <= 0) return hipSuccess;
    const size_t lds = lse_sink_lds_bytes(max_m, max_n);
    const bool staged = sizeof(double) * lse_lds_doubles(max_m, max_n, true) <= kStageLds;
    const void* kern = staged ? (const void*)k_sink_lse<true> : (const void*)k_sink_lse<false>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return launch_kernel(staged ? k_sink_lse<true> : k_sink_lse<false>, dim3((unsigned)nitems), dim3(64),
                         (uint32_t)lds, s, a);
}

}  // namespace wmd
