// Fused Sinkhorn iterations and final WMD step, one team of lanes per
// (query, document) pair.
//
// The paper's dense-to-sparse transformation (Sec. 4) evaluates K^T u only at
// the nonzeros of c (SDDMM) and fuses it with x = diag(1/r) K v (SpMM) into
// one pass over the nonzeros ("SDDMM_SpMM").  Column j of x depends only on
// column j of x and of c, so every document is an independent small Sinkhorn
// problem on the n_j x v_r block A = Kt[words(j), :].  Here one team owns one
// document: it loads A into registers once and runs every iteration and the
// final step on it, so c, the gathered K block and x never travel to memory
// between iterations.
//
// Per team of R x C lanes (lane (a, b)), lane (a, b) holds
//   A[a + R p][kb + q] for p < P, q < Q, with kb = (wave-in-team * C + b) * Q,
// i.e. rows strided over a and a contiguous block of Q columns per b.
//   u     = 1 / x                        (formed on the column's owner lane,
//                                         then copied to every a)
//   s_i   = sum_k A[i][k] u_k            (partial over q, then summed over b)
//   v_i   = c_i / s_i                    (rows; every b holds a copy)
//   x_k   = (1 / r_k) sum_i A[i][k] v_i  (partial over p, then reduce-scattered
//                                         over a: each column's sum, x and u
//                                         are formed on one owner lane)
// Teams with R <= Q and C < 16 pass the column partial sums and u through
// LDS (each lane stores its partials, the owner of a column adds them in
// row-lane order, stores u, and every lane reads its columns' u back); the
// others use lane shuffles (permlane swaps and DPP), as do the row sums.
// Final: u = 1/x, v = c / (A u), WMD = sum_{i,k} ((K .* M)[i][k] u_k) v_i with
// the products and each lane's sum over its (at most 8) columns of a row in
// FP32 and the sum beyond in FP64, where K .* M is rebuilt from the
// K block already in registers (M = n_i - ln K / lambda, n_i the row's
// log-domain shift or 0) for lambda >= 0.5, else gathered from KMt; the
// absolute error of the rebuilt M is about ulp(lambda M) / lambda, so its
// relative error stays at FP32 rounding level.  Optionally the FP64 residual
// sum_k |u_k (A^T v)_k - r_k| of the plan's row marginal (its column marginal
// is c by construction).
#include <atomic>

#include "wmd_device.h"
#include "launch.h"
#include "wmd_internal.h"

// No implicit multiply-add contraction in this file: every fused operation is
// an explicit fmaf/fma.  The lane-exchange sums rely on both partners of a
// butterfly adding the same two rounded values; a product contracted into the
// exchange add (fma(a, b, partner) on one lane, fma(a', b', mine) on the other)
// would give the copies different bits.
#pragma clang fp contract(off)

namespace wmd {

namespace {

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// v of lane k of this lane's quad (k a compile-time constant after unrolling)
__device__ __forceinline__ float quad_bcast(float v, int k) {
    switch (k) {
        case 0: return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x00, 0xF, 0xF, true));
        case 1: return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x55, 0xF, 0xF, true));
        case 2: return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xAA, 0xF, 0xF, true));
        default: return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xFF, 0xF, 0xF, true));
    }
}

// lane ^ 16 and lane ^ 32 partner sums with the gfx950 row-swap VALU ops:
// with both operands = v, the two results hold v of this lane and of its
// partner, in the same order on both lanes, so both get identical bits.
__device__ __forceinline__ float add_xor16(float v) {
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float add_xor32(float v) {
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// lane ^ 4 within each 16-lane row: row_shl:4 into banks 0 and 2 (lanes 0-3,
// 8-11), row_shr:4 into banks 1 and 3.
__device__ __forceinline__ float xor4(float v) {
    const int i = __float_as_int(v);
    int t = __builtin_amdgcn_update_dpp(i, i, 0x104, 0xF, 0x5, false);
    t = __builtin_amdgcn_update_dpp(t, i, 0x114, 0xF, 0xA, false);
    return __int_as_float(t);
}

template <int C>
__device__ __forceinline__ float sum_over_b(float v) {
    if constexpr (C >= 2) v += dpp<0xB1>(v);    // quad_perm [1,0,3,2]: lane ^ 1
    if constexpr (C >= 4) v += dpp<0x4E>(v);    // quad_perm [2,3,0,1]: lane ^ 2
    if constexpr (C >= 8) v += dpp<0x141>(v);   // row_half_mirror: the other quad (quads uniform)
    if constexpr (C >= 16) v += dpp<0x140>(v);  // row_mirror: the other half-row (halves uniform)
    return v;
}

// Sum over the R lanes with the same b (lane stride C) of an R*C-lane team.
// Every step pairs lane l with lane l ^ o; IEEE addition is commutative, so
// both partners get the same bits and the R copies of x stay identical.
// sum_over_b for K values at once, step-major so that no DPP op reads a
// value written by the instruction just before it
template <int C, int K>
__device__ __forceinline__ void sum_over_b_n(float* v) {
    if constexpr (C >= 2) {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] += dpp<0xB1>(v[k]);
    }
    if constexpr (C >= 4) {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] += dpp<0x4E>(v[k]);
    }
    if constexpr (C >= 8) {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] += dpp<0x141>(v[k]);
    }
    if constexpr (C >= 16) {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] += dpp<0x140>(v[k]);
    }
}

template <int R, int C>
__device__ __forceinline__ float sum_over_a(float v) {
    constexpr int T = R * C;
    if constexpr (C <= 1 && T > 1) v += dpp<0xB1>(v);    // lane ^ 1
    if constexpr (C <= 2 && T > 2) v += dpp<0x4E>(v);    // lane ^ 2
    if constexpr (C <= 4 && T > 4) v += xor4(v);         // lane ^ 4
    if constexpr (C <= 8 && T > 8) v += dpp<0x128>(v);   // row_ror:8 == lane ^ 8 within a row
    if constexpr (T > 16) v = add_xor16(v);              // lane ^ 16
    if constexpr (T > 32) v = add_xor32(v);              // lane ^ 32
    return v;
}

// (K .* M) of a kernel value kk = exp(-lambda (M - n)): kk (n - ln(kk) / lambda),
// with log2(kk) = exponent + log2(mantissa) (the hardware log2 flushes
// denormal inputs; the mantissa is always normal, so denormal kk are exact),
// and kk = 0 giving 0.  c = ln 2 / lambda.  The absolute error of the rebuilt
// M is about ulp(lambda M) / lambda, so its relative error stays at FP32
// rounding level.
__device__ __forceinline__ float km_of(float kk, float n, float c) {
    const float mant = fmaxf(__builtin_amdgcn_frexp_mantf(kk), 0.5f);
    const float l2 = __builtin_amdgcn_logf(mant) + (float)__builtin_amdgcn_frexp_expf(kk);
    return kk * fmaf(-l2, c, n);
}

// sum_q (K .* M)[q] u[q] over one row of Q kernel values (FP32): the plain
// hardware log2 when no value of the row, in any lane of the team's part of
// the wave, is a denormal (the common case; a zero gives a finite logarithm
// of 2^-126 and so adds K = 0), else km_of for each value.  The choice
// depends on the team's own document only (T < 64 masks the ballot to the
// team's lanes), so a document's result does not depend on its neighbours.
template <int Q, int T>
__device__ __forceinline__ float km_row(const float (&kk)[Q], const float (&u)[Q], float n, float c) {
    // bits - 1 as unsigned: +0 wraps to the maximum, denormals fall below 0x7fffff
    uint32_t mn = __float_as_uint(kk[0]) - 1u;
#pragma unroll
    for (int q = 1; q < Q; ++q) mn = min(mn, __float_as_uint(kk[q]) - 1u);
    uint64_t sub = __builtin_amdgcn_ballot_w64(mn < 0x7fffffu);
    if constexpr (T < 64) sub &= ((1ull << T) - 1ull) << (__lane_id() & (64 - T));
    float rsum = 0.f;
    if (sub == 0) {
#pragma unroll
        for (int q = 0; q < Q; ++q)
            rsum = fmaf(kk[q] * u[q], fmaf(-__builtin_amdgcn_logf(fmaxf(kk[q], 0x1p-126f)), c, n), rsum);
    } else {
#pragma unroll
        for (int q = 0; q < Q; ++q) rsum = fmaf(km_of(kk[q], n, c), u[q], rsum);
    }
    return rsum;
}

// Reduce-scatter over lane bit BETA (2..5) of N values: afterwards the lanes
// with that bit clear hold, in v[0, N/2), the pair sums of the first half,
// the lanes with it set those of the second half.  Each sum is formed on one
// lane only, so the copies that the matching all-gather hands out agree bit
// for bit.
template <int BETA, int N>
__device__ __forceinline__ void rs_bit(float* v) {
    static_assert(BETA >= 2 && BETA <= 5 && N % 2 == 0, "lane bits 2..5, even counts");
    constexpr int H = N / 2;
    if constexpr (BETA >= 4) {
        // the row swap exchanges the second half of one lane pair's registers
        // with the first half of the other's
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const uint32_t lo = __float_as_uint(v[j]), hi = __float_as_uint(v[j + H]);
            auto r = (BETA == 4) ? __builtin_amdgcn_permlane16_swap(lo, hi, false, false)
                                 : __builtin_amdgcn_permlane32_swap(lo, hi, false, false);
            v[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
        }
    } else {
        const bool up = (__lane_id() >> BETA) & 1;
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const float keep = up ? v[j + H] : v[j];
            const float send = up ? v[j] : v[j + H];
            float other;
            if constexpr (BETA == 2)   // lane ^ 4 through the LDS crossbar
                other = __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(send), 0x101F));
            else                       // row_ror:8 == lane ^ 8 within a row
                other = dpp<0x128>(send);
            v[j] = keep + other;
        }
    }
}

// All-gather over lane bit BETA: v[0, N) holds the first-half values on the
// lanes with the bit clear and the second-half values on the others;
// afterwards every lane holds all 2N values in order.
template <int BETA, int N>
__device__ __forceinline__ void ag_bit(float* v) {
    static_assert(BETA >= 2 && BETA <= 5, "lane bits 2..5");
    if constexpr (BETA >= 4) {
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const uint32_t w = __float_as_uint(v[j]);
            auto r = (BETA == 4) ? __builtin_amdgcn_permlane16_swap(w, w, false, false)
                                 : __builtin_amdgcn_permlane32_swap(w, w, false, false);
            v[j] = __uint_as_float(r[0]);
            v[j + N] = __uint_as_float(r[1]);
        }
    } else {
        // lanes with the bit clear sit in banks 0, 2 (BETA 2) or 0, 1 (BETA 3)
        // of each 16-lane row and read their partner with row_shl; the others
        // read theirs with row_shr; lanes outside the bank mask keep their own
        constexpr int SHL = (BETA == 2) ? 0x104 : 0x108, SHR = (BETA == 2) ? 0x114 : 0x118;
        constexpr int LO = (BETA == 2) ? 0x5 : 0x3, HI = (BETA == 2) ? 0xA : 0xC;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const int w = __float_as_int(v[j]);
            v[j + N] = __int_as_float(__builtin_amdgcn_update_dpp(w, w, SHL, 0xF, LO, false));
            v[j] = __int_as_float(__builtin_amdgcn_update_dpp(w, w, SHR, 0xF, HI, false));
        }
    }
}

// Reduce-scatter over lane bits LO .. LO+NB-1, highest first: N values become
// N >> NB, the lane whose bits read i in that field keeping values
// [i (N >> NB), (i + 1) (N >> NB)) of the sums.
template <int LO, int NB, int N>
__device__ __forceinline__ void rs_bits(float* v) {
    if constexpr (NB > 0) {
        rs_bit<LO + NB - 1, N>(v);
        rs_bits<LO, NB - 1, N / 2>(v);
    }
}

// The inverse spread: all-gather over lane bits LO .. LO+NB-1, lowest first.
template <int LO, int NB, int N>
__device__ __forceinline__ void ag_bits(float* v) {
    if constexpr (NB > 0) {
        ag_bit<LO, N>(v);
        ag_bits<LO + 1, NB - 1, N * 2>(v);
    }
}

// All-reduce of N values over lane bits LO .. LO+NB-1 (xor butterflies, so
// both partners of a step get the same bits).
template <int LO, int NB, int N>
__device__ __forceinline__ void allreduce_bits(float* v) {
    if constexpr (NB > 0) {
        static_assert(LO >= 0 && LO <= 5, "lane bits 0..5");
#pragma unroll
        for (int i = 0; i < N; ++i) {
            if constexpr (LO == 0) v[i] += dpp<0xB1>(v[i]);
            else if constexpr (LO == 1) v[i] += dpp<0x4E>(v[i]);
            else if constexpr (LO == 2) v[i] += xor4(v[i]);
            else if constexpr (LO == 3) v[i] += dpp<0x128>(v[i]);
            else if constexpr (LO == 4) v[i] = add_xor16(v[i]);
            else v[i] = add_xor32(v[i]);
        }
        allreduce_bits<LO + 1, NB - 1, N>(v);
    }
}

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

template <int T>
__device__ __forceinline__ double team_sum_f64(double v) {
#pragma unroll
    for (int o = 1; o < T; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// A launch whose queries each carry their own progress (per_query: the
// step-wise server, where queries join and leave between launches) runs each
// query's it_count iterations from its it_base, with the final step once the
// query's iterations are done; other launches share one range.  Uniform over
// a block (the query is), so the fields stay scalar.
__device__ __forceinline__ void take_iteration_range(SinkArgs& g, const QueryDev* qp) {
    if (g.per_query) {
        g.it_begin = qp->it_base;
        g.final_step = (int64_t)qp->it_base + g.it_count >= qp->iters ? 1 : 0;
    }
}

// added to every x update (see sink_team)
constexpr float kXPad = 0x1p-126f;

// One team's work on its document with PN rows per lane (fixed at compile
// time so the code is straight-line; the kernel picks PN per wave from the
// longest document of the wave).
template <int R, int C, int P, int Q, int W, int PN>
__device__ __forceinline__ void sink_team(const SinkArgs& g, const QueryDev* qp, const bool valid, const int d,
                                          const int rs, const int n, const int m, const int ldk, const int a,
                                          const int b, const int tl, const int wi, const int team, const int kb,
                                          const int it_end, float* s_part, double* s_red,
                                          float* s_rho, float* s_x) {
    constexpr int T = R * C;
    constexpr int Q4 = Q / 4;
    // The SpMM's column sums are reduce-scattered over the R lanes of a column
    // group (lane bits LC .. LC+LR-1), so lane (a, b) owns F of its Q columns,
    // kb + (a >> ARB) F + f: it forms their sums, x and u = 1/x, and the u
    // values are then spread back to the group.  With more row lanes than
    // columns (R > Q) the lowest ARB row-lane bits are all-reduced instead, so
    // 2^ARB lanes form each owned column identically and one of them (lead)
    // counts it in the residuals and stores it.
    constexpr int LC = ilog2(C), LR = ilog2(R), LQ = ilog2(Q);
    constexpr int RSB = (LR < LQ) ? LR : LQ;
    constexpr int ARB = LR - RSB;
    constexpr bool XLDS0 = (ARB == 0) && (C < 16);
    // Q need not be a power of two when the sums go through LDS: the R row
    // lanes then own ceil(Q / R) columns each, the last lanes fewer or none
    constexpr int F = XLDS0 ? (Q + R - 1) / R : Q >> RSB;
    constexpr bool EXACT = F * R == Q || !XLDS0;
    static_assert((1 << LC) == C && (1 << LR) == R && C >= 4, "team shape");
    static_assert((1 << LQ) == Q || XLDS0, "Q is a power of two unless the sums go through LDS");
    const int kf = kb + (a >> ARB) * F;              // first owned column
    const bool lead = (a & ((1 << ARB) - 1)) == 0;
    // owned column f lies in this lane's column group (always, unless Q is not R F)
    auto owned = [&](int f) -> bool { return EXACT || (a >> ARB) * F + f < Q; };
    // Teams with at least as many columns as row lanes, whose row lanes sit
    // on the low lane bits (C < 16, where the shuffles need DPP bank moves,
    // selects and wait states; the permlane swaps of bits 4 and 5 are cheaper
    // than a round trip through LDS), exchange through LDS instead: each lane
    // stores its Q column partial sums, the owner of a column adds the R
    // partials of it in row-lane order, and every lane reads the Q values of
    // u of its columns back.  s_x is this wave's region (each wave of a team
    // has its own C Q columns): R x XS partials, then C Q values of u,
    // indexed by the column within the wave (kbl, kfl).
    constexpr bool XLDS = XLDS0;
    constexpr int XS = C * Q + 4;                    // partial-sum row stride (floats)
    float* const s_u = s_x + R * XS;
    const int kbl = b * Q, kfl = kbl + (a >> ARB) * F;

    // A and every per-row / per-column vector are zero outside the document's
    // n x m block, except that a padded row holds 1 in column 0 (which every
    // query has) and x on a padded column is 2^-126: the update adds 2^-126
    // to y / r (which leaves every x >= 2^-102 unchanged, and is all of x where
    // y and 1/r are zero), so the reciprocals stay finite, padded rows get
    // v = 0 and padded columns add exact zeros; the arithmetic needs no
    // per-element guards and no per-column padding register.
    const auto Kt = gmem(qp->Kt);
    const int doc = g.sdoc[d];   // output slot, loaded with the indices
    int col[PN];
    float cval[PN];
    float A[PN][Q];
    if constexpr (W == 1) {
        // Branch-free loads, all in flight at once (a branch per row makes the
        // compiler wait for each row's loads before issuing the next): the
        // indices and weights of the lane's rows first, then the rows of Kt.
        // A row beyond the document reads index 0 (present: every document has
        // a word) and its Kt values from the zero block, whose first four
        // values are (1, 0, 0, 0); a column group beyond m reads zeros there
        // too.  Choosing the address instead of the loaded value keeps the
        // loads' destinations in A (no second set of registers).
#pragma unroll
        for (int p = 0; p < PN; ++p) {
            const int i = a + R * p;
            const int e = (valid && i < n) ? rs + i : 0;
            col[p] = g.scol[e];
            cval[p] = g.scw[e];
        }
        const auto zp = gmem(g.zpad);
#pragma unroll
        for (int p = 0; p < PN; ++p) {
            const bool row = valid && a + R * p < n;
            cval[p] = row ? cval[p] : 0.f;
#pragma unroll
            for (int q4 = 0; q4 < Q4; ++q4) {
                const int k0 = kb + 4 * q4;
                const bool ld = row && k0 < m;   // columns m..ldk-1 of Kt hold zeros
                const float4 t = ld4(ld ? Kt + (int64_t)col[p] * ldk + k0
                                        : zp + ((!row && kb == 0 && q4 == 0) ? 0 : 4 + k0));
                A[p][4 * q4 + 0] = t.x;
                A[p][4 * q4 + 1] = t.y;
                A[p][4 * q4 + 2] = t.z;
                A[p][4 * q4 + 3] = t.w;
            }
        }
    } else {
        // Multi-wave teams (the largest A blocks) load row by row, which needs
        // fewer registers; their rows' indices are read again where needed.
#pragma unroll
        for (int p = 0; p < PN; ++p) {
            const int i = a + R * p;
            const bool row = valid && i < n;
            cval[p] = row ? g.scw[rs + i] : 0.f;
#pragma unroll
            for (int q = 0; q < Q; ++q) A[p][q] = 0.f;
            if (!row && kb == 0) A[p][0] = 1.f;
            if (row) {
                const auto rowp = Kt + (int64_t)g.scol[rs + i] * ldk;
#pragma unroll
                for (int q4 = 0; q4 < Q4; ++q4) {
                    const int k0 = kb + 4 * q4;
                    if (k0 < m) {   // columns m..ldk-1 of Kt hold zeros
                        const float4 t = ld4(rowp + k0);
                        A[p][4 * q4 + 0] = t.x;
                        A[p][4 * q4 + 1] = t.y;
                        A[p][4 * q4 + 2] = t.z;
                        A[p][4 * q4 + 3] = t.w;
                    }
                }
            }
        }
    }
    // the act row index of row p (valid rows only), read again where needed
    // (the final step, with the column shift or K .* M gathered) rather than
    // held in registers through the iterations
    auto col_of = [&](int p) -> int { return g.scol[rs + a + R * p]; };

    // per-column vectors, also branch-free; a column beyond m reads element 0
    const auto rinvp = gmem(qp->rinv);
    const auto rp = gmem(qp->r);
    // convergence check (uniform over the launch: one tol per call)
    const float tol = qp->tol;
    const bool adaptive = tol > 0.f;
    float x[F], rinv[F], rq[F];
#pragma unroll
    for (int f = 0; f < F; ++f) {
        const int k = kf + f;
        const bool kv = k < m && owned(f);
        const int kc = kv ? k : 0;
        const float ri = rinvp[kc];
        const float rv = rp[kc];
        rinv[f] = kv ? ri : 0.f;
        rq[f] = (kv && adaptive && lead) ? rv : 0.f;
        x[f] = kv ? 1.0f / (float)m : 1.f;
    }
    if (g.it_begin != 0) {
        const auto xp = gmem(qp->x) + (int64_t)d * ldk;
#pragma unroll
        for (int f = 0; f < F; ++f) {
            const bool kv = kf + f < m && owned(f);
            const float xv = xp[kv ? kf + f : 0];
            x[f] = kv ? xv : 1.f;
        }
    }

    // u = 1/x on the owned columns (uo), spread to all Q columns of the lane (u)
    float u[Q], uo[F], s[PN], v[PN], y[Q];
    auto make_u = [&](void) {
        if constexpr (XLDS) {
#pragma unroll
            for (int f = 0; f < F; ++f) {
                uo[f] = rcp(x[f]);
                if (owned(f)) s_u[kfl + f] = uo[f];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int q4 = 0; q4 < Q4; ++q4) {
                const float4 t = *reinterpret_cast<const float4*>(s_u + kbl + 4 * q4);
                u[4 * q4 + 0] = t.x;
                u[4 * q4 + 1] = t.y;
                u[4 * q4 + 2] = t.z;
                u[4 * q4 + 3] = t.w;
            }
        } else {
#pragma unroll
            for (int f = 0; f < F; ++f) uo[f] = u[f] = rcp(x[f]);
            ag_bits<LC + ARB, RSB, F>(u);
        }
    };
    int par = 0;
    bool done = false;
    int t_done = g.it_begin;

    // s = A u summed over the team (lanes b, then waves); v = c / s
    // (the scheduling barriers keep each phase step-major: every reduction step
    // and reciprocal then has independent work between it and its consumer)
    auto sddmm = [&](void) {
#pragma unroll
        for (int p = 0; p < PN; ++p) {
            float acc = A[p][0] * u[0];
#pragma unroll
            for (int q = 1; q < Q; ++q) acc = fmaf(A[p][q], u[q], acc);
            s[p] = acc;
        }
        __builtin_amdgcn_sched_barrier(0);
        sum_over_b_n<C, PN>(s);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (W > 1) {
            float* sp = s_part + ((team * 2 + par) * W) * (R * P);
            if (b == 0) {
#pragma unroll
                for (int p = 0; p < PN; ++p) sp[wi * R * P + a + R * p] = s[p];
            }
            __syncthreads();
#pragma unroll
            for (int p = 0; p < PN; ++p) {
                float t = 0.f;
                for (int w2 = 0; w2 < W; ++w2) t += sp[w2 * R * P + a + R * p];
                s[p] = t;
            }
            par ^= 1;
        }
        if constexpr (C <= 8) {
            // Every lane of a row group (C lanes, whole quads) holds the same
            // sums: lane b forms the reciprocals of rows p with p mod 4 = b
            // mod 4 only, and each lane reads the others' with a quad
            // broadcast (the same values, a quarter of the reciprocals; with
            // C = 8 both quads of the group form their own copy).  The
            // 16-row tiles (C = 16) measured no gain from it.
            // (the picks are bit masks: selects between array elements would
            // be folded into an indexed access, i.e. scratch memory)
            constexpr int K = (PN + 3) / 4;
            const int bq = b & 3;
            const uint32_t m1 = 0u - (uint32_t)(bq == 1), m2 = 0u - (uint32_t)(bq == 2), m3 = 0u - (uint32_t)(bq == 3);
            float rq[K];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                uint32_t x = __float_as_uint(s[4 * j]);
                if (4 * j + 1 < PN) x = (__float_as_uint(s[4 * j + 1]) & m1) | (x & ~m1);
                if (4 * j + 2 < PN) x = (__float_as_uint(s[4 * j + 2]) & m2) | (x & ~m2);
                if (4 * j + 3 < PN) x = (__float_as_uint(s[4 * j + 3]) & m3) | (x & ~m3);
                rq[j] = rcp(__uint_as_float(x));
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int p = 0; p < PN; ++p) v[p] = cval[p] * quad_bcast(rq[p / 4], p % 4);
        } else {
#pragma unroll
            for (int p = 0; p < PN; ++p) s[p] = rcp(s[p]);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int p = 0; p < PN; ++p) v[p] = cval[p] * s[p];
        }
    };

    // y = A^T v summed over the team's rows (lanes a), the owned columns'
    // sums left in y[0, F)
    auto spmm = [&](void) {
#pragma unroll
        for (int q = 0; q < Q; ++q) y[q] = A[0][q] * v[0];
#pragma unroll
        for (int p = 1; p < PN; ++p) {
#pragma unroll
            for (int q = 0; q < Q; ++q) y[q] = fmaf(A[p][q], v[p], y[q]);
        }
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (XLDS) {
            // the previous readers of this region (last iteration's owners)
            // are this wave's own earlier LDS reads: in order, no wait needed
#pragma unroll
            for (int q4 = 0; q4 < Q4; ++q4)
                *reinterpret_cast<float4*>(s_x + a * XS + kbl + 4 * q4) =
                    make_float4(y[4 * q4 + 0], y[4 * q4 + 1], y[4 * q4 + 2], y[4 * q4 + 3]);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            float part[R][F];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int f = 0; f < F; ++f) part[r][f] = s_x[r * XS + kfl + f];
#pragma unroll
            for (int f = 0; f < F; ++f) {
                float t = part[0][f];
#pragma unroll
                for (int r = 1; r < R; ++r) t += part[r][f];
                y[f] = t;
            }
        } else {
            rs_bits<LC + ARB, RSB, Q>(y);
            allreduce_bits<LC, ARB, F>(y);
        }
        __builtin_amdgcn_sched_barrier(0);
    };

    for (int it = g.it_begin; it < it_end; ++it) {
        if constexpr (W == 1) {
            // a wave leaves once every team in it has converged
            if (adaptive && __builtin_amdgcn_ballot_w64(!done) == 0) break;
        }
        make_u();
        sddmm();
        spmm();
        if (!adaptive) {
#pragma unroll
            for (int f = 0; f < F; ++f) x[f] = fmaf(y[f], rinv[f], kXPad);
            t_done = it + 1;
        } else {
            // rho = sum_k r_k |x_new / x_old - 1|, with u = 1 / x_old from above,
            // over the owned columns, then over the whole team
            float xn[F];
            float rho = 0.f;
#pragma unroll
            for (int f = 0; f < F; ++f) {
                xn[f] = fmaf(y[f], rinv[f], kXPad);
                rho = fmaf(rq[f], fabsf(xn[f] * uo[f] - 1.f), rho);
            }
            sum_over_b_n<C, 1>(&rho);
            rho = sum_over_a<R, C>(rho);
            if constexpr (W > 1) {
                if (b == 0 && a == 0) s_rho[team * W + wi] = rho;
                __syncthreads();
                rho = 0.f;
                for (int w2 = 0; w2 < W; ++w2) rho += s_rho[team * W + w2];
            }
            if (!done) {
#pragma unroll
                for (int f = 0; f < F; ++f) x[f] = xn[f];
                t_done = it + 1;
                done = rho <= tol;
            }
        }
    }
    if (g.final_step && qp->it_out && valid && tl == 0 && wi == 0) gmem(qp->it_out)[doc] = t_done;

    if (!g.final_step) {
        if (valid && lead) {
#pragma unroll
            for (int f = 0; f < F; ++f)
                if (kf + f < m && owned(f)) gmem(qp->x)[(int64_t)d * ldk + kf + f] = x[f];
        }
        return;
    }

    // final step: u = 1/x (finite on padded columns, where A is zero), v = c / (K^T u)
    make_u();
    sddmm();

    double rho = 0.0;
    const bool want_resid = valid && qp->resid != nullptr;
    if (__builtin_amdgcn_readfirstlane((int)(qp->resid != nullptr))) {
        spmm();
        if (want_resid && lead) {
#pragma unroll
            for (int f = 0; f < F; ++f)
                if (kf + f < m && owned(f)) rho += fabs((double)uo[f] * (double)y[f] - (double)gmem(qp->r)[kf + f]);
        }
    }

    // WMD = sum_i v_i sum_k (K .* M)[i][k] u_k: products and each lane's sum over
    // its Q columns of a row in FP32, everything beyond in FP64.  K .* M is
    // rebuilt from the K block in registers (M = n_i - ln K / lambda) or
    // gathered from KMt when lambda is too small for that.
    double wsum = 0.0;
    if (qp->km_from_k) {
        const float cl = 0.693147180559945309f * qp->inv_lambda;
        // the rows' log-domain shifts, loaded together (the pointer is uniform)
        float nr[PN];
        const auto nrowp = gmem(qp->nrow);
        if (nrowp) {
            const auto zp = gmem(g.zpad) + 4;
#pragma unroll
            for (int p = 0; p < PN; ++p) nr[p] = *((valid && a + R * p < n) ? nrowp + col_of(p) : zp);
        } else {
#pragma unroll
            for (int p = 0; p < PN; ++p) nr[p] = 0.f;
        }
#pragma unroll
        for (int p = 0; p < PN; ++p) {
            const float rsum = km_row<Q, T>(A[p], u, nr[p], cl);
            wsum = fma((double)rsum, (double)v[p], wsum);
        }
    } else {
        const auto KMt = gmem(qp->KMt);
        float4 t[PN][Q4];
#pragma unroll
        for (int p = 0; p < PN; ++p) {
            const bool row = valid && a + R * p < n;
#pragma unroll
            for (int q4 = 0; q4 < Q4; ++q4) {
                const int k0 = kb + 4 * q4;
                const bool ld = row && k0 < m;
                t[p][q4] = ld4(ld ? KMt + (int64_t)col_of(p) * ldk + k0 : gmem(g.zpad) + 4 + k0);
            }
        }
        // padded rows and columns add exact zeros (u is zero beyond m, v on padded rows)
#pragma unroll
        for (int p = 0; p < PN; ++p) {
            float rsum = 0.f;
#pragma unroll
            for (int q4 = 0; q4 < Q4; ++q4) {
                rsum = fmaf(t[p][q4].x, u[4 * q4 + 0], rsum);
                rsum = fmaf(t[p][q4].y, u[4 * q4 + 1], rsum);
                rsum = fmaf(t[p][q4].z, u[4 * q4 + 2], rsum);
                rsum = fmaf(t[p][q4].w, u[4 * q4 + 3], rsum);
            }
            wsum = fma((double)rsum, (double)v[p], wsum);
        }
    }
    wsum = team_sum_f64<T>(wsum);
    if (__builtin_amdgcn_readfirstlane((int)(qp->resid != nullptr))) rho = team_sum_f64<T>(rho);
    if constexpr (W > 1) {
        if (tl == 0) {
            s_red[(team * W + wi) * 2 + 0] = wsum;
            s_red[(team * W + wi) * 2 + 1] = rho;
        }
        __syncthreads();
        if (wi == 0 && tl == 0) {
            wsum = 0.0;
            rho = 0.0;
            for (int w2 = 0; w2 < W; ++w2) {
                wsum += s_red[(team * W + w2) * 2 + 0];
                rho += s_red[(team * W + w2) * 2 + 1];
            }
        }
    }
    if (valid && tl == 0 && wi == 0) {
        gmem(qp->out)[doc] = wsum;
        if (want_resid) gmem(qp->resid)[doc] = rho;
    }
}

// Occupancy targets (waves per SIMD) of the one-wave register tiles: 5 for 4
// rows per lane, 3 for 8 rows of up to 12 columns (12 columns spill a few
// registers of the load phase to reach it, still faster than 2 waves), 2 for
// 16 rows or 16 columns.  The multi-wave teams with 8 rows of up to 12
// columns per lane target 3 too; the others take what their registers allow.
// `dense`: a second build of the one-wave tiles with 8 rows and 8 columns per
// lane at 4 waves (spilling a few registers), faster when the launch has more
// waves than 3 per SIMD, slower for a single query on a small corpus.
template <int P, int Q, int W, bool dense>
constexpr int sink_occupancy() {
    if constexpr (W > 1) return (P <= 8 && Q <= 12) ? 3 : 1;
    else if constexpr (P >= 16 || Q > 12) return 2;
    else if constexpr (P <= 4) return 5;
    else if constexpr (dense && Q <= 8) return 4;
    else return 3;
}

// The smallest compiled PN (a multiple of STEP, at most P) that covers pr
// rows per lane.  Results do not depend on PN: padded rows add exact zeros.
template <int R, int C, int P, int Q, int W, int PN, int STEP, typename... Args>
__device__ __forceinline__ void sink_dispatch(const int pr, Args&&... args) {
    if constexpr (PN >= P) {
        sink_team<R, C, P, Q, W, P>(args...);
    } else {
        if (pr <= PN) sink_team<R, C, P, Q, W, PN>(args...);
        else sink_dispatch<R, C, P, Q, W, PN + STEP, STEP>(pr, args...);
    }
}

// Occupancy target OCC (waves per SIMD), see sink_occupancy.
template <int R, int C, int P, int Q, int W, int OCC>
__global__ __launch_bounds__(256, OCC) void k_sink(SinkArgs g) {
    constexpr int T = R * C;
    static_assert(W == 1 || T == 64, "multi-wave teams use whole waves");
    static_assert(Q % 4 == 0, "columns are loaded as float4");
    static_assert(P % 4 == 0, "rows come in groups of 4");
    static_assert(4 + C * Q * W <= kZpadFloats, "padded loads stay inside the zero block");
    constexpr int TPW = 64 / T;
    constexpr int TEAMS = (W == 1) ? 4 * TPW : 4 / W;

    __shared__ float s_part[(W > 1) ? TEAMS * 2 * W * R * P : 1];
    __shared__ double s_red[(W > 1) ? TEAMS * W * 2 : 1];
    __shared__ float s_rho[(W > 1) ? TEAMS * W : 1];
    // per-team exchange region of the one-wave tiles (see sink_team)
    constexpr bool XL = (R <= Q) && (C < 16);
    constexpr int XTEAM = XL ? R * (C * Q + 4) + C * Q + 4 : 1;
    __shared__ __attribute__((aligned(16))) float s_x[XL ? TEAMS * W * XTEAM : 1];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int team = (W == 1) ? wave * TPW + lane / T : wave / W;
    const int tl = (W == 1) ? lane % T : lane;
    const int wi = (W == 1) ? 0 : wave % W;
    const int a = tl / C, b = tl % C;

    // Each query's documents fill whole blocks (the launch pads them to a
    // multiple of TEAMS), so the query, and every field of its record, is
    // uniform over the block: the compiler reads them with scalar loads.
    const int nd = g.d_end - g.d_begin;
    const int bpq = (nd + TEAMS - 1) / TEAMS;   // blocks per query
    const int qi = (int)(blockIdx.x / bpq);
    const int dd = (int)(blockIdx.x % bpq) * TEAMS + team;
    const bool valid = qi < g.nq && dd < nd;
    const int qidx = g.single ? 0 : g.qlist[qi < g.nq ? qi : 0];
    const int d = g.d_begin + (valid ? dd : 0);
    const QueryDev* qp = g.qd + qidx;
    take_iteration_range(g, qp);
    // the record's fields are read unconditionally (qp always points at a
    // record of the launch), so no branch waits for them
    const int qm = qp->m, qiters = qp->iters;
    const int m = valid ? qm : 0;
    const int ldk = qp->ldk;
    // d is a document of the launch even for a team without one, so these
    // loads need no guard (a guarded load would be waited for inside its branch)
    const int rs = g.sptr[d];
    const int re = g.sptr[d + 1];
    const int n = valid ? re - rs : 0;
    const int kb = (wi * C + b) * Q;

    // Every team of a multi-wave block runs the query's iteration count (the
    // query is uniform over the block), a padding team too, so all waves run
    // the same barriers; a padding team stores nothing.
    const int it_end = (valid || W > 1) ? min(g.it_begin + g.it_count, qiters) : g.it_begin;

    // rows per lane for this wave: the most any of its teams needs (documents
    // of a launch are sorted by length, so the teams of a wave have similar n).
    // n is uniform over a team, so its first lane stands for it; uniform, SGPR
    const int nrl = (n + R - 1) / R;
    int pr = __builtin_amdgcn_readlane(nrl, 0);
    if constexpr (W == 1) {
#pragma unroll
        for (int t = 1; t < TPW; ++t) pr = max(pr, __builtin_amdgcn_readlane(nrl, t * T));
    }
    sink_dispatch<R, C, P, Q, W, (P >= 16) ? 2 : 1, (P >= 16) ? 2 : 1>(
        pr, g, qp, valid, d, rs, n, m, ldk, a, b, tl, wi, team, kb, it_end, s_part, s_red, s_rho,
        s_x + (XL ? (team * W + wi) * XTEAM : 0));
}

// Any size: one 256-thread block per (query, document); the K block is
// re-read from memory in every iteration.  Dynamic LDS: x, u, rinv (m each)
// and v (n).
__global__ __launch_bounds__(256) void k_sink_stream(SinkArgs g) {
    extern __shared__ float sh[];
    __shared__ double red[2][4];
    const int tid = threadIdx.x;
    const int64_t item = blockIdx.x;
    const int nd = g.d_end - g.d_begin;
    const int qidx = g.single ? 0 : g.qlist[item / nd];
    const int d = g.d_begin + (int)(item % nd);
    const QueryDev* qp = g.qd + qidx;
    take_iteration_range(g, qp);
    const int m = qp->m, ldk = qp->ldk;
    const int rs = g.sptr[d], n = g.sptr[d + 1] - rs;
    float* x = sh;
    float* u = sh + m;
    float* ri = sh + 2 * m;
    float* v = sh + 3 * m;
    for (int k = tid; k < m; k += 256) {
        ri[k] = gmem(qp->rinv)[k];
        x[k] = (g.it_begin == 0) ? 1.0f / (float)m : gmem(qp->x)[(int64_t)d * ldk + k];
    }
    __syncthreads();
    const int it_end = min(g.it_begin + g.it_count, qp->iters);
    auto sddmm = [&](void) {
        for (int k = tid; k < m; k += 256) u[k] = rcp(x[k]);
        __syncthreads();
        for (int i = tid; i < n; i += 256) {
            const auto row = gmem(qp->Kt) + (int64_t)g.scol[rs + i] * ldk;
            float acc = 0.f;
            for (int k = 0; k < m; ++k) acc = fmaf(row[k], u[k], acc);
            v[i] = g.scw[rs + i] * rcp(acc);
        }
        __syncthreads();
    };
    const float tol = qp->tol;
    __shared__ float s_rho[4];
    int t_done = g.it_begin;
    for (int it = g.it_begin; it < it_end; ++it) {
        sddmm();
        float rho = 0.f;
        for (int k = tid; k < m; k += 256) {
            float acc = 0.f;
            for (int i = 0; i < n; ++i)
                acc = fmaf(gmem(qp->Kt)[(int64_t)g.scol[rs + i] * ldk + k], v[i], acc);
            const float xn = acc * ri[k];
            // convergence check: rho = sum_k r_k |x_new / x_old - 1|, u = 1 / x_old
            if (tol > 0.f) rho = fmaf(gmem(qp->r)[k], fabsf(xn * u[k] - 1.f), rho);
            x[k] = xn;
        }
        __syncthreads();
        t_done = it + 1;
        if (tol > 0.f) {
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) rho += __shfl_xor(rho, o, 64);
            if ((tid & 63) == 0) s_rho[tid >> 6] = rho;
            __syncthreads();
            const float tot = s_rho[0] + s_rho[1] + s_rho[2] + s_rho[3];
            if (tot <= tol) break;
        }
    }
    if (g.final_step && qp->it_out && tid == 0) gmem(qp->it_out)[g.sdoc[d]] = t_done;
    if (!g.final_step) {
        for (int k = tid; k < m; k += 256) gmem(qp->x)[(int64_t)d * ldk + k] = x[k];
        return;
    }
    sddmm();
    double rho = 0.0, wsum = 0.0;
    if (qp->resid) {
        for (int k = tid; k < m; k += 256) {
            float acc = 0.f;
            for (int i = 0; i < n; ++i)
                acc = fmaf(gmem(qp->Kt)[(int64_t)g.scol[rs + i] * ldk + k], v[i], acc);
            rho += fabs((double)u[k] * (double)acc - (double)gmem(qp->r)[k]);
        }
    }
    // per document word: FP32 sum over the query words in chunks of 8 (as the
    // register tiles sum a lane's columns), FP64 beyond
    for (int i = tid; i < n; i += 256) {
        const int col = g.scol[rs + i];
        const double vi = (double)v[i];
        if (qp->km_from_k) {   // K .* M rebuilt from K: M = n_i - ln K / lambda
            const auto row = gmem(qp->Kt) + (int64_t)col * ldk;
            const float nr = qp->nrow ? gmem(qp->nrow)[col] : 0.f, cl = 0.693147180559945309f * qp->inv_lambda;
            for (int k0 = 0; k0 < m; k0 += 8) {
                float rsum = 0.f;
                for (int k = k0; k < min(k0 + 8, m); ++k) rsum = fmaf(km_of(row[k], nr, cl), u[k], rsum);
                wsum = fma((double)rsum, vi, wsum);
            }
        } else {
            const auto row = gmem(qp->KMt) + (int64_t)col * ldk;
            for (int k0 = 0; k0 < m; k0 += 8) {
                float rsum = 0.f;
                for (int k = k0; k < min(k0 + 8, m); ++k) rsum = fmaf(row[k], u[k], rsum);
                wsum = fma((double)rsum, vi, wsum);
            }
        }
    }
    wsum = team_sum_f64<64>(wsum);
    if (qp->resid) rho = team_sum_f64<64>(rho);
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = wsum;
        red[1][tid >> 6] = rho;
    }
    __syncthreads();
    if (tid == 0) {
        const int doc = g.sdoc[d];
        gmem(qp->out)[doc] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        if (qp->resid) gmem(qp->resid)[doc] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
}

// Row-lane form for short queries: one wave per (query, document).  Lane l
// holds rows l + 64 r (r < RP) of the document's K block in registers, so the
// SDDMM s_i = sum_k A[i][k] u_k is an in-lane dot product with u broadcast
// from LDS.  The block is also kept transposed in LDS, and for the SpMM lane l
// owns column l % MQ and sums part l / MQ of the rows, so neither phase needs
// cross-lane reductions; the H = 64 / MQ row parts are combined with lane
// swaps.  One reciprocal per lane and row / column per iteration.
template <int MQ, int RP>
__global__ __launch_bounds__(64) void k_sink_rows(SinkArgs g) {
    constexpr int H = 64 / MQ;              // row parts in the SpMM
    constexpr int NR = 64 * RP;             // rows held by the wave
    constexpr int LDT = NR + 4;             // transposed block row stride (floats)
    constexpr int MQ4 = MQ / 4;
    static_assert(H == 1 || H == 2 || H == 4, "MQ in {16, 32, 64}");
    __shared__ __attribute__((aligned(16))) float At[MQ * LDT];
    __shared__ __attribute__((aligned(16))) float uS[MQ];
    __shared__ __attribute__((aligned(16))) float vS[NR];
    __shared__ double red[2];

    const int lane = threadIdx.x;
    const int64_t item = blockIdx.x;
    const int nd = g.d_end - g.d_begin;
    const int qidx = g.single ? 0 : g.qlist[item / nd];
    const int d = g.d_begin + (int)(item % nd);
    const QueryDev* qp = g.qd + qidx;
    take_iteration_range(g, qp);
    const int m = qp->m, ldk = qp->ldk;
    const int rs = g.sptr[d];
    const int n = g.sptr[d + 1] - rs;

    // rows: registers and the transposed LDS copy (zeros outside n x m)
    float A[RP][MQ];
    float cval[RP];
#pragma unroll
    for (int r = 0; r < RP; ++r) {
        const int i = lane + 64 * r;
        cval[r] = 0.f;
#pragma unroll
        for (int k = 0; k < MQ; ++k) A[r][k] = 0.f;
        if (i < n) {
            cval[r] = g.scw[rs + i];
            const auto row = gmem(qp->Kt) + (int64_t)g.scol[rs + i] * ldk;
#pragma unroll
            for (int k4 = 0; k4 < MQ4; ++k4) {
                if (4 * k4 < m) {   // columns m..ldk-1 of Kt hold zeros
                    const float4 t = ld4(row + 4 * k4);
                    A[r][4 * k4 + 0] = t.x;
                    A[r][4 * k4 + 1] = t.y;
                    A[r][4 * k4 + 2] = t.z;
                    A[r][4 * k4 + 3] = t.w;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < MQ; ++k) At[k * LDT + i] = A[r][k];
    }

    // SpMM lane roles: column kc, rows [i0, i1) in steps of 4
    const int kc = lane % MQ, h = lane / MQ;
    const bool kv = kc < m;
    const int n4 = (n + 3) & ~3;
    const int part = (((n4 / 4) + H - 1) / H) * 4;
    const int i0 = min(h * part, n4), i1 = min(i0 + part, n4);
    const float rinv = kv ? gmem(qp->rinv)[kc] : 0.f;
    float x = kv ? 1.0f / (float)m : 1.f;
    if (g.it_begin > 0 && kv) x = gmem(qp->x)[(int64_t)d * ldk + kc];
    float u = 0.f, v[RP];

    auto sddmm = [&](void) {
        if (h == 0) uS[kc] = u;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RP; ++r) {
            float acc = 0.f;
#pragma unroll
            for (int k4 = 0; k4 < MQ4; ++k4) {
                const float4 uu = *reinterpret_cast<const float4*>(&uS[4 * k4]);
                acc = fmaf(A[r][4 * k4 + 0], uu.x, acc);
                acc = fmaf(A[r][4 * k4 + 1], uu.y, acc);
                acc = fmaf(A[r][4 * k4 + 2], uu.z, acc);
                acc = fmaf(A[r][4 * k4 + 3], uu.w, acc);
            }
            v[r] = (cval[r] > 0.f) ? cval[r] * rcp(acc) : 0.f;
            vS[lane + 64 * r] = v[r];
        }
        __syncthreads();
    };
    // y_kc = sum_i At[kc][i] v_i over this lane's row part, then over the parts
    auto spmm = [&](void) -> float {
        float y = 0.f;
        const float* at = &At[kc * LDT];
        for (int i = i0; i < i1; i += 4) {
            const float4 a4 = *reinterpret_cast<const float4*>(at + i);
            const float4 v4 = *reinterpret_cast<const float4*>(&vS[i]);
            y = fmaf(a4.x, v4.x, y);
            y = fmaf(a4.y, v4.y, y);
            y = fmaf(a4.z, v4.z, y);
            y = fmaf(a4.w, v4.w, y);
        }
        if constexpr (H >= 4) y = add_xor16(y);
        if constexpr (H >= 2) y = add_xor32(y);
        return y;
    };

    const int it_end = min(g.it_begin + g.it_count, qp->iters);
    for (int it = g.it_begin; it < it_end; ++it) {
        u = kv ? rcp(x) : 0.f;
        sddmm();
        x = spmm() * rinv;
    }
    if (!g.final_step) {
        if (h == 0 && kv) gmem(qp->x)[(int64_t)d * ldk + kc] = x;
        return;
    }
    u = kv ? rcp(x) : 0.f;
    sddmm();
    double rho = 0.0;
    if (qp->resid) {
        const float y = spmm();
        if (h == 0 && kv) rho = fabs((double)u * (double)y - (double)gmem(qp->r)[kc]);
    }
    // WMD = sum_i v_i sum_k (K .* M)[i][k] u_k: products and sums over 8 query
    // words in FP32, FP64 beyond; K .* M rebuilt from the registers
    // (M = n_i - ln K / lambda) or gathered from KMt
    double wsum = 0.0;
#pragma unroll
    for (int r = 0; r < RP; ++r) {
        const int i = lane + 64 * r;
        if (i < n) {
            const double vr = (double)v[r];
            if (qp->km_from_k) {
                const float cl = 0.693147180559945309f * qp->inv_lambda;
                const float nr = qp->nrow ? gmem(qp->nrow)[g.scol[rs + i]] : 0.f;
#pragma unroll
                for (int k8 = 0; k8 < MQ / 8; ++k8) {   // FP32 over 8 query words, FP64 beyond
                    float rsum = 0.f;
#pragma unroll
                    for (int e = 0; e < 8; ++e) rsum = fmaf(km_of(A[r][8 * k8 + e], nr, cl), uS[8 * k8 + e], rsum);
                    wsum = fma((double)rsum, vr, wsum);
                }
            } else {
                const auto row = gmem(qp->KMt) + (int64_t)g.scol[rs + i] * ldk;
#pragma unroll
                for (int k8 = 0; k8 < MQ / 8; ++k8) {
                    float rsum = 0.f;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int k4 = 2 * k8 + h;
                        if (4 * k4 < m) {
                            const float4 t = ld4(row + 4 * k4);
                            const float4 uu = *reinterpret_cast<const float4*>(&uS[4 * k4]);
                            // uS is zero past m, so the padded columns add nothing
                            rsum = fmaf(t.x, uu.x, rsum);
                            rsum = fmaf(t.y, uu.y, rsum);
                            rsum = fmaf(t.z, uu.z, rsum);
                            rsum = fmaf(t.w, uu.w, rsum);
                        }
                    }
                    wsum = fma((double)rsum, vr, wsum);
                }
            }
        }
    }
    wsum = team_sum_f64<64>(wsum);
    if (qp->resid) rho = team_sum_f64<64>(rho);
    (void)red;
    if (lane == 0) {
        const int doc = g.sdoc[d];
        gmem(qp->out)[doc] = wsum;
        if (qp->resid) gmem(qp->resid)[doc] = rho;
        if (qp->it_out) gmem(qp->it_out)[doc] = it_end;
    }
}

// Compute units of the current device (cached per device).
int device_cus() {
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int n = cache[dev].load(std::memory_order_relaxed);
    if (n == 0) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cache[dev].store(n, std::memory_order_relaxed);
    }
    return n;
}

struct Shape {
    int max_m, max_n, teams_per_block, threads;
    bool tile;   // a register tile (implements the convergence check)
    int occ;     // waves per SIMD of kern
    void (*kern)(SinkArgs);
    void (*kern_dense)(SinkArgs);   // the build for launches beyond occ waves per SIMD
};

template <int R, int C, int P, int Q, int W>
constexpr Shape make_shape() {
    constexpr int occ = sink_occupancy<P, Q, W, false>();
    constexpr int occ_dense = sink_occupancy<P, Q, W, true>();
    return Shape{C * Q * W, R * P, (W == 1) ? 4 * (64 / (R * C)) : 4 / W, 256, true, occ,
                 &k_sink<R, C, P, Q, W, occ>, &k_sink<R, C, P, Q, W, occ_dense>};
}

template <int MQ, int RP>
constexpr Shape make_rows_shape() {
    return Shape{MQ, 64 * RP, 1, 64, false, 0, &k_sink_rows<MQ, RP>, &k_sink_rows<MQ, RP>};
}

const Shape kShapes[] = {
    make_shape<4, 4, 16, 4, 1>(),    // 0: m <= 16,  16-lane teams
    make_shape<4, 4, 16, 8, 1>(),    // 1: m <= 32,  16-lane teams
    make_shape<8, 4, 8, 8, 1>(),     // 2: m <= 32,  32-lane teams
    make_shape<4, 8, 16, 8, 1>(),    // 3: m <= 64,  32-lane teams
    make_shape<8, 8, 8, 8, 1>(),     // 4: m <= 64,  one wave
    make_shape<4, 16, 16, 8, 1>(),   // 5: m <= 128, one wave
    make_shape<4, 16, 16, 8, 2>(),   // 6: m <= 256, two waves
    make_shape<4, 16, 16, 8, 4>(),   // 7: m <= 512, four waves
    make_rows_shape<16, 1>(),        // 8: m <= 16,  row lanes
    make_rows_shape<32, 1>(),        // 9: m <= 32,  row lanes
    make_rows_shape<64, 1>(),        // 10: m <= 64, row lanes
    make_shape<16, 4, 4, 8, 1>(),    // 11: m <= 32,  one wave per document
    make_shape<8, 4, 8, 12, 1>(),    // 12: m <= 48,  32-lane teams, 12 columns per lane
    make_shape<8, 8, 8, 12, 1>(),    // 13: m <= 96,  one wave, 12 columns per lane
    make_shape<8, 8, 8, 12, 2>(),    // 14: m <= 192, two waves, 12 columns per lane
    make_shape<8, 8, 8, 12, 4>(),    // 15: m <= 384, four waves, 12 columns per lane
    make_shape<8, 8, 8, 8, 4>(),     // 16: m <= 256, four waves
};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);
// default shape per query-length class, smallest first: the first entry
// whose max_m covers the query (measured on corpora of 5000 and 20000
// documents of 10-60 words, one query and batches of 8-16: the 12-column
// tiles run 33-48, 65-96, 129-192 and 257-384-word queries 13-21 % faster
// than the next power-of-two tile; the 8 x 8 tiles at three or four waves per
// SIMD run 49-64 and 193-256-word queries 2-15 % faster than the 16-row tiles
// at two)
const int kDefaultShapes[] = {8, 2, 12, 4, 13, 5, 14, 16, 15, 7};
const int kAdaptiveShapes[] = {0, 2, 12, 4, 13, 5, 14, 16, 15, 7};  // register tiles only (convergence check)

}  // namespace

int sinkhorn_num_shapes() { return kNumShapes; }

bool sinkhorn_shape_adaptive(int shape) { return shape < 0 || kShapes[shape].tile; }

int sinkhorn_shape_for(int m, int max_n, bool adaptive) {
    for (int s : (adaptive ? kAdaptiveShapes : kDefaultShapes))
        if (m <= kShapes[s].max_m && max_n <= kShapes[s].max_n) return s;
    return -1;
}

bool sinkhorn_shape_fits(int shape, int m, int max_n) {
    return shape >= 0 && shape < kNumShapes && m <= kShapes[shape].max_m && max_n <= kShapes[shape].max_n;
}

int sinkhorn_shape_max_m(int shape) { return shape < 0 ? 4096 : kShapes[shape].max_m; }
int sinkhorn_shape_max_n(int shape) { return shape < 0 ? 16384 : kShapes[shape].max_n; }

hipError_t launch_sinkhorn(int shape, const SinkArgs& a, int max_m, int max_n, hipStream_t s) {
    const int64_t nitems = (int64_t)a.nq * (a.d_end - a.d_begin);
    if (nitems <= 0) return hipSuccess;
    if (shape < 0) {
        // dynamic LDS: x, u, 1/r for the largest query, v for the largest document
        const size_t lds = (size_t)(3 * max_m + max_n) * sizeof(float);
        if (lds > 64 * 1024) {
            hipError_t e = hipFuncSetAttribute((const void*)k_sink_stream,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        return launch_kernel(k_sink_stream, dim3((unsigned)nitems), dim3(256), (uint32_t)lds, s, a);
    }
    const Shape& sh = kShapes[shape];
    // register tiles: each query's documents padded to whole blocks; the row
    // kernel has one team per block, so this is nitems for it
    const int64_t blocks = (int64_t)a.nq * ((a.d_end - a.d_begin + sh.teams_per_block - 1) / sh.teams_per_block);
    const bool dense = sh.occ > 0 && blocks * (sh.threads / 64) > (int64_t)sh.occ * 4 * device_cus();
    return launch_kernel(dense ? sh.kern_dense : sh.kern, dim3((unsigned)blocks), dim3(sh.threads), 0, s, a);
}

}  // namespace wmd
