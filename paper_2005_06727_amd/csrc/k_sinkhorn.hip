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
//   u     = 1 / x                        (columns; every a holds a copy)
//   s_i   = sum_k A[i][k] u_k            (partial over q, then summed over b)
//   v_i   = c_i / s_i                    (rows; every b holds a copy)
//   x_k   = (1 / r_k) sum_i A[i][k] v_i  (partial over p, then summed over a)
// Final: u = 1/x, v = c / (A u), WMD = sum_{i,k} (KMt[i][k] u_k) v_i with the
// products in FP32 and the sum in FP64; optionally the FP64 residual
// sum_k |u_k (A^T v)_k - r_k| of the plan's row marginal (its column marginal
// is c by construction).
#include "wmd_internal.h"

namespace wmd {

namespace {

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float swz_xor16(float v) {
    // ds_swizzle bit mode: and 0x1f, or 0, xor 0x10 -> lane ^ 16 within 32 lanes
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
}

__device__ __forceinline__ float shfl_xor32(float v) {
    return __shfl_xor(v, 32, 64);
}

// Sum over the C consecutive lanes (C a power of two <= 16) sharing a team row.
template <int C>
__device__ __forceinline__ float sum_over_b(float v) {
    if constexpr (C >= 2) v += dpp<0xB1>(v);    // quad_perm [1,0,3,2]: lane ^ 1
    if constexpr (C >= 4) v += dpp<0x4E>(v);    // quad_perm [2,3,0,1]: lane ^ 2
    if constexpr (C >= 8) v += dpp<0x141>(v);   // row_half_mirror: the other quad (quads uniform)
    if constexpr (C >= 16) v += dpp<0x140>(v);  // row_mirror: the other half-row (halves uniform)
    return v;
}

__device__ __forceinline__ float swz_xor4(float v) {
    // ds_swizzle bit mode: and 0x1f, or 0, xor 0x04 -> lane ^ 4 within 32 lanes
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x101F));
}

// Sum over the R lanes with the same b (lane stride C) of an R*C-lane team.
// Every step pairs lane l with lane l ^ o, so all R lanes end with the same
// bits (a + b == b + a): the R copies of x stay identical.
template <int R, int C>
__device__ __forceinline__ float sum_over_a(float v) {
    constexpr int T = R * C;
    if constexpr (C <= 1 && T > 1) v += dpp<0xB1>(v);    // lane ^ 1
    if constexpr (C <= 2 && T > 2) v += dpp<0x4E>(v);    // lane ^ 2
    if constexpr (C <= 4 && T > 4) v += swz_xor4(v);     // lane ^ 4
    if constexpr (C <= 8 && T > 8) v += dpp<0x128>(v);   // row_ror:8 == lane ^ 8 within a row
    if constexpr (T > 16) v += swz_xor16(v);             // lane ^ 16
    if constexpr (T > 32) v += shfl_xor32(v);            // lane ^ 32
    return v;
}

template <int T>
__device__ __forceinline__ double team_sum_f64(double v) {
#pragma unroll
    for (int o = 1; o < T; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

template <int R, int C, int P, int Q, int W>
__global__ __launch_bounds__(256) void k_sink(SinkArgs g) {
    constexpr int T = R * C;
    static_assert(W == 1 || T == 64, "multi-wave teams use whole waves");
    static_assert(Q % 4 == 0, "columns are loaded as float4");
    constexpr int TPW = 64 / T;
    constexpr int TEAMS = (W == 1) ? 4 * TPW : 4 / W;
    constexpr int Q4 = Q / 4;

    __shared__ float s_part[(W > 1) ? TEAMS * 2 * W * R * P : 1];
    __shared__ double s_red[(W > 1) ? TEAMS * W * 2 : 1];
    __shared__ int s_itmax[(W > 1) ? TEAMS : 1];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int team = (W == 1) ? wave * TPW + lane / T : wave / W;
    const int tl = (W == 1) ? lane % T : lane;
    const int wi = (W == 1) ? 0 : wave % W;
    const int a = tl / C, b = tl % C;

    const int64_t item = (int64_t)blockIdx.x * TEAMS + team;
    const int nd = g.d_end - g.d_begin;
    const bool valid = item < (int64_t)g.nq * nd;
    int qidx = 0, d = g.d_begin;
    if (valid) {
        qidx = g.qlist[item / nd];
        d = g.d_begin + (int)(item % nd);
    }
    const QueryDev* qp = g.qd + qidx;
    const int m = valid ? qp->m : 0;
    const int ldk = qp->ldk;
    const int rs = g.sptr[d];
    const int n = valid ? g.sptr[d + 1] - rs : 0;
    const int kb = (wi * C + b) * Q;

    const int pn_w = wave_max((n + R - 1) / R);                        // row blocks in use (wave)
    const int qb_w = wave_max((min(max(m - kb, 0), Q) + 3) >> 2);      // float4 column blocks in use

    float A[P][Q];
    float cval[P];
    // load the document's block of Kt (and its weights) once
#pragma unroll
    for (int p = 0; p < P; ++p) {
        cval[p] = 0.f;
#pragma unroll
        for (int q = 0; q < Q; ++q) A[p][q] = 0.f;
        if (p < pn_w) {
            const int i = a + R * p;
            if (i < n) {
                cval[p] = g.scw[rs + i];
                const float* row = qp->Kt + (int64_t)g.scol[rs + i] * ldk;
#pragma unroll
                for (int q4 = 0; q4 < Q4; ++q4) {
                    const int k0 = kb + 4 * q4;
                    if (q4 < qb_w && k0 < m) {
                        float4 t = *reinterpret_cast<const float4*>(row + k0);
                        A[p][4 * q4 + 0] = t.x;
                        A[p][4 * q4 + 1] = (k0 + 1 < m) ? t.y : 0.f;
                        A[p][4 * q4 + 2] = (k0 + 2 < m) ? t.z : 0.f;
                        A[p][4 * q4 + 3] = (k0 + 3 < m) ? t.w : 0.f;
                    }
                }
            }
        }
    }

    float x[Q], rinv[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int k = kb + q;
        const bool kv = k < m;
        rinv[q] = kv ? qp->rinv[k] : 0.f;
        if (g.it_begin == 0) x[q] = kv ? 1.0f / (float)m : 1.f;
        else x[q] = kv ? qp->x[(int64_t)d * ldk + k] : 1.f;
    }

    int it_end = valid ? min(g.it_begin + g.it_count, qp->iters) : g.it_begin;
    if constexpr (W > 1) {
        // every wave of the block must run the same number of barriers
        if (tid < TEAMS) s_itmax[tid] = g.it_begin;
        __syncthreads();
        if (tl == 0 && wi == 0) atomicMax(&s_itmax[team], it_end);
        __syncthreads();
        int mx = g.it_begin;
        for (int t2 = 0; t2 < TEAMS; ++t2) mx = max(mx, s_itmax[t2]);
        __syncthreads();
        it_end = mx;
    }
    const int my_end = valid ? min(g.it_begin + g.it_count, qp->iters) : g.it_begin;

    float u[Q], s[P], v[P];
#pragma unroll
    for (int p = 0; p < P; ++p) s[p] = 0.f;
    int par = 0;

    // s = A u summed over the whole team (lanes b, then waves)
    auto sddmm = [&](void) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (p < pn_w) {
                float acc = 0.f;
#pragma unroll
                for (int q = 0; q < Q; ++q)
                    if (q / 4 < qb_w) acc = fmaf(A[p][q], u[q], acc);
                s[p] = sum_over_b<C>(acc);
            }
        }
        if constexpr (W > 1) {
            float* sp = s_part + ((team * 2 + par) * W) * (R * P);
            if (b == 0) {
#pragma unroll
                for (int p = 0; p < P; ++p)
                    if (p < pn_w) sp[wi * R * P + a + R * p] = s[p];
            }
            __syncthreads();
#pragma unroll
            for (int p = 0; p < P; ++p) {
                if (p < pn_w) {
                    float t = 0.f;
                    for (int w2 = 0; w2 < W; ++w2) t += sp[w2 * R * P + a + R * p];
                    s[p] = t;
                }
            }
            par ^= 1;
        }
#pragma unroll
        for (int p = 0; p < P; ++p) v[p] = (cval[p] > 0.f) ? cval[p] * rcp(s[p]) : 0.f;
    };

    for (int it = g.it_begin; it < it_end; ++it) {
        const bool act = it < my_end;
#pragma unroll
        for (int q = 0; q < Q; ++q) u[q] = (act && kb + q < m) ? rcp(x[q]) : 0.f;
        sddmm();
        if (act) {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                if (q / 4 < qb_w) {
                    float acc = 0.f;
#pragma unroll
                    for (int p = 0; p < P; ++p)
                        if (p < pn_w) acc = fmaf(A[p][q], v[p], acc);
                    x[q] = sum_over_a<R, C>(acc) * rinv[q];
                }
            }
        }
    }

    if (!g.final_step) {
        if (valid && a == 0) {
#pragma unroll
            for (int q = 0; q < Q; ++q)
                if (kb + q < m) qp->x[(int64_t)d * ldk + kb + q] = x[q];
        }
        return;
    }

    // final step: u = 1/x, v = c / (K^T u)
#pragma unroll
    for (int q = 0; q < Q; ++q) u[q] = (kb + q < m) ? rcp(x[q]) : 0.f;
    sddmm();

    double rho = 0.0;
    const bool want_resid = valid && qp->resid != nullptr;
    if (want_resid) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (q / 4 < qb_w) {
                float acc = 0.f;
#pragma unroll
                for (int p = 0; p < P; ++p)
                    if (p < pn_w) acc = fmaf(A[p][q], v[p], acc);
                const float y = sum_over_a<R, C>(acc);
                if (a == 0 && kb + q < m)
                    rho += fabs((double)u[q] * (double)y - (double)qp->r[kb + q]);
            }
        }
    }

    // WMD = sum_i v_i sum_k KMt[i][k] u_k
    double wsum = 0.0;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        if (p < pn_w) {
            const int i = a + R * p;
            if (i < n) {
                const float* row = qp->KMt + (int64_t)g.scol[rs + i] * ldk;
                const double vp = (double)v[p];
#pragma unroll
                for (int q4 = 0; q4 < Q4; ++q4) {
                    const int k0 = kb + 4 * q4;
                    if (q4 < qb_w && k0 < m) {
                        float4 t = *reinterpret_cast<const float4*>(row + k0);
                        wsum = fma((double)(t.x * u[4 * q4 + 0]), vp, wsum);
                        if (k0 + 1 < m) wsum = fma((double)(t.y * u[4 * q4 + 1]), vp, wsum);
                        if (k0 + 2 < m) wsum = fma((double)(t.z * u[4 * q4 + 2]), vp, wsum);
                        if (k0 + 3 < m) wsum = fma((double)(t.w * u[4 * q4 + 3]), vp, wsum);
                    }
                }
            }
        }
    }
    wsum = team_sum_f64<T>(wsum);
    rho = team_sum_f64<T>(rho);
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
        const int doc = g.sdoc[d];
        qp->out[doc] = wsum;
        if (want_resid) qp->resid[doc] = rho;
    }
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
    const int qidx = g.qlist[item / nd];
    const int d = g.d_begin + (int)(item % nd);
    const QueryDev* qp = g.qd + qidx;
    const int m = qp->m, ldk = qp->ldk;
    const int rs = g.sptr[d], n = g.sptr[d + 1] - rs;
    float* x = sh;
    float* u = sh + m;
    float* ri = sh + 2 * m;
    float* v = sh + 3 * m;
    for (int k = tid; k < m; k += 256) {
        ri[k] = qp->rinv[k];
        x[k] = (g.it_begin == 0) ? 1.0f / (float)m : qp->x[(int64_t)d * ldk + k];
    }
    __syncthreads();
    const int it_end = min(g.it_begin + g.it_count, qp->iters);
    auto sddmm = [&](void) {
        for (int k = tid; k < m; k += 256) u[k] = rcp(x[k]);
        __syncthreads();
        for (int i = tid; i < n; i += 256) {
            const float* row = qp->Kt + (int64_t)g.scol[rs + i] * ldk;
            float acc = 0.f;
            for (int k = 0; k < m; ++k) acc = fmaf(row[k], u[k], acc);
            v[i] = g.scw[rs + i] * rcp(acc);
        }
        __syncthreads();
    };
    for (int it = g.it_begin; it < it_end; ++it) {
        sddmm();
        for (int k = tid; k < m; k += 256) {
            float acc = 0.f;
            for (int i = 0; i < n; ++i)
                acc = fmaf(qp->Kt[(int64_t)g.scol[rs + i] * ldk + k], v[i], acc);
            x[k] = acc * ri[k];
        }
        __syncthreads();
    }
    if (!g.final_step) {
        for (int k = tid; k < m; k += 256) qp->x[(int64_t)d * ldk + k] = x[k];
        return;
    }
    sddmm();
    double rho = 0.0, wsum = 0.0;
    if (qp->resid) {
        for (int k = tid; k < m; k += 256) {
            float acc = 0.f;
            for (int i = 0; i < n; ++i)
                acc = fmaf(qp->Kt[(int64_t)g.scol[rs + i] * ldk + k], v[i], acc);
            rho += fabs((double)u[k] * (double)acc - (double)qp->r[k]);
        }
    }
    for (int i = tid; i < n; i += 256) {
        const float* row = qp->KMt + (int64_t)g.scol[rs + i] * ldk;
        const double vi = (double)v[i];
        for (int k = 0; k < m; ++k) wsum = fma((double)(row[k] * u[k]), vi, wsum);
    }
    wsum = team_sum_f64<64>(wsum);
    rho = team_sum_f64<64>(rho);
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = wsum;
        red[1][tid >> 6] = rho;
    }
    __syncthreads();
    if (tid == 0) {
        const int doc = g.sdoc[d];
        qp->out[doc] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        if (qp->resid) qp->resid[doc] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
}

struct Shape {
    int max_m, max_n, teams_per_block;
    void (*kern)(SinkArgs);
};

template <int R, int C, int P, int Q, int W>
constexpr Shape make_shape() {
    return Shape{C * Q * W, R * P, (W == 1) ? 4 * (64 / (R * C)) : 4 / W, &k_sink<R, C, P, Q, W>};
}

const Shape kShapes[] = {
    make_shape<4, 4, 16, 4, 1>(),    // 0: m <= 16,  16-lane teams
    make_shape<8, 4, 8, 8, 1>(),     // 1: m <= 32,  32-lane teams
    make_shape<8, 8, 8, 8, 1>(),     // 2: m <= 64,  one wave
    make_shape<4, 16, 16, 8, 1>(),   // 3: m <= 128, one wave
    make_shape<4, 16, 16, 8, 2>(),   // 4: m <= 256, two waves
    make_shape<4, 16, 16, 8, 4>(),   // 5: m <= 512, four waves
};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

}  // namespace

int sinkhorn_shape_for(int m, int max_n) {
    for (int s = 0; s < kNumShapes; ++s)
        if (m <= kShapes[s].max_m && max_n <= kShapes[s].max_n) return s;
    return -1;
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
        hipLaunchKernelGGL(k_sink_stream, dim3((unsigned)nitems), dim3(256), lds, s, a);
        return hipGetLastError();
    }
    const Shape& sh = kShapes[shape];
    const int64_t blocks = (nitems + sh.teams_per_block - 1) / sh.teams_per_block;
    hipLaunchKernelGGL(sh.kern, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace wmd
