// Internal declarations shared by the host runtime and the HIP kernels of libwmd.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "wmd.h"

namespace wmd {

// Embedding rows on the device are zero-padded to a multiple of this many
// floats, so the distance GEMM's k loop needs no tail handling.
constexpr int kRowAlign = 64;

// Per-query descriptor in device memory, read by every kernel of a query.
struct QueryDev {
    const int32_t* qid;    // m vocabulary ids of the query words
    const float* r;        // m query weights r_k (sum 1)
    const float* rinv;     // m values 1 / r_k
    float* Kt;             // U x ldk: Kt[i, k] = K[k, word(i)] (optionally column-shifted)
    float* KMt;            // U x ldk: Kt[i, k] * M[k, word(i)] (written only when km_from_k == 0)
    float* nrow;           // U: log-domain shift n_i = min_k M[k, word(i)] (shift != 0 only)
    float* x;              // N x ldk iterate x (documents in length-sorted order),
                           // used only when iterations span several launches
    double* out;           // N distances, input document order
    double* resid;         // N row-marginal residuals or nullptr
    float lambda;
    float tau2;            // squared recompute threshold of the distance epilogue
    int32_t m;             // query words (v_r)
    int32_t ldk;           // row stride of Kt / KMt / x (multiple of 4, >= m)
    int32_t iters;         // x updates
    int32_t shift;         // log-domain column shift on/off
    int32_t km_from_k;     // the final step rebuilds K .* M from K: M = n_i - ln(K) / lambda
    float inv_lambda;      // 1 / lambda (km_from_k only)
    float tol;             // > 0: stop a document once its x-change residual <= tol
    int32_t* it_out;       // N x updates made per document (input order) or nullptr
    int32_t it_base;       // x updates done before this launch (per-query launches only)
};

// Device-resident corpus (all arrays on `device`).
struct DevCorpus {
    int device = 0;
    int64_t V = 0, N = 0, nnz = 0, U = 0;
    int32_t dim = 0, ldv = 0, max_doc = 0;
    float* vecs = nullptr;          // V x ldv FP32, every vocabulary word
    float* act = nullptr;           // U x ldv FP32, the words the documents use
    float* act_norm = nullptr;      // U: |row|^2 of act
    int32_t* act_word = nullptr;    // U: vocabulary id of each act row
    uint16_t* act_bf16 = nullptr;   // U x ldv BF16 copy of act (optional)
    float* act_norm_bf16 = nullptr; // U: |bf16 row|^2 (optional)
    int32_t* sptr = nullptr;        // N+1: CSR row pointer, documents sorted by length desc
    int32_t* scol = nullptr;        // nnz: act row index of each nonzero
    float* scw = nullptr;           // nnz: normalised weight c_ij
    int32_t* sdoc = nullptr;        // N: input id of each sorted document
    float* zpad = nullptr;          // kZpadFloats: 1, 0, 0, ...: source of padding loads
};

// Floats in the corpus's padding block (1 followed by zeros), read by the
// Sinkhorn kernels in place of the rows and columns beyond a document or query.
constexpr int kZpadFloats = 1024;

// Arguments of one fused Sinkhorn launch: every (query, document) pair with
// query in qlist[0..nq) and document rank in [d_begin, d_end).
struct SinkArgs {
    const QueryDev* qd;
    const int32_t* qlist;
    int32_t nq;
    int32_t d_begin, d_end;
    const int32_t* sptr;
    const int32_t* scol;
    const float* scw;
    const int32_t* sdoc;
    int32_t it_begin;      // first iteration index handled by this launch
    int32_t it_count;      // iterations in this launch (clamped to each query's iters)
    int32_t final_step;    // nonzero: run the final u/v/WMD step at the end
    const float* zpad;     // the corpus's zero block
    // nonzero: the launch has one query whose record is qd[0]; qlist is not
    // read, so the record's load does not wait for a load of qlist
    int32_t single = 0;
    // nonzero: each query runs it_count iterations from its own it_base (its
    // record), with the final step when that reaches its iteration count;
    // it_begin and final_step are then ignored
    int32_t per_query = 0;
};

// Kernel timing by dispatch.  While `stop` is set on the calling thread, the
// query kernels are launched through hipExtLaunchKernel: the first launch
// after `start` is set writes its dispatch's start time into `start`, and
// every launch writes its dispatch's end time into `stop`.  The pair then spans
// exactly the dispatches of one phase, without the command-processor gap that
// an event record before the first launch would add.
struct DispatchClock {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
};
DispatchClock& dispatch_clock();

// launch_kernel() (launch.h, device sources only) implements it.

// ---- launchers (return hipError_t of the launch) ----
// Log-domain iteration: FP64 distance kernel (Kt of each query holds U x ldk
// doubles) and the log-sum-exp Sinkhorn, one wave per (query, document).
constexpr size_t kLseMaxLds = 160 * 1024;
size_t lse_dist_lds_bytes(int ldv);
size_t lse_sink_lds_bytes(int max_m, int max_n);
hipError_t launch_dist_lse(const DevCorpus& c, const QueryDev* qd, const int32_t* kofs, int B, int ncols,
                           hipStream_t s);
hipError_t launch_sinkhorn_lse(const SinkArgs& a, int max_m, int max_n, hipStream_t s);
// Its register-tile form: queries of at most kLseTileMaxM words against
// documents of at most kTileMaxDoc (64) words, the distance block in registers.
constexpr int kLseTileMaxM = 40;
hipError_t launch_sinkhorn_lse_tile(const SinkArgs& a, hipStream_t s);
hipError_t launch_prep_norms(const float* rows, int64_t nrows, int ldv, float* norms, hipStream_t s);
hipError_t launch_prep_bf16(const float* src, uint16_t* dst, float* norms, int64_t nrows, int ldv,
                            hipStream_t s);
hipError_t launch_prep_docs(const int32_t* ptr, const float* w, float* cw, int64_t N, hipStream_t s);
// Parameter blocks up to kUploadMaxBytes are uploaded as kernel arguments, in
// chunks of kUploadChunkBytes (one small launch each).
constexpr int kUploadChunkBytes = 2048;
constexpr int kUploadMaxBytes = 4 * kUploadChunkBytes;
hipError_t launch_upload(const void* src, size_t bytes, void* dst, hipStream_t s);
hipError_t launch_gather_rows(const float* vecs, const int32_t* ids, float* out, int64_t nrows, int ldv,
                              hipStream_t s);

// Distance GEMM + epilogue: writes Kt / KMt of every query; the queries are
// split into `groups` contiguous groups, qgroup[g] .. qgroup[g+1] (device).
// K1 over all queries of a call: kofs[B + 1] holds each query's first column
// (prefix sums of ldk, kofs[B] = ncols).  With shift, each query's nrow (U
// floats) receives its row minima and a second pass turns Kt into
// exp(-lambda (d - n)).
hipError_t launch_dist(const DevCorpus& c, const QueryDev* qd, const int32_t* kofs, int B, int ncols, int bf16,
                       int shift, hipStream_t s);
// k smallest (distance, index) pairs of n distances, ascending; scratch of
// topk_scratch_bytes(n, k) device bytes.  k <= kMaxTopK.
constexpr int kMaxTopK = WMD_MAX_TOPK;
size_t topk_scratch_bytes(int64_t n, int k);
hipError_t launch_topk(const double* dist, int64_t n, int k, void* scratch, size_t scratch_bytes, int32_t* res_idx,
                       double* res_dist, hipStream_t s);
// K1 for one short query whose parameter block (at most kUploadChunkBytes, host
// image with device pointers) travels as kernel arguments; block 0 stores it
// at params_dev for the launches that follow.  hq: the query's fields.  One
// launch, the column shift included.
bool dist_narrow_fits(const DevCorpus& c, int bf16, int B, int ncols, size_t pbytes);
hipError_t launch_dist_narrow(const DevCorpus& c, const QueryDev& hq, const void* blob,
                              size_t pbytes, size_t off_id, void* params_dev, int bf16, hipStream_t s);

// Fused Sinkhorn iterations + final WMD step.  `shape` selects the register
// tile (see k_sinkhorn.hip); shape < 0 selects the streaming kernel that
// handles any size.
int sinkhorn_num_shapes();
// -1 when only the streaming kernel fits; adaptive: the convergence check is
// on (register tiles and the streaming kernel implement it, the row-lane
// kernels do not)
int sinkhorn_shape_for(int m, int max_n, bool adaptive = false);
bool sinkhorn_shape_adaptive(int shape);
bool sinkhorn_shape_fits(int shape, int m, int max_n);
int sinkhorn_shape_max_m(int shape);
int sinkhorn_shape_max_n(int shape);
hipError_t launch_sinkhorn(int shape, const SinkArgs& a, int max_m, int max_n, hipStream_t s);

}  // namespace wmd
