// Host-side state of a corpus and its query workspace.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "wmd_internal.h"

namespace wmd {

constexpr int kMaxQueryWords = 4096;   // streaming kernel LDS: 3 floats per query word
constexpr int kMaxDocWords = 16384;    // streaming kernel LDS: 1 float per document word
constexpr int kTileMaxDoc = 64;        // documents up to this length use the register tiles
constexpr float kKmFromKMinLambda = 0.5f;  // from this lambda on, K .* M is rebuilt from K

// Device buffers of one query call.  A corpus has kWorkSlots of them, used
// round-robin, so a call can run while the previous one is still on the
// device (when the two are on different streams); a slot is reused only after
// its previous call's work has finished (event `done`, waited on the device).
struct Workspace {
    float* Kt = nullptr;
    float* KMt = nullptr;
    size_t kcap = 0;          // floats in Kt
    size_t kmcap = 0;         // floats in KMt (only queries with small lambda read it)
    float* x = nullptr;
    size_t xcap = 0;
    float* nrow = nullptr;    // per-query log-domain row shifts (U each)
    size_t ncap = 0;
    char* params = nullptr;   // device parameter block
    size_t pcap = 0;
    double* out = nullptr;    // device results of synchronous calls
    size_t ocap = 0;          // bytes
    double* h_out = nullptr;  // pinned copy of `out`
    size_t hocap = 0;
    char* tk = nullptr;       // top-k scratch and results (device)
    size_t tkcap = 0;
    char* tk_host = nullptr;  // pinned top-k results
    size_t tkhcap = 0;
    hipEvent_t done = nullptr;
    bool done_valid = false;
    hipStream_t last_stream = nullptr;   // stream of the slot's previous call
    bool carved = false;      // buffers point into memory owned elsewhere (fixed capacity)
};
constexpr int kWorkSlots = 3;   // calls cycling over three streams overlap without cross-stream waits

// Sizes and offsets of one call's workspace and parameter block.
struct Layout {
    size_t kfloats = 0, kmfloats = 0, xfloats = 0, nfloats = 0, pbytes = 0, obytes = 0;
    size_t sum_ldk = 0, sum_m = 0;
    size_t off_ql = 0, off_qg = 0, off_id = 0, off_r = 0, off_ri = 0;
    int max_m = 0, max_iters = 0, per_launch = 0;
    bool chunked = false;
    size_t device_bytes() const;
};

// Pinned host staging of the parameter blocks: a ring, so the host can enqueue
// several calls ahead of the device; slot i is reusable once its upload
// (event ev[i]) has run.
struct Staging {
    static constexpr int kSlots = 8;
    char* h[kSlots] = {};
    hipEvent_t ev[kSlots] = {};
    bool pending[kSlots] = {};
    int next = 0;
    size_t cap = 0;
};

struct PlannedQuery {
    std::vector<int32_t> ids;    // words with positive weight, input order
    std::vector<float> r, rinv;  // r_k (sum 1) and 1 / r_k, each rounded once from FP64
    int m = 0, ldk = 0, iters = 0;
    float lambda = 0.f;
};

class DeviceGuard {
  public:
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
    bool ok() const { return ok_; }

  private:
    int dev_, prev_ = -1;
    bool ok_ = false;
};

int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
// hipMalloc behind the library's fault-injection switch (WMD_TEST_FAIL_ALLOC_BYTES)
hipError_t device_alloc(void** p, size_t bytes);
extern thread_local std::string g_err;

}  // namespace wmd

struct wmd_corpus {
    wmd::DevCorpus dc;
    std::vector<int32_t> h_sorted_len;  // document lengths in sorted order, plus a trailing 0
    int64_t d_tile = 0;                 // first sorted document that fits the register tiles
    int64_t device_bytes = 0;
    std::mutex mu;
    hipStream_t stream = nullptr;       // stream of the synchronous entry points
    // timing ring: slot i holds the events of one timed call (distance phase
    // start and end, Sinkhorn phase start and end, each taken from the phase's
    // own kernel dispatches); a slot is folded into the totals before reuse
    static constexpr int kTimingSlots = 64;
    static constexpr int kTimingEvents = 4;
    hipEvent_t ev[kTimingSlots][kTimingEvents] = {};
    bool slot_pending[kTimingSlots] = {};
    int next_slot = 0, last_slot = -1;
    int32_t timing = 0;                 // 0: off; k: record every k-th call
    int64_t timing_seq = 0;
    int64_t timed_calls = 0;
    double dist_ms_total = 0.0, sink_ms_total = 0.0;
    float last_dist_ms = 0.f, last_sink_ms = 0.f;
    int last_launches = 0;
    wmd::Workspace ws[wmd::kWorkSlots];
    int next_ws = 0;
    wmd::Staging stage;
};

namespace wmd {
// host_out: results go to the workspace's output buffer (B x N distances, then
// B x N residuals when resid, then B x N int32 iteration counts when iters_out)
Layout make_layout(const wmd_corpus* c, const std::vector<PlannedQuery>& qs, const wmd_query_options& opt,
                   bool resid, bool host_out, bool iters_out = false);
int plan_query(const wmd_corpus* c, const int32_t* qids, const float* qw, int32_t n, float lambda,
               int32_t iters, int bf16, PlannedQuery* out);
// Enqueue a call on the corpus's own workspace slots; *slot receives the slot used.
int run_queries(wmd_corpus* c, const std::vector<PlannedQuery>& qs, const wmd_query_options& opt,
                double* dev_out, double* dev_res, hipStream_t stream, bool need_host_out, int* slot,
                bool iters_out = false);
int fold_timing_slot(wmd_corpus* c, int slot);
// Enqueue a call on an explicit workspace and staging ring (the server's own).
int enqueue_queries(wmd_corpus* c, const std::vector<PlannedQuery>& qs, const wmd_query_options& opt,
                    double* dev_out, double* dev_res, hipStream_t stream, bool need_host_out, Workspace& w,
                    Staging& st, bool timed, bool iters_out = false);
// Device bytes a call's workspace needs (K buffers, row shifts, iterate, results).
size_t workspace_bytes(const wmd_corpus* c, const std::vector<PlannedQuery>& qs, const wmd_query_options& opt,
                       bool resid);
void free_workspace(Workspace& w);
void carve_workspace(Workspace& w, char* base, const Layout& L);
void free_staging(Staging& st);
int check_query_options(const wmd_query_options* in, wmd_query_options* out);
// Resolve the fixed scratch array's address on device `dev` (the current
// device), once per device; the allocation-free entry point works in it.
int scratch_setup(int dev);
}  // namespace wmd
