// Host runtime of libwmd: argument validation, corpus upload, per-corpus
// workspace, query planning and kernel launches.  Every entry point declared
// in include/wmd.h except the server lives here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "wmd_corpus.h"

namespace wmd {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? WMD_ENOMEM : WMD_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Fault injection for tests: with WMD_TEST_FAIL_ALLOC_BYTES=X in the
// environment, every device allocation of at least X bytes fails as if the
// device were out of memory (read at each allocation, so a test can switch it
// on and off around one call).
hipError_t device_alloc(void** p, size_t bytes) {
    if (const char* lim = std::getenv("WMD_TEST_FAIL_ALLOC_BYTES")) {
        const unsigned long long x = std::strtoull(lim, nullptr, 10);
        if (x > 0 && bytes >= x) return hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

DeviceGuard::DeviceGuard(int dev) : dev_(dev) {
    if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
    ok_ = (prev_ == dev_) || hipSetDevice(dev_) == hipSuccess;
}
DeviceGuard::~DeviceGuard() {
    if (prev_ >= 0 && prev_ != dev_) (void)hipSetDevice(prev_);
}

namespace {

template <typename T>
hipError_t dalloc(T** p, size_t count) {
    return device_alloc(reinterpret_cast<void**>(p), std::max<size_t>(count, 1) * sizeof(T));
}

template <typename T>
void dfree(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

template <typename T>
void hfree(T*& p) {
    if (p) (void)hipHostFree(p);
    p = nullptr;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

void free_workspace(Workspace& w) {
    dfree(w.tk);
    hfree(w.tk_host);
    w.tkcap = w.tkhcap = 0;
    if (!w.carved) {
        dfree(w.Kt);
        dfree(w.KMt);
        dfree(w.x);
        dfree(w.nrow);
        dfree(w.params);
        dfree(w.out);
    }
    w.Kt = w.KMt = w.x = w.nrow = nullptr;
    w.params = nullptr;
    w.out = nullptr;
    hfree(w.h_out);
    w.kcap = w.kmcap = w.xcap = w.ncap = w.pcap = w.ocap = w.hocap = 0;
    w.carved = false;
    if (w.done) (void)hipEventDestroy(w.done);
    w.done = nullptr;
    w.done_valid = false;
    w.last_stream = nullptr;
}

void free_staging(Staging& st) {
    for (int i = 0; i < Staging::kSlots; ++i) {
        hfree(st.h[i]);
        if (st.ev[i]) (void)hipEventDestroy(st.ev[i]);
        st.ev[i] = nullptr;
        st.pending[i] = false;
    }
    st.cap = 0;
}

int check_query_options(const wmd_query_options* in, wmd_query_options* o) {
    wmd_query_options_init(o);
    if (in) *o = *in;
    if (o->precision != WMD_DIST_FP32 && o->precision != WMD_DIST_BF16)
        return fail(WMD_EINVAL, "options: unknown precision %d", o->precision);
    if (!std::isfinite(o->recompute_below)) return fail(WMD_EINVAL, "options: recompute_below not finite");
    if (o->iters_per_launch < 0) return fail(WMD_EINVAL, "options: iters_per_launch < 0");
    if (o->tile < -2 || o->tile >= sinkhorn_num_shapes())
        return fail(WMD_EINVAL, "options: tile %d outside [-2, %d)", o->tile, sinkhorn_num_shapes());
    if (!std::isfinite(o->tol) || o->tol < 0.f) return fail(WMD_EINVAL, "options: tol must be finite and >= 0");
    if (o->tol > 0.f && o->iters_per_launch > 0)
        return fail(WMD_EINVAL, "options: the convergence check (tol > 0) needs iters_per_launch = 0");
    if (o->tol > 0.f && o->tile >= 0 && !sinkhorn_shape_adaptive(o->tile))
        return fail(WMD_EINVAL, "options: tile %d has no convergence check", o->tile);
    if (o->lse && (o->precision != WMD_DIST_FP32 || o->tol > 0.f || o->iters_per_launch > 0 || o->tile != -1 ||
                   o->log_domain))
        return fail(WMD_EINVAL, "options: lse needs FP32 precision, tol = 0, iters_per_launch = 0, tile = -1 "
                                "and log_domain = 0");
    return WMD_OK;
}

// ---------------------------------------------------------------- queries

int plan_query(const wmd_corpus* c, const int32_t* qids, const float* qw, int32_t n, float lambda,
               int32_t iters, int bf16, PlannedQuery* out) {
    if (n <= 0 || !qids || !qw) return fail(WMD_EINVAL, "query: empty or null word arrays");
    if (!std::isfinite(lambda) || lambda < 0.f) return fail(WMD_EINVAL, "query: lambda must be finite and >= 0");
    if (iters < 0) return fail(WMD_EINVAL, "query: iters must be >= 0");
    if (bf16 && !c->dc.act_bf16) return fail(WMD_EINVAL, "query: BF16 distances need a corpus created with bf16 copies");
    std::vector<int32_t> sorted(qids, qids + n);
    std::sort(sorted.begin(), sorted.end());
    for (int32_t k = 0; k < n; ++k) {
        if (sorted[k] < 0 || sorted[k] >= c->dc.V) return fail(WMD_EINVAL, "query: word id %d out of range", sorted[k]);
        if (k > 0 && sorted[k] == sorted[k - 1]) return fail(WMD_EINVAL, "query: word id %d repeated", sorted[k]);
    }
    out->ids.clear();
    std::vector<double> w;
    double total = 0.0;
    for (int32_t k = 0; k < n; ++k) {
        const float wk = qw[k];
        if (!std::isfinite(wk) || wk < 0.f) return fail(WMD_EINVAL, "query: weight %d is negative or not finite", k);
        if (wk > 0.f) {   // I = (r > 0)
            out->ids.push_back(qids[k]);
            w.push_back((double)wk);
            total += (double)wk;
        }
    }
    const int m = (int)out->ids.size();
    if (m == 0) return fail(WMD_EINVAL, "query: no word with positive weight");
    if (m > kMaxQueryWords) return fail(WMD_EINVAL, "query: %d words exceed the limit of %d", m, kMaxQueryWords);
    out->r.resize(m);
    out->rinv.resize(m);
    for (int k = 0; k < m; ++k) {
        out->r[k] = (float)(w[k] / total);
        out->rinv[k] = (float)(total / w[k]);
    }
    out->m = m;
    // K block rows start on 128-byte lines once they exceed 16 floats, so a
    // document's row gather reads whole lines
    out->ldk = m <= 4 ? 4 : m <= 8 ? 8 : m <= 16 ? 16 : (int)align_up((size_t)m, 32);
    out->lambda = lambda;
    out->iters = iters;
    return WMD_OK;
}

Layout make_layout(const wmd_corpus* c, const std::vector<PlannedQuery>& qs, const wmd_query_options& opt,
                   bool resid, bool host_out, bool iters_out) {
    Layout L;
    const int B = (int)qs.size();
    const int64_t N = c->dc.N, U = c->dc.U;
    bool any_km = false;
    for (const auto& q : qs) {
        L.sum_ldk += q.ldk;
        L.sum_m += q.m;
        L.max_iters = std::max(L.max_iters, q.iters);
        L.max_m = std::max(L.max_m, q.m);
        any_km = any_km || q.lambda < kKmFromKMinLambda;
    }
    L.per_launch = opt.iters_per_launch > 0 ? opt.iters_per_launch : INT_MAX;
    L.chunked = L.per_launch < L.max_iters;
    L.kfloats = (size_t)U * L.sum_ldk * (opt.lse ? 2 : 1);   // the log-domain form keeps FP64 distances
    L.kmfloats = (any_km && !opt.lse) ? L.kfloats : 0;
    L.xfloats = L.chunked ? (size_t)N * L.sum_ldk : 0;
    L.nfloats = opt.log_domain ? (size_t)U * B : 0;
    // parameter block: QueryDev[B] | qlist[B] | kofs[B+1] | qid[sum_m] | r[sum_m] | rinv[sum_m]
    // (64-byte aligned sub-arrays: a one-query block stays small enough to
    // travel as kernel arguments)
    L.off_ql = align_up(sizeof(QueryDev) * B, 64);
    L.off_qg = align_up(L.off_ql + sizeof(int32_t) * B, 64);
    L.off_id = align_up(L.off_qg + sizeof(int32_t) * (B + 1), 64);
    L.off_r = align_up(L.off_id + sizeof(int32_t) * L.sum_m, 64);
    L.off_ri = align_up(L.off_r + sizeof(float) * L.sum_m, 64);
    L.pbytes = align_up(L.off_ri + sizeof(float) * L.sum_m, 64);
    L.obytes = host_out ? sizeof(double) * (size_t)B * N * (resid ? 2 : 1) : 0;
    if (host_out && iters_out) L.obytes += sizeof(int32_t) * (size_t)B * N;
    return L;
}

size_t Layout::device_bytes() const {
    return align_up(sizeof(float) * kfloats, 256) + align_up(sizeof(float) * kmfloats, 256) +
           align_up(sizeof(float) * xfloats, 256) + align_up(sizeof(float) * nfloats, 256) + pbytes +
           align_up(obytes, 256);
}

// Point w's buffers into one device allocation of at least L.device_bytes().
void carve_workspace(Workspace& w, char* base, const Layout& L) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base + off;
        off += align_up(bytes, 256);
        return p;
    };
    w.Kt = reinterpret_cast<float*>(take(sizeof(float) * L.kfloats));
    w.KMt = reinterpret_cast<float*>(take(sizeof(float) * L.kmfloats));
    w.x = reinterpret_cast<float*>(take(sizeof(float) * L.xfloats));
    w.nrow = reinterpret_cast<float*>(take(sizeof(float) * L.nfloats));
    w.params = take(L.pbytes);
    w.out = reinterpret_cast<double*>(take(L.obytes));
    w.kcap = L.kfloats;
    w.kmcap = L.kmfloats;
    w.xcap = L.xfloats;
    w.ncap = L.nfloats;
    w.pcap = L.pbytes;
    w.ocap = L.obytes;
    w.carved = true;
}

static int ensure_workspace(Workspace& w, const Layout& L, bool need_host_out) {
    const size_t kfloats = L.kfloats, kmfloats = L.kmfloats, xfloats = L.xfloats, nfloats = L.nfloats;
    const size_t pbytes = L.pbytes, obytes = L.obytes;
    const bool grow_dev = kfloats > w.kcap || kmfloats > w.kmcap || xfloats > w.xcap || nfloats > w.ncap ||
                          pbytes > w.pcap || obytes > w.ocap;
    if (grow_dev && w.carved) return fail(WMD_ENOMEM, "workspace: batch exceeds its carved device memory");
    const bool grow = grow_dev || (need_host_out && obytes > w.hocap);
    if (!grow) return WMD_OK;
    // nothing queued may still use this slot's old buffers
    if (w.done_valid) {
        hipError_t e = hipEventSynchronize(w.done);
        if (e != hipSuccess) return hip_fail(e, "workspace: wait for previous work");
    }
    hipError_t e = hipSuccess;
    auto grown = [](size_t need) { return need + need / 4; };
    if (kfloats > w.kcap) {
        dfree(w.Kt);
        w.kcap = 0;
        size_t cap = grown(kfloats);
        if ((e = dalloc(&w.Kt, cap)) != hipSuccess) return hip_fail(e, "workspace: K buffer");
        w.kcap = cap;
    }
    if (kmfloats > w.kmcap) {
        dfree(w.KMt);
        w.kmcap = 0;
        size_t cap = grown(kmfloats);
        if ((e = dalloc(&w.KMt, cap)) != hipSuccess) return hip_fail(e, "workspace: K.*M buffer");
        w.kmcap = cap;
    }
    if (xfloats > w.xcap) {
        dfree(w.x);
        w.xcap = 0;
        size_t cap = grown(xfloats);
        if ((e = dalloc(&w.x, cap)) != hipSuccess) return hip_fail(e, "workspace: x buffer");
        w.xcap = cap;
    }
    if (nfloats > w.ncap) {
        dfree(w.nrow);
        w.ncap = 0;
        size_t cap = grown(nfloats);
        if ((e = dalloc(&w.nrow, cap)) != hipSuccess) return hip_fail(e, "workspace: row shifts");
        w.ncap = cap;
    }
    if (pbytes > w.pcap) {
        dfree(w.params);
        w.pcap = 0;
        size_t cap = grown(pbytes);
        if ((e = dalloc(&w.params, cap)) != hipSuccess) return hip_fail(e, "workspace: query parameters");
        w.pcap = cap;
    }
    if (obytes > w.ocap) {
        dfree(w.out);
        w.ocap = 0;
        size_t cap = grown(obytes);
        if ((e = dalloc(reinterpret_cast<char**>(&w.out), cap)) != hipSuccess)
            return hip_fail(e, "workspace: output buffer");
        w.ocap = cap;
    }
    if (need_host_out && obytes > w.hocap) {
        hfree(w.h_out);
        w.hocap = 0;
        size_t cap = grown(obytes);
        if ((e = hipHostMalloc(reinterpret_cast<void**>(&w.h_out), cap, hipHostMallocDefault)) != hipSuccess)
            return hip_fail(e, "workspace: pinned output");
        w.hocap = cap;
    }
    return WMD_OK;
}

// A pinned staging slot of at least `bytes`, free for writing.
static int take_staging(Staging& st, size_t bytes, int* slot_out) {
    hipError_t e;
    if (bytes > st.cap) {
        for (int i = 0; i < Staging::kSlots; ++i) {
            if (st.pending[i] && (e = hipEventSynchronize(st.ev[i])) != hipSuccess)
                return hip_fail(e, "staging: wait");
            st.pending[i] = false;
            hfree(st.h[i]);
        }
        st.cap = 0;
        const size_t cap = bytes + bytes / 4;
        for (int i = 0; i < Staging::kSlots; ++i)
            if ((e = hipHostMalloc(reinterpret_cast<void**>(&st.h[i]), cap, hipHostMallocDefault)) != hipSuccess)
                return hip_fail(e, "staging: pinned allocation");
        st.cap = cap;
    }
    const int slot = st.next;
    st.next = (st.next + 1) % Staging::kSlots;
    if (st.pending[slot]) {
        if ((e = hipEventSynchronize(st.ev[slot])) != hipSuccess) return hip_fail(e, "staging: wait");
        st.pending[slot] = false;
    }
    *slot_out = slot;
    return WMD_OK;
}

DispatchClock& dispatch_clock() {
    thread_local DispatchClock clock;
    return clock;
}

namespace {

// Clears the calling thread's dispatch clock when it leaves scope.
struct ClockReset {
    ~ClockReset() { dispatch_clock() = DispatchClock{}; }
};

// End of a timed phase: a phase that launched nothing records both of its
// events here, so its duration reads as zero.
hipError_t close_phase(hipStream_t s) {
    DispatchClock& k = dispatch_clock();
    if (!k.start) return hipSuccess;
    hipError_t e = hipEventRecord(k.start, s);
    return e != hipSuccess ? e : hipEventRecord(k.stop, s);
}

}  // namespace

// Wait for a timed call's events and add its kernel times to the totals.
int fold_timing_slot(wmd_corpus* c, int slot) {
    hipError_t e;
    float d = 0.f, k = 0.f;
    if ((e = hipEventSynchronize(c->ev[slot][3])) != hipSuccess) return hip_fail(e, "timing: wait");
    if ((e = hipEventElapsedTime(&d, c->ev[slot][0], c->ev[slot][1])) != hipSuccess ||
        (e = hipEventElapsedTime(&k, c->ev[slot][2], c->ev[slot][3])) != hipSuccess)
        return hip_fail(e, "timing: elapsed");
    c->slot_pending[slot] = false;
    c->timed_calls += 1;
    c->dist_ms_total += d;
    c->sink_ms_total += k;
    if (slot == c->last_slot) {
        c->last_dist_ms = d;
        c->last_sink_ms = k;
    }
    return WMD_OK;
}

// Enqueue K1 + the fused Sinkhorn launches for `qs` on `stream`.  Row b of
// dev_out (and dev_res when non-null) receives query b's N results.
int run_queries(wmd_corpus* c, const std::vector<PlannedQuery>& qs, const wmd_query_options& opt,
                double* dev_out, double* dev_res, hipStream_t stream, bool need_host_out, int* slot_used,
                bool iters_out) {
    const int wslot = c->next_ws;
    c->next_ws = (c->next_ws + 1) % kWorkSlots;
    *slot_used = wslot;
    // timing on: every c->timing-th call records its kernel events
    const bool timed = c->timing > 0 && (c->timing_seq++ % c->timing) == 0;
    return enqueue_queries(c, qs, opt, dev_out, dev_res, stream, need_host_out, c->ws[wslot], c->stage, timed,
                           iters_out);
}

size_t workspace_bytes(const wmd_corpus* c, const std::vector<PlannedQuery>& qs, const wmd_query_options& opt,
                       bool resid) {
    return make_layout(c, qs, opt, resid, true).device_bytes();
}

int enqueue_queries(wmd_corpus* c, const std::vector<PlannedQuery>& qs, const wmd_query_options& opt,
                    double* dev_out, double* dev_res, hipStream_t stream, bool need_host_out, Workspace& w,
                    Staging& st, bool timed, bool iters_out) {
    const DevCorpus& dc = c->dc;
    const int B = (int)qs.size();
    const int64_t N = dc.N, U = dc.U;
    const Layout L = make_layout(c, qs, opt, dev_res != nullptr, need_host_out, iters_out);
    const int max_m = L.max_m, max_iters = L.max_iters, per_launch = L.per_launch;
    const bool chunked = L.chunked;
    const size_t sum_ldk = L.sum_ldk;
    const size_t off_ql = L.off_ql, off_qg = L.off_qg, off_id = L.off_id, off_r = L.off_r, off_ri = L.off_ri;
    const size_t pbytes = L.pbytes;
    (void)max_iters;
    if (opt.tile >= 0 && !sinkhorn_shape_fits(opt.tile, max_m, 1))
        return fail(WMD_EINVAL, "options: tile %d cannot hold a %d-word query", opt.tile, max_m);
    if (opt.lse && (lse_dist_lds_bytes(dc.ldv) > kLseMaxLds || lse_sink_lds_bytes(max_m, dc.max_doc) > kLseMaxLds))
        return fail(WMD_EINVAL, "options: lse: a %d-word query against %d-word documents (dimension %d) exceeds "
                                "the local memory of one workgroup", max_m, dc.max_doc, dc.dim);
    int rc = ensure_workspace(w, L, need_host_out);
    if (rc) return rc;
    int32_t* dev_iters = nullptr;
    if (need_host_out) {
        dev_out = w.out;
        if (dev_res) dev_res = w.out + (size_t)B * N;
        if (iters_out) dev_iters = reinterpret_cast<int32_t*>(w.out + (size_t)B * N * (dev_res ? 2 : 1));
    }

    // small parameter blocks go up as kernel arguments (built in host memory
    // here), larger ones through a pinned staging slot and a copy
    const bool by_args = pbytes <= (size_t)kUploadMaxBytes;
    thread_local std::vector<char> arg_block;
    int slot_s = -1;
    char* hp = nullptr;
    if (by_args) {
        arg_block.assign(pbytes, 0);
        hp = arg_block.data();
    } else {
        if ((rc = take_staging(st, pbytes, &slot_s))) return rc;
        hp = st.h[slot_s];
    }
    char* dp = w.params;
    QueryDev* hq = reinterpret_cast<QueryDev*>(hp);
    int32_t* hql = reinterpret_cast<int32_t*>(hp + off_ql);
    int32_t* hqg = reinterpret_cast<int32_t*>(hp + off_qg);
    int32_t* hid = reinterpret_cast<int32_t*>(hp + off_id);
    float* hr = reinterpret_cast<float*>(hp + off_r);
    float* hri = reinterpret_cast<float*>(hp + off_ri);
    const float tau = opt.recompute_below >= 0.f ? opt.recompute_below
                                                 : (opt.precision == WMD_DIST_BF16 ? 1e-2f : 0.5f);
    size_t ko = 0, mo = 0;
    for (int b = 0; b < B; ++b) {
        const PlannedQuery& q = qs[b];
        QueryDev& d = hq[b];
        d.qid = reinterpret_cast<const int32_t*>(dp + off_id) + mo;
        d.r = reinterpret_cast<const float*>(dp + off_r) + mo;
        d.rinv = reinterpret_cast<const float*>(dp + off_ri) + mo;
        d.Kt = w.Kt + (size_t)U * ko * (opt.lse ? 2 : 1);   // log domain: U x ldk doubles per query
        d.KMt = L.kmfloats ? w.KMt + (size_t)U * ko : nullptr;
        d.x = chunked ? w.x + (size_t)N * ko : nullptr;
        d.out = dev_out + (size_t)b * N;
        d.resid = dev_res ? dev_res + (size_t)b * N : nullptr;
        d.lambda = q.lambda;
        d.tau2 = tau * tau;
        d.m = q.m;
        d.ldk = q.ldk;
        d.iters = q.iters;
        d.shift = opt.log_domain ? 1 : 0;
        d.nrow = opt.log_domain ? w.nrow + (size_t)U * b : nullptr;
        d.km_from_k = q.lambda >= kKmFromKMinLambda ? 1 : 0;
        d.inv_lambda = d.km_from_k ? 1.0f / q.lambda : 0.f;
        d.tol = opt.tol;
        d.it_out = dev_iters ? dev_iters + (size_t)b * N : nullptr;
        d.it_base = 0;
        std::memcpy(hid + mo, q.ids.data(), sizeof(int32_t) * q.m);
        std::memcpy(hr + mo, q.r.data(), sizeof(float) * q.m);
        std::memcpy(hri + mo, q.rinv.data(), sizeof(float) * q.m);
        ko += q.ldk;
        mo += q.m;
    }
    hqg[0] = 0;   // kofs: first global distance-GEMM column of each query
    for (int b = 0; b < B; ++b) hqg[b + 1] = hqg[b] + qs[b].ldk;
    // group queries by Sinkhorn launch shape: streaming-only first, then each register shape
    std::vector<int> shape_of(B);
    const int nshape = sinkhorn_num_shapes();
    std::vector<int> cnt(nshape + 1, 0);
    for (int b = 0; b < B; ++b) {
        if (opt.lse) shape_of[b] = qs[b].m <= kLseTileMaxM ? 0 : -1;   // log-domain register tile or stream form
        else if (opt.tile == -2) shape_of[b] = -1;
        else if (opt.tile >= 0) shape_of[b] = opt.tile;
        else shape_of[b] = sinkhorn_shape_for(qs[b].m, kTileMaxDoc, opt.tol > 0.f);
        cnt[shape_of[b] + 1]++;
    }
    std::vector<int> start(nshape + 2, 0);
    for (int s = 0; s <= nshape; ++s) start[s + 1] = start[s] + cnt[s];
    {
        std::vector<int> fill(start.begin(), start.end() - 1);
        for (int b = 0; b < B; ++b) hql[fill[shape_of[b] + 1]++] = b;
    }

    hipError_t e;
    // the slot's previous call must be done with its buffers; on the same
    // stream that order holds already
    if (w.done_valid && w.last_stream != stream && (e = hipStreamWaitEvent(stream, w.done, 0)) != hipSuccess)
        return hip_fail(e, "query: order after the slot's previous call");
    // one short query: its parameters ride along with the distance kernel
    const int bf16 = opt.precision == WMD_DIST_BF16 ? 1 : 0;
    const bool narrow = !opt.lse && by_args && dist_narrow_fits(dc, bf16, B, (int)sum_ldk, pbytes);
    if (by_args) {
        if (!narrow && (e = launch_upload(hp, pbytes, dp, stream)) != hipSuccess)
            return hip_fail(e, "query: upload parameters");
    } else {
        if ((e = hipMemcpyAsync(dp, hp, pbytes, hipMemcpyHostToDevice, stream)) != hipSuccess)
            return hip_fail(e, "query: upload parameters");
        if ((e = hipEventRecord(st.ev[slot_s], stream)) != hipSuccess) return hip_fail(e, "query: record");
        st.pending[slot_s] = true;
    }

    const QueryDev* dq = reinterpret_cast<const QueryDev*>(dp);
    const int32_t* dql = reinterpret_cast<const int32_t*>(dp + off_ql);
    int launches = 0;
    int slot = -1;
    ClockReset clock_reset;   // the dispatch clock is off again however this returns
    if (timed) {
        slot = c->next_slot;
        c->next_slot = (c->next_slot + 1) % wmd_corpus::kTimingSlots;
        if (c->slot_pending[slot] && (rc = fold_timing_slot(c, slot))) return rc;
        dispatch_clock() = DispatchClock{c->ev[slot][0], c->ev[slot][1]};
    }
    const int32_t* dqg = reinterpret_cast<const int32_t*>(dp + off_qg);
    if (opt.lse) e = launch_dist_lse(dc, dq, dqg, B, (int)sum_ldk, stream);
    else if (narrow) e = launch_dist_narrow(dc, hq[0], hp, pbytes, off_id, dp, bf16, stream);
    else e = launch_dist(dc, dq, dqg, B, (int)sum_ldk, bf16, opt.log_domain, stream);
    if (e != hipSuccess) return hip_fail(e, "query: distance kernel launch");
    ++launches;
    if (slot >= 0) {
        if ((e = close_phase(stream)) != hipSuccess) return hip_fail(e, "query: record");
        dispatch_clock() = DispatchClock{c->ev[slot][2], c->ev[slot][3]};
    }

    const int d_tile = (int)c->d_tile;   // sorted docs [d_tile, N) fit the register tiles
    if (opt.lse) {
        // queries of at most kLseTileMaxM words against documents that fit the
        // register tiles: the tile form; everything else: the stream form
        auto golse = [&](bool tile, int q0, int q1, int d0, int d1) -> hipError_t {
            if (q1 <= q0 || d1 <= d0) return hipSuccess;
            SinkArgs a;
            a.qd = dq;
            a.qlist = dql + q0;
            a.nq = q1 - q0;
            a.d_begin = d0;
            a.d_end = d1;
            a.sptr = dc.sptr;
            a.scol = dc.scol;
            a.scw = dc.scw;
            a.sdoc = dc.sdoc;
            a.zpad = dc.zpad;
            a.it_begin = 0;
            a.it_count = max_iters;
            a.final_step = 1;
            int mm = 0;
            for (int i = q0; i < q1; ++i) mm = std::max(mm, qs[hql[i]].m);
            ++launches;
            return tile ? launch_sinkhorn_lse_tile(a, stream) : launch_sinkhorn_lse(a, mm, c->h_sorted_len[d0], stream);
        };
        if ((e = golse(false, start[0], start[1], 0, (int)N)) != hipSuccess ||
            (e = golse(false, start[1], B, 0, d_tile)) != hipSuccess ||
            (e = golse(true, start[1], B, d_tile, (int)N)) != hipSuccess)
            return hip_fail(e, "query: log-domain sinkhorn launch");
    }
    for (int it0 = 0; !opt.lse; it0 += per_launch) {
        SinkArgs a;
        a.qd = dq;
        a.sptr = dc.sptr;
        a.scol = dc.scol;
        a.scw = dc.scw;
        a.sdoc = dc.sdoc;
        a.zpad = dc.zpad;
        a.it_begin = it0;
        a.it_count = per_launch;
        a.final_step = (int64_t)it0 + per_launch >= max_iters ? 1 : 0;
        auto go = [&](int shape, int q0, int q1, int d0, int d1) -> hipError_t {
            if (q1 <= q0 || d1 <= d0) return hipSuccess;
            a.qlist = dql + q0;
            a.nq = q1 - q0;
            a.single = (a.nq == 1) ? 1 : 0;
            a.qd = a.single ? dq + hql[q0] : dq;
            a.d_begin = d0;
            a.d_end = d1;
            int mm = 0;
            for (int i = q0; i < q1; ++i) mm = std::max(mm, qs[hql[i]].m);
            ++launches;
            return launch_sinkhorn(shape, a, mm, c->h_sorted_len[d0], stream);
        };
        // queries too long for any register tile: streaming kernel over every document
        if ((e = go(-1, start[0], start[1], 0, (int)N)) != hipSuccess) return hip_fail(e, "query: sinkhorn launch");
        // documents too long for the register tiles: streaming kernel
        if ((e = go(-1, start[1], B, 0, d_tile)) != hipSuccess) return hip_fail(e, "query: sinkhorn launch");
        for (int s = 0; s < nshape; ++s)
            if ((e = go(s, start[s + 1], start[s + 2], d_tile, (int)N)) != hipSuccess)
                return hip_fail(e, "query: sinkhorn launch");
        if (a.final_step) break;
    }
    if (slot >= 0) {
        if ((e = close_phase(stream)) != hipSuccess) return hip_fail(e, "query: record");
        dispatch_clock() = DispatchClock{};
        c->slot_pending[slot] = true;
        c->last_slot = slot;
        c->last_launches = launches;
    }
    if (w.done) {   // a workspace without an event (fixed scratch) orders nothing
        if ((e = hipEventRecord(w.done, stream)) != hipSuccess) return hip_fail(e, "query: record");
        w.done_valid = true;
        w.last_stream = stream;
    }
    return WMD_OK;
}

}  // namespace wmd

using namespace wmd;

// ---------------------------------------------------------------- C ABI

extern "C" {

const char* wmd_last_error(void) { return g_err.c_str(); }

void wmd_corpus_options_init(wmd_corpus_options* opt) {
    if (!opt) return;
    opt->device = -1;
    opt->bf16 = 0;
}

void wmd_query_options_init(wmd_query_options* opt) {
    if (!opt) return;
    opt->precision = WMD_DIST_FP32;
    opt->recompute_below = -1.f;
    opt->log_domain = 0;
    opt->iters_per_launch = 0;
    opt->tile = -1;
    opt->tol = 0.f;
    opt->lse = 0;
}

static void corpus_free(wmd_corpus* c) {
    DevCorpus& d = c->dc;
    dfree(d.vecs);
    dfree(d.act);
    dfree(d.act_norm);
    dfree(d.act_word);
    dfree(d.act_bf16);
    dfree(d.act_norm_bf16);
    dfree(d.sptr);
    dfree(d.scol);
    dfree(d.scw);
    dfree(d.sdoc);
    dfree(d.zpad);
    for (int sl = 0; sl < kWorkSlots; ++sl) free_workspace(c->ws[sl]);
    free_staging(c->stage);
    for (int i = 0; i < wmd_corpus::kTimingSlots; ++i)
        for (int j = 0; j < wmd_corpus::kTimingEvents; ++j)
            if (c->ev[i][j]) (void)hipEventDestroy(c->ev[i][j]);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

// Documents of equal length are interchangeable for the kernels (a wave's rows
// per lane depend on the lengths only, and every document's result on itself
// only), so within each run of equal length the order puts documents that
// share words on the same XCD.  A word's K row is fetched from memory once per
// XCD whose L2 misses it, and the register-tile launch of a query (8
// documents per block for the 17-48-word tiles) sends block b to XCD b mod 8:
// sorted position p, counted from the first document of at most kTileMaxDoc
// words, runs on XCD (p / 8) mod 8 (for every query of a batch alike, up to a
// rotation).  Greedy: the documents of a run in order of their rarest word,
// each to the XCD with positions left in the run that already holds most of
// its words.  Longer documents (the streaming kernel) keep their order.
static void cluster_by_xcd(std::vector<int32_t>& order, const std::vector<int32_t>& len,
                           const std::vector<int64_t>& fptr, const std::vector<int32_t>& ids,
                           const std::vector<int32_t>& remap, int64_t U) {
    constexpr int kXcds = 8, kDocsPerBlock = 8;
    const int64_t N = (int64_t)order.size();
    int64_t p0 = 0;
    while (p0 < N && len[order[p0]] > kTileMaxDoc) ++p0;
    const int64_t d_tile = p0;
    std::vector<int32_t> df((size_t)U, 0);
    for (int32_t id : ids) ++df[remap[id]];
    std::vector<uint8_t> on((size_t)U * kXcds, 0);   // on[w * 8 + x]: word w's row is on XCD x
    auto xcd_of = [&](int64_t p) { return (int)(((p - d_tile) / kDocsPerBlock) % kXcds); };
    std::vector<int32_t> run, key, bins[kXcds];
    while (p0 < N) {
        int64_t p1 = p0;
        while (p1 < N && len[order[p1]] == len[order[p0]]) ++p1;
        int quota[kXcds] = {0};
        for (int64_t p = p0; p < p1; ++p) ++quota[xcd_of(p)];
        run.assign(order.begin() + p0, order.begin() + p1);
        key.assign(run.size(), 0);
        for (size_t i = 0; i < run.size(); ++i) {
            int32_t k = INT32_MAX;
            for (int64_t e = fptr[run[i]]; e < fptr[run[i] + 1]; ++e) k = std::min(k, df[remap[ids[e]]]);
            key[i] = k;
        }
        std::vector<size_t> idx(run.size());
        for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
        std::stable_sort(idx.begin(), idx.end(), [&](size_t x, size_t y) { return key[x] < key[y]; });
        for (auto& b : bins) b.clear();
        for (size_t i : idx) {
            const int32_t j = run[i];
            int best = -1;
            int64_t best_new = INT64_MAX;
            for (int x = 0; x < kXcds; ++x) {
                if ((int)bins[x].size() >= quota[x]) continue;
                int64_t fresh = 0;
                for (int64_t e = fptr[j]; e < fptr[j + 1]; ++e) fresh += on[(size_t)remap[ids[e]] * kXcds + x] == 0;
                if (fresh < best_new) {
                    best_new = fresh;
                    best = x;
                }
            }
            bins[best].push_back(j);
            for (int64_t e = fptr[j]; e < fptr[j + 1]; ++e) on[(size_t)remap[ids[e]] * kXcds + best] = 1;
        }
        size_t next[kXcds] = {0};
        for (int64_t p = p0; p < p1; ++p) {
            const int x = xcd_of(p);
            order[p] = bins[x][next[x]++];
        }
        p0 = p1;
    }
}

int wmd_corpus_create(const float* vecs, int64_t V, int32_t dim, const int64_t* doc_ptr,
                      const int32_t* word_ids, const float* weights, int64_t N,
                      const wmd_corpus_options* opt_in, wmd_corpus** out) {
    if (!out) return fail(WMD_EINVAL, "corpus: null output handle");
    if (!vecs || !doc_ptr || (!word_ids && N > 0) || (!weights && N > 0))
        return fail(WMD_EINVAL, "corpus: null input array");
    if (V <= 0 || V > INT32_MAX) return fail(WMD_EINVAL, "corpus: V must be in [1, 2^31)");
    if (dim <= 0) return fail(WMD_EINVAL, "corpus: dim must be > 0");
    if (N <= 0 || N > INT32_MAX) return fail(WMD_EINVAL, "corpus: N must be in [1, 2^31)");
    wmd_corpus_options opt;
    wmd_corpus_options_init(&opt);
    if (opt_in) opt = *opt_in;
    if (doc_ptr[0] != 0) return fail(WMD_EINVAL, "corpus: doc_ptr[0] must be 0");
    for (int64_t j = 0; j < N; ++j)
        if (doc_ptr[j + 1] < doc_ptr[j]) return fail(WMD_EINVAL, "corpus: doc_ptr decreases at %lld", (long long)j);
    const int64_t nnz_in = doc_ptr[N];

    // validate, drop zero weights, mark the vocabulary in use
    std::vector<int32_t> stamp((size_t)V, -1);
    std::vector<int32_t> remap((size_t)V, -1);
    std::vector<int32_t> len((size_t)N);
    std::vector<int32_t> ids;
    std::vector<float> wts;
    std::vector<int64_t> fptr((size_t)N + 1, 0);
    ids.reserve((size_t)nnz_in);
    wts.reserve((size_t)nnz_in);
    for (int64_t j = 0; j < N; ++j) {
        for (int64_t p = doc_ptr[j]; p < doc_ptr[j + 1]; ++p) {
            const int32_t id = word_ids[p];
            const float wt = weights[p];
            if (id < 0 || id >= V) return fail(WMD_EINVAL, "corpus: document %lld has word id %d out of range", (long long)j, id);
            if (stamp[id] == (int32_t)j) return fail(WMD_EINVAL, "corpus: document %lld repeats word %d", (long long)j, id);
            stamp[id] = (int32_t)j;
            if (!std::isfinite(wt) || wt < 0.f)
                return fail(WMD_EINVAL, "corpus: document %lld has a negative or non-finite weight", (long long)j);
            if (wt > 0.f) {
                ids.push_back(id);
                wts.push_back(wt);
                remap[id] = 0;
            }
        }
        fptr[j + 1] = (int64_t)ids.size();
        len[j] = (int32_t)(fptr[j + 1] - fptr[j]);
        if (len[j] == 0) return fail(WMD_EINVAL, "corpus: document %lld has no word with positive weight", (long long)j);
        if (len[j] > kMaxDocWords)
            return fail(WMD_EINVAL, "corpus: document %lld has %d words, above the limit of %d", (long long)j, len[j], kMaxDocWords);
    }
    const int64_t nnz = (int64_t)ids.size();
    if (nnz > INT32_MAX) return fail(WMD_EINVAL, "corpus: more than 2^31-1 nonzeros");
    std::vector<int32_t> act_word;
    for (int64_t i = 0; i < V; ++i)
        if (remap[i] == 0) {
            remap[i] = (int32_t)act_word.size();
            act_word.push_back((int32_t)i);
        }
    const int64_t U = (int64_t)act_word.size();
    // documents sorted by length, longest first (stable), then within each
    // run of equal length grouped by the XCD that will run them
    std::vector<int32_t> order((size_t)N);
    for (int64_t j = 0; j < N; ++j) order[j] = (int32_t)j;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return len[x] > len[y]; });
    cluster_by_xcd(order, len, fptr, ids, remap, U);
    std::vector<int32_t> sptr((size_t)N + 1, 0), scol((size_t)nnz), slen((size_t)N);
    std::vector<float> sw((size_t)nnz);
    for (int64_t d = 0; d < N; ++d) {
        const int32_t j = order[d];
        slen[d] = len[j];
        sptr[d + 1] = sptr[d] + len[j];
        for (int32_t t = 0; t < len[j]; ++t) {
            scol[sptr[d] + t] = remap[ids[fptr[j] + t]];
            sw[sptr[d] + t] = wts[fptr[j] + t];
        }
    }

    int dev = opt.device;
    if (dev < 0 && hipGetDevice(&dev) != hipSuccess) return fail(WMD_EDEVICE, "corpus: no current HIP device");
    DeviceGuard guard(dev);
    if (!guard.ok()) return fail(WMD_EDEVICE, "corpus: cannot select HIP device %d", dev);
    int rc_scratch = scratch_setup(dev);
    if (rc_scratch) return rc_scratch;

    wmd_corpus* c = new wmd_corpus();
    DevCorpus& d = c->dc;
    d.device = dev;
    d.V = V;
    d.N = N;
    d.nnz = nnz;
    d.U = U;
    d.dim = dim;
    d.ldv = (int32_t)align_up((size_t)dim, kRowAlign);
    d.max_doc = slen[0];
    c->h_sorted_len = slen;
    c->h_sorted_len.push_back(0);
    c->d_tile = 0;
    while (c->d_tile < N && slen[c->d_tile] > kTileMaxDoc) ++c->d_tile;

    hipError_t e = hipSuccess;
    auto bail = [&](hipError_t err, const char* what) {
        int code = hip_fail(err, what);
        (void)hipDeviceSynchronize();
        corpus_free(c);
        return code;
    };
    if ((e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking)) != hipSuccess) return bail(e, "corpus: stream");
    for (int sl = 0; sl < kWorkSlots; ++sl)
        if ((e = hipEventCreateWithFlags(&c->ws[sl].done, hipEventDisableTiming)) != hipSuccess)
            return bail(e, "corpus: events");
    for (int i = 0; i < Staging::kSlots; ++i)
        if ((e = hipEventCreateWithFlags(&c->stage.ev[i], hipEventDisableTiming)) != hipSuccess)
            return bail(e, "corpus: events");
    for (int i = 0; i < wmd_corpus::kTimingSlots; ++i)
        for (int j = 0; j < wmd_corpus::kTimingEvents; ++j)
            if ((e = hipEventCreate(&c->ev[i][j])) != hipSuccess) return bail(e, "corpus: timing events");
    const size_t ldv = (size_t)d.ldv;
    if ((e = dalloc(&d.vecs, (size_t)V * ldv)) != hipSuccess || (e = dalloc(&d.act, (size_t)U * ldv)) != hipSuccess ||
        (e = dalloc(&d.act_norm, (size_t)U)) != hipSuccess || (e = dalloc(&d.act_word, (size_t)U)) != hipSuccess ||
        (e = dalloc(&d.sptr, (size_t)N + 1)) != hipSuccess || (e = dalloc(&d.scol, (size_t)nnz)) != hipSuccess ||
        (e = dalloc(&d.scw, (size_t)nnz)) != hipSuccess || (e = dalloc(&d.sdoc, (size_t)N)) != hipSuccess ||
        (e = dalloc(&d.zpad, (size_t)kZpadFloats)) != hipSuccess)
        return bail(e, "corpus: device allocation");
    if (opt.bf16) {
        if ((e = dalloc(&d.act_bf16, (size_t)U * ldv)) != hipSuccess ||
            (e = dalloc(&d.act_norm_bf16, (size_t)U)) != hipSuccess)
            return bail(e, "corpus: BF16 allocation");
    }
    std::vector<float> zpad((size_t)kZpadFloats, 0.f);
    zpad[0] = 1.f;
    hipStream_t s = c->stream;
    if ((e = hipMemsetAsync(d.vecs, 0, (size_t)V * ldv * sizeof(float), s)) != hipSuccess ||
        (e = hipMemcpy2DAsync(d.vecs, ldv * sizeof(float), vecs, (size_t)dim * sizeof(float),
                              (size_t)dim * sizeof(float), (size_t)V, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(d.act_word, act_word.data(), sizeof(int32_t) * U, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(d.sptr, sptr.data(), sizeof(int32_t) * (N + 1), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(d.scol, scol.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(d.scw, sw.data(), sizeof(float) * nnz, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(d.sdoc, order.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(d.zpad, zpad.data(), sizeof(float) * kZpadFloats, hipMemcpyHostToDevice, s)) != hipSuccess)
        return bail(e, "corpus: upload");
    if ((e = launch_gather_rows(d.vecs, d.act_word, d.act, U, d.ldv, s)) != hipSuccess ||
        (e = launch_prep_norms(d.act, U, d.ldv, d.act_norm, s)) != hipSuccess ||
        (e = launch_prep_docs(d.sptr, d.scw, d.scw, N, s)) != hipSuccess)
        return bail(e, "corpus: preparation kernels");
    if (opt.bf16 && (e = launch_prep_bf16(d.act, d.act_bf16, d.act_norm_bf16, U, d.ldv, s)) != hipSuccess)
        return bail(e, "corpus: BF16 preparation");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return bail(e, "corpus: preparation");
    c->device_bytes = (int64_t)((V + U) * ldv * sizeof(float) + U * (sizeof(float) + sizeof(int32_t)) +
                                (N + 1 + N) * sizeof(int32_t) + nnz * (sizeof(int32_t) + sizeof(float)) +
                                kZpadFloats * sizeof(float) + (opt.bf16 ? U * (ldv * sizeof(uint16_t) + sizeof(float)) : 0));
    *out = c;
    return WMD_OK;
}

void wmd_corpus_destroy(wmd_corpus* c) {
    if (!c) return;
    DeviceGuard guard(c->dc.device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (int sl = 0; sl < kWorkSlots; ++sl)
        if (c->ws[sl].done_valid) (void)hipEventSynchronize(c->ws[sl].done);
    corpus_free(c);
}

int wmd_corpus_info_get(const wmd_corpus* c, wmd_corpus_info* out) {
    if (!c || !out) return fail(WMD_EINVAL, "info: null argument");
    out->V = c->dc.V;
    out->N = c->dc.N;
    out->nnz = c->dc.nnz;
    out->U = c->dc.U;
    out->dim = c->dc.dim;
    out->max_doc_words = c->dc.max_doc;
    out->device = c->dc.device;
    out->has_bf16 = c->dc.act_bf16 != nullptr;
    out->device_bytes = c->device_bytes;
    return WMD_OK;
}

static int batch_plan(wmd_corpus* c, int32_t B, const int64_t* q_ptr, const int32_t* qids, const float* qw,
                      const float* lambdas, const int32_t* iters, const wmd_query_options& o,
                      std::vector<PlannedQuery>* qs) {
    if (B <= 0 || !q_ptr || !lambdas || !iters) return fail(WMD_EINVAL, "batch: bad arguments");
    if (q_ptr[0] != 0) return fail(WMD_EINVAL, "batch: q_ptr[0] must be 0");
    qs->resize(B);
    for (int32_t b = 0; b < B; ++b) {
        const int64_t n = q_ptr[b + 1] - q_ptr[b];
        if (n <= 0 || n > INT32_MAX) return fail(WMD_EINVAL, "batch: query %d has no words", b);
        int rc = plan_query(c, qids + q_ptr[b], qw + q_ptr[b], (int32_t)n, lambdas[b], iters[b],
                            o.precision == WMD_DIST_BF16, &(*qs)[b]);
        if (rc) {
            std::string msg = g_err;
            return fail(rc, "batch query %d: %s", b, msg.c_str());
        }
    }
    return WMD_OK;
}

static int finish_sync(wmd_corpus* c, int slot, int B, double* out_dist, double* out_resid) {
    Workspace& w = c->ws[slot];
    const size_t n = (size_t)B * c->dc.N;
    const size_t bytes = sizeof(double) * n * (out_resid ? 2 : 1);
    hipError_t e;
    if ((e = hipMemcpyAsync(w.h_out, w.out, bytes, hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
        return hip_fail(e, "query: download results");
    if ((e = hipEventRecord(w.done, c->stream)) != hipSuccess) return hip_fail(e, "query: record");
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(e, "query: execution");
    std::memcpy(out_dist, w.h_out, sizeof(double) * n);
    if (out_resid) std::memcpy(out_resid, w.h_out + n, sizeof(double) * n);
    return WMD_OK;
}

int wmd_query(wmd_corpus* c, const int32_t* qids, const float* qweights, int32_t n, float lambda, int32_t iters,
              const wmd_query_options* opt, double* out_dist, double* out_resid) {
    if (!c || !out_dist) return fail(WMD_EINVAL, "query: null corpus or output");
    wmd_query_options o;
    int rc = wmd::check_query_options(opt, &o);
    if (rc) return rc;
    std::vector<PlannedQuery> qs(1);
    if ((rc = plan_query(c, qids, qweights, n, lambda, iters, o.precision == WMD_DIST_BF16, &qs[0]))) return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard guard(c->dc.device);
    if (!guard.ok()) return fail(WMD_EDEVICE, "query: cannot select device");
    double dummy = 0.0;
    int slot = 0;
    if ((rc = run_queries(c, qs, o, &dummy, out_resid ? &dummy : nullptr, c->stream, true, &slot))) return rc;
    return finish_sync(c, slot, 1, out_dist, out_resid);
}

int wmd_query_adaptive(wmd_corpus* c, const int32_t* qids, const float* qweights, int32_t n, float lambda,
                       int32_t max_iters, const wmd_query_options* opt, double* out_dist, double* out_resid,
                       int32_t* out_iters) {
    if (!c || !out_dist) return fail(WMD_EINVAL, "query: null corpus or output");
    wmd_query_options o;
    int rc = wmd::check_query_options(opt, &o);
    if (rc) return rc;
    std::vector<PlannedQuery> qs(1);
    if ((rc = plan_query(c, qids, qweights, n, lambda, max_iters, o.precision == WMD_DIST_BF16, &qs[0]))) return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard guard(c->dc.device);
    if (!guard.ok()) return fail(WMD_EDEVICE, "query: cannot select device");
    double dummy = 0.0;
    int slot = 0;
    if ((rc = run_queries(c, qs, o, &dummy, out_resid ? &dummy : nullptr, c->stream, true, &slot, true))) return rc;
    Workspace& w = c->ws[slot];
    const size_t N = (size_t)c->dc.N;
    const size_t nd = N * (out_resid ? 2 : 1);
    const size_t bytes = sizeof(double) * nd + sizeof(int32_t) * N;
    hipError_t e;
    if ((e = hipMemcpyAsync(w.h_out, w.out, bytes, hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
        return hip_fail(e, "query: download results");
    if ((e = hipEventRecord(w.done, c->stream)) != hipSuccess) return hip_fail(e, "query: record");
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(e, "query: execution");
    std::memcpy(out_dist, w.h_out, sizeof(double) * N);
    if (out_resid) std::memcpy(out_resid, w.h_out + N, sizeof(double) * N);
    if (out_iters) std::memcpy(out_iters, w.h_out + nd, sizeof(int32_t) * N);
    return WMD_OK;
}

int wmd_query_async(wmd_corpus* c, const int32_t* qids, const float* qweights, int32_t n, float lambda,
                    int32_t iters, const wmd_query_options* opt, double* dev_dist, double* dev_resid,
                    void* stream) {
    if (!c || !dev_dist) return fail(WMD_EINVAL, "query: null corpus or output");
    wmd_query_options o;
    int rc = wmd::check_query_options(opt, &o);
    if (rc) return rc;
    std::vector<PlannedQuery> qs(1);
    if ((rc = plan_query(c, qids, qweights, n, lambda, iters, o.precision == WMD_DIST_BF16, &qs[0]))) return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard guard(c->dc.device);
    if (!guard.ok()) return fail(WMD_EDEVICE, "query: cannot select device");
    int slot = 0;
    return run_queries(c, qs, o, dev_dist, dev_resid, (hipStream_t)stream, false, &slot);
}

int wmd_query_batch(wmd_corpus* c, int32_t B, const int64_t* q_ptr, const int32_t* qids, const float* qweights,
                    const float* lambdas, const int32_t* iters, const wmd_query_options* opt, double* out_dist,
                    double* out_resid) {
    if (!c || !out_dist) return fail(WMD_EINVAL, "batch: null corpus or output");
    wmd_query_options o;
    int rc = wmd::check_query_options(opt, &o);
    if (rc) return rc;
    std::vector<PlannedQuery> qs;
    if ((rc = batch_plan(c, B, q_ptr, qids, qweights, lambdas, iters, o, &qs))) return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard guard(c->dc.device);
    if (!guard.ok()) return fail(WMD_EDEVICE, "batch: cannot select device");
    double dummy = 0.0;
    int slot = 0;
    if ((rc = run_queries(c, qs, o, &dummy, out_resid ? &dummy : nullptr, c->stream, true, &slot))) return rc;
    return finish_sync(c, slot, B, out_dist, out_resid);
}

int wmd_query_batch_async(wmd_corpus* c, int32_t B, const int64_t* q_ptr, const int32_t* qids,
                          const float* qweights, const float* lambdas, const int32_t* iters,
                          const wmd_query_options* opt, double* dev_dist, double* dev_resid, void* stream) {
    if (!c || !dev_dist) return fail(WMD_EINVAL, "batch: null corpus or output");
    wmd_query_options o;
    int rc = wmd::check_query_options(opt, &o);
    if (rc) return rc;
    std::vector<PlannedQuery> qs;
    if ((rc = batch_plan(c, B, q_ptr, qids, qweights, lambdas, iters, o, &qs))) return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard guard(c->dc.device);
    if (!guard.ok()) return fail(WMD_EDEVICE, "batch: cannot select device");
    int slot = 0;
    return run_queries(c, qs, o, dev_dist, dev_resid, (hipStream_t)stream, false, &slot);
}

// Top-k of the distances in w.out: scratch and results in w.tk (grown when
// needed, after the slot's previous work).  Leaves the results at w.tk and
// re-records w.done after the selection.
static int enqueue_topk(wmd_corpus* c, Workspace& w, int32_t k, hipStream_t stream, int32_t** res_idx,
                        double** res_dist) {
    const int64_t N = c->dc.N;
    const size_t sb = align_up(topk_scratch_bytes(N, k), 256);
    const size_t need = sb + align_up(sizeof(int32_t) * k, 256) + sizeof(double) * k;
    hipError_t e;
    if (need > w.tkcap) {
        if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(e, "top-k: wait");
        dfree(w.tk);
        w.tkcap = 0;
        const size_t cap = need + need / 4;
        if ((e = dalloc(&w.tk, cap)) != hipSuccess) return hip_fail(e, "top-k: scratch");
        w.tkcap = cap;
    }
    *res_idx = reinterpret_cast<int32_t*>(w.tk + sb);
    *res_dist = reinterpret_cast<double*>(w.tk + sb + align_up(sizeof(int32_t) * k, 256));
    if ((e = launch_topk(w.out, N, k, w.tk, sb, *res_idx, *res_dist, stream)) != hipSuccess)
        return hip_fail(e, "top-k: launch");
    if ((e = hipEventRecord(w.done, stream)) != hipSuccess) return hip_fail(e, "top-k: record");
    return WMD_OK;
}

static int check_topk(const wmd_corpus* c, int32_t k) {
    if (k < 1 || (int64_t)k > c->dc.N || k > WMD_MAX_TOPK)
        return fail(WMD_EINVAL, "top-k: k = %d outside [1, min(N, %d)]", k, WMD_MAX_TOPK);
    return WMD_OK;
}

int wmd_query_topk(wmd_corpus* c, const int32_t* qids, const float* qweights, int32_t n, float lambda,
                   int32_t iters, const wmd_query_options* opt, int32_t k, int32_t* out_idx, double* out_dist) {
    if (!c || !out_idx || !out_dist) return fail(WMD_EINVAL, "top-k: null corpus or output");
    int rc = check_topk(c, k);
    if (rc) return rc;
    wmd_query_options o;
    if ((rc = wmd::check_query_options(opt, &o))) return rc;
    std::vector<PlannedQuery> qs(1);
    if ((rc = plan_query(c, qids, qweights, n, lambda, iters, o.precision == WMD_DIST_BF16, &qs[0]))) return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard guard(c->dc.device);
    if (!guard.ok()) return fail(WMD_EDEVICE, "top-k: cannot select device");
    double dummy = 0.0;
    int slot = 0;
    if ((rc = run_queries(c, qs, o, &dummy, nullptr, c->stream, true, &slot))) return rc;
    Workspace& w = c->ws[slot];
    int32_t* ri = nullptr;
    double* rd = nullptr;
    if ((rc = enqueue_topk(c, w, k, c->stream, &ri, &rd))) return rc;
    hipError_t e;
    // the indices and distances sit in one region of the scratch (indices first,
    // distances 256-byte aligned after them): one copy brings both
    const size_t doff = align_up(sizeof(int32_t) * k, 256);
    const size_t hb = doff + sizeof(double) * k;
    if (hb > w.tkhcap) {
        if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(e, "top-k: wait");
        hfree(w.tk_host);
        w.tkhcap = 0;
        if ((e = hipHostMalloc(reinterpret_cast<void**>(&w.tk_host), hb, hipHostMallocDefault)) != hipSuccess)
            return hip_fail(e, "top-k: pinned results");
        w.tkhcap = hb;
    }
    (void)rd;
    if ((e = hipMemcpyAsync(w.tk_host, ri, hb, hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
        return hip_fail(e, "top-k: download");
    if ((e = hipEventRecord(w.done, c->stream)) != hipSuccess) return hip_fail(e, "top-k: record");
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(e, "top-k: execution");
    std::memcpy(out_idx, w.tk_host, sizeof(int32_t) * k);
    std::memcpy(out_dist, w.tk_host + doff, sizeof(double) * k);
    return WMD_OK;
}

int wmd_query_topk_async(wmd_corpus* c, const int32_t* qids, const float* qweights, int32_t n, float lambda,
                         int32_t iters, const wmd_query_options* opt, int32_t k, int32_t* dev_idx, double* dev_dist,
                         void* stream) {
    if (!c || !dev_idx || !dev_dist) return fail(WMD_EINVAL, "top-k: null corpus or output");
    int rc = check_topk(c, k);
    if (rc) return rc;
    wmd_query_options o;
    if ((rc = wmd::check_query_options(opt, &o))) return rc;
    std::vector<PlannedQuery> qs(1);
    if ((rc = plan_query(c, qids, qweights, n, lambda, iters, o.precision == WMD_DIST_BF16, &qs[0]))) return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard guard(c->dc.device);
    if (!guard.ok()) return fail(WMD_EDEVICE, "top-k: cannot select device");
    const hipStream_t s = (hipStream_t)stream;
    double dummy = 0.0;
    int slot = 0;
    if ((rc = run_queries(c, qs, o, &dummy, nullptr, s, true, &slot))) return rc;
    Workspace& w = c->ws[slot];
    int32_t* ri = nullptr;
    double* rd = nullptr;
    if ((rc = enqueue_topk(c, w, k, s, &ri, &rd))) return rc;
    hipError_t e;
    if ((e = hipMemcpyAsync(dev_dist, rd, sizeof(double) * k, hipMemcpyDeviceToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(dev_idx, ri, sizeof(int32_t) * k, hipMemcpyDeviceToDevice, s)) != hipSuccess)
        return hip_fail(e, "top-k: copy results");
    if ((e = hipEventRecord(w.done, s)) != hipSuccess) return hip_fail(e, "top-k: record");
    return WMD_OK;
}

int wmd_set_timing(wmd_corpus* c, int32_t enable) {
    if (!c) return fail(WMD_EINVAL, "timing: null corpus");
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard guard(c->dc.device);
    for (int i = 0; i < wmd_corpus::kTimingSlots; ++i)
        if (c->slot_pending[i]) {
            hipError_t e = hipEventSynchronize(c->ev[i][3]);
            if (e != hipSuccess) return hip_fail(e, "timing: wait");
            c->slot_pending[i] = false;
        }
    if (enable < 0) return fail(WMD_EINVAL, "timing: enable must be >= 0");
    c->timing = enable;
    c->timing_seq = 0;
    c->timed_calls = 0;
    c->dist_ms_total = c->sink_ms_total = 0.0;
    c->last_dist_ms = c->last_sink_ms = 0.f;
    c->last_slot = -1;
    return WMD_OK;
}

int wmd_timing_get(wmd_corpus* c, wmd_timing* out) {
    if (!c || !out) return fail(WMD_EINVAL, "timing: null argument");
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard guard(c->dc.device);
    for (int i = 0; i < wmd_corpus::kTimingSlots; ++i) {
        const int slot = (c->next_slot + i) % wmd_corpus::kTimingSlots;   // oldest first
        if (c->slot_pending[slot]) {
            int rc = fold_timing_slot(c, slot);
            if (rc) return rc;
        }
    }
    out->calls = c->timed_calls;
    out->dist_ms = c->dist_ms_total;
    out->sinkhorn_ms = c->sink_ms_total;
    out->last_dist_ms = c->last_dist_ms;
    out->last_sinkhorn_ms = c->last_sink_ms;
    out->launches = c->last_launches;
    return WMD_OK;
}

}  // extern "C"
