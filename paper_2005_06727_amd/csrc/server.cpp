// Continuous-batching server: a worker thread admits queued queries into
// batches as streams and device memory free up, so batches overlap on the
// device; results and latency statistics are kept per ticket.
//
// Two schedules.  Batch mode: each admitted batch runs its whole path (K1,
// every iteration, final step, download) on a stream of its own.  Step mode
// (step_iters > 0, iteration-level batching): every in-flight query holds its
// own device region (K block, iterate x, results) across launches, and the
// worker enqueues steps on one stream; a step runs K1 for the queries
// admitted into it, then one Sinkhorn launch per shape class over all
// in-flight queries, each advancing step_iters iterations from its own iteration count
// (the final step included once its count is reached), then downloads the
// results of the queries that finished.  Queries join and leave at step
// boundaries, so a short query admitted next to a long one finishes after
// its own few steps.
//
// Memory: one device allocation of the whole HBM budget, carved per batch by
// a first-fit pool (byte accounting: a batch is admitted when its workspace
// fits the largest free range, and its bytes return to the pool when it
// completes).  Completion: the worker polls each running batch's event
// (cheaper and quicker than a host callback), so it keeps one host core busy
// while batches are in flight and sleeps on a condition variable otherwise.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pool.h"
#include "wmd_corpus.h"

using namespace wmd;
using Clock = std::chrono::steady_clock;

namespace {

struct Ticket {
    PlannedQuery q;
    size_t bytes = 0;                // device workspace of this query alone
    Clock::time_point t_submit, t_done;
    std::vector<double> dist, resid;
    int status = WMD_OK;
    std::atomic<bool> done{false};   // set under the server lock, read without it by its waiter
    bool waited = false;             // a thread is in wmd_server_wait on it
};

struct Slot {
    hipStream_t stream = nullptr;
    Workspace w;                     // carved from the pool per batch; pinned output and staging own
    Staging st;
    bool busy = false;
    size_t off = 0, bytes = 0;       // the running batch's pool range
    std::vector<int64_t> ids;        // tickets of the running batch
    int status = WMD_OK;
};

// Step mode: one in-flight query, its device region in the pool (K block,
// K .* M when lambda is small, row shifts with the column shift, iterate x,
// results) and its progress.
struct Active {
    int64_t id = 0;
    const PlannedQuery* q = nullptr;   // the ticket's (tickets do not move)
    size_t off = 0, bytes = 0;         // pool range
    int hslot = -1;                    // pinned result buffer
    int it_base = 0;                   // x updates done before the next step
    int shape = -1;                    // Sinkhorn launch shape
    bool fresh = true;                 // its distance kernel has not run yet
    float* Kt = nullptr;
    float* KMt = nullptr;
    float* nrow = nullptr;
    float* x = nullptr;
    double* out = nullptr;             // N distances, then N residuals
};

struct Step {
    hipEvent_t ev = nullptr;
    std::vector<Active> finishing;     // queries whose results this step downloads
    int queries = 0;                   // queries the step advanced
};

struct StepState {
    static constexpr int kRing = 2;    // steps in flight at most
    hipStream_t stream = nullptr;
    std::vector<Active> active;        // in-flight queries (worker thread only)
    Step ring[kRing];
    int next = 0;                      // ring entry of the next step
    std::deque<int> order;             // ring entries in flight, oldest first
    char* dparams[kRing] = {};         // device parameter block of each ring entry
    size_t dcap[kRing] = {};
    char* hparams[kRing] = {};         // its pinned host image
    size_t hcap[kRing] = {};
    double* h_out = nullptr;           // max_batch pinned result buffers
    std::vector<int> free_hslots;
};

}  // namespace

struct wmd_server {
    wmd_corpus* corpus = nullptr;
    wmd_server_options opt{};
    std::mutex mu;
    std::condition_variable cv_work;   // worker: submissions, shutdown
    std::condition_variable cv_done;   // waiters: finished tickets
    std::deque<int64_t> pending;
    // node-based: a Ticket's address stays valid while other tickets are
    // inserted or erased (only its own waiter erases it)
    std::unordered_map<int64_t, Ticket> tickets;
    int64_t next_id = 0;
    bool stop = false;
    char* base = nullptr;              // the budget, one device allocation
    RegionPool pool;
    std::vector<Slot*> slots;
    std::thread worker;
    StepState* steps = nullptr;        // step mode only
    // statistics
    int64_t submitted = 0, completed = 0, batches = 0, batched_queries = 0;
    double doc_iters = 0.0;
    std::vector<double> latencies_ms;
    Clock::time_point t_first, t_last;
    bool have_first = false;
};

namespace {

// Enqueue one batch on its slot's stream, in its pool range (worker thread,
// without the server lock).
int launch_batch(wmd_server* S, Slot* sl, const std::vector<PlannedQuery>& qs, const Layout& L) {
    carve_workspace(sl->w, S->base + sl->off, L);
    double dummy = 0.0;
    const bool resid = S->opt.want_resid != 0;
    int rc = enqueue_queries(S->corpus, qs, S->opt.query, &dummy, resid ? &dummy : nullptr, sl->stream, true,
                             sl->w, sl->st, false);
    if (rc) return rc;
    hipError_t e;
    if ((e = hipMemcpyAsync(sl->w.h_out, sl->w.out, L.obytes, hipMemcpyDeviceToHost, sl->stream)) != hipSuccess)
        return hip_fail(e, "server: download results");
    if ((e = hipEventRecord(sl->w.done, sl->stream)) != hipSuccess) return hip_fail(e, "server: record");
    return WMD_OK;
}

// Hand a finished batch's results to its tickets and return its memory
// (worker thread, lock held on entry and exit; the copies run unlocked).
void complete_batch(wmd_server* S, Slot* sl, std::unique_lock<std::mutex>& lk) {
    const int64_t N = S->corpus->dc.N;
    const size_t B = sl->ids.size();
    const bool resid = S->opt.want_resid != 0;
    std::vector<Ticket*> ts(B);
    for (size_t b = 0; b < B; ++b) ts[b] = &S->tickets.at(sl->ids[b]);
    int status = sl->status;
    lk.unlock();
    if (status == WMD_OK && hipEventSynchronize(sl->w.done) != hipSuccess) status = WMD_EDEVICE;
    if (status == WMD_OK) {
        for (size_t b = 0; b < B; ++b) {
            ts[b]->dist.assign(sl->w.h_out + b * N, sl->w.h_out + (b + 1) * N);
            if (resid) ts[b]->resid.assign(sl->w.h_out + (B + b) * N, sl->w.h_out + (B + b + 1) * N);
        }
    }
    lk.lock();
    const Clock::time_point now = Clock::now();
    for (size_t b = 0; b < B; ++b) {
        Ticket* t = ts[b];
        t->status = status;
        t->t_done = now;
        t->done.store(true, std::memory_order_release);
        if (status == WMD_OK) {
            S->completed += 1;
            S->doc_iters += (double)N * t->q.iters;
            S->latencies_ms.push_back(std::chrono::duration<double, std::milli>(now - t->t_submit).count());
        }
    }
    S->t_last = now;
    S->pool.release(sl->off, sl->bytes);
    sl->ids.clear();
    sl->busy = false;
    sl->bytes = 0;
    S->cv_done.notify_all();
}

// Whether a running batch has finished (or failed) on the device.
bool batch_finished(Slot* sl) {
    const hipError_t e = hipEventQuery(sl->w.done);
    if (e == hipErrorNotReady) return false;
    if (e != hipSuccess && sl->status == WMD_OK) sl->status = WMD_EDEVICE;
    return true;
}

void worker_main(wmd_server* S) {
    (void)hipSetDevice(S->corpus->dc.device);
    const bool resid = S->opt.want_resid != 0;
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        bool any_busy = false;
        for (Slot* sl : S->slots) {
            if (sl->busy && batch_finished(sl)) complete_batch(S, sl, lk);
            any_busy = any_busy || sl->busy;
        }
        if (S->stop && S->pending.empty() && !any_busy) break;

        bool launched = false;
        Clock::time_point deadline = Clock::time_point::max();
        for (Slot* sl : S->slots) {
            if (sl->busy || S->pending.empty()) continue;
            if (S->opt.batch_wait_us > 0 && !S->stop && (int)S->pending.size() < S->opt.max_batch) {
                const Clock::time_point due =
                    S->tickets.at(S->pending.front()).t_submit + std::chrono::microseconds(S->opt.batch_wait_us);
                if (Clock::now() < due) {
                    deadline = due;
                    break;
                }
            }
            // the longest FIFO prefix whose workspace fits the largest free
            // range of the budget; the head waits (no overtaking) when even it
            // does not fit until running batches return their memory
            const size_t room = S->pool.largest_free();
            std::vector<PlannedQuery> qs;
            int64_t words = 0;
            Layout L;
            size_t n_take = 0;
            while (n_take < S->pending.size() && (int)n_take < S->opt.max_batch) {
                const Ticket& t = S->tickets.at(S->pending[n_take]);
                if (n_take > 0 && S->opt.max_batch_words > 0 && words + t.q.m > S->opt.max_batch_words) break;
                if (t.bytes > room) break;
                qs.push_back(t.q);
                const Layout L2 = make_layout(S->corpus, qs, S->opt.query, resid, true);
                if (RegionPool::rounded(L2.device_bytes()) > room) {
                    qs.pop_back();
                    break;
                }
                L = L2;
                words += t.q.m;
                ++n_take;
            }
            if (n_take == 0) break;
            size_t off = 0;
            const size_t bytes = L.device_bytes();
            if (!S->pool.alloc(bytes, &off)) break;   // cannot happen: bytes <= room
            sl->busy = true;
            sl->off = off;
            sl->bytes = bytes;
            sl->ids.assign(S->pending.begin(), S->pending.begin() + (std::ptrdiff_t)n_take);
            S->pending.erase(S->pending.begin(), S->pending.begin() + (std::ptrdiff_t)n_take);
            sl->status = WMD_OK;
            S->batches += 1;
            S->batched_queries += (int64_t)n_take;
            lk.unlock();
            const int rc = launch_batch(S, sl, qs, L);
            if (rc != WMD_OK) (void)hipStreamSynchronize(sl->stream);   // drain what was enqueued
            lk.lock();
            if (rc != WMD_OK) {
                sl->status = rc;
                complete_batch(S, sl, lk);
            }
            launched = true;
            any_busy = true;
        }
        if (launched) continue;
        if (any_busy) {
            // poll the running batches; a submission needs no wake-up here
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        } else if (deadline != Clock::time_point::max()) {
            S->cv_work.wait_until(lk, deadline);
        } else {
            S->cv_work.wait(lk, [&] { return S->stop || !S->pending.empty(); });
        }
    }
}

// ---- step mode ----

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }
size_t al64(size_t b) { return (b + 63) & ~(size_t)63; }

// Device bytes of one query's region in step mode.
size_t region_bytes(const wmd_corpus* c, const PlannedQuery& q, const wmd_query_options& o, bool resid) {
    const size_t U = (size_t)c->dc.U, N = (size_t)c->dc.N, ldk = (size_t)q.ldk;
    size_t b = al256(sizeof(float) * U * ldk);                                       // K block
    if (q.lambda < kKmFromKMinLambda) b += al256(sizeof(float) * U * ldk);           // K .* M
    if (o.log_domain) b += al256(sizeof(float) * U);                                 // row shifts
    b += al256(sizeof(float) * N * ldk);                                             // x
    b += al256(sizeof(double) * N * (resid ? 2 : 1));                                // results
    return b;
}

void carve_region(const wmd_server* S, Active& a) {
    const wmd_corpus* c = S->corpus;
    const size_t U = (size_t)c->dc.U, N = (size_t)c->dc.N, ldk = (size_t)a.q->ldk;
    char* p = S->base + a.off;
    auto take = [&](size_t bytes) {
        char* r = p;
        p += al256(bytes);
        return r;
    };
    a.Kt = reinterpret_cast<float*>(take(sizeof(float) * U * ldk));
    a.KMt = a.q->lambda < kKmFromKMinLambda ? reinterpret_cast<float*>(take(sizeof(float) * U * ldk)) : nullptr;
    a.nrow = S->opt.query.log_domain ? reinterpret_cast<float*>(take(sizeof(float) * U)) : nullptr;
    a.x = reinterpret_cast<float*>(take(sizeof(float) * N * ldk));
    a.out = reinterpret_cast<double*>(take(sizeof(double) * N * (S->opt.want_resid ? 2 : 1)));
}

// Grow a step's parameter buffers (its previous step has retired, so neither
// is in use).
int ensure_step_buffers(StepState& st, int k, size_t bytes) {
    hipError_t e;
    if (bytes > st.dcap[k]) {
        if (st.dparams[k]) (void)hipFree(st.dparams[k]);
        st.dparams[k] = nullptr;
        st.dcap[k] = 0;
        const size_t cap = bytes + bytes / 2;
        if ((e = device_alloc(reinterpret_cast<void**>(&st.dparams[k]), cap)) != hipSuccess)
            return hip_fail(e, "server: step parameters");
        st.dcap[k] = cap;
    }
    if (bytes > st.hcap[k]) {
        if (st.hparams[k]) (void)hipHostFree(st.hparams[k]);
        st.hparams[k] = nullptr;
        st.hcap[k] = 0;
        const size_t cap = bytes + bytes / 2;
        if ((e = hipHostMalloc(reinterpret_cast<void**>(&st.hparams[k]), cap, hipHostMallocDefault)) != hipSuccess)
            return hip_fail(e, "server: pinned step parameters");
        st.hcap[k] = cap;
    }
    return WMD_OK;
}

// Move queued queries into the in-flight set, FIFO without overtaking, while
// a result buffer is free, the query's region fits the largest free range of
// the budget and the in-flight words stay within max_batch_words (lock held).
void admit_step(wmd_server* S) {
    StepState& st = *S->steps;
    const bool resid = S->opt.want_resid != 0;
    int64_t words = 0;
    for (const Active& a : st.active) words += a.q->m;
    while (!S->pending.empty() && !st.free_hslots.empty()) {
        const Ticket& t = S->tickets.at(S->pending.front());
        if (!st.active.empty() && S->opt.max_batch_words > 0 && words + t.q.m > S->opt.max_batch_words) break;
        Active a;
        a.id = S->pending.front();
        a.q = &t.q;
        a.bytes = region_bytes(S->corpus, t.q, S->opt.query, resid);
        if (!S->pool.alloc(a.bytes, &a.off)) break;
        a.hslot = st.free_hslots.back();
        st.free_hslots.pop_back();
        a.shape = sinkhorn_shape_for(t.q.m, kTileMaxDoc, false);
        carve_region(S, a);
        words += t.q.m;
        S->pending.pop_front();
        // fresh queries go first: the step's distance kernel covers the first records
        size_t pos = 0;
        while (pos < st.active.size() && st.active[pos].fresh) ++pos;
        st.active.insert(st.active.begin() + (std::ptrdiff_t)pos, a);
    }
}

// Enqueue one step over the in-flight queries on ring entry k (worker thread,
// without the lock).  `finishing` receives the queries this step completes.
int enqueue_step(wmd_server* S, int k, std::vector<Active>& act, std::vector<Active>& finishing) {
    StepState& st = *S->steps;
    wmd_corpus* c = S->corpus;
    const DevCorpus& dc = c->dc;
    const wmd_query_options& o = S->opt.query;
    const int A = (int)act.size();
    const int64_t N = dc.N;
    const int iters_step = S->opt.step_iters;
    int nnew = 0;
    size_t m_new = 0, m_all = 0;
    for (const Active& a : act) {
        if (a.fresh) {
            ++nnew;
            m_new += (size_t)a.q->m;
        }
        m_all += (size_t)a.q->m;
    }
    // parameter block: QueryDev[A] | qlist[A] | kofs[nnew + 1] | qid of the new
    // queries | r | 1/r of every query
    const size_t off_ql = al64(sizeof(QueryDev) * A);
    const size_t off_qg = al64(off_ql + sizeof(int32_t) * A);
    const size_t off_id = al64(off_qg + sizeof(int32_t) * (nnew + 1));
    const size_t off_r = al64(off_id + sizeof(int32_t) * m_new);
    const size_t off_ri = al64(off_r + sizeof(float) * m_all);
    const size_t pbytes = al64(off_ri + sizeof(float) * m_all);
    int rc = ensure_step_buffers(st, k, pbytes);
    if (rc) return rc;
    char* hp = st.hparams[k];
    char* dp = st.dparams[k];
    std::memset(hp, 0, pbytes);
    QueryDev* hq = reinterpret_cast<QueryDev*>(hp);
    int32_t* hql = reinterpret_cast<int32_t*>(hp + off_ql);
    int32_t* hqg = reinterpret_cast<int32_t*>(hp + off_qg);
    const float tau = o.recompute_below >= 0.f ? o.recompute_below : (o.precision == WMD_DIST_BF16 ? 1e-2f : 0.5f);
    size_t mi = 0, mr = 0;
    hqg[0] = 0;
    for (int b = 0; b < A; ++b) {
        const Active& a = act[b];
        const PlannedQuery& q = *a.q;
        QueryDev& d = hq[b];
        if (a.fresh) {
            d.qid = reinterpret_cast<const int32_t*>(dp + off_id) + mi;
            std::memcpy(hp + off_id + sizeof(int32_t) * mi, q.ids.data(), sizeof(int32_t) * q.m);
            mi += (size_t)q.m;
            hqg[b + 1] = hqg[b] + q.ldk;
        }
        d.r = reinterpret_cast<const float*>(dp + off_r) + mr;
        d.rinv = reinterpret_cast<const float*>(dp + off_ri) + mr;
        std::memcpy(hp + off_r + sizeof(float) * mr, q.r.data(), sizeof(float) * q.m);
        std::memcpy(hp + off_ri + sizeof(float) * mr, q.rinv.data(), sizeof(float) * q.m);
        mr += (size_t)q.m;
        d.Kt = a.Kt;
        d.KMt = a.KMt;
        d.nrow = a.nrow;
        d.x = a.x;
        d.out = a.out;
        d.resid = S->opt.want_resid ? a.out + N : nullptr;
        d.lambda = q.lambda;
        d.tau2 = tau * tau;
        d.m = q.m;
        d.ldk = q.ldk;
        d.iters = q.iters;
        d.shift = o.log_domain ? 1 : 0;
        d.km_from_k = q.lambda >= kKmFromKMinLambda ? 1 : 0;
        d.inv_lambda = d.km_from_k ? 1.0f / q.lambda : 0.f;
        d.tol = 0.f;
        d.it_out = nullptr;
        d.it_base = a.it_base;
    }
    // Sinkhorn launches grouped by shape, the streaming-only queries first
    const int nshape = sinkhorn_num_shapes();
    std::vector<int> start(nshape + 2, 0);
    for (const Active& a : act) start[a.shape + 2]++;
    for (int sh = 0; sh <= nshape; ++sh) start[sh + 1] += start[sh];
    {
        std::vector<int> fill(start.begin(), start.end() - 1);
        for (int b = 0; b < A; ++b) hql[fill[act[b].shape + 1]++] = b;
    }

    // One stream: a step's distance kernel of the admitted queries, then its
    // Sinkhorn launches.  (Running the distance kernels on a second stream, to
    // overlap the previous step, measured no gain: each cross-stream event wait
    // costs microseconds.)
    const hipStream_t s = st.stream;
    hipError_t e;
    if ((e = hipMemcpyAsync(dp, hp, pbytes, hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_fail(e, "server: step parameters");
    const QueryDev* dq = reinterpret_cast<const QueryDev*>(dp);
    const int32_t* dql = reinterpret_cast<const int32_t*>(dp + off_ql);
    if (nnew > 0 &&
        (e = launch_dist(dc, dq, reinterpret_cast<const int32_t*>(dp + off_qg), nnew, hqg[nnew],
                         o.precision == WMD_DIST_BF16 ? 1 : 0, o.log_domain, s)) != hipSuccess)
        return hip_fail(e, "server: distance kernel launch");
    const int d_tile = (int)c->d_tile;
    auto go = [&](int shape, int q0, int q1, int d0, int d1) -> hipError_t {
        if (q1 <= q0 || d1 <= d0) return hipSuccess;
        SinkArgs g;
        g.sptr = dc.sptr;
        g.scol = dc.scol;
        g.scw = dc.scw;
        g.sdoc = dc.sdoc;
        g.zpad = dc.zpad;
        g.it_begin = 0;
        g.it_count = iters_step;
        g.final_step = 0;
        g.per_query = 1;
        g.qlist = dql + q0;
        g.nq = q1 - q0;
        g.single = (g.nq == 1) ? 1 : 0;
        g.qd = g.single ? dq + hql[q0] : dq;
        g.d_begin = d0;
        g.d_end = d1;
        int mm = 0;
        for (int i = q0; i < q1; ++i) mm = std::max(mm, act[hql[i]].q->m);
        return launch_sinkhorn(shape, g, mm, c->h_sorted_len[d0], s);
    };
    if ((e = go(-1, start[0], start[1], 0, (int)N)) != hipSuccess ||
        (e = go(-1, start[1], A, 0, d_tile)) != hipSuccess)
        return hip_fail(e, "server: sinkhorn launch");
    for (int sh = 0; sh < nshape; ++sh)
        if ((e = go(sh, start[sh + 1], start[sh + 2], d_tile, (int)N)) != hipSuccess)
            return hip_fail(e, "server: sinkhorn launch");
    // results of the queries that reach their iteration count in this step
    const size_t per = sizeof(double) * (size_t)N * (S->opt.want_resid ? 2 : 1);
    for (const Active& a : act) {
        if ((int64_t)a.it_base + iters_step < a.q->iters) continue;
        if ((e = hipMemcpyAsync(reinterpret_cast<char*>(st.h_out) + per * (size_t)a.hslot, a.out, per,
                                hipMemcpyDeviceToHost, s)) != hipSuccess)
            return hip_fail(e, "server: download results");
        finishing.push_back(a);
    }
    if ((e = hipEventRecord(st.ring[k].ev, s)) != hipSuccess) return hip_fail(e, "server: record");
    return WMD_OK;
}

// Hand the results of a finished step's queries to their tickets and return
// their memory (lock held on entry and exit).
void retire_step(wmd_server* S, Step& sp, int status, std::unique_lock<std::mutex>& lk) {
    StepState& st = *S->steps;
    const int64_t N = S->corpus->dc.N;
    const bool resid = S->opt.want_resid != 0;
    const size_t per = (size_t)N * (resid ? 2 : 1);
    std::vector<Ticket*> ts;
    for (const Active& a : sp.finishing) ts.push_back(&S->tickets.at(a.id));
    lk.unlock();
    if (status == WMD_OK) {
        for (size_t i = 0; i < ts.size(); ++i) {
            const double* h = st.h_out + per * (size_t)sp.finishing[i].hslot;
            ts[i]->dist.assign(h, h + N);
            if (resid) ts[i]->resid.assign(h + N, h + 2 * N);
        }
    }
    lk.lock();
    const Clock::time_point now = Clock::now();
    for (size_t i = 0; i < ts.size(); ++i) {
        Ticket* t = ts[i];
        t->status = status;
        t->t_done = now;
        t->done.store(true, std::memory_order_release);
        if (status == WMD_OK) {
            S->completed += 1;
            S->doc_iters += (double)N * t->q.iters;
            S->latencies_ms.push_back(std::chrono::duration<double, std::milli>(now - t->t_submit).count());
        }
        S->pool.release(sp.finishing[i].off, sp.finishing[i].bytes);
        st.free_hslots.push_back(sp.finishing[i].hslot);
    }
    if (!ts.empty()) S->t_last = now;
    sp.finishing.clear();
    S->cv_done.notify_all();
}

void step_worker_main(wmd_server* S) {
    (void)hipSetDevice(S->corpus->dc.device);
    StepState& st = *S->steps;
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        // retire finished steps, oldest first
        while (!st.order.empty()) {
            Step& sp = st.ring[st.order.front()];
            const hipError_t e = hipEventQuery(sp.ev);
            if (e == hipErrorNotReady) break;
            retire_step(S, sp, e == hipSuccess ? WMD_OK : WMD_EDEVICE, lk);
            st.order.pop_front();
        }
        if (S->stop && S->pending.empty() && st.active.empty() && st.order.empty()) break;
        if ((int)st.order.size() < StepState::kRing) {
            admit_step(S);
            if (!st.active.empty()) {
                const int k = st.next;
                st.next = (st.next + 1) % StepState::kRing;
                std::vector<Active> act = st.active;   // the worker alone changes st.active
                S->batches += 1;
                S->batched_queries += (int64_t)act.size();
                lk.unlock();
                std::vector<Active> finishing;
                const int rc = enqueue_step(S, k, act, finishing);
                if (rc != WMD_OK) (void)hipStreamSynchronize(st.stream);   // drain what was enqueued
                lk.lock();
                Step& sp = st.ring[k];
                if (rc != WMD_OK) {
                    // the step failed: every query it carried fails with it
                    sp.finishing = st.active;
                    st.active.clear();
                    retire_step(S, sp, rc, lk);
                    continue;
                }
                sp.finishing = std::move(finishing);
                sp.queries = (int)act.size();
                st.order.push_back(k);
                // advance the in-flight set: finishing queries leave it (their
                // memory returns when the step retires)
                std::vector<Active> keep;
                for (Active a : st.active) {
                    a.fresh = false;
                    a.it_base += S->opt.step_iters;
                    if (a.it_base < a.q->iters) keep.push_back(a);
                }
                st.active.swap(keep);
                continue;
            }
        }
        if (!st.order.empty()) {
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        } else {
            S->cv_work.wait(lk, [&] { return S->stop || !S->pending.empty(); });
        }
    }
}

void step_state_free(StepState* st) {
    if (!st) return;
    if (st->stream) (void)hipStreamSynchronize(st->stream);
    for (int k = 0; k < StepState::kRing; ++k) {
        if (st->ring[k].ev) (void)hipEventDestroy(st->ring[k].ev);
        if (st->dparams[k]) (void)hipFree(st->dparams[k]);
        if (st->hparams[k]) (void)hipHostFree(st->hparams[k]);
    }
    if (st->h_out) (void)hipHostFree(st->h_out);
    if (st->stream) (void)hipStreamDestroy(st->stream);
    delete st;
}

int step_state_create(wmd_server* S) {
    StepState* st = new StepState();
    S->steps = st;
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&st->stream, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "server: step stream");
    for (int k = 0; k < StepState::kRing; ++k)
        if ((e = hipEventCreateWithFlags(&st->ring[k].ev, hipEventDisableTiming)) != hipSuccess)
            return hip_fail(e, "server: step events");
    const size_t per = sizeof(double) * (size_t)S->corpus->dc.N * (S->opt.want_resid ? 2 : 1);
    if ((e = hipHostMalloc(reinterpret_cast<void**>(&st->h_out), per * (size_t)S->opt.max_batch,
                           hipHostMallocDefault)) != hipSuccess)
        return hip_fail(e, "server: pinned results");
    for (int i = S->opt.max_batch - 1; i >= 0; --i) st->free_hslots.push_back(i);
    return WMD_OK;
}

void server_free(wmd_server* S) {
    for (Slot* sl : S->slots) {
        if (sl->stream) (void)hipStreamSynchronize(sl->stream);
        free_workspace(sl->w);
        free_staging(sl->st);
        if (sl->stream) (void)hipStreamDestroy(sl->stream);
        delete sl;
    }
    S->slots.clear();
    step_state_free(S->steps);
    S->steps = nullptr;
    if (S->base) (void)hipFree(S->base);
    delete S;
}

// Pinned host memory a stream slot needs for its usual batches, taken at
// creation so that no batch pays for it: the result download of max_batch
// queries and the staging ring for parameter blocks of up to 64 KB.
int prealloc_slot_host(wmd_server* S, Slot* sl) {
    const size_t out_bytes =
        sizeof(double) * (size_t)S->opt.max_batch * (size_t)S->corpus->dc.N * (S->opt.want_resid ? 2 : 1);
    hipError_t e;
    if ((e = hipHostMalloc(reinterpret_cast<void**>(&sl->w.h_out), out_bytes, hipHostMallocDefault)) != hipSuccess)
        return hip_fail(e, "server: pinned results");
    sl->w.hocap = out_bytes;
    const size_t stage = 64 * 1024;
    for (int j = 0; j < Staging::kSlots; ++j)
        if ((e = hipHostMalloc(reinterpret_cast<void**>(&sl->st.h[j]), stage, hipHostMallocDefault)) != hipSuccess)
            return hip_fail(e, "server: pinned staging");
    sl->st.cap = stage;
    return WMD_OK;
}

}  // namespace

extern "C" {

void wmd_server_options_init(wmd_server_options* opt) {
    if (!opt) return;
    opt->hbm_budget_bytes = (int64_t)4 << 30;
    opt->max_batch = 16;
    opt->max_inflight = 2;
    opt->want_resid = 0;
    opt->batch_wait_us = 0;
    wmd_query_options_init(&opt->query);
    opt->max_batch_words = 512;
    opt->step_iters = 0;
}

int wmd_server_create(wmd_corpus* corpus, const wmd_server_options* opt_in, wmd_server** out) {
    if (!corpus || !out) return fail(WMD_EINVAL, "server: null corpus or output handle");
    wmd_server_options opt;
    wmd_server_options_init(&opt);
    if (opt_in) opt = *opt_in;
    if (opt.hbm_budget_bytes < (int64_t)RegionPool::kAlign)
        return fail(WMD_EINVAL, "server: hbm_budget_bytes must be at least %zu", RegionPool::kAlign);
    if (opt.max_batch < 1) return fail(WMD_EINVAL, "server: max_batch must be >= 1");
    if (opt.max_inflight < 1 || opt.max_inflight > 16) return fail(WMD_EINVAL, "server: max_inflight outside 1..16");
    if (opt.batch_wait_us < 0) return fail(WMD_EINVAL, "server: batch_wait_us < 0");
    if (opt.max_batch_words < 0) return fail(WMD_EINVAL, "server: max_batch_words < 0");
    if (opt.step_iters < 0) return fail(WMD_EINVAL, "server: step_iters < 0");
    wmd_query_options qo;
    int rc = check_query_options(&opt.query, &qo);
    if (rc) return rc;
    if (qo.tile != -1) return fail(WMD_EINVAL, "server: the query tile must be automatic (-1)");
    if (opt.step_iters > 0 && (qo.lse || qo.tol > 0.f || qo.iters_per_launch > 0))
        return fail(WMD_EINVAL, "server: step mode runs the plain iteration (no lse, tol or iters_per_launch)");
    if (qo.precision == WMD_DIST_BF16 && !corpus->dc.act_bf16)
        return fail(WMD_EINVAL, "server: BF16 distances need a corpus created with bf16 copies");
    opt.query = qo;
    DeviceGuard guard(corpus->dc.device);
    if (!guard.ok()) return fail(WMD_EDEVICE, "server: cannot select device");

    wmd_server* S = new wmd_server();
    S->corpus = corpus;
    S->opt = opt;
    S->pool.reset((size_t)opt.hbm_budget_bytes);
    hipError_t e;
    if ((e = device_alloc(reinterpret_cast<void**>(&S->base), S->pool.capacity())) != hipSuccess) {
        const int code = hip_fail(e, "server: device budget");
        S->base = nullptr;
        server_free(S);
        return code;
    }
    if (opt.step_iters > 0) {
        if ((rc = step_state_create(S)) != WMD_OK) {
            server_free(S);
            return rc;
        }
        S->worker = std::thread(step_worker_main, S);
        *out = S;
        return WMD_OK;
    }
    for (int i = 0; i < opt.max_inflight; ++i) {
        Slot* sl = new Slot();
        S->slots.push_back(sl);
        if ((e = hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&sl->w.done, hipEventDisableTiming)) != hipSuccess) {
            const int code = hip_fail(e, "server: stream resources");
            server_free(S);
            return code;
        }
        for (int j = 0; j < Staging::kSlots; ++j)
            if ((e = hipEventCreateWithFlags(&sl->st.ev[j], hipEventDisableTiming)) != hipSuccess) {
                const int code = hip_fail(e, "server: events");
                server_free(S);
                return code;
            }
        if ((rc = prealloc_slot_host(S, sl)) != WMD_OK) {
            server_free(S);
            return rc;
        }
    }
    S->worker = std::thread(worker_main, S);
    *out = S;
    return WMD_OK;
}

int64_t wmd_server_submit(wmd_server* S, const int32_t* qids, const float* qweights, int32_t n, float lambda,
                          int32_t iters) {
    if (!S) return fail(WMD_EINVAL, "server: null handle");
    PlannedQuery q;
    int rc = plan_query(S->corpus, qids, qweights, n, lambda, iters, S->opt.query.precision == WMD_DIST_BF16, &q);
    if (rc) return rc;
    const std::vector<PlannedQuery> one{q};
    const size_t need = S->opt.step_iters > 0
                            ? region_bytes(S->corpus, q, S->opt.query, S->opt.want_resid != 0)
                            : make_layout(S->corpus, one, S->opt.query, S->opt.want_resid != 0, true).device_bytes();
    if (RegionPool::rounded(need) > S->pool.capacity())
        return fail(WMD_ENOMEM, "server: query needs %zu device bytes, the whole budget is %zu", need,
                    S->pool.capacity());
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return fail(WMD_ESHUTDOWN, "server: shutting down");
    const int64_t id = S->next_id++;
    Ticket& t = S->tickets[id];
    t.q = std::move(q);
    t.bytes = RegionPool::rounded(need);
    t.t_submit = Clock::now();
    if (!S->have_first) {
        S->have_first = true;
        S->t_first = t.t_submit;
    }
    S->pending.push_back(id);
    S->submitted += 1;
    S->cv_work.notify_all();
    return id;
}

int wmd_server_wait(wmd_server* S, int64_t ticket, double* out_dist, double* out_resid, int64_t timeout_us) {
    if (!S || !out_dist) return fail(WMD_EINVAL, "server: null handle or output");
    Ticket* t = nullptr;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->tickets.find(ticket);
        if (it == S->tickets.end()) return fail(WMD_ENOTFOUND, "server: unknown ticket %lld", (long long)ticket);
        t = &it->second;   // stays valid: only this waiter erases it
        if (t->waited) return fail(WMD_EINVAL, "server: ticket %lld already has a waiter", (long long)ticket);
        t->waited = true;
    }
    // spin briefly (results of short queries arrive within microseconds of
    // the device finishing), then sleep on the condition variable
    const Clock::time_point t0 = Clock::now();
    const Clock::time_point spin_until = t0 + std::chrono::microseconds(2000);
    while (!t->done.load(std::memory_order_acquire) && Clock::now() < spin_until) {
        if (timeout_us >= 0 && Clock::now() - t0 >= std::chrono::microseconds(timeout_us)) break;
        std::this_thread::yield();
    }
    std::unique_lock<std::mutex> lk(S->mu);
    auto ready = [&] { return t->done.load(std::memory_order_acquire); };
    if (timeout_us < 0) {
        S->cv_done.wait(lk, ready);
    } else if (!S->cv_done.wait_until(lk, t0 + std::chrono::microseconds(timeout_us), ready)) {
        t->waited = false;
        return fail(WMD_ETIMEDOUT, "server: ticket %lld not finished", (long long)ticket);
    }
    const int status = t->status;
    std::vector<double> dist = std::move(t->dist), resid = std::move(t->resid);
    S->tickets.erase(ticket);
    lk.unlock();
    if (status != WMD_OK) return fail(status, "server: ticket %lld failed", (long long)ticket);
    std::memcpy(out_dist, dist.data(), sizeof(double) * dist.size());
    if (out_resid && !resid.empty()) std::memcpy(out_resid, resid.data(), sizeof(double) * resid.size());
    return WMD_OK;
}

int wmd_server_stats_get(wmd_server* S, wmd_server_stats* out) {
    if (!S || !out) return fail(WMD_EINVAL, "server: null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    std::memset(out, 0, sizeof *out);
    out->submitted = S->submitted;
    out->completed = S->completed;
    out->batches = S->batches;
    out->mean_batch = S->batches ? (double)S->batched_queries / (double)S->batches : 0.0;
    out->workspace_bytes = (int64_t)S->pool.capacity();
    if (!S->latencies_ms.empty()) {
        std::vector<double> l = S->latencies_ms;
        std::sort(l.begin(), l.end());
        auto pct = [&](double p) {
            const double pos = p * (double)(l.size() - 1);
            const size_t i = (size_t)pos;
            const double f = pos - (double)i;
            return i + 1 < l.size() ? l[i] * (1.0 - f) + l[i + 1] * f : l[i];
        };
        out->latency_p50_ms = pct(0.50);
        out->latency_p99_ms = pct(0.99);
        double sum = 0.0;
        for (double v : l) sum += v;
        out->latency_mean_ms = sum / (double)l.size();
        out->latency_max_ms = l.back();
        const double span = std::chrono::duration<double>(S->t_last - S->t_first).count();
        if (span > 0) {
            out->queries_per_s = (double)S->completed / span;
            out->doc_iters_per_s = S->doc_iters / span;
        }
    }
    return WMD_OK;
}

int wmd_server_stats_reset(wmd_server* S) {
    if (!S) return fail(WMD_EINVAL, "server: null handle");
    std::lock_guard<std::mutex> lk(S->mu);
    S->submitted = (int64_t)S->pending.size();
    for (Slot* sl : S->slots) S->submitted += (int64_t)sl->ids.size();
    if (S->steps) {
        S->submitted += (int64_t)S->steps->active.size();
        for (int k : S->steps->order) S->submitted += (int64_t)S->steps->ring[k].finishing.size();
    }
    S->completed = S->batches = S->batched_queries = 0;
    S->doc_iters = 0.0;
    S->latencies_ms.clear();
    S->have_first = false;
    if (S->submitted > 0) {   // queries still queued or running count from now
        S->have_first = true;
        S->t_first = Clock::now();
    }
    return WMD_OK;
}

void wmd_server_destroy(wmd_server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    DeviceGuard guard(S->corpus->dc.device);
    server_free(S);
}

}  // extern "C"
