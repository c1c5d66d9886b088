// Continuous-batching server: a worker thread admits queued queries into
// batches as streams and device memory free up, so batches overlap on the
// device; results and latency statistics are kept per ticket.
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

void server_free(wmd_server* S) {
    for (Slot* sl : S->slots) {
        if (sl->stream) (void)hipStreamSynchronize(sl->stream);
        free_workspace(sl->w);
        free_staging(sl->st);
        if (sl->stream) (void)hipStreamDestroy(sl->stream);
        delete sl;
    }
    S->slots.clear();
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
    wmd_query_options qo;
    int rc = check_query_options(&opt.query, &qo);
    if (rc) return rc;
    if (qo.tile != -1) return fail(WMD_EINVAL, "server: the query tile must be automatic (-1)");
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
    const size_t need = make_layout(S->corpus, one, S->opt.query, S->opt.want_resid != 0, true).device_bytes();
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
