// Continuous-batching server: a worker thread admits queued queries into
// batches as streams and their workspace shares free up, so batches overlap
// on the device; results and latency statistics are kept per ticket.
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

#include "wmd_corpus.h"

using namespace wmd;
using Clock = std::chrono::steady_clock;

namespace {

struct Ticket {
    PlannedQuery q;
    Clock::time_point t_submit, t_done;
    std::vector<double> dist, resid;
    int status = WMD_OK;
    bool done = false;
};

struct Slot {
    hipStream_t stream = nullptr;
    char* base = nullptr;       // this stream's share of the budget
    size_t cap = 0;
    Workspace w;
    Staging st;
    bool busy = false;
    std::atomic<bool> finished{false};
    std::vector<int64_t> ids;   // tickets of the running batch
    int status = WMD_OK;
    wmd_server* server = nullptr;
};

}  // namespace

struct wmd_server {
    wmd_corpus* corpus = nullptr;
    wmd_server_options opt{};
    std::mutex mu;
    std::condition_variable cv_work;   // worker: submissions, completions, shutdown
    std::condition_variable cv_done;   // waiters: finished tickets
    std::deque<int64_t> pending;
    std::unordered_map<int64_t, Ticket> tickets;
    int64_t next_id = 0;
    bool stop = false;
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

void on_batch_done(void* p) {
    // HIP host callback: no HIP calls here, just flag and wake the worker
    Slot* sl = static_cast<Slot*>(p);
    wmd_server* S = sl->server;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        sl->finished.store(true);
    }
    S->cv_work.notify_all();
}

// Enqueue one batch on its slot's stream (worker thread, without the server lock).
int launch_batch(wmd_server* S, Slot* sl, const std::vector<PlannedQuery>& qs) {
    const bool resid = S->opt.want_resid != 0;
    const Layout L = make_layout(S->corpus, qs, S->opt.query, resid, true);
    if (L.device_bytes() > sl->cap) return fail(WMD_ENOMEM, "server: batch exceeds the stream's budget share");
    carve_workspace(sl->w, sl->base, L);
    double dummy = 0.0;
    int rc = enqueue_queries(S->corpus, qs, S->opt.query, &dummy, resid ? &dummy : nullptr, sl->stream, true,
                             sl->w, sl->st, false);
    if (rc) return rc;
    hipError_t e;
    const size_t bytes = L.obytes;
    if ((e = hipMemcpyAsync(sl->w.h_out, sl->w.out, bytes, hipMemcpyDeviceToHost, sl->stream)) != hipSuccess)
        return hip_fail(e, "server: download results");
    if ((e = hipEventRecord(sl->w.done, sl->stream)) != hipSuccess) return hip_fail(e, "server: record");
    if ((e = hipLaunchHostFunc(sl->stream, on_batch_done, sl)) != hipSuccess)
        return hip_fail(e, "server: completion callback");
    return WMD_OK;
}

// Hand a finished batch's results to its tickets (worker thread, lock held on
// entry and exit; the copies run unlocked).
void complete_batch(wmd_server* S, Slot* sl, std::unique_lock<std::mutex>& lk) {
    const int64_t N = S->corpus->dc.N;
    const size_t B = sl->ids.size();
    const bool resid = S->opt.want_resid != 0;
    std::vector<Ticket*> ts(B);
    for (size_t b = 0; b < B; ++b) ts[b] = &S->tickets.at(sl->ids[b]);
    int status = sl->status;
    lk.unlock();
    // the callback ran after the download; this also surfaces a device error of the batch
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
        t->done = true;
        t->t_done = now;
        if (status == WMD_OK) {
            S->completed += 1;
            S->doc_iters += (double)N * t->q.iters;
            S->latencies_ms.push_back(std::chrono::duration<double, std::milli>(now - t->t_submit).count());
        }
    }
    S->t_last = now;
    sl->ids.clear();
    sl->busy = false;
    sl->finished.store(false);
    S->cv_done.notify_all();
}

void worker_main(wmd_server* S) {
    (void)hipSetDevice(S->corpus->dc.device);
    const bool resid = S->opt.want_resid != 0;
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        for (Slot* sl : S->slots)
            if (sl->busy && sl->finished.load()) complete_batch(S, sl, lk);
        bool any_busy = false;
        for (Slot* sl : S->slots) any_busy = any_busy || sl->busy;
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
            // the longest FIFO prefix that fits this stream's share
            std::vector<PlannedQuery> qs;
            std::vector<int64_t> ids;
            int64_t words = 0;
            while (!S->pending.empty() && (int)ids.size() < S->opt.max_batch) {
                const PlannedQuery& nq = S->tickets.at(S->pending.front()).q;
                if (!ids.empty() && S->opt.max_batch_words > 0 && words + nq.m > S->opt.max_batch_words) break;
                qs.push_back(nq);
                if (make_layout(S->corpus, qs, S->opt.query, resid, true).device_bytes() > sl->cap) {
                    qs.pop_back();
                    break;
                }
                words += nq.m;
                ids.push_back(S->pending.front());
                S->pending.pop_front();
            }
            if (ids.empty()) {   // cannot happen: submit rejects queries larger than a share
                const int64_t id = S->pending.front();
                S->pending.pop_front();
                Ticket& t = S->tickets.at(id);
                t.status = WMD_ENOMEM;
                t.done = true;
                S->cv_done.notify_all();
                continue;
            }
            sl->busy = true;
            sl->finished.store(false);
            sl->ids = ids;
            sl->status = WMD_OK;
            S->batches += 1;
            S->batched_queries += (int64_t)ids.size();
            lk.unlock();
            const int rc = launch_batch(S, sl, qs);
            if (rc != WMD_OK) (void)hipStreamSynchronize(sl->stream);   // drain what was enqueued
            lk.lock();
            if (rc != WMD_OK) {
                // no completion callback was enqueued: fail the batch's tickets now
                sl->status = rc;
                complete_batch(S, sl, lk);
            }
            launched = true;
        }
        if (launched) continue;
        if (any_busy || deadline != Clock::time_point::max()) {
            const Clock::time_point until = std::min(deadline, Clock::now() + std::chrono::milliseconds(5));
            S->cv_work.wait_until(lk, until);
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
        if (sl->base) (void)hipFree(sl->base);
        if (sl->stream) (void)hipStreamDestroy(sl->stream);
        delete sl;
    }
    S->slots.clear();
    delete S;
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
    if (opt.hbm_budget_bytes <= 0) return fail(WMD_EINVAL, "server: hbm_budget_bytes must be > 0");
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
    const size_t share = ((size_t)opt.hbm_budget_bytes / (size_t)opt.max_inflight) / 256 * 256;
    hipError_t e;
    for (int i = 0; i < opt.max_inflight; ++i) {
        Slot* sl = new Slot();
        sl->server = S;
        S->slots.push_back(sl);
        sl->cap = share;
        if ((e = hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipMalloc(reinterpret_cast<void**>(&sl->base), std::max<size_t>(share, 256))) != hipSuccess ||
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
    if (need > S->slots[0]->cap)
        return fail(WMD_ENOMEM, "server: query needs %zu device bytes, one stream's share is %zu", need,
                    S->slots[0]->cap);
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return fail(WMD_ESHUTDOWN, "server: shutting down");
    const int64_t id = S->next_id++;
    Ticket& t = S->tickets[id];
    t.q = std::move(q);
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
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) return fail(WMD_ENOTFOUND, "server: unknown ticket %lld", (long long)ticket);
    auto ready = [&] { return it->second.done; };
    if (timeout_us < 0) {
        S->cv_done.wait(lk, ready);
    } else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
        return fail(WMD_ETIMEDOUT, "server: ticket %lld not finished", (long long)ticket);
    }
    Ticket t = std::move(it->second);
    S->tickets.erase(it);
    lk.unlock();
    if (t.status != WMD_OK) return fail(t.status, "server: ticket %lld failed", (long long)ticket);
    std::memcpy(out_dist, t.dist.data(), sizeof(double) * t.dist.size());
    if (out_resid && !t.resid.empty()) std::memcpy(out_resid, t.resid.data(), sizeof(double) * t.resid.size());
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
    for (Slot* sl : S->slots) out->workspace_bytes += (int64_t)sl->cap;
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
