"""Throughput of the sparse Sinkhorn WMD hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
    python bench.py --serve c5 [--queries Q] [--qps R]
    python bench.py --lse
    python bench.py --profile-batch

One step = a group of 128 queries (--queries-per-step), each issued as its own
call and taken through the whole path (query preparation, distance GEMM + K
epilogue, 15 fused Sinkhorn iterations + final WMD step) against the
device-resident corpus, results written to device memory.  A group, not one
query, so that the pipeline's fill and drain (the first distance kernel has
nothing to overlap, the last Sinkhorn kernel neither) and any short stall
weigh the same in a 20-step run (about 50 ms) as in a long one.  Workload: the
paper-shaped single query (V=100000 words, 300-dim embeddings, N=5000
documents of 10-60 distinct Zipf(1.1) words, one query of 20-40 words,
lambda=10, 15 iterations), seeded synthetic data standing in for the paper's
crawl embeddings and DBpedia documents.  Consecutive queries cycle over
three streams (one per workspace slot of the corpus), so one query's
distance GEMM overlaps the Sinkhorn kernels of the queries before it.  Before the K timed steps the queries run for W
steps and at least 0.3 s (the GPU's clocks ramp up under load).

Prints one JSON line: value = documents x iterations / second.  Beside it:
the kernels' roofline figures from HIP events that hold each kernel
dispatch's own start and end (hipExtLaunchKernel), on one stream (the same
single-stream run a kernel trace reproduces), the synchronous per-call
figure (host query in, host distances out), the 64-query batch on the same
corpus served three ways with the batched distance GEMM's MFMA rate, the
precision workload (BF16 distances, column shift, lambda = 50, N = 20000)
with its per-distance error against the FP64 oracle, a bounded served stream
on the 100000-document corpus (plain FP32 calls vs served FP32 vs served
BF16, p50/p99 at 50% and 90% load, served results checked), and the FP64
oracle on the host cores.

``--serve c5`` runs the served stream alone with its full 10000 queries.
``--lse`` runs the log-domain iteration (FP64 distances and potentials) on the
20000-document precision corpus at lambda = 1000.  ``--profile-batch`` runs
only the 64-query batch calls (FP32 and BF16 distances), for counter runs.
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
# independent queries in flight on their own streams, one per workspace slot
# of the corpus (three), so no call waits on another stream
STREAMS = 3
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0            # MI355X HBM3E
PEAK_FP32_TFLOPS = 157.3         # MI355X published FP32 peak (vector, counting packed FP32, and matrix)
# FP32 vector issue rate of this build: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA)
# x 2.4 GHz; the library is compiled without packed (two-wide) FP32 instructions
PEAK_FP32_UNPACKED_TFLOPS = 78.6
PEAK_BF16_TFLOPS = 2500.0        # MI355X dense BF16 matrix
PEAK_FP64_VALU_TFLOPS = 78.6     # MI355X FP64 vector
# FP32 exponentials (v_exp_f32, a quarter-rate transcendental): 256 CUs x 4 SIMDs
# x 16 lanes / 4 x 2.4 GHz
PEAK_EXP_TPS = 256 * 4 * 16 / 4 * 2.4e9 / 1e12
MIN_WARMUP_S = 0.3
# server step mode (iteration-level batching): iterations per step, queries
# and query words in flight
STEP_ITERS = 5
STEP_BATCH = 16
STEP_WORDS = 1024


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=100)
    p.add_argument("--queries-per-step", type=int, default=128,
                   help="queries of one step, each issued as its own call")
    p.add_argument("--workload", default="c2", choices=["c1", "c2"])
    p.add_argument("--min-warmup-s", type=float, default=MIN_WARMUP_S,
                   help="the warm-up runs --warmup steps and at least this many seconds")
    p.add_argument("--headline-streams", type=int, default=STREAMS,
                   help="streams the headline queries alternate over (1: every kernel runs alone, as the "
                        "single-stream kernel trace in profiles/ is taken)")
    p.add_argument("--latency-calls", type=int, default=300)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-batch", action="store_true", help="skip the 64-query batch section")
    p.add_argument("--no-c4", action="store_true", help="skip the precision-workload section")
    p.add_argument("--no-c5", action="store_true", help="skip the bounded served-stream section")
    p.add_argument("--c5-queries", type=int, default=2000, help="queries of the bounded served stream")
    p.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                   help="also run one device copy of this many MiB (reference for HBM counters)")
    p.add_argument("--serve", default=None, choices=["c5"], help="run the served-stream benchmark alone")
    p.add_argument("--lse", action="store_true",
                   help="run the log-domain iteration on the precision corpus at lambda = 1000")
    p.add_argument("--lse-lambda", type=float, default=1000.0)
    p.add_argument("--profile-batch", action="store_true", help="run only the 64-query batch calls")
    p.add_argument("--queries", type=int, default=10000, help="--serve: queries of the stream")
    p.add_argument("--qps", type=float, default=0.0,
                   help="--serve: offered rate (0: 50%% and 90%% of the served closed-loop capacity)")
    p.add_argument("--max-batch", type=int, default=16)
    p.add_argument("--streams", type=int, default=2, help="server streams (batches in flight)")
    p.add_argument("--batch-words", type=int, default=512, help="server cap on query words per batch")
    p.add_argument("--hbm-budget-gib", type=float, default=16.0)
    p.add_argument("--step-iters", type=int, default=STEP_ITERS, help="server step mode: iterations per step")
    p.add_argument("--step-batch", type=int, default=STEP_BATCH, help="server step mode: queries in flight")
    p.add_argument("--step-words", type=int, default=STEP_WORDS, help="server step mode: query words in flight")
    return p.parse_args()


def source_digest(*names) -> str:
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2005_06727_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counter_traffic(kernel: str, sources) -> float | None:
    """Per-launch HBM bytes of `kernel` from a committed counter summary, if it
    was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_counters.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256_16") != source_digest(*sources):
        return None
    return rec.get("hbm_bytes_per_launch")


def pct(lat):
    lat = np.asarray(lat)
    return {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
            "mean": float(np.mean(lat)), "max": float(np.max(lat))}


def rel_stats(err):
    err = np.asarray(err)
    return {"max": float(err.max()), "p99": float(np.percentile(err, 99)), "median": float(np.median(err)),
            "count": int(err.size)}


# ---------------------------------------------------------------- CPU baseline

def host_info() -> dict:
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    blas = None
    try:
        from threadpoolctl import threadpool_info
        blas = [{"api": d.get("internal_api"), "threads": d.get("num_threads")} for d in threadpool_info()]
    except Exception:
        pass
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "usable_cpus": usable, "blas_pools": blas}


_POOL_WL = None   # the workload, inherited by forked workers


def _oracle_slice(job):
    """Worker: the oracle on one contiguous slice of the documents."""
    from threadpoolctl import threadpool_limits
    from oracle import sinkhorn_wmd_sparse
    from paper_2005_06727_amd import synth
    wl, q, qw = _POOL_WL
    lo, hi = job
    sptr, sids, sw = synth.subcorpus(wl.doc_ptr, wl.word_ids, wl.weights, np.arange(lo, hi))
    with threadpool_limits(1):
        sinkhorn_wmd_sparse(wl.vecs, q, qw, sptr, sids, sw, wl.spec.lam, wl.spec.iters)
    return hi - lo


def cpu_baseline(wl, q, qw) -> dict:
    """The FP64 oracle as it stands on the host: the sparse form single-threaded
    on the whole query, the sparse form over all usable cores (one process per
    core, each on a contiguous slice of the documents, balanced by nonzeros),
    and the dense form (Algorithm 1 over the whole vocabulary, the analogue of
    the paper's Python code) on a sample of the documents."""
    global _POOL_WL
    from threadpoolctl import threadpool_limits
    from oracle import dense_doc_matrix, sinkhorn_wmd_dense, sinkhorn_wmd_sparse
    from paper_2005_06727_amd import synth
    sp = wl.spec
    info = host_info()
    times = []
    with threadpool_limits(1):
        for _ in range(3):
            t0 = time.perf_counter()
            sinkhorn_wmd_sparse(wl.vecs, q, qw, wl.doc_ptr, wl.word_ids, wl.weights, sp.lam, sp.iters)
            times.append(time.perf_counter() - t0)
    t1 = float(np.median(times))
    cores = max(1, min(int(info["usable_cpus"] or 1), 16))
    # slices of about equal nonzeros, a few per worker
    nslice = 4 * cores
    cum = wl.doc_ptr[1:]
    cuts = [0] + [int(np.searchsorted(cum, cum[-1] * k / nslice)) + 1 for k in range(1, nslice)] + [sp.N]
    jobs = [(a, b) for a, b in zip(cuts[:-1], cuts[1:]) if b > a]
    _POOL_WL = (wl, q, qw)
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_slice, jobs[:cores])          # warm the workers (imports)
        t0 = time.perf_counter()
        done = sum(pool.map(_oracle_slice, jobs))
        tall = time.perf_counter() - t0
    _POOL_WL = None
    assert done == sp.N
    # dense form on every 25th document (all V rows of K per document)
    docs = np.arange(0, sp.N, 25)
    sptr, sids, sw = synth.subcorpus(wl.doc_ptr, wl.word_ids, wl.weights, docs)
    Cd = dense_doc_matrix(sp.V, sptr, sids, sw)
    t0 = time.perf_counter()
    sinkhorn_wmd_dense(wl.vecs, q, qw, Cd, sp.lam, sp.iters)
    tdense = time.perf_counter() - t0
    work = sp.N * sp.iters
    return {"value": work / tall, "unit": "doc*iters/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 numpy oracle (sparse form) on the whole workload, 1 query x {sp.N} documents x "
                      f"{sp.iters} iterations, split over {cores} worker processes (one per usable core, BLAS "
                      f"limited to 1 thread each) in {len(jobs)} nonzero-balanced slices: {tall:.2f} s",
            "single_thread": {"value": work / t1, "seconds": t1,
                              "sample": f"same workload, one process, 1 BLAS thread, median of {len(times)}"},
            "dense_form": {"value": docs.size * sp.iters / tdense, "seconds": tdense,
                           "sample": f"Algorithm 1 over the whole vocabulary (V={sp.V}) on {docs.size} of the "
                                     f"{sp.N} documents (every 25th), one run, default BLAS threads"},
            "host": info}


# ---------------------------------------------------------------- helpers

def warm(step, steps: int, min_s: float = MIN_WARMUP_S):
    """Run `steps` steps, then more until `min_s` seconds have passed."""
    import torch
    t0 = time.perf_counter()
    i = 0
    while i < steps or time.perf_counter() - t0 < min_s:
        step(i)
        i += 1
        if i % 256 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    return i


def open_loop_plain(call, queries, arrivals_s):
    """FIFO single-caller service of Poisson arrivals: latency = completion - arrival."""
    lat = []
    t0 = time.perf_counter()
    for qa, a in zip(queries, arrivals_s):
        while time.perf_counter() - t0 < a:
            pass
        call(qa)
        lat.append((time.perf_counter() - t0 - a) * 1e3)
    return np.array(lat), time.perf_counter() - t0


def open_loop_served(server, queries, arrivals_s, lam, iters, keep=()):
    """Submit at the arrival times from one thread, collect from another; the
    server measures submit -> result latency itself.  Returns the span and
    the results of the query indices in `keep`."""
    import threading
    tickets = [None] * len(queries)
    ready = threading.Semaphore(0)

    def submitter():
        t0 = time.perf_counter()
        for i, ((q, qw), a) in enumerate(zip(queries, arrivals_s)):
            while time.perf_counter() - t0 < a:
                time.sleep(0)
            tickets[i] = server.submit(q, qw, lam, iters)
            ready.release()

    kept = {}
    t0 = time.perf_counter()
    th = threading.Thread(target=submitter)
    th.start()
    for i in range(len(queries)):
        ready.acquire()
        d, _ = server.wait(tickets[i])
        if i in keep:
            kept[i] = d
    th.join()
    return time.perf_counter() - t0, kept


def server_latency(st):
    return {"p50": st["latency_p50_ms"], "p99": st["latency_p99_ms"], "mean": st["latency_mean_ms"],
            "max": st["latency_max_ms"]}


# ---------------------------------------------------------------- sections

def batch_section(wmd, corpus, reps: int = 3) -> dict:
    """The 64-query batch (v_r 5-200) on the single-query corpus: back-to-back
    plain calls vs one batch call vs the server; the batched distance GEMM's
    MFMA rate; open-loop latency of plain calls and the server."""
    from paper_2005_06727_amd import synth
    wl3 = synth.make("c3")
    qs = [(np.ascontiguousarray(q, np.int32), np.ascontiguousarray(w, np.float32)) for q, w in wl3.queries]
    lam, iters = wl3.spec.lam, wl3.spec.iters
    info = corpus.info
    N, U, dim = info["N"], info["U"], info["dim"]
    h = corpus.handle
    B = len(qs)
    work = B * N * iters

    def best(f):
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            f()
            ts.append(time.perf_counter() - t)
        return min(ts)

    ref = [corpus.query(q, w, lam, iters)[0] for q, w in qs]   # warm-up + reference
    t_b2b = best(lambda: [corpus.query(q, w, lam, iters) for q, w in qs])
    corpus.query_batch(qs, lam, iters)
    t_batch = best(lambda: corpus.query_batch(qs, lam, iters))
    out = {"workload": f"{B} queries, v_r {min(len(q) for q, _ in qs)}-{max(len(q) for q, _ in qs)} "
                       f"(uniform 5-200), same corpus, lambda={lam}, {iters} iterations, FP32",
           "back_to_back": {"ms": t_b2b * 1e3, "doc_iters_per_s": work / t_b2b},
           "batch_call": {"ms": t_batch * 1e3, "doc_iters_per_s": work / t_batch}}
    # the batched distance GEMM (one launch over all 64 queries' columns), HIP events
    sum_m = sum(len(q) for q, _ in qs)
    flops = 2.0 * sum_m * dim * U
    gemm = {}
    for name, prec, peak in (("fp32", wmd.WMD_DIST_FP32, PEAK_FP32_TFLOPS), ("bf16", wmd.WMD_DIST_BF16,
                                                                              PEAK_BF16_TFLOPS)):
        corpus.query_batch(qs, lam, iters, precision=prec)
        wmd.wmd_set_timing(h, 1)
        for _ in range(5):
            corpus.query_batch(qs, lam, iters, precision=prec)
        tm = wmd.wmd_timing_get(h)
        wmd.wmd_set_timing(h, 0)
        us = 1e3 * tm["dist_ms"] / tm["calls"]
        tf = flops / (us * 1e-6) / 1e12
        gemm[name] = {"avg_us": us, "TFLOPs": tf, "peak": peak, "frac": tf / peak,
                      "sinkhorn_avg_us": 1e3 * tm["sinkhorn_ms"] / tm["calls"]}
    out["dist_gemm_batched"] = dict(gemm, algorithmic_flops=flops,
                                    what=f"2 * sum(v_r) * dim * U = 2 * {sum_m} * {dim} * {U} per launch "
                                         f"(the corpus words only); HIP events, 5 batch calls, one stream")
    with wmd.Server(corpus, max_batch=16, max_inflight=2) as srv:
        def closed():
            ts = [srv.submit(q, w, lam, iters) for q, w in qs]
            return [srv.wait(t)[0] for t in ts]
        got = closed()
        assert all(np.array_equal(g, r) for g, r in zip(got, ref)), "served != plain"
        t_srv = best(closed)
        st = srv.stats()
        out["served"] = {"ms": t_srv * 1e3, "doc_iters_per_s": work / t_srv, "mean_batch": st["mean_batch"],
                         "max_batch": 16, "streams": 2, "vs_back_to_back": t_b2b / t_srv}
    step_kw = dict(step_iters=STEP_ITERS, max_batch=STEP_BATCH, max_batch_words=STEP_WORDS)
    with wmd.Server(corpus, **step_kw) as srv:
        def closed_step():
            ts = [srv.submit(q, w, lam, iters) for q, w in qs]
            return [srv.wait(t)[0] for t in ts]
        got = closed_step()
        assert all(np.array_equal(g, r) for g, r in zip(got, ref)), "served (step mode) != plain"
        t_step = best(closed_step)
        st = srv.stats()
        out["served_step"] = {"ms": t_step * 1e3, "doc_iters_per_s": work / t_step,
                              "mean_queries_per_step": st["mean_batch"], "step_iters": STEP_ITERS,
                              "max_queries_in_flight": STEP_BATCH, "max_words_in_flight": STEP_WORDS,
                              "vs_back_to_back": t_b2b / t_step}
    # open loop: Poisson arrivals at 70% of the back-to-back capacity, the same
    # sequence for both; each path warmed on the first 64 queries first
    rate = 0.7 * B / t_b2b
    n_open = 16 * B
    arr = np.cumsum(np.random.default_rng(7).exponential(1.0 / rate, size=n_open))
    stream = [qs[i % B] for i in range(n_open)]
    lat_plain, _ = open_loop_plain(lambda qa: corpus.query(qa[0], qa[1], lam, iters), stream, arr)
    served = {}
    for name, kw in (("served", dict(max_batch=16, max_inflight=2)), ("served_step", step_kw)):
        with wmd.Server(corpus, **kw) as srv:
            for t in [srv.submit(q, w, lam, iters) for q, w in qs]:
                srv.wait(t)
            srv.reset_stats()
            open_loop_served(srv, stream, arr, lam, iters)
            served[name] = srv.stats()
    out["open_loop"] = {"qps": rate, "queries": n_open,
                        "plain_latency_ms": pct(lat_plain),
                        "served_latency_ms": server_latency(served["served"]),
                        "served_mean_batch": served["served"]["mean_batch"],
                        "served_step_latency_ms": server_latency(served["served_step"]),
                        "served_step_mean_queries_per_step": served["served_step"]["mean_batch"]}
    return out


def extensions_section(wmd, corpus, sp, q, qw, calls: int = 200) -> dict:
    """The convergence-checked iteration and the k-nearest selection on the same
    query, against the plain query, all synchronous (host in, host out)."""
    N = corpus.info["N"]

    def per_call(f):
        for _ in range(20):
            f()
        t = time.perf_counter()
        for _ in range(calls):
            r = f()
        return (time.perf_counter() - t) / calls, r

    t_plain, _ = per_call(lambda: corpus.query(q, qw, sp.lam, sp.iters))
    tol = 1e-3
    t_ad, (_, _, its) = per_call(lambda: corpus.query_adaptive(q, qw, sp.lam, sp.iters, tol))
    k = 100
    t_topk, _ = per_call(lambda: corpus.topk(q, qw, sp.lam, sp.iters, k))
    return {
        "what": "synchronous calls on the headline query: per-call wall time",
        "plain": {"us_per_query": t_plain * 1e6, "doc_iters_per_s": N * sp.iters / t_plain},
        "convergence_check": {"tol": tol, "max_iters": sp.iters, "mean_iters": float(np.mean(its)),
                              "docs_stopped_early": float(np.mean(its < sp.iters)),
                              "us_per_query": t_ad * 1e6,
                              "doc_iters_per_s": float(np.sum(its)) / t_ad},
        "topk": {"k": k, "us_per_query": t_topk * 1e6, "difference_us_vs_plain": (t_topk - t_plain) * 1e6},
    }


def precision_section(wmd, steps: int = 400, sample_docs: int = 400) -> dict:
    """The precision workload: BF16 distances with FP32 accumulation, FP32
    recompute below 1e-2, column-shifted K, lambda = 50, N = 20000; throughput
    on three streams and per-distance error against the FP64 oracle on sampled
    documents (the FP32 path's error beside it)."""
    import torch
    from oracle import sinkhorn_wmd_sparse
    from paper_2005_06727_amd import synth
    wl = synth.make("c4")
    sp = wl.spec
    qs = [(np.ascontiguousarray(q, np.int32), np.ascontiguousarray(w, np.float32)) for q, w in wl.queries]
    corpus = wmd.Corpus(wl.vecs, wl.doc_ptr, wl.word_ids, wl.weights, device=0, bf16=True)
    info = corpus.info
    N, h = info["N"], corpus.handle
    opts = dict(precision=wmd.WMD_DIST_BF16, log_domain=1)
    streams = [torch.cuda.Stream() for _ in range(STREAMS)]
    outs = [torch.empty(N, dtype=torch.float64, device="cuda") for _ in streams]

    def step(i):
        q, w = qs[i % len(qs)]
        j = i % STREAMS
        wmd.wmd_query_async(h, q, w, sp.lam, sp.iters, outs[j], None, streams[j], **opts)

    warm(step, 50)
    t0 = time.perf_counter()
    for i in range(steps):
        step(i)
    torch.cuda.synchronize()
    per_q = (time.perf_counter() - t0) / steps
    wmd.wmd_set_timing(h, 1)
    for i in range(50):
        q, w = qs[i % len(qs)]
        wmd.wmd_query_async(h, q, w, sp.lam, sp.iters, outs[0], None, streams[0], **opts)
    torch.cuda.synchronize()
    tm = wmd.wmd_timing_get(h)
    wmd.wmd_set_timing(h, 0)
    docs = np.linspace(0, N - 1, sample_docs).astype(np.int64)
    sptr, sids, sw = synth.subcorpus(wl.doc_ptr, wl.word_ids, wl.weights, docs)
    err_bf16, err_fp32 = [], []
    for q, w in qs[:2]:
        want, _ = sinkhorn_wmd_sparse(wl.vecs, q, w, sptr, sids, sw, sp.lam, sp.iters)
        got16 = corpus.query(q, w, sp.lam, sp.iters, **opts)[0][docs]
        got32 = corpus.query(q, w, sp.lam, sp.iters, log_domain=1)[0][docs]
        err_bf16.append(np.abs(got16 - want) / np.abs(want))
        err_fp32.append(np.abs(got32 - want) / np.abs(want))
    corpus.close()
    return {"workload": f"c4: {len(qs)} queries (v_r {min(len(q) for q, _ in qs)}-{max(len(q) for q, _ in qs)}) "
                        f"in turn vs N={N} docs, V={sp.V}, dim={sp.dim}, nnz={info['nnz']}, U={info['U']}, "
                        f"lambda={sp.lam}, {sp.iters} iterations; BF16 distance GEMM (FP32 accumulation, FP32 "
                        f"recompute below 1e-2), column-shifted K, FP32 Sinkhorn, FP64 WMD sum; {STREAMS} streams",
            "doc_iters_per_s": N * sp.iters / per_q, "us_per_query": per_q * 1e6,
            "kernels_us": {"dist_gemm": 1e3 * tm["dist_ms"] / tm["calls"],
                           "sinkhorn_fused": 1e3 * tm["sinkhorn_ms"] / tm["calls"]},
            "rel_error_vs_fp64_oracle": {
                "bf16_path": rel_stats(np.concatenate(err_bf16)),
                "fp32_path": rel_stats(np.concatenate(err_fp32)),
                "sample": f"2 queries x {docs.size} documents spread over the corpus"}}


def served_stream(wmd, wl, nq: int, rates=None, sample_queries: int = 6, sample_docs: int = 150,
                  budget: int = 16 << 30, max_batch: int = 16, streams: int = 2, batch_words: int = 512,
                  step_iters: int = STEP_ITERS, step_batch: int = STEP_BATCH, step_words: int = STEP_WORDS) -> dict:
    """Served stream on the large corpus: plain FP32 synchronous calls vs the
    server in FP32 (same accuracy) vs the server with BF16 distances, each in
    batch mode and in step mode (iteration-level batching), same queries and
    Poisson arrival times; served results checked bitwise against plain calls
    (FP32) and against the FP64 oracle on sampled documents."""
    from oracle import sinkhorn_wmd_sparse
    from paper_2005_06727_amd import synth
    sp = wl.spec
    corpus = wmd.Corpus(wl.vecs, wl.doc_ptr, wl.word_ids, wl.weights, device=0, bf16=True)
    info = corpus.info
    qs = [(np.ascontiguousarray(q, np.int32), np.ascontiguousarray(w, np.float32)) for q, w in wl.queries[:nq]]
    nq = len(qs)
    lam, iters, N = sp.lam, sp.iters, info["N"]
    lens = np.array([len(q) for q, _ in qs])
    keep = set(int(i) for i in np.argsort(lens)[np.linspace(0, nq - 1, sample_queries).astype(int)])
    work = nq * N * iters
    kw = dict(hbm_budget_bytes=budget, max_batch=max_batch, max_inflight=streams, max_batch_words=batch_words)
    kws = dict(hbm_budget_bytes=budget, max_batch=step_batch, max_batch_words=step_words, step_iters=step_iters)
    paths = {"served_fp32": dict(kw, precision=wmd.WMD_DIST_FP32),
             "served_bf16": dict(kw, precision=wmd.WMD_DIST_BF16),
             "served_step_fp32": dict(kws, precision=wmd.WMD_DIST_FP32),
             "served_step_bf16": dict(kws, precision=wmd.WMD_DIST_BF16)}

    for q, w in qs[:8]:
        corpus.query(q, w, lam, iters)
    # closed loop: every query submitted at once (served) / back to back (plain)
    closed, kept = {}, {}
    t = time.perf_counter()
    kept["plain_fp32"] = {}
    for i, (q, w) in enumerate(qs):
        d = corpus.query(q, w, lam, iters)[0]
        if i in keep:
            kept["plain_fp32"][i] = d
    closed["plain_fp32"] = nq / (time.perf_counter() - t)
    for name in paths:
        with wmd.Server(corpus, **paths[name]) as srv:
            for tk in [srv.submit(q, w, lam, iters) for q, w in qs[:32]]:
                srv.wait(tk)
            t = time.perf_counter()
            ts = [srv.submit(q, w, lam, iters) for q, w in qs]
            kept[name] = {}
            for i, tk in enumerate(ts):
                d = srv.wait(tk)[0]
                if i in keep:
                    kept[name][i] = d
            closed[name] = nq / (time.perf_counter() - t)
    same = {name: all(np.array_equal(kept[name][i], kept["plain_fp32"][i]) for i in keep)
            for name in ("served_fp32", "served_step_fp32")}
    # accuracy on sampled queries x sampled documents
    docs = np.linspace(0, N - 1, sample_docs).astype(np.int64)
    sptr, sids, sw = synth.subcorpus(wl.doc_ptr, wl.word_ids, wl.weights, docs)
    errs = {name: [] for name in paths}
    for i in sorted(keep):
        q, w = qs[i]
        want, _ = sinkhorn_wmd_sparse(wl.vecs, q, w, sptr, sids, sw, lam, iters)
        for name in errs:
            errs[name].append(np.abs(kept[name][i][docs] - want) / np.abs(want))
    # open loop at fixed fractions of the served BF16 capacity
    X = closed["served_bf16"]
    rates = rates or [0.5 * X, 0.9 * X]
    runs = []
    for qps in rates:
        arr = wl.arrivals[:nq] / qps          # unit-rate Poisson times scaled to the offered rate
        run = {"qps": qps, "load_of_served_bf16_capacity": qps / X}
        lat, span = open_loop_plain(lambda qa: corpus.query(qa[0], qa[1], lam, iters), qs, arr)
        run["plain_fp32"] = {"latency_ms": pct(lat), "doc_iters_per_s": work / span}
        for name in paths:
            with wmd.Server(corpus, **paths[name]) as srv:
                for tk in [srv.submit(q, w, lam, iters) for q, w in qs[:16]]:
                    srv.wait(tk)
                srv.reset_stats()
                span, _ = open_loop_served(srv, qs, arr, lam, iters)
                st = srv.stats()
            run[name] = {"latency_ms": server_latency(st), "doc_iters_per_s": work / span,
                         "mean_batch": st["mean_batch"]}
        runs.append(run)
        print(f"# served stream: {qps:.0f} q/s done", file=sys.stderr, flush=True)
    corpus.close()
    return {"workload": f"{sp.name}: Poisson stream of {nq} queries, v_r log-uniform 3-500 "
                        f"(here {lens.min()}-{lens.max()}), V={sp.V}, dim={sp.dim}, N={N}, nnz={info['nnz']}, "
                        f"U={info['U']}, lambda={lam}, {iters} iterations",
            "server": {"hbm_budget_bytes": budget, "max_batch": max_batch, "streams": streams,
                       "max_batch_words": batch_words},
            "server_step_mode": {"hbm_budget_bytes": budget, "step_iters": step_iters,
                                 "max_queries_in_flight": step_batch, "max_words_in_flight": step_words},
            "closed_loop_qps": closed,
            "closed_loop_doc_iters_per_s": {k: v * N * iters for k, v in closed.items()},
            "served_fp32_equals_plain_fp32_bitwise": bool(same["served_fp32"]),
            "served_step_fp32_equals_plain_fp32_bitwise": bool(same["served_step_fp32"]),
            "rel_error_vs_fp64_oracle": {k: rel_stats(np.concatenate(v)) for k, v in errs.items()},
            "error_sample": f"{len(keep)} queries across the v_r range x {docs.size} documents",
            "open_loop": runs}


def serve_main(args):
    import torch
    from paper_2005_06727_amd import synth, wmd
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    wl = synth.make(args.serve, n_queries=args.queries)
    res = served_stream(wmd, wl, args.queries, [args.qps] if args.qps > 0 else None,
                        budget=int(args.hbm_budget_gib * (1 << 30)), max_batch=args.max_batch,
                        streams=args.streams, batch_words=args.batch_words, step_iters=args.step_iters,
                        step_batch=args.step_batch, step_words=args.step_words)
    top = res["open_loop"][-1]
    line = {"metric": "served doc*iters/s + p50/p99 query latency", "value": top["served_bf16"]["doc_iters_per_s"],
            "unit": "doc*iters/s", "n_gpus": 1, "higher_is_better": True,
            "dtype": "bf16 distances, f32 Sinkhorn", "data": "synthetic",
            "config": {"workload": res["workload"] + "; value: served BF16 at the highest offered rate"}}
    line.update(res)
    print(json.dumps(line), flush=True)


def lse_main(args):
    import torch
    from oracle import sinkhorn_wmd_lse
    from paper_2005_06727_amd import synth, wmd

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    wl = synth.make("c4")
    sp = wl.spec
    lam, t = args.lse_lambda, sp.iters
    qs = [(np.ascontiguousarray(q, np.int32), np.ascontiguousarray(w, np.float32)) for q, w in wl.queries]
    corpus = wmd.Corpus(wl.vecs, wl.doc_ptr, wl.word_ids, wl.weights, device=0)
    info = corpus.info
    N, U, nnz, dim = info["N"], info["U"], info["nnz"], info["dim"]
    h = corpus.handle
    streams = [torch.cuda.Stream() for _ in range(STREAMS)]
    outs = [torch.empty(N, dtype=torch.float64, device="cuda") for _ in streams]

    def step(i):
        q, w = qs[i % len(qs)]
        j = i % STREAMS
        wmd.wmd_query_async(h, q, w, lam, t, outs[j], None, streams[j], lse=True)

    warm(step, 40)
    steps = max(args.steps // 50, 80)
    t0 = time.perf_counter()
    for i in range(steps):
        step(i)
    torch.cuda.synchronize()
    per_q = (time.perf_counter() - t0) / steps
    # kernel durations, one stream (events on the launching stream)
    wmd.wmd_set_timing(h, 1)
    for i in range(40):
        q, w = qs[i % len(qs)]
        wmd.wmd_query_async(h, q, w, lam, t, outs[0], None, streams[0], lse=True)
    torch.cuda.synchronize()
    tm = wmd.wmd_timing_get(h)
    wmd.wmd_set_timing(h, 0)
    dist_us = 1e3 * tm["dist_ms"] / tm["calls"]
    sink_us = 1e3 * tm["sinkhorn_ms"] / tm["calls"]
    m_mean = float(np.mean([len(q) for q, _ in qs]))
    exps = (2 * t + 1) * nnz * m_mean                 # one per (nonzero, query word) per log-sum-exp
    fl64 = 3.0 * U * m_mean * dim                    # subtract + FMA per (word, query word, dimension)
    kernels = {
        "sinkhorn_lse": {"avg_us": sink_us, "bound": "alu", "achieved": exps / (sink_us * 1e-6) / 1e12,
                         "peak": PEAK_EXP_TPS, "unit": "Texp/s",
                         "frac": exps / (sink_us * 1e-6) / 1e12 / PEAK_EXP_TPS, "algorithmic_exps": exps},
        "dist_lse": {"avg_us": dist_us, "bound": "alu", "achieved": fl64 / (dist_us * 1e-6) / 1e12,
                     "peak": PEAK_FP64_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": fl64 / (dist_us * 1e-6) / 1e12 / PEAK_FP64_VALU_TFLOPS, "algorithmic_flops": fl64},
    }
    line = {"metric": "target-doc*Sinkhorn-iters/sec, log-domain iteration", "value": N * t / per_q,
            "unit": "doc*iters/s", "n_gpus": 1, "steps": steps, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "ms_per_step": per_q * 1e3,
            "dtype": "f64 distances and potentials, f32 exponentials", "data": "synthetic",
            "config": {"workload": f"precision corpus (V={info['V']}, dim={dim}, N={N}, nnz={nnz}, U={U}) at "
                                   f"lambda={lam:g}, {t} iterations, log-domain iteration; {len(qs)} queries "
                                   f"(v_r {min(len(q) for q, _ in qs)}-{max(len(q) for q, _ in qs)}) in turn "
                                   f"on {STREAMS} streams"},
            "roofline": kernels["sinkhorn_lse"], "kernels": kernels}
    if not args.no_cpu_baseline:
        docs = np.arange(0, N, max(1, N // 1000))
        sptr, sids, sw = synth.subcorpus(wl.doc_ptr, wl.word_ids, wl.weights, docs)
        q, w = qs[0]
        t1 = time.perf_counter()
        sinkhorn_wmd_lse(wl.vecs, q, w, sptr, sids, sw, lam, t)
        dt = time.perf_counter() - t1
        line["cpu_baseline"] = {"value": docs.size * t / dt, "unit": "doc*iters/s", "cores": 1, "kind": "oracle",
                                "sample": f"FP64 numpy log-domain oracle, 1 query x {docs.size} of the {N} "
                                          f"documents (every {N // docs.size}th), {t} iterations, one run "
                                          f"({dt:.2f} s); single-threaded numpy"}
    corpus.close()
    print(json.dumps(line), flush=True)


def profile_batch_main(args):
    """Only the 64-query batch calls (FP32, then BF16 distances), a few times
    each, so that a counter run sees just these kernels."""
    import torch
    from paper_2005_06727_amd import synth, wmd
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    wl = synth.make("c2")
    wl3 = synth.make("c3")
    qs = [(np.ascontiguousarray(q, np.int32), np.ascontiguousarray(w, np.float32)) for q, w in wl3.queries]
    corpus = wmd.Corpus(wl.vecs, wl.doc_ptr, wl.word_ids, wl.weights, device=0, bf16=True)
    for prec in (wmd.WMD_DIST_FP32, wmd.WMD_DIST_BF16):
        for _ in range(5):
            corpus.query_batch(qs, wl3.spec.lam, wl3.spec.iters, precision=prec)
    corpus.close()
    print(json.dumps({"profile_batch": "done", "queries": len(qs)}), flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(documents would shard across GPUs with one all-gather of the N distances). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.serve:
        serve_main(args)
        return
    if args.lse:
        lse_main(args)
        return
    if args.profile_batch:
        profile_batch_main(args)
        return

    from paper_2005_06727_amd import synth
    wl = synth.make(args.workload)
    sp = wl.spec
    q, qw = wl.queries[0]
    q = np.ascontiguousarray(q, np.int32)
    qw = np.ascontiguousarray(qw, np.float32)
    # the host-core oracle runs first, in worker processes forked before the
    # GPU runtime starts
    cpu = None if args.no_cpu_baseline else cpu_baseline(wl, q, qw)

    import torch
    from paper_2005_06727_amd import wmd
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    corpus = wmd.Corpus(wl.vecs, wl.doc_ptr, wl.word_ids, wl.weights, device=0, bf16=True)
    info = corpus.info
    N, U, nnz, m, dim = info["N"], info["U"], info["nnz"], q.size, info["dim"]
    h = corpus.handle
    # consecutive queries cycle over STREAMS streams (and the library's three
    # workspace slots), so one query's distance GEMM overlaps the Sinkhorn
    # kernels of the queries before it
    nstr = max(1, args.headline_streams)
    streams = [torch.cuda.Stream() for _ in range(nstr)]
    outs = [torch.empty(N, dtype=torch.float64, device="cuda") for _ in streams]

    qps_step = max(1, args.queries_per_step)
    seq = [0]

    def one(nstreams):
        j = seq[0] % nstreams
        seq[0] += 1
        wmd.wmd_query_async(h, q, qw, sp.lam, sp.iters, outs[j], None, streams[j])

    def step(i, nstreams=nstr):
        for _ in range(qps_step):
            one(nstreams)

    # no garbage-collector pause in the launching thread from here to the end
    # of the timed region (collected first, so that no pause leaves the GPU
    # idle between the warm-up and the timed steps)
    gc.collect()
    gc.disable()
    warmed = warm(step, args.warmup, args.min_warmup_s)

    # timed region: K steps, no kernel timing inside it
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gc.enable()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = N * sp.iters * qps_step / (ms_per_step * 1e-3)

    # the same pipeline again with every 8th call timed: the kernels' durations
    # while they share the GPU with the other stream's (the sampling slows the
    # pipeline by a few per cent, so the value above is taken without it)
    wmd.wmd_set_timing(h, 8)
    for i in range(max(1, 2000 // qps_step)):
        step(i)
    torch.cuda.synchronize()
    tim = wmd.wmd_timing_get(h)
    wmd.wmd_set_timing(h, False)

    # the same query on one stream, every call timed: each kernel's own
    # duration, with nothing beside it on the GPU
    for i in range(100):
        one(1)
    wmd.wmd_set_timing(h, True)
    for i in range(400):
        one(1)
    torch.cuda.synchronize()
    iso = wmd.wmd_timing_get(h)
    wmd.wmd_set_timing(h, False)

    if args.calibrate_copy > 0:
        # a plain copy of known size: the profiler's byte counters read on it
        # scale the counters read on the library's kernels
        src = torch.ones(args.calibrate_copy << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    got = [o.cpu().numpy() for o in outs]
    assert all(np.all(np.isfinite(g)) and np.all(g > 0) for g in got)
    assert all(np.array_equal(got[0], g) for g in got[1:])

    # per-query latency of the synchronous host API (host arrays in, host results out)
    lat = []
    for _ in range(args.latency_calls):
        t = time.perf_counter()
        corpus.query(q, qw, sp.lam, sp.iters)
        lat.append((time.perf_counter() - t) * 1e3)
    lat = np.array(lat)

    # roofline figures per kernel: algorithmic work per launch / average launch time
    calls = max(iso["calls"], 1)
    dist_s = iso["dist_ms"] / calls * 1e-3
    sink_s = iso["sinkhorn_ms"] / calls * 1e-3
    t_it = sp.iters
    # 4 nnz v_r t: one FMA per (nonzero, query word) in each of the SDDMM and
    # the SpMM of every one of the t x-updates; the final step (one more
    # SDDMM and the K .* M sum) is not counted
    sink_flops = 4.0 * nnz * m * t_it
    sink_flops_exec = 2.0 * nnz * m * (2 * t_it + 1) + 2.0 * nnz * m
    # compulsory bytes: K block of the corpus words (once), CSR, results
    sink_bytes = 4.0 * U * m + 8.0 * nnz + 8.0 * (N + 1) + 8.0 * N
    it_bytes = 4.0 * m * U + 8.0 * nnz + 4.0 * (N + 1) + 8.0 * m * N
    dist_bytes = 4.0 * U * dim + 4.0 * m * dim + 4.0 * U * m
    dist_flops = 2.0 * U * dim * m
    tcalls = max(tim["calls"], 1)
    in_pipeline = lambda ms: ms / tcalls * 1e3
    kernels = {
        "sinkhorn_fused": {
            "avg_us": sink_s * 1e6, "avg_us_in_pipeline": in_pipeline(tim["sinkhorn_ms"]),
            "bound": "alu", "achieved": sink_flops / sink_s / 1e12, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": sink_flops / sink_s / 1e12 / PEAK_FP32_TFLOPS,
            "frac_of_unpacked_fp32_issue_rate": sink_flops / sink_s / 1e12 / PEAK_FP32_UNPACKED_TFLOPS,
            "algorithmic_flops": sink_flops, "flops_as_executed": sink_flops_exec,
            "compulsory_bytes": sink_bytes, "compulsory_GBps": sink_bytes / sink_s / 1e9,
            # the per-iteration form's bound: it would move B_it = 4 v_r U + 8 nnz + 4 (N + 1)
            # + 8 v_r N bytes in every iteration; t of them in the fused kernel's time
            "per_iteration_form_equivalent": {
                "bytes_per_iteration": it_bytes, "GBps": it_bytes * t_it / sink_s / 1e9,
                "frac_of_hbm_peak": it_bytes * t_it / sink_s / 1e9 / PEAK_HBM_GBS}},
        "dist_gemm": {
            "avg_us": dist_s * 1e6, "avg_us_in_pipeline": in_pipeline(tim["dist_ms"]),
            "bound": "hbm", "achieved": dist_bytes / dist_s / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": dist_bytes / dist_s / 1e9 / PEAK_HBM_GBS,
            "algorithmic_bytes": dist_bytes, "mfma_TFLOPs": dist_flops / dist_s / 1e12},
    }
    dom = "sinkhorn_fused" if sink_s >= dist_s else "dist_gemm"
    kd = kernels[dom]
    traffic = counter_traffic(dom, ["k_sinkhorn.hip" if dom == "sinkhorn_fused" else "k_dist.hip", "wmd_device.h",
                                    "wmd_internal.h"])
    roofline = {"kernel": dom, "bound": kd["bound"], "achieved": kd["achieved"], "peak": kd["peak"],
                "unit": kd["unit"], "frac": kd["frac"], "traffic": traffic,
                "time_source": f"HIP events holding the kernel dispatches' own start and end "
                               f"(hipExtLaunchKernel), {calls} calls on one stream",
                "work": ("4 * nnz * v_r * t flops, t = 15 x-updates (final step not counted)"
                         if dom == "sinkhorn_fused" else "corpus rows + query rows + K block bytes")}
    if dom == "sinkhorn_fused":
        roofline["frac_of_unpacked_fp32_issue_rate"] = kd["frac_of_unpacked_fp32_issue_rate"]

    sync_us = float(np.mean(lat)) * 1e3
    line = {
        "metric": "target-doc·Sinkhorn-iters/sec per query + p50/p99 query latency (served)",
        "value": value, "unit": "doc*iters/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{sp.name}: 1 query (v_r={m}) vs N={N} docs, V={sp.V}, dim={dim}, "
                               f"nnz={nnz}, U={U}, lambda={sp.lam}, {sp.iters} iterations, FP32 distances; "
                               f"consecutive queries on {nstr} streams, results in device memory; "
                               f"one step = {qps_step} queries, each its own call",
                   "queries_per_step": qps_step, "V": sp.V, "dim": dim, "N": N, "nnz": nnz, "U": U, "v_r": int(m), "lambda": sp.lam,
                   "iters": sp.iters, "parallelism": "single GPU"},
        "warmup_steps_run": warmed,
        "us_per_query": ms_per_step * 1e3 / qps_step,
        "latency_ms": ({"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                        "what": "synchronous wmd_query: host query in, host distances out"}
                       if lat.size else None),
        "sync_call": ({"us_per_query": sync_us, "doc_iters_per_s": N * sp.iters / (sync_us * 1e-6),
                       "what": "one synchronous wmd_query at a time, PCIe copy of the distances included"}
                      if lat.size else None),
        "roofline": roofline,
        "kernels": kernels,
        "streams": nstr,
        "launches_per_query": iso["launches"],
    }
    if not args.no_batch:
        line["batch64"] = batch_section(wmd, corpus)
        line["extensions"] = extensions_section(wmd, corpus, sp, q, qw)
    corpus.close()
    if not args.no_c4:
        line["precision_c4"] = precision_section(wmd)
    if not args.no_c5:
        wl5 = synth.make("c5", n_queries=args.c5_queries)
        line["served_c5"] = served_stream(wmd, wl5, args.c5_queries)
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
