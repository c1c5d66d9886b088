/*
 * wmd.h -- C ABI of libwmd: sparse Sinkhorn-Knopp Word Mover's Distance of
 * one query document against many target documents, on an AMD MI355X
 * (gfx950) GPU.
 *
 * What is computed (Algorithm 1 of Tithi & Petrini, "An Efficient
 * Shared-memory Parallel Sinkhorn-Knopp Algorithm to Compute the Word
 * Mover's Distance", in the sparse form of its Sec. 4):
 *
 *   r      query histogram over its v_r words with positive weight, sum 1
 *   c_j    histogram of target document j, sum 1
 *   M      v_r x V Euclidean distances between query words and vocabulary
 *          words (Sec. 2), computed only for the query rows
 *   K      exp(-lambda M)
 *   x      v_r x N, starts at 1/v_r; repeated `iters` times:
 *            u = 1/x;  v = c .* (1 ./ (K^T u))   [only where c != 0: SDDMM]
 *            x = diag(1/r) K v                   [SpMM]
 *   final  u = 1/x;  v = c .* (1 ./ (K^T u));
 *          WMD_j = sum_k u_kj ((K .* M) v)_kj = <P_j, M>, P_j = diag(u_j) K diag(v_j)
 *          (Eq. 1; no entropy term)
 *
 * Conventions for every entry point:
 *  - Status: 0 (WMD_OK) on success, a negative WMD_E* code on failure; then
 *    wmd_last_error() returns a message for the calling thread and no output
 *    argument has been written.
 *  - Host pointers are read during the call only; the caller keeps ownership.
 *  - Device pointers are HIP device addresses on the corpus's device.
 *  - Streams are hipStream_t values passed as void* (NULL = null stream).
 *  - Nothing here allocates or frees caller memory.
 */
#ifndef WMD_H
#define WMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WMD_OK         0
#define WMD_EINVAL    (-1)  /* invalid argument or input data */
#define WMD_ENOMEM    (-2)  /* device (or pinned host) allocation failed */
#define WMD_EDEVICE   (-3)  /* a HIP runtime call failed */
#define WMD_ETIMEDOUT (-4)  /* wmd_server_wait timed out; the ticket stays valid */
#define WMD_ESHUTDOWN (-5)  /* the server is shutting down */
#define WMD_ENOTFOUND (-6)  /* unknown or already collected server ticket */

#define WMD_DIST_FP32 0     /* distance GEMM in FP32 (MFMA 16x16x4 f32) */
#define WMD_DIST_BF16 1     /* distance GEMM in BF16 with FP32 accumulation */

typedef struct wmd_corpus wmd_corpus;

typedef struct wmd_corpus_options {
    int32_t device;   /* HIP device ordinal; -1 = the calling thread's current device */
    int32_t bf16;     /* nonzero: also keep BF16 copies of the corpus's embedding rows,
                         required by WMD_DIST_BF16 queries */
} wmd_corpus_options;

typedef struct wmd_query_options {
    int32_t precision;        /* WMD_DIST_FP32 (default) or WMD_DIST_BF16 */
    float   recompute_below;  /* distances below this value are recomputed as a direct
                                 FP32 sum of squared differences (the expansion
                                 |a|^2 + |b|^2 - 2 a.b cancels there); < 0 selects the
                                 default: 0.5 for FP32, 1e-2 for BF16 */
    int32_t log_domain;       /* nonzero: divide each vocabulary column of K by its
                                 largest entry exp(-lambda min_k M[k, i]); the
                                 iterates x, u and the result are unchanged in exact
                                 arithmetic, and K cannot underflow for large lambda */
    int32_t iters_per_launch; /* 0: all iterations and the final step in one fused
                                 launch; k > 0: at most k iterations per launch, x kept
                                 in device memory between launches */
    int32_t tile;             /* Sinkhorn launch shape: -1 picks by query length; 0..7
                                 and 11..16 force that register tile, 8..10 that row-lane
                                 tile (WMD_EINVAL when the query is
                                 longer than the tile holds); -2 uses the streaming
                                 kernel for every document.  Results are identical
                                 between calls with the same tile, and agree across
                                 tiles to FP32 rounding. */
    float   tol;              /* 0: exactly `iters` x updates per document (default).
                                 > 0: the convergence check of Algorithm 1 (iterate
                                 while x still changes): after each x update a document stops once
                                 rho = sum_k r_k |x_k(t) / x_k(t-1) - 1| <= tol (rho is
                                 the row-marginal residual of the plan built from
                                 x(t-1)), else after `iters` updates.  The decision is
                                 taken in FP32.  Needs iters_per_launch = 0 and a tile
                                 of -1, -2, 0..7 or 11..16. */
    int32_t lse;              /* nonzero: the same iteration carried in the log domain
                                 (Algorithm 1 on log u and log v, every product with K
                                 evaluated as a log-sum-exp over the same nonzeros, Sec. 4),
                                 for lambda beyond the range of K = exp(-lambda M) even
                                 with the column shift.  Distances are computed in FP64 as
                                 direct differences, the potentials are FP64 and only the
                                 exponentials of non-positive arguments are FP32, so the
                                 FP32 accuracy bar holds at any lambda.  Needs precision
                                 WMD_DIST_FP32, tol = 0, iters_per_launch = 0, tile = -1
                                 and log_domain = 0 (WMD_EINVAL otherwise).  Limits:
                                 32 * (embedding row + 4) floats (the distance kernel's
                                 staged query rows) and 16 (v_r + longest document) +
                                 4 (longest document + 1) bytes (the iteration's
                                 vectors) of LDS, each at most 160 KB (WMD_EINVAL
                                 beyond). */
} wmd_query_options;

typedef struct wmd_corpus_info {
    int64_t V, N, nnz;        /* vocabulary size, documents, nonzeros after dropping
                                 zero weights */
    int64_t U;                /* distinct vocabulary words used by the documents */
    int32_t dim;              /* embedding dimension */
    int32_t max_doc_words;    /* largest document (distinct words) */
    int32_t device;           /* HIP device ordinal holding the corpus */
    int32_t has_bf16;
    int64_t device_bytes;     /* device memory held by the corpus itself */
} wmd_corpus_info;

/* Fill *opt with the defaults (device -1, no BF16 copies). */
void wmd_corpus_options_init(wmd_corpus_options* opt);

/* Fill *opt with the defaults (FP32, recompute_below -1, no log domain,
 * fused launch, tile -1). */
void wmd_query_options_init(wmd_query_options* opt);

/*
 * Upload a vocabulary embedding table and a bag-of-words corpus (Sec. 4,
 * "A Python Implementation" and "Dataset": vecs is V x dim, c is V x N
 * sparse with normalised columns).
 *
 *  vecs      host, V*dim floats, row-major: row i is the embedding of word i
 *  doc_ptr   host, N+1 int64, CSR by document (the transpose of the paper's
 *            V x N c): document j holds entries doc_ptr[j] .. doc_ptr[j+1]-1;
 *            doc_ptr[0] == 0, non-decreasing
 *  word_ids  host, doc_ptr[N] int32 vocabulary ids in [0, V), distinct within
 *            a document
 *  weights   host, doc_ptr[N] floats >= 0 (raw counts or frequencies); the
 *            library drops zeros and normalises each document to sum 1
 *  opt       nullable
 *  out       receives the corpus handle (untouched on error)
 *
 * Errors: WMD_EINVAL for V <= 0, dim <= 0, N <= 0, a bad doc_ptr, an id out
 * of range, a repeated id within a document, a negative or non-finite
 * weight, a document with no positive weight, more than 2^31-1 nonzeros;
 * WMD_ENOMEM, WMD_EDEVICE.
 */
int wmd_corpus_create(const float* vecs, int64_t V, int32_t dim,
                      const int64_t* doc_ptr, const int32_t* word_ids,
                      const float* weights, int64_t N,
                      const wmd_corpus_options* opt, wmd_corpus** out);

/* Release every device and host resource of the corpus after waiting for its
 * outstanding work.  NULL is a no-op.  The handle must not be in use by
 * another thread or by a server. */
void wmd_corpus_destroy(wmd_corpus* corpus);

/* Sizes and resources of a corpus. */
int wmd_corpus_info_get(const wmd_corpus* corpus, wmd_corpus_info* out);

/*
 * Distances from one query to every document (Algorithm 1; lazily computed
 * M rows, Sec. 4), synchronous.
 *
 *  qids, qweights  host, n entries; query word ids in [0, V), distinct, and
 *                  weights >= 0 (zeros dropped: I = (r > 0); the rest are
 *                  normalised to sum 1)
 *  lambda          >= 0, finite; K = exp(-lambda M)
 *  iters           >= 0 x-updates; the final u/v/WMD step always runs once
 *  out_dist        host, N doubles: out_dist[j] = WMD to document j (input
 *                  order)
 *  out_resid       host, N doubles or NULL: sum_k |(P_j 1)_k - r_k|, the row
 *                  marginal residual of the final plan, accumulated in FP64
 *
 * Errors: WMD_EINVAL (no positive weight, id out of range or repeated,
 * lambda < 0 or not finite, iters < 0, BF16 without BF16 copies),
 * WMD_ENOMEM, WMD_EDEVICE.  Thread-safe: calls on one corpus are serialised.
 */
int wmd_query(wmd_corpus* corpus, const int32_t* qids, const float* qweights,
              int32_t n, float lambda, int32_t iters,
              const wmd_query_options* opt, double* out_dist, double* out_resid);

/*
 * Same computation, stream-ordered: the query arrays are host memory (read
 * before return), the outputs are DEVICE pointers to N doubles (dev_resid
 * nullable), written in stream order on `stream`.  The call returns after
 * enqueueing; argument errors are reported synchronously, device faults at
 * the caller's next synchronisation.  A corpus has three workspace slots used
 * in turn: consecutive calls on different streams may run concurrently, and a
 * call never starts before the call that last used its slot has finished,
 * whatever the streams (calls cycling over three streams keep each slot on
 * one stream, so no call waits on another stream).  Host-side state is locked, so threads may share a
 * corpus.
 */
int wmd_query_async(wmd_corpus* corpus, const int32_t* qids, const float* qweights,
                    int32_t n, float lambda, int32_t iters,
                    const wmd_query_options* opt, double* dev_dist,
                    double* dev_resid, void* stream);

/*
 * wmd_query_async for callers that cannot allocate memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.  The
 * call makes no device or pinned-host allocation: the query's whole device
 * workspace (K block, K .* M when lambda < 0.5, row shifts, iterate, kernel
 * parameters) lives in one fixed array of WMD_NOALLOC_SCRATCH_BYTES that
 * each device holds from the first corpus created on it until the process
 * ends.  Arguments, results and options as wmd_query_async (outputs are
 * DEVICE pointers written in stream order on `stream`).
 *
 * Every call on a device shares that device's array, which keeps the last
 * call's contents (nothing in it needs to start at zero): calls that may
 * overlap on one device (different streams, or threads) race and give wrong
 * results; order them on one stream.  Calls on different devices do not
 * interact.
 *
 * Errors: as wmd_query_async, plus WMD_EINVAL when the workspace exceeds the
 * array (about 4 U v_r bytes, U the corpus's distinct words: v_r up to
 * 16M / U query words, half that when lambda < 0.5, which keeps K .* M too)
 * or the kernel parameter block exceeds 8 KB (about 600 query words).
 */
#define WMD_NOALLOC_SCRATCH_BYTES (64ull << 20)
int wmd_query_noalloc(wmd_corpus* corpus, const int32_t* qids, const float* qweights,
                      int32_t n, float lambda, int32_t iters,
                      const wmd_query_options* opt, double* dev_dist,
                      double* dev_resid, void* stream);

/*
 * B queries against the corpus in one distance-GEMM launch and one fused
 * Sinkhorn launch per shape class (the paper's one-to-many evaluation, Sec. 3,
 * applied to many queries at once).
 *
 *  q_ptr     host, B+1 int64: query b holds entries q_ptr[b] .. q_ptr[b+1]-1
 *  qids, qweights  host, q_ptr[B] entries, as in wmd_query per query
 *  lambdas, iters  host, B entries each (per-query lambda and iteration count)
 *  out_dist  host, B*N doubles, row b = distances of query b
 *  out_resid host, B*N doubles or NULL
 *
 * Results are bitwise identical to B separate wmd_query calls with the same
 * options.  Errors as wmd_query, for any query of the batch.
 */
int wmd_query_batch(wmd_corpus* corpus, int32_t B, const int64_t* q_ptr,
                    const int32_t* qids, const float* qweights,
                    const float* lambdas, const int32_t* iters,
                    const wmd_query_options* opt, double* out_dist,
                    double* out_resid);

/* Stream-ordered wmd_query_batch: outputs are DEVICE pointers (B*N doubles). */
int wmd_query_batch_async(wmd_corpus* corpus, int32_t B, const int64_t* q_ptr,
                          const int32_t* qids, const float* qweights,
                          const float* lambdas, const int32_t* iters,
                          const wmd_query_options* opt, double* dev_dist,
                          double* dev_resid, void* stream);

/* wmd_query with the convergence check (opt->tol > 0; tol = 0 runs exactly
 * max_iters updates): out_iters (nullable, N int32, input document order)
 * receives the number of x updates each document made.  Errors as
 * wmd_query, plus WMD_EINVAL for tol < 0 or not finite, or tol > 0 with
 * iters_per_launch > 0 or a row-lane tile (8..10). */
int wmd_query_adaptive(wmd_corpus* corpus, const int32_t* qids, const float* qweights,
                       int32_t n, float lambda, int32_t max_iters, const wmd_query_options* opt,
                       double* out_dist, double* out_resid, int32_t* out_iters);

/*
 * Retrieval (the k nearest documents of a query, the use of WMD the paper
 * motivates in Sec. 3): distances as wmd_query computes them, then the k
 * smallest selected on the device.  Results ascend by (distance, document
 * index): equal distances are ordered by the smaller index, so the answer is
 * unique.  k in [1, min(N, WMD_MAX_TOPK)], else WMD_EINVAL; other errors as
 * wmd_query.  out_idx receives k document indices (input order numbering),
 * out_dist their k distances.
 */
#define WMD_MAX_TOPK 2048
int wmd_query_topk(wmd_corpus* corpus, const int32_t* qids, const float* qweights,
                   int32_t n, float lambda, int32_t iters, const wmd_query_options* opt,
                   int32_t k, int32_t* out_idx, double* out_dist);

/* Stream-ordered wmd_query_topk: dev_idx (k int32) and dev_dist (k doubles)
 * are DEVICE pointers written in order on `stream`. */
int wmd_query_topk_async(wmd_corpus* corpus, const int32_t* qids, const float* qweights,
                         int32_t n, float lambda, int32_t iters, const wmd_query_options* opt,
                         int32_t k, int32_t* dev_idx, double* dev_dist, void* stream);

/*
 * Kernel timing with HIP events on the stream the kernels run on.  A timed
 * call launches its kernels through hipExtLaunchKernel, so each phase's pair
 * of events holds the start of its first kernel dispatch and the end of its
 * last (the times a kernel trace reports), not the gaps around them.
 * wmd_set_timing(corpus, k) with k > 0 clears the totals and times every
 * k-th query or batch call from then on (1: every call; timed launches cost
 * some host time, so sparse sampling disturbs a pipeline less); 0 disables
 * it.  wmd_timing_get waits for the recorded events and returns
 * milliseconds.  Errors: WMD_EINVAL for k < 0.
 */
typedef struct wmd_timing {
    int64_t calls;            /* timed calls since timing was enabled */
    double dist_ms;           /* distance GEMM + epilogue, summed over the calls */
    double sinkhorn_ms;       /* Sinkhorn iterations + final WMD step, summed */
    float last_dist_ms;       /* the most recent timed call */
    float last_sinkhorn_ms;
    int32_t launches;         /* kernel launches of the most recent timed call */
} wmd_timing;

int wmd_set_timing(wmd_corpus* corpus, int32_t enable);
int wmd_timing_get(wmd_corpus* corpus, wmd_timing* out);

/*
 * Serving: continuous batching of queries against a device-resident corpus
 * (the paper's one-query-against-many evaluation, Sec. 3, applied to a stream
 * of queries).
 *
 * A server owns a worker thread, `max_inflight` HIP streams and one device
 * allocation of `hbm_budget_bytes`.  Submitted queries wait in FIFO order;
 * whenever a stream is free the worker launches the longest FIFO prefix (at
 * most `max_batch` queries and `max_batch_words` query words) whose workspace
 * fits the largest free range of the budget, and the batch's bytes return to
 * the budget when it completes.  So batches admitted while others run
 * overlap on the device, and a query waits only while the budget is in use
 * by running batches (the head of the queue is never overtaken).  The worker
 * polls the running batches' completion, keeping one host core busy while
 * any batch is on the device.  Every query's result is bitwise the one
 * wmd_query returns for it with the same options: a document's computation
 * does not depend on the rest of the batch.
 *
 * Step mode (step_iters > 0): iteration-level continuous batching.  Each
 * admitted query holds its own region of the budget (K block, iterate x,
 * results: about 4 (U + N) ldk bytes) until it completes, and at most
 * max_batch queries are in flight.  The worker enqueues steps (at most two
 * ahead, on one stream): a step runs the distance kernel of the queries
 * admitted into it, then one Sinkhorn launch per shape class over every
 * in-flight query, each advancing step_iters iterations from its own count
 * (with the final step once it reaches its iteration count), then downloads
 * the results of the queries that finished.  Queries join and leave between
 * steps, so a short query does not wait for a long one to finish.  Results are bitwise
 * those of wmd_query (the iterate is kept in FP32 between launches, as in a
 * call with iters_per_launch).  Needs tol = 0, lse = 0, iters_per_launch = 0;
 * batch_wait_us and max_inflight are not used.
 */
typedef struct wmd_server wmd_server;

typedef struct wmd_server_options {
    int64_t hbm_budget_bytes;  /* device memory for the workspaces of all running batches
                                  together (>= 256), allocated once at creation */
    int32_t max_batch;         /* queries per device batch (>= 1) */
    int32_t max_inflight;      /* concurrent batches, one stream each (1..16) */
    int32_t want_resid;        /* also keep the FP64 row-marginal residuals */
    int32_t batch_wait_us;     /* how long a lone waiting query may wait for others to
                                  batch with (0: launch at once) */
    wmd_query_options query;   /* options of every query */
    int32_t max_batch_words;   /* cap on the query words of one batch (its work), so a
                                  burst of queries does not form one long batch; a
                                  query longer than the cap runs alone (0: no cap).
                                  Step mode: cap on the words in flight */
    int32_t step_iters;        /* 0: batch mode.  > 0: step mode (iteration-level
                                  batching, below), each step advancing every
                                  in-flight query by this many iterations */
} wmd_server_options;

typedef struct wmd_server_stats {
    int64_t submitted, completed, batches;
    double latency_p50_ms;     /* submit -> result ready, over completed queries */
    double latency_p99_ms;
    double latency_mean_ms;
    double latency_max_ms;
    double queries_per_s;      /* completed / (last completion - first submission) */
    double doc_iters_per_s;    /* sum over completed queries of N * iters, per second */
    double mean_batch;         /* queries per launched batch */
    int64_t workspace_bytes;   /* device memory held by the server (the budget) */
} wmd_server_stats;

/* Defaults: 4 GiB budget, batches of 16 and at most 512 query words, 2
 * streams, no residuals, no batching wait, default query options, batch
 * mode. */
void wmd_server_options_init(wmd_server_options* opt);

/* Create a server on `corpus` (which must outlive it).  Errors: WMD_EINVAL for
 * bad options (budget < 256, max_batch < 1, max_inflight outside 1..16,
 * step_iters < 0, invalid query options, BF16 without BF16 corpus copies,
 * step mode with lse, tol or iters_per_launch), WMD_ENOMEM, WMD_EDEVICE. */
int wmd_server_create(wmd_corpus* corpus, const wmd_server_options* opt, wmd_server** out);

/* Queue one query (arguments as wmd_query; host arrays copied before return).
 * Returns a ticket >= 0, or WMD_EINVAL for an invalid query, WMD_ENOMEM when
 * the query's workspace alone is larger than the whole budget (any smaller
 * query is admitted once running batches leave room for it),
 * WMD_ESHUTDOWN while the server is being destroyed. */
int64_t wmd_server_submit(wmd_server* server, const int32_t* qids, const float* qweights, int32_t n,
                          float lambda, int32_t iters);

/* Wait up to timeout_us (< 0: forever) for a ticket; on success write N
 * distances (and N residuals when requested at creation and out_resid is
 * non-null) and forget the ticket.  Any thread may wait on any ticket, one
 * waiter per ticket at a time.  WMD_ETIMEDOUT keeps the ticket;
 * WMD_ENOTFOUND for an unknown or collected ticket; WMD_EINVAL while another
 * thread waits on the same ticket; a device error of the ticket's batch is
 * returned as WMD_EDEVICE. */
int wmd_server_wait(wmd_server* server, int64_t ticket, double* out_dist, double* out_resid,
                    int64_t timeout_us);

/* Counters and latency percentiles since creation or the last reset. */
int wmd_server_stats_get(wmd_server* server, wmd_server_stats* out);

/* Restart the statistics (e.g. after a warm-up): completed queries and
 * latencies are forgotten; queries still queued or running count as
 * submitted from now. */
int wmd_server_stats_reset(wmd_server* server);

/* Finish every queued and running query, then release the server.  Results
 * not collected by then are dropped.  NULL is a no-op. */
void wmd_server_destroy(wmd_server* server);

/* Message describing the last non-zero status returned to this thread. */
const char* wmd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* WMD_H */
