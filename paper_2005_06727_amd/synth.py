"""Seeded synthetic inputs for one-query-against-many-documents Sinkhorn WMD.

This module only *draws* inputs; it holds none of the method's arithmetic
(no distances, no kernel matrix, no normalisation of histograms).  Both the
FP64 oracle (through the tests) and the GPU library consume what it returns.

Stand-in for the paper's data (Sec. 4, "Dataset"): a 100 000-word subset of a
300-dimensional crawl embedding, and the first 5000 documents of a DBpedia
training file as targets.  Neither is available here, so the shapes are kept
and the values are synthetic:

* embeddings: i.i.d. N(0,1) in FP64, each row scaled to unit L2 norm in FP64,
  then rounded to FP32.  The FP32 values are canonical for every consumer.
* document words: each document draws its length uniformly from an integer
  range, then that many *distinct* word ids from a Zipf(s) law over ranks
  1..V (id = rank-1), rejecting repeats.  Rank order stands in for a
  frequency-sorted vocabulary file.
* weights: raw counts ~ Geometric(p=0.5) on {1, 2, ...}, passed as floats
  (exact in FP32); every consumer normalises them itself.
* queries: distinct ids, uniform over the vocabulary (small correctness case)
  or Zipf like the documents (the paper's queries are documents of the same
  corpus), with Geometric(0.5) counts.

Seeds: ``numpy.random.SeedSequence(config_seed).spawn(4)`` gives independent
streams for embeddings, corpus, queries and arrival times.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

__all__ = [
    "WorkloadSpec", "Workload", "SPECS", "embeddings", "zipf_cdf",
    "corpus", "query", "loguniform_lengths", "make", "subcorpus", "near_duplicates",
]


@dataclasses.dataclass(frozen=True)
class WorkloadSpec:
    name: str
    seed: int              # SeedSequence entropy for embeddings + corpus
    query_seed: int        # SeedSequence entropy for the query stream
    V: int
    dim: int
    N: int
    doc_len: Tuple[int, int]
    n_queries: int
    q_len: Tuple[int, int]
    q_len_law: str         # "uniform" (integer) or "loguniform"
    q_words: str           # "uniform" or "zipf"
    lam: float
    iters: int
    zipf_s: float = 1.1


# The five workloads: a tiny correctness case, the paper-shaped single query
# (V=100k, w=300, N=5000, Sec. 4 "Dataset"), a 64-query batch on that corpus,
# a large-lambda precision case and a served stream on a larger corpus.
SPECS = {
    "c1": WorkloadSpec("c1", 1, 1, V=2000, dim=64, N=100, doc_len=(5, 20),
                       n_queries=1, q_len=(10, 10), q_len_law="uniform",
                       q_words="uniform", lam=10.0, iters=15),
    "c2": WorkloadSpec("c2", 2, 2, V=100_000, dim=300, N=5000, doc_len=(10, 60),
                       n_queries=1, q_len=(20, 40), q_len_law="uniform",
                       q_words="zipf", lam=10.0, iters=15),
    "c3": WorkloadSpec("c3", 2, 3, V=100_000, dim=300, N=5000, doc_len=(10, 60),
                       n_queries=64, q_len=(5, 200), q_len_law="uniform",
                       q_words="zipf", lam=10.0, iters=15),
    "c4": WorkloadSpec("c4", 4, 4, V=100_000, dim=300, N=20_000, doc_len=(10, 60),
                       n_queries=8, q_len=(20, 40), q_len_law="uniform",
                       q_words="zipf", lam=50.0, iters=15),
    "c5": WorkloadSpec("c5", 5, 5, V=200_000, dim=300, N=100_000, doc_len=(10, 60),
                       n_queries=10_000, q_len=(3, 500), q_len_law="loguniform",
                       q_words="zipf", lam=10.0, iters=15),
}


@dataclasses.dataclass
class Workload:
    spec: WorkloadSpec
    vecs: np.ndarray          # (V, dim) float32, C-contiguous
    doc_ptr: np.ndarray       # (N+1,) int64
    word_ids: np.ndarray      # (nnz,) int32
    weights: np.ndarray       # (nnz,) float32 raw counts
    queries: List[Tuple[np.ndarray, np.ndarray]]   # (ids int32, counts float32)
    arrivals: Optional[np.ndarray] = None          # unit-rate Poisson times


def embeddings(V: int, dim: int, rng: np.random.Generator) -> np.ndarray:
    e = rng.standard_normal((V, dim))
    e /= np.sqrt(np.einsum("ij,ij->i", e, e))[:, None]
    return np.ascontiguousarray(e.astype(np.float32))


def zipf_cdf(V: int, s: float) -> np.ndarray:
    p = np.arange(1, V + 1, dtype=np.float64) ** (-s)
    c = np.cumsum(p)
    return c / c[-1]


def _distinct_zipf(cdf: np.ndarray, n: int, rng: np.random.Generator) -> np.ndarray:
    """n distinct ids, drawn Zipf in order of first appearance (rejection)."""
    out: List[int] = []
    seen = set()
    while len(out) < n:
        draw = np.searchsorted(cdf, rng.random(2 * n + 8), side="right")
        for w in draw.tolist():
            if w not in seen:
                seen.add(w)
                out.append(w)
                if len(out) == n:
                    break
    return np.asarray(out, dtype=np.int32)


def corpus(V: int, N: int, doc_len: Tuple[int, int], rng: np.random.Generator,
           s: float = 1.1):
    lo, hi = doc_len
    lens = rng.integers(lo, hi + 1, size=N)
    cdf = zipf_cdf(V, s)
    ptr = np.zeros(N + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(lens)
    ids = np.empty(int(ptr[-1]), dtype=np.int32)
    for j in range(N):
        ids[ptr[j]:ptr[j + 1]] = _distinct_zipf(cdf, int(lens[j]), rng)
    counts = rng.geometric(0.5, size=ids.size).astype(np.float32)
    return ptr, ids, counts


def query(V: int, n: int, rng: np.random.Generator, words: str = "zipf",
          s: float = 1.1, cdf: Optional[np.ndarray] = None):
    if words == "uniform":
        ids = rng.choice(V, size=n, replace=False).astype(np.int32)
    else:
        ids = _distinct_zipf(zipf_cdf(V, s) if cdf is None else cdf, n, rng)
    counts = rng.geometric(0.5, size=n).astype(np.float32)
    return ids, counts


def loguniform_lengths(n: int, lo: int, hi: int, rng: np.random.Generator) -> np.ndarray:
    v = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n))
    return np.clip(np.rint(v), lo, hi).astype(np.int64)


def make(name: str, n_queries: Optional[int] = None) -> Workload:
    """Build workload ``name`` ("c1".."c5"); ``n_queries`` caps the query count."""
    sp = SPECS[name]
    s_emb, s_corp, _, _ = np.random.SeedSequence(sp.seed).spawn(4)
    _, _, s_q, s_arr = np.random.SeedSequence(sp.query_seed).spawn(4)
    vecs = embeddings(sp.V, sp.dim, np.random.default_rng(s_emb))
    ptr, ids, counts = corpus(sp.V, sp.N, sp.doc_len, np.random.default_rng(s_corp), sp.zipf_s)
    rq = np.random.default_rng(s_q)
    nq = sp.n_queries if n_queries is None else min(n_queries, sp.n_queries)
    if sp.q_len_law == "loguniform":
        lens = loguniform_lengths(sp.n_queries, sp.q_len[0], sp.q_len[1], rq)
    else:
        lens = rq.integers(sp.q_len[0], sp.q_len[1] + 1, size=sp.n_queries)
    cdf = zipf_cdf(sp.V, sp.zipf_s) if sp.q_words == "zipf" else None
    queries = [query(sp.V, int(lens[q]), rq, sp.q_words, sp.zipf_s, cdf) for q in range(nq)]
    arrivals = None
    if name == "c5":
        arrivals = np.cumsum(np.random.default_rng(s_arr).exponential(1.0, size=sp.n_queries))
    return Workload(sp, vecs, ptr, ids, counts, queries, arrivals)


def subcorpus(doc_ptr: np.ndarray, word_ids: np.ndarray, weights: np.ndarray,
              docs: np.ndarray):
    """CSR restricted to the documents ``docs`` (in that order)."""
    docs = np.asarray(docs, dtype=np.int64)
    lens = doc_ptr[docs + 1] - doc_ptr[docs]
    ptr = np.zeros(docs.size + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(lens)
    sel = np.concatenate([np.arange(doc_ptr[d], doc_ptr[d + 1]) for d in docs]) \
        if docs.size else np.zeros(0, dtype=np.int64)
    return ptr, word_ids[sel].copy(), weights[sel].copy()


def near_duplicates(vecs: np.ndarray, bases: np.ndarray, rows: np.ndarray, dists: np.ndarray,
                    rng: np.random.Generator) -> np.ndarray:
    """A copy of ``vecs`` in which row ``rows[i]`` is replaced by a unit vector
    at Euclidean (chord) distance ``dists[i]`` from row ``bases[i]``: the base
    rotated by the angle 2 asin(d / 2) towards a random direction orthogonal
    to it, in FP64, then rounded to FP32 like every embedding.  Real
    embedding tables hold such near-synonyms; the synthetic N(0, 1) rows do
    not (their pairwise distances lie near sqrt(2))."""
    out = np.array(vecs, dtype=np.float32, copy=True)
    for b, r, d in zip(np.asarray(bases), np.asarray(rows), np.asarray(dists, dtype=np.float64)):
        e = out[b].astype(np.float64)
        e /= np.linalg.norm(e)
        z = rng.standard_normal(e.size)
        z -= (z @ e) * e
        z /= np.linalg.norm(z)
        th = 2.0 * np.arcsin(d / 2.0)
        out[r] = (np.cos(th) * e + np.sin(th) * z).astype(np.float32)
    return out
