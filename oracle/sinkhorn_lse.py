"""FP64 CPU oracle: the Sinkhorn WMD iteration carried in the log domain.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the GPU library.

Algorithm 1 multiplies by K = exp(-lambda M).  Once lambda M passes the
exponent range of the format (FP64: about 745) the entries of K underflow to
zero and the iteration breaks down (0/0 in v = c / (K^T u)).  Writing the
scaling vectors by their logarithms, every product with K becomes a
log-sum-exp over the same index set, evaluated after taking out its largest
term, so no quantity leaves the range.  In exact arithmetic the iterates are
those of Algorithm 1 (sparse form, Sec. 4), step for step:

  x = 1/v_r                      ->  lx = -log v_r
  u = 1/x                        ->  lu = -lx
  v_e = c_e / (K^T u)_e          ->  lv_e = log c_e - LSE_k(lu_k - lambda M[k, i_e])
  x = diag(1/r) K v  (per doc)   ->  lx_k = LSE_{e in doc}(lv_e - lambda M[k, i_e]) - log r_k
  WMD = sum u_k K_ke v_e M_ke    ->  sum_{k, e} exp(lu_k - lambda M[k, i_e] + lv_e) M[k, i_e]

with LSE_j(a_j) = max_j a + log sum_j exp(a_j - max_j a).  The iteration
count, the final step and every reading of the paper are those of
``sinkhorn_wmd_sparse`` (oracle/sinkhorn_wmd.py).

Pins (tests/test_oracle_lse.py): equality with the plain oracle wherever the
latter does not underflow; the one-word-query and one-word-document closed
forms at lambda where the plain form fails; exact column marginals; the shift
identity WMD(M + delta) = WMD(M) + delta far beyond the exponent range; the
entropic bound against the exact earth mover's distance at large lambda.
"""
from __future__ import annotations

import math

import numpy as np

from .sinkhorn_wmd import doc_histograms, query_histogram, word_distances

__all__ = ["sinkhorn_wmd_lse", "sinkhorn_lse_core"]


def _lse_rows(A: np.ndarray) -> np.ndarray:
    """LSE down each column of A (over axis 0)."""
    m = A.max(axis=0)
    return m + np.log(np.exp(A - m[None, :]).sum(axis=0))


def _lse_segments(B: np.ndarray, ptr: np.ndarray) -> np.ndarray:
    """LSE along axis 1 over each segment [ptr[j], ptr[j+1]) of the columns."""
    m = np.maximum.reduceat(B, ptr[:-1], axis=1)
    doc_of = np.repeat(np.arange(ptr.size - 1), np.diff(ptr))
    return m + np.log(np.add.reduceat(np.exp(B - m[:, doc_of]), ptr[:-1], axis=1))


def sinkhorn_lse_core(Mg: np.ndarray, r: np.ndarray, c: np.ndarray, ptr: np.ndarray,
                      lam: float, iters: int, return_plans: bool = False):
    """The log-domain iteration on given distances.

    ``Mg`` is v_r x nnz: column e holds M[:, i_e] for the e-th nonzero of the
    document-major CSR ``ptr``; ``r`` (v_r) and ``c`` (nnz) are normalised
    weights.  Returns (wmd, resid[, plans]) as ``sinkhorn_wmd_sparse`` does.
    """
    if lam < 0 or not math.isfinite(lam):
        raise ValueError("lambda must be finite and >= 0")
    if iters < 0:
        raise ValueError("iters must be >= 0")
    ptr = np.asarray(ptr, dtype=np.int64)
    N = ptr.size - 1
    doc_of = np.repeat(np.arange(N), np.diff(ptr))
    vr = r.size
    lKg = -lam * Mg                                   # log K at the nonzeros
    log_r, log_c = np.log(r), np.log(c)

    def lv_of(lu):       # SDDMM: lv_e = log c_e - LSE_k(lu_k + log K[k, e])
        return log_c - _lse_rows(lKg + lu[:, doc_of])

    lx = np.full((vr, N), -math.log(vr))
    for _ in range(iters):
        lv = lv_of(-lx)
        lx = _lse_segments(lKg + lv[None, :], ptr) - log_r[:, None]   # SpMM
    lu = -lx
    lv = lv_of(lu)
    lP = lu[:, doc_of] + lKg + lv[None, :]            # log of the plan entries
    P = np.exp(lP)
    wmd = np.add.reduceat((P * Mg).sum(axis=0), ptr[:-1])
    row = np.add.reduceat(P, ptr[:-1], axis=1)        # P 1, per document
    resid = np.abs(row - r[:, None]).sum(axis=0)
    out = (wmd, resid)
    if return_plans:
        out = out + ([P[:, ptr[j]:ptr[j + 1]] for j in range(N)],)
    return out


def sinkhorn_wmd_lse(vecs, qids, qweights, doc_ptr, word_ids, weights, lam: float, iters: int,
                     return_plans: bool = False):
    """Log-domain Sinkhorn WMD of one query against every document.

    Same inputs, outputs and readings as ``sinkhorn_wmd_sparse`` (fixed
    iteration count), for any lambda >= 0.
    """
    ptr = np.asarray(doc_ptr, dtype=np.int64)
    if np.any(np.diff(ptr) <= 0):
        raise ValueError("every document needs at least one word")
    ids, r = query_histogram(qids, qweights)
    c = doc_histograms(ptr, weights)
    words, row_of = np.unique(np.asarray(word_ids, dtype=np.int64), return_inverse=True)
    M = word_distances(vecs, ids, words)
    return sinkhorn_lse_core(M[:, row_of], r, c, ptr, lam, int(iters), return_plans)
