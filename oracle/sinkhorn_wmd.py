"""FP64 CPU oracle for one-query-against-many-documents Sinkhorn WMD.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the GPU library.

It is a plain, slow statement of Algorithm 1 of the paper (Cuturi's
Sinkhorn-Knopp scaling for the entropic transport distance), as the paper's
Sec. 4 walk-through of its Python implementation applies it to WMD, and of the
paper's sparse reformulation of the same iteration (Sec. 4, "Dense to Sparse
Kernel" and "The SDDMM_SpMM Kernel").  Every float is FP64; FP32 inputs are
widened exactly.

Two forms are given:

* ``sinkhorn_wmd_dense``  -- Algorithm 1 as printed: K is v_r x V, c is the
  dense V x N matrix of document histograms, K^T u is a dense product and the
  result is masked by c afterwards.
* ``sinkhorn_wmd_sparse`` -- the paper's transformation: K^T u is evaluated
  only at the nonzeros of c (SDDMM), then x = diag(1/r) K v (SpMM).

With ``exact=True`` every sum is an exactly rounded sum (``math.fsum``) of the
same rounded FP64 products, so the two forms agree bit for bit: the dense form
only adds exact zeros.  That mode is for tiny inputs.

Readings of the paper taken here (where it is silent, garbled or at odds with
itself):

* distance is the Euclidean norm (not its square): Sec. 2 prints a squared
  norm but defines it as sqrt(sum(pow(diff, 2))), as does the cdist call of
  Table 1;
* lambda >= 0 and K = exp(-lambda M) (the Python passes lambda pre-negated);
* ``iters`` = number of x updates; the final u/v/WMD step always runs once
  more, so iters = 0 is legal;
* at zeros of c, v = 0 and no division is made (c.multiply keeps the pattern);
* document and query weights are normalised to sum to one (Sec. 4);
* the result is <P, M> with P = diag(u) K diag(v) (Eq. 1), with no entropy
  term.

Pins (tests/test_oracle_pins.py): cdist; closed forms at lambda = 0, at t = 0,
for a one-word query, a one-word document and the symmetric 2 x 2 problem;
exact column marginals; row marginals -> r; dense == sparse bit for bit;
brute-force / assignment / LP earth mover's distance within the entropic
bound; WMD(d, d) -> 0 as lambda grows; symmetry at convergence.
"""
from __future__ import annotations

import math
from typing import List, Optional, Tuple

import numpy as np

__all__ = [
    "query_histogram", "doc_histograms", "dense_doc_matrix", "word_distances",
    "sinkhorn_wmd_dense", "sinkhorn_wmd_sparse",
]


# -- o1: inputs (Algorithm 1 first step; Sec. 4 Python walk-through) ---------

def query_histogram(qids, qweights) -> Tuple[np.ndarray, np.ndarray]:
    """Select the query words with r > 0 (I = (r > 0); r = r(I)) and
    normalise so that sum(r) = 1.  Returns (word ids int64, r FP64)."""
    ids = np.asarray(qids, dtype=np.int64)
    w = np.asarray(qweights, dtype=np.float32).astype(np.float64)
    if ids.shape != w.shape or ids.ndim != 1:
        raise ValueError("query ids and weights must be 1-D of equal length")
    if np.unique(ids).size != ids.size:
        raise ValueError("a histogram holds each word once")
    if np.any(~np.isfinite(w)) or np.any(w < 0):
        raise ValueError("query weights must be finite and >= 0")
    keep = w > 0
    ids, w = ids[keep], w[keep]
    if ids.size == 0:
        raise ValueError("query has no word with positive weight")
    return ids, w / math.fsum(w)


def doc_histograms(doc_ptr, weights) -> np.ndarray:
    """Per-nonzero values of c: each document's weights divided by their sum
    (columns of c sum to one, Sec. 4)."""
    ptr = np.asarray(doc_ptr, dtype=np.int64)
    w = np.asarray(weights, dtype=np.float32).astype(np.float64)
    c = np.empty_like(w)
    for j in range(ptr.size - 1):
        seg = w[ptr[j]:ptr[j + 1]]
        c[ptr[j]:ptr[j + 1]] = seg / math.fsum(seg)
    return c


def dense_doc_matrix(V: int, doc_ptr, word_ids, weights) -> np.ndarray:
    """The V x N matrix c of Algorithm 1, column j = histogram of document j."""
    ptr = np.asarray(doc_ptr, dtype=np.int64)
    N = ptr.size - 1
    C = np.zeros((V, N))
    c = doc_histograms(ptr, weights)
    for j in range(N):
        C[np.asarray(word_ids[ptr[j]:ptr[j + 1]], dtype=np.int64), j] = c[ptr[j]:ptr[j + 1]]
    return C


# -- o2: the cost matrix (Sec. 2 definition of m(i, j)) ----------------------

def word_distances(vecs, rows, cols) -> np.ndarray:
    """M[k, i] = sqrt(sum_d (E[rows[k], d] - E[cols[i], d])^2), the Euclidean
    distance written as a direct difference, in FP64."""
    E = np.asarray(vecs, dtype=np.float32).astype(np.float64)
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    B = E[cols]
    M = np.empty((rows.size, cols.size))
    for k in range(rows.size):
        diff = B - E[rows[k]]
        M[k] = np.sqrt(np.sum(diff * diff, axis=1))
    return M


# -- reductions: numpy by default, exactly rounded on request ---------------

def _matmul(A: np.ndarray, B: np.ndarray, exact: bool) -> np.ndarray:
    if not exact:
        return A @ B
    out = np.empty((A.shape[0], B.shape[1]))
    for i in range(A.shape[0]):
        prod = A[i][:, None] * B
        for j in range(B.shape[1]):
            out[i, j] = math.fsum(prod[:, j])
    return out


def _colsum(A: np.ndarray, exact: bool) -> np.ndarray:
    if not exact:
        return A.sum(axis=0)
    return np.array([math.fsum(A[:, j]) for j in range(A.shape[1])])


# -- Algorithm 1, dense ------------------------------------------------------

def sinkhorn_wmd_dense(vecs, qids, qweights, C, lam: float, iters: int,
                       exact: bool = False, return_plans: bool = False):
    """Algorithm 1 over the whole vocabulary.

    ``C`` is the dense V x N matrix of normalised document histograms
    (``dense_doc_matrix``).  Returns the N distances, and with
    ``return_plans`` also the plans P_j = diag(u_j) K diag(v_j) (Eq. 1) as a
    v_r x V x N array.
    """
    if lam < 0 or not math.isfinite(lam):
        raise ValueError("lambda must be finite and >= 0")
    if iters < 0:
        raise ValueError("iters must be >= 0")
    C = np.asarray(C, dtype=np.float64)
    V, N = C.shape
    ids, r = query_histogram(qids, qweights)
    vr = ids.size
    M = word_distances(vecs, ids, np.arange(V))        # M = M(I, :), computed lazily
    K = np.exp(-lam * M)
    K_over_r = K / r[:, None]                          # diag(1./r) * K
    nz = C > 0

    def v_of(u):                                       # c .* (1./(K^T u)) at c != 0
        KTu = _matmul(K.T, u, exact)
        v = np.zeros_like(C)
        np.divide(C, KTu, out=v, where=nz)
        return v

    x = np.ones((vr, N)) / vr
    for _ in range(iters):
        x = _matmul(K_over_r, v_of(1.0 / x), exact)
    u = 1.0 / x
    v = v_of(u)
    wmd = _colsum(u * _matmul(K * M, v, exact), exact)
    if return_plans:
        P = u[:, None, :] * K[:, :, None] * v[None, :, :]
        return wmd, P
    return wmd


# -- the sparse transformation (SDDMM at the nonzeros of c, then SpMM) -------

def sinkhorn_wmd_sparse(vecs, qids, qweights, doc_ptr, word_ids, weights,
                        lam: float, iters, exact: bool = False,
                        return_plans: bool = False, tol: float = 0.0,
                        return_history: bool = False):
    """Same iteration, evaluated only where c != 0.

    Returns ``(wmd, resid)``: the N distances and, per document, the row
    marginal residual sum_k |(P 1)_k - r_k| of the final plan (its column
    marginal equals c exactly).  With ``return_plans`` a third item lists the
    plans P_j (v_r x nnz_j, columns in the document's CSR order).

    ``iters`` is one count for every document or an array of N counts (each
    document stops its x updates after its own count; column j of x depends
    only on column j, so this is the same as running the documents alone).

    ``tol > 0`` is Algorithm 1's stopping test (iterate while x still changes): after each x update,
    document j computes rho_j = sum_k r_k |x_new[k, j] / x_old[k, j] - 1| and
    makes no further update once rho_j <= tol (at most ``iters`` updates).
    With ``return_history`` the result gains the number of updates t_j of
    each document and the list of its rho values.
    """
    if lam < 0 or not math.isfinite(lam):
        raise ValueError("lambda must be finite and >= 0")
    if np.any(np.asarray(iters) < 0):
        raise ValueError("iters must be >= 0")
    if not (tol >= 0 and math.isfinite(tol)):
        raise ValueError("tol must be finite and >= 0")
    ptr = np.asarray(doc_ptr, dtype=np.int64)
    word_ids = np.asarray(word_ids, dtype=np.int64)
    N = ptr.size - 1
    if np.any(np.diff(ptr) <= 0):
        raise ValueError("every document needs at least one word")
    ids, r = query_histogram(qids, qweights)
    vr = ids.size
    c = doc_histograms(ptr, weights)
    doc_of = np.repeat(np.arange(N), np.diff(ptr))     # column j of each nonzero
    words, row_of = np.unique(word_ids, return_inverse=True)
    M = word_distances(vecs, ids, words)               # only the words c uses
    K = np.exp(-lam * M)
    K_over_r = K / r[:, None]
    KM = K * M
    Kg, KoRg, KMg = K[:, row_of], K_over_r[:, row_of], KM[:, row_of]

    def sddmm(u):        # s_e = sum_k K[k, i_e] u[k, j_e] for each nonzero e
        prod = Kg * u[:, doc_of]
        if not exact:
            return prod.sum(axis=0)
        return np.array([math.fsum(prod[:, e]) for e in range(prod.shape[1])])

    def spmm(Ag, v):     # out[k, j] = sum_{e in doc j} Ag[k, e] v_e
        prod = Ag * v[None, :]
        if not exact:
            return np.add.reduceat(prod, ptr[:-1], axis=1)
        out = np.empty((vr, N))
        for j in range(N):
            for k in range(vr):
                out[k, j] = math.fsum(prod[k, ptr[j]:ptr[j + 1]])
        return out

    t_max = np.broadcast_to(np.asarray(iters, dtype=np.int64), (N,))
    x = np.ones((vr, N)) / vr
    t = np.zeros(N, dtype=np.int64)                 # x updates made so far
    active = t_max > 0
    history = [[] for _ in range(N)]
    while np.any(active):
        x_new = spmm(KoRg, c / sddmm(1.0 / x))
        rho = _colsum(r[:, None] * np.abs(x_new / x - 1.0), exact)
        for j in np.flatnonzero(active):
            history[j].append(float(rho[j]))
        x = np.where(active[None, :], x_new, x)
        t = t + active
        active = active & (t < t_max)
        if tol > 0:
            active = active & (rho > tol)
    u = 1.0 / x
    v = c / sddmm(u)
    wmd = _colsum(u * spmm(KMg, v), exact)
    resid = _colsum(np.abs(u * spmm(Kg, v) - r[:, None]), exact)
    out = (wmd, resid)
    if return_plans:
        plans = [u[:, j][:, None] * Kg[:, ptr[j]:ptr[j + 1]] * v[None, ptr[j]:ptr[j + 1]]
                 for j in range(N)]
        out = out + (plans,)
    if return_history:
        out = out + (t, history)
    return out
