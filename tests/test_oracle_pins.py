"""Pins of the FP64 oracle against facts fixed by the paper and by the
mathematics, independently of the oracle's own code.

* Sec. 2 / Table 1: word distance is the Euclidean (cdist) distance.
* Algorithm 1 with lambda = 0: K = 1 and the plan is r c_j^T after one
  update, so WMD_j = r^T M c_j for any t >= 1.
* Algorithm 1 with t = 0: u = v_r * 1, so P[k, i] = c_i K[k, i] / sum_k K[k, i].
* One query word: x stays 1, so P = c_j and WMD_j = sum_i c_ij M[0, i].
* One-word document: P = r after one update, WMD = sum_k r_k M[k, i].
* Symmetric 2 x 2 (uniform r = c over the same two words): x is a fixed point
  from the start, WMD = d / (1 + exp(lambda d)).
* General 2 x 2 at convergence: the plan with the given marginals whose
  cross ratio is exp(lambda (M12 + M21 - M11 - M22)) (Eq. 1).
* Eq. 1 plan: column marginals equal c exactly after every final step; row
  marginals tend to r.
* At convergence: EMD <= d <= EMD + min(H(r), H(c)) / lambda, with EMD from
  brute force, assignment and LP; d(a, a) falls with lambda; d is symmetric.
"""
import math

import numpy as np
import pytest
from scipy.spatial.distance import cdist

from oracle import (dense_doc_matrix, doc_histograms, query_histogram,
                    sinkhorn_wmd_dense, sinkhorn_wmd_sparse, word_distances)
from paper_2005_06727_amd import synth
from tests.emd_exact import (emd_assignment_uniform, emd_bruteforce_uniform,
                             emd_lp, entropy)


def tiny(V=60, dim=8, N=7, doc_len=(1, 6), vr=4, seed=0):
    rng = np.random.default_rng(seed)
    vecs = synth.embeddings(V, dim, rng)
    ptr, ids, w = synth.corpus(V, N, doc_len, rng)
    qids, qw = synth.query(V, vr, rng, "uniform")
    return vecs, ptr, ids, w, qids, qw


def cdist64(vecs, a, b):
    E = vecs.astype(np.float64)
    return cdist(E[np.asarray(a)], E[np.asarray(b)])


def both_forms(vecs, ptr, ids, w, qids, qw, lam, t, exact=False):
    V = vecs.shape[0]
    C = dense_doc_matrix(V, ptr, ids, w)
    d = sinkhorn_wmd_dense(vecs, qids, qw, C, lam, t, exact=exact)
    s, _ = sinkhorn_wmd_sparse(vecs, qids, qw, ptr, ids, w, lam, t, exact=exact)
    return d, s


def test_distances_match_cdist():
    rng = np.random.default_rng(3)
    vecs = synth.embeddings(300, 64, rng)
    a, b = rng.choice(300, 17, replace=False), np.arange(300)
    M = word_distances(vecs, a, b)
    np.testing.assert_allclose(M, cdist64(vecs, a, b), rtol=1e-13, atol=1e-15)
    assert np.all(word_distances(vecs, a, a).diagonal() == 0.0)
    # Euclidean, not squared (Sec. 2 definition)
    assert not np.allclose(M, cdist64(vecs, a, b) ** 2)


@pytest.mark.parametrize("t", [1, 2, 15])
def test_lambda_zero_closed_form(t):
    vecs, ptr, ids, w, qids, qw = tiny(seed=1)
    d, s = both_forms(vecs, ptr, ids, w, qids, qw, 0.0, t)
    wq = qw.astype(np.float64)
    r = wq / wq.sum()
    for j in range(ptr.size - 1):
        words = ids[ptr[j]:ptr[j + 1]]
        c = w[ptr[j]:ptr[j + 1]].astype(np.float64)
        c /= c.sum()
        want = r @ cdist64(vecs, qids, words) @ c
        assert d[j] == pytest.approx(want, rel=1e-13)
        assert s[j] == pytest.approx(want, rel=1e-13)


@pytest.mark.parametrize("lam", [0.5, 10.0, 40.0])
def test_zero_iterations_closed_form(lam):
    vecs, ptr, ids, w, qids, qw = tiny(seed=2)
    d, s = both_forms(vecs, ptr, ids, w, qids, qw, lam, 0)
    for j in range(ptr.size - 1):
        words = ids[ptr[j]:ptr[j + 1]]
        c = w[ptr[j]:ptr[j + 1]].astype(np.float64)
        c /= c.sum()
        M = cdist64(vecs, qids, words)
        K = np.exp(-lam * M)
        want = float((c * (K * M).sum(0) / K.sum(0)).sum())
        assert d[j] == pytest.approx(want, rel=1e-12)
        assert s[j] == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("lam,t", [(3.0, 0), (10.0, 1), (25.0, 15)])
def test_one_word_query(lam, t):
    vecs, ptr, ids, w, _, _ = tiny(seed=4)
    q = np.array([5], dtype=np.int32)
    d, s = both_forms(vecs, ptr, ids, w, q, np.array([3.0], np.float32), lam, t)
    for j in range(ptr.size - 1):
        words = ids[ptr[j]:ptr[j + 1]]
        c = w[ptr[j]:ptr[j + 1]].astype(np.float64)
        c /= c.sum()
        want = float(cdist64(vecs, q, words)[0] @ c)
        assert d[j] == pytest.approx(want, rel=1e-12)
        assert s[j] == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("lam,t", [(3.0, 1), (10.0, 4), (25.0, 15)])
def test_one_word_document(lam, t):
    vecs, _, _, _, qids, qw = tiny(seed=5, vr=6)
    ptr = np.array([0, 1, 2, 3], np.int64)
    ids = np.array([7, int(qids[0]), 33], np.int32)     # one shares a query word
    w = np.array([2.0, 1.0, 5.0], np.float32)
    d, s = both_forms(vecs, ptr, ids, w, qids, qw, lam, t)
    r = qw.astype(np.float64) / qw.astype(np.float64).sum()
    for j in range(3):
        want = float(r @ cdist64(vecs, qids, ids[j:j + 1])[:, 0])
        assert d[j] == pytest.approx(want, rel=1e-12)
        assert s[j] == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("lam", [0.0, 1.0, 7.5, 30.0])
@pytest.mark.parametrize("t", [0, 1, 9])
def test_symmetric_two_by_two(lam, t):
    vecs = synth.embeddings(10, 5, np.random.default_rng(6))
    q = np.array([2, 7], np.int32)
    ptr = np.array([0, 2], np.int64)
    d, s = both_forms(vecs, ptr, q[::-1].copy(), np.array([4, 4], np.float32),
                      q, np.array([1, 1], np.float32), lam, t)
    dist = float(np.linalg.norm(vecs[2].astype(np.float64) - vecs[7].astype(np.float64)))
    want = dist / (1.0 + math.exp(lam * dist))
    assert d[0] == pytest.approx(want, rel=1e-13)
    assert s[0] == pytest.approx(want, rel=1e-13)


def test_general_two_by_two_converged():
    vecs = synth.embeddings(10, 3, np.random.default_rng(7))
    q, qw = np.array([1, 4], np.int32), np.array([3, 1], np.float32)
    doc, dw = np.array([6, 8], np.int32), np.array([1, 2], np.float32)
    lam = 6.0
    d, s = both_forms(vecs, np.array([0, 2]), doc, dw, q, qw, lam, 3000)
    M = cdist64(vecs, q, doc)
    r1, r2 = 0.75, 0.25
    c1 = 1.0 / 3.0
    rho = math.exp(lam * (M[0, 1] + M[1, 0] - M[0, 0] - M[1, 1]))
    # (1 - rho) a^2 + (r2 - c1 + rho (r1 + c1)) a - rho r1 c1 = 0
    A, B, Cc = 1.0 - rho, r2 - c1 + rho * (r1 + c1), -rho * r1 * c1
    roots = np.roots([A, B, Cc])
    lo, hi = max(0.0, c1 - r2), min(r1, c1)
    a = [x.real for x in roots if abs(x.imag) < 1e-14 and lo < x.real < hi]
    assert len(a) == 1
    a = a[0]
    P = np.array([[a, r1 - a], [c1 - a, r2 - c1 + a]])
    want = float((P * M).sum())
    assert d[0] == pytest.approx(want, rel=1e-11)
    assert s[0] == pytest.approx(want, rel=1e-11)


@pytest.mark.parametrize("t", [0, 1, 6])
def test_marginals(t):
    vecs, ptr, ids, w, qids, qw = tiny(seed=8, N=9)
    _, resid, plans = sinkhorn_wmd_sparse(vecs, qids, qw, ptr, ids, w, 8.0, t,
                                          return_plans=True)
    c = doc_histograms(ptr, w)
    _, r = query_histogram(qids, qw)
    for j, P in enumerate(plans):
        np.testing.assert_allclose(P.sum(0), c[ptr[j]:ptr[j + 1]], rtol=1e-14, atol=0)
        assert resid[j] == pytest.approx(np.abs(P.sum(1) - r).sum(), rel=1e-10, abs=1e-16)
    # dense plans agree with the sparse ones
    C = dense_doc_matrix(vecs.shape[0], ptr, ids, w)
    _, Pd = sinkhorn_wmd_dense(vecs, qids, qw, C, 8.0, t, return_plans=True)
    for j, P in enumerate(plans):
        np.testing.assert_allclose(Pd[:, ids[ptr[j]:ptr[j + 1]], j], P, rtol=1e-12)


def test_row_marginals_converge():
    vecs, ptr, ids, w, qids, qw = tiny(seed=9)
    _, r5 = sinkhorn_wmd_sparse(vecs, qids, qw, ptr, ids, w, 4.0, 5)
    _, r2k = sinkhorn_wmd_sparse(vecs, qids, qw, ptr, ids, w, 4.0, 2000)
    assert np.all(r2k < 1e-10)
    assert np.all(r2k <= r5 + 1e-15)


def test_dense_equals_sparse_bitwise():
    vecs, ptr, ids, w, qids, qw = tiny(V=40, N=6, vr=3, seed=10)
    for lam, t in [(0.0, 1), (5.0, 0), (12.0, 4)]:
        d, s = both_forms(vecs, ptr, ids, w, qids, qw, lam, t, exact=True)
        assert np.array_equal(d, s), (lam, t, d - s)
        d2, s2 = both_forms(vecs, ptr, ids, w, qids, qw, lam, t)
        np.testing.assert_allclose(d2, d, rtol=1e-13)
        np.testing.assert_allclose(s2, s, rtol=1e-13)


def _converged(vecs, q, qw, doc, dw, lam, iters=4000, tol=1e-9):
    d, resid = sinkhorn_wmd_sparse(vecs, q, qw, np.array([0, len(doc)]), doc, dw, lam, iters)
    assert resid[0] < tol, resid
    return float(d[0])


@pytest.mark.parametrize("n", [2, 3, 5, 6])
@pytest.mark.parametrize("lam", [50.0, 100.0, 200.0])
def test_entropic_bound_bruteforce(n, lam):
    # low-dimensional points scaled so lambda * M stays moderate and Sinkhorn converges
    rng = np.random.default_rng(100 + n)
    vecs = (rng.uniform(0, 0.2, size=(2 * n, 2))).astype(np.float32)
    q, doc = np.arange(n, dtype=np.int32), np.arange(n, 2 * n, dtype=np.int32)
    ones = np.ones(n, np.float32)
    d = _converged(vecs, q, ones, doc, ones, lam, iters=20000)
    M = cdist64(vecs, q, doc)
    emd = emd_bruteforce_uniform(M)
    assert emd == pytest.approx(emd_assignment_uniform(M), rel=1e-12)
    assert emd - 1e-9 <= d <= emd + math.log(n) / lam + 1e-9


def test_entropic_bound_lp_general_weights():
    rng = np.random.default_rng(11)
    vecs = rng.uniform(0, 0.3, size=(12, 3)).astype(np.float32)
    q, doc = np.array([0, 1, 2, 3], np.int32), np.array([4, 5, 6, 7, 8], np.int32)
    qw = np.array([1, 2, 3, 1], np.float32)
    dw = np.array([2, 1, 1, 4, 1], np.float32)
    r = qw.astype(np.float64) / qw.sum()
    c = dw.astype(np.float64) / dw.sum()
    M = cdist64(vecs, q, doc)
    emd = emd_lp(M, r, c)
    for lam in (30.0, 60.0, 120.0):
        d = _converged(vecs, q, qw, doc, dw, lam, iters=20000)
        assert emd - 1e-9 <= d <= emd + min(entropy(r), entropy(c)) / lam + 1e-9


def test_self_distance_falls_with_lambda():
    vecs = 0.1 * synth.embeddings(30, 4, np.random.default_rng(12))
    q, qw = np.array([1, 5, 9, 20], np.int32), np.array([1, 1, 2, 1], np.float32)
    prev = np.inf
    r = qw.astype(np.float64) / qw.sum()
    for lam in (1.0, 4.0, 16.0, 64.0):
        d = _converged(vecs, q, qw, q, qw, lam, iters=40000, tol=1e-8)
        assert 0.0 <= d <= entropy(r) / lam + 1e-8
        assert d < prev
        prev = d


def test_symmetry_at_convergence():
    vecs = synth.embeddings(30, 4, np.random.default_rng(13))
    a, aw = np.array([1, 5, 9], np.int32), np.array([1, 3, 2], np.float32)
    b, bw = np.array([2, 5, 17, 28], np.int32), np.array([2, 1, 1, 1], np.float32)
    ab = _converged(vecs, a, aw, b, bw, 6.0)
    ba = _converged(vecs, b, bw, a, aw, 6.0)
    assert ab == pytest.approx(ba, rel=1e-10)


def test_zero_weight_query_words_are_dropped():
    vecs, ptr, ids, w, qids, qw = tiny(seed=14)
    qz = np.concatenate([qids, [59]]).astype(np.int32)
    wz = np.concatenate([qw, [0.0]]).astype(np.float32)
    if 59 in qids:
        pytest.skip("id collision")
    a, _ = sinkhorn_wmd_sparse(vecs, qids, qw, ptr, ids, w, 10.0, 15)
    b, _ = sinkhorn_wmd_sparse(vecs, qz, wz, ptr, ids, w, 10.0, 15)
    assert np.array_equal(a, b)


def test_input_errors():
    vecs, ptr, ids, w, qids, qw = tiny(seed=15)
    with pytest.raises(ValueError):
        query_histogram(np.array([1, 1]), np.array([1.0, 1.0]))
    with pytest.raises(ValueError):
        query_histogram(np.array([1, 2]), np.array([0.0, 0.0]))
    with pytest.raises(ValueError):
        sinkhorn_wmd_sparse(vecs, qids, qw, ptr, ids, w, -1.0, 3)
    with pytest.raises(ValueError):
        sinkhorn_wmd_sparse(vecs, qids, qw, ptr, ids, w, 1.0, -1)


# -- convergence check (Algorithm 1 iterates while x still changes; rho = row-marginal residual)

def _adaptive_case():
    rng = np.random.default_rng(31)
    vecs = synth.embeddings(60, 8, rng)
    ptr, ids, w = synth.corpus(60, 7, (1, 9), rng)
    q, qw = synth.query(60, 5, rng, "uniform")
    return vecs, q, qw, ptr, ids, w


def test_rho_is_residual_of_previous_plan():
    vecs, q, qw, ptr, ids, w = _adaptive_case()
    _, _, t, hist = sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, 6.0, 10, return_history=True)
    assert np.all(t == 10)
    for tt in range(1, 11):
        prev = sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, 6.0, tt - 1)[1]
        np.testing.assert_allclose([h[tt - 1] for h in hist], prev, rtol=1e-10, atol=1e-16)


def test_adaptive_stops_at_first_small_rho_and_matches_fixed_counts():
    vecs, q, qw, ptr, ids, w = _adaptive_case()
    tol = 2e-3
    d, res, t, hist = sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, 6.0, 40, tol=tol, return_history=True)
    for j, h in enumerate(hist):
        assert len(h) == t[j]
        assert all(v > tol for v in h[:-1])
        assert h[-1] <= tol or t[j] == 40
    d_fix, res_fix = sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, 6.0, t)
    assert np.array_equal(d, d_fix) and np.array_equal(res, res_fix)
    # a one-word document's plan is exact after one update: rho(2) = 0
    d1, _, t1, h1 = sinkhorn_wmd_sparse(vecs, q, qw, np.array([0, 1]), np.array([7]), np.array([1.0]),
                                        6.0, 9, tol=1e-14, return_history=True)
    assert t1[0] == 2 and h1[0][1] == 0.0


def test_huge_tol_is_one_update():
    vecs, q, qw, ptr, ids, w = _adaptive_case()
    d, _, t, _ = sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, 6.0, 25, tol=1e9, return_history=True)
    assert np.all(t == 1)
    assert np.array_equal(d, sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, 6.0, 1)[0])
