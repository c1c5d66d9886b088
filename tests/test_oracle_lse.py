"""Pins of the log-domain oracle (oracle/sinkhorn_lse.py).

None of them re-types its arithmetic: it must equal the plain oracle wherever
that one does not underflow, reproduce closed forms and the shift identity far
beyond the exponent range, keep the column marginals exact, and land inside
the entropic bound around the exact earth mover's distance at large lambda.
A few planted mistakes in a copy of the module must each trip the battery.
"""
import math
import os
import types

import numpy as np
import pytest
from scipy.spatial.distance import cdist

from oracle import sinkhorn_lse_core, sinkhorn_wmd_lse, sinkhorn_wmd_sparse
from paper_2005_06727_amd import synth
from tests.emd_exact import emd_assignment_uniform, emd_lp


def _case(seed=0, V=60, dim=8, N=7, q=5):
    rng = np.random.default_rng(seed)
    vecs = synth.embeddings(V, dim, rng)
    ptr, ids, w = synth.corpus(V, N, (1, 6), rng)
    qq, qw = synth.query(V, q, rng, "uniform")
    return vecs, qq, qw, ptr, ids, w


def _d64(vecs, a, b):
    E = np.asarray(vecs, np.float32).astype(np.float64)
    return cdist(E[np.asarray(a)], E[np.asarray(b)])


@pytest.mark.parametrize("lam", [0.0, 1.0, 10.0, 50.0])
@pytest.mark.parametrize("t", [0, 1, 5, 20])
def test_equals_plain_oracle_in_range(lam, t):
    vecs, q, qw, ptr, ids, w = _case()
    d, res = sinkhorn_wmd_lse(vecs, q, qw, ptr, ids, w, lam, t)
    d0, res0 = sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, lam, t)
    np.testing.assert_allclose(d, d0, rtol=1e-12)
    np.testing.assert_allclose(res, res0, rtol=1e-9, atol=1e-13)


def test_plain_form_breaks_down_where_log_domain_holds():
    vecs, q, qw, ptr, ids, w = _case()
    with np.errstate(all="ignore"):
        d0, _ = sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, 2000.0, 5)
    assert not np.all(np.isfinite(d0))          # K underflows to 0 in FP64
    d, res = sinkhorn_wmd_lse(vecs, q, qw, ptr, ids, w, 2000.0, 5)
    assert np.all(np.isfinite(d)) and np.all(np.isfinite(res))


@pytest.mark.parametrize("t", [0, 3])
def test_one_word_query_beyond_range(t):
    # v_r = 1: the plan is c itself, WMD = sum_i c_i M[0, i] for any lambda, t
    vecs, _, _, ptr, ids, w = _case(1)
    q, qw = np.array([11], np.int32), np.array([3.0], np.float32)
    d, res = sinkhorn_wmd_lse(vecs, q, qw, ptr, ids, w, 3000.0, t)
    for j in range(ptr.size - 1):
        c = w[ptr[j]:ptr[j + 1]].astype(np.float64)
        want = float(_d64(vecs, q, ids[ptr[j]:ptr[j + 1]])[0] @ (c / c.sum()))
        assert math.isclose(d[j], want, rel_tol=1e-12)
    assert np.all(res < 1e-12)


def test_one_word_document_beyond_range():
    # n_j = 1: the plan is r itself after one update, WMD = sum_k r_k M[k, i]
    vecs, q, qw, _, _, _ = _case(2)
    ptr = np.array([0, 1, 2])
    ids = np.array([4, 9], np.int32)
    w = np.array([2.0, 0.5], np.float32)
    r = qw.astype(np.float64) / qw.astype(np.float64).sum()
    for t in (1, 4):
        d, res = sinkhorn_wmd_lse(vecs, q, qw, ptr, ids, w, 3000.0, t)
        for j, word in enumerate(ids):
            assert math.isclose(d[j], float(r @ _d64(vecs, q, [word])[:, 0]), rel_tol=1e-12)
        assert np.all(res < 1e-12)


def test_column_marginals_exact_beyond_range():
    vecs, q, qw, ptr, ids, w = _case(3)
    _, _, plans = sinkhorn_wmd_lse(vecs, q, qw, ptr, ids, w, 1500.0, 7, return_plans=True)
    for j, P in enumerate(plans):
        c = w[ptr[j]:ptr[j + 1]].astype(np.float64)
        np.testing.assert_allclose(P.sum(axis=0), c / c.sum(), rtol=1e-12)


def test_shift_identity_far_beyond_range():
    # M + delta rescales K by exp(-lambda delta), which v absorbs: the plan is
    # unchanged and WMD grows by exactly delta (the plan has mass one)
    vecs, q, qw, ptr, ids, w = _case(4)
    M = _d64(vecs, q, ids)
    r = qw.astype(np.float64) / qw.astype(np.float64).sum()
    c = np.concatenate([w[ptr[j]:ptr[j + 1]].astype(np.float64) / w[ptr[j]:ptr[j + 1]].astype(np.float64).sum()
                        for j in range(ptr.size - 1)])
    lam, delta = 40.0, 125.0                      # lambda * delta = 5000
    d, res = sinkhorn_lse_core(M, r, c, ptr, lam, 9)
    d2, res2 = sinkhorn_lse_core(M + delta, r, c, ptr, lam, 9)
    np.testing.assert_allclose(d2, d + delta, rtol=1e-12)
    np.testing.assert_allclose(res2, res, rtol=1e-6, atol=1e-12)


def _pairs(n, jitter, rng):
    """n points on a line and n partners near them (each is closest to its own)."""
    a = np.stack([np.arange(n) / n, np.zeros(n)], 1)
    b = a + np.array([0.03, 0.02])
    if jitter:
        b = b + rng.uniform(-0.01, 0.01, size=b.shape)
    return np.concatenate([a, b]).astype(np.float32), np.arange(n, dtype=np.int32), np.arange(n, 2 * n, dtype=np.int32)


@pytest.mark.parametrize("lam", [300.0, 1000.0, 3000.0])
def test_entropic_bound_at_large_lambda_uniform(lam):
    # at convergence EMD <= d <= EMD + min(H(r), H(c)) / lambda; uniform
    # weights: EMD by the assignment problem (Birkhoff-von Neumann)
    pts, a, b = _pairs(5, True, np.random.default_rng(7))
    ones = np.ones(5, np.float32)
    d, res = sinkhorn_wmd_lse(pts, a, ones, np.array([0, 5]), b, ones, lam, 200)
    assert res[0] < 1e-9
    emd = emd_assignment_uniform(_d64(pts, a, b))
    assert emd - 1e-9 <= d[0] <= emd + math.log(5) / lam + 1e-9


@pytest.mark.parametrize("lam", [300.0, 1000.0])
def test_entropic_bound_at_large_lambda_general_weights(lam):
    # general weights against the transportation LP (HiGHS); the seed is one
    # whose iteration converges within the budget at both lambdas (at very
    # large lambda, terms more than ~745 below a sum's largest underflow and
    # some weightings stall short of the marginals; convergence is asserted)
    rng = np.random.default_rng(9)
    pts, a, b = _pairs(5, False, rng)
    wa = rng.uniform(0.5, 2, 5).astype(np.float32)
    wb = rng.uniform(0.5, 2, 5).astype(np.float32)
    d, res = sinkhorn_wmd_lse(pts, a, wa, np.array([0, 5]), b, wb, lam, 6000)
    assert res[0] < 1e-9
    ra = wa.astype(np.float64) / wa.astype(np.float64).sum()
    cb = wb.astype(np.float64) / wb.astype(np.float64).sum()
    H = min(-(ra * np.log(ra)).sum(), -(cb * np.log(cb)).sum())
    emd = emd_lp(_d64(pts, a, b), ra, cb)
    assert emd - 1e-9 <= d[0] <= emd + H / lam + 1e-9


def test_errors():
    vecs, q, qw, ptr, ids, w = _case()
    with pytest.raises(ValueError):
        sinkhorn_wmd_lse(vecs, q, qw, ptr, ids, w, -1.0, 3)
    with pytest.raises(ValueError):
        sinkhorn_wmd_lse(vecs, q, qw, ptr, ids, w, 1.0, -1)


# -- planted mistakes -------------------------------------------------------

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "sinkhorn_lse.py")


def _load(replace=None):
    text = open(SRC).read()
    if replace is not None:
        old, new = replace
        assert text.count(old) == 1, old
        text = text.replace(old, new)
    text = text.replace("from .sinkhorn_wmd import", "from oracle.sinkhorn_wmd import")
    mod = types.ModuleType("lse_mutant")
    exec(compile(text, "lse_mutant", "exec"), mod.__dict__)
    return mod


def _battery(o) -> bool:
    vecs, q, qw, ptr, ids, w = _case()
    ok = True
    with np.errstate(all="ignore"):
        try:
            d = o.sinkhorn_wmd_lse(vecs, q, qw, ptr, ids, w, 10.0, 5)[0]
            ok &= bool(np.allclose(d, sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, 10.0, 5)[0], rtol=1e-12))
            q1, w1 = np.array([11], np.int32), np.array([3.0], np.float32)
            d = o.sinkhorn_wmd_lse(vecs, q1, w1, ptr, ids, w, 3000.0, 3)[0]
            for j in range(ptr.size - 1):
                c = w[ptr[j]:ptr[j + 1]].astype(np.float64)
                ok &= math.isclose(d[j], float(_d64(vecs, q1, ids[ptr[j]:ptr[j + 1]])[0] @ (c / c.sum())),
                                   rel_tol=1e-12)
            pd, idd, wd = np.array([0, 1, 2]), np.array([4, 9], np.int32), np.array([2.0, 0.5], np.float32)
            d = o.sinkhorn_wmd_lse(vecs, q, qw, pd, idd, wd, 3000.0, 2)[0]
            r = qw.astype(np.float64) / qw.astype(np.float64).sum()
            for j, word in enumerate(idd):
                ok &= math.isclose(d[j], float(r @ _d64(vecs, q, [word])[:, 0]), rel_tol=1e-12)
            M = _d64(vecs, q, ids)
            c = np.concatenate([w[ptr[j]:ptr[j + 1]].astype(np.float64) / w[ptr[j]:ptr[j + 1]].astype(np.float64).sum()
                                for j in range(ptr.size - 1)])
            d1 = o.sinkhorn_lse_core(M, r, c, ptr, 40.0, 9)[0]
            d2 = o.sinkhorn_lse_core(M + 125.0, r, c, ptr, 40.0, 9)[0]
            ok &= bool(np.allclose(d2, d1 + 125.0, rtol=1e-12))
        except (ValueError, FloatingPointError, IndexError, TypeError):
            return False
    return bool(ok)


MUTANTS = {
    "no_max_shift_rows": ("    m = A.max(axis=0)\n", "    m = 0.0 * A.max(axis=0)\n"),
    "no_max_shift_segments": ("    m = np.maximum.reduceat(B, ptr[:-1], axis=1)\n",
                              "    m = 0.0 * np.maximum.reduceat(B, ptr[:-1], axis=1)\n"),
    "kernel_sign": ("lKg = -lam * Mg", "lKg = lam * Mg"),
    "r_dropped": ("lx = _lse_segments(lKg + lv[None, :], ptr) - log_r[:, None]",
                  "lx = _lse_segments(lKg + lv[None, :], ptr)"),
    "c_dropped": ("return log_c - _lse_rows(lKg + lu[:, doc_of])", "return -_lse_rows(lKg + lu[:, doc_of])"),
    "stale_final_v": ("    lu = -lx\n    lv = lv_of(lu)\n", "    lu = -lx\n    lv = lv_of(-lx * 0.5)\n"),
    "u_not_inverted": ("        lv = lv_of(-lx)\n", "        lv = lv_of(lx)\n"),
}


def test_battery_passes_on_the_oracle():
    assert _battery(_load())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name):
    assert not _battery(_load(MUTANTS[name])), name
