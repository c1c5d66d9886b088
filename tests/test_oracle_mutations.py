"""Planted mistakes in a copy of the oracle must each trip at least one pin.

Each mutant is the oracle's source with one plausible slip (a dropped term, a
wrong sign, r on the wrong side, an off-by-one iteration count...), executed
on the CPU as a throw-away module.  The battery below restates the closed-form
pins of test_oracle_pins against a module argument.
"""
import math
import os
import types

import numpy as np
import pytest
from scipy.spatial.distance import cdist

from paper_2005_06727_amd import synth
from tests.emd_exact import emd_bruteforce_uniform

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "sinkhorn_wmd.py")


def load(replace=None):
    text = open(SRC).read()
    if replace is not None:
        old, new = replace
        assert text.count(old) >= 1, old
        text = text.replace(old, new)
    mod = types.ModuleType("oracle_mutant")
    exec(compile(text, "oracle_mutant", "exec"), mod.__dict__)
    return mod


def _d64(vecs, a, b):
    E = vecs.astype(np.float64)
    return cdist(E[np.asarray(a)], E[np.asarray(b)])


def battery(o) -> bool:
    """True when every pin holds for oracle module ``o``."""
    rng = np.random.default_rng(0)
    vecs = synth.embeddings(40, 6, rng)
    ptr, ids, w = synth.corpus(40, 5, (1, 5), rng)
    q, qw = synth.query(40, 4, rng, "uniform")
    r = qw.astype(np.float64) / qw.sum()
    ok = True
    try:
        ok &= np.allclose(o.word_distances(vecs, q, np.arange(40)), _d64(vecs, q, np.arange(40)),
                          rtol=1e-12)
        for form in ("dense", "sparse"):
            def run(lam, t, qq=q, qqw=qw, p=ptr, ii=ids, ww=w):
                if form == "dense":
                    C = o.dense_doc_matrix(40, p, ii, ww)
                    return o.sinkhorn_wmd_dense(vecs, qq, qqw, C, lam, t)
                return o.sinkhorn_wmd_sparse(vecs, qq, qqw, p, ii, ww, lam, t)[0]
            d0, dt0 = run(0.0, 3), run(7.0, 0)
            one_q = run(5.0, 4, qq=np.array([3], np.int32), qqw=np.array([2.0], np.float32))
            one_d = run(9.0, 2, p=np.array([0, 1, 2]), ii=np.array([4, int(q[1])], np.int32),
                        ww=np.array([1.0, 3.0], np.float32))
            for j in range(ptr.size - 1):
                words = ids[ptr[j]:ptr[j + 1]]
                c = w[ptr[j]:ptr[j + 1]].astype(np.float64)
                c /= c.sum()
                M = _d64(vecs, q, words)
                ok &= math.isclose(d0[j], r @ M @ c, rel_tol=1e-12)
                K = np.exp(-7.0 * M)
                ok &= math.isclose(dt0[j], float((c * (K * M).sum(0) / K.sum(0)).sum()),
                                   rel_tol=1e-12)
                ok &= math.isclose(one_q[j], float(_d64(vecs, [3], words)[0] @ c), rel_tol=1e-12)
            for j, word in enumerate([4, int(q[1])]):
                ok &= math.isclose(one_d[j], float(r @ _d64(vecs, q, [word])[:, 0]), rel_tol=1e-12)
        # entropic bound at convergence
        pts = np.random.default_rng(1).uniform(0, 0.2, size=(8, 2)).astype(np.float32)
        a, b = np.arange(4, dtype=np.int32), np.arange(4, 8, dtype=np.int32)
        ones = np.ones(4, np.float32)
        d, res = o.sinkhorn_wmd_sparse(pts, a, ones, np.array([0, 4]), b, ones, 60.0, 5000)
        emd = emd_bruteforce_uniform(_d64(pts, a, b))
        ok &= bool(res[0] < 1e-9) and emd - 1e-9 <= d[0] <= emd + math.log(4) / 60.0 + 1e-9
        # convergence check: rho(t) is the row-marginal residual after t - 1 updates,
        # and a document stops at the first t with rho(t) <= tol
        _, _, t, hist = o.sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, 4.0, 12, tol=1e-3,
                                              return_history=True)
        for tt in range(1, 7):
            res_prev = o.sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, 4.0, tt - 1)[1]
            for j in range(ptr.size - 1):
                if len(hist[j]) >= tt:
                    ok &= math.isclose(hist[j][tt - 1], res_prev[j], rel_tol=1e-9, abs_tol=1e-15)
        for j in range(ptr.size - 1):
            below = [i for i, v in enumerate(hist[j]) if v <= 1e-3]
            ok &= int(t[j]) == (below[0] + 1 if below else 12) and len(hist[j]) == int(t[j])
        d_ad = o.sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, 4.0, 12, tol=1e-3)[0]
        d_fix = o.sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, 4.0, np.asarray(t))[0]
        ok &= bool(np.array_equal(d_ad, d_fix))
    except (ValueError, FloatingPointError, ZeroDivisionError, IndexError, TypeError):
        return False
    return bool(ok)


MUTANTS = {
    "squared_distance": ("M[k] = np.sqrt(np.sum(diff * diff, axis=1))",
                         "M[k] = np.sum(diff * diff, axis=1)"),
    "kernel_sign": ("K = np.exp(-lam * M)", "K = np.exp(lam * M)"),
    "r_wrong_side": ("K_over_r = K / r[:, None]", "K_over_r = K * r[:, None]"),
    "wmd_drops_M_sparse": ("wmd = _colsum(u * spmm(KMg, v), exact)",
                           "wmd = _colsum(u * spmm(Kg, v), exact)"),
    "wmd_drops_u_dense": ("wmd = _colsum(u * _matmul(K * M, v, exact), exact)",
                          "wmd = _colsum(_matmul(K * M, v, exact), exact)"),
    "v_multiplies": ("v = c / sddmm(u)", "v = c * sddmm(u)"),
    "extra_iteration_dense": ("for _ in range(iters):\n        x = _matmul(",
                              "for _ in range(iters + 1):\n        x = _matmul("),
    "extra_iteration_sparse": ("t_max = np.broadcast_to(np.asarray(iters, dtype=np.int64), (N,))",
                               "t_max = np.broadcast_to(np.asarray(iters, dtype=np.int64) + 1, (N,))"),
    "rho_unweighted": ("rho = _colsum(r[:, None] * np.abs(x_new / x - 1.0), exact)",
                       "rho = _colsum(np.abs(x_new / x - 1.0), exact)"),
    "rho_absolute_change": ("rho = _colsum(r[:, None] * np.abs(x_new / x - 1.0), exact)",
                            "rho = _colsum(r[:, None] * np.abs(x_new - x), exact)"),
    "stop_one_late": ("            active = active & (rho > tol)",
                      "            active = active & (np.roll(rho, 0) > tol * 0.5)"),
    "r_not_normalised": ("return ids, w / math.fsum(w)", "return ids, w"),
    "c_not_normalised": ("c[ptr[j]:ptr[j + 1]] = seg / math.fsum(seg)",
                         "c[ptr[j]:ptr[j + 1]] = seg"),
    "transposed_gather": ("Kg, KoRg, KMg = K[:, row_of], K_over_r[:, row_of], KM[:, row_of]",
                          "Kg, KoRg, KMg = K[:, row_of], K_over_r[:, row_of], KM[:, row_of[::-1]]"),
    "no_final_step_u": ("u = 1.0 / x\n    v = c / sddmm(u)", "u = x\n    v = c / sddmm(u)"),
}


def test_unmutated_oracle_passes_battery():
    assert battery(load())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    with np.errstate(all="ignore"):
        assert not battery(load(MUTANTS[name])), name
