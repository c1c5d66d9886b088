"""Convergence-checked iteration (tol > 0) through the C ABI.

The GPU decides each document's stop in FP32 and the oracle's residuals are
FP64, so a document's iteration count is checked for validity instead of
equality: the oracle's rho at the GPU's count is at most tol, and at the
count before it above tol, both within an absolute slack that covers FP32
rounding of rho.  The distances are then compared with the oracle run for
exactly the GPU's per-document counts, at the FP32 bar.
"""
import numpy as np
import pytest

from oracle import sinkhorn_wmd_sparse
from tests.test_gpu_parity import FP32_RTOL, RESID_ATOL, RESID_RTOL, ragged_corpus, rel_err

pytestmark = pytest.mark.gpu

SLACK = 2e-6   # |rho_fp32 - rho_fp64|: a sum of r_k-weighted ratios near 1, each rounded at ~6e-8


@pytest.fixture(scope="module")
def wmd():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2005_06727_amd import wmd as w
    return w


@pytest.fixture(scope="module")
def ragged(wmd):
    vecs, ptr, ids, w = ragged_corpus(seed=55)
    c = wmd.Corpus(vecs, ptr, ids, w, device=0)
    yield (vecs, ptr, ids, w), c
    c.close()


def check_counts(t_gpu, hist, tol, max_iters):
    bad = []
    for j, (t, h) in enumerate(zip(t_gpu, hist)):
        ok = 1 <= t <= max_iters
        if ok and t < max_iters:
            ok = h[t - 1] <= tol + SLACK
        if ok and t > 1:
            ok = h[t - 2] > tol - SLACK
        if not ok:
            bad.append((j, int(t), h[:t + 1]))
    assert not bad, bad[:3]


@pytest.mark.parametrize("m,tile", [(6, -1), (26, -1), (60, -1), (120, -1), (250, -1), (450, -1),
                                    (26, -2), (12, 0), (26, 2)])
def test_adaptive_counts_and_distances(ragged, wmd, m, tile):
    (vecs, ptr, ids, w), c = ragged
    rng = np.random.default_rng(m)
    q = rng.choice(vecs.shape[0], m, replace=False).astype(np.int32)
    qw = rng.random(m, dtype=np.float32) + 0.1
    lam, max_iters, tol = 8.0, 60, 1e-3
    d, res, t = c.query_adaptive(q, qw, lam, max_iters, tol, resid=True, tile=tile)
    _, _, t_full, hist = sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, lam, max_iters, return_history=True)
    check_counts(t, hist, tol, max_iters)
    assert np.any(t < max_iters) and np.any(t > 1)
    want, wres = sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, lam, t.astype(np.int64))
    assert rel_err(d, want).max() <= FP32_RTOL
    np.testing.assert_allclose(res, wres, rtol=RESID_RTOL, atol=RESID_ATOL)


@pytest.mark.parametrize("tile", [0, 1, 2, 3, 4, 5, 6, 7, 11, 12, 13, 14, 15, 16])   # the register tiles
def test_adaptive_every_tile_shape(ragged, wmd, tile):
    # the stop decision sums rho over every lane of a team (each lane owns some
    # columns), across waves for the multi-wave shapes
    from tests.test_gpu_parity import TILE_MAX_M
    (vecs, ptr, ids, w), c = ragged
    m = TILE_MAX_M[tile]
    rng = np.random.default_rng(300 + tile)
    q = rng.choice(vecs.shape[0], m, replace=False).astype(np.int32)
    qw = rng.random(m, dtype=np.float32) + 0.1
    lam, max_iters, tol = 8.0, 40, 2e-3
    d, _, t = c.query_adaptive(q, qw, lam, max_iters, tol, tile=tile)
    _, _, _, hist = sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, lam, max_iters, return_history=True)
    check_counts(t, hist, tol, max_iters)
    want, _ = sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, lam, t.astype(np.int64))
    assert rel_err(d, want).max() <= FP32_RTOL


def test_tol_zero_is_the_fixed_iteration(ragged, wmd):
    (vecs, ptr, ids, w), c = ragged
    q, qw = np.arange(3, 40, 3, dtype=np.int32), np.ones(13, np.float32)
    d, _, t = c.query_adaptive(q, qw, 10.0, 15, 0.0)
    assert np.all(t == 15)
    np.testing.assert_array_equal(d, c.query(q, qw, 10.0, 15)[0])


def test_adaptive_is_deterministic_and_tile_independent(ragged, wmd):
    (vecs, ptr, ids, w), c = ragged
    q, qw = np.arange(5, 95, 3, dtype=np.int32), np.ones(30, np.float32)
    d1, _, t1 = c.query_adaptive(q, qw, 8.0, 50, 5e-4)
    d2, _, t2 = c.query_adaptive(q, qw, 8.0, 50, 5e-4)
    np.testing.assert_array_equal(d1, d2)
    np.testing.assert_array_equal(t1, t2)
    d3, _, t3 = c.query_adaptive(q, qw, 8.0, 50, 5e-4, tile=-2)
    # counts can only differ where rho sits within rounding of tol; distances stay within the bar
    assert np.mean(t1 == t3) > 0.95
    assert rel_err(d3, d1).max() <= 2 * FP32_RTOL


def test_adaptive_errors(ragged, wmd):
    (vecs, ptr, ids, w), c = ragged
    q, qw = np.array([1, 2, 3], np.int32), np.ones(3, np.float32)
    for kw in ({"tol": -1.0}, {"tol": float("nan")}, {"tol": 1e-3, "iters_per_launch": 4}, {"tol": 1e-3, "tile": 8}):
        tol = kw.pop("tol")
        with pytest.raises(wmd.WmdError) as e:
            c.query_adaptive(q, qw, 10.0, 10, tol, **kw)
        assert e.value.code == wmd.WMD_EINVAL
