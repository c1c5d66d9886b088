"""On-device k-nearest-document retrieval through the C ABI.

The selection is exact integer/ordering work on the GPU's own distances: the
returned (index, distance) list must equal the oracle's knn applied to the
GPU's full distance vector, bit for bit.  Against the FP64 oracle's distances,
the i-th smallest distance is 1-Lipschitz in the per-document errors, so the
sorted values must agree rank by rank within the FP32 bar.
"""
import numpy as np
import pytest

from oracle import knn, sinkhorn_wmd_sparse
from paper_2005_06727_amd import synth
from tests.test_gpu_parity import FP32_RTOL, ragged_corpus

pytestmark = pytest.mark.gpu


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
    vecs, ptr, ids, w = ragged_corpus(seed=44)
    c = wmd.Corpus(vecs, ptr, ids, w, device=0)
    yield (vecs, ptr, ids, w), c
    c.close()


@pytest.mark.parametrize("m,k", [(5, 1), (26, 10), (26, 260), (90, 37), (300, 100)])
def test_topk_equals_selection_of_full_vector(ragged, wmd, m, k):
    (vecs, ptr, ids, w), c = ragged
    rng = np.random.default_rng(m + k)
    q = rng.choice(vecs.shape[0], m, replace=False).astype(np.int32)
    qw = rng.random(m, dtype=np.float32) + 0.1
    full, _ = c.query(q, qw, 10.0, 15)
    idx, dist = c.topk(q, qw, 10.0, 15, k)
    want_idx, want_dist = knn(full, k)
    np.testing.assert_array_equal(idx, want_idx)
    np.testing.assert_array_equal(dist, want_dist)
    # rank-wise against the FP64 oracle
    ref, _ = sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, 10.0, 15)
    _, ref_sorted = knn(ref, k)
    assert np.all(np.abs(dist - ref_sorted) <= FP32_RTOL * ref_sorted)


def test_ties_break_by_index(wmd):
    # identical documents give bitwise identical distances
    rng = np.random.default_rng(5)
    vecs = synth.embeddings(300, 32, rng)
    base = [np.array([3, 17, 40], np.int32), np.array([5, 6], np.int32), np.array([100, 7, 8, 9], np.int32)]
    docs = [base[i % 3] for i in range(30)]
    ptr = np.zeros(31, np.int64)
    ptr[1:] = np.cumsum([len(d) for d in docs])
    ids = np.concatenate(docs)
    wts = np.ones(ids.size, np.float32)
    with wmd.Corpus(vecs, ptr, ids, wts, device=0) as c:
        q, qw = np.array([3, 5, 200], np.int32), np.array([1, 2, 1], np.float32)
        full, _ = c.query(q, qw, 10.0, 15)
        assert len(np.unique(full)) == 3
        idx, dist = c.topk(q, qw, 10.0, 15, 30)
        np.testing.assert_array_equal(idx, knn(full, 30)[0])
        first = np.argmin([full[0], full[1], full[2]])
        assert list(idx[:10]) == [first + 3 * i for i in range(10)]


def test_several_selection_passes(wmd):
    # N = 20000 and k = 2048 need four passes of 4096-key tiles
    rng = np.random.default_rng(9)
    vecs, ptr, ids, w = ragged_corpus(V=2000, dim=64, N=20000, seed=9, max_len=30)
    with wmd.Corpus(vecs, ptr, ids, w, device=0) as c:
        q = rng.choice(2000, 12, replace=False).astype(np.int32)
        qw = np.ones(12, np.float32)
        full, _ = c.query(q, qw, 10.0, 5)
        for k in (2048, 1500, 1000):
            idx, dist = c.topk(q, qw, 10.0, 5, k)
            want_idx, want_dist = knn(full, k)
            np.testing.assert_array_equal(idx, want_idx)
            np.testing.assert_array_equal(dist, want_dist)


def test_async_equals_sync(ragged, wmd):
    import torch
    (vecs, ptr, ids, w), c = ragged
    q = np.array([1, 2, 3, 50, 60], np.int32)
    qw = np.ones(5, np.float32)
    idx, dist = c.topk(q, qw, 10.0, 15, 25)
    s = torch.cuda.Stream()
    di = torch.empty(25, dtype=torch.int32, device="cuda")
    dd = torch.empty(25, dtype=torch.float64, device="cuda")
    wmd.wmd_query_topk_async(c.handle, q, qw, 10.0, 15, 25, di, dd, s)
    s.synchronize()
    np.testing.assert_array_equal(di.cpu().numpy(), idx)
    np.testing.assert_array_equal(dd.cpu().numpy(), dist)


def test_topk_errors(ragged, wmd):
    (vecs, ptr, ids, w), c = ragged
    q, qw = np.array([1, 2], np.int32), np.ones(2, np.float32)
    for k in (0, -1, c.info["N"] + 1, wmd.WMD_MAX_TOPK + 1):
        with pytest.raises(wmd.WmdError) as e:
            c.topk(q, qw, 10.0, 5, k)
        assert e.value.code == wmd.WMD_EINVAL


def test_ties_across_tiles_and_passes(wmd):
    # 20 000 documents repeating 3 contents: one distance value covers ~6 700
    # documents, so the first k are all tied and must be the k smallest indices
    # of that value, across several tiles and a second selection pass
    rng = np.random.default_rng(12)
    vecs = synth.embeddings(400, 32, rng)
    base = [np.array([3, 17, 40], np.int32), np.array([5, 6], np.int32), np.array([100, 7, 8, 9], np.int32)]
    N = 20000
    docs = [base[(i * 7) % 3] for i in range(N)]
    ptr = np.zeros(N + 1, np.int64)
    ptr[1:] = np.cumsum([len(d) for d in docs])
    ids = np.concatenate(docs)
    wts = np.ones(ids.size, np.float32)
    with wmd.Corpus(vecs, ptr, ids, wts, device=0) as c:
        q, qw = np.array([3, 5, 200], np.int32), np.array([1, 2, 1], np.float32)
        full, _ = c.query(q, qw, 10.0, 15)
        assert len(np.unique(full)) == 3
        for k in (1000, 2048, 7):
            idx, dist = c.topk(q, qw, 10.0, 15, k)
            want_idx, want_dist = knn(full, k)
            np.testing.assert_array_equal(idx, want_idx)
            np.testing.assert_array_equal(dist, want_dist)
