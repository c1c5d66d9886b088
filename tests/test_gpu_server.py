"""Continuous-batching server through the C ABI: every served result equals
the single-query result bitwise (and the oracle to the FP32 bar), admission
respects the device budget, and the statistics add up."""
import numpy as np
import pytest

from oracle import sinkhorn_wmd_sparse
from paper_2005_06727_amd import synth
from tests.test_gpu_parity import FP32_RTOL, ragged_corpus, rel_err

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
    vecs, ptr, ids, w = ragged_corpus(seed=33)
    c = wmd.Corpus(vecs, ptr, ids, w, device=0)
    yield (vecs, ptr, ids, w), c
    c.close()


def mixed_queries(V, n, seed, lo=1, hi=300):
    rng = np.random.default_rng(seed)
    lens = synth.loguniform_lengths(n, lo, hi, rng)
    out = []
    for m in lens:
        q = rng.choice(V, int(m), replace=False).astype(np.int32)
        out.append((q, rng.random(int(m), dtype=np.float32) + 0.05))
    return out


@pytest.mark.parametrize("max_inflight,max_batch,words", [(1, 1, 0), (2, 8, 0), (4, 16, 0), (2, 16, 100)])
def test_served_equals_single_bitwise(ragged, wmd, max_inflight, max_batch, words):
    (vecs, ptr, ids, w), c = ragged
    qs = mixed_queries(vecs.shape[0], 40, seed=max_batch + words)
    lam, iters = 10.0, 12
    with wmd.Server(c, max_inflight=max_inflight, max_batch=max_batch, want_resid=True,
                    max_batch_words=words) as s:
        tickets = [s.submit(q, qw, lam, iters) for q, qw in qs]
        served = [s.wait(t) for t in tickets]
        st = s.stats()
    assert st["submitted"] == st["completed"] == len(qs)
    assert 1 <= st["batches"] <= len(qs)
    assert st["mean_batch"] <= max_batch
    assert 0 < st["latency_p50_ms"] <= st["latency_p99_ms"] <= st["latency_max_ms"]
    for (q, qw), (d, r) in zip(qs, served):
        d1, r1 = c.query(q, qw, lam, iters, resid=True)
        np.testing.assert_array_equal(d, d1)
        np.testing.assert_array_equal(r, r1)
    # and the oracle, for a short and a long query
    for k in (int(np.argmin([len(q) for q, _ in qs])), int(np.argmax([len(q) for q, _ in qs]))):
        q, qw = qs[k]
        want, _ = sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, lam, iters)
        assert rel_err(served[k][0], want).max() <= FP32_RTOL


def test_mixed_lambda_and_iters(ragged, wmd):
    (vecs, ptr, ids, w), c = ragged
    qs = mixed_queries(vecs.shape[0], 12, seed=5, hi=80)
    params = [(0.0, 3), (1.0, 0), (10.0, 7), (0.25, 5), (50.0, 20), (5.0, 1)] * 2
    with wmd.Server(c, max_batch=6, max_inflight=2) as s:
        tickets = [s.submit(q, qw, lam, t) for (q, qw), (lam, t) in zip(qs, params)]
        for (q, qw), (lam, t), tk in zip(qs, params, tickets):
            d, _ = s.wait(tk)
            np.testing.assert_array_equal(d, c.query(q, qw, lam, t)[0])


def test_budget_admission(ragged, wmd):
    (vecs, ptr, ids, w), c = ragged
    U = c.info["U"]
    rng = np.random.default_rng(3)
    small = (rng.choice(vecs.shape[0], 8, replace=False).astype(np.int32), np.ones(8, np.float32))
    big = (rng.choice(vecs.shape[0], 600, replace=False).astype(np.int32), np.ones(600, np.float32))
    # a share that holds K for ~64 query words but not 600
    budget = 2 * (4 * U * 64 + (1 << 20))
    with wmd.Server(c, hbm_budget_bytes=budget, max_inflight=2, max_batch=32) as s:
        with pytest.raises(wmd.WmdError) as e:
            s.submit(*big, 10.0, 5)
        assert e.value.code == wmd.WMD_ENOMEM
        tickets = [s.submit(*small, 10.0, 5) for _ in range(20)]
        ref = c.query(*small, 10.0, 5)[0]
        for t in tickets:
            np.testing.assert_array_equal(s.wait(t)[0], ref)
        assert s.stats()["workspace_bytes"] <= budget


def test_ticket_errors_and_options(ragged, wmd):
    (vecs, ptr, ids, w), c = ragged
    for kw in ({"max_inflight": 0}, {"max_inflight": 17}, {"max_batch": 0}, {"hbm_budget_bytes": 0},
               {"batch_wait_us": -1}, {"max_batch_words": -1}, {"tile": 3}, {"precision": wmd.WMD_DIST_BF16}):
        with pytest.raises(wmd.WmdError) as e:
            wmd.Server(c, **kw)
        assert e.value.code == wmd.WMD_EINVAL, kw
    q = np.arange(5, dtype=np.int32)
    with wmd.Server(c, batch_wait_us=2000) as s:
        with pytest.raises(wmd.WmdError) as e:
            s.wait(12345)
        assert e.value.code == wmd.WMD_ENOTFOUND
        with pytest.raises(wmd.WmdError) as e:
            s.submit(q, -np.ones(5, np.float32), 1.0, 3)
        assert e.value.code == wmd.WMD_EINVAL
        t = s.submit(q, np.ones(5, np.float32), 1.0, 3)
        d, _ = s.wait(t)
        np.testing.assert_array_equal(d, c.query(q, np.ones(5, np.float32), 1.0, 3)[0])
        with pytest.raises(wmd.WmdError) as e:
            s.wait(t)
        assert e.value.code == wmd.WMD_ENOTFOUND


def test_destroy_drains_pending(ragged, wmd):
    (vecs, ptr, ids, w), c = ragged
    qs = mixed_queries(vecs.shape[0], 30, seed=9, hi=200)
    s = wmd.Server(c, max_batch=4, max_inflight=2)
    for q, qw in qs:
        s.submit(q, qw, 10.0, 10)
    s.close()   # returns once every queued query ran; results are dropped
    # the corpus is still usable afterwards
    q, qw = qs[0]
    want, _ = sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, 10.0, 10)
    assert rel_err(c.query(q, qw, 10.0, 10)[0], want).max() <= FP32_RTOL
