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
    """Admission is byte accounting against the whole budget: a query larger
    than budget / max_inflight but within the budget runs (it waits until the
    budget has room); only a query larger than the whole budget is refused."""
    (vecs, ptr, ids, w), c = ragged
    U, N = c.info["U"], c.info["N"]
    rng = np.random.default_rng(3)

    def query(m):
        return rng.choice(vecs.shape[0], m, replace=False).astype(np.int32), np.ones(m, np.float32)

    small, mid, big = query(8), query(300), query(600)
    # K buffer: U x ldk floats per query; the budget holds K for ~400 query words
    budget = 4 * U * 400 + (1 << 16)
    with wmd.Server(c, hbm_budget_bytes=budget, max_inflight=2, max_batch=32) as s:
        with pytest.raises(wmd.WmdError) as e:
            s.submit(*big, 10.0, 5)
        assert e.value.code == wmd.WMD_ENOMEM
        # mid needs more than half of the budget: it cannot share it with a
        # second mid, but runs
        tickets = [s.submit(*small, 10.0, 5) for _ in range(10)] + [s.submit(*mid, 10.0, 5) for _ in range(3)] + \
                  [s.submit(*small, 10.0, 5) for _ in range(10)]
        ref_small = c.query(*small, 10.0, 5)[0]
        ref_mid = c.query(*mid, 10.0, 5)[0]
        for i, t in enumerate(tickets):
            np.testing.assert_array_equal(s.wait(t)[0], ref_mid if 10 <= i < 13 else ref_small)
        st = s.stats()
        assert st["completed"] == len(tickets)
        assert st["workspace_bytes"] <= budget
    assert 4 * U * 300 > budget // 2


def test_concurrent_submit_and_wait(ragged, wmd):
    """Several threads submit and wait at once (the ticket table grows while
    others wait on it); every result equals the single call."""
    import threading
    (vecs, ptr, ids, w), c = ragged
    qs = mixed_queries(vecs.shape[0], 24, seed=77, hi=60)
    refs = [c.query(q, qw, 10.0, 6)[0] for q, qw in qs]
    errors = []
    with wmd.Server(c, max_inflight=3, max_batch=4) as s:
        def worker(k):
            try:
                for rep in range(6):
                    mine = [(i, s.submit(*qs[i], 10.0, 6)) for i in range(k, len(qs), 4)]
                    for i, t in mine:
                        np.testing.assert_array_equal(s.wait(t)[0], refs[i])
            except Exception as ex:   # reported by the main thread
                errors.append(ex)

        # tickets submitted here are collected by another thread
        shared = [s.submit(*qs[i], 10.0, 6) for i in range(len(qs))]

        def collector():
            try:
                for i, t in enumerate(shared):
                    np.testing.assert_array_equal(s.wait(t)[0], refs[i])
            except Exception as ex:
                errors.append(ex)

        ths = [threading.Thread(target=worker, args=(k,)) for k in range(4)] + [threading.Thread(target=collector)]
        for th in ths:
            th.start()
        for th in ths:
            th.join()
        st = s.stats()
    assert not errors, errors[:3]
    assert st["completed"] == st["submitted"] == len(qs) * 7


def test_one_waiter_per_ticket(ragged, wmd):
    """A second wait on a ticket that already has a waiter is refused; the
    first waiter still gets the result; stats reset forgets the warm-up."""
    import threading
    import time
    (vecs, ptr, ids, w), c = ragged
    q = np.arange(7, dtype=np.int32)
    qw = np.ones(7, np.float32)
    ref = c.query(q, qw, 10.0, 4)[0]
    got = {}
    # a lone query waits up to batch_wait_us for company, so it is still pending below
    with wmd.Server(c, batch_wait_us=400_000, max_batch=8) as s:
        t = s.submit(q, qw, 10.0, 4)
        th = threading.Thread(target=lambda: got.setdefault("d", s.wait(t)[0]))
        th.start()
        time.sleep(0.1)
        with pytest.raises(wmd.WmdError) as e:
            s.wait(t, timeout_us=0)
        assert e.value.code == wmd.WMD_EINVAL
        th.join()
        np.testing.assert_array_equal(got["d"], ref)
        assert s.stats()["completed"] == 1
        s.reset_stats()
        st = s.stats()
        assert st["completed"] == st["submitted"] == 0 and st["latency_p50_ms"] == 0.0
        t2 = s.submit(q, qw, 10.0, 4)
        np.testing.assert_array_equal(s.wait(t2)[0], ref)
        assert s.stats()["completed"] == 1


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


# ---- step mode (iteration-level batching) ----

@pytest.mark.parametrize("step_iters,max_batch,words", [(1, 1, 0), (4, 6, 0), (7, 16, 0), (5, 16, 120)])
def test_step_mode_equals_single_bitwise(ragged, wmd, step_iters, max_batch, words):
    """Queries that join and leave between steps, each at its own iteration
    count (lambdas on both sides of the K .* M switch, 0 iterations, counts
    that are and are not multiples of the step), give wmd_query's results bit
    for bit, residuals included."""
    (vecs, ptr, ids, w), c = ragged
    qs = mixed_queries(vecs.shape[0], 30, seed=100 + step_iters, hi=260)
    params = [(10.0, 12), (0.25, 5), (50.0, 0), (1.0, 9), (10.0, 1), (3.0, 14)] * 5
    with wmd.Server(c, step_iters=step_iters, max_batch=max_batch, want_resid=True, max_batch_words=words) as s:
        tickets = [s.submit(q, qw, lam, t) for (q, qw), (lam, t) in zip(qs, params)]
        served = [s.wait(t) for t in tickets]
        st = s.stats()
    assert st["submitted"] == st["completed"] == len(qs)
    assert 0 < st["mean_batch"] <= max_batch
    for (q, qw), (lam, t), (d, r) in zip(qs, params, served):
        d1, r1 = c.query(q, qw, lam, t, resid=True)
        np.testing.assert_array_equal(d, d1)
        np.testing.assert_array_equal(r, r1)
    q, qw = qs[0]
    want, _ = sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, 10.0, 12)
    assert rel_err(served[0][0], want).max() <= FP32_RTOL


def test_step_mode_log_domain(ragged, wmd):
    """Column-shifted K (each query's row minima in its own region) at a large
    lambda, stepped: equal to the single call."""
    (vecs, ptr, ids, w), c = ragged
    qs = mixed_queries(vecs.shape[0], 10, seed=41, hi=120)
    with wmd.Server(c, step_iters=3, max_batch=5, log_domain=True) as s:
        tickets = [s.submit(q, qw, 200.0, 8) for q, qw in qs]
        for (q, qw), t in zip(qs, tickets):
            np.testing.assert_array_equal(s.wait(t)[0], c.query(q, qw, 200.0, 8, log_domain=True)[0])


def test_step_mode_short_query_overtakes_long(ragged, wmd):
    """A short query admitted beside a long one finishes while the long one is
    still iterating (it does not wait for the long query's batch)."""
    (vecs, ptr, ids, w), c = ragged
    rng = np.random.default_rng(8)
    ql = rng.choice(vecs.shape[0], 200, replace=False).astype(np.int32)
    qs = rng.choice(vecs.shape[0], 6, replace=False).astype(np.int32)
    ones = lambda q: np.ones(q.size, np.float32)
    with wmd.Server(c, step_iters=4, max_batch=4) as s:
        t_long = s.submit(ql, ones(ql), 10.0, 20000)
        t_short = s.submit(qs, ones(qs), 10.0, 3)
        np.testing.assert_array_equal(s.wait(t_short)[0], c.query(qs, ones(qs), 10.0, 3)[0])
        with pytest.raises(wmd.WmdError) as e:
            s.wait(t_long, timeout_us=0)
        assert e.value.code == wmd.WMD_ETIMEDOUT
        np.testing.assert_array_equal(s.wait(t_long)[0], c.query(ql, ones(ql), 10.0, 20000)[0])


def test_step_mode_budget_and_options(ragged, wmd):
    (vecs, ptr, ids, w), c = ragged
    U, N = c.info["U"], c.info["N"]
    rng = np.random.default_rng(4)

    def query(m):
        return rng.choice(vecs.shape[0], m, replace=False).astype(np.int32), np.ones(m, np.float32)

    # a query's region: K block (U x ldk) + x (N x ldk) + results; the budget
    # holds regions for about 300 query words in flight
    budget = 4 * (U + N) * 300 + (1 << 16)
    small, mid, big = query(8), query(200), query(700)
    with wmd.Server(c, step_iters=4, hbm_budget_bytes=budget, max_batch=8) as s:
        with pytest.raises(wmd.WmdError) as e:
            s.submit(*big, 10.0, 5)
        assert e.value.code == wmd.WMD_ENOMEM
        tickets = [s.submit(*mid, 10.0, 9) for _ in range(3)] + [s.submit(*small, 10.0, 9) for _ in range(6)]
        ref_mid, ref_small = c.query(*mid, 10.0, 9)[0], c.query(*small, 10.0, 9)[0]
        for i, t in enumerate(tickets):
            np.testing.assert_array_equal(s.wait(t)[0], ref_mid if i < 3 else ref_small)
        assert s.stats()["completed"] == len(tickets)
    for kw in ({"step_iters": -1}, {"step_iters": 2, "tol": 1e-3}, {"step_iters": 2, "lse": True},
               {"step_iters": 2, "iters_per_launch": 3}):
        with pytest.raises(wmd.WmdError) as e:
            wmd.Server(c, **kw)
        assert e.value.code == wmd.WMD_EINVAL, kw
