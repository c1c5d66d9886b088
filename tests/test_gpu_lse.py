"""Log-domain iteration (option lse) through the C ABI.

Against the FP64 log-domain oracle at every lambda, at the FP32 bar (the GPU
keeps the distances and potentials in FP64 and only the exponentials of
non-positive arguments in FP32); against the plain oracle where that one is in
range; closed forms beyond the range; batch == single bitwise; top-k; errors;
and the precision corpus at full size on sampled documents at lambda = 1000,
where the plain FP32 path cannot run.
"""
import numpy as np
import pytest

from oracle import knn, sinkhorn_wmd_lse, sinkhorn_wmd_sparse
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
    vecs, ptr, ids, w = ragged_corpus(seed=66)
    c = wmd.Corpus(vecs, ptr, ids, w, device=0)
    yield (vecs, ptr, ids, w), c
    c.close()


def _query(V, m, seed):
    rng = np.random.default_rng(seed)
    return rng.choice(V, m, replace=False).astype(np.int32), rng.random(m, dtype=np.float32) + 0.1


@pytest.mark.parametrize("lam", [10.0, 300.0, 3000.0])
@pytest.mark.parametrize("m", [1, 6, 26, 40, 41, 70, 300])   # 40 / 41: the register tile's bound
def test_lse_matches_log_domain_oracle(ragged, m, lam):
    (vecs, ptr, ids, w), c = ragged
    q, qw = _query(vecs.shape[0], m, m)
    d, res = c.query(q, qw, lam, 15, resid=True, lse=True)
    want, wres = sinkhorn_wmd_lse(vecs, q, qw, ptr, ids, w, lam, 15)
    e = rel_err(d, want)
    print(f"lse m={m} lambda={lam}: max rel err {e.max():.2e}")
    assert e.max() <= FP32_RTOL
    np.testing.assert_allclose(res, wres, rtol=1e-3, atol=1e-6)


@pytest.mark.parametrize("t", [0, 1, 15])
def test_lse_matches_plain_oracle_in_range(ragged, t):
    (vecs, ptr, ids, w), c = ragged
    q, qw = _query(vecs.shape[0], 20, 3)
    d, _ = c.query(q, qw, 10.0, t, lse=True)
    want, _ = sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, 10.0, t)
    assert rel_err(d, want).max() <= FP32_RTOL


def test_one_word_query_beyond_range(ragged):
    # v_r = 1: the plan is c itself at any lambda; the plain oracle at lambda = 0 gives it
    (vecs, ptr, ids, w), c = ragged
    q, qw = np.array([17], np.int32), np.array([2.0], np.float32)
    d, res = c.query(q, qw, 5000.0, 9, resid=True, lse=True)
    want, _ = sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, 0.0, 1)
    assert rel_err(d, want).max() <= FP32_RTOL
    assert np.all(res <= 1e-6)


def test_batch_equals_single_bitwise(ragged, wmd):
    (vecs, ptr, ids, w), c = ragged
    qs = [_query(vecs.shape[0], m, 40 + m) for m in (4, 30, 90, 1)]
    lams = np.array([800.0, 50.0, 2000.0, 10.0], np.float32)
    its = np.array([0, 15, 3, 7], np.int32)
    out, res = c.query_batch(qs, lams, its, resid=True, lse=True)
    for b, (q, qw) in enumerate(qs):
        one, r1 = c.query(q, qw, float(lams[b]), int(its[b]), resid=True, lse=True)
        np.testing.assert_array_equal(out[b], one)
        np.testing.assert_array_equal(res[b], r1)


def test_topk_with_lse(ragged):
    (vecs, ptr, ids, w), c = ragged
    q, qw = _query(vecs.shape[0], 12, 5)
    full, _ = c.query(q, qw, 1500.0, 15, lse=True)
    idx, dist = c.topk(q, qw, 1500.0, 15, 40, lse=True)
    want_idx, want_dist = knn(full, 40)
    np.testing.assert_array_equal(idx, want_idx)
    np.testing.assert_array_equal(dist, want_dist)


def test_lse_option_errors(ragged, wmd):
    (vecs, ptr, ids, w), c = ragged
    q, qw = np.array([1, 2, 3], np.int32), np.ones(3, np.float32)
    for kw in ({"iters_per_launch": 4}, {"tile": 2}, {"tile": -2}, {"log_domain": True}):
        with pytest.raises(wmd.WmdError) as e:
            c.query(q, qw, 100.0, 5, lse=True, **kw)
        assert e.value.code == wmd.WMD_EINVAL
    with pytest.raises(wmd.WmdError) as e:
        c.query_adaptive(q, qw, 100.0, 5, 1e-3, lse=True)
    assert e.value.code == wmd.WMD_EINVAL


def test_lse_bf16_rejected(wmd):
    vecs, ptr, ids, w = ragged_corpus(V=500, N=120, seed=3, max_len=20)
    with wmd.Corpus(vecs, ptr, ids, w, device=0, bf16=True) as c:
        with pytest.raises(wmd.WmdError) as e:
            c.query(np.array([1, 2], np.int32), np.ones(2, np.float32), 100.0, 5, lse=True,
                    precision=wmd.WMD_DIST_BF16)
        assert e.value.code == wmd.WMD_EINVAL


def test_precision_corpus_lambda_1000_sampled(wmd):
    # N = 20 000 documents, 300-d embeddings: lambda M ~ 1400, far beyond FP32's
    # exp range even after the column shift
    wl = synth.make("c4")
    sp = wl.spec
    with wmd.Corpus(wl.vecs, wl.doc_ptr, wl.word_ids, wl.weights, device=0) as c:
        outs = [c.query(np.asarray(q, np.int32), np.asarray(qw, np.float32), 1000.0, sp.iters, lse=True)[0]
                for q, qw in wl.queries[:2]]
    worst = 0.0
    for i, (q, qw) in enumerate(wl.queries[:2]):
        docs = np.concatenate([np.random.default_rng(30 + i).choice(sp.N, 120, replace=False), [0, sp.N - 1]])
        sptr, sids, sw = synth.subcorpus(wl.doc_ptr, wl.word_ids, wl.weights, docs)
        want, _ = sinkhorn_wmd_lse(wl.vecs, q, qw, sptr, sids, sw, 1000.0, sp.iters)
        worst = max(worst, rel_err(outs[i][docs], want).max())
        assert np.all(np.isfinite(outs[i]))
    print(f"c4 corpus at lambda = 1000 (log domain): max rel err {worst:.2e}")
    assert worst <= FP32_RTOL


def test_server_with_lse_equals_single(ragged, wmd):
    # the served batches carve their workspaces with the log-domain layout (FP64 distances)
    (vecs, ptr, ids, w), c = ragged
    qs = [_query(vecs.shape[0], m, 70 + m) for m in (5, 33, 12, 48)]
    with wmd.Server(c, lse=True, max_batch=4, max_inflight=2, hbm_budget_bytes=1 << 30) as s:
        tickets = [s.submit(q, qw, 900.0, 12) for q, qw in qs]
        got = [s.wait(t)[0] for t in tickets]
    for (q, qw), d in zip(qs, got):
        np.testing.assert_array_equal(d, c.query(q, qw, 900.0, 12, lse=True)[0])
