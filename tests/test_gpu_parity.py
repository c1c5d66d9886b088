"""GPU path vs the FP64 oracle, element by element, through the C ABI.

Bar: FP32 distance path <= 1e-5 relative error per distance; BF16 distance
path <= 1e-3.  Residuals (row-marginal, FP64 on the GPU) are compared to
RESID_ATOL + RESID_RTOL * |residual|: rho = sum_k |u_k y_k - r_k| is a sum of
differences of nearly equal terms, each formed from the FP32 u_k and
y_k = (K^T v)_k, whose relative errors against the FP64 iteration are a few
units of FP32 rounding (2^-24); the terms sum to about sum_k r_k = 1, so the
absolute error is a few 1e-7 (measured at most 2.3e-7 over query lengths
1-300, lambda 0.25-50 and up to 200 iterations).
"""
import numpy as np
import pytest

from oracle import sinkhorn_wmd_sparse
from paper_2005_06727_amd import synth

pytestmark = pytest.mark.gpu

FP32_RTOL = 1e-5
BF16_RTOL = 1e-3
RESID_ATOL = 5e-7
RESID_RTOL = 1e-3


@pytest.fixture(scope="module")
def wmd():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2005_06727_amd import wmd as w
    return w


def rel_err(got, want):
    return np.abs(got - want) / np.abs(want)


def oracle_docs(wl_vecs, ptr, ids, w, docs, q, qw, lam, iters):
    sp, si, sw = synth.subcorpus(ptr, ids, w, docs)
    return sinkhorn_wmd_sparse(wl_vecs, q, qw, sp, si, sw, lam, iters)


def ragged_corpus(V=3000, dim=64, N=260, seed=21, max_len=100):
    """Document lengths 1..max_len (all present), Zipf words; some > 64 words."""
    rng = np.random.default_rng(seed)
    vecs = synth.embeddings(V, dim, rng)
    lens = np.concatenate([np.arange(1, max_len + 1), rng.integers(1, max_len + 1, N - max_len)])
    rng.shuffle(lens)
    cdf = synth.zipf_cdf(V, 1.1)
    ptr = np.zeros(N + 1, np.int64)
    ptr[1:] = np.cumsum(lens)
    ids = np.concatenate([synth._distinct_zipf(cdf, int(n), rng) for n in lens]).astype(np.int32)
    w = rng.geometric(0.5, ids.size).astype(np.float32)
    return vecs, ptr, ids, w


@pytest.fixture(scope="module")
def c1(wmd):
    wl = synth.make("c1")
    c = wmd.Corpus(wl.vecs, wl.doc_ptr, wl.word_ids, wl.weights, device=0, bf16=True)
    yield wl, c
    c.close()


@pytest.fixture(scope="module")
def ragged(wmd):
    vecs, ptr, ids, w = ragged_corpus()
    c = wmd.Corpus(vecs, ptr, ids, w, device=0, bf16=True)
    yield (vecs, ptr, ids, w), c
    c.close()


def test_c1_full_parity(c1):
    wl, c = c1
    q, qw = wl.queries[0]
    got, res = c.query(q, qw, wl.spec.lam, wl.spec.iters, resid=True)
    want, wres = sinkhorn_wmd_sparse(wl.vecs, q, qw, wl.doc_ptr, wl.word_ids, wl.weights,
                                     wl.spec.lam, wl.spec.iters)
    print("c1 max rel err", rel_err(got, want).max())
    assert rel_err(got, want).max() <= FP32_RTOL
    np.testing.assert_allclose(res, wres, rtol=RESID_RTOL, atol=RESID_ATOL)


@pytest.mark.parametrize("m", [1, 2, 3, 15, 16, 17, 31, 32, 33, 64, 65, 127, 128, 129, 256, 257,
                               511, 512, 513, 700])
def test_query_lengths_and_ragged_docs(ragged, m):
    (vecs, ptr, ids, w), c = ragged
    rng = np.random.default_rng(1000 + m)
    q = rng.choice(vecs.shape[0], m, replace=False).astype(np.int32)
    qw = rng.geometric(0.5, m).astype(np.float32)
    got, res = c.query(q, qw, 10.0, 15, resid=True)
    want, wres = sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, 10.0, 15)
    e = rel_err(got, want)
    print(f"m={m} max rel err {e.max():.2e} (docs 1..100 words)")
    assert e.max() <= FP32_RTOL
    np.testing.assert_allclose(res, wres, rtol=RESID_RTOL, atol=RESID_ATOL)


@pytest.mark.parametrize("lam,t", [(0.0, 1), (0.0, 15), (10.0, 0), (3.0, 1), (25.0, 40)])
def test_special_lambda_and_iters(ragged, lam, t):
    (vecs, ptr, ids, w), c = ragged
    rng = np.random.default_rng(7)
    q = rng.choice(vecs.shape[0], 24, replace=False).astype(np.int32)
    qw = rng.geometric(0.5, 24).astype(np.float32)
    got, _ = c.query(q, qw, lam, t)
    want, _ = sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, lam, t)
    assert rel_err(got, want).max() <= FP32_RTOL


def test_shared_words_give_zero_distance_terms(ragged):
    (vecs, ptr, ids, w), c = ragged
    # the query is document 0's words plus a few more: d = 0 on shared words
    q = np.unique(np.concatenate([ids[ptr[0]:ptr[1]], ids[ptr[5]:ptr[6]], [11, 23]])).astype(np.int32)
    qw = np.ones(q.size, np.float32)
    got, _ = c.query(q, qw, 10.0, 15)
    want, _ = sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, 10.0, 15)
    assert rel_err(got, want).max() <= FP32_RTOL


def test_zero_weight_words_dropped(ragged, wmd):
    (vecs, ptr, ids, w), c = ragged
    q = np.array([5, 17, 29, 101], np.int32)
    a, _ = c.query(q, np.array([1, 2, 3, 1], np.float32), 10.0, 15)
    b, _ = c.query(np.array([5, 17, 29, 101, 7], np.int32), np.array([1, 2, 3, 1, 0], np.float32), 10.0, 15)
    assert np.array_equal(a, b)


def test_deterministic(ragged):
    (vecs, ptr, ids, w), c = ragged
    q = np.arange(3, 90, 3, dtype=np.int32)
    qw = np.ones(q.size, np.float32)
    a, ra = c.query(q, qw, 10.0, 15, resid=True)
    b, rb = c.query(q, qw, 10.0, 15, resid=True)
    assert np.array_equal(a, b) and np.array_equal(ra, rb)


def test_iters_per_launch_matches_fused_bitwise(ragged):
    (vecs, ptr, ids, w), c = ragged
    rng = np.random.default_rng(3)
    for m in (9, 40, 200, 600):
        q = rng.choice(vecs.shape[0], m, replace=False).astype(np.int32)
        qw = rng.geometric(0.5, m).astype(np.float32)
        a, ra = c.query(q, qw, 10.0, 15, resid=True)
        for k in (1, 4, 15, 16):
            b, rb = c.query(q, qw, 10.0, 15, resid=True, iters_per_launch=k)
            assert np.array_equal(a, b), (m, k)
            assert np.array_equal(ra, rb), (m, k)


def test_batch_equals_single_bitwise(ragged, wmd):
    (vecs, ptr, ids, w), c = ragged
    rng = np.random.default_rng(4)
    ms = [1, 5, 16, 30, 64, 100, 200, 400, 520]
    queries = [(rng.choice(vecs.shape[0], m, replace=False).astype(np.int32),
                rng.geometric(0.5, m).astype(np.float32)) for m in ms]
    lams = np.array([10.0, 5.0, 10.0, 20.0, 10.0, 1.0, 10.0, 8.0, 10.0], np.float32)
    its = np.array([15, 3, 15, 0, 15, 20, 15, 15, 7], np.int32)
    out, res = c.query_batch(queries, lams, its, resid=True)
    for b, (q, qw) in enumerate(queries):
        one, r1 = c.query(q, qw, float(lams[b]), int(its[b]), resid=True)
        assert np.array_equal(out[b], one), b
        assert np.array_equal(res[b], r1), b
    want, _ = sinkhorn_wmd_sparse(vecs, queries[3][0], queries[3][1], ptr, ids, w, 20.0, 0)
    assert rel_err(out[3], want).max() <= FP32_RTOL


@pytest.mark.parametrize("tile", [2, 4])
def test_dense_occupancy_build_equals_default_bitwise(wmd, tile):
    """The 8-row, 8-column tiles have a second build at four waves per SIMD,
    which a launch takes when it has more waves than three per SIMD: a batch
    of 16 queries on 1200 documents (9600 waves) runs it, each query alone
    (600 waves) the default build; the bits agree."""
    vecs, ptr, ids, w = ragged_corpus(N=1200, seed=71, max_len=64)
    rng = np.random.default_rng(72)
    top = TILE_MAX_M[tile]
    with wmd.Corpus(vecs, ptr, ids, w, device=0) as c:
        queries = [(rng.choice(vecs.shape[0], m, replace=False).astype(np.int32),
                    rng.geometric(0.5, m).astype(np.float32)) for m in rng.integers(top // 2 + 1, top + 1, 16)]
        out, res = c.query_batch(queries, 10.0, 15, resid=True, tile=tile)
        for b, (q, qw) in enumerate(queries):
            one, r1 = c.query(q, qw, 10.0, 15, resid=True, tile=tile)
            assert np.array_equal(out[b], one), b
            assert np.array_equal(res[b], r1), b
        want, _ = sinkhorn_wmd_sparse(vecs, queries[0][0], queries[0][1], ptr, ids, w, 10.0, 15)
        assert rel_err(out[0], want).max() <= FP32_RTOL


@pytest.mark.parametrize("bf16", [False, True])
def test_shift_one_query_kernel_equals_batched_bitwise(wmd, bf16):
    """With the column shift, a single query of up to 64 words runs the
    one-query distance kernel (row minimum reduced inside the wave, K written
    once; two passes beyond 32 words) and a batch the tiled kernel (row minima
    by atomics, then a second pass): the same bits, with K .* M rebuilt from K
    (lambda 50) and gathered (lambda 0.25)."""
    vecs, ptr, ids, w = ragged_corpus(seed=61)
    rng = np.random.default_rng(62)
    with wmd.Corpus(vecs, ptr, ids, w, device=0, bf16=bf16) as c:
        opts = dict(log_domain=True, precision=wmd.WMD_DIST_BF16 if bf16 else wmd.WMD_DIST_FP32)
        queries = [(rng.choice(vecs.shape[0], m, replace=False).astype(np.int32),
                    rng.geometric(0.5, m).astype(np.float32)) for m in (1, 7, 26, 32, 33, 40, 64)]
        for lam in (50.0, 0.25):
            out, _ = c.query_batch(queries, np.full(len(queries), lam, np.float32),
                                   np.full(len(queries), 12, np.int32), **opts)
            for b, (q, qw) in enumerate(queries):
                one, _ = c.query(q, qw, lam, 12, **opts)
                assert np.array_equal(out[b], one), (lam, b)


def test_async_equals_sync(ragged, wmd):
    import torch
    (vecs, ptr, ids, w), c = ragged
    N = c.info["N"]
    q = np.arange(100, 140, dtype=np.int32)
    qw = np.ones(q.size, np.float32)
    sync, rsync = c.query(q, qw, 10.0, 15, resid=True)
    s = torch.cuda.Stream()
    d = torch.full((N,), -1.0, dtype=torch.float64, device="cuda")
    r = torch.full((N,), -1.0, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(s):
        wmd.wmd_query_async(c.handle, q, qw, 10.0, 15, d, r, stream=s)
    s.synchronize()
    assert np.array_equal(d.cpu().numpy(), sync)
    assert np.array_equal(r.cpu().numpy(), rsync)
    # batch async
    queries = [(q, qw), (q[:7], qw[:7])]
    out = torch.empty((2, N), dtype=torch.float64, device="cuda")
    wmd.wmd_query_batch_async(c.handle, queries, 10.0, 15, out)
    torch.cuda.synchronize()
    assert np.array_equal(out[0].cpu().numpy(), sync)


@pytest.mark.parametrize("log_domain", [False, True])
def test_large_lambda(ragged, log_domain):
    (vecs, ptr, ids, w), c = ragged
    rng = np.random.default_rng(5)
    q = rng.choice(vecs.shape[0], 30, replace=False).astype(np.int32)
    qw = rng.geometric(0.5, 30).astype(np.float32)
    got, _ = c.query(q, qw, 50.0, 15, log_domain=log_domain)
    want, _ = sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, 50.0, 15)
    e = rel_err(got, want)
    print(f"lambda=50 log_domain={log_domain}: max rel err {e.max():.2e}")
    assert e.max() <= FP32_RTOL


def test_bf16_distances(ragged, wmd):
    (vecs, ptr, ids, w), c = ragged
    rng = np.random.default_rng(6)
    for m in (12, 40, 150):
        q = rng.choice(vecs.shape[0], m, replace=False).astype(np.int32)
        q[:3] = ids[:3]      # shared words: exact zero distances
        q = np.unique(q)
        qw = rng.geometric(0.5, q.size).astype(np.float32)
        got, _ = c.query(q, qw, 50.0, 15, precision=wmd.WMD_DIST_BF16, log_domain=True)
        want, _ = sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, 50.0, 15)
        e = rel_err(got, want)
        print(f"bf16 m={q.size}: max rel err {e.max():.2e} median {np.median(e):.2e}")
        assert e.max() <= BF16_RTOL


def near_duplicate_corpus(seed=12, V=3000, dim=64, N=200, nbase=20):
    """Query words with planted near-synonyms at distances 1e-3 .. 0.3 (where
    |a|^2 + |b|^2 - 2 a.b cancels): every document holds three of them beside
    5-30 Zipf words."""
    rng = np.random.default_rng(seed)
    vecs = synth.embeddings(V, dim, rng)
    dists = np.array([1e-3, 3e-3, 1e-2, 3e-2, 0.1, 0.3])
    bases = rng.choice(V, nbase, replace=False)
    others = np.setdiff1d(np.arange(V), bases)
    planted = rng.choice(others, nbase * dists.size, replace=False)
    vecs = synth.near_duplicates(vecs, np.repeat(bases, dists.size), planted, np.tile(dists, nbase), rng)
    cdf = synth.zipf_cdf(V, 1.1)
    docs = []
    for _ in range(N):
        near = rng.choice(planted, 3, replace=False)
        rest = [x for x in synth._distinct_zipf(cdf, int(rng.integers(5, 31)), rng) if x not in near]
        docs.append(np.concatenate([near, np.asarray(rest, np.int64)]))
    ptr = np.zeros(N + 1, np.int64)
    ptr[1:] = np.cumsum([d.size for d in docs])
    ids = np.concatenate(docs).astype(np.int32)
    w = rng.geometric(0.5, ids.size).astype(np.float32)
    q = bases.astype(np.int32)
    qw = rng.geometric(0.5, q.size).astype(np.float32)
    return vecs, ptr, ids, w, q, qw


@pytest.mark.parametrize("lam", [10.0, 50.0])
def test_near_duplicate_words_recompute(wmd, lam):
    """Distances below the recompute threshold are taken as direct FP32 sums
    of squared differences: the FP32 path keeps its bar on near-synonyms, and
    so does the BF16 path with its default threshold."""
    vecs, ptr, ids, w, q, qw = near_duplicate_corpus()
    want, _ = sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, lam, 15)
    with wmd.Corpus(vecs, ptr, ids, w, device=0, bf16=True) as c:
        for log_domain in (False, True):
            e32 = rel_err(c.query(q, qw, lam, 15, log_domain=log_domain)[0], want)
            e16 = rel_err(c.query(q, qw, lam, 15, log_domain=log_domain, precision=wmd.WMD_DIST_BF16)[0], want)
            print(f"near duplicates lambda={lam} log_domain={log_domain}: FP32 max {e32.max():.2e}, "
                  f"BF16 max {e16.max():.2e} median {np.median(e16):.2e}")
            assert e32.max() <= FP32_RTOL
            assert e16.max() <= BF16_RTOL


def test_query_errors(ragged, wmd):
    (vecs, ptr, ids, w), c = ragged
    V = vecs.shape[0]
    bad = [
        (np.array([1, 1], np.int32), np.ones(2, np.float32), 10.0, 15),
        (np.array([1, V], np.int32), np.ones(2, np.float32), 10.0, 15),
        (np.array([1, -2], np.int32), np.ones(2, np.float32), 10.0, 15),
        (np.array([1, 2], np.int32), np.zeros(2, np.float32), 10.0, 15),
        (np.array([1, 2], np.int32), np.array([1, -1], np.float32), 10.0, 15),
        (np.array([1, 2], np.int32), np.ones(2, np.float32), -1.0, 15),
        (np.array([1, 2], np.int32), np.ones(2, np.float32), float("nan"), 15),
        (np.array([1, 2], np.int32), np.ones(2, np.float32), 10.0, -1),
    ]
    for q, qw, lam, t in bad:
        with pytest.raises(wmd.WmdError) as e:
            c.query(q, qw, lam, t)
        assert e.value.code == wmd.WMD_EINVAL


def test_bf16_needs_copies(wmd):
    vecs, ptr, ids, w = ragged_corpus(V=500, N=120, seed=3)
    with wmd.Corpus(vecs, ptr, ids, w, device=0, bf16=False) as c:
        with pytest.raises(wmd.WmdError) as e:
            c.query(np.array([1, 2], np.int32), np.ones(2, np.float32), 10.0, 5,
                    precision=wmd.WMD_DIST_BF16)
        assert e.value.code == wmd.WMD_EINVAL


def test_single_document_and_single_word_corpus(wmd):
    vecs = synth.embeddings(50, 64, np.random.default_rng(9))
    for ptr, ids, w in [([0, 1], [7], [2.0]), ([0, 3], [7, 8, 9], [1.0, 0.0, 2.0])]:
        with wmd.Corpus(vecs, ptr, ids, w, device=0) as c:
            q = np.array([3, 7, 40], np.int32)
            qw = np.array([1, 2, 1], np.float32)
            got, _ = c.query(q, qw, 10.0, 15)
            keep = np.asarray(w) > 0
            want, _ = sinkhorn_wmd_sparse(vecs, q, qw, [0, int(keep.sum())],
                                          np.asarray(ids)[keep], np.asarray(w, np.float32)[keep], 10.0, 15)
            assert rel_err(got, want).max() <= FP32_RTOL


def test_c2_paper_shape_sampled(wmd):
    wl = synth.make("c2")
    q, qw = wl.queries[0]
    sp = wl.spec
    with wmd.Corpus(wl.vecs, wl.doc_ptr, wl.word_ids, wl.weights, device=0) as c:
        got, res = c.query(q, qw, sp.lam, sp.iters, resid=True)
        info = c.info
    print("c2 corpus:", info)
    docs = np.random.default_rng(0).choice(sp.N, 400, replace=False)
    docs = np.concatenate([docs, [0, sp.N - 1]])
    want, wres = oracle_docs(wl.vecs, wl.doc_ptr, wl.word_ids, wl.weights, docs, q, qw, sp.lam, sp.iters)
    e = rel_err(got[docs], want)
    print(f"c2 (V=100k, N=5000, v_r={q.size}): max rel err {e.max():.2e} on {docs.size} sampled docs")
    assert e.max() <= FP32_RTOL
    assert np.all(np.isfinite(got)) and np.all(got > 0)


TILE_MAX_M = {0: 16, 1: 32, 2: 32, 3: 64, 4: 64, 5: 128, 6: 256, 7: 512, 8: 16, 9: 32, 10: 64, 11: 32, 12: 48, 13: 96, 14: 192, 15: 384, 16: 256}


@pytest.mark.parametrize("tile", [-2] + sorted(TILE_MAX_M))
def test_every_tile_shape(ragged, wmd, tile):
    (vecs, ptr, ids, w), c = ragged
    rng = np.random.default_rng(50 + tile)
    top = TILE_MAX_M.get(tile, 600)
    for m in sorted({1, 3, top // 2 + 1, top}):
        q = rng.choice(vecs.shape[0], m, replace=False).astype(np.int32)
        qw = rng.geometric(0.5, m).astype(np.float32)
        got, res = c.query(q, qw, 10.0, 15, resid=True, tile=tile)
        want, wres = sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, 10.0, 15)
        e = rel_err(got, want)
        print(f"tile={tile} m={m}: max rel err {e.max():.2e}")
        assert e.max() <= FP32_RTOL
        np.testing.assert_allclose(res, wres, rtol=RESID_RTOL, atol=RESID_ATOL)
        again, _ = c.query(q, qw, 10.0, 15, tile=tile, iters_per_launch=4)
        assert np.array_equal(got, again)
    if tile >= 0:
        m = top + 1
        q = rng.choice(vecs.shape[0], m, replace=False).astype(np.int32)
        with pytest.raises(wmd.WmdError) as ex:
            c.query(q, np.ones(m, np.float32), 10.0, 15, tile=tile)
        assert ex.value.code == wmd.WMD_EINVAL
