"""Parity at the full workload sizes, on sampled documents.

The oracle computes each sampled document on its own (the iteration of one
document never reads another's), so a few hundred documents of a 5 000- to
100 000-document corpus can be checked one by one at the real shapes:

* the 64-query batch (v_r 5-200) on the paper-shaped corpus, one batch call;
* the precision configuration (N = 20 000, lambda = 50, BF16 distances with
  FP32 recompute, log-domain column shift), and its FP32 form;
* the served stream's corpus (V = 200 000, N = 100 000): BF16 queries through
  the continuous-batching server, and a plain FP32 query.
"""
import numpy as np
import pytest

from oracle import sinkhorn_wmd_sparse
from paper_2005_06727_amd import synth
from tests.test_gpu_parity import BF16_RTOL, FP32_RTOL, oracle_docs, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wmd():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2005_06727_amd import wmd as w
    return w


def sample_docs(N, n, seed):
    d = np.random.default_rng(seed).choice(N, n, replace=False)
    return np.concatenate([d, [0, N - 1]])


def test_batch64_sampled(wmd):
    wl = synth.make("c3")
    sp = wl.spec
    qs = [(np.asarray(q, np.int32), np.asarray(w, np.float32)) for q, w in wl.queries]
    with wmd.Corpus(wl.vecs, wl.doc_ptr, wl.word_ids, wl.weights, device=0) as c:
        got, _ = c.query_batch(qs, sp.lam, sp.iters)
        for b in (0, 31):
            np.testing.assert_array_equal(got[b], c.query(*qs[b], sp.lam, sp.iters)[0])
    lens = [len(q) for q, _ in qs]
    picks = sorted({int(np.argmin(lens)), int(np.argmax(lens)), 7, 40})
    worst = 0.0
    for b in picks:
        docs = sample_docs(sp.N, 120, b)
        want, _ = oracle_docs(wl.vecs, wl.doc_ptr, wl.word_ids, wl.weights, docs, *qs[b], sp.lam, sp.iters)
        worst = max(worst, rel_err(got[b][docs], want).max())
    print(f"64-query batch: max rel err {worst:.2e} over queries {picks} (v_r {[lens[b] for b in picks]})")
    assert worst <= FP32_RTOL


@pytest.mark.parametrize("bf16", [True, False])
def test_precision_config_sampled(wmd, bf16):
    wl = synth.make("c4")
    sp = wl.spec
    opts = {"precision": wmd.WMD_DIST_BF16 if bf16 else wmd.WMD_DIST_FP32, "log_domain": True}
    if bf16:
        opts["recompute_below"] = 1e-2
    tol = BF16_RTOL if bf16 else FP32_RTOL
    with wmd.Corpus(wl.vecs, wl.doc_ptr, wl.word_ids, wl.weights, device=0, bf16=bf16) as c:
        outs = [c.query(np.asarray(q, np.int32), np.asarray(w, np.float32), sp.lam, sp.iters, resid=True, **opts)
                for q, w in wl.queries[:3]]
    errs = []
    for i, (q, w) in enumerate(wl.queries[:3]):
        docs = sample_docs(sp.N, 150, 10 + i)
        want, _ = oracle_docs(wl.vecs, wl.doc_ptr, wl.word_ids, wl.weights, docs, q, w, sp.lam, sp.iters)
        e = rel_err(outs[i][0][docs], want)
        errs.append((float(e.max()), float(np.percentile(e, 99)), float(np.median(e))))
        assert np.all(np.isfinite(outs[i][0]))
    print(f"lambda=50 {'BF16' if bf16 else 'FP32'} + log-domain: (max, p99, median) rel err per query {errs}")
    assert max(e[0] for e in errs) <= tol


def test_served_stream_corpus_sampled(wmd):
    wl = synth.make("c5", n_queries=40)
    sp = wl.spec
    qs = [(np.asarray(q, np.int32), np.asarray(w, np.float32)) for q, w in wl.queries]
    lens = np.array([len(q) for q, _ in qs])
    picks = [int(np.argmin(lens)), int(np.argmax(lens)), 3, 17]
    with wmd.Corpus(wl.vecs, wl.doc_ptr, wl.word_ids, wl.weights, device=0, bf16=True) as c:
        with wmd.Server(c, precision=wmd.WMD_DIST_BF16, max_batch=8, max_inflight=2,
                        hbm_budget_bytes=8 << 30) as s:
            tickets = [s.submit(q, w, sp.lam, sp.iters) for q, w in qs]
            served = [s.wait(t)[0] for t in tickets]
        plain = c.query(*qs[picks[1]], sp.lam, sp.iters)[0]   # FP32 path, the longest query
    worst_bf16 = 0.0
    for b in picks:
        docs = sample_docs(sp.N, 80, 100 + b)
        want, _ = oracle_docs(wl.vecs, wl.doc_ptr, wl.word_ids, wl.weights, docs, *qs[b], sp.lam, sp.iters)
        worst_bf16 = max(worst_bf16, rel_err(served[b][docs], want).max())
        if b == picks[1]:
            e32 = rel_err(plain[docs], want).max()
    print(f"N=100k corpus: served BF16 max rel err {worst_bf16:.2e} (v_r {lens[picks].tolist()}), "
          f"plain FP32 (v_r {lens[picks[1]]}) {e32:.2e}")
    assert worst_bf16 <= BF16_RTOL
    assert e32 <= FP32_RTOL


def test_paper_corpus_uniform_query_words_sampled(wmd):
    # the paper-shaped corpus with a query whose words are uniform over the
    # vocabulary (mostly words no document shares), beside the Zipf queries
    wl = synth.make("c2")
    sp = wl.spec
    q, qw = synth.query(sp.V, 30, np.random.default_rng(2024), "uniform")
    with wmd.Corpus(wl.vecs, wl.doc_ptr, wl.word_ids, wl.weights, device=0) as c:
        got, _ = c.query(q, qw, sp.lam, sp.iters)
    docs = sample_docs(sp.N, 200, 77)
    want, _ = oracle_docs(wl.vecs, wl.doc_ptr, wl.word_ids, wl.weights, docs, q, qw, sp.lam, sp.iters)
    e = rel_err(got[docs], want)
    print(f"c2 corpus, uniform query words (v_r=30): max rel err {e.max():.2e}")
    assert e.max() <= FP32_RTOL
