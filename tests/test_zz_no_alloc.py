"""The allocation-free entry point (wmd_query_noalloc) through the C ABI
(the ctypes binding of the same name):
its results equal wmd_query_async's bitwise and the FP64 oracle to the FP32
bar, on two calls in a row (the second with a smaller query) and after a
call with a different workspace layout; sizes beyond the fixed scratch are
refused."""
import numpy as np
import pytest

from oracle import sinkhorn_wmd_sparse
from tests.test_gpu_parity import FP32_RTOL, ragged_corpus, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2005_06727_amd import wmd
    vecs, ptr, ids, w = ragged_corpus(seed=41)
    c = wmd.Corpus(vecs, ptr, ids, w, device=0)
    yield torch, wmd, (vecs, ptr, ids, w), c
    c.close()


def noalloc(env, q, qw, lam, iters, resid=True, **opts):
    torch, wmd, _, c = env
    N = c.info["N"]
    d = torch.full((N,), -1.0, dtype=torch.float64, device="cuda")
    r = torch.full((N,), -1.0, dtype=torch.float64, device="cuda") if resid else None
    wmd.wmd_query_noalloc(c.handle, q, qw, lam, iters, d, r, torch.cuda.current_stream(), **opts)
    torch.cuda.synchronize()
    return d.cpu().numpy(), (r.cpu().numpy() if resid else None)


def plain_async(env, q, qw, lam, iters, **opts):
    torch, wmd, _, c = env
    N = c.info["N"]
    d = torch.empty(N, dtype=torch.float64, device="cuda")
    r = torch.empty(N, dtype=torch.float64, device="cuda")
    wmd.wmd_query_async(c.handle, q, qw, lam, iters, d, r, torch.cuda.current_stream(), **opts)
    torch.cuda.synchronize()
    return d.cpu().numpy(), r.cpu().numpy()


@pytest.mark.parametrize("opts", [{}, {"log_domain": 1}, {"iters_per_launch": 4}])
def test_noalloc_matches_async_twice(env, opts):
    vecs, ptr, ids, w = env[2]
    rng = np.random.default_rng(5)
    big = rng.choice(vecs.shape[0], 90, replace=False).astype(np.int32)
    small = rng.choice(vecs.shape[0], 7, replace=False).astype(np.int32)
    for q in (big, small):   # second call: smaller query, stale scratch from the first
        qw = rng.random(q.size, dtype=np.float32) + 0.1
        got, gres = noalloc(env, q, qw, 10.0, 9, **opts)
        want, wres = plain_async(env, q, qw, 10.0, 9, **opts)
        np.testing.assert_array_equal(got, want)
        np.testing.assert_array_equal(gres, wres)
        ref, _ = sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, 10.0, 9)
        assert rel_err(got, ref).max() <= FP32_RTOL


def test_noalloc_small_lambda_and_refusals(env):
    torch, wmd, (vecs, ptr, ids, w), c = env
    q = np.arange(12, dtype=np.int32)
    qw = np.linspace(1, 2, 12).astype(np.float32)
    got, _ = noalloc(env, q, qw, 0.25, 6, resid=False)     # K .* M gathered from its own buffer
    want, _ = plain_async(env, q, qw, 0.25, 6)
    np.testing.assert_array_equal(got, want)
    # a query whose parameter block is too large to travel as kernel arguments
    long_q = np.arange(2000, dtype=np.int32)
    with pytest.raises(wmd.WmdError) as e:
        noalloc(env, long_q, np.ones(2000, np.float32), 10.0, 3)
    assert e.value.code == wmd.WMD_EINVAL
    with pytest.raises(wmd.WmdError) as e:
        noalloc(env, q, -qw, 10.0, 3)
    assert e.value.code == wmd.WMD_EINVAL
