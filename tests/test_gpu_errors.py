"""Device-allocation failure through the C ABI: with the library's
fault-injection switch (WMD_TEST_FAIL_ALLOC_BYTES) a query, a server and a
corpus whose device memory cannot be had fail with WMD_ENOMEM, leave their
outputs untouched, and the corpus works again once memory is available."""
import ctypes as C

import numpy as np
import pytest

from oracle import sinkhorn_wmd_sparse
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


def test_allocation_failure_is_enomem(wmd, monkeypatch):
    vecs, ptr, ids, w = ragged_corpus(seed=8)
    rng = np.random.default_rng(4)
    q = rng.choice(vecs.shape[0], 300, replace=False).astype(np.int32)
    qw = rng.geometric(0.5, q.size).astype(np.float32)
    with wmd.Corpus(vecs, ptr, ids, w, device=0) as c:
        N, U = c.info["N"], c.info["U"]
        kblock = 4 * U * 300                      # the query's K block, its largest buffer
        out = np.full(N, -7.0)
        res = np.full(N, -7.0)
        o = wmd.wmd_query_options_init()
        monkeypatch.setenv("WMD_TEST_FAIL_ALLOC_BYTES", str(kblock // 2))
        rc = wmd._lib.wmd_query(c.handle, q.ctypes.data, qw.ctypes.data, q.size, 10.0, 15, C.byref(o),
                                out.ctypes.data, res.ctypes.data)
        assert rc == wmd.WMD_ENOMEM, wmd.wmd_last_error()
        assert "K buffer" in wmd.wmd_last_error()
        assert np.all(out == -7.0) and np.all(res == -7.0)
        with pytest.raises(wmd.WmdError) as e:
            wmd.Server(c, hbm_budget_bytes=kblock)
        assert e.value.code == wmd.WMD_ENOMEM
        monkeypatch.delenv("WMD_TEST_FAIL_ALLOC_BYTES")
        got, _ = c.query(q, qw, 10.0, 15)
        want, _ = sinkhorn_wmd_sparse(vecs, q, qw, ptr, ids, w, 10.0, 15)
        assert rel_err(got, want).max() <= FP32_RTOL
    monkeypatch.setenv("WMD_TEST_FAIL_ALLOC_BYTES", "4096")
    with pytest.raises(wmd.WmdError) as e:
        wmd.Corpus(vecs, ptr, ids, w, device=0)
    assert e.value.code == wmd.WMD_ENOMEM
