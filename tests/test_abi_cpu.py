"""C ABI checks that need no GPU: the library loads, exports every function
include/wmd.h declares, fills option defaults, and rejects invalid corpora
during host-side validation (before any device call)."""
import numpy as np
import pytest

from paper_2005_06727_amd import wmd


def test_every_declared_function_is_exported():
    names = wmd.declared_functions()
    assert len(names) >= 12
    missing = [n for n in names if not wmd.exported(n)]
    assert not missing, missing


def test_option_defaults():
    o = wmd.wmd_query_options_init()
    assert (o.precision, o.recompute_below, o.log_domain, o.iters_per_launch, o.tile, o.tol, o.lse) == (
        0, -1.0, 0, 0, -1, 0.0, 0)
    c = wmd.wmd_corpus_options_init()
    assert (c.device, c.bf16) == (-1, 0)


V = np.eye(6, 4, dtype=np.float32)


@pytest.mark.parametrize("ptr,ids,w,msg", [
    ([0, 2], [1, 1], [1.0, 1.0], "repeats"),
    ([0, 2], [1, 9], [1.0, 1.0], "out of range"),
    ([0, 2], [1, -1], [1.0, 1.0], "out of range"),
    ([0, 2], [1, 2], [1.0, -1.0], "negative"),
    ([0, 2], [1, 2], [1.0, np.nan], "non-finite"),
    ([0, 2], [1, 2], [0.0, 0.0], "no word with positive weight"),
    ([0, 0, 1], [1], [1.0], "no word with positive weight"),
    ([1, 2], [1, 2], [1.0, 1.0], "doc_ptr[0]"),
    ([0, 2, 1], [1, 2], [1.0, 1.0], "decreases"),
])
def test_invalid_corpus_rejected(ptr, ids, w, msg):
    with pytest.raises(wmd.WmdError) as e:
        wmd.wmd_corpus_create(V, ptr, ids, w)
    assert e.value.code == wmd.WMD_EINVAL
    assert msg in str(e.value)
    assert msg in wmd.wmd_last_error()


def test_invalid_sizes_rejected():
    with pytest.raises(wmd.WmdError) as e:
        wmd.wmd_corpus_create(np.zeros((0, 4), np.float32), [0, 1], [0], [1.0])
    assert e.value.code == wmd.WMD_EINVAL
    with pytest.raises(wmd.WmdError) as e:
        wmd.wmd_corpus_create(np.zeros((4, 0), np.float32), [0, 1], [0], [1.0])
    assert e.value.code == wmd.WMD_EINVAL


def test_null_handle_info_is_einval():
    with pytest.raises(wmd.WmdError) as e:
        wmd.wmd_corpus_info_get(None)
    assert e.value.code == wmd.WMD_EINVAL


def test_product_path_does_not_import_oracle():
    import ast
    import os
    pkg = os.path.dirname(wmd.__file__)
    for f in os.listdir(pkg):
        if f.endswith(".py"):
            tree = ast.parse(open(os.path.join(pkg, f)).read())
            for node in ast.walk(tree):
                if isinstance(node, (ast.Import, ast.ImportFrom)):
                    mods = [a.name for a in node.names] if isinstance(node, ast.Import) else [node.module or ""]
                    assert not any(m.split(".")[0] == "oracle" for m in mods), f


def test_server_option_defaults_and_null_corpus():
    o = wmd.wmd_server_options_init()
    assert (o.hbm_budget_bytes, o.max_batch, o.max_inflight, o.want_resid, o.batch_wait_us, o.max_batch_words,
            o.step_iters) == (4 << 30, 16, 2, 0, 0, 512, 0)
    assert (o.query.precision, o.query.tile) == (0, -1)
    with pytest.raises(wmd.WmdError) as e:
        wmd.wmd_server_create(None)
    assert e.value.code == wmd.WMD_EINVAL
    with pytest.raises(wmd.WmdError) as e:
        wmd.wmd_server_submit(None, [1], [1.0], 1.0, 1)
    assert e.value.code == wmd.WMD_EINVAL
    wmd.wmd_server_destroy(None)


def test_valid_corpus_host_preparation_without_gpu():
    """A valid ragged corpus passes the host-side preparation (validation,
    vocabulary remap, the length sort and the grouping of equal-length
    documents by XCD) and then stops at device selection when there is no
    GPU: under the sanitizer build this runs that host code on the CPU."""
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present: the corpus would be created")
    rng = np.random.default_rng(5)
    V, N = 500, 300
    vecs = rng.standard_normal((V, 8)).astype(np.float32)
    lens = np.concatenate([np.arange(1, 101), rng.integers(1, 101, N - 100)])
    ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    ids = np.concatenate([rng.choice(V, n, replace=False) for n in lens]).astype(np.int32)
    w = rng.random(ids.size).astype(np.float32) + 0.1
    with pytest.raises(wmd.WmdError) as e:
        wmd.wmd_corpus_create(vecs, ptr, ids, w, device=0)
    assert e.value.code == wmd.WMD_EDEVICE
