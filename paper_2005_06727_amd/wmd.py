"""ctypes binding of libwmd (include/wmd.h): argument marshalling only.

Every function here has the name of the C entry point it calls; all the
arithmetic runs in the library's HIP kernels.  Importing this module loads
``libwmd.so`` and raises ImportError when it has not been built
(``python -m paper_2005_06727_amd.build``).  The environment variable
``WMD_LIBRARY`` names another build of the same library to load instead (for
example one whose host code is instrumented with sanitizers).

torch, when importable, is imported before the library so that the process
holds a single HIP runtime (torch ships its own copy under the same soname);
it is used only for device buffers and streams of the ``*_async`` calls.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from typing import Optional, Sequence, Tuple

import numpy as np

try:  # one HIP runtime per process: let torch's copy be the one
    import torch
except ImportError:  # pragma: no cover - torch is part of the image
    torch = None

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("WMD_LIBRARY") or os.path.join(PKG, "libwmd.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "wmd.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run: python -m paper_2005_06727_amd.build")
_lib = C.CDLL(LIB_PATH)

WMD_OK, WMD_EINVAL, WMD_ENOMEM, WMD_EDEVICE = 0, -1, -2, -3
WMD_ETIMEDOUT, WMD_ESHUTDOWN, WMD_ENOTFOUND = -4, -5, -6
WMD_DIST_FP32, WMD_DIST_BF16 = 0, 1


class WmdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libwmd error {code}: {msg}")
        self.code = code


class wmd_corpus_options(C.Structure):
    _fields_ = [("device", C.c_int32), ("bf16", C.c_int32)]


class wmd_query_options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("recompute_below", C.c_float),
                ("log_domain", C.c_int32), ("iters_per_launch", C.c_int32), ("tile", C.c_int32),
                ("tol", C.c_float), ("lse", C.c_int32)]


class wmd_corpus_info(C.Structure):
    _fields_ = [("V", C.c_int64), ("N", C.c_int64), ("nnz", C.c_int64), ("U", C.c_int64),
                ("dim", C.c_int32), ("max_doc_words", C.c_int32), ("device", C.c_int32),
                ("has_bf16", C.c_int32), ("device_bytes", C.c_int64)]


class wmd_timing(C.Structure):
    _fields_ = [("calls", C.c_int64), ("dist_ms", C.c_double), ("sinkhorn_ms", C.c_double),
                ("last_dist_ms", C.c_float), ("last_sinkhorn_ms", C.c_float), ("launches", C.c_int32)]


class wmd_server_options(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_int64), ("max_batch", C.c_int32), ("max_inflight", C.c_int32),
                ("want_resid", C.c_int32), ("batch_wait_us", C.c_int32), ("query", wmd_query_options),
                ("max_batch_words", C.c_int32), ("step_iters", C.c_int32)]


class wmd_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("batches", C.c_int64),
                ("latency_p50_ms", C.c_double), ("latency_p99_ms", C.c_double),
                ("latency_mean_ms", C.c_double), ("latency_max_ms", C.c_double),
                ("queries_per_s", C.c_double), ("doc_iters_per_s", C.c_double),
                ("mean_batch", C.c_double), ("workspace_bytes", C.c_int64)]


_P = C.c_void_p
# array arguments travel as plain addresses (the element type is the header's):
# building a typed ctypes pointer per call costs several microseconds
_i32p = _i64p = _f32p = _f64p = C.c_void_p


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype, f.argtypes = res, list(args)
    return f


_sig("wmd_last_error", C.c_char_p)
_sig("wmd_corpus_options_init", None, C.POINTER(wmd_corpus_options))
_sig("wmd_query_options_init", None, C.POINTER(wmd_query_options))
_sig("wmd_corpus_create", C.c_int, _f32p, C.c_int64, C.c_int32, _i64p, _i32p, _f32p, C.c_int64,
     C.POINTER(wmd_corpus_options), C.POINTER(_P))
_sig("wmd_corpus_destroy", None, _P)
_sig("wmd_corpus_info_get", C.c_int, _P, C.POINTER(wmd_corpus_info))
_sig("wmd_query", C.c_int, _P, _i32p, _f32p, C.c_int32, C.c_float, C.c_int32,
     C.POINTER(wmd_query_options), _f64p, _f64p)
_sig("wmd_query_async", C.c_int, _P, _i32p, _f32p, C.c_int32, C.c_float, C.c_int32,
     C.POINTER(wmd_query_options), _P, _P, _P)
_sig("wmd_query_noalloc", C.c_int, _P, _i32p, _f32p, C.c_int32, C.c_float, C.c_int32,
     C.POINTER(wmd_query_options), _P, _P, _P)
_sig("wmd_query_batch", C.c_int, _P, C.c_int32, _i64p, _i32p, _f32p, _f32p, _i32p,
     C.POINTER(wmd_query_options), _f64p, _f64p)
_sig("wmd_query_batch_async", C.c_int, _P, C.c_int32, _i64p, _i32p, _f32p, _f32p, _i32p,
     C.POINTER(wmd_query_options), _P, _P, _P)
_sig("wmd_query_adaptive", C.c_int, _P, _i32p, _f32p, C.c_int32, C.c_float, C.c_int32,
     C.POINTER(wmd_query_options), _f64p, _f64p, _i32p)
_sig("wmd_query_topk", C.c_int, _P, _i32p, _f32p, C.c_int32, C.c_float, C.c_int32,
     C.POINTER(wmd_query_options), C.c_int32, _i32p, _f64p)
_sig("wmd_query_topk_async", C.c_int, _P, _i32p, _f32p, C.c_int32, C.c_float, C.c_int32,
     C.POINTER(wmd_query_options), C.c_int32, _P, _P, _P)
_sig("wmd_set_timing", C.c_int, _P, C.c_int32)
_sig("wmd_timing_get", C.c_int, _P, C.POINTER(wmd_timing))
_sig("wmd_server_options_init", None, C.POINTER(wmd_server_options))
_sig("wmd_server_create", C.c_int, _P, C.POINTER(wmd_server_options), C.POINTER(_P))
_sig("wmd_server_submit", C.c_int64, _P, _i32p, _f32p, C.c_int32, C.c_float, C.c_int32)
_sig("wmd_server_wait", C.c_int, _P, C.c_int64, _f64p, _f64p, C.c_int64)
_sig("wmd_server_stats_get", C.c_int, _P, C.POINTER(wmd_server_stats))
_sig("wmd_server_stats_reset", C.c_int, _P)
_sig("wmd_server_destroy", None, _P)


def declared_functions() -> list:
    """Names of the functions include/wmd.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w]+\s*\*?\s*(wmd_\w+)\s*\(", text, flags=re.M)))


def exported(name: str) -> bool:
    return hasattr(_lib, name)


def wmd_last_error() -> str:
    return (_lib.wmd_last_error() or b"").decode()


def _check(rc: int) -> None:
    if rc != WMD_OK:
        raise WmdError(rc, wmd_last_error())


def _arr(a, dtype) -> np.ndarray:
    if type(a) is np.ndarray and a.dtype == dtype and a.flags.c_contiguous:
        return a
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


def _ptr(a: np.ndarray, ctype=None) -> int:
    """Address of a C-contiguous array (``ctype`` names the element type the C side reads)."""
    return a.__array_interface__["data"][0]


def _make_qopts(precision, recompute_below, log_domain, iters_per_launch, tile, tol, lse):
    o = wmd_query_options()
    _lib.wmd_query_options_init(C.byref(o))
    o.precision = int(precision)
    o.recompute_below = float(recompute_below)
    o.log_domain = int(bool(log_domain))
    o.iters_per_launch = int(iters_per_launch)
    o.tile = int(tile)
    o.tol = float(tol)
    o.lse = int(bool(lse))
    return o


_DEFAULT_QOPTS = (WMD_DIST_FP32, -1.0, False, 0, -1, 0.0, False)
_default_qopts = None


def _qopts(precision=WMD_DIST_FP32, recompute_below=-1.0, log_domain=False, iters_per_launch=0,
           tile=-1, tol=0.0, lse=False):
    global _default_qopts
    args = (precision, recompute_below, log_domain, iters_per_launch, tile, tol, lse)
    if args == _DEFAULT_QOPTS:
        # the library copies the options at the call, so one default object serves every call
        if _default_qopts is None:
            _default_qopts = _make_qopts(*args)
        return _default_qopts
    return _make_qopts(*args)


def _devptr(x, numel: int = 0, device: int = -1, dtype=None) -> Optional[int]:
    """Address of a device output.  A torch tensor must be a contiguous GPU
    tensor of ``dtype`` (float64 by default) on ``device`` holding at least
    ``numel`` elements, since the kernels write that many; a plain int is
    taken as a device address the caller vouches for."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if torch is not None and isinstance(x, torch.Tensor):
        want = torch.float64 if dtype is None else dtype
        if not x.is_cuda or x.dtype != want or not x.is_contiguous():
            raise ValueError(f"device outputs must be contiguous {want} GPU tensors")
        if x.numel() < numel:
            raise ValueError(f"device output holds {x.numel()} elements, the call writes {numel}")
        if device >= 0 and x.device.index != device:
            raise ValueError(f"device output is on cuda:{x.device.index}, the corpus on cuda:{device}")
        return x.data_ptr()
    raise TypeError("device pointer must be an int or a torch tensor")


# (N, device) of each corpus handle, for the checks of the device-output calls
_corpus_shape = {}


def _corpus_nd(corpus: int) -> Tuple[int, int]:
    nd = _corpus_shape.get(corpus)
    if nd is None:
        info = wmd_corpus_info_get(corpus)
        nd = _corpus_shape[corpus] = (int(info["N"]), int(info["device"]))
    return nd


def _query_arrays(qids, qweights):
    q, w = _arr(qids, np.int32), _arr(qweights, np.float32)
    if q.shape != w.shape or q.ndim != 1:
        raise ValueError("query ids and weights must be 1-D of equal length")
    return q, w


def _stream(s) -> Optional[int]:
    if s is None:
        return torch.cuda.current_stream().cuda_stream if torch is not None else None
    if isinstance(s, int):
        return s
    return s.cuda_stream


def wmd_corpus_options_init() -> wmd_corpus_options:
    o = wmd_corpus_options()
    _lib.wmd_corpus_options_init(C.byref(o))
    return o


def wmd_query_options_init() -> wmd_query_options:
    o = wmd_query_options()
    _lib.wmd_query_options_init(C.byref(o))
    return o


def wmd_corpus_create(vecs, doc_ptr, word_ids, weights, device: int = -1, bf16: bool = False) -> int:
    v = _arr(vecs, np.float32)
    if v.ndim != 2:
        raise ValueError("vecs must be V x dim")
    p, ids, w = _arr(doc_ptr, np.int64), _arr(word_ids, np.int32), _arr(weights, np.float32)
    if p.ndim != 1 or p.size < 1 or ids.shape != w.shape or int(p[-1]) > ids.size:
        raise ValueError("doc_ptr / word_ids / weights do not form a CSR")
    o = wmd_corpus_options_init()
    o.device, o.bf16 = int(device), int(bool(bf16))
    h = _P()
    _check(_lib.wmd_corpus_create(_ptr(v, C.c_float), v.shape[0], v.shape[1], _ptr(p, C.c_int64),
                                  _ptr(ids, C.c_int32), _ptr(w, C.c_float), p.size - 1,
                                  C.byref(o), C.byref(h)))
    return h.value


def wmd_corpus_destroy(corpus: int) -> None:
    _corpus_shape.pop(corpus, None)
    _lib.wmd_corpus_destroy(corpus)


def wmd_corpus_info_get(corpus: int) -> dict:
    info = wmd_corpus_info()
    _check(_lib.wmd_corpus_info_get(corpus, C.byref(info)))
    return {f: getattr(info, f) for f, _ in info._fields_}


def wmd_query(corpus: int, qids, qweights, lam: float, iters: int, resid: bool = False,
              **opts) -> Tuple[np.ndarray, Optional[np.ndarray]]:
    q, w = _query_arrays(qids, qweights)
    N = _corpus_nd(corpus)[0]
    out = np.empty(N, np.float64)
    res = np.empty(N, np.float64) if resid else None
    o = _qopts(**opts)
    _check(_lib.wmd_query(corpus, _ptr(q, C.c_int32), _ptr(w, C.c_float), q.size, float(lam), int(iters),
                          C.byref(o), _ptr(out, C.c_double), _ptr(res, C.c_double) if resid else None))
    return out, res


def wmd_query_async(corpus: int, qids, qweights, lam: float, iters: int, dev_dist, dev_resid=None,
                    stream=None, **opts) -> None:
    q, w = _query_arrays(qids, qweights)
    N, dev = _corpus_nd(corpus)
    o = _qopts(**opts)
    _check(_lib.wmd_query_async(corpus, _ptr(q, C.c_int32), _ptr(w, C.c_float), q.size, float(lam),
                                int(iters), C.byref(o), _devptr(dev_dist, N, dev), _devptr(dev_resid, N, dev),
                                _stream(stream)))


def wmd_query_noalloc(corpus: int, qids, qweights, lam: float, iters: int, dev_dist, dev_resid=None,
                      stream=None, **opts) -> None:
    """wmd_query_async without allocation: the workspace is the library's
    fixed per-device scratch array (calls that overlap on one device race)."""
    q, w = _query_arrays(qids, qweights)
    N, dev = _corpus_nd(corpus)
    o = _qopts(**opts)
    _check(_lib.wmd_query_noalloc(corpus, _ptr(q, C.c_int32), _ptr(w, C.c_float), q.size, float(lam),
                                  int(iters), C.byref(o), _devptr(dev_dist, N, dev), _devptr(dev_resid, N, dev),
                                  _stream(stream)))


def _batch_args(queries: Sequence[Tuple[np.ndarray, np.ndarray]], lambdas, iters):
    B = len(queries)
    for b, (qi, qw) in enumerate(queries):
        if np.ndim(qi) != 1 or np.shape(qi) != np.shape(qw):
            raise ValueError(f"query {b}: ids and weights must be 1-D of equal length")
    qp = np.zeros(B + 1, np.int64)
    qp[1:] = np.cumsum([len(q[0]) for q in queries])
    ids = _arr(np.concatenate([np.asarray(q[0]) for q in queries]), np.int32)
    w = _arr(np.concatenate([np.asarray(q[1]) for q in queries]), np.float32)
    lam = _arr(np.broadcast_to(np.asarray(lambdas, np.float32), (B,)), np.float32)
    it = _arr(np.broadcast_to(np.asarray(iters, np.int32), (B,)), np.int32)
    return B, qp, ids, w, lam, it


def wmd_query_batch(corpus: int, queries, lambdas, iters, resid: bool = False, **opts):
    B, qp, ids, w, lam, it = _batch_args(queries, lambdas, iters)
    N = _corpus_nd(corpus)[0]
    out = np.empty((B, N), np.float64)
    res = np.empty((B, N), np.float64) if resid else None
    o = _qopts(**opts)
    _check(_lib.wmd_query_batch(corpus, B, _ptr(qp, C.c_int64), _ptr(ids, C.c_int32), _ptr(w, C.c_float),
                                _ptr(lam, C.c_float), _ptr(it, C.c_int32), C.byref(o),
                                _ptr(out, C.c_double), _ptr(res, C.c_double) if resid else None))
    return out, res


def wmd_query_batch_async(corpus: int, queries, lambdas, iters, dev_dist, dev_resid=None, stream=None,
                          **opts) -> None:
    B, qp, ids, w, lam, it = _batch_args(queries, lambdas, iters)
    N, dev = _corpus_nd(corpus)
    o = _qopts(**opts)
    _check(_lib.wmd_query_batch_async(corpus, B, _ptr(qp, C.c_int64), _ptr(ids, C.c_int32),
                                      _ptr(w, C.c_float), _ptr(lam, C.c_float), _ptr(it, C.c_int32),
                                      C.byref(o), _devptr(dev_dist, B * N, dev), _devptr(dev_resid, B * N, dev),
                                      _stream(stream)))


def wmd_query_adaptive(corpus: int, qids, qweights, lam: float, max_iters: int, tol: float, resid: bool = False,
                       **opts):
    """Convergence-checked query: (distances, residuals or None, x updates per document)."""
    q, w = _query_arrays(qids, qweights)
    N = _corpus_nd(corpus)[0]
    out = np.empty(N, np.float64)
    res = np.empty(N, np.float64) if resid else None
    its = np.empty(N, np.int32)
    o = _qopts(tol=tol, **opts)
    _check(_lib.wmd_query_adaptive(corpus, _ptr(q, C.c_int32), _ptr(w, C.c_float), q.size, float(lam),
                                   int(max_iters), C.byref(o), _ptr(out, C.c_double),
                                   _ptr(res, C.c_double) if resid else None, _ptr(its, C.c_int32)))
    return out, res, its


WMD_MAX_TOPK = 2048


def wmd_query_topk(corpus: int, qids, qweights, lam: float, iters: int, k: int, **opts):
    """(indices, distances) of the k nearest documents, ascending by (distance, index)."""
    q, w = _query_arrays(qids, qweights)
    idx = np.empty(max(int(k), 0), np.int32)
    dist = np.empty(max(int(k), 0), np.float64)
    o = _qopts(**opts)
    _check(_lib.wmd_query_topk(corpus, _ptr(q, C.c_int32), _ptr(w, C.c_float), q.size, float(lam), int(iters),
                               C.byref(o), int(k), _ptr(idx, C.c_int32), _ptr(dist, C.c_double)))
    return idx, dist


def wmd_query_topk_async(corpus: int, qids, qweights, lam: float, iters: int, k: int, dev_idx, dev_dist,
                         stream=None, **opts) -> None:
    q, w = _query_arrays(qids, qweights)
    dev = _corpus_nd(corpus)[1]
    o = _qopts(**opts)
    kk = max(int(k), 0)
    idx_p = _devptr(dev_idx, kk, dev, torch.int32 if torch is not None else None)
    _check(_lib.wmd_query_topk_async(corpus, _ptr(q, C.c_int32), _ptr(w, C.c_float), q.size, float(lam),
                                     int(iters), C.byref(o), int(k), idx_p, _devptr(dev_dist, kk, dev),
                                     _stream(stream)))


def wmd_set_timing(corpus: int, every) -> None:
    """every: False/0 off, True/1 every call, k: every k-th call."""
    _check(_lib.wmd_set_timing(corpus, int(every)))


def wmd_timing_get(corpus: int) -> dict:
    t = wmd_timing()
    _check(_lib.wmd_timing_get(corpus, C.byref(t)))
    return {f: getattr(t, f) for f, _ in t._fields_}


def wmd_server_options_init() -> wmd_server_options:
    o = wmd_server_options()
    _lib.wmd_server_options_init(C.byref(o))
    return o


def wmd_server_create(corpus: int, hbm_budget_bytes: Optional[int] = None, max_batch: Optional[int] = None,
                      max_inflight: Optional[int] = None, want_resid: bool = False,
                      batch_wait_us: int = 0, max_batch_words: Optional[int] = None, step_iters: int = 0,
                      **opts) -> int:
    o = wmd_server_options_init()
    if hbm_budget_bytes is not None:
        o.hbm_budget_bytes = int(hbm_budget_bytes)
    if max_batch is not None:
        o.max_batch = int(max_batch)
    if max_inflight is not None:
        o.max_inflight = int(max_inflight)
    o.want_resid = int(bool(want_resid))
    o.batch_wait_us = int(batch_wait_us)
    if max_batch_words is not None:
        o.max_batch_words = int(max_batch_words)
    o.step_iters = int(step_iters)
    o.query = _qopts(**opts)
    h = _P()
    _check(_lib.wmd_server_create(corpus, C.byref(o), C.byref(h)))
    return h.value


def wmd_server_submit(server: int, qids, qweights, lam: float, iters: int) -> int:
    q, w = _query_arrays(qids, qweights)
    t = _lib.wmd_server_submit(server, _ptr(q, C.c_int32), _ptr(w, C.c_float), q.size, float(lam), int(iters))
    if t < 0:
        raise WmdError(int(t), wmd_last_error())
    return int(t)


def wmd_server_wait(server: int, ticket: int, N: int, resid: bool = False, timeout_us: int = -1):
    out = np.empty(N, np.float64)
    res = np.empty(N, np.float64) if resid else None
    _check(_lib.wmd_server_wait(server, int(ticket), _ptr(out, C.c_double),
                                _ptr(res, C.c_double) if resid else None, int(timeout_us)))
    return out, res


def wmd_server_stats_get(server: int) -> dict:
    st = wmd_server_stats()
    _check(_lib.wmd_server_stats_get(server, C.byref(st)))
    return {f: getattr(st, f) for f, _ in st._fields_}


def wmd_server_stats_reset(server: int) -> None:
    _check(_lib.wmd_server_stats_reset(server))


def wmd_server_destroy(server: int) -> None:
    _lib.wmd_server_destroy(server)


class Corpus:
    """Owning handle: ``Corpus(vecs, doc_ptr, word_ids, weights).query(ids, w, lam, iters)``."""

    def __init__(self, vecs, doc_ptr, word_ids, weights, device: int = -1, bf16: bool = False):
        self.handle = wmd_corpus_create(vecs, doc_ptr, word_ids, weights, device, bf16)
        self.info = wmd_corpus_info_get(self.handle)

    def query(self, qids, qweights, lam, iters, resid=False, **opts):
        return wmd_query(self.handle, qids, qweights, lam, iters, resid, **opts)

    def query_batch(self, queries, lambdas, iters, resid=False, **opts):
        return wmd_query_batch(self.handle, queries, lambdas, iters, resid, **opts)

    def query_adaptive(self, qids, qweights, lam, max_iters, tol, resid=False, **opts):
        return wmd_query_adaptive(self.handle, qids, qweights, lam, max_iters, tol, resid, **opts)

    def topk(self, qids, qweights, lam, iters, k, **opts):
        return wmd_query_topk(self.handle, qids, qweights, lam, iters, k, **opts)

    def close(self):
        if getattr(self, "handle", None):
            wmd_corpus_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Owning handle of a continuous-batching server on a Corpus."""

    def __init__(self, corpus: Corpus, **kw):
        self.corpus = corpus
        self.N = corpus.info["N"]
        self.resid = bool(kw.get("want_resid", False))
        self.handle = wmd_server_create(corpus.handle, **kw)

    def submit(self, qids, qweights, lam, iters) -> int:
        return wmd_server_submit(self.handle, qids, qweights, lam, iters)

    def wait(self, ticket, timeout_us=-1):
        return wmd_server_wait(self.handle, ticket, self.N, self.resid, timeout_us)

    def stats(self) -> dict:
        return wmd_server_stats_get(self.handle)

    def reset_stats(self) -> None:
        wmd_server_stats_reset(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            wmd_server_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
