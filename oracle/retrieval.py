"""FP64 CPU oracle: k nearest documents by WMD.

TEST INFRASTRUCTURE ONLY (imported by the tests, never by the product path).

Sec. 3 motivates computing the distances of one query to many documents with
retrieval in mind (the k nearest neighbours under WMD).  Given the distances,
the answer is plain: order the documents by (distance, document index) -- the
index breaks ties so the answer is unique -- and keep the first k.
"""
from __future__ import annotations

import numpy as np

__all__ = ["knn"]


def knn(dist: np.ndarray, k: int):
    """(indices, distances) of the k smallest entries of ``dist``, ascending by
    (distance, index).  A NaN sorts after every number."""
    d = np.asarray(dist, dtype=np.float64)
    if not 1 <= k <= d.size:
        raise ValueError("k outside [1, N]")
    key = np.where(np.isnan(d), np.inf, d)
    nan_last = np.isnan(d).astype(np.int8)
    order = np.lexsort((np.arange(d.size), key, nan_last))[:k]
    return order.astype(np.int64), d[order]
