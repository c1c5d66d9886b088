"""FP64 CPU oracle for sparse Sinkhorn WMD.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.  It shares no
code with the GPU library.
"""
from .sinkhorn_wmd import (  # noqa: F401
    query_histogram, doc_histograms, dense_doc_matrix, word_distances,
    sinkhorn_wmd_dense, sinkhorn_wmd_sparse,
)
from .retrieval import knn  # noqa: F401
from .sinkhorn_lse import sinkhorn_wmd_lse, sinkhorn_lse_core  # noqa: F401
