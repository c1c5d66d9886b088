"""Write tests/golden/c1_oracle.json: the FP64 oracle's distances and
row-marginal residuals on the small synthetic workload (V=2000, w=64, N=100,
one 10-word query, lambda=10, 15 iterations), plus a digest of the inputs.

Calls only the oracle and the seeded input generator.  Run from the repo root:
    python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import sinkhorn_wmd_sparse, sinkhorn_wmd_dense, dense_doc_matrix  # noqa: E402
from paper_2005_06727_amd import synth  # noqa: E402


def digest(wl) -> str:
    h = hashlib.sha256()
    for a in (wl.vecs, wl.doc_ptr, wl.word_ids, wl.weights, *wl.queries[0]):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def main():
    wl = synth.make("c1")
    q, qw = wl.queries[0]
    sp = wl.spec
    wmd, resid = sinkhorn_wmd_sparse(wl.vecs, q, qw, wl.doc_ptr, wl.word_ids, wl.weights,
                                     sp.lam, sp.iters)
    C = dense_doc_matrix(sp.V, wl.doc_ptr, wl.word_ids, wl.weights)
    dense = sinkhorn_wmd_dense(wl.vecs, q, qw, C, sp.lam, sp.iters)
    assert np.allclose(dense, wmd, rtol=1e-12)
    out = {
        "what": "FP64 oracle (sparse form) on the small synthetic workload",
        "cite": "Algorithm 1 and Sec. 4 (SDDMM at nonzeros of c, then SpMM)",
        "workload": {"V": sp.V, "dim": sp.dim, "N": sp.N, "lam": sp.lam, "iters": sp.iters},
        "inputs_sha256": digest(wl),
        "wmd": [float(x) for x in wmd],
        "resid": [float(x) for x in resid],
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
