"""The stored small-workload fixture still matches the generator and the oracle."""
import json
import os

import numpy as np

from oracle import sinkhorn_wmd_sparse
from paper_2005_06727_amd import synth
from tests.golden.make_golden import digest

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c1_oracle.json")


def test_c1_fixture_reproduces():
    g = json.load(open(GOLD))
    wl = synth.make("c1")
    assert digest(wl) == g["inputs_sha256"]
    q, qw = wl.queries[0]
    wmd, resid = sinkhorn_wmd_sparse(wl.vecs, q, qw, wl.doc_ptr, wl.word_ids, wl.weights,
                                     wl.spec.lam, wl.spec.iters)
    np.testing.assert_allclose(wmd, g["wmd"], rtol=1e-13)
    np.testing.assert_allclose(resid, g["resid"], rtol=1e-9, atol=1e-15)
