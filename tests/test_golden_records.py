"""The stored oracle records under tests/golden/ agree with the oracle as it
stands: a few entries are recomputed here (a stale record would fail)."""
import json
import os

import numpy as np

import oracle
from paper_2008_05171_amd import datagen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_clara256_record_matches_oracle():
    rec = json.load(open(os.path.join(GOLDEN, "clara256_int_reference.json")))["instances"]
    assert len(rec) == 256
    Xi = np.rint(datagen.workload_gmm8_pool() * 16.0).astype(np.int32)
    off, idx, ks = datagen.clara_samples(Xi.shape[0], 256, 10, 50, 2000, seed=1004)
    sizes = np.diff(off)
    for j in np.argsort(sizes, kind="stable")[:2]:   # the two smallest samples
        j = int(j)
        sample = idx[off[j]:off[j + 1]]
        ref = oracle.pam(int(ks[j]), D=oracle.dist_matrix(Xi[sample], oracle.L1))
        med = [int(m) for m in sample[np.asarray(ref.medoids)]]
        assert rec[j]["medoids"] == med
        assert rec[j]["td_sample"] == int(ref.td)
        tdf, _ = oracle.td(np.asarray(med), X=Xi, metric=oracle.L1)
        assert rec[j]["td_full"] == int(tdf)
