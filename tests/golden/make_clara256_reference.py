#!/usr/bin/env python3
"""Write clara256_int_reference.json: the oracle's PAM result for every one of
the 256 CLARA instances of the batched workload on its integer pool, the
values the batched GPU run is compared with bit for bit.

The pool is the batched workload's 1e6 points (8 dimensions, seed 1004)
scaled by 16 and rounded to int32; the instances are its 256 seeded samples
(100 to 2000 points, k from 10 to 50).  Distances are exact Manhattan
integers, so every sum is exact and the GPU must give the same medoids
(PAM BUILD, Alg. 1, then PAM SWAP, Alg. 2, ties by (change, slot,
candidate)), the same TD on the sample and the same TD over all 1e6 pool
points.  Calls only the oracle and the seeded input generators; about seven
minutes on eight host cores.

    python tests/golden/make_clara256_reference.py
"""
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2008_05171_amd import datagen  # noqa: E402

OUT = os.path.join(HERE, "clara256_int_reference.json")
SEED = 1004
_POOL = {}


def pool():
    if "X" not in _POOL:
        _POOL["X"] = np.rint(datagen.workload_gmm8_pool() * 16.0).astype(np.int32)
        _POOL["s"] = datagen.clara_samples(_POOL["X"].shape[0], 256, 10, 50, 2000, seed=SEED)
    return _POOL["X"], _POOL["s"]


def one(j):
    Xi, (off, idx, ks) = pool()
    sample = idx[off[j]:off[j + 1]]
    D = oracle.dist_matrix(Xi[sample], oracle.L1)
    ref = oracle.pam(int(ks[j]), D=D)
    med = sample[np.asarray(ref.medoids)]
    tdf, _ = oracle.td(med, X=Xi, metric=oracle.L1)
    return j, [int(m) for m in med], int(ref.td), int(tdf), int(ref.swaps)


def main():
    t0 = time.time()
    with ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        rows = sorted(ex.map(one, range(256)))
    rec = {"what": "oracle PAM (BUILD then SWAP to convergence) on each of the 256 CLARA "
                   "instances; pool = rint(16 * batched workload points), int32 Manhattan",
           "writer": "tests/golden/make_clara256_reference.py",
           "pool": "datagen.workload_gmm8_pool() * 16, rounded; samples: "
                   "datagen.clara_samples(1000000, 256, 10, 50, 2000, seed=1004)",
           "instances": [{"j": j, "medoids": m, "td_sample": td, "td_full": tdf, "swaps": sw}
                         for j, m, td, tdf, sw in rows]}
    with open(OUT, "w") as f:
        json.dump(rec, f, separators=(",", ":"))
        f.write("\n")
    print("wrote", OUT, "in %.0f s" % (time.time() - t0))


if __name__ == "__main__":
    main()
