#!/usr/bin/env python3
"""Write fp64_reference.json: the FP64 oracle's own k-medoids results on the
benchmark's seeded workloads, the values that GPU results in FP32 or BF16 are
compared with (medoid agreement, TD relative error).

Calls only the oracle (PAM BUILD, Alg. 1, then PAM SWAP, Alg. 2, or the
FastPAM2 reading, every distance in FP64 from the points) and the seeded
input generators.  Runs on the host; about ten minutes on eight cores.

    python tests/golden/make_fp64_reference.py [--only NAME]

Workloads:
  gmm16        n = 20000, d = 16, 50 components, k = 100 (PAM and FastPAM2)
  gmm64_n5000  the 64-dimensional, 200-component mixture at n = 5000, k = 200
The 1e5-point workload is left out: one PAM SWAP search there is 5e12 loss
change evaluations in FP64 (hours on the host per search).
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2008_05171_amd import datagen  # noqa: E402

OUT = os.path.join(HERE, "fp64_reference.json")

WORKLOADS = {
    "gmm16": dict(desc="n=20000 d=16, 50 equal components (seed 1002), FP64 Euclidean, k=100",
                  points=lambda: datagen.workload_gmm16(), k=100,
                  variants={"pam": oracle.PAM, "fastpam2": oracle.FASTPAM2}),
    "gmm64_n5000": dict(desc="n=5000 d=64, 200 components, sigma U[0.5,2] (seed 1003), FP64 "
                             "Euclidean, k=200",
                        points=lambda: datagen.workload_gmm64(n=5000), k=200,
                        variants={"pam": oracle.PAM}),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", choices=sorted(WORKLOADS))
    args = ap.parse_args()
    rec = {"what": "FP64 oracle results (BUILD, then SWAP to convergence) on seeded workloads",
           "writer": "tests/golden/make_fp64_reference.py", "workloads": {}}
    if os.path.exists(OUT):
        rec = json.load(open(OUT))
    for name, w in WORKLOADS.items():
        if args.only and name != args.only:
            continue
        X = w["points"]()
        D = oracle.dist_matrix(X, oracle.L2)
        runs = {}
        for vname, variant in w["variants"].items():
            t = time.time()
            r = oracle.pam(w["k"], D=D, variant=variant)
            runs[vname] = {"medoids": [int(m) for m in r.medoids], "td": float(r.td),
                           "td_build": float(r.td_build), "swaps": int(r.swaps),
                           "iterations": int(r.iterations), "converged": r.rc == 0,
                           "host_s": round(time.time() - t, 1)}
            print(name, vname, runs[vname]["td"], runs[vname]["swaps"], runs[vname]["host_s"],
                  flush=True)
        rec["workloads"][name] = {"desc": w["desc"], "n": int(X.shape[0]), "dim": int(X.shape[1]),
                                  "k": w["k"], "runs": runs}
        with open(OUT, "w") as fh:
            json.dump(rec, fh, indent=1)


if __name__ == "__main__":
    main()
