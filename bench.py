#!/usr/bin/env python3
"""k-medoids benchmark on one MI355X: PAM BUILD + eager FastPAM2 SWAP.

One step = one whole fit on points already resident in HBM: Euclidean
distance matrix (FP32, Gram term on MFMA), BUILD, eager FastPAM2 SWAP to
convergence, labels and TD -- every kernel of the hot path.

Workload (the largest single-GPU configuration): n = 100000 points in 32
dimensions from a 500-component isotropic Gaussian mixture with Zipf(1.1)
component weights (centers uniform in [-10, 10]^32, sigma 1, seed 1005),
k = 500, stored FP32 matrix (40 GB).  Synthetic data (the paper's data sets
are not available).

Reported (one JSON line):
  value            SWAP loss-change pair evaluations per second: candidate-
                   object pairs (n - k) * n per SWAP search, over the SWAP
                   phase device time of the timed fits
  ms_per_step      wall time of one whole fit
  roofline         the FastPAM2 SWAP pass kernel: algorithmic bytes
                   4 * n * (n - k) per launch over its average duration (HIP
                   events on the library's stream), against 8 TB/s HBM;
                   read_probe is a plain read of an n x n FP32 matrix in the
                   pass's launch shape (pamx_read_probe), the rate the access
                   can reach; traffic = HBM bytes per launch from committed
                   rocprofv3 counter runs, while the kernel is unchanged
  cpu_baseline     the CPU oracle (the Eq. change sums of a PAM SWAP search,
                   FP64, distances from the points) on a bounded sample of
                   candidates of the same workload, all host threads and one
  gmm16            the 20000-point, k = 100 workload (FastPAM1 and eager
                   FastPAM2), with medoid agreement and TD relative error
                   against the FP64 oracle's own results on it
  paper            the paper's SWAP speedups with its stated hardware, beside
                   this run's search time against the oracle's

--next fasterpam|init|clarans|starts [--large] times a row beyond the
headline instead (FasterPAM from BUILD; distance-weighted and LAB seeding;
one FastCLARANS search; whole fits for every start x SWAP variant) on the
20000-point workload, or with --large on the 1e5-point one, and prints one
JSON line of its timings.

--form bf16|clara|gmm16|l1int times one of the other forms on its own
workload and prints one JSON line: the mixed-precision form (n = 50000,
d = 64, 200 components, k = 200, no stored matrix; and at n = 5000 against
the FP64 oracle's result), 256 batched CLARA instances drawn from 1e6 points
in 8 dimensions (also run as 256 separate single-instance fits, for
comparison), FastPAM1 on the 20000-point workload, or exact Manhattan
distances of n = 1000 integer points (coordinates uniform on {0..999}^2,
k = 5).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# headline workload: 1e5 x 32, 500 Zipf(1.1)-weighted components, k = 500
N5, DIM5, K5, SEED5 = 100000, 32, 500, 1005
# the 20000-point workload (extra keys, --form gmm16, --next)
N, DIM, K, COMPONENTS, SEED = 20000, 16, 100, 50, 1002

PAPER = {
    "swap_speedup_vs_pam": {"k100": 458, "k200": 1191},
    "what": "FasterPAM SWAP against the original PAM SWAP (the abstract; Sec. 4.4: 100plants, "
            "n = 1600, BUILD start, k = 200); O(k) fewer loss-change evaluations per search "
            "plus eager swaps, same implementation and machine on both sides",
    "hardware": "Java (ELKI) on Intel Xeon E5-2697v2 CPUs at 2.70 GHz, thread count not stated",
}
REFERENCE_JSON = os.path.join(ROOT, "tests", "golden", "fp64_reference.json")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# HBM traffic records from rocprofv3 counter runs, one per timed pass kernel
TRAFFIC = {
    "fastpam2_gmm32": (os.path.join(ROOT, "profiles", "swap_pass_fastpam2_gmm32_traffic.json"),
                       "pamx::k_swap_pass<float, 4, true, false, true>", N5, K5),
    "fastpam1_gmm16": (os.path.join(ROOT, "profiles", "swap_pass_gmm16_traffic.json"),
                       "pamx::k_swap_pass<float, 4, false, false, false>", N, K),
}
# the SWAP pass kernel and the header it shares (its launch shape, the chunk
# length, is recorded with the counters and compared with the timed fits')
KERNEL_SOURCES = ("swap.hip", "pamx_internal.h")


def kernel_sha256():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2008_05171_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def traffic_from_profiles(which, chunk):
    """HBM bytes per SWAP pass from committed rocprofv3 counter runs, or None
    when the kernel sources or the chunk length changed since the counters
    were taken."""
    path, _, n, k = TRAFFIC[which]
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if (rec.get("src_sha256") != kernel_sha256() or rec.get("n") != n or rec.get("k") != k
            or rec.get("chunk") != chunk):
        return None
    return float(rec["bytes_per_launch"])


def write_traffic(which, fetch_csv, write_csv, probe_mib, chunk):
    """Turn two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE; KiB per
    dispatch) of this script with --copy-probe-mib M into the traffic record
    read by traffic_from_profiles.  Each counter is scaled by what it reads
    for the probe's plain copy of M MiB (M MiB read, M MiB written).  SWAP
    passes enqueued after convergence, which return at once, are left out."""
    import csv
    import re

    def per_kernel(path):
        out = {}
        for r in csv.DictReader(open(path)):
            name = re.sub(r"\(.*", "", r["Kernel_Name"]).replace("void ", "").strip()
            out.setdefault(name, []).append(float(r["Counter_Value"]))
        return out

    path, key, n, k = TRAFFIC[which]
    f, w = per_kernel(fetch_csv), per_kernel(write_csv)
    fetch_scale = probe_mib * 1024.0 / max(f["__amd_rocclr_copyBuffer"])
    write_scale = probe_mib * 1024.0 / max(w["__amd_rocclr_copyBuffer"])
    pairs = [(a, b) for a, b in zip(f[key], w[key]) if a > 1024.0]
    fetch_kib = sum(a for a, _ in pairs) / len(pairs)
    write_kib = sum(b for _, b in pairs) / len(pairs)
    rec = {"kernel": key, "n": n, "k": k, "chunk": chunk, "src_sha256": kernel_sha256(),
           "launches": len(pairs), "fetch_kib": fetch_kib, "write_kib": write_kib,
           "fetch_scale": fetch_scale, "write_scale": write_scale,
           "bytes_per_launch": (fetch_kib * fetch_scale + write_kib * write_scale) * 1024.0,
           "algorithmic_bytes_per_launch": 4.0 * n * (n - k)}
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


def cpu_baseline(X, k, target_s):
    """The oracle's PAM SWAP search arithmetic (Alg. 2: Eq. change summed over
    the objects for every slot of every candidate, FP64, distances computed
    from the points) over a bounded sample of candidates, with all host
    threads and with one.  A pair is a (candidate, object) pair with all k
    slots evaluated, the unit of the GPU rate.  The nearest / second-nearest
    set-up of a search (2 n k distances) is timed alone and left out."""
    import numpy as np
    import oracle
    n = X.shape[0]
    X64 = X.astype(np.float64)
    rng = np.random.default_rng(SEED5)
    perm = rng.permutation(n)
    med, cand = perm[:k].astype(np.int32), np.sort(perm[k:])
    all_threads = oracle.num_threads()
    out = {}
    for threads in (all_threads, 1):
        oracle.set_num_threads(threads)
        t0 = time.perf_counter()
        oracle.swap_list(med, cand[:0], X=X64)
        setup = time.perf_counter() - t0
        m0 = max(2, threads)
        t0 = time.perf_counter()
        oracle.swap_list(med, cand[:m0], X=X64)
        dt0 = max(time.perf_counter() - t0 - setup, 1e-3)
        m = int(max(m0, min(len(cand), m0 * target_s / dt0)))
        t0 = time.perf_counter()
        oracle.swap_list(med, cand[:m], X=X64)
        dt = max(time.perf_counter() - t0 - setup, 1e-6)
        out[threads] = (m * n / dt, m, dt, setup)
        log("cpu baseline: %d thread(s): %d candidates x %d objects x %d slots in %.1f s "
            "(+%.1f s set-up): %.3g pair-evals/s" % (threads, m, n, k, dt, setup, m * n / dt))
    oracle.set_num_threads(all_threads)
    v, m, dt, setup = out[all_threads]
    v1, m1, dt1, setup1 = out[1]
    return {"value": v, "unit": "pair-evals/s", "cores": all_threads, "kind": "oracle",
            "value_1_thread": v1,
            "sample": "Eq. change sums of a PAM SWAP search (all %d slots per pair, FP64, "
                      "distances from the points) for the first %d (%d threads) and %d (1 "
                      "thread) non-medoid candidates of a seeded random medoid set on the "
                      "same %d-point workload: %.1f s and %.1f s, plus %.1f s and %.1f s of "
                      "nearest / second-nearest set-up, not counted"
                      % (k, m, all_threads, m1, n, dt, dt1, setup, setup1)}


def fp64_agreement(name, variant, medoids, td):
    """Medoid agreement and TD relative error of a GPU result against the
    FP64 oracle's own result on the same workload (committed record written
    by tests/golden/make_fp64_reference.py), or None without that record."""
    if not os.path.exists(REFERENCE_JSON):
        return None
    ref = json.load(open(REFERENCE_JSON))["workloads"].get(name)
    if ref is None or variant not in ref["runs"]:
        return None
    r = ref["runs"][variant]
    a, b = set(int(v) for v in medoids), set(r["medoids"])
    return {"fp64_td": r["td"], "td_rel_err": (td - r["td"]) / r["td"],
            "medoids_shared": len(a & b), "k": len(b), "jaccard": len(a & b) / len(a | b),
            "same_set": a == b, "fp64_swaps": r["swaps"]}


def run_next(which, large, reps):
    """Time one of the rows beyond the headline (see the module docstring)."""
    import torch
    import paper_2008_05171_amd as px
    from paper_2008_05171_amd import datagen
    if large:
        X = torch.from_numpy(datagen.workload_gmm32_zipf()).cuda()
        k, name = 500, "gmm32 zipf: n=100000 d=32, 500 Zipf(1.1)-weighted components, k=500"
    else:
        X = torch.from_numpy(datagen.gaussian_mixture(N, DIM, COMPONENTS, seed=SEED)).cuda()
        k, name = K, "gmm16: n=20000 d=16, 50 components, k=100"
    out = {"next": which, "workload": name, "runs": []}
    if which == "starts":
        # whole fits from the points; the second of two runs is reported
        # (one run each at 1e5 points, where a slow combination takes seconds)
        variants = ("fastpam1", "fastpam2", "fasterpam")
        combos = [(i, v) for i in ("build", "random", "dw", "lab") for v in variants]
        if large:
            combos = [c for c in combos if c not in (("random", "fastpam1"), ("dw", "fastpam1"),
                                                     ("lab", "fastpam1"), ("lab", "fastpam2"))]
        for init, v in combos:
            for _ in range(1 if large else 2):
                torch.cuda.synchronize()
                t = time.perf_counter()
                res = px.fit(X, k, init=init, variant=v, seed=3)
                torch.cuda.synchronize()
                wall = (time.perf_counter() - t) * 1e3
            s = res.stats
            run = {"start": init, "variant": v, "wall_ms": wall, "start_ms": s["ms_build"],
                   "swap_ms": s["ms_swap"], "swaps": s["swaps"], "td": res.td}
            out["runs"].append(run)
            log("starts: %s" % run)
        print(json.dumps(out))
        return
    D = px.dist(X) if which in ("init", "clarans") else None
    for r in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        if which == "fasterpam":
            res = px.fit(X, k, variant="fasterpam")
            torch.cuda.synchronize()
            s = res.stats
            run = {"fit_ms": s["ms_total"], "swap_ms": s["ms_swap"], "windows": s["windows"],
                   "swaps": s["swaps"], "passes": s["iterations"], "td": res.td}
        elif which == "init":
            px.init_dw(D, k, seed=1)
            torch.cuda.synchronize()
            a = time.perf_counter()
            px.init_lab(D, k, seed=1)
            torch.cuda.synchronize()
            run = {"dw_ms": (a - t) * 1e3, "lab_ms": (time.perf_counter() - a) * 1e3}
        else:
            res = px.clarans(D, k, numlocal=1, seed=1)
            torch.cuda.synchronize()
            s = res.stats
            run = {"search_ms": s["ms_swap"], "windows": s["windows"], "swaps": s["swaps"],
                   "draws_evaluated": s["scan_positions"], "td": res.td}
        run["wall_ms"] = (time.perf_counter() - t) * 1e3
        out["runs"].append(run)
        log("%s run %d: %s" % (which, r, run))
    print(json.dumps(out))


def run_form(which, reps):
    """Time one of the other forms on its workload (see the module docstring)."""
    import torch
    import paper_2008_05171_amd as px
    from paper_2008_05171_amd import datagen
    from paper_2008_05171_amd import pamx as abi
    out = {"form": which, "runs": []}
    if which == "clara":
        Xh = datagen.workload_gmm8_pool()
        off, idx, ks = datagen.clara_samples(Xh.shape[0], 256, 10, 50, 2000, seed=1004)
        X = torch.from_numpy(Xh).cuda()
        idxd = torch.from_numpy(idx).cuda()
        out["workload"] = ("gmm8 pool: 1e6 points d=8, 100 components; 256 CLARA instances, "
                           "k ~ U{10..50}, n' ~ U{40+2k..2000}")
        for r in range(reps):
            # team sizes timed on the first call (the fastest kept)
            res = px.fit_batched(X, off, idxd, ks, tune=True)
            s = res.stats
            run = {"pam_ms": s["ms_pam"], "full_td_ms": s["ms_assign"], "pairs": s["pairs"],
                   "team_scale": s["team_scale"],
                   "pair_evals_per_s": s["pairs"] / (s["ms_pam"] / 1e3),
                   "iterations": s["iterations"], "swaps": s["swaps"], "best": res.best,
                   "td_full_best": res.td_full[res.best]}
            out["runs"].append(run)
            log("clara run %d: %s" % (r, run))
        # the same instances as separate fits (one pamx_fit per instance, the
        # stored-matrix path on the sample's points)
        torch.cuda.synchronize()
        t = time.perf_counter()
        same = 0
        for j in range(len(ks)):
            sample = idxd[int(off[j]):int(off[j + 1])].long()
            fr = px.fit(X[sample].contiguous(), int(ks[j]))
            same += int(set(sample[fr.medoids.long()].tolist()) == set(res.medoids[j].tolist()))
        torch.cuda.synchronize()
        out["separate_fits"] = {"ms": (time.perf_counter() - t) * 1e3,
                                "same_medoid_sets": same, "instances": len(ks)}
        log("separate fits: %s" % out["separate_fits"])
        print(json.dumps(out))
        return
    if which == "l1int":
        out["workload"] = "l1 int: n=1000 d=2, coordinates uniform on {0..999}, k=5, exact Manhattan"
        for seed in range(1001, 1001 + reps):
            Xi = torch.from_numpy(datagen.int_points(1000, 2, 0, 1000, seed=seed)).cuda()
            opt = px._options()
            opt.profile = 1
            ws = torch.empty(abi.pamx_workspace_bytes(1000, 5, 2, abi.PAMX_INPUT_X, abi.PAMX_I32,
                                                      opt), dtype=torch.uint8, device="cuda")
            med = torch.empty(5, dtype=torch.int32, device="cuda")
            lab = torch.empty(1000, dtype=torch.int32, device="cuda")
            for _ in range(2):   # the second fit is reported
                rc, td, st = abi.pamx_fit(Xi, abi.PAMX_INPUT_X, 5, med, lab, ws,
                                          metric=abi.PAMX_L1, opt=opt)
            us = 1e3 * st.ms_swap_pass / max(st.n_swap_pass, 1)
            run = {"seed": seed, "rc": rc, "fit_ms": st.ms_total, "searches": st.iterations,
                   "swaps": st.swaps, "us_per_pass": us,
                   "pair_evals_per_s": 1000 * 995 / (us * 1e-6), "td": td}
            out["runs"].append(run)
            log("l1int: %s" % run)
        print(json.dumps(out))
        return
    if which == "bf16":
        out["workload"] = ("gmm64: n=50000 d=64, 200 components, k=200, BF16 form (no stored "
                           "matrix): FP32 loss-change sums, FP64 re-scoring of near-ties")
        X = torch.from_numpy(datagen.workload_gmm64()).cuda()
        stats, td, med = fits(X, 200, "fastpam1", reps, 0, dist_mode="bf16", accum="f32")
        out["runs"] = [run_summary(st, t) for st, t in zip(stats, td)]
        # the same form with FP64 sums
        st64, td64, med64 = fits(X, 200, "fastpam1", 1, 0, dist_mode="bf16")
        out["fp64_sums"] = dict(run_summary(st64[-1], td64[-1]),
                                same_medoids=set(med64.tolist()) == set(med.tolist()))
        # the plain FP32 path (stored 10 GB matrix) on the same points
        st32, td32, med32 = fits(X, 200, "fastpam1", 1, 0)
        a, b = set(med.tolist()), set(med32.tolist())
        out["vs_stored_fp32"] = {"fit_ms": st32[-1]["ms_total"], "td": td32[-1],
                                 "td_rel_diff": (td[-1] - td32[-1]) / td32[-1],
                                 "medoids_shared": len(a & b), "same_set": a == b}
        del X
        torch.cuda.empty_cache()
        # at n = 5000 against the FP64 oracle's own result
        Xs = torch.from_numpy(datagen.workload_gmm64(n=5000)).cuda()
        sts, tds, meds = fits(Xs, 200, "fastpam1", 1, 1, dist_mode="bf16", accum="f32")
        out["n5000_vs_fp64_oracle"] = dict(fp64_agreement("gmm64_n5000", "pam", meds.tolist(),
                                                          tds[-1]) or {},
                                           swaps=sts[-1]["swaps"], rescored=sts[-1]["rescored"])
        log("bf16: %s" % out)
        print(json.dumps(out))
        return
    # the 20000-point workload, FastPAM1
    out["workload"] = "gmm16: n=20000 d=16, 50 components, k=100, FastPAM1 (1.6 GB matrix)"
    X = torch.from_numpy(datagen.workload_gmm16()).cuda()
    stats, td, med = fits(X, K, "fastpam1", reps, 1)
    out["runs"] = [run_summary(st, t) for st, t in zip(stats, td)]
    out["vs_fp64_oracle"] = fp64_agreement("gmm16", "pam", med.tolist(), td[-1])
    print(json.dumps(out))


def fits(X, k, variant, steps, warmup, dist_mode="stored", stream=None, on_step=None,
         accum="f64"):
    """`warmup` untimed then `steps` whole fits of the points X (profiling
    events on); returns (per-fit stats dicts, TDs, medoids of the last fit).
    accum: "f64" or "f32" loss-change sums (FP32 only with dist_mode bf16)."""
    import torch
    import paper_2008_05171_amd as px
    from paper_2008_05171_amd import pamx as abi
    n, dim = X.shape
    opt = px._options(variant=variant, dist_mode=dist_mode,
                      accum=px.PAMX_ACC_F32 if accum == "f32" else px.PAMX_ACC_F64)
    opt.profile = 1
    nbytes = abi.pamx_workspace_bytes(n, k, dim, abi.PAMX_INPUT_X, abi.PAMX_F32, opt)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=X.device)
    med = torch.empty(k, dtype=torch.int32, device=X.device)
    lab = torch.empty(n, dtype=torch.int32, device=X.device)
    stats, tds = [], []
    for j in range(warmup + steps):
        rc, td, st = abi.pamx_fit(X, abi.PAMX_INPUT_X, k, med, lab, ws, metric=abi.PAMX_L2,
                                  opt=opt, stream=stream)
        if rc != 0:
            raise RuntimeError("pamx_fit returned %d" % rc)
        if j >= warmup:
            stats.append({f: getattr(st, f) for f, _ in abi.pamx_stats._fields_})
            tds.append(td)
        if on_step:
            on_step(j, warmup, st, td)
    out = med.cpu()
    del ws
    return stats, tds, out


def run_summary(st, td):
    return {"fit_ms": st["ms_total"], "dist_ms": st["ms_dist"], "build_ms": st["ms_build"],
            "swap_ms": st["ms_swap"], "searches": st["iterations"], "swaps": st["swaps"],
            "rescored": st["rescored"],
            "swap_pass_ms": st["ms_swap_pass"] / max(st["n_swap_pass"], 1), "td": td}


def pass_roofline(stats, n, k, which):
    """roofline of the SWAP pass over the timed fits."""
    pass_ms = sum(s["ms_swap_pass"] for s in stats)
    n_pass = sum(s["n_swap_pass"] for s in stats)
    avg = pass_ms / max(n_pass, 1)
    alg = 4.0 * n * (n - k)                  # FP32 entries of the non-medoid candidates
    achieved = alg / (avg / 1e3) / 1e9
    _, key, _, _ = TRAFFIC[which]
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic_from_profiles(which, int(stats[-1]["chunk"])),
            "kernel": key.replace("pamx::", ""), "bytes_per_launch": alg, "avg_launch_ms": avg,
            "launches": n_pass}


def read_probe(n, chunk, stream, launches=10):
    """Average duration of pamx_read_probe over an n x n FP32 matrix (row
    stride rounded up to 64, as the fit stores it) in the pass's shape."""
    import torch
    from paper_2008_05171_amd import pamx as abi
    ld = (n + 63) // 64 * 64
    Dp = torch.ones(n, ld, dtype=torch.float32, device="cuda")
    tiles, nq = (n + 1023) // 1024, (n + chunk - 1) // chunk
    psums = torch.empty(tiles * nq, dtype=torch.float32, device="cuda")
    for _ in range(2):
        abi.pamx_read_probe(Dp, chunk, psums, n=n, ld=ld, stream=stream)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms = []
    for _ in range(launches):
        ev0.record(stream)
        abi.pamx_read_probe(Dp, chunk, psums, n=n, ld=ld, stream=stream)
        ev1.record(stream)
        ev1.synchronize()
        ms.append(ev0.elapsed_time(ev1))
    del Dp, psums
    torch.cuda.empty_cache()
    avg = sum(ms) / len(ms)
    gbs = 4.0 * n * n / (avg / 1e3) / 1e9
    return {"avg_launch_ms": avg, "achieved": gbs, "frac": gbs / HBM_PEAK_GBS,
            "bytes_per_launch": 4.0 * n * n, "launches": len(ms)}


def write_probe(n, stream, launches=10):
    """Average duration of pamx_write_probe over an n x n FP32 matrix (row
    stride rounded up to 64, as the fit stores it): the distance kernel's
    stores alone, in its launch shape."""
    import torch
    from paper_2008_05171_amd import pamx as abi
    ld = (n + 63) // 64 * 64
    Dp = torch.empty(n, ld, dtype=torch.float32, device="cuda")
    for _ in range(2):
        abi.pamx_write_probe(Dp, 1.0, n=n, ld=ld, stream=stream)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms = []
    for _ in range(launches):
        ev0.record(stream)
        abi.pamx_write_probe(Dp, 1.0, n=n, ld=ld, stream=stream)
        ev1.record(stream)
        ev1.synchronize()
        ms.append(ev0.elapsed_time(ev1))
    # a plain fill of the same matrix by torch (16-byte stores along the rows)
    fill = []
    for _ in range(3):
        ev0.record(stream)
        Dp.fill_(2.0)
        ev1.record(stream)
        ev1.synchronize()
        fill.append(ev0.elapsed_time(ev1))
    del Dp
    torch.cuda.empty_cache()
    avg = sum(ms) / len(ms)
    gbs = 4.0 * n * n / (avg / 1e3) / 1e9
    fgbs = 4.0 * n * ld / (min(fill) / 1e3) / 1e9
    return {"avg_launch_ms": avg, "achieved": gbs, "frac": gbs / HBM_PEAK_GBS,
            "bytes_per_launch": 4.0 * n * n, "launches": len(ms),
            "torch_fill_gbs": fgbs}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=6.0,
                    help="target seconds of each cpu_baseline sample (all threads, one thread)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline fits (no read probe, no 20000-point workload)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first copy a device buffer of this many MiB three times (a plain copy "
                         "kernel of known size that calibrates HBM byte counters)")
    ap.add_argument("--write-traffic", nargs=4,
                    metavar=("WHICH", "FETCH_CSV", "WRITE_CSV", "CHUNK"),
                    help="write a SWAP pass traffic record (WHICH: %s) from two rocprofv3 --pmc "
                         "runs of this script with --copy-probe-mib, whose fits used chunk "
                         "length CHUNK (printed as config.chunk; no GPU work)" % ", ".join(TRAFFIC))
    ap.add_argument("--next", choices=("fasterpam", "init", "clarans", "starts"),
                    help="time a row beyond the headline instead (one JSON line)")
    ap.add_argument("--large", action="store_true",
                    help="with --next: the 1e5-point, k=500 workload")
    ap.add_argument("--form", choices=("bf16", "clara", "gmm16", "l1int"),
                    help="time another form on its own workload instead (one JSON line)")
    args = ap.parse_args()
    if args.write_traffic:
        if args.copy_probe_mib <= 0:
            sys.exit("--write-traffic needs the --copy-probe-mib size of the profiled runs")
        which, f_csv, w_csv, chunk = args.write_traffic
        print(json.dumps(write_traffic(which, f_csv, w_csv, args.copy_probe_mib, int(chunk))))
        return
    if args.gpus != 1:
        print("bench.py: one GPU only; --gpus %d is not supported (the path runs on a "
              "single GPU; sharding across GPUs is a design, not built)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.form:
        run_form(args.form, max(args.steps, 1))
        return
    if args.next:
        run_next(args.next, args.large, max(args.steps, 1))
        return

    import torch
    from paper_2008_05171_amd import datagen

    dev = torch.device("cuda:0")
    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: 3 copies of %d MiB (read %d + write %d bytes each)" % (
            args.copy_probe_mib, src.numel() * 4, src.numel() * 4))
        del src, dst
    X_np = datagen.workload_gmm32_zipf()
    X = torch.from_numpy(X_np).to(dev)
    stream = torch.cuda.current_stream()

    def on_step(j, warmup, st, td):
        tag = "warmup %d/%d" % (j + 1, warmup) if j < warmup else "step %d/%d" % (
            j - warmup + 1, args.steps)
        log("%s: %.1f ms (dist %.1f, build %.1f, swap %.1f), %d searches, %d swaps, TD %.6f" % (
            tag, st.ms_total, st.ms_dist, st.ms_build, st.ms_swap, st.iterations, st.swaps, td))

    # warm-up fits first, then the timed ones (the same workspace throughout)
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    walls = []

    def timed(j, warmup, st, td):
        on_step(j, warmup, st, td)
        torch.cuda.synchronize()
        walls.append(time.perf_counter())

    stats, tds, med = fits(X, K5, "fastpam2", args.steps, args.warmup, stream=stream,
                           on_step=timed)
    torch.cuda.synchronize()
    marks = [t_all] + walls
    ms_steps = [(marks[i + 1] - marks[i]) * 1e3 for i in range(args.warmup, len(walls))]
    ms_per_step = sum(ms_steps) / max(len(ms_steps), 1)
    last = stats[-1]
    swap_pairs = sum(s["pass_pairs"] for s in stats)
    swap_s = sum(s["ms_swap"] for s in stats) / 1e3
    roof = pass_roofline(stats, N5, K5, "fastpam2_gmm32")
    chunk = int(last["chunk"])
    avg_bpass = sum(s["ms_build_pass"] for s in stats) / max(sum(s["n_build_pass"] for s in stats), 1)
    out = {
        "metric": "SWAP dTD pair-evals/s + achieved HBM GB/s; end-to-end k-medoids fit time",
        "value": swap_pairs / swap_s,
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "accum_dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "gmm32 zipf: n=100000 d=32, 500-component Gaussian mixture with "
                               "Zipf(1.1) weights, stored FP32 Euclidean matrix (40 GB), k=500, "
                               "BUILD init, eager FastPAM2 to convergence",
                   "n": N5, "dim": DIM5, "k": K5, "components": 500, "zipf_s": 1.1,
                   "seed": SEED5, "variant": "fastpam2", "chunk": chunk,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": None,
        "fit_ms": round(last["ms_total"], 3),
        "phase_ms": {"dist": round(last["ms_dist"], 3), "build": round(last["ms_build"], 3),
                     "swap": round(last["ms_swap"], 3)},
        "searches": last["iterations"], "swaps": last["swaps"], "td": tds[-1],
        "td_build": last["td_build"],
        "swap_pass_pairs_per_s": N5 * (N5 - K5) / (roof["avg_launch_ms"] / 1e3),
        "build_pass": {"avg_launch_ms": avg_bpass,
                       "achieved_gbs": 4.0 * N5 * N5 / (avg_bpass / 1e3) / 1e9,
                       "launches_per_fit": last["n_build_pass"]},
        "build_incremental": {"launches_per_fit": last["n_build_delta"],
                              "rows_read_per_fit": last["build_rows"],
                              "ms_per_fit": round(last["ms_build_delta"], 3)},
    }
    med_np = med.numpy()
    del X
    torch.cuda.empty_cache()

    if not args.no_extras:
        probe = read_probe(N5, chunk, stream)
        roof["read_probe"] = probe
        roof["frac_of_read_probe"] = roof["achieved"] / probe["achieved"]
        log("read probe: %.3f ms per launch, %.0f GB/s" % (probe["avg_launch_ms"],
                                                           probe["achieved"]))
        # the distance kernel (its phase: mean + Gram kernel) against its stores alone
        wp = write_probe(N5, stream)
        dist_ms = sum(s["ms_dist"] for s in stats) / len(stats)
        dist_gbs = 4.0 * N5 * N5 / (dist_ms / 1e3) / 1e9
        out["distance_roofline"] = {
            "bound": "hbm", "kernel": "k_dist_l2_f32_upper<32> (with k_center_mean)",
            "achieved": dist_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": dist_gbs / HBM_PEAK_GBS, "avg_ms": dist_ms, "bytes": 4.0 * N5 * N5,
            "mfma_flops": 2.0 * DIM5 * N5 * N5, "write_probe": wp,
            "frac_of_write_probe": dist_gbs / wp["achieved"]}
        log("write probe: %.3f ms per launch, %.0f GB/s; distances %.3f ms, %.0f GB/s" % (
            wp["avg_launch_ms"], wp["achieved"], dist_ms, dist_gbs))
        Xc = torch.from_numpy(datagen.workload_gmm16()).to(dev)
        g = {"workload": "gmm16: n=20000 d=16, 50 equal components, stored FP32 matrix (1.6 GB), "
                         "k=100, BUILD init"}
        for variant in ("fastpam1", "fastpam2"):
            st2, td2, m2 = fits(Xc, K, variant, 5, 1, stream=stream)
            which = "fastpam1_gmm16" if variant == "fastpam1" else None
            r = {"fit_ms": st2[-1]["ms_total"], "swap_ms": st2[-1]["ms_swap"],
                 "searches": st2[-1]["iterations"], "swaps": st2[-1]["swaps"], "td": td2[-1],
                 "value": sum(s["pass_pairs"] for s in st2) / (sum(s["ms_swap"] for s in st2) / 1e3),
                 "vs_fp64_oracle": fp64_agreement("gmm16", "pam" if variant == "fastpam1"
                                                  else "fastpam2", m2.tolist(), td2[-1])}
            if which:
                r["roofline"] = pass_roofline(st2, N, K, which)
            else:
                p = sum(s["ms_swap_pass"] for s in st2) / max(sum(s["n_swap_pass"] for s in st2), 1)
                r["swap_pass_ms_avg"] = p
            g[variant] = r
            log("gmm16 %s: %s" % (variant, r))
        out["gmm16"] = g
        del Xc
        torch.cuda.empty_cache()

    if not args.no_cpu_baseline:
        cpu = cpu_baseline(X_np, K5, args.cpu_seconds)
        out["cpu_baseline"] = cpu
        gpu_search_s = sum(s["ms_swap"] for s in stats) / 1e3 / sum(s["iterations"] for s in stats)
        orc_search_s = N5 * (N5 - K5) / cpu["value"]
        out["paper"] = dict(PAPER, this_run={
            "gpu_fastpam2_search_ms": gpu_search_s * 1e3,
            "oracle_pam_search_s": orc_search_s,
            "oracle_pam_search_s_1_thread": N5 * (N5 - K5) / cpu["value_1_thread"],
            "search_speedup_vs_oracle": orc_search_s / gpu_search_s,
            "note": "one SWAP search of the GPU (pass, reductions, eager apply) against the "
                    "oracle's PAM search arithmetic over all (n - k) candidates, extrapolated from "
                    "its sample (cpu_baseline); both evaluate every slot of every pair"})
    out["medoids_sha"] = hashlib.sha256(med_np.tobytes()).hexdigest()[:16]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
