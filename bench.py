#!/usr/bin/env python3
"""k-medoids benchmark on one MI355X: PAM BUILD + FastPAM1 SWAP.

One step = one whole fit on points already resident in HBM: Euclidean
distance matrix (FP32, Gram term on MFMA), BUILD, FastPAM1 SWAP to
convergence, labels and TD -- every kernel of the hot path.

Workload: n = 20000 points in 16 dimensions from a 50-component isotropic
Gaussian mixture (centers uniform in [-10, 10]^16, sigma 1, seed 1002),
k = 100, stored FP32 matrix (1.6 GB).  Synthetic data (the paper's data sets
are not available).

Reported (one JSON line):
  value            SWAP loss-change pair evaluations per second: candidate-
                   object pairs (n - k) * n per SWAP pass, over the SWAP phase
                   device time of the timed fits
  ms_per_step      wall time of one whole fit
  roofline         SWAP pass kernel: algorithmic bytes 4 * n * (n - k) per
                   launch over its average duration (HIP events on the
                   library's stream), against 8 TB/s HBM; read_probe is a
                   plain read of an n x n FP32 matrix in the pass's launch
                   shape (pamx_read_probe), the rate the access can reach
  cpu_baseline     the CPU oracle (original PAM SWAP, FP64, OpenMP) on a
                   bounded sample of candidates of the same workload

--next fasterpam|init|clarans|starts [--large] times a row beyond the
headline instead (FasterPAM from BUILD; distance-weighted and LAB seeding;
one FastCLARANS search; whole fits for every start x SWAP variant) on this
workload, or with --large on the 1e5 x 32 Zipf mixture (k = 500, 40 GB
matrix), and prints one JSON line of its timings.

--form bf16|clara|eager-large|l1int times one of the other forms on its own
workload and prints one JSON line: the mixed-precision form (n = 50000,
d = 64, 200 components, k = 200, no stored matrix), 256 batched CLARA
instances drawn from 1e6 points in 8 dimensions (also run as 256 separate
single-instance fits, for comparison), eager FastPAM2 on the 1e5 x 32 Zipf
mixture (k = 500, 40 GB matrix), or exact Manhattan distances of n = 1000
integer points (coordinates uniform on {0..999}^2, k = 5).
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
N, DIM, K, COMPONENTS, SEED = 20000, 16, 100, 50, 1002


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


TRAFFIC_JSON = os.path.join(ROOT, "profiles", "swap_pass_gmm16_traffic.json")
# the SWAP pass kernel and the header it shares (its launch shape, the chunk
# length, is recorded with the counters and compared with the timed fits')
KERNEL_SOURCES = ("swap.hip", "pamx_internal.h")


def kernel_sha256():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2008_05171_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def traffic_from_profiles(n, k, chunk):
    """HBM bytes per SWAP pass from committed rocprofv3 counter runs, or None
    when the kernel sources or the chunk length changed since the counters
    were taken."""
    if not os.path.exists(TRAFFIC_JSON):
        return None
    rec = json.load(open(TRAFFIC_JSON))
    if (rec.get("src_sha256") != kernel_sha256() or rec.get("n") != n or rec.get("k") != k
            or rec.get("chunk") != chunk):
        return None
    return float(rec["bytes_per_launch"])


def write_traffic(fetch_csv, write_csv, probe_mib, chunk):
    """Turn two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE; KiB per
    dispatch) of `bench.py --copy-probe-mib M` into the traffic record read by
    traffic_from_profiles.  Each counter is scaled by what it reads for the
    probe's plain copy of M MiB (M MiB read, M MiB written).  SWAP passes
    enqueued after convergence, which return at once, are left out."""
    import csv
    import re

    def per_kernel(path):
        out = {}
        for r in csv.DictReader(open(path)):
            name = re.sub(r"\(.*", "", r["Kernel_Name"]).replace("void ", "").strip()
            out.setdefault(name, []).append(float(r["Counter_Value"]))
        return out

    f, w = per_kernel(fetch_csv), per_kernel(write_csv)
    fetch_scale = probe_mib * 1024.0 / max(f["__amd_rocclr_copyBuffer"])
    write_scale = probe_mib * 1024.0 / max(w["__amd_rocclr_copyBuffer"])
    key = "pamx::k_swap_pass<float, 4, false, false>"   # FastPAM1, full candidate range
    pairs = [(a, b) for a, b in zip(f[key], w[key]) if a > 1024.0]
    fetch_kib = sum(a for a, _ in pairs) / len(pairs)
    write_kib = sum(b for _, b in pairs) / len(pairs)
    rec = {"kernel": key, "n": N, "k": K, "chunk": chunk, "src_sha256": kernel_sha256(),
           "launches": len(pairs), "fetch_kib": fetch_kib, "write_kib": write_kib,
           "fetch_scale": fetch_scale, "write_scale": write_scale,
           "bytes_per_launch": (fetch_kib * fetch_scale + write_kib * write_scale) * 1024.0,
           "algorithmic_bytes_per_launch": 4.0 * N * (N - K)}
    with open(TRAFFIC_JSON, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


def cpu_baseline(X, k, target_s):
    """Original PAM SWAP search (Alg. 2 with Eq. change, FP64) of the oracle
    over a bounded sample of candidates; pairs = candidates * n."""
    import numpy as np
    import oracle
    n = X.shape[0]
    log("cpu baseline: oracle distance matrix (FP64) ...")
    D = oracle.dist_matrix(X.astype(np.float64), oracle.L2)
    rng = np.random.default_rng(SEED)
    med = rng.choice(n, size=k, replace=False).astype(np.int32)
    m0 = 8
    t0 = time.perf_counter()
    oracle.swap_search(med, D=D, c_begin=0, c_end=m0)
    dt0 = time.perf_counter() - t0
    m = int(max(m0, min(n, m0 * target_s / max(dt0, 1e-3))))
    log("cpu baseline: %d candidates x %d objects x %d slots (calibration %.2fs)" % (m, n, k, dt0))
    t0 = time.perf_counter()
    oracle.swap_search(med, D=D, c_begin=0, c_end=m)
    dt = time.perf_counter() - t0
    del D
    return {"value": m * n / dt, "unit": "pair-evals/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "one PAM SWAP search (all %d slots, Eq. change per pair, FP64) over "
                      "candidates 0..%d of the same %d-point workload, %.1f s" % (k, m - 1, n, dt)}


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
            res = px.fit_batched(X, off, idxd, ks)
            s = res.stats
            run = {"pam_ms": s["ms_pam"], "full_td_ms": s["ms_assign"], "pairs": s["pairs"],
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
        X = torch.from_numpy(datagen.workload_gmm64()).cuda()
        k, kw = 200, dict(dist_mode="bf16")
        out["workload"] = "gmm64: n=50000 d=64, 200 components, k=200, BF16 form (no stored matrix)"
    else:
        X = torch.from_numpy(datagen.workload_gmm32_zipf()).cuda()
        k, kw = 500, dict(variant="fastpam2")
        out["workload"] = ("gmm32 zipf: n=100000 d=32, 500 Zipf(1.1)-weighted components, k=500, "
                           "eager FastPAM2 (40 GB matrix)")
    n, dim = X.shape
    opt = px._options(**kw)
    opt.profile = 1
    ws = torch.empty(abi.pamx_workspace_bytes(n, k, dim, abi.PAMX_INPUT_X, abi.PAMX_F32, opt),
                     dtype=torch.uint8, device="cuda")
    med = torch.empty(k, dtype=torch.int32, device="cuda")
    lab = torch.empty(n, dtype=torch.int32, device="cuda")
    for r in range(reps):
        rc, td, st = abi.pamx_fit(X, abi.PAMX_INPUT_X, k, med, lab, ws, opt=opt)
        run = {"rc": rc, "fit_ms": st.ms_total, "dist_ms": st.ms_dist, "build_ms": st.ms_build,
               "swap_ms": st.ms_swap, "searches": st.iterations, "swaps": st.swaps,
               "rescored": st.rescored,
               "swap_pass_ms": st.ms_swap_pass / max(st.n_swap_pass, 1), "td": td}
        out["runs"].append(run)
        log("%s run %d: %s" % (which, r, run))
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fastpam2", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first copy a device buffer of this many MiB three times (a plain copy "
                         "kernel of known size that calibrates HBM byte counters)")
    ap.add_argument("--write-traffic", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "CHUNK"),
                    help="write the SWAP pass traffic record from two rocprofv3 --pmc runs of "
                         "this script with --copy-probe-mib, whose fits used chunk length CHUNK "
                         "(printed as config.chunk; no GPU work)")
    ap.add_argument("--next", choices=("fasterpam", "init", "clarans", "starts"),
                    help="time a row beyond the headline instead (one JSON line)")
    ap.add_argument("--large", action="store_true",
                    help="with --next: the 1e5-point, k=500 workload")
    ap.add_argument("--form", choices=("bf16", "clara", "eager-large", "l1int"),
                    help="time another form on its own workload instead (one JSON line)")
    args = ap.parse_args()
    if args.form:
        run_form(args.form, max(args.steps, 1))
        return
    if args.next:
        run_next(args.next, args.large, max(args.steps, 1))
        return
    if args.write_traffic:
        if args.copy_probe_mib <= 0:
            sys.exit("--write-traffic needs the --copy-probe-mib size of the profiled runs")
        f_csv, w_csv, chunk = args.write_traffic
        print(json.dumps(write_traffic(f_csv, w_csv, args.copy_probe_mib, int(chunk))))
        return
    if args.gpus != 1:
        print("bench.py: one GPU only; --gpus %d is not supported (the path runs on a "
              "single GPU; sharding across GPUs is a design, not built)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2008_05171_amd import datagen
    from paper_2008_05171_amd import pamx as abi

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
    X_np = datagen.gaussian_mixture(N, DIM, COMPONENTS, seed=SEED, sigma=1.0)
    X = torch.from_numpy(X_np).to(dev)

    def make(variant):
        opt = abi.pamx_default_options()
        opt.variant = variant
        opt.profile = 1
        nbytes = abi.pamx_workspace_bytes(N, K, DIM, abi.PAMX_INPUT_X, abi.PAMX_F32, opt)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        med = torch.empty(K, dtype=torch.int32, device=dev)
        lab = torch.empty(N, dtype=torch.int32, device=dev)
        return opt, ws, med, lab

    opt, ws, med, lab = make(abi.PAMX_FASTPAM1)
    stream = torch.cuda.current_stream()

    def step():
        rc, td, st = abi.pamx_fit(X, abi.PAMX_INPUT_X, K, med, lab, ws, metric=abi.PAMX_L2,
                                  opt=opt, stream=stream)
        return rc, td, st

    for w in range(args.warmup):
        step()
        log("warmup %d/%d done" % (w + 1, args.warmup))
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for s in range(args.steps):
        rc, td, st = step()
        stats.append((rc, td, {f: getattr(st, f) for f, _ in abi.pamx_stats._fields_}))
        log("step %d/%d: %.1f ms (dist %.1f, build %.1f, swap %.1f), %d iterations, TD %.6f" % (
            s + 1, args.steps, st.ms_total, st.ms_dist, st.ms_build, st.ms_swap, st.iterations, td))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    swap_pairs = sum(s[2]["pass_pairs"] for s in stats)
    swap_s = sum(s[2]["ms_swap"] for s in stats) / 1e3
    pass_ms = sum(s[2]["ms_swap_pass"] for s in stats)
    n_pass = sum(s[2]["n_swap_pass"] for s in stats)
    bpass_ms = sum(s[2]["ms_build_pass"] for s in stats)
    n_bpass = sum(s[2]["n_build_pass"] for s in stats)
    avg_pass_ms = pass_ms / max(n_pass, 1)
    avg_bpass_ms = bpass_ms / max(n_bpass, 1)
    alg_bytes = 4.0 * N * (N - K)            # D entries of the non-medoid candidates
    achieved = alg_bytes / (avg_pass_ms / 1e3) / 1e9
    build_gbs = 4.0 * N * N / (avg_bpass_ms / 1e3) / 1e9
    chunk = int(stats[-1][2]["chunk"])
    traffic = traffic_from_profiles(N, K, chunk)
    last = stats[-1][2]

    # the reference read: the same bytes in the pass's launch shape, no arithmetic
    ld_fit = (N + 63) // 64 * 64
    Dp = torch.rand(N, ld_fit, dtype=torch.float32, device=dev)
    tiles, nq = (N + 1023) // 1024, (N + chunk - 1) // chunk
    psums = torch.empty(tiles * nq, dtype=torch.float32, device=dev)
    for _ in range(3):
        abi.pamx_read_probe(Dp, chunk, psums, n=N, ld=ld_fit, stream=stream)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    probe_ms = []
    for _ in range(20):
        ev0.record(stream)
        abi.pamx_read_probe(Dp, chunk, psums, n=N, ld=ld_fit, stream=stream)
        ev1.record(stream)
        ev1.synchronize()
        probe_ms.append(ev0.elapsed_time(ev1))
    del Dp, psums
    probe_avg = sum(probe_ms) / len(probe_ms)
    probe_gbs = 4.0 * N * N / (probe_avg / 1e3) / 1e9
    log("read probe: %.1f us per launch, %.0f GB/s" % (probe_avg * 1e3, probe_gbs))

    extra = {}
    if not args.no_fastpam2:
        opt2, ws2, med2, lab2 = make(abi.PAMX_FASTPAM2)
        for _ in range(2):   # the second fit is reported (the first loads its kernels)
            rc2, td2, st2 = abi.pamx_fit(X, abi.PAMX_INPUT_X, K, med2, lab2, ws2,
                                         metric=abi.PAMX_L2, opt=opt2, stream=stream)
        extra = {"fastpam2_eager": {
            "fit_ms": round(st2.ms_total, 3), "swap_ms": round(st2.ms_swap, 3),
            "iterations": st2.iterations, "swaps": st2.swaps, "td": td2,
            "td_rel_vs_fastpam1": (td2 - stats[-1][1]) / stats[-1][1],
            "swap_pass_ms_avg": round(st2.ms_swap_pass / max(st2.n_swap_pass, 1), 4)}}
        del ws2
        log("fastpam2: %.1f ms, %d iterations, %d swaps, TD %.6f" % (
            st2.ms_total, st2.iterations, st2.swaps, td2))

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(X_np, K, args.cpu_seconds)

    out = {
        "metric": "SWAP dTD pair-evals/s + achieved HBM GB/s; end-to-end k-medoids fit time",
        "value": swap_pairs / swap_s,
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "accum_dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "gmm16: n=20000 d=16, 50-component Gaussian mixture, stored FP32 "
                               "Euclidean matrix (1.6 GB), k=100, BUILD init, FastPAM1",
                   "n": N, "dim": DIM, "k": K, "components": COMPONENTS, "seed": SEED,
                   "chunk": chunk, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_swap_pass", "bytes_per_launch": alg_bytes,
                     "avg_launch_ms": avg_pass_ms, "launches": n_pass,
                     "read_probe": {"avg_launch_ms": probe_avg, "achieved": probe_gbs,
                                    "frac": probe_gbs / HBM_PEAK_GBS,
                                    "bytes_per_launch": 4.0 * N * N, "launches": len(probe_ms)},
                     "frac_of_read_probe": achieved / probe_gbs},
        "cpu_baseline": cpu,
        "fit_ms": round(last["ms_total"], 3),
        "phase_ms": {"dist": round(last["ms_dist"], 3), "build": round(last["ms_build"], 3),
                     "swap": round(last["ms_swap"], 3)},
        "iterations": last["iterations"], "swaps": last["swaps"], "td": stats[-1][1],
        "td_build": last["td_build"],
        "build_pass": {"avg_launch_ms": avg_bpass_ms, "achieved_gbs": build_gbs,
                       "bytes_per_launch": 4.0 * N * N, "launches_per_fit": last["n_build_pass"]},
        "build_incremental": {"launches_per_fit": last["n_build_delta"],
                              "rows_read_per_fit": last["build_rows"],
                              "ms_per_fit": round(last["ms_build_delta"], 3),
                              "achieved_gbs": (4.0 * N * last["build_rows"] /
                                               max(last["ms_build_delta"], 1e-9) / 1e6)},
        "swap_pass_pairs_per_s": N * (N - K) / (avg_pass_ms / 1e3),
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
