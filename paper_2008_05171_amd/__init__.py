"""MI355X-native k-medoids: PAM BUILD with FastPAM1 / eager FastPAM2 /
FasterPAM SWAP.

Schubert & Rousseeuw, "Fast and Eager k-Medoids Clustering: O(k) Runtime
Improvement of the PAM, CLARA, and CLARANS Algorithms", arXiv 2008.05171.

All compute runs in libpamx.so (hand-written HIP for gfx950); the functions
here allocate outputs and the workspace with torch and call the C ABI through
``paper_2008_05171_amd.pamx``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

from . import pamx as _abi
from .pamx import (PAMX_ACC_F32, PAMX_ACC_F64, PAMX_CHUNK_TUNE, PAMX_DIST_BF16, PAMX_DIST_STORED,
                   PAMX_FASTERPAM, PAMX_FASTPAM1,
                   PAMX_FASTPAM2, PAMX_INPUT_D, PAMX_INPUT_X, PAMX_L1, PAMX_L2, PamxError)

__all__ = ["fit", "build", "swap", "dist", "check_dissimilarity", "init_dw", "init_lab",
           "clarans", "fit_rect",
           "fit_batched", "FitResult", "BatchResult", "PamxError", "PAMX_FASTPAM1",
           "PAMX_FASTPAM2", "PAMX_FASTERPAM", "PAMX_L1", "PAMX_L2", "PAMX_ACC_F64", "PAMX_ACC_F32",
           "PAMX_INPUT_D", "PAMX_INPUT_X", "PAMX_CHUNK_TUNE"]

_VARIANTS = {"fastpam1": PAMX_FASTPAM1, "fastpam2": PAMX_FASTPAM2, "fasterpam": PAMX_FASTERPAM,
             PAMX_FASTPAM1: PAMX_FASTPAM1, PAMX_FASTPAM2: PAMX_FASTPAM2,
             PAMX_FASTERPAM: PAMX_FASTERPAM}


def _trace_cap(variant, max_iter, n, k):
    """Swap records to reserve: one per search (FastPAM1), k per search
    (FastPAM2), for FasterPAM up to four per object."""
    v = _VARIANTS[variant]
    if v == PAMX_FASTERPAM:
        return 4 * n + 16
    return max_iter * (k if v == PAMX_FASTPAM2 else 1) + 16


@dataclass
class FitResult:
    medoids: object          # torch.int32 [k] on the device, slot order
    labels: object           # torch.int32 [n] on the device
    td: float
    rc: int
    stats: dict
    trace: list = field(default_factory=list)   # [(slot, candidate, delta)]


_DIST = {"stored": PAMX_DIST_STORED, "bf16": PAMX_DIST_BF16,
         PAMX_DIST_STORED: PAMX_DIST_STORED, PAMX_DIST_BF16: PAMX_DIST_BF16}


def _options(variant="fastpam1", accum=PAMX_ACC_F64, max_iter=10000, exclude_self=False,
             chunk=0, trace_buf=None, trace_cap=0, dist_mode="stored", graph=False, window=0):
    o = _abi.pamx_default_options()
    o.graph = int(bool(graph))
    o.window = int(window)
    o.dist_mode = _DIST[dist_mode]
    o.variant = _VARIANTS[variant]
    o.accum = int(accum)
    o.max_iter = int(max_iter)
    o.build_exclude_self = int(bool(exclude_self))
    o.chunk = int(chunk)
    if trace_buf is not None:
        o.trace = trace_buf.data_ptr()
        o.trace_cap = int(trace_cap)
    return o


def _workspace(nbytes, device):
    import torch
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _trace_list(buf, count):
    import numpy as np
    if buf is None or count <= 0:
        return []
    raw = buf[: count * 16].cpu().numpy()
    rec = np.frombuffer(raw.tobytes(), dtype=np.dtype([("slot", "<i4"), ("cand", "<i4"),
                                                         ("delta", "<f8")]))
    return [(int(r["slot"]), int(r["cand"]), float(r["delta"])) for r in rec]


def _stats_dict(st):
    return {f: getattr(st, f) for f, _ in _abi.pamx_stats._fields_}


def fit(data, k, *, input_kind=PAMX_INPUT_X, metric=None, variant="fastpam1",
        accum=PAMX_ACC_F64, max_iter=10000, exclude_self=False, trace=False, chunk=0,
        dist_mode="stored", graph=False, window=0, init="build", seed=0,
        stream=None) -> FitResult:
    """Distances (for points), BUILD, SWAP, labels and TD on the GPU.

    data: device tensor, n x dim points (int32 -> L1, float32 -> L2) or an
    n x n dissimilarity matrix with input_kind=PAMX_INPUT_D.
    dist_mode="bf16": the mixed-precision form (no matrix; BF16 Gram
    distances, FP32 sums, FP64 re-scoring of every possible best swap).
    chunk: objects per pass work-group, 0 = automatic, PAMX_CHUNK_TUNE = timed
    once per process and shape on this matrix (stats["chunk"] reports it).
    variant="fasterpam": Alg. 4; window = candidates scored per pass (0 =
    automatic).
    init: "build" (PAM BUILD, default), or one of the initialisations of
    Sec. 3.3 drawn from `seed`: "random" (k uniform distinct objects), "dw"
    (distance-weighted seeding), "lab" (linear approximative BUILD); these
    run on the stored matrix (computed first for points), then SWAP."""
    import torch
    if init != "build":
        return _fit_init(data, k, input_kind=input_kind, metric=metric, variant=variant,
                         max_iter=max_iter, exclude_self=exclude_self, trace=trace, chunk=chunk,
                         graph=graph, window=window, init=init, seed=seed, stream=stream)
    n = data.shape[0]
    dim = data.shape[1] if input_kind == PAMX_INPUT_X else 0
    dtype = _abi._dtype_code(data)
    if metric is None:
        metric = PAMX_L1 if dtype == _abi.PAMX_I32 else PAMX_L2
    cap = _trace_cap(variant, max_iter, n, k) if trace else 0
    tbuf = torch.empty(cap * 16, dtype=torch.uint8, device=data.device) if trace else None
    opt = _options(variant, accum, max_iter, exclude_self, chunk, tbuf, cap, dist_mode, graph,
                   window)
    nbytes = _abi.pamx_workspace_bytes(n, k, dim, input_kind, dtype, opt)
    ws = _workspace(nbytes, data.device)
    med = torch.empty(k, dtype=torch.int32, device=data.device)
    lab = torch.empty(n, dtype=torch.int32, device=data.device)
    rc, td, st = _abi.pamx_fit(data, input_kind, k, med, lab, ws, metric=metric, opt=opt,
                               stream=stream)
    return FitResult(med, lab, td, rc, _stats_dict(st), _trace_list(tbuf, min(st.swaps, cap)))


def _fit_init(data, k, *, input_kind, metric, variant, max_iter, exclude_self, trace, chunk,
              graph, window, init, seed, stream):
    import time
    import torch
    from . import datagen
    n = data.shape[0]
    torch.cuda.synchronize(data.device)
    t0 = time.perf_counter()
    D = dist(data, metric=metric, stream=stream) if input_kind == PAMX_INPUT_X else data
    torch.cuda.synchronize(data.device)
    t1 = time.perf_counter()
    if init == "random":
        med = torch.from_numpy(datagen.random_subset(n, k, seed)).to(data.device)
    elif init == "dw":
        med = init_dw(D, k, seed=seed, stream=stream)
    elif init == "lab":
        med = init_lab(D, k, seed=seed, exclude_self=exclude_self, stream=stream)
    else:
        raise ValueError("unknown init %r" % (init,))
    torch.cuda.synchronize(data.device)
    t2 = time.perf_counter()
    r = swap(D, med, variant=variant, max_iter=max_iter, trace=trace, chunk=chunk, graph=graph,
             window=window, stream=stream)
    r.stats["init"] = init
    r.stats["init_medoids"] = med
    r.stats["ms_dist"] = (t1 - t0) * 1e3
    r.stats["ms_build"] = (t2 - t1) * 1e3
    r.stats["ms_total"] = r.stats["ms_dist"] + r.stats["ms_build"] + r.stats["ms_swap"]
    return r


def build(D, k, *, exclude_self=False, stream=None):
    """BUILD only: returns (medoids tensor [k], TD)."""
    import torch
    n = D.shape[0]
    opt = _options(exclude_self=exclude_self)
    nbytes = _abi.pamx_workspace_bytes(n, k, 0, PAMX_INPUT_D, _abi._dtype_code(D), opt)
    ws = _workspace(nbytes, D.device)
    med = torch.empty(k, dtype=torch.int32, device=D.device)
    _, td = _abi.pamx_build(D, k, med, ws, opt=opt, stream=stream)
    return med, td


def swap(D, medoids, *, variant="fastpam1", accum=PAMX_ACC_F64, max_iter=10000, trace=False,
         chunk=0, graph=False, window=0, stream=None) -> FitResult:
    """SWAP from the given medoids (device int32 tensor, slot order; copied)."""
    import torch
    n = D.shape[0]
    k = int(medoids.numel())
    cap = _trace_cap(variant, max_iter, n, k) if trace else 0
    tbuf = torch.empty(cap * 16, dtype=torch.uint8, device=D.device) if trace else None
    opt = _options(variant, accum, max_iter, False, chunk, tbuf, cap, graph=graph, window=window)
    nbytes = _abi.pamx_workspace_bytes(n, k, 0, PAMX_INPUT_D, _abi._dtype_code(D), opt)
    ws = _workspace(nbytes, D.device)
    med = medoids.to(device=D.device, dtype=torch.int32).clone()
    lab = torch.empty(n, dtype=torch.int32, device=D.device)
    rc, td, st = _abi.pamx_swap(D, k, med, ws, labels=lab, opt=opt, stream=stream)
    return FitResult(med, lab, td, rc, _stats_dict(st), _trace_list(tbuf, min(st.swaps, cap)))


def init_dw(D, k, *, seed=0, u=None, stream=None):
    """Distance-weighted seeds (Sec. 3.3) from k uniforms (drawn from `seed`
    unless given): device int32 [k]."""
    import torch
    from . import datagen
    n = D.shape[0]
    if u is None:
        u = datagen.uniforms(k, seed)
    ud = torch.as_tensor(u, dtype=torch.float64).to(D.device)
    ws = _workspace(_abi.pamx_init_workspace_bytes(n, 0), D.device)
    med = torch.empty(k, dtype=torch.int32, device=D.device)
    _abi.pamx_init_dw(D, k, ud, med, ws, stream=stream)
    return med


def lab_sample_size(n):
    """LAB's per-step subsample, 10 + ceil(sqrt(n)) points (Sec. 3.3), at most n."""
    import math
    return min(n, 10 + math.isqrt(n - 1) + 1 if n > 1 else 1)


def init_lab(D, k, *, seed=0, m=None, samples=None, exclude_self=False, stream=None):
    """LAB seeds (Sec. 3.3): BUILD on a fresh subsample of m points per step
    (default 10 + ceil(sqrt(n)); rows of `samples` if given).  Device int32 [k]."""
    import torch
    from . import datagen
    n = D.shape[0]
    if samples is None:
        m = lab_sample_size(n) if m is None else int(m)
        samples = datagen.subsamples(n, k, m, seed)
    sd = torch.as_tensor(samples, dtype=torch.int32).to(D.device).contiguous()
    ws = _workspace(_abi.pamx_init_workspace_bytes(n, sd.shape[1]), D.device)
    med = torch.empty(k, dtype=torch.int32, device=D.device)
    _abi.pamx_init_lab(D, k, sd, med, ws, exclude_self=exclude_self, stream=stream)
    return med


def clarans_maxneighbor(n, k):
    """Failures that end a FastCLARANS search: 2.5% of the non-medoids
    (the paper's setting, Sec. 3.4), at least 1."""
    return max(1, int(round(0.025 * (n - k))))


def clarans(D, k, *, numlocal=2, seed=0, maxneighbor=None, draws_per_search=None,
            stream=None) -> FitResult:
    """FastCLARANS (Sec. 3.4) on a stored matrix: `numlocal` local searches,
    each from k uniform random medoids over its own list of random draws
    (seeded), keeping the smallest TD (the first search on ties), in one
    library call (pamx_clarans_numlocal).  stats gain "search_td" (every
    search's TD), "best" (the search kept), "starts" [numlocal, k], "draws"
    [numlocal, len] and "maxneighbor"."""
    import numpy as np
    import torch
    from . import datagen
    n = D.shape[0]
    if maxneighbor is None:
        maxneighbor = clarans_maxneighbor(n, k)
    length = draws_per_search or (64 * maxneighbor + 4 * n)
    starts = np.stack([datagen.random_subset(n, k, seed * 1000 + 2 * r) for r in range(numlocal)])
    draws = np.stack([datagen.int_points(length, 1, 0, n, seed=seed * 1000 + 2 * r + 1).reshape(-1)
                      for r in range(numlocal)])
    opt = _options()
    ws = _workspace(_abi.pamx_best_of_workspace_bytes(n, k, _abi._dtype_code(D), opt), D.device)
    med = torch.empty(k, dtype=torch.int32, device=D.device)
    lab = torch.empty(n, dtype=torch.int32, device=D.device)
    rc, td, st, each, best = _abi.pamx_clarans_numlocal(
        D, k, torch.from_numpy(starts.astype(np.int32)).to(D.device),
        torch.from_numpy(draws.astype(np.int32)).to(D.device), maxneighbor, med, ws, labels=lab,
        opt=opt, stream=stream)
    res = FitResult(med, lab, td, rc, _stats_dict(st), [])
    res.stats.update(search_td=each, best=best, starts=starts, draws=draws, maxneighbor=maxneighbor)
    return res


def restart_starts(D, k, restarts, init="random", seed=0):
    """Starts for `restarts` local searches (Sec. 3.3): uniform random medoid
    sets, distance-weighted seeds or LAB, each from its own seed; host int32
    array [restarts, k]."""
    import numpy as np
    from . import datagen
    n = D.shape[0]
    out = []
    for r in range(restarts):
        sr = seed * 1000 + r
        if init == "random":
            out.append(datagen.random_subset(n, k, sr))
        elif init == "dw":
            out.append(init_dw(D, k, seed=sr).cpu().numpy())
        elif init == "lab":
            out.append(init_lab(D, k, seed=sr).cpu().numpy())
        else:
            raise ValueError("init must be random, dw or lab")
    return np.stack(out).astype(np.int32)


def fit_restarts(D, k, *, restarts=4, init="random", variant="fasterpam", seed=0, starts=None,
                 max_iter=10000, stream=None) -> FitResult:
    """Several cheap starts then SWAP (Sec. 3.3; the paper finds random starts
    with FasterPAM fastest at equal quality, Sec. 4.3), keeping the smallest
    TD (the first restart on ties), in one library call (pamx_swap_restarts)
    on a stored matrix D.  `starts` (host or device int32 [R, k]) overrides
    init/restarts/seed.  stats gain "restart_td", "best" and "starts"."""
    import numpy as np
    import torch
    n = D.shape[0]
    if starts is None:
        starts = restart_starts(D, k, restarts, init, seed)
    st_d = torch.as_tensor(np.asarray(starts) if not torch.is_tensor(starts) else starts,
                           dtype=torch.int32).to(D.device).contiguous()
    opt = _options(variant=variant, max_iter=max_iter)
    ws = _workspace(_abi.pamx_best_of_workspace_bytes(n, k, _abi._dtype_code(D), opt), D.device)
    med = torch.empty(k, dtype=torch.int32, device=D.device)
    lab = torch.empty(n, dtype=torch.int32, device=D.device)
    rc, td, st, each, best = _abi.pamx_swap_restarts(D, k, st_d, med, ws, labels=lab, opt=opt,
                                                     stream=stream)
    res = FitResult(med, lab, td, rc, _stats_dict(st), [])
    res.stats.update(restart_td=each, best=best, starts=st_d.cpu().numpy())
    return res


def fit_rect(D, k, *, medoids=None, max_iter=10000, trace=False, stream=None) -> FitResult:
    """Bichromatic medoids (Sec. 5) on a consumers x locations matrix D
    (device, int32 or float32): BUILD then FastPAM1, or FastPAM1 from the
    location `medoids` given.  Medoids are location indices, labels slots."""
    import torch
    nco, nl = D.shape
    cap = max_iter + 16 if trace else 0
    tbuf = torch.empty(cap * 16, dtype=torch.uint8, device=D.device) if trace else None
    opt = _options(max_iter=max_iter, trace_buf=tbuf, trace_cap=cap)
    nbytes = _abi.pamx_rect_workspace_bytes(nco, nl, k, _abi._dtype_code(D), opt)
    ws = _workspace(nbytes, D.device)
    if medoids is None:
        med = torch.empty(k, dtype=torch.int32, device=D.device)
    else:
        med = medoids.to(device=D.device, dtype=torch.int32).clone()
    lab = torch.empty(nco, dtype=torch.int32, device=D.device)
    rc, td, st = _abi.pamx_rect(D, k, med, ws, labels=lab, opt=opt, build=medoids is None,
                                stream=stream)
    return FitResult(med, lab, td, rc, _stats_dict(st), _trace_list(tbuf, min(st.swaps, cap)))


def check_dissimilarity(D, *, stream=None) -> dict:
    """Validate an n x n device matrix: {"valid", "asymmetric", "diagonal",
    "negative", "nonfinite", "pairs"} (pairs = offending pairs {i, j}, i <= j)."""
    flags, count = _abi.pamx_check_dissimilarity(D, stream=stream)
    return {"valid": flags == 0,
            "asymmetric": bool(flags & _abi.PAMX_DIS_ASYMMETRIC),
            "diagonal": bool(flags & _abi.PAMX_DIS_DIAGONAL),
            "negative": bool(flags & _abi.PAMX_DIS_NEGATIVE),
            "nonfinite": bool(flags & _abi.PAMX_DIS_NONFINITE),
            "pairs": count}


def dist(X, *, metric=None, ld=None, stream=None):
    """n x n dissimilarity matrix of points X (int32 -> L1, float32 -> L2)."""
    import torch
    n = X.shape[0]
    dtype = _abi._dtype_code(X)
    if metric is None:
        metric = PAMX_L1 if dtype == _abi.PAMX_I32 else PAMX_L2
    ld = ((n + 3) // 4) * 4 if ld is None else ld
    D = torch.empty((n, ld), dtype=X.dtype, device=X.device)
    _abi.pamx_dist(X, metric, D, ld=ld, stream=stream)
    return D[:, :n]


@dataclass
class BatchResult:
    medoids: list            # per instance: torch.int32 [k_j] global point indices
    td_sample: object        # numpy float64 [n_inst]
    td_full: object          # numpy float64 [n_inst] or None
    best: int                # instance with the smallest full-data TD (-1 if not computed)
    rc: int
    stats: dict


def fit_batched(X, sample_off, sample_idx, k_inst, *, metric=None, max_iter=10000,
                exclude_self=False, full_td=True, tune=False, stream=None) -> BatchResult:
    """Batched CLARA: PAM (BUILD + FastPAM1) on every subsample in one launch,
    then the TD of each run over all points of X.  sample_off/k_inst are host
    arrays, sample_idx a device int32 tensor.  tune=True: the team sizes are
    timed on the first call of this instance shape and the fastest kept
    (stats["team_scale"])."""
    import numpy as np
    import torch
    dtype = _abi._dtype_code(X)
    if metric is None:
        metric = PAMX_L1 if dtype == _abi.PAMX_I32 else PAMX_L2
    k_inst = np.asarray(k_inst, dtype=np.int32)
    sample_off = np.asarray(sample_off, dtype=np.int64)
    opt = _options(max_iter=max_iter, exclude_self=exclude_self,
                   chunk=PAMX_CHUNK_TUNE if tune else 0)
    ws = _workspace(_abi.pamx_batched_workspace_bytes(len(k_inst), X.shape[0]), X.device)
    med = torch.empty(int(k_inst.sum()), dtype=torch.int32, device=X.device)
    rc, tds, tdf, st = _abi.pamx_fit_batched(X, metric, sample_off, sample_idx, k_inst, med, ws,
                                             opt=opt, want_full=full_td, stream=stream)
    offs = np.concatenate([[0], np.cumsum(k_inst)])
    meds = [med[offs[j]:offs[j + 1]] for j in range(len(k_inst))]
    stats = {f: getattr(st, f) for f, _ in _abi.pamx_batch_stats._fields_}
    return BatchResult(meds, tds, tdf, st.best_inst, rc, stats)
