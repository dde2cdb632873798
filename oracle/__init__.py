"""CPU oracle of PAM (BUILD + SWAP) in FP64 -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product library never loads it.

The arithmetic lives in ``pam_oracle.c`` (plain C, OpenMP, FP64); this module
only builds it (gcc) and marshals numpy arrays.  Paper references
(Schubert & Rousseeuw, arXiv 2008.05171):

* ``dist_matrix``   -- the dissimilarity matrix PAM consumes (Sec. 2).
* ``build``         -- PAM BUILD, Alg. 1 (self-term reading R1, see the C file).
* ``nearest``/``td``-- nearest/second-nearest caches and Eq. td.
* ``change``        -- Eq. change, the per-object loss change of a swap.
* ``delta``         -- Delta TD of one swap, Eq. td2 summed with Eq. change.
* ``swap``          -- PAM SWAP, Alg. 2 (variant 1), the FastPAM2 reading
                       (variant 2: best swap per medoid, applied eagerly), or
                       FasterPAM, Alg. 4 (variant 3: the first candidate in scan
                       order with an improving swap, applied at once).
* ``pam``           -- BUILD followed by SWAP, with labels.
* ``init_dw``       -- distance-weighted seeding (Sec. 3.3, reading R14).
* ``init_lab``      -- LAB, BUILD on per-step subsamples (Sec. 3.3, reading R15).
* ``clarans``       -- one FastCLARANS local search over given draws (Sec. 3.4,
                       reading R16).
* ``rect_build``, ``rect_swap``, ``rect_td``, ``rect_pam`` -- BUILD and PAM SWAP
                       for bichromatic medoids: consumers x locations matrix
                       (Sec. 5, reading R17).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pam_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

L1 = 1
L2 = 2
L2F32 = 3        # Euclidean, each distance rounded to the nearest FP32 value
PAM = 1          # best swap per iteration (PAM == FastPAM1 result)
FASTPAM2 = 2     # best swap per medoid, applied eagerly
FASTERPAM = 3    # Alg. 4: eager swap of each improving candidate in scan order

_lib = None


def compile_oracle(force: bool = False) -> str:
    """Compile pam_oracle.c into liboracle.so with gcc (OpenMP, -O3 for the
    host's own CPU).  Floating-point contraction stays off and no fast-math
    flag is given, so every FP64 operation is rounded as written and the
    results do not depend on the CPU it was built for."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O3", "-march=native", "-ffp-contract=off", "-std=c11", "-fopenmp", "-fPIC",
             "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    lib = ctypes.CDLL(compile_oracle())
    P = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_set_num_threads.argtypes = [ctypes.c_int]
    lib.orc_set_num_threads.restype = ctypes.c_int
    lib.orc_dist_matrix.argtypes = [P, i64, i32, i32, P]
    lib.orc_nearest.argtypes = [P, P, i64, i32, i32, P, i32, P, P, P]
    lib.orc_td.argtypes = [P, P, i64, i32, i32, P, i32, P]
    lib.orc_td.restype = f64
    lib.orc_change.argtypes = [f64, i32, f64, f64]
    lib.orc_change.restype = f64
    lib.orc_delta.argtypes = [P, P, i64, i32, i32, P, i32, i32, i64]
    lib.orc_delta.restype = f64
    lib.orc_build.argtypes = [P, P, i64, i32, i32, i32, i32, P, P, P]
    lib.orc_swap_search.argtypes = [P, P, i64, i32, i32, P, i32, i64, i64, P, P, P]
    lib.orc_swap.argtypes = [P, P, i64, i32, i32, P, i32, i32, i32, P, P, P, i32, P, P, P]
    lib.orc_dist_rows.argtypes = [P, i64, i32, i32, P, i64, P]
    lib.orc_swap_list.argtypes = [P, P, i64, i32, i32, P, i32, P, i64, P]
    lib.orc_build_list.argtypes = [P, P, i64, i32, i32, P, i32, i32, P, i64, P]
    lib.orc_init_dw.argtypes = [P, P, i64, i32, i32, i32, P, P]
    lib.orc_init_lab.argtypes = [P, P, i64, i32, i32, i32, P, i32, i32, P]
    lib.orc_clarans.argtypes = [P, P, i64, i32, i32, P, i32, P, i64, i64, P, P, P, i32, P, P, P]
    lib.orc_rect_td.argtypes = [P, i64, i64, P, i32, P]
    lib.orc_rect_td.restype = f64
    lib.orc_rect_build.argtypes = [P, i64, i64, i32, P, P]
    lib.orc_rect_swap.argtypes = [P, i64, i64, P, i32, i32, P, P, P, i32, P, P, P]
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class _Src:
    """Holds the FP64 arrays handed to C (dense matrix, or points + metric)."""

    def __init__(self, D=None, X=None, metric=L2):
        if (D is None) == (X is None):
            raise ValueError("give exactly one of D (n x n) or X (n x dim)")
        if D is not None:
            D = np.ascontiguousarray(D, dtype=np.float64)
            if D.ndim != 2 or D.shape[0] != D.shape[1]:
                raise ValueError("D must be square")
            self.n, self.dim = D.shape[0], 0
        else:
            X = np.ascontiguousarray(X, dtype=np.float64)
            if X.ndim != 2:
                raise ValueError("X must be 2-D")
            self.n, self.dim = X.shape
        self.D, self.X, self.metric = D, X, int(metric)

    def args(self):
        return (_ptr(self.D), _ptr(self.X), self.n, self.dim, self.metric)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(t: int) -> int:
    """Threads of the oracle's parallel loops from now on; returns the count."""
    return int(_load().orc_set_num_threads(int(t)))


def dist_matrix(X, metric=L2) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float64)
    n, dim = X.shape
    D = np.empty((n, n), dtype=np.float64)
    rc = _load().orc_dist_matrix(_ptr(X), n, dim, int(metric), _ptr(D))
    if rc:
        raise ValueError("orc_dist_matrix rc=%d" % rc)
    return D


def dist_rows(X, rows, metric=L2) -> np.ndarray:
    """Rows ``rows`` of the dissimilarity matrix of points X, FP64."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    n, dim = X.shape
    out = np.empty((len(rows), n), dtype=np.float64)
    rc = _load().orc_dist_rows(_ptr(X), n, dim, int(metric), _ptr(rows), len(rows), _ptr(out))
    if rc:
        raise ValueError("orc_dist_rows rc=%d" % rc)
    return out


def change(d, is_i, dn, ds) -> float:
    return float(_load().orc_change(float(d), int(bool(is_i)), float(dn), float(ds)))


def nearest(med, D=None, X=None, metric=L2):
    s = _Src(D, X, metric)
    med = np.ascontiguousarray(med, dtype=np.int32)
    near = np.empty(s.n, np.int32)
    dn = np.empty(s.n, np.float64)
    ds = np.empty(s.n, np.float64)
    rc = _load().orc_nearest(*s.args(), _ptr(med), len(med), _ptr(near), _ptr(dn), _ptr(ds))
    if rc:
        raise ValueError("orc_nearest rc=%d" % rc)
    return near, dn, ds


def td(med, D=None, X=None, metric=L2):
    """Return (TD, labels) for the medoid slots ``med``."""
    s = _Src(D, X, metric)
    med = np.ascontiguousarray(med, dtype=np.int32)
    labels = np.empty(s.n, np.int32)
    v = _load().orc_td(*s.args(), _ptr(med), len(med), _ptr(labels))
    return float(v), labels


def delta(med, i, c, D=None, X=None, metric=L2) -> float:
    s = _Src(D, X, metric)
    med = np.ascontiguousarray(med, dtype=np.int32)
    return float(_load().orc_delta(*s.args(), _ptr(med), len(med), int(i), int(c)))


def build(k, D=None, X=None, metric=L2, exclude_self=False):
    """PAM BUILD: returns (medoids in slot order, TD, per-step chosen change)."""
    s = _Src(D, X, metric)
    med = np.empty(k, np.int32)
    tdv = np.zeros(1, np.float64)
    steps = np.empty(k, np.float64)
    rc = _load().orc_build(*s.args(), int(k), int(bool(exclude_self)), _ptr(med), _ptr(tdv),
                           _ptr(steps))
    if rc:
        raise ValueError("orc_build rc=%d" % rc)
    return med, float(tdv[0]), steps


def swap_search(med, D=None, X=None, metric=L2, c_begin=0, c_end=None):
    """One SWAP search (Alg. 2 order) over candidates [c_begin, c_end)."""
    s = _Src(D, X, metric)
    med = np.ascontiguousarray(med, dtype=np.int32)
    c_end = s.n if c_end is None else int(c_end)
    bd = ctypes.c_double()
    bi = ctypes.c_int32()
    bc = ctypes.c_int64()
    rc = _load().orc_swap_search(*s.args(), _ptr(med), len(med), int(c_begin), c_end,
                                 ctypes.byref(bd), ctypes.byref(bi), ctypes.byref(bc))
    if rc < 0:
        raise ValueError("orc_swap_search rc=%d" % rc)
    return bool(rc), bd.value, bi.value, bc.value


def swap_list(med, cand, D=None, X=None, metric=L2) -> np.ndarray:
    """Delta TD of every (candidate in ``cand``, slot) swap: array (len(cand), k),
    NaN rows for candidates that are medoids (Alg. 2 inner sum, Eq. change)."""
    s = _Src(D, X, metric)
    med = np.ascontiguousarray(med, dtype=np.int32)
    cand = np.ascontiguousarray(cand, dtype=np.int64)
    out = np.empty((len(cand), len(med)), np.float64)
    rc = _load().orc_swap_list(*s.args(), _ptr(med), len(med), _ptr(cand), len(cand), _ptr(out))
    if rc:
        raise ValueError("orc_swap_list rc=%d" % rc)
    return out


def build_list(prefix, cand, D=None, X=None, metric=L2, exclude_self=False) -> np.ndarray:
    """BUILD change (Alg. 1) of taking each of ``cand`` as the next medoid after
    the medoids ``prefix``; an empty prefix gives the first step's column sums."""
    s = _Src(D, X, metric)
    prefix = np.ascontiguousarray(prefix, dtype=np.int32)
    cand = np.ascontiguousarray(cand, dtype=np.int64)
    out = np.empty(len(cand), np.float64)
    rc = _load().orc_build_list(*s.args(), _ptr(prefix) if len(prefix) else None, len(prefix),
                                int(bool(exclude_self)), _ptr(cand), len(cand), _ptr(out))
    if rc:
        raise ValueError("orc_build_list rc=%d" % rc)
    return out


@dataclass
class SwapResult:
    medoids: np.ndarray
    td: float
    iterations: int
    swaps: int
    rc: int
    trace: list = field(default_factory=list)   # [(slot, candidate, delta)]


def swap(med, D=None, X=None, metric=L2, variant=PAM, max_iter=10000, trace_cap=100000):
    s = _Src(D, X, metric)
    med = np.array(med, dtype=np.int32, copy=True)
    ts = np.empty(trace_cap, np.int32)
    tc = np.empty(trace_cap, np.int64)
    tdl = np.empty(trace_cap, np.float64)
    it = ctypes.c_int32()
    sw = ctypes.c_int32()
    tdv = ctypes.c_double()
    rc = _load().orc_swap(*s.args(), _ptr(med), len(med), int(variant), int(max_iter),
                          _ptr(ts), _ptr(tc), _ptr(tdl), int(trace_cap),
                          ctypes.byref(it), ctypes.byref(sw), ctypes.byref(tdv))
    if rc < 0:
        raise ValueError("orc_swap rc=%d" % rc)
    m = min(sw.value, trace_cap)
    trace = [(int(ts[j]), int(tc[j]), float(tdl[j])) for j in range(m)]
    return SwapResult(med, tdv.value, it.value, sw.value, rc, trace)


@dataclass
class PamResult:
    medoids: np.ndarray
    labels: np.ndarray
    td: float
    td_build: float
    build_medoids: np.ndarray
    iterations: int
    swaps: int
    rc: int
    trace: list


def pam(k, D=None, X=None, metric=L2, variant=PAM, exclude_self=False, max_iter=10000):
    """BUILD (Alg. 1) then SWAP (Alg. 2, the FastPAM2 reading or Alg. 4)."""
    bm, td_b, _ = build(k, D=D, X=X, metric=metric, exclude_self=exclude_self)
    r = swap(bm, D=D, X=X, metric=metric, variant=variant, max_iter=max_iter)
    tdv, labels = td(r.medoids, D=D, X=X, metric=metric)
    return PamResult(r.medoids, labels, tdv, td_b, bm, r.iterations, r.swaps, r.rc, r.trace)


def init_dw(k, u, D=None, X=None, metric=L2) -> np.ndarray:
    """Distance-weighted seeds (reading R14) from the uniforms u[0..k-1]."""
    s = _Src(D, X, metric)
    u = np.ascontiguousarray(u, dtype=np.float64)
    if len(u) < k:
        raise ValueError("need k uniforms")
    med = np.empty(k, np.int32)
    rc = _load().orc_init_dw(*s.args(), int(k), _ptr(u), _ptr(med))
    if rc:
        raise ValueError("orc_init_dw rc=%d" % rc)
    return med


def init_lab(k, samples, D=None, X=None, metric=L2, exclude_self=False) -> np.ndarray:
    """LAB (reading R15): samples is a (k, m) array, row t = step t's subsample."""
    s = _Src(D, X, metric)
    samples = np.ascontiguousarray(samples, dtype=np.int32)
    if samples.ndim != 2 or samples.shape[0] != k:
        raise ValueError("samples must be (k, m)")
    med = np.empty(k, np.int32)
    rc = _load().orc_init_lab(*s.args(), int(k), _ptr(samples), int(samples.shape[1]),
                              int(bool(exclude_self)), _ptr(med))
    if rc:
        raise ValueError("orc_init_lab rc=%d" % rc)
    return med


@dataclass
class ClaransResult:
    medoids: np.ndarray
    td: float
    evaluations: int
    swaps: int
    rc: int
    trace: list = field(default_factory=list)


def clarans(med, draws, maxneighbor, D=None, X=None, metric=L2, trace_cap=100000):
    """One FastCLARANS local search (reading R16) from medoids `med` over the
    random draws `draws` (object indices, in order)."""
    s = _Src(D, X, metric)
    med = np.array(med, dtype=np.int32, copy=True)
    draws = np.ascontiguousarray(draws, dtype=np.int32)
    ts = np.empty(trace_cap, np.int32)
    tc = np.empty(trace_cap, np.int64)
    tdl = np.empty(trace_cap, np.float64)
    ev = ctypes.c_int64()
    sw = ctypes.c_int32()
    tdv = ctypes.c_double()
    rc = _load().orc_clarans(*s.args(), _ptr(med), len(med), _ptr(draws), len(draws),
                             int(maxneighbor), _ptr(ts), _ptr(tc), _ptr(tdl), int(trace_cap),
                             ctypes.byref(ev), ctypes.byref(sw), ctypes.byref(tdv))
    if rc < 0:
        raise ValueError("orc_clarans rc=%d" % rc)
    m = min(sw.value, trace_cap)
    trace = [(int(ts[j]), int(tc[j]), float(tdl[j])) for j in range(m)]
    return ClaransResult(med, tdv.value, ev.value, sw.value, rc, trace)


def _rect(D):
    D = np.ascontiguousarray(D, dtype=np.float64)
    if D.ndim != 2:
        raise ValueError("D must be consumers x locations")
    return D, D.shape[0], D.shape[1]


def rect_td(med, D):
    """(TD, labels) of location medoids `med` for the consumers x locations D."""
    D, nc, nl = _rect(D)
    med = np.ascontiguousarray(med, dtype=np.int32)
    labels = np.empty(nc, np.int32)
    v = _load().orc_rect_td(_ptr(D), nc, nl, _ptr(med), len(med), _ptr(labels))
    return float(v), labels


def rect_build(k, D):
    """BUILD over locations (reading R17): (medoids, TD)."""
    D, nc, nl = _rect(D)
    med = np.empty(k, np.int32)
    tdv = np.zeros(1, np.float64)
    rc = _load().orc_rect_build(_ptr(D), nc, nl, int(k), _ptr(med), _ptr(tdv))
    if rc:
        raise ValueError("orc_rect_build rc=%d" % rc)
    return med, float(tdv[0])


def rect_swap(med, D, max_iter=10000, trace_cap=100000):
    """PAM SWAP over locations (reading R17)."""
    D, nc, nl = _rect(D)
    med = np.array(med, dtype=np.int32, copy=True)
    ts = np.empty(trace_cap, np.int32)
    tc = np.empty(trace_cap, np.int64)
    tdl = np.empty(trace_cap, np.float64)
    it = ctypes.c_int32()
    sw = ctypes.c_int32()
    tdv = ctypes.c_double()
    rc = _load().orc_rect_swap(_ptr(D), nc, nl, _ptr(med), len(med), int(max_iter), _ptr(ts),
                               _ptr(tc), _ptr(tdl), int(trace_cap), ctypes.byref(it),
                               ctypes.byref(sw), ctypes.byref(tdv))
    if rc < 0:
        raise ValueError("orc_rect_swap rc=%d" % rc)
    m = min(sw.value, trace_cap)
    trace = [(int(ts[j]), int(tc[j]), float(tdl[j])) for j in range(m)]
    return SwapResult(med, tdv.value, it.value, sw.value, rc, trace)


def rect_pam(k, D, max_iter=10000):
    """Bichromatic BUILD then SWAP: PamResult with location medoids."""
    bm, td_b = rect_build(k, D)
    r = rect_swap(bm, D, max_iter=max_iter)
    tdv, labels = rect_td(r.medoids, D)
    return PamResult(r.medoids, labels, tdv, td_b, bm, r.iterations, r.swaps, r.rc, r.trace)
