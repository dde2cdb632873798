"""ctypes binding of libpamx.so (C ABI in include/pamx.h).

Argument marshalling only: every step of BUILD and SWAP runs in the HIP
kernels of libpamx.so.  Torch tensors provide device memory and the stream.
If the library is missing this module raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libpamx.so")

# constants of include/pamx.h
PAMX_I32, PAMX_F32 = 1, 2
PAMX_INPUT_D, PAMX_INPUT_X = 0, 1
PAMX_L1, PAMX_L2 = 1, 2
PAMX_FASTPAM1, PAMX_FASTPAM2, PAMX_FASTERPAM = 1, 2, 3
PAMX_ACC_F64, PAMX_ACC_F32 = 0, 1
PAMX_DIST_STORED, PAMX_DIST_BF16 = 0, 1
PAMX_CHUNK_TUNE = -1
PAMX_OK, PAMX_WARN_MAXITER = 0, 1
PAMX_ERR_ARG, PAMX_ERR_WORKSPACE, PAMX_ERR_HIP = -1, -2, -3
PAMX_ERR_INVALID_MEDOIDS, PAMX_ERR_UNSUPPORTED = -4, -5
PAMX_DIS_ASYMMETRIC, PAMX_DIS_DIAGONAL, PAMX_DIS_NEGATIVE, PAMX_DIS_NONFINITE = 1, 2, 4, 8


class pamx_options(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("accum", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("build_exclude_self", ctypes.c_int32),
                ("trace_cap", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("dist_mode", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("window", ctypes.c_int32),
                ("trace", ctypes.c_void_p)]


class pamx_swap_record(ctypes.Structure):
    _fields_ = [("slot", ctypes.c_int32), ("cand", ctypes.c_int32), ("delta", ctypes.c_double)]


class pamx_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("swaps", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("rescored", ctypes.c_int32),
                ("td_build", ctypes.c_double), ("td", ctypes.c_double),
                ("ms_dist", ctypes.c_double), ("ms_build", ctypes.c_double),
                ("ms_swap", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("pass_pairs", ctypes.c_int64), ("build_pairs", ctypes.c_int64),
                ("ms_swap_pass", ctypes.c_double), ("ms_build_pass", ctypes.c_double),
                ("n_swap_pass", ctypes.c_int32), ("n_build_pass", ctypes.c_int32),
                ("ms_build_delta", ctypes.c_double), ("build_rows", ctypes.c_int64),
                ("n_build_delta", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("scan_positions", ctypes.c_int64), ("windows", ctypes.c_int32),
                ("window", ctypes.c_int32)]


class pamx_batch_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("swaps", ctypes.c_int32),
                ("best_inst", ctypes.c_int32), ("team_scale", ctypes.c_int32),
                ("ms_pam", ctypes.c_double), ("ms_assign", ctypes.c_double),
                ("ms_total", ctypes.c_double), ("pairs", ctypes.c_int64)]


EXPORTS = ("pamx_default_options", "pamx_workspace_bytes", "pamx_dist", "pamx_build",
           "pamx_swap", "pamx_fit", "pamx_batched_workspace_bytes", "pamx_fit_batched",
           "pamx_init_workspace_bytes", "pamx_init_dw", "pamx_init_lab", "pamx_clarans",
           "pamx_rect_workspace_bytes", "pamx_fit_rect", "pamx_swap_rect",
           "pamx_check_dissimilarity", "pamx_read_probe", "pamx_write_probe", "pamx_swap_noalloc",
           "pamx_best_of_workspace_bytes", "pamx_swap_restarts", "pamx_clarans_numlocal",
           "pamx_last_error")


class PamxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("pamx error %d: %s" % (code, msg))
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libpamx.so and declare its signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libpamx.so is not built (%s); run "
                           "`python -m paper_2008_05171_amd.buildlib`" % path)
    lib = ctypes.CDLL(path)
    P, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    opt_p = ctypes.POINTER(pamx_options)
    st_p = ctypes.POINTER(pamx_stats)
    dbl_p = ctypes.POINTER(ctypes.c_double)
    lib.pamx_default_options.argtypes = [opt_p]
    lib.pamx_default_options.restype = None
    lib.pamx_workspace_bytes.argtypes = [i64, i32, i32, i32, i32, opt_p, ctypes.POINTER(sz)]
    lib.pamx_dist.argtypes = [P, i32, i64, i32, i32, P, i64, P, sz, P]
    lib.pamx_build.argtypes = [P, i32, i64, i64, i32, opt_p, P, dbl_p, P, sz, P]
    lib.pamx_swap.argtypes = [P, i32, i64, i64, i32, opt_p, P, P, dbl_p, st_p, P, sz, P]
    lib.pamx_fit.argtypes = [P, i32, i32, i64, i32, i32, i32, opt_p, P, P, dbl_p, st_p, P, sz, P]
    lib.pamx_batched_workspace_bytes.argtypes = [i32, i64, ctypes.POINTER(sz)]
    lib.pamx_fit_batched.argtypes = [P, i32, i64, i32, i32, i32, P, P, P, opt_p, P, P, P,
                                     ctypes.POINTER(pamx_batch_stats), P, sz, P]
    lib.pamx_init_workspace_bytes.argtypes = [i64, i32, ctypes.POINTER(sz)]
    lib.pamx_init_dw.argtypes = [P, i32, i64, i64, i32, P, P, P, sz, P]
    lib.pamx_init_lab.argtypes = [P, i32, i64, i64, i32, P, i32, i32, P, P, sz, P]
    lib.pamx_clarans.argtypes = [P, i32, i64, i64, i32, P, i64, i64, opt_p, P, P, dbl_p, st_p, P,
                                 sz, P]
    lib.pamx_rect_workspace_bytes.argtypes = [i64, i64, i32, i32, opt_p, ctypes.POINTER(sz)]
    lib.pamx_fit_rect.argtypes = [P, i32, i64, i64, i64, i32, opt_p, P, P, dbl_p, st_p, P, sz, P]
    lib.pamx_swap_rect.argtypes = [P, i32, i64, i64, i64, i32, opt_p, P, P, dbl_p, st_p, P, sz, P]
    lib.pamx_check_dissimilarity.argtypes = [P, i32, i64, i64, ctypes.POINTER(ctypes.c_int32),
                                             ctypes.POINTER(ctypes.c_int64), P, sz, P]
    lib.pamx_read_probe.argtypes = [P, i64, i64, i32, P, i64, P]
    lib.pamx_write_probe.argtypes = [P, i64, i64, ctypes.c_float, P]
    lib.pamx_swap_noalloc.argtypes = [P, i32, i64, i64, i32, opt_p, P, P, dbl_p, st_p, P]
    lib.pamx_best_of_workspace_bytes.argtypes = [i64, i32, i32, opt_p, ctypes.POINTER(sz)]
    lib.pamx_swap_restarts.argtypes = [P, i32, i64, i64, i32, i32, P, opt_p, P, P, dbl_p, st_p,
                                       dbl_p, ctypes.POINTER(i32), P, sz, P]
    lib.pamx_clarans_numlocal.argtypes = [P, i32, i64, i64, i32, i32, P, P, i64, i64, opt_p, P, P,
                                          dbl_p, st_p, dbl_p, ctypes.POINTER(i32), P, sz, P]
    lib.pamx_last_error.argtypes = []
    lib.pamx_last_error.restype = ctypes.c_char_p
    for name in ("pamx_workspace_bytes", "pamx_dist", "pamx_build", "pamx_swap", "pamx_fit",
                 "pamx_batched_workspace_bytes", "pamx_fit_batched", "pamx_init_workspace_bytes",
                 "pamx_init_dw", "pamx_init_lab", "pamx_clarans", "pamx_rect_workspace_bytes",
                 "pamx_fit_rect", "pamx_swap_rect", "pamx_check_dissimilarity", "pamx_read_probe",
                 "pamx_write_probe",
                 "pamx_swap_noalloc", "pamx_best_of_workspace_bytes", "pamx_swap_restarts",
                 "pamx_clarans_numlocal"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc):
    if rc < 0:
        raise PamxError(rc, load().pamx_last_error().decode())
    return rc


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dtype_code(t):
    import torch
    if t.dtype == torch.int32:
        return PAMX_I32
    if t.dtype == torch.float32:
        return PAMX_F32
    raise TypeError("dissimilarities/points must be int32 or float32, got %s" % t.dtype)


def pamx_default_options() -> pamx_options:
    o = pamx_options()
    load().pamx_default_options(ctypes.byref(o))
    return o


def pamx_workspace_bytes(n, k, dim, input_kind, dtype, opt=None) -> int:
    out = ctypes.c_size_t()
    _check(load().pamx_workspace_bytes(int(n), int(k), int(dim), int(input_kind), int(dtype),
                                       ctypes.byref(opt) if opt is not None else None,
                                       ctypes.byref(out)))
    return int(out.value)


def pamx_dist(X, metric, D, ws=None, ld=None, stream=None):
    """ws: device scratch of >= 4*dim bytes (float32 points) or 8*dim bytes
    (int32 points), allocated here if None."""
    import torch
    n, dim = X.shape
    ld = D.stride(0) if ld is None else ld
    if ws is None:
        ws = torch.empty(max(8 * dim, 256), dtype=torch.uint8, device=X.device)
    return _check(load().pamx_dist(_ptr(X), _dtype_code(X), n, dim, int(metric), _ptr(D), int(ld),
                                   _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))


def pamx_check_dissimilarity(D, ws=None, n=None, ld=None, stream=None):
    """(flags, count): PAMX_DIS_* bits found in the n x n matrix D and the
    number of offending pairs; ws: >= 8 bytes of device scratch."""
    import torch
    n = D.shape[0] if n is None else n
    ld = D.stride(0) if ld is None else ld
    if ws is None:
        ws = torch.empty(256, dtype=torch.uint8, device=D.device)
    flags = ctypes.c_int32()
    count = ctypes.c_int64()
    _check(load().pamx_check_dissimilarity(_ptr(D), _dtype_code(D), int(n), int(ld),
                                           ctypes.byref(flags), ctypes.byref(count), _ptr(ws),
                                           ws.numel() * ws.element_size(), _stream(stream)))
    return flags.value, count.value


def pamx_read_probe(D, chunk, sums, n=None, ld=None, stream=None):
    """Plain read of the n x n FP32 matrix D in the SWAP pass's launch shape
    (rows in chunks of `chunk`); sums: device float32, one per work-group."""
    n = D.shape[0] if n is None else n
    ld = D.stride(0) if ld is None else ld
    return _check(load().pamx_read_probe(_ptr(D), int(n), int(ld), int(chunk), _ptr(sums),
                                         sums.numel(), _stream(stream)))


def pamx_write_probe(D, value=1.0, n=None, ld=None, stream=None):
    """Writes `value` to the n x n FP32 matrix D in the distance kernel's launch
    shape and store pattern (no loads, no arithmetic)."""
    n = D.shape[0] if n is None else n
    ld = D.stride(0) if ld is None else ld
    return _check(load().pamx_write_probe(_ptr(D), int(n), int(ld), float(value), _stream(stream)))


def pamx_build(D, k, medoids, ws, opt=None, n=None, ld=None, stream=None):
    n = D.shape[0] if n is None else n
    ld = D.stride(0) if ld is None else ld
    td = ctypes.c_double()
    rc = _check(load().pamx_build(_ptr(D), _dtype_code(D), int(n), int(ld), int(k),
                                  ctypes.byref(opt) if opt is not None else None, _ptr(medoids),
                                  ctypes.byref(td), _ptr(ws), ws.numel() * ws.element_size(),
                                  _stream(stream)))
    return rc, td.value


def pamx_swap(D, k, medoids, ws, labels=None, opt=None, n=None, ld=None, stream=None):
    n = D.shape[0] if n is None else n
    ld = D.stride(0) if ld is None else ld
    td = ctypes.c_double()
    st = pamx_stats()
    rc = _check(load().pamx_swap(_ptr(D), _dtype_code(D), int(n), int(ld), int(k),
                                 ctypes.byref(opt) if opt is not None else None, _ptr(medoids),
                                 _ptr(labels), ctypes.byref(td), ctypes.byref(st), _ptr(ws),
                                 ws.numel() * ws.element_size(), _stream(stream)))
    return rc, td.value, st


def pamx_swap_noalloc(D, k, medoids, labels=None, opt=None, n=None, ld=None, stream=None):
    """pamx_swap with the library's fixed scratch array instead of a workspace."""
    n = D.shape[0] if n is None else n
    ld = D.stride(0) if ld is None else ld
    td = ctypes.c_double()
    st = pamx_stats()
    rc = _check(load().pamx_swap_noalloc(_ptr(D), _dtype_code(D), int(n), int(ld), int(k),
                                         ctypes.byref(opt) if opt is not None else None,
                                         _ptr(medoids), _ptr(labels), ctypes.byref(td),
                                         ctypes.byref(st), _stream(stream)))
    return rc, td.value, st


PAMX_NOALLOC_SCRATCH_BYTES = 64 << 20


def pamx_fit(XorD, input_kind, k, medoids, labels, ws, metric=PAMX_L2, opt=None, stream=None):
    n = XorD.shape[0]
    dim = XorD.shape[1] if input_kind == PAMX_INPUT_X else 0
    td = ctypes.c_double()
    st = pamx_stats()
    rc = _check(load().pamx_fit(_ptr(XorD), int(input_kind), _dtype_code(XorD), int(n), int(dim),
                                int(metric), int(k),
                                ctypes.byref(opt) if opt is not None else None, _ptr(medoids),
                                _ptr(labels), ctypes.byref(td), ctypes.byref(st), _ptr(ws),
                                ws.numel() * ws.element_size(), _stream(stream)))
    return rc, td.value, st


def pamx_batched_workspace_bytes(n_inst, N) -> int:
    out = ctypes.c_size_t()
    _check(load().pamx_batched_workspace_bytes(int(n_inst), int(N), ctypes.byref(out)))
    return int(out.value)


def pamx_fit_batched(X, metric, sample_off, sample_idx, k_inst, medoids, ws, opt=None,
                     want_full=True, stream=None):
    """sample_off (int64) and k_inst (int32) are host numpy arrays; X,
    sample_idx, medoids and ws are device tensors.  Returns
    (rc, td_sample ndarray, td_full ndarray or None, stats)."""
    import numpy as np
    N, dim = X.shape
    so = np.ascontiguousarray(sample_off, dtype=np.int64)
    ki = np.ascontiguousarray(k_inst, dtype=np.int32)
    n_inst = len(ki)
    tds = np.zeros(n_inst, np.float64)
    tdf = np.zeros(n_inst, np.float64) if want_full else None
    st = pamx_batch_stats()
    rc = _check(load().pamx_fit_batched(
        _ptr(X), _dtype_code(X), int(N), int(dim), int(metric), int(n_inst),
        so.ctypes.data_as(ctypes.c_void_p), _ptr(sample_idx), ki.ctypes.data_as(ctypes.c_void_p),
        ctypes.byref(opt) if opt is not None else None, _ptr(medoids),
        tds.ctypes.data_as(ctypes.c_void_p),
        tdf.ctypes.data_as(ctypes.c_void_p) if tdf is not None else None, ctypes.byref(st),
        _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))
    return rc, tds, tdf, st


def pamx_last_error() -> str:
    return load().pamx_last_error().decode()


def pamx_init_workspace_bytes(n, m=0) -> int:
    out = ctypes.c_size_t()
    _check(load().pamx_init_workspace_bytes(int(n), int(m), ctypes.byref(out)))
    return int(out.value)


def pamx_init_dw(D, k, u, medoids, ws, n=None, ld=None, stream=None):
    """u: device float64 [k] uniforms in [0, 1)."""
    n = D.shape[0] if n is None else n
    ld = D.stride(0) if ld is None else ld
    return _check(load().pamx_init_dw(_ptr(D), _dtype_code(D), int(n), int(ld), int(k), _ptr(u),
                                      _ptr(medoids), _ptr(ws), ws.numel() * ws.element_size(),
                                      _stream(stream)))


def pamx_init_lab(D, k, samples, medoids, ws, exclude_self=False, n=None, ld=None, stream=None):
    """samples: device int32 (k, m), row t = step t's subsample."""
    n = D.shape[0] if n is None else n
    ld = D.stride(0) if ld is None else ld
    m = int(samples.shape[1])
    return _check(load().pamx_init_lab(_ptr(D), _dtype_code(D), int(n), int(ld), int(k),
                                       _ptr(samples), m, int(bool(exclude_self)), _ptr(medoids),
                                       _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))


def pamx_clarans(D, k, draws, maxneighbor, medoids, ws, labels=None, opt=None, n=None, ld=None,
                 stream=None):
    """draws: device int32 [len]; medoids: device int32 [k], read and overwritten."""
    n = D.shape[0] if n is None else n
    ld = D.stride(0) if ld is None else ld
    td = ctypes.c_double()
    st = pamx_stats()
    rc = _check(load().pamx_clarans(_ptr(D), _dtype_code(D), int(n), int(ld), int(k), _ptr(draws),
                                    int(draws.numel()), int(maxneighbor),
                                    ctypes.byref(opt) if opt is not None else None, _ptr(medoids),
                                    _ptr(labels), ctypes.byref(td), ctypes.byref(st), _ptr(ws),
                                    ws.numel() * ws.element_size(), _stream(stream)))
    return rc, td.value, st


def pamx_best_of_workspace_bytes(n, k, dtype, opt=None) -> int:
    out = ctypes.c_size_t()
    _check(load().pamx_best_of_workspace_bytes(int(n), int(k), int(dtype),
                                               ctypes.byref(opt) if opt is not None else None,
                                               ctypes.byref(out)))
    return int(out.value)


def pamx_swap_restarts(D, k, starts, medoids, ws, labels=None, opt=None, n=None, ld=None,
                       stream=None):
    """starts: device int32 [R, k]; medoids: device int32 [k] output.
    Returns (rc, td, stats, per-restart TDs, best restart)."""
    n = D.shape[0] if n is None else n
    ld = D.stride(0) if ld is None else ld
    R = starts.shape[0]
    td = ctypes.c_double()
    st = pamx_stats()
    each = (ctypes.c_double * R)()
    best = ctypes.c_int32()
    rc = _check(load().pamx_swap_restarts(_ptr(D), _dtype_code(D), int(n), int(ld), int(k), int(R),
                                          _ptr(starts), ctypes.byref(opt) if opt is not None else None,
                                          _ptr(medoids), _ptr(labels), ctypes.byref(td),
                                          ctypes.byref(st), each, ctypes.byref(best), _ptr(ws),
                                          ws.numel() * ws.element_size(), _stream(stream)))
    return rc, td.value, st, list(each), best.value


def pamx_clarans_numlocal(D, k, starts, draws, maxneighbor, medoids, ws, labels=None, opt=None,
                          n=None, ld=None, stream=None):
    """starts: device int32 [numlocal, k]; draws: device int32 [numlocal, len];
    medoids: device int32 [k] output.  Returns (rc, td, stats, per-search
    TDs, best search)."""
    n = D.shape[0] if n is None else n
    ld = D.stride(0) if ld is None else ld
    R, length = draws.shape
    td = ctypes.c_double()
    st = pamx_stats()
    each = (ctypes.c_double * R)()
    best = ctypes.c_int32()
    rc = _check(load().pamx_clarans_numlocal(_ptr(D), _dtype_code(D), int(n), int(ld), int(k),
                                             int(R), _ptr(starts), _ptr(draws), int(length),
                                             int(maxneighbor),
                                             ctypes.byref(opt) if opt is not None else None,
                                             _ptr(medoids), _ptr(labels), ctypes.byref(td),
                                             ctypes.byref(st), each, ctypes.byref(best), _ptr(ws),
                                             ws.numel() * ws.element_size(), _stream(stream)))
    return rc, td.value, st, list(each), best.value


def pamx_rect_workspace_bytes(n_cons, n_loc, k, dtype, opt=None) -> int:
    out = ctypes.c_size_t()
    _check(load().pamx_rect_workspace_bytes(int(n_cons), int(n_loc), int(k), int(dtype),
                                            ctypes.byref(opt) if opt is not None else None,
                                            ctypes.byref(out)))
    return int(out.value)


def pamx_rect(D, k, medoids, ws, labels=None, opt=None, build=True, ld=None, stream=None):
    """D: device (n_cons, n_loc) matrix (row stride ld); build=False starts
    from `medoids` (pamx_swap_rect), else pamx_fit_rect."""
    nco, nl = D.shape
    ld = D.stride(0) if ld is None else ld
    td = ctypes.c_double()
    st = pamx_stats()
    f = load().pamx_fit_rect if build else load().pamx_swap_rect
    rc = _check(f(_ptr(D), _dtype_code(D), int(nco), int(nl), int(ld), int(k),
                  ctypes.byref(opt) if opt is not None else None, _ptr(medoids), _ptr(labels),
                  ctypes.byref(td), ctypes.byref(st), _ptr(ws), ws.numel() * ws.element_size(),
                  _stream(stream)))
    return rc, td.value, st
