"""C-ABI checks that need no GPU: the library loads, exports every entry
point declared in include/pamx.h, and rejects bad arguments on the host
before any device work (so these calls never touch HIP)."""
import ctypes
import os
import re

import pytest

from paper_2008_05171_amd import pamx as abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(abi.LIB_PATH):
        from paper_2008_05171_amd import buildlib
        buildlib.build()
    return abi.load()


def _declared():
    txt = open(os.path.join(ROOT, "include", "pamx.h")).read()
    return sorted(set(re.findall(r"\b(pamx_[a-z_]+)\s*\(", txt)))


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert set(names) == set(abi.EXPORTS)
    for name in names:
        assert hasattr(lib, name), name


def test_struct_sizes_match_header():
    assert ctypes.sizeof(abi.pamx_options) == 48
    assert ctypes.sizeof(abi.pamx_swap_record) == 16
    assert ctypes.sizeof(abi.pamx_stats) == 144


def test_default_options(lib):
    o = abi.pamx_default_options()
    assert (o.variant, o.accum, o.max_iter, o.build_exclude_self, o.trace_cap, o.chunk,
            o.profile) == (abi.PAMX_FASTPAM1, abi.PAMX_ACC_F64, 10000, 0, 0, 0, 0)


def test_workspace_bytes_grows_and_validates(lib):
    a = abi.pamx_workspace_bytes(1000, 5, 0, abi.PAMX_INPUT_D, abi.PAMX_I32)
    b = abi.pamx_workspace_bytes(20000, 100, 0, abi.PAMX_INPUT_D, abi.PAMX_F32)
    c = abi.pamx_workspace_bytes(20000, 100, 16, abi.PAMX_INPUT_X, abi.PAMX_F32)
    assert 0 < a < b < c
    assert c - b >= 20000 * 20032 * 4          # stored matrix, 64-padded rows
    o = abi.pamx_default_options()
    o.variant = abi.PAMX_FASTPAM2
    d = abi.pamx_workspace_bytes(20000, 100, 0, abi.PAMX_INPUT_D, abi.PAMX_F32, o)
    assert d >= b + 100 * 20480 * 8            # per-medoid change buffer
    for args in [(0, 1), (10, 0), (10, 11), (10, 20000), (30000, 16001)]:
        with pytest.raises(abi.PamxError) as e:
            abi.pamx_workspace_bytes(args[0], args[1], 0, abi.PAMX_INPUT_D, abi.PAMX_F32)
        assert e.value.code == abi.PAMX_ERR_ARG
    with pytest.raises(abi.PamxError):
        abi.pamx_workspace_bytes(10, 2, 0, abi.PAMX_INPUT_X, abi.PAMX_F32)   # dim 0
    with pytest.raises(abi.PamxError):
        abi.pamx_workspace_bytes(10, 2, 0, 7, abi.PAMX_F32)


def _call_build(lib, D, dtype, n, ld, k, ws, wsb, opt=None):
    td = ctypes.c_double()
    med = ctypes.c_void_p(0x1000)
    return lib.pamx_build(D, dtype, n, ld, k, ctypes.byref(opt) if opt else None, med,
                          ctypes.byref(td), ws, wsb, None)


def test_host_argument_errors_before_device_work(lib):
    fake = ctypes.c_void_p(0x100000)          # never dereferenced: rejected first
    ws = ctypes.c_void_p(0x200000)
    assert _call_build(lib, None, abi.PAMX_F32, 10, 10, 2, ws, 1 << 30) == abi.PAMX_ERR_ARG
    assert "D is NULL" in abi.pamx_last_error()
    assert _call_build(lib, fake, 9, 10, 10, 2, ws, 1 << 30) == abi.PAMX_ERR_ARG
    assert _call_build(lib, fake, abi.PAMX_F32, 10, 9, 2, ws, 1 << 30) == abi.PAMX_ERR_ARG
    assert _call_build(lib, fake, abi.PAMX_F32, 10, 10, 11, ws, 1 << 30) == abi.PAMX_ERR_ARG
    assert _call_build(lib, fake, abi.PAMX_F32, 10, 10, 0, ws, 1 << 30) == abi.PAMX_ERR_ARG
    assert _call_build(lib, fake, abi.PAMX_F32, 10, 10, 2, ws, 16) == abi.PAMX_ERR_WORKSPACE
    assert "too small" in abi.pamx_last_error()
    assert _call_build(lib, fake, abi.PAMX_F32, 10, 10, 2, ctypes.c_void_p(0x200010),
                       1 << 30) == abi.PAMX_ERR_WORKSPACE
    assert _call_build(lib, fake, abi.PAMX_F32, 10, 10, 2, None, 1 << 30) == abi.PAMX_ERR_WORKSPACE
    o = abi.pamx_default_options()
    o.variant = 4
    assert _call_build(lib, fake, abi.PAMX_F32, 10, 10, 2, ws, 1 << 30, o) == abi.PAMX_ERR_ARG
    o = abi.pamx_default_options()
    o.variant = abi.PAMX_FASTERPAM
    o.window = -1
    assert _call_build(lib, fake, abi.PAMX_F32, 10, 10, 2, ws, 1 << 30, o) == abi.PAMX_ERR_ARG
    assert "window" in abi.pamx_last_error()
    o = abi.pamx_default_options()
    o.accum = abi.PAMX_ACC_F32
    assert _call_build(lib, fake, abi.PAMX_I32, 10, 10, 2, ws, 1 << 30, o) == abi.PAMX_ERR_ARG
    o = abi.pamx_default_options()
    o.trace_cap = 5
    rc = lib.pamx_swap(fake, abi.PAMX_F32, 10, 10, 2, ctypes.byref(o), fake, None, None, None,
                       ws, 1 << 30, None)
    assert rc == abi.PAMX_ERR_ARG and "trace" in abi.pamx_last_error()
    # overflow of n * ld
    assert _call_build(lib, fake, abi.PAMX_F32, 1 << 30, 1 << 40, 2, ws, 1 << 62) == abi.PAMX_ERR_ARG


def test_chunk_tuning_option(lib):
    """chunk = PAMX_CHUNK_TUNE is accepted and sizes the workspace for the
    largest chunk count the tuner may pick; other negative values are errors."""
    o = abi.pamx_default_options()
    base = abi.pamx_workspace_bytes(20000, 100, 16, abi.PAMX_INPUT_X, abi.PAMX_F32, o)
    o.chunk = abi.PAMX_CHUNK_TUNE
    tuned = abi.pamx_workspace_bytes(20000, 100, 16, abi.PAMX_INPUT_X, abi.PAMX_F32, o)
    assert tuned >= base
    o.chunk = -2
    with pytest.raises(abi.PamxError):
        abi.pamx_workspace_bytes(20000, 100, 16, abi.PAMX_INPUT_X, abi.PAMX_F32, o)


def test_fasterpam_window_option(lib):
    """FasterPAM sizes the workspace for its window passes; a wider window
    needs more partials; BF16 distances run FastPAM1 only."""
    o = abi.pamx_default_options()
    o.variant = abi.PAMX_FASTERPAM
    o.window = 1024
    a = abi.pamx_workspace_bytes(20000, 100, 0, abi.PAMX_INPUT_D, abi.PAMX_F32, o)
    o.window = 8192
    b = abi.pamx_workspace_bytes(20000, 100, 0, abi.PAMX_INPUT_D, abi.PAMX_F32, o)
    assert 0 < a <= b
    o.window = 0
    o.dist_mode = abi.PAMX_DIST_BF16
    with pytest.raises(abi.PamxError) as e:
        abi.pamx_workspace_bytes(2000, 10, 8, abi.PAMX_INPUT_X, abi.PAMX_F32, o)
    assert e.value.code == abi.PAMX_ERR_UNSUPPORTED


def test_init_argument_errors(lib):
    """The initialisation entry points reject bad arguments before any
    device work."""
    fake = ctypes.c_void_p(0x100000)
    ws = ctypes.c_void_p(0x200000)
    need = abi.pamx_init_workspace_bytes(1000, 42)
    assert need >= abi.pamx_init_workspace_bytes(1000, 0) > 1000 * 8
    with pytest.raises(abi.PamxError):
        abi.pamx_init_workspace_bytes(1000, 1001)
    dw = lib.pamx_init_dw
    assert dw(None, abi.PAMX_F32, 1000, 1000, 5, fake, fake, ws, 1 << 30, None) == abi.PAMX_ERR_ARG
    assert dw(fake, abi.PAMX_F32, 1000, 1000, 1001, fake, fake, ws, 1 << 30, None) == abi.PAMX_ERR_ARG
    assert dw(fake, abi.PAMX_F32, 1000, 1000, 0, fake, fake, ws, 1 << 30, None) == abi.PAMX_ERR_ARG
    assert dw(fake, 9, 1000, 1000, 5, fake, fake, ws, 1 << 30, None) == abi.PAMX_ERR_ARG
    assert dw(fake, abi.PAMX_F32, 1000, 999, 5, fake, fake, ws, 1 << 30, None) == abi.PAMX_ERR_ARG
    assert dw(fake, abi.PAMX_F32, 1000, 1000, 5, None, fake, ws, 1 << 30, None) == abi.PAMX_ERR_ARG
    assert dw(fake, abi.PAMX_F32, 1000, 1000, 5, fake, None, ws, 1 << 30, None) == abi.PAMX_ERR_ARG
    assert dw(fake, abi.PAMX_F32, 1000, 1000, 5, fake, fake, ws, 64, None) == abi.PAMX_ERR_WORKSPACE
    assert dw(fake, abi.PAMX_F32, 1000, 1000, 5, fake, fake, ctypes.c_void_p(0x200010), 1 << 30,
              None) == abi.PAMX_ERR_WORKSPACE
    lab = lib.pamx_init_lab
    assert lab(fake, abi.PAMX_I32, 1000, 1000, 5, fake, 0, 0, fake, ws, 1 << 30, None) == abi.PAMX_ERR_ARG
    assert lab(fake, abi.PAMX_I32, 1000, 1000, 5, fake, 1001, 0, fake, ws, 1 << 30, None) == abi.PAMX_ERR_ARG
    assert lab(fake, abi.PAMX_I32, 1000, 1000, 5, None, 42, 0, fake, ws, 1 << 30, None) == abi.PAMX_ERR_ARG
    assert lab(fake, abi.PAMX_I32, 1000, 1000, 5, fake, 42, 2, fake, ws, 1 << 30, None) == abi.PAMX_ERR_ARG
    assert lab(fake, abi.PAMX_I32, 1000, 1000, 5, fake, 42, 0, fake, ws, 100, None) == abi.PAMX_ERR_WORKSPACE


def test_clarans_argument_errors(lib):
    fake = ctypes.c_void_p(0x100000)
    ws = ctypes.c_void_p(0x200000)
    cl = lib.pamx_clarans

    def call(D=fake, dtype=abi.PAMX_F32, n=1000, ld=1000, k=5, draws=fake, ln=100, mx=10, opt=None,
             med=fake, wsb=1 << 30):
        return cl(D, dtype, n, ld, k, draws, ln, mx, ctypes.byref(opt) if opt else None, med, None,
                  None, None, ws, wsb, None)
    assert call(D=None) == abi.PAMX_ERR_ARG
    assert call(k=1001) == abi.PAMX_ERR_ARG
    assert call(draws=None) == abi.PAMX_ERR_ARG
    assert call(ln=-1) == abi.PAMX_ERR_ARG
    assert call(mx=0) == abi.PAMX_ERR_ARG
    assert call(med=None) == abi.PAMX_ERR_ARG
    o = abi.pamx_default_options()
    o.variant = abi.PAMX_FASTERPAM
    assert call(opt=o) == abi.PAMX_ERR_ARG
    assert call(wsb=64) == abi.PAMX_ERR_WORKSPACE


def test_rect_argument_errors(lib):
    fake = ctypes.c_void_p(0x100000)
    ws = ctypes.c_void_p(0x200000)

    def call(f, D=fake, nco=500, nl=300, ld=300, k=5, opt=None, med=fake, wsb=1 << 30):
        return f(D, abi.PAMX_F32, nco, nl, ld, k, ctypes.byref(opt) if opt else None, med, None,
                 None, None, ws, wsb, None)
    for f in (lib.pamx_fit_rect, lib.pamx_swap_rect):
        assert call(f, D=None) == abi.PAMX_ERR_ARG
        assert call(f, nco=0) == abi.PAMX_ERR_ARG
        assert call(f, k=301) == abi.PAMX_ERR_ARG
        assert call(f, ld=299) == abi.PAMX_ERR_ARG
        assert call(f, med=None) == abi.PAMX_ERR_ARG
        for v in (abi.PAMX_FASTPAM2, abi.PAMX_FASTERPAM):
            o = abi.pamx_default_options()
            o.variant = v
            assert call(f, opt=o) == abi.PAMX_ERR_UNSUPPORTED
        assert call(f, wsb=64) == abi.PAMX_ERR_WORKSPACE
    a = abi.pamx_rect_workspace_bytes(20000, 500, 50, abi.PAMX_F32)
    assert a > 500 * 20032 * 4                 # holds the transposed matrix
    with pytest.raises(abi.PamxError):
        abi.pamx_rect_workspace_bytes(20000, 500, 501, abi.PAMX_F32)


def test_points_metric_rules(lib):
    fake = ctypes.c_void_p(0x100000)
    rc = lib.pamx_dist(fake, abi.PAMX_I32, 10, 2, abi.PAMX_L2, fake, 12, None, 0, None)
    assert rc == abi.PAMX_ERR_UNSUPPORTED
    rc = lib.pamx_dist(fake, abi.PAMX_F32, 10, 2, abi.PAMX_L1, fake, 12, fake, 256, None)
    assert rc == abi.PAMX_ERR_UNSUPPORTED
    rc = lib.pamx_dist(fake, abi.PAMX_F32, 10, 2, abi.PAMX_L2, fake, 10, fake, 256, None)
    assert rc == abi.PAMX_ERR_ARG          # ld not a multiple of 4
    rc = lib.pamx_dist(fake, abi.PAMX_F32, 10, 0, abi.PAMX_L2, fake, 12, fake, 256, None)
    assert rc == abi.PAMX_ERR_ARG
    rc = lib.pamx_dist(fake, abi.PAMX_F32, 10, 8, abi.PAMX_L2, fake, 12, fake, 31, None)
    assert rc == abi.PAMX_ERR_WORKSPACE    # the 8 coordinate means need 32 bytes
    rc = lib.pamx_dist(fake, abi.PAMX_F32, 10, 8, abi.PAMX_L2, fake, 12, None, 0, None)
    assert rc == abi.PAMX_ERR_WORKSPACE


def test_no_oracle_in_product_path():
    """The product package never imports or loads the CPU oracle."""
    pkg = os.path.join(ROOT, "paper_2008_05171_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "liboracle" not in txt, f


def test_batched_host_argument_errors(lib):
    import numpy as np
    fake = ctypes.c_void_p(0x100000)
    ws = ctypes.c_void_p(0x200000)

    def call(so, ki, dim=8, dtype=abi.PAMX_F32, metric=abi.PAMX_L2, wsb=1 << 30, N=1000):
        so = np.asarray(so, np.int64)
        ki = np.asarray(ki, np.int32)
        tds = np.zeros(len(ki))
        return lib.pamx_fit_batched(fake, dtype, N, dim, metric, len(ki),
                                    so.ctypes.data_as(ctypes.c_void_p), fake,
                                    ki.ctypes.data_as(ctypes.c_void_p), None, fake,
                                    tds.ctypes.data_as(ctypes.c_void_p), None, None, ws, wsb, None)
    assert call([0, 50, 100], [5, 5], wsb=16) == abi.PAMX_ERR_WORKSPACE
    assert call([1, 50], [5]) == abi.PAMX_ERR_ARG                 # sample_off[0] != 0
    assert call([0, 0], [1]) == abi.PAMX_ERR_ARG                  # empty sample
    assert call([0, 10], [11]) == abi.PAMX_ERR_ARG                # k > n'
    assert call([0, 10], [0]) == abi.PAMX_ERR_ARG
    assert call([0, 3000], [5]) == abi.PAMX_ERR_UNSUPPORTED       # n' > 2048
    assert call([0, 2000], [300]) == abi.PAMX_ERR_UNSUPPORTED     # k > 256
    assert call([0, 100], [5], dim=17) == abi.PAMX_ERR_UNSUPPORTED
    assert call([0, 100], [5], dtype=abi.PAMX_I32) == abi.PAMX_ERR_UNSUPPORTED  # int + L2
    assert abi.pamx_batched_workspace_bytes(256, 10 ** 6) > 256 * 256 * 8


def test_check_dissimilarity_argument_errors(lib):
    fake = ctypes.c_void_p(0x100000)
    ws = ctypes.c_void_p(0x200000)
    flags = ctypes.c_int32(-7)

    def call(D=fake, dtype=abi.PAMX_F32, n=100, ld=100, fl=True, w=ws, wsb=256):
        return lib.pamx_check_dissimilarity(D, dtype, n, ld, ctypes.byref(flags) if fl else None,
                                            None, w, wsb, None)
    assert call(D=None) == abi.PAMX_ERR_ARG
    assert call(dtype=7) == abi.PAMX_ERR_ARG
    assert call(n=0) == abi.PAMX_ERR_ARG
    assert call(ld=99) == abi.PAMX_ERR_ARG
    assert call(fl=False) == abi.PAMX_ERR_ARG
    assert call(w=None) == abi.PAMX_ERR_WORKSPACE
    assert call(wsb=4) == abi.PAMX_ERR_WORKSPACE
    assert flags.value == -7   # nothing written on an argument error


def test_read_probe_argument_errors(lib):
    fake = ctypes.c_void_p(0x100000)
    sums = ctypes.c_void_p(0x200000)

    def call(D=fake, n=2000, ld=2000, chunk=100, s=sums, slen=40):
        return lib.pamx_read_probe(D, n, ld, chunk, s, slen, None)
    assert call(D=None) == abi.PAMX_ERR_ARG
    assert call(n=0) == abi.PAMX_ERR_ARG
    assert call(ld=1999) == abi.PAMX_ERR_ARG
    assert call(ld=2002) == abi.PAMX_ERR_ARG                    # ld % 4 != 0
    assert call(D=ctypes.c_void_p(0x100004)) == abi.PAMX_ERR_ARG  # not 16-byte aligned
    assert call(chunk=0) == abi.PAMX_ERR_ARG
    assert call(n=100000, ld=100000, chunk=1, slen=10 ** 9) == abi.PAMX_ERR_ARG  # > 65535 chunks
    assert call(s=None) == abi.PAMX_ERR_ARG
    assert call(slen=39) == abi.PAMX_ERR_ARG   # 2 tiles x 20 chunks = 40 sums


def test_noalloc_host_errors(lib):
    """pamx_swap_noalloc refuses, before any device work, arguments whose
    workspace exceeds its fixed scratch and the options that would create
    events or graphs."""
    fake = ctypes.c_void_p(0x100000)          # never dereferenced: rejected first

    def call(n, k, opt=None, dtype=abi.PAMX_F32):
        return lib.pamx_swap_noalloc(fake, dtype, n, n, k, ctypes.byref(opt) if opt else None,
                                     fake, None, None, None, None)

    o2 = abi.pamx_default_options()
    o2.variant = abi.PAMX_FASTPAM2        # 500 x 1e5 per-medoid changes: 400 MB
    assert abi.pamx_workspace_bytes(100000, 500, 0, abi.PAMX_INPUT_D, abi.PAMX_F32,
                                    o2) > abi.PAMX_NOALLOC_SCRATCH_BYTES
    assert call(100000, 500, o2) == abi.PAMX_ERR_WORKSPACE
    assert "scratch" in abi.pamx_last_error()
    for field in ("profile", "graph"):
        o = abi.pamx_default_options()
        setattr(o, field, 1)
        assert call(1000, 5, o) == abi.PAMX_ERR_ARG
        assert field in abi.pamx_last_error()
    o = abi.pamx_default_options()
    o.chunk = abi.PAMX_CHUNK_TUNE
    assert call(1000, 5, o) == abi.PAMX_ERR_ARG
    assert call(10, 11) == abi.PAMX_ERR_ARG
    assert lib.pamx_swap_noalloc(None, abi.PAMX_F32, 10, 10, 2, None, fake, None, None, None,
                                 None) == abi.PAMX_ERR_ARG


def test_int_points_workspace_rule(lib):
    """Integer points need 8 bytes per coordinate of scratch (the range check)."""
    fake = ctypes.c_void_p(0x100000)
    rc = lib.pamx_dist(fake, abi.PAMX_I32, 10, 2, abi.PAMX_L1, fake, 12, None, 0, None)
    assert rc == abi.PAMX_ERR_WORKSPACE
    rc = lib.pamx_dist(fake, abi.PAMX_I32, 10, 2, abi.PAMX_L1, fake, 12, fake, 15, None)
    assert rc == abi.PAMX_ERR_WORKSPACE
    a = abi.pamx_workspace_bytes(1000, 5, 8, abi.PAMX_INPUT_X, abi.PAMX_I32)
    b = abi.pamx_workspace_bytes(1000, 5, 8, abi.PAMX_INPUT_D, abi.PAMX_I32)
    assert a >= b + 1000 * 1000 * 4 + 64


def test_best_of_host_argument_errors(lib):
    """Restarts and numlocal searches: argument errors come back before any
    device work (fake device pointers are never touched)."""
    fake = ctypes.c_void_p(0x100000)
    ws = ctypes.c_void_p(0x200000)
    n, k = 300, 5
    need = abi.pamx_best_of_workspace_bytes(n, k, abi.PAMX_I32)
    assert need > abi.pamx_workspace_bytes(n, k, 0, abi.PAMX_INPUT_D, abi.PAMX_I32) + n * 4
    td, st, best = ctypes.c_double(), abi.pamx_stats(), ctypes.c_int32()

    def restarts(R=3, starts=fake, wsb=need, opt=None):
        return lib.pamx_swap_restarts(fake, abi.PAMX_I32, n, n, k, R, starts, opt, fake, None,
                                      ctypes.byref(td), ctypes.byref(st), None,
                                      ctypes.byref(best), ws, wsb, None)

    assert restarts(R=0) == abi.PAMX_ERR_ARG
    assert restarts(starts=None) == abi.PAMX_ERR_ARG
    assert restarts(wsb=need - 1) == abi.PAMX_ERR_WORKSPACE

    def numlocal(R=2, starts=fake, draws=fake, length=100, maxn=5, wsb=need, opt=None):
        return lib.pamx_clarans_numlocal(fake, abi.PAMX_I32, n, n, k, R, starts, draws, length,
                                         maxn, opt, fake, None, ctypes.byref(td),
                                         ctypes.byref(st), None, ctypes.byref(best), ws, wsb, None)

    assert numlocal(R=0) == abi.PAMX_ERR_ARG
    assert numlocal(starts=None) == abi.PAMX_ERR_ARG
    assert numlocal(draws=None) == abi.PAMX_ERR_ARG
    assert numlocal(maxn=0) == abi.PAMX_ERR_ARG
    assert numlocal(wsb=need - 1) == abi.PAMX_ERR_WORKSPACE
    o = abi.pamx_default_options()
    o.trace = 0x300000
    o.trace_cap = 10
    assert numlocal(opt=ctypes.byref(o)) == abi.PAMX_ERR_ARG
    o = abi.pamx_default_options()
    o.variant = abi.PAMX_FASTPAM2
    assert numlocal(opt=ctypes.byref(o)) == abi.PAMX_ERR_ARG
