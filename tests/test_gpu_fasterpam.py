"""GPU parity of FasterPAM (Alg. 4): the HIP window scan against the oracle.

Integer dissimilarities: bit-exact medoids, labels, TD, the whole swap
trajectory (slot, candidate, change) and the number of passes, against the
oracle's sequential scan (reading R13), for several window widths (one
window per pass, many windows per pass with wrap-around, the 1-wide load
path).  Float dissimilarities: the same FP32 matrix on both sides; the GPU's
swaps are replayed on the oracle: each change agrees within the FP64
summation bound, the chosen slot is the candidate's best, and every candidate
the scan passed without a swap has no change below minus that bound.
"""
import numpy as np
import pytest

import oracle
from paper_2008_05171_amd import datagen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def px():
    import paper_2008_05171_amd as m
    return m


def _say(*a):
    print("[case]", *a, flush=True)


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _int_case(n, seed, hi=1000, dim=2):
    X = datagen.int_points(n, dim, 0, hi, seed=seed)
    return X, oracle.dist_matrix(X, oracle.L1)


def _check_same(res, ref):
    assert list(res.medoids.cpu().numpy()) == list(ref.medoids)
    assert res.td == ref.td
    assert res.trace == ref.trace
    assert res.stats["swaps"] == ref.swaps
    assert res.stats["iterations"] == ref.iterations


# ------------------------------------------------------------------ integer: exact
@pytest.mark.parametrize("seed", list(range(1001, 1009)))
def test_fit_l1_int_bitexact(seed):
    """n=1000 integer points, Manhattan, k=5: BUILD + FasterPAM vs the oracle."""
    _say("fasterpam_fit_l1_int", seed)
    X, D = _int_case(1000, seed)
    ref = oracle.pam(5, D=D, variant=oracle.FASTERPAM)
    res = px().fit(_t(X), 5, variant="fasterpam", trace=True)
    assert res.rc == 0 and res.stats["converged"] == 1
    assert res.stats["td_build"] == ref.td_build
    _check_same(res, ref)
    assert np.array_equal(res.labels.cpu().numpy(), ref.labels)


@pytest.mark.parametrize("n,k,hi,seed,window", [
    (200, 2, 10, 1, 0), (200, 5, 10, 2, 0), (1000, 10, 10, 3, 256), (1000, 5, 10, 4, 0),
    (333, 7, 6, 5, 0), (1000, 30, 30, 6, 0), (3000, 12, 40, 7, 1024), (3000, 40, 100, 8, 2048)])
def test_swap_random_start_bitexact(n, k, hi, seed, window):
    """Random starting medoids (many swaps, dense at first), tie-heavy
    coordinates; windows narrower than n make each pass several windows and
    the scan wrap around."""
    _say("fasterpam_random_start", n, k, hi, seed, window)
    X, D = _int_case(n, seed, hi=hi)
    start = np.random.default_rng(seed).choice(n, size=k, replace=False).astype(np.int32)
    ref = oracle.swap(start, D=D, variant=oracle.FASTERPAM)
    res = px().swap(_t(D.astype(np.int32)), _t(start), variant="fasterpam", trace=True,
                    window=window)
    assert res.rc == 0
    _check_same(res, ref)
    assert res.stats["windows"] >= 1 and res.stats["window"] >= 256
    assert (res.stats["scan_positions"] + n - 1) // n == ref.iterations


@pytest.mark.parametrize("window", [256, 1024, 4096])
def test_window_width_does_not_change_results(window):
    _say("fasterpam_window", window)
    X, D = _int_case(2500, 21, hi=300)
    start = np.arange(0, 2500, 125, dtype=np.int32)[:20]
    ref = oracle.swap(start, D=D, variant=oracle.FASTERPAM)
    res = px().swap(_t(D.astype(np.int32)), _t(start), variant="fasterpam", trace=True,
                    window=window)
    _check_same(res, ref)


_GROUP_CASE = {}


@pytest.mark.parametrize("group", [1, 2, 4])
def test_window_chunk_groups(group, monkeypatch):
    """The window pass merges 1, 2 or 4 consecutive object chunks in each
    work-group (PAMX_FP_GROUP fixes the choice): n = 2990 makes 187 chunks of
    16 objects, so the last group is short for 2 and 4.  Bit-exact against
    the oracle's scan on integer distances (rows padded to 2992: 4-wide
    loads); on an FP32 matrix (rows of 2990: 1-wide loads; the FP64 sums of a
    chunk group are added in another order) every choice gives the same
    swaps, medoids and labels as 4, the changes and TD equal to 1e-12."""
    _say("fasterpam_groups", group)
    if not _GROUP_CASE:
        X, D = _int_case(2990, 91, hi=400)
        start = np.random.default_rng(91).choice(2990, size=40, replace=False).astype(np.int32)
        _GROUP_CASE["int"] = (D, start, oracle.swap(start, D=D, variant=oracle.FASTERPAM))
        Xf = datagen.gaussian_mixture(2990, 8, 30, seed=92)
        Df = oracle.dist_matrix(Xf.astype(np.float64), oracle.L2).astype(np.float32)
        monkeypatch.setenv("PAMX_FP_GROUP", "4")
        _GROUP_CASE["float"] = (Df, px().fit(_t(Df), 30, input_kind=px().PAMX_INPUT_D,
                                             variant="fasterpam", trace=True))
    D, start, ref = _GROUP_CASE["int"]
    monkeypatch.setenv("PAMX_FP_GROUP", str(group))
    Dp = np.zeros((2990, 2992), np.int32)
    Dp[:, :2990] = D
    res = px().swap(_t(Dp)[:, :2990], _t(start), variant="fasterpam", trace=True)
    _check_same(res, ref)
    Df, f4 = _GROUP_CASE["float"]
    f = px().fit(_t(Df), 30, input_kind=px().PAMX_INPUT_D, variant="fasterpam", trace=True)
    assert [(i, c) for i, c, _ in f.trace] == [(i, c) for i, c, _ in f4.trace]
    for (_, _, v), (_, _, v4) in zip(f.trace, f4.trace):
        assert abs(v - v4) <= 1e-12 * f4.td
    assert torch.equal(f.medoids, f4.medoids) and torch.equal(f.labels, f4.labels)
    assert abs(f.td - f4.td) <= 1e-12 * f4.td


def test_more_medoids_than_lds_staging():
    """k above the 4096 medoids a work-group stages in LDS: the window step
    falls back to the separate decision, rescan and count launches (random
    start, integer distances, bit-exact against the oracle's scan)."""
    _say("fasterpam_k4100")
    X, D = _int_case(4300, 95, hi=3000)
    start = np.random.default_rng(95).choice(4300, size=4100, replace=False).astype(np.int32)
    ref = oracle.swap(start, D=D, variant=oracle.FASTERPAM)
    res = px().swap(_t(D.astype(np.int32)), _t(start), variant="fasterpam", trace=True)
    assert res.rc == 0
    _check_same(res, ref)


def test_unaligned_ld_uses_scalar_loads():
    """A leading dimension that is not a multiple of 4 takes the 1-wide
    load path (256-candidate tiles, windows at any position)."""
    _say("fasterpam_unaligned")
    X, D = _int_case(901, 31, hi=200)
    Dp = np.zeros((901, 903), np.int32)
    Dp[:, :901] = D
    start = np.random.default_rng(31).choice(901, size=9, replace=False).astype(np.int32)
    ref = oracle.swap(start, D=D, variant=oracle.FASTERPAM)
    Dt = _t(Dp)[:, :901]
    res = px().swap(Dt, _t(start), variant="fasterpam", trace=True, window=512)
    _check_same(res, ref)


def test_max_iter_and_converged_start():
    _say("fasterpam_max_iter")
    X, D = _int_case(1200, 41, hi=500)
    Di = _t(D.astype(np.int32))
    start = np.arange(8, dtype=np.int32)
    full = oracle.swap(start, D=D, variant=oracle.FASTERPAM)
    assert full.iterations >= 2
    capped = px().swap(Di, _t(start), variant="fasterpam", trace=True, max_iter=1)
    assert capped.rc == 1 and capped.stats["converged"] == 0
    assert capped.stats["iterations"] == 1
    assert capped.stats["scan_positions"] == 1200
    assert capped.trace == full.trace[:capped.stats["swaps"]]
    again = px().swap(Di, _t(np.array(full.medoids, np.int32)), variant="fasterpam", trace=True)
    assert again.rc == 0 and again.stats["swaps"] == 0 and again.stats["iterations"] == 1
    assert again.td == full.td
    none = px().swap(Di, _t(start), variant="fasterpam", max_iter=0)
    assert none.rc == 1 and none.stats["swaps"] == 0


@pytest.mark.parametrize("n,k", [(1, 1), (2, 1), (2, 2), (3, 2), (5, 5), (50, 1)])
def test_degenerate_sizes(n, k):
    _say("fasterpam_degenerate", n, k)
    X, D = _int_case(n, 50 + n, hi=20)
    ref = oracle.pam(k, D=D, variant=oracle.FASTERPAM)
    res = px().fit(_t(X), k, variant="fasterpam", trace=True)
    assert list(res.medoids.cpu().numpy()) == list(ref.medoids)
    assert res.td == ref.td
    assert res.trace == ref.trace


def test_duplicates_and_bitwise_rerun():
    _say("fasterpam_duplicates")
    X, D = _int_case(800, 61, hi=4)        # 16 distinct points
    ref = oracle.pam(6, D=D, variant=oracle.FASTERPAM)
    a = px().fit(_t(X), 6, variant="fasterpam", trace=True)
    b = px().fit(_t(X), 6, variant="fasterpam", trace=True)
    _check_same(a, ref)
    assert a.trace == b.trace and torch.equal(a.labels, b.labels)


def test_graph_replays_equal_direct_launches():
    """Window steps replayed from a captured HIP graph equal direct launches."""
    _say("fasterpam_graph")
    X, D = _int_case(1500, 71, hi=80)
    start = np.random.default_rng(71).choice(1500, size=10, replace=False).astype(np.int32)
    ref = oracle.swap(start, D=D, variant=oracle.FASTERPAM)
    Di = _t(D.astype(np.int32))
    g = px().swap(Di, _t(start), variant="fasterpam", trace=True, graph=True, window=512)
    torch.cuda.synchronize()
    d = px().swap(Di, _t(start), variant="fasterpam", trace=True, graph=False, window=512)
    _check_same(g, ref)
    _check_same(d, ref)


# ------------------------------------------------------------------ float: replayed on the oracle
def check_float_trajectory(D64, start, res, sample=None, seed=0):
    """Replays the GPU's swaps on the oracle (FP64 sums of the same matrix).

    tol = 16 n 2^-53 S with S = sum(dn + ds) bounds the difference of two FP64
    summation orders plus the GPU's acceptance threshold (a swap is taken
    when its change is below minus the summation bound).  Candidates scanned
    between swaps are checked all, or `sample` of them per gap."""
    n = D64.shape[0]
    rng = np.random.default_rng(seed)
    med = [int(v) for v in start]
    pos = 0
    visited = 0
    checked = 0
    trace = list(res.trace)
    assert len(trace) == res.stats["swaps"]

    def tol_of(m):
        _, dn, ds = oracle.nearest(m, D=D64)
        return 16 * n * 2.0 ** -53 * float((dn + ds).sum())

    def quiet_ok(m, cands, tol):
        nonlocal checked
        cands = [c for c in cands if c not in set(m)]
        if sample is not None and len(cands) > sample:
            cands = sorted(rng.choice(cands, size=sample, replace=False).tolist())
        if not cands:
            return
        ch = oracle.swap_list(m, cands, D=D64)
        assert np.nanmin(ch) >= -tol, (float(np.nanmin(ch)), tol)
        checked += len(cands)

    for (i, c, dl) in trace:
        tol = tol_of(med)
        gap = (c - pos) % n
        quiet_ok(med, [(pos + j) % n for j in range(gap)], tol)
        ch = oracle.swap_list(med, [c], D=D64)[0]
        assert dl < 0
        assert abs(ch[i] - dl) <= tol, (i, c, float(ch[i]), dl, tol)
        assert ch[i] <= np.nanmin(ch) + 2 * tol
        visited += gap + 1
        med[i] = c
        pos = (c + 1) % n
    # the final pass found nothing: every candidate is certified
    tol = tol_of(med)
    quiet_ok(med, [(pos + j) % n for j in range(n)], tol)
    visited += n
    assert list(res.medoids.cpu().numpy()) == med
    if res.stats["converged"]:
        assert res.stats["scan_positions"] == visited
    td, lab = oracle.td(med, D=D64)
    assert abs(res.td - td) <= 8 * n * 2.0 ** -53 * td
    assert np.array_equal(res.labels.cpu().numpy(), lab)
    return checked


@pytest.mark.parametrize("window", [0, 256])
def test_float_matrix_replayed_on_oracle(window):
    _say("fasterpam_float", window)
    X = datagen.gaussian_mixture(1500, 8, 12, seed=81)
    D32 = oracle.dist_matrix(X.astype(np.float64)).astype(np.float32)
    D64 = D32.astype(np.float64)
    start = np.random.default_rng(81).choice(1500, size=15, replace=False).astype(np.int32)
    res = px().swap(_t(D32), _t(start), variant="fasterpam", trace=True, window=window)
    assert res.rc == 0 and res.stats["swaps"] > 5
    n_checked = check_float_trajectory(D64, start, res)
    assert n_checked > 1500


def test_float_fit_points_build_init():
    """Points through the GPU's own FP32 matrix, BUILD then FasterPAM: the
    result is a local optimum of that matrix (full certificate) and its TD is
    no worse than FastPAM1's beyond the paper's reported noise."""
    _say("fasterpam_points")
    X = datagen.gaussian_mixture(3000, 16, 20, seed=91)
    a = px().fit(_t(X), 20, variant="fasterpam", trace=True)
    b = px().fit(_t(X), 20, variant="fastpam1")
    assert a.rc == 0 and b.rc == 0
    Dg = px().dist(_t(X))
    bm = px().build(Dg, 20)[0]
    s = px().swap(Dg, bm, variant="fasterpam", trace=True)
    assert torch.equal(s.medoids, a.medoids) and s.trace == a.trace and s.td == a.td
    D64 = Dg.cpu().numpy().astype(np.float64)
    check_float_trajectory(D64, bm.cpu().numpy(), a, sample=256, seed=91)
    assert a.td <= b.td * 1.01
