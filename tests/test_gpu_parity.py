"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Integer dissimilarities: bit-exact medoids, labels, TD and the whole swap
trajectory (FastPAM1 performs exactly PAM's swaps, Sec. 3.1; ties broken by
(change, slot, candidate), the order of Alg. 2).  Float dissimilarities:
the same FP32 matrix is given to both sides (the oracle widens it to FP64);
the GPU sums in FP64, so results agree up to FP64 rounding.
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


# ------------------------------------------------------------------ distances
@pytest.mark.parametrize("n", [1000, 1001, 37, 64])
def test_dist_l1_int_exact(n):
    _say("dist_l1", n)
    X, Dref = _int_case(n, seed=7 + n)
    D = px().dist(_t(X)).cpu().numpy()
    assert np.array_equal(D.astype(np.float64), Dref)


@pytest.mark.parametrize("n,dim", [(500, 16), (1001, 3), (130, 70), (65, 1), (300, 17), (257, 33),
                                   (200, 64), (129, 65)])
def test_dist_l2_f32(n, dim):
    _say("dist_l2", n, dim)
    X = datagen.gaussian_mixture(n, dim, 5, seed=n + dim)
    D = px().dist(_t(X)).cpu().numpy()
    Dref = oracle.dist_matrix(X.astype(np.float64), oracle.L2)
    assert np.array_equal(D, D.T), "not bitwise symmetric"
    assert np.all(np.diag(D) == 0)
    # Gram-form error: |d^2 - d_ref^2| <= c * u * (|x|^2 + |y|^2) (uncentred X here)
    nrm = (X.astype(np.float64) ** 2).sum(1)
    bound = (dim + 8) * 2.0 ** -23 * (nrm[:, None] + nrm[None, :]) + 1e-6
    err = np.abs(D.astype(np.float64) ** 2 - Dref ** 2)
    assert np.all(err <= bound), float((err / bound).max())


# ------------------------------------------------------------------ integer FastPAM1 == PAM
def _check_same(res, ref, k):
    med = res.medoids.cpu().numpy()
    lab = res.labels.cpu().numpy()
    assert list(med) == list(ref.medoids)
    assert np.array_equal(lab, ref.labels)
    assert res.td == ref.td
    assert [(s, c) for s, c, _ in res.trace] == [(s, c) for s, c, _ in ref.trace]
    assert [d for _, _, d in res.trace] == [d for _, _, d in ref.trace]


@pytest.mark.parametrize("seed", list(range(1001, 1033)))
def test_l1_int_fit_bitexact(seed):
    """n=1000, d=2 integer points, Manhattan, k=5: BUILD + FastPAM1 vs PAM."""
    _say("fit_l1_int", seed)
    X, D = _int_case(1000, seed)
    ref = oracle.pam(5, D=D)
    res = px().fit(_t(X), 5, trace=True)
    assert res.rc == 0
    assert res.stats["td_build"] == ref.td_build
    assert res.stats["iterations"] == ref.iterations == ref.swaps + 1
    _check_same(res, ref, 5)


@pytest.mark.parametrize("n,k,hi,seed", [(200, 2, 10, 1), (200, 5, 10, 2), (1000, 10, 10, 3),
                                         (1000, 5, 10, 4), (333, 7, 6, 5), (1000, 30, 30, 6)])
def test_tie_stress_bitexact(n, k, hi, seed):
    """Coordinates in [0, hi): many equal distances and duplicate points."""
    _say("tie_stress", n, k, hi, seed)
    X, D = _int_case(n, seed, hi=hi)
    ref = oracle.pam(k, D=D)
    res = px().fit(_t(X), k, trace=True)
    _check_same(res, ref, k)


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_swap_from_random_medoids_bitexact(seed):
    _say("swap_random_init", seed)
    X, D = _int_case(700, seed, hi=300)
    rng = np.random.default_rng(seed)
    start = rng.choice(700, size=12, replace=False).astype(np.int32)
    ref = oracle.swap(start, D=D)
    res = px().swap(_t(D.astype(np.int32)), _t(start), trace=True)
    assert list(res.medoids.cpu().numpy()) == list(ref.medoids)
    assert res.td == ref.td
    assert [(s, c, d) for s, c, d in res.trace] == ref.trace
    assert res.stats["iterations"] == ref.iterations


@pytest.mark.parametrize("chunk", [8, 16, 40, 1000])
def test_chunk_carries_do_not_change_results(chunk):
    """Small object chunks cut segments in many places (carry merging)."""
    _say("chunk", chunk)
    X, D = _int_case(611, 99, hi=200)
    ref = oracle.pam(9, D=D)
    res = px().fit(_t(X), 9, trace=True, chunk=chunk)
    _check_same(res, ref, 9)


@pytest.mark.parametrize("variant", ["fastpam1", "fastpam2"])
@pytest.mark.parametrize("n,chunk", [(4200, 4096), (5000, 4104), (6000, 6000)])
def test_long_chunks_prefetching_loop(n, chunk, variant):
    """Chunks of 4096 rows and more take the prefetching row loop (the next
    block's rows issued before the current block is summed): one chunk, two
    chunks with a ragged second one, segments cut at a chunk edge; bit-exact
    against the oracle's PAM and FastPAM2 reading."""
    _say("long_chunk", n, chunk, variant)
    X, D = _int_case(n, 123 + n)
    ref = oracle.pam(6, D=D, variant=oracle.PAM if variant == "fastpam1" else oracle.FASTPAM2)
    res = px().fit(_t(X), 6, trace=True, chunk=chunk, variant=variant)
    assert res.stats["chunk"] == chunk
    _check_same(res, ref, 6)


_MANY_SEG = {}


@pytest.mark.parametrize("chunk", [4096, 4200])
def test_long_chunks_many_segments(chunk):
    """FastPAM2 over long chunks holding many segments (k = 40: about 40
    segment values per wave and chunk, several times the per-wave ring of P
    values that the pass's writer wave drains): bit-exact against the
    oracle's FastPAM2 reading, with two chunks (ragged second) and one."""
    _say("long_chunk_many_segments", chunk)
    if not _MANY_SEG:
        X, D = _int_case(4200, 4209)
        _MANY_SEG["X"] = X
        _MANY_SEG["ref"] = oracle.pam(40, D=D, variant=oracle.FASTPAM2)
    res = px().fit(_t(_MANY_SEG["X"]), 40, trace=True, chunk=chunk, variant="fastpam2")
    assert res.stats["chunk"] == chunk
    _check_same(res, _MANY_SEG["ref"], 40)


def test_chunk_tuning_keeps_results():
    """Chunk tuning times the pass for several chunk lengths and keeps the
    fastest; on integer distances every chunking gives the same sums, so the
    run equals the oracle's, and a second call reuses the tuned length."""
    _say("chunk_tune")
    X, D = _int_case(4000, 41, hi=300)
    ref = oracle.pam(12, D=D)
    a = px().fit(_t(X), 12, trace=True, chunk=px().PAMX_CHUNK_TUNE)
    _check_same(a, ref, 12)
    b = px().fit(_t(X), 12, trace=True, chunk=px().PAMX_CHUNK_TUNE)
    _check_same(b, ref, 12)
    assert a.stats["chunk"] == b.stats["chunk"] > 0
    print("tuned chunk", a.stats["chunk"], flush=True)


@pytest.mark.parametrize("variant", ["fastpam1", "fastpam2"])
def test_graph_replays_equal_direct_launches(variant):
    """The searches replayed from a captured HIP graph (with host polls and
    the caller's own work between batches) equal directly launched ones, bit
    for bit, on integer and float matrices, and the integer run is the oracle's."""
    _say("graph", variant)
    X, D = _int_case(1500, 51, hi=60)
    ref = oracle.pam(7, D=D, variant=oracle.FASTPAM2 if variant == "fastpam2" else oracle.PAM)
    g = px().fit(_t(X), 7, variant=variant, trace=True, graph=True)
    d = px().fit(_t(X), 7, variant=variant, trace=True, graph=False)
    _check_same(g, ref, 7)
    assert g.trace == d.trace and torch.equal(g.medoids, d.medoids)
    assert torch.equal(g.labels, d.labels) and g.td == d.td
    Xf = datagen.gaussian_mixture(3000, 8, 12, seed=52)
    g = px().fit(_t(Xf), 15, variant=variant, trace=True, graph=True)
    torch.cuda.synchronize()
    filler = torch.ones(1 << 20, device=DEV).cumsum(0)   # the caller's own work in between
    d = px().fit(_t(Xf), 15, variant=variant, trace=True, graph=False)
    assert g.trace == d.trace and torch.equal(g.medoids, d.medoids) and g.td == d.td
    assert float(filler[-1]) == float(1 << 20)


def test_unaligned_leading_dimension():
    """n not a multiple of 4 with ld = n: the scalar-load pass variant."""
    _say("ld_unaligned")
    X, D = _int_case(517, 5, hi=100)
    ref = oracle.pam(6, D=D)
    res = px().fit(_t(D.astype(np.int32)), 6, input_kind=px().PAMX_INPUT_D, trace=True)
    _check_same(res, ref, 6)


# ------------------------------------------------------------------ FastPAM2 reading
@pytest.mark.parametrize("seed,n,k,hi", [(21, 400, 8, 50), (22, 1000, 5, 1000), (23, 300, 12, 10)])
def test_fastpam2_int_bitexact(seed, n, k, hi):
    _say("fastpam2", seed, n, k)
    X, D = _int_case(n, seed, hi=hi)
    ref = oracle.pam(k, D=D, variant=oracle.FASTPAM2)
    res = px().fit(_t(X), k, variant="fastpam2", trace=True)
    _check_same(res, ref, k)
    assert res.stats["iterations"] == ref.iterations


@pytest.mark.parametrize("seed,n,k,hi", [(24, 900, 20, 100), (25, 2000, 40, 1000)])
def test_fastpam2_one_workgroup_apply_equals_grid(seed, n, k, hi, monkeypatch):
    """The eager apply over the whole chip (cooperative launch) and the
    one-work-group form (PAMX_COOPERATIVE=0) perform the same visits and
    swaps: both bit-exact against the oracle on integer distances."""
    _say("fastpam2_coop", seed, n, k)
    X, D = _int_case(n, seed, hi=hi)
    ref = oracle.pam(k, D=D, variant=oracle.FASTPAM2)
    grid = px().fit(_t(X), k, variant="fastpam2", trace=True)
    monkeypatch.setenv("PAMX_COOPERATIVE", "0")
    one = px().fit(_t(X), k, variant="fastpam2", trace=True)
    _check_same(grid, ref, k)
    _check_same(one, ref, k)


_EG_CASES = {}


@pytest.mark.parametrize("case,cap", [("n2000", 4), ("n2000", 8), ("n4200", 1), ("n4200", 2),
                                      ("n4200", 4), ("n4200", 8)])
def test_fastpam2_eager_register_forms(case, cap, monkeypatch):
    """The cooperative eager apply holds each thread's objects in registers,
    in forms for 1, 2, 4, 8 and 16 objects per thread, and reads them from
    memory at every visit above that.  Capping the grid (PAMX_EAGER_GRID)
    sends small inputs through each form: n = 2000 on 4 and 8 work-groups
    (2 and 1 objects per thread), n = 4200 on 1, 2, 4 and 8 (17: the memory
    form, then 9, 5, 3: the 16, 8 and 4 forms).  Bit-exact against the
    oracle's FastPAM2 reading on integer distances."""
    _say("fastpam2_eager_forms", case, cap)
    if case not in _EG_CASES:
        if case == "n2000":
            X, D = _int_case(2000, 25, hi=1000)
            _EG_CASES[case] = (X, oracle.pam(40, D=D, variant=oracle.FASTPAM2))
        else:
            if not _MANY_SEG:
                X, D = _int_case(4200, 4209)
                _MANY_SEG["X"] = X
                _MANY_SEG["ref"] = oracle.pam(40, D=D, variant=oracle.FASTPAM2)
            _EG_CASES[case] = (_MANY_SEG["X"], _MANY_SEG["ref"])
    X, ref = _EG_CASES[case]
    monkeypatch.setenv("PAMX_EAGER_GRID", str(cap))
    res = px().fit(_t(X), 40, variant="fastpam2", trace=True)
    _check_same(res, ref, 40)


def test_fastpam2_one_workgroup_apply_float(monkeypatch):
    """FP32 matrix: the two forms add the re-score sums in different orders,
    so only rounding may differ; the swaps are the same."""
    _say("fastpam2_coop_float")
    X = datagen.gaussian_mixture(3000, 8, 30, seed=26)
    D32 = oracle.dist_matrix(X.astype(np.float64), oracle.L2).astype(np.float32)
    grid = px().fit(_t(D32), 30, input_kind=px().PAMX_INPUT_D, variant="fastpam2", trace=True)
    monkeypatch.setenv("PAMX_COOPERATIVE", "0")
    one = px().fit(_t(D32), 30, input_kind=px().PAMX_INPUT_D, variant="fastpam2", trace=True)
    assert [(s, c) for s, c, _ in grid.trace] == [(s, c) for s, c, _ in one.trace]
    assert torch.equal(grid.medoids, one.medoids) and torch.equal(grid.labels, one.labels)
    assert abs(grid.td - one.td) <= 1e-12 * one.td


# ------------------------------------------------------------------ float matrices
@pytest.mark.parametrize("variant", ["fastpam1", "fastpam2"])
def test_float_matrix_matches_oracle(variant):
    """Same FP32 matrix on both sides; FP64 sums on the GPU."""
    _say("float_D", variant)
    X = datagen.gaussian_mixture(1500, 8, 12, seed=5)
    D32 = oracle.dist_matrix(X.astype(np.float64), oracle.L2).astype(np.float32)
    D64 = D32.astype(np.float64)
    ref = oracle.pam(15, D=D64, variant=oracle.PAM if variant == "fastpam1" else oracle.FASTPAM2)
    res = px().fit(_t(D32), 15, input_kind=px().PAMX_INPUT_D, variant=variant, trace=True)
    assert list(res.medoids.cpu().numpy()) == list(ref.medoids)
    assert np.array_equal(res.labels.cpu().numpy(), ref.labels)
    assert abs(res.td - ref.td) <= 1e-9 * ref.td
    assert [(s, c) for s, c, _ in res.trace] == [(s, c) for s, c, _ in ref.trace]
    np.testing.assert_allclose([d for *_, d in res.trace], [d for *_, d in ref.trace],
                               rtol=1e-9, atol=1e-9 * ref.td)


def test_float_points_fit_close_to_oracle():
    """Distances computed on the GPU (FP32 Gram on MFMA) vs FP64 oracle ones."""
    _say("float_X")
    X = datagen.gaussian_mixture(2000, 16, 20, seed=1002)
    D64 = oracle.dist_matrix(X.astype(np.float64), oracle.L2)
    ref = oracle.pam(20, D=D64)
    res = px().fit(_t(X), 20)
    med = set(res.medoids.cpu().numpy().tolist())
    agree = len(med & set(ref.medoids.tolist())) / 20
    td_true, _ = oracle.td(res.medoids.cpu().numpy(), D=D64)
    print("medoid agreement", agree, "TD", res.td, ref.td, td_true, flush=True)
    assert abs(res.td - td_true) <= 1e-5 * td_true
    assert abs(td_true - ref.td) <= 1e-4 * ref.td
    assert agree >= 0.9


# ------------------------------------------------------------------ edge cases
def test_k1_and_k_equals_n():
    _say("k1_kn")
    X, D = _int_case(50, 3, hi=20)
    for k in (1, 50, 49):
        ref = oracle.pam(k, D=D)
        res = px().fit(_t(X), k, trace=True)
        assert sorted(res.medoids.cpu().numpy().tolist()) == sorted(ref.medoids.tolist()), k
        assert res.td == ref.td
        assert res.stats["iterations"] == ref.iterations


@pytest.mark.parametrize("seed,n,k", [(31, 800, 600), (32, 1200, 1100)])
@pytest.mark.parametrize("variant", ["fastpam1", "fastpam2"])
def test_large_k_bitexact(seed, n, k, variant):
    # k well above the 256 threads of the segment kernels: each thread scans
    # a run of several slot totals into the segment offsets
    _say("large_k", seed, n, k, variant)
    X, D = _int_case(n, seed)
    if variant == "fastpam2":
        ref = oracle.pam(k, D=D, variant=oracle.FASTPAM2)
    else:
        ref = oracle.pam(k, D=D)
    res = px().fit(_t(X), k, variant=variant, trace=True)
    _check_same(res, ref, k)
    assert res.stats["iterations"] == ref.iterations


def test_tiny_n():
    _say("tiny_n")
    for n in (1, 2, 3):
        X, D = _int_case(n, 4, hi=5)
        for k in range(1, n + 1):
            ref = oracle.pam(k, D=D)
            res = px().fit(_t(X), k)
            assert res.td == ref.td
            assert list(res.medoids.cpu().numpy()) == list(ref.medoids)


def test_duplicate_points():
    _say("duplicates")
    X = np.repeat(datagen.int_points(40, 2, 0, 30, seed=8), 3, axis=0)
    D = oracle.dist_matrix(X, oracle.L1)
    for k in (3, 10):
        ref = oracle.pam(k, D=D)
        res = px().fit(_t(X), k, trace=True)
        _check_same(res, ref, k)


def test_invalid_medoids_and_maxiter():
    _say("invalid_medoids")
    X, D = _int_case(300, 9, hi=300)
    Dt = _t(D.astype(np.int32))
    with pytest.raises(px().PamxError) as e:
        px().swap(Dt, _t(np.array([1, 1, 2], np.int32)))
    assert e.value.code == -4
    with pytest.raises(px().PamxError):
        px().swap(Dt, _t(np.array([1, 300], np.int32)))
    start = np.arange(8, dtype=np.int32)
    ref = oracle.swap(start, D=D, max_iter=2)
    res = px().swap(Dt, _t(start), max_iter=2, trace=True)
    assert res.rc == 1 and ref.rc == 1
    assert list(res.medoids.cpu().numpy()) == list(ref.medoids)
    assert res.stats["iterations"] == 2 and res.stats["converged"] == 0


def test_deterministic_rerun():
    _say("determinism")
    X = datagen.gaussian_mixture(3000, 16, 30, seed=77)
    a = px().fit(_t(X), 30, variant="fastpam2")
    b = px().fit(_t(X), 30, variant="fastpam2")
    assert torch.equal(a.medoids, b.medoids) and torch.equal(a.labels, b.labels)
    assert a.td == b.td


# ------------------------------------------------------------------ int32 range
def test_int_points_range_limit():
    """Integer points whose coordinate ranges sum past INT32_MAX - 1 are
    refused by the distance call, the fit and the batched fit (an L1
    distance could leave int32); at exactly INT32_MAX - 1 the distances and
    the fit are exact (Eq. td with int64 sums)."""
    _say("int_range_limit")
    big = np.array([[-2 ** 30, 5], [2 ** 30 - 1, -7], [0, 2 ** 30 - 1], [3, -2 ** 30]], np.int32)
    Xb = _t(big)
    with pytest.raises(px().PamxError):
        px().dist(Xb)
    with pytest.raises(px().PamxError):
        px().fit(Xb, 2)
    off = np.array([0, 4], np.int64)
    with pytest.raises(px().PamxError):
        px().fit_batched(Xb, off, _t(np.arange(4, dtype=np.int32)), np.array([2], np.int32))
    # one coordinate spanning INT32_MAX - 1, the other constant
    lim = 2 ** 31 - 2
    X = np.array([[0, 9], [lim, 9], [1, 9], [lim - 1, 9], [lim // 2, 9], [5, 9]], np.int32)
    D = px().dist(_t(X)).cpu().numpy().astype(np.int64)
    Dref = oracle.dist_matrix(X, oracle.L1)
    assert np.array_equal(D.astype(np.float64), Dref)
    assert D.max() == lim
    ref = oracle.pam(2, D=Dref)
    res = px().fit(_t(X), 2)
    assert list(res.medoids.cpu().numpy()) == list(ref.medoids)
    assert res.td == ref.td
