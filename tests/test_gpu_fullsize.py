"""GPU parity at the full workload sizes, on outputs the FP64 oracle can
compute one at a time: the change of a BUILD step (Alg. 1) for sampled
candidates, the change of each recorded swap (Eq. change summed as in
Alg. 2), and a local-optimum certificate over sampled candidates.

* n = 20000, d = 16, k = 100, FP32 matrix (the benchmark workload), FastPAM1
  and eager FastPAM2.  The oracle computes the matrix in FP64 and it is
  rounded to FP32 once; the GPU and the oracle read the same FP32 values, so
  every decision agrees up to the order of FP64 sums (bounded below).
* The same workload from points, as the benchmark runs it: the GPU's own FP32
  matrix is within the rounding bound of its Gram form everywhere, fitting
  the points equals fitting that matrix bit for bit, and the TD is within the
  summed per-object distance error of the exact TD.
* n = 100000, d = 32, k = 500 (a 40 GB matrix), eager FastPAM2: on integer
  coordinates with Manhattan distance every check is exact; on the FP32
  Euclidean workload the TD is within the rounding bound.
* n = 50000, d = 64, k = 200, BF16 Gram recompute with FP64 re-scoring: the
  decisions are the FP64 oracle's.
* 256 CLARA instances from a 1e6-point pool: sampled instances against the
  oracle, bit-exact on an integer pool.

Summation-order tolerance: two FP64 sums of the same n terms in different
orders differ by at most about 2 n u S (u = 2^-53, S = sum of |terms|); every
Eq. change term is bounded by the object's second-nearest distance, so
S <= sum(dn + ds).  The tests allow 8 n u S.
"""
import numpy as np
import pytest

import oracle
from paper_2008_05171_amd import datagen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"
U53 = 2.0 ** -53
U24 = 2.0 ** -24


def px():
    import paper_2008_05171_amd as m
    return m


def _say(*a):
    print("[case]", *a, flush=True)


def _sum_tol(n, S):
    return 8.0 * n * U53 * float(S) + 1e-300


def _medoid_sets(start, trace):
    """Medoid slots before each recorded swap, and the final set."""
    meds = [np.asarray(start, np.int32).copy()]
    for slot, cand, _ in trace:
        m = meds[-1].copy()
        m[slot] = cand
        meds.append(m)
    return meds


def _non_medoid_sample(rng, n, med, size, must=()):
    is_med = np.zeros(n, bool)
    is_med[np.asarray(med)] = True
    pool = np.flatnonzero(~is_med)
    s = rng.choice(pool, size=min(size, len(pool)), replace=False)
    return np.unique(np.concatenate([s, np.asarray(must, np.int64)])).astype(np.int64)


def _swap_tol(med, n, **src):
    _, dn, ds = oracle.nearest(med, **src)
    return _sum_tol(n, dn.sum() + ds.sum())


def _check_build_step(bm, t, cand, exact=False, full=False, **src):
    """The GPU's medoid for step t has the smallest change among cand."""
    n = src["D"].shape[0] if "D" in src else src["X"].shape[0]
    cand = np.unique(np.concatenate([cand, [bm[t]]])).astype(np.int64)
    v = oracle.build_list(bm[:t], cand, **src)
    v = np.where(np.isnan(v), np.inf, v)
    g = v[np.searchsorted(cand, bm[t])]
    if exact:
        assert g == v.min(), (t, g, v.min())
        tied = cand[v == g]
        assert bm[t] == tied.min(), (t, "tie order")
        return
    if t == 0:                       # column sums: the terms are the distances
        S = max(abs(g), abs(v.min()))
    else:                            # terms min(d - dn, 0) lie in [-dn, 0]
        _, dn, _ = oracle.nearest(bm[:t], **src)
        S = dn.sum()
    tol = _sum_tol(n, S)
    assert g <= v.min() + tol, (t, g, v.min(), tol)
    if full:
        order = np.argsort(v, kind="stable")
        if v[order[1]] - v[order[0]] > 2 * tol:
            assert cand[order[0]] == bm[t], t


def _assert_best_swap(tab, cands, slot, cand, tol):
    """(slot, cand) is the first minimum of the oracle's table (rows: cands,
    columns: slots) in (change, slot, candidate) order, whenever the
    runner-up lies more than 2 tol above it (closer values may trade places
    under a different FP64 summation order)."""
    vals = np.where(np.isnan(tab), np.inf, tab)
    k = vals.shape[1]
    slots = np.broadcast_to(np.arange(k)[None, :], vals.shape).ravel()
    cidx = np.broadcast_to(np.asarray(cands)[:, None], vals.shape).ravel()
    flat = vals.ravel()
    order = np.lexsort((cidx, slots, flat))
    best, second = int(order[0]), int(order[1])
    if flat[second] - flat[best] > 2 * tol:
        assert (int(slots[best]), int(cidx[best])) == (slot, cand), (slots[best], cidx[best])


# ============================================================ n = 20000, FP32 matrix
@pytest.fixture(scope="module")
def gmm16():
    X = datagen.workload_gmm16()
    D64 = oracle.dist_matrix(X)
    D32 = D64.astype(np.float32)
    Dq = D32.astype(np.float64)         # the FP32 values both sides read
    return X, D64, D32, Dq


def test_gmm16_build_full(gmm16):
    X, _, D32, Dq = gmm16
    n, k = D32.shape[0], 100
    _say("gmm16 build", n, k)
    Dt = torch.from_numpy(D32).to(DEV)
    bm, tdb = px().build(Dt, k)
    bm = bm.cpu().numpy()
    assert len(set(bm.tolist())) == k
    assert tdb == pytest.approx(oracle.td(bm, D=Dq)[0], rel=1e-12)
    rng = np.random.default_rng(7)
    for t in (0, 1, 2, k - 1):                       # every candidate
        _check_build_step(bm, t, np.arange(n), full=True, D=Dq)
    for t in (10, 30, 50, 75):                       # 2048 sampled candidates
        _check_build_step(bm, t, _non_medoid_sample(rng, n, bm[:t], 2048), D=Dq)


@pytest.mark.parametrize("variant", ["fastpam1", "fastpam2"])
def test_gmm16_swap_full(gmm16, variant):
    X, _, D32, Dq = gmm16
    n, k = D32.shape[0], 100
    _say("gmm16 swap", variant, n, k)
    Dt = torch.from_numpy(D32).to(DEV)
    bm, tdb = px().build(Dt, k)
    bm = bm.cpu().numpy()
    r = px().fit(Dt, k, input_kind=px().PAMX_INPUT_D, variant=variant, trace=True)
    assert r.rc == 0 and r.stats["swaps"] == len(r.trace) >= 1
    assert r.stats["td_build"] == tdb
    if variant == "fastpam1":
        assert r.stats["iterations"] == r.stats["swaps"] + 1
    meds = _medoid_sets(bm, r.trace)
    rng = np.random.default_rng(11)
    m = len(r.trace)
    if variant == "fastpam1":
        check = sorted(set([0, 1, 2, m // 3, m // 2, 2 * m // 3, m - 2, m - 1]) & set(range(m)))
    else:
        check = range(m)                             # every eager swap is re-scored
    for j in check:
        slot, cand, dl = r.trace[j]
        tol = _swap_tol(meds[j], n, D=Dq)
        want = oracle.swap_list(meds[j], [cand], D=Dq)[0, slot]
        assert dl < 0 and abs(dl - want) <= tol, (j, dl, want, tol)
        if variant == "fastpam1" and j == 0:         # the first search over every candidate
            allc = np.arange(n)
            tab = oracle.swap_list(meds[0], allc, D=Dq)
            assert dl <= np.nanmin(tab) + tol, (dl, np.nanmin(tab))
            _assert_best_swap(tab, allc, slot, cand, tol)
        elif variant == "fastpam1":                  # the best swap of its iteration
            tab = oracle.swap_list(meds[j], _non_medoid_sample(rng, n, meds[j], 512), D=Dq)
            assert dl <= np.nanmin(tab) + tol, (j, dl, np.nanmin(tab))
    final = r.medoids.cpu().numpy()
    assert np.array_equal(final, meds[-1])
    td_ref, lab_ref = oracle.td(final, D=Dq)
    assert r.td == pytest.approx(td_ref, rel=1e-12)
    assert np.array_equal(r.labels.cpu().numpy(), lab_ref)
    assert abs(tdb + sum(d for _, _, d in r.trace) - r.td) <= 8 * _swap_tol(final, n, D=Dq)
    # local optimum: no sampled swap lowers TD beyond rounding
    tab = oracle.swap_list(final, _non_medoid_sample(rng, n, final, 2048), D=Dq)
    assert np.nanmin(tab) >= -_swap_tol(final, n, D=Dq)
    print("TD", variant, r.td, "swaps", m, "iterations", r.stats["iterations"], flush=True)


def test_gmm16_points_path(gmm16):
    """Fitting the points (distances computed on the GPU) as the benchmark does."""
    X, D64, _, _ = gmm16
    n, dim, k = X.shape[0], X.shape[1], 100
    _say("gmm16 points", n, dim, k)
    Xt = torch.from_numpy(X).to(DEV)
    Dg = px().dist(Xt)
    assert torch.equal(Dg, Dg.t()) and bool((torch.diagonal(Dg) == 0).all())
    # Gram-form rounding bound on every entry: |d~^2 - d^2| <= 2 (dim+4) u32 (|x|+|y|)^2
    # for centred coordinates
    Xc = X.astype(np.float64) - X.astype(np.float64).mean(axis=0)
    nrm = np.sqrt((Xc * Xc).sum(axis=1))
    eps = np.empty(n)
    for r0 in range(0, n, 2000):
        r1 = min(r0 + 2000, n)
        g = Dg[r0:r1].cpu().numpy().astype(np.float64)
        e = D64[r0:r1]
        bound = 2.0 * (dim + 4) * U24 * (nrm[r0:r1, None] + nrm[None, :]) ** 2
        assert (np.abs(g * g - e * e) <= bound).all(), r0
        eps[r0:r1] = np.abs(g - e).max(axis=1)
    rx = px().fit(Xt, k, trace=True)
    rd = px().fit(Dg.contiguous(), k, input_kind=px().PAMX_INPUT_D, trace=True)
    assert rx.rc == 0 and rd.rc == 0
    assert torch.equal(rx.medoids, rd.medoids) and torch.equal(rx.labels, rd.labels)
    assert rx.td == rd.td and rx.trace == rd.trace
    td_ref, _ = oracle.td(rx.medoids.cpu().numpy(), D=D64)
    assert abs(rx.td - td_ref) <= eps.sum(), (rx.td, td_ref, eps.sum())
    print("TD", rx.td, "exact", td_ref, "bound", eps.sum(), flush=True)


# ============================================================ n = 100000, 40 GB matrix
def test_zipf32_int_fastpam2_full():
    """Integer coordinates (the FP32 workload scaled by 4 and rounded),
    Manhattan distance, 40 GB int32 matrix, k = 500, eager FastPAM2."""
    Xi = np.rint(datagen.workload_gmm32_zipf() * 4.0).astype(np.int32)
    n, k = Xi.shape[0], 500
    _say("zipf32 int fastpam2", n, k)
    Xt = torch.from_numpy(Xi).to(DEV)
    rb = px().fit(Xt, k, max_iter=0)
    assert rb.stats["swaps"] == 0
    bm = rb.medoids.cpu().numpy()
    assert rb.td == oracle.td(bm, X=Xi, metric=oracle.L1)[0]
    rng = np.random.default_rng(13)
    for t in (0, 1, 250, k - 1):
        _check_build_step(bm, t, _non_medoid_sample(rng, n, bm[:t], 512), exact=True, X=Xi,
                          metric=oracle.L1)
    del rb
    r = px().fit(Xt, k, variant="fastpam2", trace=True)
    assert r.rc == 0 and r.stats["swaps"] == len(r.trace) >= 1
    meds = _medoid_sets(bm, r.trace)
    m = len(r.trace)
    check = sorted(set(range(4)) | set(range(m - 4, m)) |
                   set(rng.choice(m, size=min(6, m), replace=False).tolist()))
    for j in check:
        if j < 0 or j >= m:
            continue
        slot, cand, dl = r.trace[j]
        want = oracle.swap_list(meds[j], [cand], X=Xi, metric=oracle.L1)[0, slot]
        assert dl == want and dl < 0, (j, dl, want)
    final = r.medoids.cpu().numpy()
    assert np.array_equal(final, meds[-1])
    td_ref, lab_ref = oracle.td(final, X=Xi, metric=oracle.L1)
    assert r.td == td_ref == _build_td_plus_changes(r, bm, Xi)
    assert np.array_equal(r.labels.cpu().numpy(), lab_ref)
    tab = oracle.swap_list(final, _non_medoid_sample(rng, n, final, 48), X=Xi, metric=oracle.L1)
    assert np.nanmin(tab) >= 0
    print("TD", r.td, "swaps", m, "iterations", r.stats["iterations"], flush=True)


def test_max_size_int_fastpam2():
    """The largest matrix this GPU holds with room to spare: n = 200000
    integer points (d = 32, 500 Zipf(1.1)-weighted components scaled by 4
    and rounded), the 160 GB int32 Manhattan matrix built from the points
    inside the fit's workspace, k = 500, BUILD + eager FastPAM2.  Every
    64-bit offset path (rows of 800 KB, 4e10 entries) against the oracle
    computing from the points: BUILD's TD and sampled steps, sampled swaps'
    changes, the final TD and labels exactly, no sampled swap improving."""
    n, k = 200000, 500
    need = n * n * 4 + (8 << 30)
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < need:
        pytest.skip("needs %.0f GB of free device memory (%.0f GB free)" % (need / 1e9, free / 1e9))
    Xi = np.rint(datagen.gaussian_mixture(n, 32, 500, seed=1006, zipf_s=1.1) * 4.0).astype(np.int32)
    _say("max size int fastpam2", n, k)
    Xt = torch.from_numpy(Xi).to(DEV)
    r = px().fit(Xt, k, variant="fastpam2", trace=True)
    assert r.rc == 0 and r.stats["swaps"] == len(r.trace) >= 1
    torch.cuda.empty_cache()
    rb = px().fit(Xt, k, max_iter=0)
    bm = rb.medoids.cpu().numpy()
    del rb
    torch.cuda.empty_cache()
    assert r.stats["td_build"] == oracle.td(bm, X=Xi, metric=oracle.L1)[0]
    rng = np.random.default_rng(17)
    for t in (0, 1, 250, k - 1):
        _check_build_step(bm, t, _non_medoid_sample(rng, n, bm[:t], 256), exact=True, X=Xi,
                          metric=oracle.L1)
    meds = _medoid_sets(bm, r.trace)
    m = len(r.trace)
    check = sorted(set(range(3)) | set(range(m - 3, m)) |
                   set(rng.choice(m, size=min(4, m), replace=False).tolist()))
    for j in check:
        if j < 0 or j >= m:
            continue
        slot, cand, dl = r.trace[j]
        want = oracle.swap_list(meds[j], [cand], X=Xi, metric=oracle.L1)[0, slot]
        assert dl == want and dl < 0, (j, dl, want)
    final = r.medoids.cpu().numpy()
    assert np.array_equal(final, meds[-1])
    td_ref, lab_ref = oracle.td(final, X=Xi, metric=oracle.L1)
    assert r.td == td_ref == _build_td_plus_changes(r, bm, Xi)
    assert np.array_equal(r.labels.cpu().numpy(), lab_ref)
    tab = oracle.swap_list(final, _non_medoid_sample(rng, n, final, 32), X=Xi, metric=oracle.L1)
    assert np.nanmin(tab) >= 0
    print("TD", r.td, "swaps", m, "iterations", r.stats["iterations"], "ms dist/build/swap",
          r.stats["ms_dist"], r.stats["ms_build"], r.stats["ms_swap"], flush=True)


def _build_td_plus_changes(r, bm, Xi):
    """BUILD TD plus every recorded change (integer sums: exact)."""
    return oracle.td(bm, X=Xi, metric=oracle.L1)[0] + sum(d for _, _, d in r.trace)


def _oracle_f32_matrix(X, block=1000):
    """The n x n matrix of Euclidean distances rounded to FP32 (the oracle's
    metric L2F32), computed by the oracle a block of rows at a time and
    copied to the device (the host never holds it whole)."""
    n = X.shape[0]
    X64 = np.ascontiguousarray(X, dtype=np.float64)
    D = torch.empty((n, n), dtype=torch.float32, device=DEV)
    for r0 in range(0, n, block):
        rows = np.arange(r0, min(r0 + block, n))
        blk = oracle.dist_rows(X64, rows, oracle.L2F32).astype(np.float32)
        D[r0:r0 + len(rows)].copy_(torch.from_numpy(blk))
    return D


def test_zipf32_f32_matrix_fastpam2_full():
    """The 40 GB FP32 workload, eager FastPAM2, on a matrix the oracle
    computed (FP64 distances of the points rounded once to FP32): both sides
    read the same FP32 values, so BUILD steps, every sampled swap's change,
    the final TD and labels agree up to the order of FP64 sums, and no
    sampled swap improves at convergence."""
    X = datagen.workload_gmm32_zipf()
    n, k = X.shape[0], 500
    _say("zipf32 f32 matrix fastpam2", n, k)
    D = _oracle_f32_matrix(X)
    src = dict(X=X, metric=oracle.L2F32)
    _say("zipf32 f32 matrix: built")
    rb = px().fit(D, k, input_kind=px().PAMX_INPUT_D, max_iter=0)
    bm = rb.medoids.cpu().numpy()
    assert len(set(bm.tolist())) == k
    assert rb.td == pytest.approx(oracle.td(bm, **src)[0], rel=1e-12)
    rng = np.random.default_rng(23)
    for t in (0, 1, 250, k - 1):
        _check_build_step(bm, t, _non_medoid_sample(rng, n, bm[:t], 512), **src)
    r = px().fit(D, k, input_kind=px().PAMX_INPUT_D, variant="fastpam2", trace=True)
    assert r.rc == 0 and r.stats["swaps"] == len(r.trace) >= 1
    assert r.stats["td_build"] == rb.td
    meds = _medoid_sets(bm, r.trace)
    m = len(r.trace)
    check = sorted((set(range(4)) | set(range(m - 4, m)) |
                    set(rng.choice(m, size=min(6, m), replace=False).tolist())) & set(range(m)))
    for j in check:
        slot, cand, dl = r.trace[j]
        tol = _swap_tol(meds[j], n, **src)
        want = oracle.swap_list(meds[j], [cand], **src)[0, slot]
        assert dl < 0 and abs(dl - want) <= tol, (j, dl, want, tol)
    final = r.medoids.cpu().numpy()
    assert np.array_equal(final, meds[-1])
    td_ref, lab_ref = oracle.td(final, **src)
    assert r.td == pytest.approx(td_ref, rel=1e-12)
    assert np.array_equal(r.labels.cpu().numpy(), lab_ref)
    ftol = _swap_tol(final, n, **src)
    assert abs(rb.td + sum(d for _, _, d in r.trace) - r.td) <= (m + 2) * ftol
    # local optimum: no sampled swap lowers TD beyond the summation bound
    tab = oracle.swap_list(final, _non_medoid_sample(rng, n, final, 2048), **src)
    assert np.nanmin(tab) >= -ftol, (np.nanmin(tab), ftol)
    print("TD", r.td, "swaps", m, "searches", r.stats["iterations"], "min change", np.nanmin(tab),
          flush=True)


def test_zipf32_float_fastpam2_full():
    """The FP32 Euclidean workload with its 40 GB matrix: sampled rows within
    the Gram rounding bound; TD within the summed per-object bound."""
    X = datagen.workload_gmm32_zipf()
    n, dim, k = X.shape[0], X.shape[1], 500
    _say("zipf32 float fastpam2", n, dim, k)
    Xt = torch.from_numpy(X).to(DEV)
    Xc = X.astype(np.float64) - X.astype(np.float64).mean(axis=0)
    nrm = np.sqrt((Xc * Xc).sum(axis=1))
    rng = np.random.default_rng(17)
    rows = rng.choice(n, size=48, replace=False)
    Dg = px().dist(Xt)
    g = Dg[torch.from_numpy(rows).to(DEV)].cpu().numpy().astype(np.float64)
    e = oracle.dist_rows(X, rows)
    bound = 2.0 * (dim + 4) * U24 * (nrm[rows, None] + nrm[None, :]) ** 2
    assert (np.abs(g * g - e * e) <= bound).all()
    r = px().fit(Xt, k, variant="fastpam2", trace=True)
    assert r.rc == 0
    # fitting the points (as the benchmark does) = fitting the GPU's own matrix
    rd = px().fit(Dg, k, input_kind=px().PAMX_INPUT_D, variant="fastpam2", trace=True)
    assert torch.equal(r.medoids, rd.medoids) and torch.equal(r.labels, rd.labels)
    assert r.td == rd.td and r.trace == rd.trace
    del Dg, rd
    torch.cuda.empty_cache()
    final = r.medoids.cpu().numpy()
    _, dn, _ = oracle.nearest(final, X=X)
    # |min_i d~_i - min_i d_i| <= max_i |d~_i - d_i|, and every d_i >= dn
    b2 = 2.0 * (dim + 4) * U24 * (nrm + nrm[final].max()) ** 2
    per_obj = np.minimum(np.sqrt(b2), b2 / np.maximum(dn, 1e-300))
    td_ref = dn.sum()
    assert abs(r.td - td_ref) <= per_obj.sum(), (r.td, td_ref, per_obj.sum())
    print("TD", r.td, "exact", td_ref, "bound", per_obj.sum(), "swaps", r.stats["swaps"],
          flush=True)


# ============================================================ n = 50000, BF16 recompute
@pytest.mark.parametrize("accum", ["f64", "f32"])
def test_gmm64_bf16_full(accum):
    """BF16 Gram distances with FP64 sums, or FP32 sums (the mixed-precision
    form as configured: FP32 loss changes, FP64 re-scoring of every candidate
    whose rigorous FP32 error bound reaches the best)."""
    X = datagen.workload_gmm64()
    n, k = X.shape[0], 200
    _say("gmm64 bf16", accum, n, X.shape[1], k)
    acc = px().PAMX_ACC_F32 if accum == "f32" else px().PAMX_ACC_F64
    Xt = torch.from_numpy(X).to(DEV)
    rb = px().fit(Xt, k, dist_mode="bf16", accum=acc, max_iter=0)
    assert rb.stats["swaps"] == 0
    bm = rb.medoids.cpu().numpy()
    assert rb.td == pytest.approx(oracle.td(bm, X=X)[0], rel=1e-12)
    rng = np.random.default_rng(19)
    for t in (0, 1, 100, k - 1):
        _check_build_step(bm, t, _non_medoid_sample(rng, n, bm[:t], 1024), X=X)
    r = px().fit(Xt, k, dist_mode="bf16", accum=acc, trace=True)
    assert r.rc == 0 and r.stats["swaps"] == len(r.trace) >= 1
    assert r.stats["iterations"] == r.stats["swaps"] + 1
    meds = _medoid_sets(bm, r.trace)
    m = len(r.trace)
    for j in sorted(set([0, 1, m // 2, m - 2, m - 1]) & set(range(m))):
        slot, cand, dl = r.trace[j]
        tol = _swap_tol(meds[j], n, X=X)
        want = oracle.swap_list(meds[j], [cand], X=X)[0, slot]
        assert dl < 0 and abs(dl - want) <= tol, (j, dl, want, tol)
        tab = oracle.swap_list(meds[j], _non_medoid_sample(rng, n, meds[j], 96), X=X)
        assert dl <= np.nanmin(tab) + tol, (j, dl, np.nanmin(tab))
    final = r.medoids.cpu().numpy()
    td_ref, lab_ref = oracle.td(final, X=X)
    assert r.td == pytest.approx(td_ref, rel=1e-12)
    assert np.array_equal(r.labels.cpu().numpy(), lab_ref)
    tab = oracle.swap_list(final, _non_medoid_sample(rng, n, final, 128), X=X)
    assert np.nanmin(tab) >= -_swap_tol(final, n, X=X)
    print("TD", r.td, "swaps", m, "rescored", r.stats.get("rescored"), flush=True)


# ============================================================ 256 CLARA instances
def _clara(X, seed=1004):
    off, idx, ks = datagen.clara_samples(X.shape[0], 256, 10, 50, 2000, seed=seed)
    res = px().fit_batched(torch.from_numpy(X).to(DEV), off, torch.from_numpy(idx).to(DEV), ks)
    assert res.rc == 0
    sizes = np.diff(off)
    rng = np.random.default_rng(seed)
    pick = sorted(set([int(np.argmax(sizes)), int(np.argmax(ks)), int(np.argmin(sizes))] +
                      rng.choice(256, size=3, replace=False).tolist()))
    return off, idx, ks, res, pick


def test_clara256_int_bitexact():
    Xi = np.rint(datagen.workload_gmm8_pool() * 16.0).astype(np.int32)
    _say("clara256 int", Xi.shape)
    off, idx, ks, res, pick = _clara(Xi)
    for j in pick:
        sample = idx[off[j]:off[j + 1]]
        D = oracle.dist_matrix(Xi[sample], oracle.L1)
        ref = oracle.pam(int(ks[j]), D=D)
        assert list(res.medoids[j].cpu().numpy()) == list(sample[ref.medoids]), j
        assert res.td_sample[j] == ref.td, j
        tdf, _ = oracle.td(sample[ref.medoids], X=Xi, metric=oracle.L1)
        assert res.td_full[j] == tdf, j
    assert res.best == int(np.argmin(res.td_full))


def test_clara256_int_all_instances():
    """Every one of the 256 instances on the integer pool against the
    oracle's record (tests/golden/clara256_int_reference.json, written by
    make_clara256_reference.py from the oracle alone): the same medoids in
    the same slots, the same sample TD and the same TD over all 1e6 points,
    and the smallest full TD picked."""
    import json
    import os
    rec = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                      "clara256_int_reference.json")))["instances"]
    assert [r["j"] for r in rec] == list(range(256))
    Xi = np.rint(datagen.workload_gmm8_pool() * 16.0).astype(np.int32)
    _say("clara256 int, all instances", Xi.shape)
    off, idx, ks, res, _ = _clara(Xi)
    med = [m.cpu().numpy().tolist() for m in res.medoids]
    bad = [r["j"] for r in rec
           if med[r["j"]] != r["medoids"]
           or res.td_sample[r["j"]] != r["td_sample"] or res.td_full[r["j"]] != r["td_full"]]
    assert not bad, bad[:10]
    tdf = np.array([r["td_full"] for r in rec])
    assert res.best == int(np.argmin(tdf))


def test_clara256_float():
    X = datagen.workload_gmm8_pool()
    _say("clara256 float", X.shape)
    off, idx, ks, res, pick = _clara(X)
    agree = 0
    for j in pick:
        sample = idx[off[j]:off[j + 1]]
        Xs = X[sample].astype(np.float64)
        D = oracle.dist_matrix(Xs)
        got = res.medoids[j].cpu().numpy()
        local = np.searchsorted(sample, got)
        td_g, _ = oracle.td(local, D=D)
        assert abs(res.td_sample[j] - td_g) <= 1e-6 * td_g, j
        ref = oracle.pam(int(ks[j]), D=D)
        assert abs(td_g - ref.td) <= 1e-3 * ref.td, (j, td_g, ref.td)
        # local optimum in FP64 up to the FP32 distance rounding
        tab = oracle.swap_list(local, np.arange(len(sample)), D=D)
        assert np.nanmin(tab) >= -1e-5 * td_g, j
        agree += set(got.tolist()) == set(sample[ref.medoids].tolist())
        tdf, _ = oracle.td(got, X=X)
        assert abs(res.td_full[j] - tdf) <= 1e-6 * tdf, j
    print("medoid-set agreement", agree, "/", len(pick), flush=True)
    assert agree >= len(pick) - 2
    assert res.best == int(np.argmin(res.td_full))
