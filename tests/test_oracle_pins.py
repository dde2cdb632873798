"""Pins of the CPU oracle against what the paper and the mathematics fix.

The oracle (plain C, FP64) is the reference the GPU path is compared with, so
it is itself checked here against things other than its own code:

* Eq. change against the definition of the change (new nearest minus old
  nearest distance), exhaustively over small integer distances with ties.
* The restructured form (Eq. better-change3 and the decomposition proved in
  the paper's appendix) against Eq. change.
* The worked example of Fig. 1 (printed losses 10 -> 7 -> 6, golden file).
* BUILD against greedy minimisation by full TD recomputation (Alg. 1).
* SWAP against best-swap steepest descent by full TD recomputation (Alg. 2):
  the whole trajectory, the local-optimum property at convergence, and the
  global optimum over all k-subsets as a lower bound.
* The FastPAM2 reading against a brute-force version of the same reading.
* Distance matrices against scipy's cdist; k = 1, k = n, duplicates.
"""
import itertools
import os

import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle
from paper_2008_05171_amd import datagen
from tests import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _tiny_int_D(rng, n, dim=2, hi=10):
    X = rng.integers(0, hi, size=(n, dim))
    return oracle.dist_matrix(X, oracle.L1), X


# ---------------------------------------------------------------- Eq. change
def test_change_matches_definition_exhaustive():
    """For k medoid distances and a candidate distance, the change of object o
    when slot i is replaced by x_c is min(d_c, min_{j!=i} d_j) - min_j d_j."""
    vals = range(0, 5)
    for k in (2, 3):
        for dm in itertools.product(vals, repeat=k):
            near = min(range(k), key=lambda j: (dm[j], j))
            dn = dm[near]
            ds = min(dm[j] for j in range(k) if j != near)
            for d in vals:
                for i in range(k):
                    want = min([d] + [dm[j] for j in range(k) if j != i]) - dn
                    got = oracle.change(d, near == i, dn, ds)
                    assert got == want, (dm, d, i)


def test_better_change3_decomposition_equals_change():
    """Appendix proof: removal loss + shared term + per-medoid term equals Eq.
    change for every object; and the per-medoid term equals med3(d,dn,ds)-ds."""
    rng = np.random.default_rng(7)
    cases = list(itertools.product(range(6), range(6), range(6), (0, 1)))
    cases += [tuple(rng.uniform(0, 5, 3)) + (int(rng.integers(0, 2)),) for _ in range(2000)]
    for d, a, b, is_i in cases:
        dn, ds = min(a, b), max(a, b)
        rem = (ds - dn) if is_i else 0.0
        shared = (d - dn) if d < dn else 0.0
        if is_i and d < dn:
            per = dn - ds
        elif is_i and d < ds:
            per = d - ds
        else:
            per = 0.0
        med3 = sorted((d, dn, ds))[1]
        assert per == ((med3 - ds) if is_i else 0.0)
        assert rem + shared + per == pytest.approx(oracle.change(d, is_i, dn, ds), abs=1e-12)


# ---------------------------------------------------------------- Fig. 1
def _read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            out[key] = vals
    return out


@pytest.mark.parametrize("variant", ["printed", "drawn"])
def test_fig1_worked_example(variant):
    g = _read_golden("fig1_swap.txt")
    pts = g["points"] if variant == "printed" else g["points_drawn"]
    losses = g["losses"] if variant == "printed" else g["losses_drawn"]
    names = [p.split("=")[0] for p in pts]
    X = np.array([[float(p.split("=")[1])] for p in pts])
    D = oracle.dist_matrix(X, oracle.L1)
    start = [names.index(s) for s in g["start"]]
    assert oracle.td(start, D=D)[0] == float(losses[0])
    r = oracle.swap(start, D=D)
    want_swaps = [(int(s.split(":")[0]), names.index(s.split(":")[1])) for s in g["swaps"]]
    assert [(s, c) for s, c, _ in r.trace] == want_swaps
    tds = [float(losses[0])]
    for _, _, dl in r.trace:
        tds.append(tds[-1] + dl)
    assert tds == [float(v) for v in losses]
    assert [names[m] for m in r.medoids] == g["final"]
    assert r.iterations == r.swaps + 1 and r.rc == 0
    # the final loss is the global optimum for k = 2 here
    assert brute.global_optimum(D.tolist(), 2) == float(losses[-1])


def test_fig1_build_readings():
    """BUILD on Fig. 1's points: with the self-term (default reading) it picks
    C then A (TD 7); with the literal loop bounds it picks C then D (TD 12).
    Both then converge to TD 6."""
    X = np.array([[-7.0], [0], [1], [2], [3], [4]])
    D = oracle.dist_matrix(X, oracle.L1)
    m, tdb, _ = oracle.build(2, D=D)
    assert list(m) == [2, 0] and tdb == 7.0
    m2, tdb2, _ = oracle.build(2, D=D, exclude_self=True)
    assert list(m2) == [2, 3] and tdb2 == 12.0
    assert oracle.pam(2, D=D).td == 6.0
    assert oracle.pam(2, D=D, exclude_self=True).td == 6.0


# ---------------------------------------------------------------- distances
def test_dist_matrix_vs_scipy():
    rng = np.random.default_rng(3)
    X = rng.normal(size=(37, 5))
    np.testing.assert_allclose(oracle.dist_matrix(X, oracle.L2), cdist(X, X), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(oracle.dist_matrix(X, oracle.L1), cdist(X, X, "cityblock"),
                               rtol=1e-13, atol=1e-13)
    Xi = datagen.int_points(50, 2, 0, 1000, seed=1)
    assert np.array_equal(oracle.dist_matrix(Xi, oracle.L1), cdist(Xi, Xi, "cityblock"))
    rows = np.array([36, 0, 7, 7])
    np.testing.assert_allclose(oracle.dist_rows(X, rows), cdist(X[rows], X), rtol=1e-13,
                               atol=1e-13)
    rows = np.array([49, 0, 7, 7])
    assert np.array_equal(oracle.dist_rows(Xi, rows, oracle.L1), cdist(Xi[rows], Xi, "cityblock"))


def test_l2f32_is_the_fp32_rounding_of_the_distance():
    """Metric L2F32: every Euclidean distance rounded to the nearest FP32
    value (what an FP32 matrix holds).  scipy's FP64 distances rounded by
    numpy agree except where the two FP64 values straddle a rounding
    boundary (then within one FP32 ulp); the swap changes in this metric
    equal those computed from that FP32 matrix, and are the TD differences
    of the swaps (brute force)."""
    rng = np.random.default_rng(31)
    X = rng.normal(size=(60, 7)) * 3.0
    ref = cdist(X, X).astype(np.float32)
    got = oracle.dist_matrix(X, oracle.L2F32)
    assert np.all(got == got.astype(np.float32))             # FP32 values
    ulp = np.spacing(ref)
    assert np.all(np.abs(got - ref.astype(np.float64)) <= ulp)
    assert np.mean(got == ref) > 0.99
    rows = np.array([59, 3, 3])
    assert np.array_equal(oracle.dist_rows(X, rows, oracle.L2F32), got[rows])
    med = [4, 17, 33, 50]
    cand = np.arange(60)
    tabx = oracle.swap_list(med, cand, X=X, metric=oracle.L2F32)
    tabd = oracle.swap_list(med, cand, D=got)
    assert np.array_equal(np.isnan(tabx), np.isnan(tabd))
    assert np.array_equal(tabx[~np.isnan(tabx)], tabd[~np.isnan(tabd)])
    Dl = got.tolist()
    td0 = brute.td_of(Dl, med)
    for c in (0, 9, 59):
        for i in range(4):
            m2 = list(med)
            m2[i] = c
            assert tabx[c, i] == pytest.approx(brute.td_of(Dl, m2) - td0, abs=1e-12)
    assert oracle.td(med, X=X, metric=oracle.L2F32)[0] == pytest.approx(td0, abs=1e-12)


# ---------------------------------------------------------------- BUILD
@pytest.mark.parametrize("exclude_self", [False, True])
def test_build_is_greedy_td(exclude_self):
    rng = np.random.default_rng(11)
    for trial in range(40):
        n = int(rng.integers(3, 13))
        k = int(rng.integers(1, n + 1))
        D, _ = _tiny_int_D(rng, n, hi=6)      # many ties
        m, tdb, _ = oracle.build(k, D=D, exclude_self=exclude_self)
        want = brute.build_greedy(D.tolist(), k, exclude_self=exclude_self)
        assert list(m) == want, (trial, n, k)
        assert tdb == brute.td_of(D.tolist(), want)


def test_k1_is_the_medoid():
    """k = 1: BUILD's first pick is the medoid of the set (Eq. def-medoid)."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        n = int(rng.integers(1, 30))
        X = rng.normal(size=(n, 3))
        D = oracle.dist_matrix(X)
        r = oracle.pam(1, D=D)
        sums = [sum(D[o][c] for o in range(n)) for c in range(n)]
        assert r.medoids[0] == int(np.argmin(sums))
        assert r.swaps == 0 and r.iterations == 0
        assert r.td == pytest.approx(min(sums), rel=1e-12)


# ---------------------------------------------------------------- SWAP
def test_swap_trajectory_is_steepest_descent():
    """Every applied swap is the best (delta, slot, cand) over all swaps by
    full TD recomputation; the result is a local optimum and no better than
    the global optimum (Alg. 2)."""
    rng = np.random.default_rng(12)
    for trial in range(30):
        n = int(rng.integers(4, 12))
        k = int(rng.integers(2, min(5, n - 1) + 1))
        D, _ = _tiny_int_D(rng, n, hi=8)
        start = [int(v) for v in rng.choice(n, size=k, replace=False)]
        r = oracle.swap(start, D=D)
        Dl = D.tolist()
        med_b, trace_b = brute.pam_swap(Dl, start)
        assert [(s, c) for s, c, _ in r.trace] == [(i, c) for i, c, _ in trace_b], trial
        assert [d for _, _, d in r.trace] == [v for _, _, v in trace_b]
        assert list(r.medoids) == med_b
        assert brute.is_local_optimum(Dl, med_b)
        assert r.td == brute.td_of(Dl, med_b) >= brute.global_optimum(Dl, k)
        assert r.iterations == r.swaps + 1


def test_swap_cross_tie_takes_pam_order():
    """Equal best changes at different (slot, cand): the swap taken is the
    first in slot-then-candidate order, as Alg. 2's loops give."""
    X = np.array([[3], [2], [4], [4], [5], [5], [2], [5]], float)
    D = oracle.dist_matrix(X, oracle.L1)
    found, dl, slot, c = oracle.swap_search([3, 0], D=D)
    b = brute.best_swap(D.tolist(), [3, 0])
    assert found and (dl, slot, c) == b
    # the brute force shows a second swap with the same change in a later slot
    sw = brute.all_swaps(D.tolist(), [3, 0])
    assert any(v == dl and i > slot for (i, _), v in sw.items())


def test_delta_matches_td_difference():
    rng = np.random.default_rng(21)
    for _ in range(30):
        n = int(rng.integers(4, 20))
        k = int(rng.integers(2, n))
        X = rng.normal(size=(n, 2))
        D = oracle.dist_matrix(X)
        med = [int(v) for v in rng.choice(n, size=k, replace=False)]
        non = [c for c in range(n) if c not in med]
        i = int(rng.integers(0, k))
        c = int(rng.choice(non))
        m2 = list(med)
        m2[i] = c
        want = brute.td_of(D.tolist(), m2) - brute.td_of(D.tolist(), med)
        assert oracle.delta(med, i, c, D=D) == pytest.approx(want, abs=1e-12)
        # points mode computes the same distances on the fly
        assert oracle.delta(med, i, c, X=X) == pytest.approx(want, abs=1e-12)


def test_swap_list_matches_td_difference():
    """The listed-candidate table equals the TD difference of every swap, on
    integer distances exactly, NaN for candidates that are medoids."""
    rng = np.random.default_rng(23)
    for trial in range(25):
        n = int(rng.integers(4, 16))
        k = int(rng.integers(2, n))
        if trial % 2:
            X = rng.integers(0, 7, size=(n, 2)).astype(float)
            D = oracle.dist_matrix(X, oracle.L1)
            metric, exact = oracle.L1, True
        else:
            X = rng.normal(size=(n, 3))
            D = oracle.dist_matrix(X)
            metric, exact = oracle.L2, False
        med = [int(v) for v in rng.choice(n, size=k, replace=False)]
        cand = rng.permutation(n)
        tab = oracle.swap_list(med, cand, D=D)
        tabx = oracle.swap_list(med, cand, X=X, metric=metric)
        Dl = D.tolist()
        td0 = brute.td_of(Dl, med)
        for j, c in enumerate(cand):
            if c in med:
                assert np.isnan(tab[j]).all() and np.isnan(tabx[j]).all()
                continue
            for i in range(k):
                m2 = list(med)
                m2[i] = int(c)
                want = brute.td_of(Dl, m2) - td0
                if exact:
                    assert tab[j, i] == want and tabx[j, i] == want, (trial, i, c)
                else:
                    assert tab[j, i] == pytest.approx(want, abs=1e-12)
                    assert tabx[j, i] == pytest.approx(want, abs=1e-12)


@pytest.mark.parametrize("exclude_self", [False, True])
def test_build_list_matches_td_difference(exclude_self):
    """BUILD change of each candidate after a prefix: the TD difference of
    adding it (self-term reading), or that plus its own nearest distance
    (literal loop bounds); the first step is the sum of distances to all
    other objects.  Along a BUILD run the chosen medoid is the first minimum."""
    rng = np.random.default_rng(29)
    for trial in range(20):
        n = int(rng.integers(3, 15))
        X = rng.integers(0, 9, size=(n, 2)).astype(float)
        D = oracle.dist_matrix(X, oracle.L1)
        Dl = D.tolist()
        t = int(rng.integers(0, n))
        prefix = [int(v) for v in rng.choice(n, size=t, replace=False)]
        cand = np.arange(n)
        got = oracle.build_list(prefix, cand, D=D, exclude_self=exclude_self)
        for c in range(n):
            if c in prefix:
                assert np.isnan(got[c])
                continue
            if t == 0:
                want = sum(Dl[o][c] for o in range(n) if o != c)
            else:
                want = brute.td_of(Dl, prefix + [c]) - brute.td_of(Dl, prefix)
                if exclude_self:
                    want += min(Dl[c][m] for m in prefix)
            assert got[c] == want, (trial, t, c)
        k = int(rng.integers(1, n + 1))
        med, _, steps = oracle.build(k, D=D, exclude_self=exclude_self)
        for s in range(k):
            v = oracle.build_list(med[:s], cand, D=D, exclude_self=exclude_self)
            v = np.where(np.isnan(v), np.inf, v)
            assert int(np.argmin(v)) == med[s] and v[med[s]] == steps[s]


def test_pam_from_build_matches_bruteforce():
    rng = np.random.default_rng(31)
    for _ in range(15):
        n = int(rng.integers(5, 13))
        k = int(rng.integers(2, 5))
        D, _ = _tiny_int_D(rng, n, hi=7)
        r = oracle.pam(k, D=D)
        Dl = D.tolist()
        bm = brute.build_greedy(Dl, k)
        med_b, _ = brute.pam_swap(Dl, bm)
        assert list(r.medoids) == med_b
        assert r.td == brute.td_of(Dl, med_b)
        assert r.td_build == brute.td_of(Dl, bm)
        near = [min(range(k), key=lambda j: (Dl[o][med_b[j]], j)) for o in range(n)]
        assert list(r.labels) == near


# ---------------------------------------------------------------- FastPAM2 reading
def test_fastpam2_reading_matches_bruteforce():
    rng = np.random.default_rng(41)
    for trial in range(30):
        n = int(rng.integers(5, 12))
        k = int(rng.integers(2, min(5, n - 1) + 1))
        D, _ = _tiny_int_D(rng, n, hi=9)
        start = [int(v) for v in rng.choice(n, size=k, replace=False)]
        r = oracle.swap(start, D=D, variant=oracle.FASTPAM2)
        med_b, trace_b = brute.fastpam2_swap(D.tolist(), start)
        assert list(r.medoids) == med_b, trial
        assert [(s, c, d) for s, c, d in r.trace] == [(i, c, v) for i, c, v in trace_b]
        assert brute.is_local_optimum(D.tolist(), med_b)


def test_fastpam2_first_swap_equals_pam_first_swap():
    rng = np.random.default_rng(43)
    for _ in range(20):
        n = int(rng.integers(6, 14))
        k = int(rng.integers(2, 5))
        D, _ = _tiny_int_D(rng, n, hi=20)
        start = [int(v) for v in rng.choice(n, size=k, replace=False)]
        a = oracle.swap(start, D=D, variant=oracle.PAM, max_iter=1)
        b = oracle.swap(start, D=D, variant=oracle.FASTPAM2, max_iter=1)
        if a.trace:
            assert b.trace[0] == a.trace[0]


# ---------------------------------------------------------------- FasterPAM (Alg. 4)
@pytest.mark.parametrize("variant", ["printed", "drawn"])
def test_fig1_fasterpam(variant):
    """The hand-worked FasterPAM run on Fig. 1's points (fixture derived from
    Alg. 4, not printed by the paper) and the losses the figure prints."""
    g = _read_golden("fig1_fasterpam.txt")
    pts = g["points"] if variant == "printed" else g["points_drawn"]
    swaps = g["swaps"] if variant == "printed" else g["swaps_drawn"]
    losses = g["losses"] if variant == "printed" else g["losses_drawn"]
    names = [p.split("=")[0] for p in pts]
    X = np.array([[float(p.split("=")[1])] for p in pts])
    D = oracle.dist_matrix(X, oracle.L1)
    start = [names.index(s) for s in g["start"]]
    r = oracle.swap(start, D=D, variant=oracle.FASTERPAM)
    want = [(int(s.split(":")[0]), names.index(s.split(":")[1]), float(s.split(":")[2]))
            for s in swaps]
    assert r.trace == want
    tds = [oracle.td(start, D=D)[0]]
    for _, _, dl in r.trace:
        tds.append(tds[-1] + dl)
    assert tds == [float(v) for v in losses]
    assert [names[m] for m in r.medoids] == g["final"]
    assert r.iterations == int(g["passes"][0]) and r.rc == 0


def test_fasterpam_matches_bruteforce():
    """Trajectory, passes and result equal the scan with full TD recomputation
    for every change, on tie-heavy integer matrices; the result is a local
    optimum (no single swap lowers TD)."""
    rng = np.random.default_rng(47)
    for trial in range(40):
        n = int(rng.integers(5, 13))
        k = int(rng.integers(2, min(5, n - 1) + 1))
        D, _ = _tiny_int_D(rng, n, hi=6 if trial % 2 else 20)
        start = [int(v) for v in rng.choice(n, size=k, replace=False)]
        r = oracle.swap(start, D=D, variant=oracle.FASTERPAM)
        med_b, trace_b, passes_b = brute.fasterpam_swap(D.tolist(), start)
        assert list(r.medoids) == med_b, trial
        assert r.trace == [(i, c, float(v)) for i, c, v in trace_b], trial
        assert r.iterations == passes_b and r.swaps == len(trace_b) and r.rc == 0
        assert brute.is_local_optimum(D.tolist(), med_b)
        assert r.td == brute.td_of(D.tolist(), med_b)


def test_fasterpam_max_iter_and_no_swap():
    """A start that is already a local optimum ends after one pass with no
    swap; a pass cap ends an unconverged run with the warning code."""
    rng = np.random.default_rng(53)
    D, _ = _tiny_int_D(rng, 40, hi=50)
    r = oracle.pam(4, D=D)
    again = oracle.swap(r.medoids, D=D, variant=oracle.FASTERPAM)
    assert again.swaps == 0 and again.iterations == 1 and again.rc == 0
    start = [0, 1, 2, 3]
    full = oracle.swap(start, D=D, variant=oracle.FASTERPAM)
    assert full.iterations >= 2 and full.rc == 0
    capped = oracle.swap(start, D=D, variant=oracle.FASTERPAM, max_iter=1)
    assert capped.rc == 1 and capped.iterations == 1
    assert capped.trace == full.trace[:capped.swaps]


def test_fasterpam_bookkeeping_on_int_workload():
    """n = 300 integer workload: TD strictly decreasing, TD_start + sum of the
    changes equals the final TD exactly, every change equals the swap's
    Eq. td difference, and the search finds no improving swap at the end."""
    rng = np.random.default_rng(59)
    X = rng.integers(0, 100, size=(300, 2)).astype(np.float64)
    D = oracle.dist_matrix(X, oracle.L1)
    start = [int(v) for v in rng.choice(300, 7, replace=False)]
    r = oracle.swap(start, D=D, variant=oracle.FASTERPAM)
    med = list(start)
    td0 = oracle.td(med, D=D)[0]
    run = td0
    for i, c, dl in r.trace:
        assert dl < 0
        before = oracle.td(med, D=D)[0]
        med[i] = c
        assert oracle.td(med, D=D)[0] - before == dl
        run += dl
    assert med == list(r.medoids) and run == r.td
    found, _, _, _ = oracle.swap_search(r.medoids, D=D)
    assert not found


# ---------------------------------------------------------------- faster initialisations
def test_init_dw_pick_frequencies_follow_distances():
    """With one seed placed, the second seed is drawn with probability
    proportional to the distance to that seed: empirical frequencies over
    many uniforms match the column of D (chi-square far below the 0.1% point),
    the seed itself (weight 0) is never drawn, and the pick is monotone in u."""
    rng = np.random.default_rng(61)
    D, _ = _tiny_int_D(rng, 12, hi=30)
    u0 = 5.5 / 12                       # first seed: floor(u0 n) = 5
    draws = 20000
    us = np.sort(rng.random(draws))
    picks = np.array([oracle.init_dw(2, [u0, u], D=D)[1] for u in us])
    assert np.all(np.diff(picks) >= 0)
    assert np.all(picks != 5)
    w = D[:, 5]
    p = w / w.sum()
    cnt = np.bincount(picks, minlength=12)
    keep = p > 0
    chi2 = float((((cnt - draws * p) ** 2)[keep] / (draws * p[keep])).sum())
    assert chi2 < 31.3                  # chi-square, 10 degrees of freedom, 0.1%
    assert oracle.init_dw(2, [u0, 0.0], D=D)[1] == int(np.flatnonzero(w > 0)[0])
    assert oracle.init_dw(2, [u0, 1 - 1e-12], D=D)[1] == int(np.flatnonzero(w > 0)[-1])


def test_init_dw_distinct_and_duplicates_never_drawn():
    """Points that coincide with a seed have weight 0: the seeds are distinct
    points; when every point coincides with a seed the smallest free index is
    taken."""
    rng = np.random.default_rng(67)
    X = np.repeat(rng.integers(0, 100, size=(8, 2)), 5, axis=0).astype(np.float64)
    D = oracle.dist_matrix(X, oracle.L1)
    for trial in range(30):
        med = oracle.init_dw(8, rng.random(8), D=D)
        assert len(set(med)) == 8
        assert len({tuple(X[m]) for m in med}) == 8
    med = oracle.init_dw(10, rng.random(10), D=D)
    assert len(set(med)) == 10
    rest = [m for m in med[8:]]
    free = [o for o in range(40) if o not in med[:8]]
    assert rest[0] == free[0] and rest[1] == [o for o in free if o != rest[0]][0]


@pytest.mark.parametrize("exclude_self", [False, True])
def test_init_lab_full_sample_is_build(exclude_self):
    """LAB with the whole data set (index order) as every step's sample is
    BUILD, and both equal the brute-force greedy TD recomputation."""
    rng = np.random.default_rng(71)
    for _ in range(10):
        n = int(rng.integers(6, 25))
        k = int(rng.integers(1, 5))
        D, _ = _tiny_int_D(rng, n, hi=15)
        S = np.tile(np.arange(n), (k, 1))
        lab = oracle.init_lab(k, S, D=D, exclude_self=exclude_self)
        assert list(lab) == list(oracle.build(k, D=D, exclude_self=exclude_self)[0])
        assert list(lab) == brute.build_greedy(D.tolist(), k, exclude_self=exclude_self)


@pytest.mark.parametrize("exclude_self", [False, True])
def test_init_lab_matches_subsample_bruteforce(exclude_self):
    """Random subsamples of 10 + ceil(sqrt n) points per step: each step picks
    the candidate with the smallest recomputed TD of its subsample."""
    rng = np.random.default_rng(73)
    for _ in range(15):
        n = int(rng.integers(20, 60))
        k = int(rng.integers(2, 7))
        m = 10 + int(np.ceil(np.sqrt(n)))
        D, _ = _tiny_int_D(rng, n, hi=25)
        S = np.array([np.sort(rng.choice(n, size=m, replace=False)) for _ in range(k)])
        lab = oracle.init_lab(k, S, D=D, exclude_self=exclude_self)
        assert list(lab) == brute.lab_greedy(D.tolist(), k, S.tolist(), exclude_self)
        assert len(set(lab)) == k


# ---------------------------------------------------------------- FastCLARANS (Sec. 3.4)
def test_clarans_matches_bruteforce():
    """Random draws (medoids among them), tie-heavy integer matrices: the
    trajectory, evaluation count and result equal the search by full TD
    recomputation."""
    rng = np.random.default_rng(83)
    for trial in range(40):
        n = int(rng.integers(5, 14))
        k = int(rng.integers(2, min(5, n - 1) + 1))
        D, _ = _tiny_int_D(rng, n, hi=6 if trial % 2 else 25)
        start = [int(v) for v in rng.choice(n, size=k, replace=False)]
        draws = rng.integers(0, n, size=400)
        mx = int(rng.integers(1, 8))
        r = oracle.clarans(start, draws, mx, D=D)
        med_b, trace_b, ev_b, exhausted = brute.clarans_search(D.tolist(), start, draws.tolist(), mx)
        assert list(r.medoids) == med_b, trial
        assert r.trace == [(i, c, float(v)) for i, c, v in trace_b], trial
        assert r.evaluations == ev_b and r.rc == (1 if exhausted else 0)
        assert r.td == brute.td_of(D.tolist(), med_b)


def test_clarans_cyclic_draws_are_fasterpam():
    """Draws in index order, repeated, with maxneighbor = n - k: the search
    stops where Alg. 4's scan completes a cycle without a swap, so it makes
    FasterPAM's swaps."""
    rng = np.random.default_rng(89)
    for _ in range(10):
        n = int(rng.integers(20, 80))
        k = int(rng.integers(2, 8))
        D, _ = _tiny_int_D(rng, n, hi=40)
        start = [int(v) for v in rng.choice(n, size=k, replace=False)]
        r = oracle.clarans(start, np.tile(np.arange(n), 50), n - k, D=D)
        f = oracle.swap(start, D=D, variant=oracle.FASTERPAM)
        assert r.rc == 0 and r.trace == f.trace and list(r.medoids) == list(f.medoids)


def test_clarans_exhausted_list_is_a_prefix():
    rng = np.random.default_rng(97)
    D, _ = _tiny_int_D(rng, 60, hi=100)
    start = [0, 1, 2, 3, 4]
    draws = rng.integers(0, 60, size=3000)
    full = oracle.clarans(start, draws, 40, D=D)
    assert full.rc == 0 and full.swaps > 2
    short = oracle.clarans(start, draws[:30], 40, D=D)
    assert short.rc == 1
    assert short.trace == full.trace[:short.swaps]


# ---------------------------------------------------------------- bichromatic medoids (Sec. 5)
def test_rect_square_symmetric_is_the_one_set_method():
    """Consumers = locations with a symmetric zero-diagonal matrix: the same
    BUILD, swap trajectory, medoids and TD as the one-set method (R1)."""
    rng = np.random.default_rng(101)
    for _ in range(10):
        n = int(rng.integers(8, 60))
        k = int(rng.integers(1, 6))
        D, _ = _tiny_int_D(rng, n, hi=25)
        a = oracle.rect_pam(k, D)
        b = oracle.pam(k, D=D)
        assert list(a.medoids) == list(b.medoids) and a.td == b.td
        assert list(a.build_medoids) == list(b.build_medoids) and a.td_build == b.td_build
        assert a.trace == b.trace and np.array_equal(a.labels, b.labels)


def test_rect_matches_bruteforce():
    """Rectangular consumer x location matrices (more, fewer or as many
    locations as consumers, tie-heavy): BUILD = greedy by full recomputation,
    SWAP = steepest descent by full recomputation, a local optimum, no better
    than the global optimum over all k-subsets of locations."""
    from itertools import combinations
    rng = np.random.default_rng(103)
    for trial in range(30):
        nc = int(rng.integers(3, 16))
        nl = int(rng.integers(3, 11))
        k = int(rng.integers(1, min(4, nl) + 1))
        D = rng.integers(0, 6 if trial % 2 else 30, size=(nc, nl)).astype(np.float64)
        Dl = D.tolist()
        bm, tdb = oracle.rect_build(k, D)
        assert list(bm) == brute.rect_build_greedy(Dl, k), trial
        assert tdb == brute.rect_td_of(Dl, list(bm))
        r = oracle.rect_swap(bm, D)
        med_b, trace_b = brute.rect_pam_swap(Dl, list(bm))
        assert list(r.medoids) == med_b and r.trace == [(i, c, float(v)) for i, c, v in trace_b]
        assert r.td == brute.rect_td_of(Dl, med_b)
        opt = min(brute.rect_td_of(Dl, list(m)) for m in combinations(range(nl), k))
        assert opt <= r.td


def test_rect_k1_is_the_bichromatic_medoid():
    """k = 1: the location minimising the summed distance to all consumers
    (the bichromatic medoid definition of Sec. 5), first on ties."""
    rng = np.random.default_rng(107)
    for _ in range(20):
        D = rng.integers(0, 50, size=(int(rng.integers(1, 30)), int(rng.integers(1, 20))))
        D = D.astype(np.float64)
        r = oracle.rect_pam(1, D)
        assert list(r.medoids) == [int(np.argmin(D.sum(0)))]


# ---------------------------------------------------------------- degenerate cases
def test_k_equals_n_and_duplicates():
    X = np.array([[0.0], [0.0], [1.0], [1.0], [5.0]])
    D = oracle.dist_matrix(X, oracle.L1)
    r = oracle.pam(5, D=D)
    assert r.td == 0.0 and sorted(r.medoids) == [0, 1, 2, 3, 4]
    r2 = oracle.pam(2, D=D)
    assert r2.td == brute.global_optimum(D.tolist(), 2)
    # duplicate points with zero distance keep caches consistent
    r3 = oracle.pam(3, D=D)
    assert r3.td == brute.td_of(D.tolist(), list(r3.medoids))
    assert brute.is_local_optimum(D.tolist(), list(r3.medoids))


def test_invalid_medoids_rejected():
    D = np.zeros((4, 4))
    with pytest.raises(ValueError):
        oracle.swap([0, 0], D=D)
    with pytest.raises(ValueError):
        oracle.swap([0, 7], D=D)


def test_running_td_bookkeeping_on_int_workload():
    """On the 1000-point integer workload shape (smaller n for speed) the
    running TD equals a fresh sum after every swap (checked inside the C code,
    rc would be negative) and iterations == swaps + 1."""
    X = datagen.workload_l1_int(n=300, seed=1001)
    D = oracle.dist_matrix(X, oracle.L1)
    r = oracle.pam(5, D=D)
    assert r.rc == 0 and r.iterations == r.swaps + 1
    tdv, _ = oracle.td(r.medoids, D=D)
    assert tdv == r.td == float(int(r.td))
