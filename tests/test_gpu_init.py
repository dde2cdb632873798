"""GPU parity of the faster initialisations (Sec. 3.3) against the oracle.

Integer dissimilarities: the seeds of distance-weighted seeding and of LAB
equal the oracle's bit for bit (weights and changes are exact integers on
both sides; the same uniforms and subsamples are inputs to both).  Float
dissimilarities: the GPU sums in another order, so its picks are replayed on
FP64 numpy sums of the same matrix and checked to be valid within the
summation bound.  Then BUILD-free fits: seeding + FasterPAM / FastPAM1 equal
the oracle's runs.
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


# ------------------------------------------------------------------ distance-weighted seeding
@pytest.mark.parametrize("n,k,hi,seed", [(1000, 5, 1000, 1), (1000, 30, 1000, 2), (1000, 50, 8, 3),
                                         (257, 20, 50, 4), (3000, 100, 300, 5), (64, 64, 4, 6)])
def test_dw_int_bitexact(n, k, hi, seed):
    _say("dw_int", n, k, hi, seed)
    X, D = _int_case(n, seed, hi=hi)
    u = datagen.uniforms(k, seed)
    ref = oracle.init_dw(k, u, D=D)
    med = px().init_dw(_t(D.astype(np.int32)), k, u=u)
    assert list(med.cpu().numpy()) == list(ref)


def test_dw_int_many_block_sums():
    """n = 70000: more than 256 blocks of weights, so the block sums are
    scanned in several chunks.  Oracle on the points (distances on the fly)."""
    _say("dw_int_70000")
    X = datagen.int_points(70000, 2, 0, 5000, seed=7)
    D = px().dist(_t(X))
    u = datagen.uniforms(12, 7)
    ref = oracle.init_dw(12, u, X=X.astype(np.float64), metric=oracle.L1)
    med = px().init_dw(D, 12, u=u)
    assert list(med.cpu().numpy()) == list(ref)
    del D


def _check_dw_float(D64, u, med):
    """Every GPU pick is valid for FP64 sums of the same weights: its running
    sum brackets u_t W within the summation bound, and it has weight > 0."""
    n = D64.shape[0]
    med = [int(v) for v in med]
    assert med[0] == min(int(np.floor(u[0] * n)), n - 1)
    w = D64[:, med[0]].copy()
    for t in range(1, len(med)):
        W = float(w.sum())
        tol = 8 * n * 2.0 ** -53 * W
        target = u[t] * W
        cs = np.cumsum(w)
        p = med[t]
        assert w[p] > 0, t
        assert cs[p] >= target - tol and (p == 0 or cs[p - 1] <= target + tol), t
        w = np.minimum(w, D64[:, p])
    assert len(set(med)) == len(med)


@pytest.mark.parametrize("n,k,seed", [(2000, 40, 11), (20000, 100, 12)])
def test_dw_float_valid(n, k, seed):
    _say("dw_float", n, k)
    X = datagen.gaussian_mixture(n, 16, 50, seed=seed)
    Dg = px().dist(_t(X))
    u = datagen.uniforms(k, seed)
    med = px().init_dw(Dg, k, u=u).cpu().numpy()
    D64 = Dg.cpu().numpy().astype(np.float64)
    _check_dw_float(D64, u, med)
    # and the oracle on the same matrix takes the same seeds (no pick lies
    # within rounding of a boundary for these draws)
    assert list(oracle.init_dw(k, u, D=D64)) == list(med)


# ------------------------------------------------------------------ LAB
@pytest.mark.parametrize("n,k,hi,seed,excl", [(1000, 5, 1000, 21, False), (1000, 30, 40, 22, False),
                                              (1000, 30, 40, 23, True), (300, 40, 10, 24, False),
                                              (5000, 60, 500, 25, False), (50, 50, 5, 26, False)])
def test_lab_int_bitexact(n, k, hi, seed, excl):
    _say("lab_int", n, k, hi, seed, excl)
    X, D = _int_case(n, seed, hi=hi)
    m = px().lab_sample_size(n)
    S = datagen.subsamples(n, k, m, seed)
    ref = oracle.init_lab(k, S, D=D, exclude_self=excl)
    med = px().init_lab(_t(D.astype(np.int32)), k, samples=S, exclude_self=excl)
    assert list(med.cpu().numpy()) == list(ref)


def test_lab_full_sample_equals_build():
    """Every step's sample the whole set in index order: LAB is BUILD."""
    _say("lab_full")
    X, D = _int_case(700, 31, hi=300)
    S = np.tile(np.arange(700, dtype=np.int32), (9, 1))
    Di = _t(D.astype(np.int32))
    med = px().init_lab(Di, 9, samples=S)
    b = px().build(Di, 9)[0]
    assert torch.equal(med, b)
    assert list(med.cpu().numpy()) == list(oracle.build(9, D=D)[0])


def test_lab_float_valid():
    """Float matrix: each step's pick has the smallest subsample change up to
    the FP64 summation bound (changes recomputed in numpy on the GPU's own
    earlier picks)."""
    _say("lab_float")
    X = datagen.gaussian_mixture(20000, 16, 50, seed=41)
    Dg = px().dist(_t(X))
    k = 100
    m = px().lab_sample_size(20000)
    S = datagen.subsamples(20000, k, m, 41)
    med = px().init_lab(Dg, k, samples=S).cpu().numpy()
    D64 = Dg.cpu().numpy().astype(np.float64)
    dn = np.full(20000, np.inf)
    chosen = []
    for t in range(k):
        s = S[t]
        cand = [c for c in s if c not in set(chosen)]
        vals = []
        for c in cand:
            if t == 0:
                v = D64[s, c].sum()
            else:
                live = np.array([o not in set(chosen) and o != c for o in s])
                dd = D64[s[live], c] - dn[s[live]]
                v = dd[dd < 0].sum() - dn[c]
            vals.append(v)
        vals = np.array(vals)
        scale = m * (float(np.abs(D64[s][:, s]).max()) + 1.0)
        tol = 8 * m * 2.0 ** -53 * scale
        p = int(med[t])
        assert p in cand
        assert vals[cand.index(p)] <= vals.min() + tol, t
        chosen.append(p)
        dn = np.minimum(dn, D64[:, p])
    assert list(oracle.init_lab(k, S, D=D64)) == list(med)


# ------------------------------------------------------------------ BUILD-free fits
@pytest.mark.parametrize("init", ["random", "dw", "lab"])
@pytest.mark.parametrize("variant", ["fasterpam", "fastpam1"])
def test_fit_with_cheap_init_bitexact(init, variant):
    _say("fit_init", init, variant)
    X, D = _int_case(1500, 51, hi=400)
    k, seed = 15, 51
    n = 1500
    if init == "random":
        start = datagen.random_subset(n, k, seed)
    elif init == "dw":
        start = oracle.init_dw(k, datagen.uniforms(k, seed), D=D)
    else:
        start = oracle.init_lab(k, datagen.subsamples(n, k, px().lab_sample_size(n), seed), D=D)
    v = oracle.FASTERPAM if variant == "fasterpam" else oracle.PAM
    ref = oracle.swap(start, D=D, variant=v)
    res = px().fit(_t(X), k, variant=variant, init=init, seed=seed, trace=True)
    assert list(res.stats["init_medoids"].cpu().numpy()) == list(start)
    assert list(res.medoids.cpu().numpy()) == list(ref.medoids)
    assert res.td == ref.td and res.trace == ref.trace
