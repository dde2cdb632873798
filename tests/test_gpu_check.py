"""GPU check of a dissimilarity matrix (the properties PAM's arithmetic relies
on, Sec. 2: symmetric, zero diagonal, finite, non-negative).  Valid matrices
from the distance kernels and the oracle pass; each planted defect is found
with its own flag and counted once per unordered pair; sizes span several
64 x 64 tiles with a ragged edge and a padded row stride."""
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


@pytest.mark.parametrize("n", [1, 63, 200, 1000])
def test_valid_matrices_pass(n):
    _say("check_valid", n)
    X = datagen.gaussian_mixture(n, 8, 4, seed=n)
    D = px().dist(torch.from_numpy(X).to(DEV))
    r = px().check_dissimilarity(D)
    assert r["valid"] and r["pairs"] == 0
    Xi = datagen.int_points(n, 2, 0, 100, seed=n)
    Di = torch.from_numpy(oracle.dist_matrix(Xi, oracle.L1).astype(np.int32)).to(DEV)
    assert px().check_dissimilarity(Di)["valid"]


@pytest.mark.parametrize("dtype", ["f32", "i32"])
def test_planted_defects(dtype):
    _say("check_defects", dtype)
    n = 333
    X = datagen.int_points(n, 2, 0, 50, seed=5)
    D = oracle.dist_matrix(X, oracle.L1)
    D = D.astype(np.float32 if dtype == "f32" else np.int32)
    # padded rows: the check reads n columns of a stride-340 matrix
    Dp = np.full((n, 340), -1, D.dtype)
    Dp[:, :n] = D

    def run(M):
        t = torch.from_numpy(M).to(DEV)[:, :n]
        return px().check_dissimilarity(t)

    assert run(Dp)["valid"]
    a = Dp.copy(); a[10, 300] += 1
    r = run(a)
    assert r["asymmetric"] and not r["diagonal"] and r["pairs"] == 1
    b = Dp.copy(); b[70, 70] = 3
    r = run(b)
    assert r["diagonal"] and not r["asymmetric"] and r["pairs"] == 1
    c = Dp.copy(); c[5, 6] = -2; c[6, 5] = -2
    r = run(c)
    assert r["negative"] and not r["asymmetric"] and r["pairs"] == 1
    d = Dp.copy(); d[300, 2] = -1       # lower entry: negative and asymmetric, one pair
    r = run(d)
    assert r["negative"] and r["asymmetric"] and r["pairs"] == 1
    if dtype == "f32":
        e = Dp.copy(); e[100, 200] = np.nan; e[200, 100] = np.nan
        r = run(e)
        assert r["nonfinite"] and r["asymmetric"] and r["pairs"] == 1
        f = Dp.copy(); f[1, 2] = np.inf; f[2, 1] = np.inf
        r = run(f)
        assert r["nonfinite"] and not r["asymmetric"] and r["pairs"] == 1
