"""Seeded synthetic inputs for k-medoids workloads.

This module only draws random numbers (numpy ``Generator(PCG64(seed))``); it
holds none of the clustering arithmetic, so both the GPU path and the CPU
oracle can take their inputs from it.

The paper's data sets (OR-Library, UCI plants/optdigits, MNIST) are not
available; these generators stand in for them with the shapes and value
distributions of the workloads the library is measured on:

* ``int_points``      -- integer coordinates, uniform in [lo, hi)
* ``gaussian_mixture``-- isotropic Gaussian mixture, centers uniform in a box,
                         equal or Zipf-distributed component weights, one sigma
                         or a per-component sigma range
* ``clara_samples``   -- subsample index lists for batched CLARA instances
"""
from __future__ import annotations

import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def int_points(n: int, dim: int, lo: int = 0, hi: int = 1000, seed: int = 0) -> np.ndarray:
    """n x dim int32 coordinates, uniform on {lo, ..., hi-1}."""
    return _rng(seed).integers(lo, hi, size=(n, dim), dtype=np.int64).astype(np.int32)


def gaussian_mixture(n: int, dim: int, n_comp: int, seed: int = 0,
                     box: float = 10.0, sigma=1.0, zipf_s: float | None = None,
                     return_labels: bool = False):
    """n x dim float32 points from an isotropic Gaussian mixture.

    Centers are uniform in [-box, box]^dim.  ``sigma`` is a scalar, or a
    (lo, hi) pair from which each component draws its own sigma uniformly.
    Component weights are equal, or proportional to j^-zipf_s (j = 1..n_comp).
    """
    g = _rng(seed)
    centers = g.uniform(-box, box, size=(n_comp, dim))
    if isinstance(sigma, (tuple, list)):
        sig = g.uniform(float(sigma[0]), float(sigma[1]), size=n_comp)
    else:
        sig = np.full(n_comp, float(sigma))
    if zipf_s is None:
        w = np.full(n_comp, 1.0 / n_comp)
    else:
        w = np.arange(1, n_comp + 1, dtype=np.float64) ** (-float(zipf_s))
        w /= w.sum()
    comp = g.choice(n_comp, size=n, p=w)
    X = centers[comp] + g.standard_normal(size=(n, dim)) * sig[comp, None]
    X = X.astype(np.float32)
    return (X, comp.astype(np.int32)) if return_labels else X


def clara_samples(N: int, n_inst: int, k_lo: int, k_hi: int, n_hi: int, seed: int = 0,
                  base: int = 40, per_k: int = 2):
    """Batched CLARA instances: for each instance j draw k_j uniform in
    {k_lo..k_hi} and a sample size n'_j uniform in {base + per_k*k_j .. n_hi},
    then n'_j distinct indices of [0, N) (without replacement, sorted).

    Returns (offsets int64[n_inst+1], indices int32[sum n'], k int32[n_inst]).
    """
    children = np.random.SeedSequence(seed).spawn(n_inst)
    ks = np.empty(n_inst, np.int32)
    idx = []
    off = np.zeros(n_inst + 1, np.int64)
    for j, ss in enumerate(children):
        g = np.random.Generator(np.random.PCG64(ss))
        k = int(g.integers(k_lo, k_hi + 1))
        lo = min(base + per_k * k, n_hi)
        m = int(g.integers(lo, n_hi + 1))
        sel = np.sort(g.choice(N, size=m, replace=False)).astype(np.int32)
        ks[j] = k
        idx.append(sel)
        off[j + 1] = off[j] + m
    return off, np.concatenate(idx) if idx else np.zeros(0, np.int32), ks


# Named workloads (shapes and distributions of the measured configurations).
def uniforms(count: int, seed: int = 0) -> np.ndarray:
    """count float64 uniforms in [0, 1)."""
    return _rng(seed).random(count)


def random_subset(n: int, size: int, seed: int = 0) -> np.ndarray:
    """size distinct indices of [0, n), drawn uniformly, int32."""
    return _rng(seed).choice(n, size=size, replace=False).astype(np.int32)


def subsamples(n: int, rows: int, size: int, seed: int = 0) -> np.ndarray:
    """(rows, size) int32: each row `size` distinct indices of [0, n) drawn
    uniformly, listed in ascending order."""
    g = _rng(seed)
    return np.stack([np.sort(g.choice(n, size=size, replace=False))
                     for _ in range(rows)]).astype(np.int32)


def workload_l1_int(n=1000, dim=2, seed=1001, hi=1000):
    """Integer coordinates uniform in [0, hi), Manhattan dissimilarity."""
    return int_points(n, dim, 0, hi, seed)


def workload_gmm16(n=20000, seed=1002):
    """20000 x 16 float32, 50 equal components, centers in [-10,10]^16, sigma 1."""
    return gaussian_mixture(n, 16, 50, seed=seed, sigma=1.0)


def workload_gmm64(n=50000, seed=1003):
    """50000 x 64 float32, 200 components, sigma uniform in [0.5, 2]."""
    return gaussian_mixture(n, 64, 200, seed=seed, sigma=(0.5, 2.0))


def workload_gmm8_pool(N=1_000_000, seed=1004):
    """1e6 x 8 float32 pool for batched CLARA, 100 equal components."""
    return gaussian_mixture(N, 8, 100, seed=seed, sigma=1.0)


def workload_gmm32_zipf(n=100000, seed=1005):
    """1e5 x 32 float32, 500 components with Zipf(1.1) weights, sigma 1."""
    return gaussian_mixture(n, 32, 500, seed=seed, sigma=1.0, zipf_s=1.1)
