"""Seeded generators for the GAME workloads.

The paper trains on a photometric catalogue of globular-cluster candidates
(Sec. 5: 2100 patterns, low-dimensional colour features, two classes).  That
catalogue is not available here, so these generators stand in with the same
shape: a handful of bounded features, a minority class, and a regression twin
whose target is a hidden polynomial plus Gaussian noise.

Everything here is data drawing.  The regression target evaluates a hidden
Chebyshev series with ``numpy.polynomial.chebyshev.chebval`` (a library
routine); neither the HIP path nor the oracle imports that code path.
"""
from __future__ import annotations

import hashlib
import math
from typing import Dict, List

import numpy as np

DATA_SEED_BASE = 12115481


def data_seed(config_index: int) -> int:
    """Seed for the patterns of workload ``config_index`` (1-based)."""
    return DATA_SEED_BASE + int(config_index)


def ga_seed(config_index: int) -> int:
    """Seed (Philox key) for the genetic algorithm of workload ``config_index``."""
    return data_seed(config_index) + 1000


def regression_dataset(n: int, f: int, degree: int, noise: float, seed: int):
    """Regression patterns: X ~ U[-1,1]^(n x f), t = hidden series + N(0, noise^2).

    The hidden target has one Chebyshev series per feature, degrees 1..degree,
    with coefficients drawn U[-1,1] (the same form as the model being fitted,
    so a perfect chromosome exists up to the noise).

    Returns (X float64 [n, f], t float64 [n], g_star float64 [f*degree]).
    """
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1.0, 1.0, size=(n, f))
    g_star = rng.uniform(-1.0, 1.0, size=f * degree)
    t = np.zeros(n)
    for i in range(f):
        coef = np.concatenate([[0.0], g_star[i * degree:(i + 1) * degree]])
        t += np.polynomial.chebyshev.chebval(X[:, i], coef)
    t += rng.normal(0.0, noise, size=n)
    return X, t, g_star


def classification_dataset(n: int, f: int, seed: int, frac1: float = 0.30,
                           offset: float = 0.5):
    """Two-class Gaussian mixture scaled to [-1, 1].

    label ~ Bernoulli(frac1); every feature x ~ N(offset * label, 1), features
    independent; each feature is then min-max scaled to [-1, 1] over all n rows.
    Returns (X float64 [n, f], t float64 [n] in {0, 1}).
    """
    rng = np.random.default_rng(seed)
    label = (rng.random(n) < frac1).astype(np.float64)
    X = rng.normal(0.0, 1.0, size=(n, f)) + offset * label[:, None]
    lo = X.min(axis=0)
    hi = X.max(axis=0)
    span = np.where(hi > lo, hi - lo, 1.0)
    X = 2.0 * (X - lo) / span - 1.0
    np.clip(X, -1.0, 1.0, out=X)
    return X, label


def batched_workload(n_runs: int, seed: int) -> List[Dict]:
    """Shapes of many independent GA runs of uneven size.

    N log-uniform in [1e4, 5e5], F uniform in {5..20}, D in {4, 6, 8},
    P in {256, 512, 1024, 2048}, task regression or classification with
    probability 1/2.  Regression runs use the Chebyshev basis and the
    regression generator, classification runs the trigonometric basis and the
    mixture generator.
    """
    rng = np.random.default_rng(seed)
    runs = []
    for r in range(n_runs):
        n = int(math.floor(math.exp(rng.uniform(math.log(1e4), math.log(5e5)))))
        f = int(rng.integers(5, 21))
        d = int(rng.choice([4, 6, 8]))
        p = int(rng.choice([256, 512, 1024, 2048]))
        cls = bool(rng.random() < 0.5)
        runs.append(dict(run=r, n=n, f=f, degree=d, pop=p,
                         task="classification" if cls else "regression",
                         basis="trig" if cls else "chebyshev",
                         data_seed=seed + r))
    return runs


def random_population(p: int, l: int, seed: int) -> np.ndarray:
    """Arbitrary chromosomes, U[-1, 1) float32, for operator tests."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(p, l)).astype(np.float32)


def random_fitness(p: int, seed: int, n_ties: int = 0, n_nan: int = 0) -> np.ndarray:
    """A fitness vector (float64) with optional exact ties and NaNs."""
    rng = np.random.default_rng(seed)
    fit = 1.0 - rng.uniform(0.0, 0.5, size=p)
    if n_ties:
        src = rng.integers(0, p, size=n_ties)
        dst = rng.integers(0, p, size=n_ties)
        fit[dst] = fit[src]
    if n_nan:
        fit[rng.choice(p, size=n_nan, replace=False)] = np.nan
    return fit


def sha256_arrays(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()
