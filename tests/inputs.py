"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

This module holds no arithmetic of the method: it only draws arrays of the shapes
and value ranges the sampler sees (prior-like coefficients, mixture parameters,
weights, uniforms) from NumPy's seeded generators.
"""
import numpy as np


def particles(N, K, seed, scale=1.0):
    """Coefficient vectors like prior draws (N x K, float64)."""
    return scale * np.random.default_rng(seed).standard_normal((N, K))


def mixture(M, kr, seed, spread=1.0):
    """(logw, mean, scale) for an M-component diagonal mixture on kr modes."""
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.5, 1.5, M)
    logw = np.log(w / w.sum())
    mean = spread * rng.standard_normal((M, kr))
    scale = rng.uniform(0.05, 1.2, (M, kr))
    return logw, mean, scale


def potentials(N, seed, spread=50.0):
    """Potential-like values: nonnegative, heavy spread."""
    rng = np.random.default_rng(seed)
    return spread * rng.chisquare(4, N)


def weights(N, seed, kind="dirichlet"):
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return np.full(N, 1.0 / N)
    if kind == "one":
        w = np.zeros(N)
        w[rng.integers(N)] = 1.0
        return w
    if kind == "sparse":
        w = np.zeros(N)
        pick = rng.choice(N, size=max(1, N // 7), replace=False)
        w[pick] = rng.exponential(1.0, pick.size)
        return w / w.sum()
    w = rng.exponential(1.0, N) ** 3
    return w / w.sum()


def u53(seed):
    return int(np.random.default_rng(seed).integers(0, 2 ** 53))


def clusters(N, D, M, seed, sep=4.0, dup=0):
    """A cloud of N points in D dimensions around M random centres (spread `sep`), with
    per-cluster, per-axis scales in [0.3, 1.2]; the last `dup` rows repeat row 0.
    Returns (X, labels, centres, scales)."""
    rng = np.random.default_rng(seed)
    centres = sep * rng.standard_normal((M, D))
    scales = rng.uniform(0.3, 1.2, (M, D))
    labels = rng.integers(0, M, N)
    X = centres[labels] + scales[labels] * rng.standard_normal((N, D))
    if dup:
        X[N - dup:] = X[0]
    return X, labels, centres, scales
