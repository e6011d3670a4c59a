"""Gaussian-mixture fit of the particle cloud (the stage input of the pCN-GM move).

TEST INFRASTRUCTURE ONLY (see the package docstring).  PARITY UNPINNED: the paper
estimates the mixture with the method of its reference [Feng2018] (Sec. 2.3,
remark on the pCN-GM proposal; Sec. 2.4), which it does not describe.  This is a
stand-in: expectation-maximisation with diagonal covariances on the active
whitened coordinates, k-means++ seeding, a fixed iteration count and a variance
floor.  Any valid mixture keeps the move invariant, so the move tests do not
depend on how good this fit is.
"""
import numpy as np
from scipy.special import logsumexp


def kmeanspp(X, M, rng):
    N = X.shape[0]
    centers = [X[rng.integers(N)]]
    for _ in range(1, M):
        d2 = np.min([np.sum((X - c) ** 2, axis=1) for c in centers], axis=0)
        p = d2 / d2.sum() if d2.sum() > 0 else np.full(N, 1.0 / N)
        centers.append(X[rng.choice(N, p=p)])
    return np.array(centers)


def fit(X, M, seed=0, iters=50, var_floor=1e-3):
    """EM for sum_j w_j N(m_j, diag(s_j)) on rows of X; returns (logw, mean, scale)."""
    X = np.asarray(X, dtype=np.float64)
    N, D = X.shape
    rng = np.random.default_rng(seed)
    mean = kmeanspp(X, M, rng)
    var = np.tile(np.maximum(X.var(axis=0), var_floor), (M, 1))
    logw = np.full(M, -np.log(M))
    for _ in range(iters):
        ll = np.stack([logw[j] - 0.5 * np.sum((X - mean[j]) ** 2 / var[j] + np.log(2 * np.pi * var[j]), axis=1)
                       for j in range(M)], axis=1)
        R = np.exp(ll - logsumexp(ll, axis=1, keepdims=True))
        Nk = R.sum(axis=0) + 1e-300
        logw = np.log(Nk / N)
        mean = (R.T @ X) / Nk[:, None]
        var = np.maximum((R.T @ (X * X)) / Nk[:, None] - mean ** 2, var_floor)
    logw = logw - logsumexp(logw)
    return logw, mean, var
