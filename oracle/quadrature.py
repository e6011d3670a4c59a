"""Posterior moments by brute-force quadrature on a tiny parameter space.

TEST INFRASTRUCTURE ONLY (see the package docstring).

For K = 1 or 2 whitened coordinates the posterior density of Sec. 2.1
(eq. (Bayes)), exp(-tau Phi(xi)) N(xi; 0, I) / Z, is tabulated on a tensor grid
and its moments are Riemann sums.  Each grid point costs one forward solve.
"""
import itertools

import numpy as np


def moments(phi_fn, K, lo=-6.0, hi=6.0, pts=400, tau=1.0):
    """(mean, covariance, weights, grid) of the tempered posterior."""
    g = np.linspace(lo, hi, pts)
    grid = np.array(list(itertools.product(g, repeat=K)))
    logp = np.array([-tau * phi_fn(x) for x in grid]) - 0.5 * np.sum(grid ** 2, axis=1)
    logp -= logp.max()
    w = np.exp(logp)
    w /= w.sum()
    mean = w @ grid
    r = grid - mean
    cov = (w[:, None] * r).T @ r
    return mean, cov, w, grid
