"""Gaussian-mixture fit of the particle cloud (the stage input of the pCN-GM move and
the mutation of SMC-GM).

TEST INFRASTRUCTURE ONLY (see the package docstring).  The paper estimates the mixture
with the method of its reference [Feng2018] (Sec. 2.3, remark on the pCN-GM proposal;
Sec. 2.4), which it does not describe, so the choice of estimator is unpinned against
the paper.  The stand-in here is expectation-maximisation with diagonal covariances on
the active whitened coordinates, k-means++ seeding, a fixed iteration count and a
variance floor; any valid mixture keeps the pCN-GM move invariant, so the move tests
do not depend on how good this fit is.  The EM steps and the seeding are pinned to
what they must compute (closed forms, monotone likelihood, selection frequencies) in
the oracle's own tests.

Two seedings:
  fit          k-means++ with NumPy's generator (the oracle's own SMC loop);
  fit_philox   k-means++ with draws from the Philox layout of `philox`, which the GPU
               fit follows:
    * the uniform of centre m is the 53-bit integer u_m = (w0 >> 5) 2^26 + (w1 >> 6) of
      block KMPP_BLOCK, particle word m, at the call's counter;
    * centre 0 is row floor(u_0 N / 2^53);
    * for m >= 1, d2_n is the smallest squared distance of row n to the centres so far,
      each squared distance the exactly rounded sum (math.fsum) of the K_r squared
      coordinate differences;
    * with D = max_n d2_n = f 2^e (f in [1/2, 1)), q_n = floor(d2_n 2^(40 - e)) are
      exact integers below 2^40; C_n = q_0 + ... + q_n, Q = C_{N-1};
    * centre m is row min{n : C_n > t}, t = floor(u_m Q / 2^53) (probability q_n / Q), or
      row floor(u_m N / 2^53) when Q = 0 (every row is a centre already).
    Integer sums make the choice independent of summation order; the floating point that
    decides it is d2_n.  Any other summation order of the K_r <= 64 non-negative terms
    (the device adds them pairwise) is within 7 eps of d2_n, which moves each q_n by at
    most 1, each C_n and Q by at most N and t by at most N + 1: a choice whose margin
    min(t - C_{n-1}, C_n - 1 - t) exceeds 2 N + 2, with D not within 7 eps of a power of
    two, is the same for every order (`kmeanspp_philox(..., margins=True)` reports both).
"""
import math

import numpy as np
from scipy.special import logsumexp

from . import philox

KMPP_BLOCK = 0x80000002
QBITS = 40


def kmeanspp(X, M, rng):
    N = X.shape[0]
    centers = [X[rng.integers(N)]]
    for _ in range(1, M):
        d2 = np.min([np.sum((X - c) ** 2, axis=1) for c in centers], axis=0)
        p = d2 / d2.sum() if d2.sum() > 0 else np.full(N, 1.0 / N)
        centers.append(X[rng.choice(N, p=p)])
    return np.array(centers)


def em(X, logw, mean, var, iters, var_floor=1e-3):
    """`iters` EM steps for sum_j w_j N(m_j, diag(s_j)) on rows of X from the given start.

    E-step: responsibilities R_nj = w_j N(x_n; m_j, s_j) / sum_i w_i N(x_n; m_i, s_i) in log
    space; M-step: N_j = sum_n R_nj, w_j = N_j / N, m_j = sum_n R_nj x_n / N_j,
    s_j = max(sum_n R_nj x_n^2 / N_j - m_j^2, var_floor).  Returns (logw, mean, var) with
    logw normalised to sum_j w_j = 1.
    """
    X = np.asarray(X, dtype=np.float64)
    N = X.shape[0]
    logw, mean, var = (np.array(a, dtype=np.float64, copy=True) for a in (logw, mean, var))
    M = logw.size
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


def start(X, centers, var_floor=1e-3):
    """EM start: equal weights, the seeded centres, the cloud's variance (floored) in every
    component."""
    X = np.asarray(X, dtype=np.float64)
    M = len(centers)
    var = np.tile(np.maximum(X.var(axis=0), var_floor), (M, 1))
    return np.full(M, -np.log(M)), X[np.asarray(centers)], var


def fit(X, M, seed=0, iters=50, var_floor=1e-3):
    """EM for sum_j w_j N(m_j, diag(s_j)) on rows of X; returns (logw, mean, scale)."""
    X = np.asarray(X, dtype=np.float64)
    rng = np.random.default_rng(seed)
    mean = kmeanspp(X, M, rng)
    var = np.tile(np.maximum(X.var(axis=0), var_floor), (M, 1))
    return em(X, np.full(M, -np.log(M)), mean, var, iters, var_floor)


# ---------------------------------------------------------------- Philox-seeded variant

def exact_row_sums(v):
    """Each row's sum, exactly rounded (math.fsum)."""
    v = np.asarray(v, dtype=np.float64)
    return np.array([math.fsum(row) for row in v.reshape(-1, v.shape[-1])]).reshape(v.shape[:-1])


def kmpp_u53(seed, ctr, m):
    """The 53-bit integer uniform of centre m."""
    c = np.array([KMPP_BLOCK, m, ctr & philox.MASK32, (ctr >> 32) & philox.MASK32], dtype=np.uint64)
    w = philox.philox4x32_10(c, philox._key(seed))
    return (int(w[0]) >> 5) * (1 << 26) + (int(w[1]) >> 6)


def kmeanspp_philox(X, M, seed, ctr, margins=False):
    """Row indices of the M seeded centres (see the module docstring).  With margins=True also
    returns, for every centre drawn with Q > 0, (margin, bound, power_of_two_clear): its
    distance in integer units from the nearest choice boundary, 2 N + 2, and whether D is more
    than 7 eps from a power of two."""
    X = np.asarray(X, dtype=np.float64)
    N = X.shape[0]
    idx = [(kmpp_u53(seed, ctr, 0) * N) >> 53]
    info = []
    d2 = np.full(N, np.inf)
    for m in range(1, M):
        r = X - X[idx[-1]]
        d2 = np.minimum(d2, exact_row_sums(r * r))
        u = kmpp_u53(seed, ctr, m)
        dmax = float(d2.max())
        if dmax == 0.0:
            idx.append((u * N) >> 53)
            continue
        f, e = math.frexp(dmax)
        q = [math.floor(math.ldexp(float(v), QBITS - e)) for v in d2]
        Q = sum(q)
        t = (u * Q) >> 53
        c = 0
        for n, qn in enumerate(q):
            prev = c
            c += qn
            if c > t:
                idx.append(n)
                eps7 = 7 * np.finfo(float).eps
                info.append((min(t - prev, c - 1 - t), 2 * N + 2, 0.5 + eps7 < f < 1.0 - eps7))
                break
    return (idx, info) if margins else idx


def fit_philox(X, M, seed, ctr, iters=50, var_floor=1e-3):
    """Philox-seeded k-means++ start, then `iters` EM steps; returns (logw, mean, var, centres)."""
    centers = kmeanspp_philox(X, M, seed, ctr)
    logw, mean, var = em(X, *start(X, centers, var_floor), iters, var_floor)
    return logw, mean, var, centers
