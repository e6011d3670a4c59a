"""Pins of the oracle's mixture fit, mixture draw and SMC-GM loop (CPU only).

The fit's estimator is a stand-in of this library (the paper's is not described), so the
pins check that it computes what it states: the exactly rounded sums of the seeding's
distances, the k-means++ selection probabilities, the EM step's closed form for one
component, the monotone likelihood of EM, and recovery of a known mixture.
"""
import math

import numpy as np
import pytest
import scipy.stats
from scipy.special import logsumexp

import inputs
from oracle import gmfit, linear, philox, smc
from oracle.moves import GM, gm_draw, pcn_gm


# ------------------------------------------------------------------ seeding

def test_squared_distances_are_exactly_rounded():
    """The seeding's distances are the exactly rounded sums of the squared differences: against
    rational arithmetic, and equal to the exact integer sum where that is representable."""
    from fractions import Fraction
    rng = np.random.default_rng(1)
    for kr in (64, 37, 1):
        v = rng.standard_normal((20, kr)) ** 2 * 10.0 ** rng.integers(-8, 8, (20, kr))
        got = gmfit.exact_row_sums(v)
        for row, g in zip(v, got):
            exact = sum(Fraction(float(x)) for x in row)
            assert g == float(exact)     # float(Fraction) rounds to nearest
    ints = rng.integers(0, 1000, (3, 64)).astype(float)
    assert np.array_equal(gmfit.exact_row_sums(ints), ints.sum(axis=1))


def test_choice_margin_covers_any_summation_order():
    """Moving each integer weight by at most 1 (what another summation order of the distances can
    do) never changes a choice whose reported margin exceeds the bound: brute force over random
    perturbations of the same weights."""
    X = inputs.particles(300, 16, 21)
    rng = np.random.default_rng(2)
    for ctr in range(6):
        idx, info = gmfit.kmeanspp_philox(X, 5, seed=4, ctr=ctr, margins=True)
        assert len(info) == 4 and all(clear for _, _, clear in info)
        assert all(mg > bound for mg, bound, _ in info)
    # the margin arithmetic itself: perturb q by +-1 and recompute the choice
    q = rng.integers(0, 1 << 40, 300)
    u = int(rng.integers(0, 1 << 53))
    def choose(qq):
        t = (u * int(sum(int(x) for x in qq))) >> 53
        c = 0
        for n, x in enumerate(qq):
            c += int(x)
            if c > t:
                return n, t, c - int(x), c
    n0, t, lo, hi = choose(q)
    margin = min(t - lo, hi - 1 - t)
    if margin > 2 * q.size + 2:
        for _ in range(200):
            assert choose(q + rng.integers(-1, 2, q.size))[0] == n0


def test_kmeanspp_all_rows_when_m_equals_n():
    """A chosen row has distance 0 and integer weight 0, so M = N distinct rows pick every row once."""
    X = inputs.particles(12, 5, 3)
    for ctr in range(5):
        assert sorted(gmfit.kmeanspp_philox(X, 12, seed=9, ctr=ctr)) == list(range(12))


def test_kmeanspp_second_centre_frequencies():
    """P(centre 1 = n | centre 0) = d2_n / sum d2 (k-means++), over many counters."""
    X = np.array([[0.0], [1.0], [3.0], [7.0]])
    counts = np.zeros((4, 4))
    T = 6000
    for ctr in range(T):
        i0, i1 = gmfit.kmeanspp_philox(X, 2, seed=5, ctr=ctr)
        counts[i0, i1] += 1
    first = counts.sum(1)
    assert np.all(np.abs(first / T - 0.25) < 4 * math.sqrt(0.25 * 0.75 / T))   # centre 0 uniform
    for i0 in range(4):
        d2 = (X[:, 0] - X[i0, 0]) ** 2
        p = d2 / d2.sum()
        f = counts[i0] / first[i0]
        assert np.all(np.abs(f - p) < 4 * np.sqrt(p * (1 - p) / first[i0]) + 1e-12), (i0, f, p)


def test_kmeanspp_identical_rows_fall_back_to_uniform():
    X = np.ones((30, 4))
    idx = gmfit.kmeanspp_philox(X, 6, seed=1, ctr=2)
    assert len(idx) == 6 and all(0 <= i < 30 for i in idx)
    u = [gmfit.kmpp_u53(1, 2, m) for m in range(6)]
    assert idx == [(x * 30) >> 53 for x in u]


def test_kmeanspp_integer_weights_are_exact_and_bounded():
    """q_n = floor(d2_n 2^(40-e)) is exact (power-of-two scaling) and the largest is in [2^39, 2^40)."""
    rng = np.random.default_rng(4)
    d2 = rng.exponential(1.0, 100) * 10.0 ** rng.integers(-200, 200)
    e = math.frexp(float(d2.max()))[1]
    q = [math.floor(math.ldexp(float(v), gmfit.QBITS - e)) for v in d2]
    assert 2 ** 39 <= max(q) < 2 ** 40
    for v, qn in zip(d2, q):
        assert abs(qn - float(v) * 2.0 ** (gmfit.QBITS - e)) < 1.0


# ------------------------------------------------------------------ EM

def _loglik(X, logw, mean, var):
    comp = [logw[j] + scipy.stats.norm(mean[j], np.sqrt(var[j])).logpdf(X).sum(1) for j in range(len(logw))]
    return float(logsumexp(np.array(comp), axis=0).sum())


def test_em_one_component_is_sample_moments():
    X = inputs.particles(500, 7, 2, 1.7) + 0.4
    logw, mean, var = gmfit.em(X, [0.0], X[:1], np.ones((1, 7)), iters=1)
    assert logw[0] == pytest.approx(0.0, abs=1e-15)
    assert np.allclose(mean[0], X.mean(0), rtol=0, atol=1e-13)
    assert np.allclose(var[0], X.var(0), rtol=1e-12)


def test_em_likelihood_never_decreases():
    X, *_ = inputs.clusters(600, 4, 3, seed=6, sep=2.0)
    logw, mean, var = gmfit.start(X, gmfit.kmeanspp_philox(X, 3, seed=1, ctr=0))
    prev = _loglik(X, logw, mean, var)
    for _ in range(25):
        logw, mean, var = gmfit.em(X, logw, mean, var, iters=1)
        cur = _loglik(X, logw, mean, var)
        assert cur >= prev - 1e-9 * abs(prev)
        prev = cur


def test_em_recovers_separated_mixture():
    X, labels, centres, scales = inputs.clusters(20000, 3, 2, seed=8, sep=5.0)
    logw, mean, var, _ = gmfit.fit_philox(X, 2, seed=3, ctr=11)
    order = np.argsort(mean[:, 0])
    true = np.argsort(centres[:, 0])
    for a, b in zip(order, true):
        assert math.exp(logw[a]) == pytest.approx(np.mean(labels == b), abs=0.01)
        assert np.allclose(mean[a], centres[b], atol=0.05)
        assert np.allclose(np.sqrt(var[a]), scales[b], rtol=0.05)
    assert logsumexp(logw) == pytest.approx(0.0, abs=1e-14)


def test_em_variance_floor():
    X = inputs.particles(200, 3, 1)
    X[:, 1] = 0.25
    _, _, var, _ = gmfit.fit_philox(X, 3, seed=0, ctr=0, iters=10, var_floor=1e-3)
    assert np.all(var[:, 1] == 1e-3) and np.all(var >= 1e-3)


# ------------------------------------------------------------------ mixture draw

def test_gm_draw_standard_mixture_is_prior_draw():
    K = 20
    v = gm_draw(pcn_gm(K, np.arange(6)), seed=3, ctr=17, ids=np.arange(9))
    assert np.array_equal(v, philox.normals(3, 17, np.arange(9), K))


def test_gm_draw_moments():
    K, kr, N = 10, 3, 40000
    logw = np.log([0.3, 0.7])
    mean = np.array([[-2.0, 0.5, 1.0], [3.0, -1.0, 0.0]])
    var = np.array([[0.5, 1.0, 0.2], [2.0, 0.3, 1.5]])
    gm = GM(logw, mean, var, np.array([1, 4, 7]), K)
    v = gm_draw(gm, seed=2, ctr=5, ids=np.arange(N))
    w = np.exp(logw)
    p_hi = sum(w[j] * scipy.stats.norm(mean[j, 0], math.sqrt(var[j, 0])).sf(0.5) for j in range(2))
    assert np.mean(v[:, 1] > 0.5) == pytest.approx(p_hi, abs=4 * math.sqrt(p_hi * (1 - p_hi) / N))
    mu = w @ mean
    var_mix = w @ (var + mean ** 2) - mu ** 2
    assert np.allclose(v[:, [1, 4, 7]].mean(0), mu, atol=4 * np.sqrt(var_mix / N))
    assert np.allclose(v[:, [1, 4, 7]].var(0), var_mix, rtol=0.03)
    rest = np.delete(v, [1, 4, 7], axis=1)
    assert abs(rest.mean()) < 4 / math.sqrt(rest.size) and rest.var() == pytest.approx(1.0, rel=0.02)


# ------------------------------------------------------------------ SMC-GM loop

def test_smc_gm_gaussian_posterior():
    """Diagonal linear-Gaussian problem: a one-component diagonal mixture holds every tempered
    posterior exactly, so SMC-GM (Alg. 3) recovers the closed-form posterior and evidence."""
    from oracle.problem import Problem
    K = 4
    H = np.diag([1.5, 0.8, 0.4, 0.2])
    sig = 0.3
    d = H @ np.array([0.8, -1.2, 0.5, 0.3]) + sig * np.array([0.3, -1.1, 0.6, 0.2])
    m_p, S_p = linear.posterior(H, d, sig)
    f = linear.phi_fn(H, d, sig)
    p = Problem(dict(name="lin", dim=1, grids=[16], kl_per_axis=K, kr=K, obs_den=16, obs=[[3]], y=[0.0],
                     sigma=1.0, f=1.0))
    N = 16000                       # resampling and the refit each stage widen the spread to about 2x iid
    out = smc.run_gm(p, 16, N, M=1, rho=0.5, seed=7, phi_fn=f, kr=K, iters=2)
    xi = out["xi"]
    sd = np.sqrt(np.diag(S_p))
    assert np.all(np.abs(xi.mean(0) - m_p) < 5 * sd / math.sqrt(N / 4))
    assert np.all(np.abs(xi.std(0) / sd - 1) < 0.05)
    assert out["log_Z"] == pytest.approx(linear.log_evidence(H, d, sig), abs=0.05)
    assert out["taus"][-1] == 1.0 and np.all(np.diff(out["taus"]) > 0)
