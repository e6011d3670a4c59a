"""Host logic of the posterior study (paper_2503_16028_amd/study.py) against closed forms and
planted structure (CPU only)."""
import math

import numpy as np
import pytest
from scipy.stats import norm

from paper_2503_16028_amd import study
from conftest import golden
from oracle.problem import Problem, synthesize


def blobs(centres, n, sd, seed):
    rng = np.random.default_rng(seed)
    return np.vstack([c + sd * rng.standard_normal((n, len(c))) for c in centres])


def test_kmeans_recovers_planted_clusters():
    centres = np.array([[0.0, 0.0, 0.0], [5.0, 0.0, 0.0], [0.0, 5.0, 1.0], [3.0, 3.0, 6.0]])
    X = blobs(centres, 200, 0.5, 1)
    k, lab, C, scores = study.count_modes(X, k_max=8, seed=2)
    assert k == 4 and scores[4] > 0.6
    order = [int(np.argmin(np.sum((C - c) ** 2, axis=1))) for c in centres]
    assert sorted(order) == [0, 1, 2, 3]
    assert np.abs(C[order] - centres).max() < 0.15            # 200 points of sd 0.5: se 0.035
    truth = np.repeat(np.arange(4), 200)
    assert all(len(set(lab[truth == j])) == 1 for j in range(4))


def test_one_gaussian_is_one_mode():
    X = np.random.default_rng(3).standard_normal((800, 5))
    k, lab, C, scores = study.count_modes(X, k_max=6, seed=0)
    assert k == 1 and max(scores.values()) < 0.25 and (lab == 0).all()
    assert np.allclose(C[0], X.mean(axis=0))


def test_silhouette_by_hand():
    """Points 0 and 1 in one cluster, 10 alone: s(0) = (10 - 1) / 10, s(1) = (9 - 1) / 9, and the
    singleton scores 0."""
    X = np.array([[0.0], [1.0], [10.0]])
    s = study.silhouette(X, np.array([0, 0, 1]))
    assert s == pytest.approx((0.9 + 8.0 / 9.0 + 0.0) / 3)


def test_rel_l2_error_is_the_function_space_norm():
    """Parseval against quadrature of the synthesised fields on the 128^2 grid (trapezoid
    rule, exact for the cosine products up to the highest mode pair)."""
    op = Problem.load(golden("problem_c3.json"))
    rng = np.random.default_rng(4)
    a, b = rng.standard_normal(op.K), rng.standard_normal(op.K)
    n = 128
    ua, ub = synthesize(op, a, n), synthesize(op, b, n)
    w = np.ones(n + 1)
    w[0] = w[-1] = 0.5
    W = np.outer(w, w) / n ** 2
    ref = math.sqrt(np.sum(W * (ua - ub) ** 2) / np.sum(W * ub ** 2))
    sl = study.sqrt_lambda(op.d)
    assert study.rel_l2_error(sl ** 2, a, b) == pytest.approx(ref, rel=1e-10)
    assert np.allclose(sl ** 2, op.lam)


def test_tv_distance_of_two_gaussians():
    """TV(N(0,1), N(1,1)) = 2 Phi(1/2) - 1; equal samples give 0; disjoint samples give 1."""
    rng = np.random.default_rng(5)
    a, b = rng.standard_normal(40000), 1.0 + rng.standard_normal(40000)
    assert study.tv_distance(a, b) == pytest.approx(2 * norm.cdf(0.5) - 1, abs=0.02)
    assert study.tv_distance(a, a) == 0.0
    assert study.tv_distance(a, a + 100.0) == pytest.approx(1.0, abs=1e-6)
    U = np.stack([a, b], axis=1)
    assert study.mean_tv(U, U + np.array([0.0, 1.0]), 2) == pytest.approx(study.tv_distance(b, b + 1.0) / 2)


def test_binned_kde_equals_the_direct_sum():
    x = np.random.default_rng(6).standard_normal(3000)
    g = np.linspace(-6.0, 6.0, 2001)
    bw = x.std(ddof=1) * x.size ** -0.2
    direct = np.exp(-0.5 * ((g[:, None] - x[None, :]) / bw) ** 2).sum(axis=1) / (x.size * bw * math.sqrt(2 * math.pi))
    assert np.abs(study.kde(x, g) - direct).max() < 1e-4 * direct.max()
    assert np.trapezoid(study.kde(x, g), g) == pytest.approx(1.0, abs=1e-6)
