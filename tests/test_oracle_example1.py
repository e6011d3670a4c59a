"""Pins of the Example 1 oracle (Sec. 3.1): the potential against function-space quadrature,
the closed-form mixture posterior and evidence against importance sampling from the prior
(CPU only)."""
import math

import numpy as np
import pytest
from scipy.special import logsumexp

from oracle import example1 as ex


def _field(prob, xi, x):
    """u(x) = sum_k sqrt(lambda_k) xi_k phi_k(x), phi_0 = 1, phi_k = sqrt(2) cos(k pi x)."""
    k = np.arange(prob["K"])
    basis = np.where(k[None, :] == 0, 1.0, np.sqrt(2.0) * np.cos(np.pi * k[None, :] * x[:, None]))
    return basis @ (prob["sqrt_lam"] * xi)


@pytest.mark.parametrize("K,sigma", [(8, 0.1), (12, 0.3)])
def test_potential_against_function_space_quadrature(K, sigma):
    prob = ex.problem(K=K, sigma=sigma)
    t, w = np.polynomial.legendre.leggauss(200)
    x, w = 0.5 * (t + 1.0), 0.5 * w
    f = [np.cos(np.pi * x), -np.cos(np.pi * x), np.cos(2 * np.pi * x), np.cos(3 * np.pi * x)]
    rng = np.random.default_rng(K)
    for _ in range(5):
        xi = rng.standard_normal(K)
        u = _field(prob, xi, x)
        d2 = np.array([np.sum(w * (u - fi) ** 2) for fi in f])
        ref = -logsumexp(-d2 / (2 * sigma ** 2))
        assert ex.phi(prob, xi) == pytest.approx(ref, rel=1e-11, abs=1e-11)


@pytest.mark.parametrize("K", [4, 16])
def test_posterior_and_evidence_against_importance_sampling(K):
    """Prior draws weighted by exp(-Phi): first and second moments of every coordinate carrying a
    centre (they fix the weights, means and variances of the mixture), and log Z."""
    prob = ex.problem(K=K, sigma=0.5)
    logW, mean, var = ex.posterior(prob)
    W = np.exp(logW)
    n = 400_000
    xi = np.random.default_rng(5).standard_normal((n, K))
    lw = -ex.phi(prob, xi)
    w = np.exp(lw - lw.max())
    w /= w.sum()
    ess = 1.0 / np.sum(w ** 2)
    assert math.log(np.mean(np.exp(lw))) == pytest.approx(ex.log_evidence(prob), abs=4 / math.sqrt(ess))
    for k in range(4):
        m1 = W @ mean[:, k]
        m2 = W @ (mean[:, k] ** 2 + var[k])
        sd1 = math.sqrt(m2 - m1 ** 2)
        assert w @ xi[:, k] == pytest.approx(m1, abs=5 * sd1 / math.sqrt(ess))
        assert w @ xi[:, k] ** 2 == pytest.approx(m2, abs=5 * 2 * m2 / math.sqrt(ess))
    rest = xi[:, 4:]
    if rest.size:                                # coordinates without a centre: N(0, v_k)
        assert np.allclose(w @ rest ** 2, var[4:], rtol=10 / math.sqrt(ess))


def test_posterior_components_are_the_linear_gaussian_updates():
    """Weights normalised, symmetric modes +-cos(pi x) equally likely, variances below the prior's."""
    prob = ex.problem()
    logW, mean, var = ex.posterior(prob)
    assert logsumexp(logW) == pytest.approx(0.0, abs=1e-14)
    assert logW[0] == logW[1] and np.allclose(mean[0], -mean[1])
    assert np.all(var < 1) and np.all(var > 0)
    assert np.all(np.diff(logW[1:]) < 0)        # cos(pi x), cos(2 pi x), cos(3 pi x): decreasing prior mass
