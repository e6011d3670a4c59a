"""Example 1 of the paper (Sec. 3.1): a multi-modal likelihood on L^2(0, 1) with no PDE.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Prior mu_0 = N(0, C), C = (I - alpha Delta)^{-2} (alpha = 0.01 in the paper), taken with the
Neumann eigenpairs of the Laplacian on (0, 1): phi_0 = 1, phi_k = sqrt(2) cos(k pi x),
lambda_k = (1 + alpha k^2 pi^2)^{-2}, k = 0 .. K-1, so u = sum_k sqrt(lambda_k) xi_k phi_k.

Likelihood (eq. (example1phi)): exp(-Phi(u)) = sum_i exp(-|u - f_i|^2 / (2 sigma^2)) with
f_1 = cos(pi x), f_2 = -cos(pi x), f_3 = cos(2 pi x), f_4 = cos(3 pi x).  Each f_i lies in the
span of the first four modes, with coefficient c_ik = <f_i, phi_k> = +-1/sqrt(2) at one k, so
by Parseval |u - f_i|^2 = sum_k (sqrt(lambda_k) xi_k - c_ik)^2 on the K-mode span.  The paper
does not give sigma; 0.1 is used.

Posterior.  Each term is a linear-Gaussian update, diagonal in xi: with a_k = sqrt(lambda_k),
    component i:  N(m_i, diag(v)),  v_k = 1 / (1 + lambda_k / sigma^2),
                  m_ik = v_k a_k c_ik / sigma^2,
    weight        W_i ∝ Z_i,  Z_i = prod_k sqrt(v_k) exp(-c_ik^2 / (2 (sigma^2 + lambda_k))),
and Z = int exp(-Phi) d mu_0 = sum_i Z_i.
"""
import numpy as np
from scipy.special import logsumexp

CENTRES = ((1, 1.0), (1, -1.0), (2, 1.0), (3, 1.0))   # (k, sign) of f_i = sign * cos(k pi x)


def problem(K=64, alpha=0.01, sigma=0.1):
    k = np.arange(K)
    lam = (1.0 + alpha * (k * np.pi) ** 2) ** -2.0
    c = np.zeros((len(CENTRES), K))
    for i, (kk, sg) in enumerate(CENTRES):
        c[i, kk] = sg / np.sqrt(2.0)
    return dict(K=K, alpha=alpha, sigma=sigma, lam=lam, sqrt_lam=np.sqrt(lam), c=c)


def phi(prob, xi):
    """Phi(xi) = -log sum_i exp(-sum_k (sqrt(lambda_k) xi_k - c_ik)^2 / (2 sigma^2))."""
    a = prob["sqrt_lam"] * np.asarray(xi, dtype=np.float64)
    d2 = np.sum((a[..., None, :] - prob["c"]) ** 2, axis=-1)
    return -logsumexp(-d2 / (2.0 * prob["sigma"] ** 2), axis=-1)


def posterior(prob):
    """(logW[4], mean[4][K], var[K]) of the exact mixture posterior in xi."""
    lam, c, s2 = prob["lam"], prob["c"], prob["sigma"] ** 2
    v = 1.0 / (1.0 + lam / s2)
    mean = v * np.sqrt(lam) * c / s2
    logz = 0.5 * np.sum(np.log(v)) - np.sum(c ** 2 / (2.0 * (s2 + lam)), axis=1)
    return logz - logsumexp(logz), mean, v


def log_evidence(prob):
    lam, c, s2 = prob["lam"], prob["c"], prob["sigma"] ** 2
    v = 1.0 / (1.0 + lam / s2)
    logz = 0.5 * np.sum(np.log(v)) - np.sum(c ** 2 / (2.0 * (s2 + lam)), axis=1)
    return float(logsumexp(logz))


def nearest_mode(prob, xi):
    """Index of the posterior component whose mean is nearest (in the whitened metric of its
    covariance) to each row of xi: the mode a particle belongs to."""
    _, mean, v = posterior(prob)
    d = np.sum((np.asarray(xi)[:, None, :] - mean[None]) ** 2 / v, axis=-1)
    return np.argmin(d, axis=1)
