"""Closed-form posterior for a linear forward map (test target).

TEST INFRASTRUCTURE ONLY (see the package docstring).

With F(xi) = H xi, prior xi ~ N(0, I) and Phi = |H xi - d|^2 / (2 sigma^2), the
posterior of Sec. 2.1 (eq. (Bayes)) is Gaussian:
    Sigma_post = (I + H^T H / sigma^2)^{-1},   m_post = Sigma_post H^T d / sigma^2,
and the normalising constant Z = int exp(-Phi) d mu_0 is
    log Z = (N_d / 2) log(2 pi sigma^2) + log N(d; 0, H H^T + sigma^2 I).
"""
import numpy as np


def posterior(H, d, sigma):
    H = np.asarray(H, dtype=np.float64)
    K = H.shape[1]
    S = np.linalg.inv(np.eye(K) + H.T @ H / sigma ** 2)
    m = S @ H.T @ np.asarray(d) / sigma ** 2
    return m, S


def log_evidence(H, d, sigma):
    H = np.asarray(H, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    Nd = d.size
    C = H @ H.T + sigma ** 2 * np.eye(Nd)
    sign, logdet = np.linalg.slogdet(C)
    quad = d @ np.linalg.solve(C, d)
    log_n = -0.5 * (quad + logdet + Nd * np.log(2 * np.pi))
    return 0.5 * Nd * np.log(2 * np.pi * sigma ** 2) + log_n


def phi_fn(H, d, sigma):
    H = np.asarray(H, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    return lambda xi: float(np.sum((H @ xi - d) ** 2) / (2 * sigma ** 2))
