"""Re-weighting and the choice of the next temperature.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Alg. 1 (re-weighting): with weights reset to 1/N at the start of the stage,
    w_hat_n = exp(-h Phi(v_n)) / N,   w_n = w_hat_n / sum_m w_hat_m.
App. C: ESS = (sum_n w_n^2)^{-1}; h is found by bisection so that ESS stays above
a fraction rho of N (the paper uses 0.6; it is a parameter here).

Conventions where the paper is silent: a fixed 64 bisection steps on (0, 1 - tau];
the step keeps ESS(lo) >= rho N and returns lo; if the whole remaining step
1 - tau already passes it is taken, so the last stage ends exactly at tau = 1.
A non-finite potential gives the particle weight zero.
The evidence increment is log Z_inc = log( (1/N) sum_n exp(-h Phi_n) ).
"""
import numpy as np
from scipy.special import logsumexp


def _clean(phi):
    phi = np.asarray(phi, dtype=np.float64)
    return np.where(np.isfinite(phi), phi, np.inf)


def log_ess(h, phi):
    """log ESS of the normalised weights exp(-h Phi) / sum."""
    lw = -h * _clean(phi)
    if h == 0.0:
        lw = np.where(np.isfinite(_clean(phi)), 0.0, -np.inf)
    w = np.exp(lw - logsumexp(lw))
    return -np.log(np.sum(w * w))


def choose_h(phi, tau, rho, steps=64):
    """(h, stalled) by the App. C bisection."""
    phi = _clean(phi)
    N = phi.size
    target = np.log(rho * N)
    rest = 1.0 - tau
    if log_ess(rest, phi) >= target:
        return rest, False
    lo, hi = 0.0, rest
    for _ in range(steps):
        mid = 0.5 * (lo + hi)
        if log_ess(mid, phi) >= target:
            lo = mid
        else:
            hi = mid
    return lo, lo == 0.0


def reweight(phi, h):
    """Normalised weights W and log Z_inc for increment h (Alg. 1 re-weighting)."""
    phi = _clean(phi)
    lw = -h * phi
    if h == 0.0:
        lw = np.where(np.isfinite(phi), 0.0, -np.inf)
    lse = logsumexp(lw)
    return np.exp(lw - lse), lse - np.log(phi.size)


def temper(phi, tau, rho):
    """One re-weighting step: (h, tau_new, W, log_Z_inc, stalled)."""
    h, stalled = choose_h(phi, tau, rho)
    W, lz = reweight(phi, h)
    tau_new = 1.0 if h == 1.0 - tau else tau + h
    return h, tau_new, W, lz, stalled
