"""Metropolis-Hastings moves in whitened KL coordinates.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Target.  At cumulative inverse temperature tau the target is
    d mu_tau / d mu_0 (u) ∝ exp(-tau Phi(u))          (Sec. 2.1, tempered measures)
which in whitened coordinates has density ∝ exp(-tau Phi(xi) - |xi|^2 / 2).

pCN-GM proposal (Sec. 2.3, eq. (pCN-GM proposal), read component-wise as in the
theorem on mu_0(du)Q(u,dv), whose joint components have means [0, (1-gamma) m_j]):
    Q(xi, dv) = sum_j w_j N(gamma xi + (1 - gamma) m_j, beta^2 C_j),  gamma = sqrt(1 - beta^2),
and in whitened coordinates C_j = diag(s_j) with s_ji = lambda_ji / lambda_i; the
mixture moves only the active modes (elsewhere m = 0, s = 1).  M = 1 with m = 0
is the plain pCN proposal (Sec. 2.3, eq. (pCNproposal)).

Acceptance (Sec. 2.3, eqs. (auv of pCN-GMM) and (auv of pCN-GMM2)):
    a(xi, v) = min{1, rho(dv) Q(v, dxi) / (rho(dxi) Q(xi, dv))}.
Here it is evaluated in the finite K-dimensional coordinates as the plain ratio of
densities: the target density times the mixture proposal density, each mixture
density a sum over components of full K-dimensional Gaussian densities.

pCN-Langevin.  The paper names it (Sec. 2.4) and gives the Langevin equation it
discretises (App. B); with the same Crank-Nicolson step as App. B and the drift
of the tempered potential kept explicit, the proposal in whitened coordinates is
    v = gamma xi - (1 - gamma) tau g(xi) + beta z,    g = grad_xi Phi,
(gamma = (2-delta)/(2+delta), beta = sqrt(8 delta)/(2+delta), so gamma^2 + beta^2 = 1),
and its acceptance is again the plain density ratio.
"""
import numpy as np
from scipy.special import logsumexp

from . import philox
from .forward import phi as phi_of


class GM:
    """Mixture parameters over the active modes (whitened)."""

    def __init__(self, logw, mean, scale, active, K):
        self.logw = np.asarray(logw, dtype=np.float64)          # (M,)
        self.mean = np.asarray(mean, dtype=np.float64)          # (M, Kr)
        self.scale = np.asarray(scale, dtype=np.float64)        # (M, Kr), s = lambda_j / lambda
        self.active = np.asarray(active, dtype=np.int64)        # (Kr,)
        self.K = int(K)

    @property
    def M(self):
        return self.logw.size

    def full(self):
        """Means and scales expanded to all K modes."""
        m = np.zeros((self.M, self.K))
        s = np.ones((self.M, self.K))
        m[:, self.active] = self.mean
        s[:, self.active] = self.scale
        return m, s


def pcn_gm(K, active):
    """The single-component, zero-mean, unit-scale mixture: plain pCN."""
    active = np.asarray(active, dtype=np.int64)
    return GM([0.0], np.zeros((1, active.size)), np.ones((1, active.size)), active, K)


def log_gauss(x, mean, var):
    """log N(x; mean, diag(var)) summed over the last axis."""
    r = x - mean
    return -0.5 * np.sum(r * r / var + np.log(2.0 * np.pi * var), axis=-1)


def log_q(gm, beta, frm, to):
    """log density of Q(frm, d to) for the pCN-GM proposal."""
    gamma = np.sqrt(1.0 - beta ** 2)
    m, s = gm.full()
    terms = [gm.logw[j] + log_gauss(to, gamma * frm + (1.0 - gamma) * m[j], beta ** 2 * s[j])
             for j in range(gm.M)]
    return logsumexp(np.array(terms), axis=0)


def log_target(xi, phi, tau):
    return -tau * phi - 0.5 * np.sum(np.asarray(xi) ** 2, axis=-1)


def log_ratio_gmpcn(gm, beta, tau, xi, phi_xi, v, phi_v):
    """log of rho(dv) Q(v, dxi) / (rho(dxi) Q(xi, dv)) by the plain density ratio."""
    if not np.isfinite(phi_v):
        return -np.inf
    num = log_target(v, phi_v, tau) + log_q(gm, beta, v, xi)
    den = log_target(xi, phi_xi, tau) + log_q(gm, beta, xi, v)
    return num - den


def log_accept_gmpcn(gm, beta, tau, xi, phi_xi, v, phi_v):
    """log a(xi, v) = min(0, log ratio)."""
    return min(0.0, log_ratio_gmpcn(gm, beta, tau, xi, phi_xi, v, phi_v))


def propose_gmpcn(gm, beta, xi, z, u_comp):
    """Component j = min{j : sum_{i<=j} w_i > U_comp}, then the proposal."""
    gamma = np.sqrt(1.0 - beta ** 2)
    cum = np.cumsum(np.exp(gm.logw))
    j = int(np.searchsorted(cum, u_comp, side="right"))
    j = min(j, gm.M - 1)
    m, s = gm.full()
    return gamma * xi + (1.0 - gamma) * m[j] + beta * np.sqrt(s[j]) * z, j


def gm_draw(gm, seed, ctr, ids):
    """Independent draws from the mixture, the mutation of SMC-GM (Alg. 3): the pCN-GM
    proposal with beta = 1 (Sec. 2.4, eq. (GMM beta=1)), where gamma = 0 removes the
    current state.  Component j = min{j : sum_{i<=j} w_i > U_comp} (U_comp of block
    UNIFORM_BLOCK), then v = m_j + sqrt(s_j) z on the active modes and v = z elsewhere,
    with z the particle's normals at counter ctr."""
    ids = np.asarray(ids, dtype=np.int64)
    z = philox.normals(seed, ctr, ids, gm.K)
    uc, _ = philox.move_uniforms(seed, ctr, ids)
    m, s = gm.full()
    cum = np.cumsum(np.exp(gm.logw))
    v = np.empty_like(z)
    for p in range(ids.size):
        j = min(int(np.searchsorted(cum, uc[p], side="right")), gm.M - 1)
        v[p] = m[j] + np.sqrt(s[j]) * z[p]
    return v


def gmpcn_moves(prob, n, xi, phi, gm, beta, tau, n_moves, seed, ctr, phi_fn=None, ids=None):
    """n_moves pCN-GM steps (Alg. 2) for every particle; returns (xi, phi, n_acc).

    Random numbers follow the layout in `philox`; particle ids are row numbers unless
    `ids` gives them.  phi_fn(xi) -> Phi overrides the PDE potential (used by tests with
    closed forms).
    """
    xi = np.array(xi, dtype=np.float64, copy=True)
    phi = np.array(phi, dtype=np.float64, copy=True)
    N, K = xi.shape
    ids = np.arange(N) if ids is None else np.asarray(ids)
    n_acc = np.zeros(N, dtype=np.int64)
    f = phi_fn if phi_fn is not None else (lambda x: phi_of(prob, x, n))
    for mv in range(n_moves):
        c = ctr + mv
        z = philox.normals(seed, c, ids, K)
        uc, ua = philox.move_uniforms(seed, c, ids)
        for p in range(N):
            v, _ = propose_gmpcn(gm, beta, xi[p], z[p], uc[p])
            pv = f(v)
            la = log_accept_gmpcn(gm, beta, tau, xi[p], phi[p], v, pv)
            if np.log(ua[p]) < la:
                xi[p], phi[p] = v, pv
                n_acc[p] += 1
    return xi, phi, n_acc


# ---------------------------------------------------------------- pCN-Langevin

def pcnl_mean(beta, tau, xi, g):
    gamma = np.sqrt(1.0 - beta ** 2)
    return gamma * xi - (1.0 - gamma) * tau * g


def log_ratio_pcnl(beta, tau, xi, phi_xi, g_xi, v, phi_v, g_v):
    """log MH ratio for the pCN-Langevin proposal by the plain density ratio."""
    if not np.isfinite(phi_v):
        return -np.inf
    var = np.full(np.size(xi), beta ** 2)
    num = log_target(v, phi_v, tau) + log_gauss(xi, pcnl_mean(beta, tau, v, g_v), var)
    den = log_target(xi, phi_xi, tau) + log_gauss(v, pcnl_mean(beta, tau, xi, g_xi), var)
    return num - den


def log_accept_pcnl(beta, tau, xi, phi_xi, g_xi, v, phi_v, g_v):
    return min(0.0, log_ratio_pcnl(beta, tau, xi, phi_xi, g_xi, v, phi_v, g_v))


def pcnl_moves(beta, tau, xi, phi, grad, n_moves, seed, ctr, value_and_grad, ids=None):
    """pCN-Langevin steps; value_and_grad(xi) -> (Phi, grad Phi).  Particle ids (the random
    streams) are row numbers unless `ids` gives them."""
    xi = np.array(xi, dtype=np.float64, copy=True)
    phi = np.array(phi, dtype=np.float64, copy=True)
    grad = np.array(grad, dtype=np.float64, copy=True)
    N, K = xi.shape
    ids = np.arange(N) if ids is None else np.asarray(ids)
    n_acc = np.zeros(N, dtype=np.int64)
    for mv in range(n_moves):
        c = ctr + mv
        z = philox.normals(seed, c, ids, K)
        _, ua = philox.move_uniforms(seed, c, ids)
        for p in range(N):
            v = pcnl_mean(beta, tau, xi[p], grad[p]) + beta * z[p]
            pv, gv = value_and_grad(v)
            la = log_accept_pcnl(beta, tau, xi[p], phi[p], grad[p], v, pv, gv)
            if np.log(ua[p]) < la:
                xi[p], phi[p], grad[p] = v, pv, gv
                n_acc[p] += 1
    return xi, phi, grad, n_acc


def prior_sample(K, N, seed, ctr):
    """xi ~ N(0, I): Alg. 1 draws the initial particles from mu_0."""
    return philox.normals(seed, ctr, np.arange(N), K)
