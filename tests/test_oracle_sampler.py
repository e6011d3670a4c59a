"""Pins of the oracle's moves, tempering, resampling, SMC loop and gradient (CPU only)."""
import math

import numpy as np
import pytest
import scipy.stats
from scipy.special import logsumexp

import inputs
from oracle import linear, philox, quadrature, smc
from oracle.forward import observe, solve
from oracle.moves import (GM, gmpcn_moves, log_accept_gmpcn, log_accept_pcnl, log_q, log_ratio_gmpcn,
                          log_ratio_pcnl, pcn_gm, pcnl_moves, propose_gmpcn)
from oracle.problem import Problem, synthesize
from oracle.resample import systematic, systematic_at
from oracle.temper import choose_h, log_ess, reweight, temper


def _gm(M, K, kr, seed, spread=1.0):
    logw, mean, scale = inputs.mixture(M, kr, seed, spread)
    return GM(logw, mean, scale, np.arange(kr), K)


# ------------------------------------------------------------------ acceptance ratio

def test_pcn_special_case_is_potential_difference():
    """M = 1, m = 0, s = 1: a = min{1, exp(tau (Phi(u) - Phi(v)))} for any pair (Sec. 2.3, eq. (a in pCN))."""
    K = 40
    gm = pcn_gm(K, np.arange(10))
    x, v = inputs.particles(2, K, 1)
    for beta in (0.1, 0.5, 1.0):
        for tau in (0.0, 0.3, 1.0):
            lr = log_ratio_gmpcn(gm, beta, tau, x, 3.0, v, 2.0 + 4 * tau)
            assert lr == pytest.approx(tau * (3.0 - 2.0 - 4 * tau), abs=1e-11)


def test_drifted_pcn_cameron_martin():
    """M = 1, s = 1, mean m: log R = m . (xi - v) (drifted pCN, Sec. 2.3, eq. (pCNproposal))."""
    K, kr = 30, 12
    m = np.random.default_rng(2).standard_normal(kr)
    gm = GM([0.0], m[None], np.ones((1, kr)), np.arange(kr), K)
    for seed in (3, 4):
        x, v = inputs.particles(2, K, seed)
        lr = log_ratio_gmpcn(gm, 0.4, 0.0, x, 0.0, v, 0.0)
        assert lr == pytest.approx(float(m @ (x[:kr] - v[:kr])), abs=1e-11)
        # the ratio is antisymmetric in (xi, v)
        assert log_ratio_gmpcn(gm, 0.4, 0.0, v, 0.0, x, 0.0) == pytest.approx(-lr, abs=1e-11)


def test_beta_one_is_independence_sampler():
    """beta = 1: ratio [g(xi)/p0(xi)] / [g(v)/p0(v)] (Sec. 2.4, eq. (GMM beta=1)); densities from scipy."""
    K, kr, M = 16, 6, 3
    gm = _gm(M, K, kr, 4)
    m, s = gm.full()
    x, v = inputs.particles(2, K, 5, 0.7)

    def log_g(y):
        return logsumexp([gm.logw[j] + scipy.stats.multivariate_normal(m[j], np.diag(s[j])).logpdf(y)
                          for j in range(M)])

    def log_p0(y):
        return scipy.stats.multivariate_normal(np.zeros(K), np.eye(K)).logpdf(y)

    ref = (log_g(x) - log_p0(x)) - (log_g(v) - log_p0(v))
    assert log_ratio_gmpcn(gm, 1.0, 0.0, x, 0.0, v, 0.0) == pytest.approx(ref, abs=1e-10)


def test_log_q_against_scipy_mixture():
    K, kr, M = 12, 5, 4
    gm = _gm(M, K, kr, 6)
    m, s = gm.full()
    x, v = inputs.particles(2, K, 7)
    beta = 0.35
    gamma = math.sqrt(1 - beta ** 2)
    ref = logsumexp([gm.logw[j] + scipy.stats.multivariate_normal(gamma * x + (1 - gamma) * m[j],
                                                                   np.diag(beta ** 2 * s[j])).logpdf(v)
                     for j in range(M)])
    assert log_q(gm, beta, x, v) == pytest.approx(ref, abs=1e-10)


def test_component_choice_rule():
    gm = GM(np.log([0.2, 0.5, 0.3]), np.zeros((3, 1)), np.ones((3, 1)), [0], 4)
    z = np.zeros(4)
    picks = [propose_gmpcn(gm, 0.5, z, z, u)[1] for u in (0.0, 0.1999, 0.2, 0.69, 0.7, 0.99999)]
    assert picks == [0, 0, 1, 1, 2, 2]


# ------------------------------------------------------------------ chains

def test_pcn_zero_potential_accepts_everything_and_keeps_prior():
    """Check (c): with Phi = 0, plain pCN accepts every move and preserves mu_0."""
    K, N = 6, 3000
    xi0 = inputs.particles(N, K, 8)
    xi, phi, n_acc = gmpcn_moves(None, None, xi0, np.zeros(N), pcn_gm(K, np.arange(K)), 0.6, 1.0, 3, 11, 100,
                                 phi_fn=lambda x: 0.0)
    assert np.all(n_acc == 3)
    assert np.abs(xi.mean(0)).max() < 4 / math.sqrt(N)
    assert np.abs(xi.var(0) - 1).max() < 5 * math.sqrt(2 / N)


def test_gmpcn_zero_potential_keeps_prior():
    """With Phi = 0 the pCN-GM kernel is mu_0-invariant though it rejects some moves."""
    K, N = 4, 3000
    gm = _gm(3, K, 2, 9, spread=1.5)
    xi, _, n_acc = gmpcn_moves(None, None, inputs.particles(N, K, 10), np.zeros(N), gm, 0.8, 1.0, 4, 12, 200,
                               phi_fn=lambda x: 0.0)
    assert 0 < n_acc.mean() < 4
    assert np.abs(xi.mean(0)).max() < 4 / math.sqrt(N)
    assert np.abs(xi.var(0) - 1).max() < 6 * math.sqrt(2 / N)


def test_gmpcn_detailed_balance_1d_against_quadrature():
    """A bimodal 1D target: chain moments equal quadrature moments."""
    def phi1(x):
        return float(-np.log(np.exp(-0.5 * (x[0] - 1.6) ** 2 / 0.09) + 0.5 * np.exp(-0.5 * (x[0] + 1.2) ** 2 / 0.16)))
    mean_q, cov_q, _, _ = quadrature.moments(phi1, 1, pts=4001)
    N = 3000
    gm = GM(np.log([0.6, 0.4]), np.array([[1.5], [-1.1]]), np.array([[0.15], [0.2]]), [0], 1)
    xi0 = inputs.particles(N, 1, 13)
    ph0 = np.array([phi1(x) for x in xi0])
    xi, _, n_acc = gmpcn_moves(None, None, xi0, ph0, gm, 0.9, 1.0, 25, 14, 300, phi_fn=phi1)
    assert 0.2 < n_acc.mean() / 25 < 0.99
    se = math.sqrt(cov_q[0, 0] / N) * 3           # chains are not fully mixed from the prior start
    assert abs(xi.mean() - mean_q[0]) < 4 * se
    assert abs(xi.var() - cov_q[0, 0]) < 0.08 * cov_q[0, 0]


def test_pcnl_reduces_to_pcn_and_keeps_gaussian_posterior():
    """g = 0 gives the pCN ratio; a quadratic Phi keeps the closed-form posterior."""
    K = 3
    x, v = inputs.particles(2, K, 15)
    lr = log_ratio_pcnl(0.3, 0.7, x, 2.0, np.zeros(K), v, 1.0, np.zeros(K))
    assert lr == pytest.approx(0.7 * (2.0 - 1.0), abs=1e-12)
    H = np.array([[1.0, 0.5, -0.2], [0.0, 1.3, 0.4]])
    d = np.array([0.7, -0.4])
    sig = 0.5
    m_p, S_p = linear.posterior(H, d, sig)

    def vg(xi):
        r = H @ xi - d
        return float(r @ r / (2 * sig ** 2)), H.T @ r / sig ** 2
    N = 3000
    xi0 = m_p + inputs.particles(N, K, 16) @ np.linalg.cholesky(S_p).T
    ph, gr = zip(*[vg(x) for x in xi0])
    xi, _, _, n_acc = pcnl_moves(0.5, 1.0, xi0, np.array(ph), np.array(gr), 6, 17, 400, vg)
    assert 0.3 < n_acc.mean() / 6 < 1.0
    assert np.abs(xi.mean(0) - m_p).max() < 5 * math.sqrt(np.diag(S_p).max() / N)
    assert np.abs(np.cov(xi.T) - S_p).max() < 0.1 * np.abs(S_p).max()


def test_pcnl_ratio_matches_published_form():
    """Cotter, Roberts, Stuart, White (Stat. Sci. 2013), pCN-Langevin with C = I:
    log a = rho(u, v) - rho(v, u),  rho(u, v) = Phi(u) + <v - u, g(u)>/2 + delta/4 <u + v, g(u)>
    + delta/4 |g(u)|^2, with delta = 2 (1 - gamma) / (1 + gamma) and the tempered Phi, g."""
    K, tau = 7, 0.6
    rng = np.random.default_rng(24)
    for beta in (0.1, 0.45, 0.9):
        gamma = math.sqrt(1 - beta ** 2)
        delta = 2 * (1 - gamma) / (1 + gamma)
        x, v, gx, gv = rng.standard_normal((4, K))

        def rho(u, w, pu, gu):
            g = tau * gu
            return tau * pu + 0.5 * (w - u) @ g + delta / 4 * (u + w) @ g + delta / 4 * g @ g
        ref = rho(x, v, 1.1, gx) - rho(v, x, 0.2, gv)
        assert log_ratio_pcnl(beta, tau, x, 1.1, gx, v, 0.2, gv) == pytest.approx(ref, abs=1e-12)


# ------------------------------------------------------------------ tempering

def test_ess_bounds_and_monotone():
    phi = inputs.potentials(500, 18)
    hs = np.linspace(0, 0.2, 41)
    ess = np.exp([log_ess(h, phi) for h in hs])
    assert ess[0] == pytest.approx(500, rel=1e-12)
    assert np.all(ess >= 1 - 1e-9) and np.all(ess <= 500 + 1e-9)
    assert np.all(np.diff(ess) <= 1e-9)


def test_bisection_hits_threshold():
    phi = inputs.potentials(1000, 19)
    h, stalled = choose_h(phi, 0.0, 0.5)
    assert not stalled and 0 < h < 1
    assert log_ess(h, phi) >= math.log(500)
    assert log_ess(h * (1 + 1e-9), phi) < math.log(500)
    W, lz = reweight(phi, h)
    assert W.sum() == pytest.approx(1.0, rel=1e-14)
    assert 1.0 / np.sum(W ** 2) >= 500 * (1 - 1e-12)


def test_equal_potentials_finish_in_one_stage():
    h, tau, W, lz, stalled = temper(np.full(64, 3.0), 0.25, 0.5)
    assert h == 0.75 and tau == 1.0 and not stalled
    assert np.allclose(W, 1 / 64) and lz == pytest.approx(-0.75 * 3.0, abs=1e-14)


def test_dominant_weight_stalls_and_nonfinite_gets_zero_weight():
    phi = np.full(32, 1e308)
    phi[3] = 0.0
    h, stalled = choose_h(phi, 0.0, 0.5)
    assert stalled and h == 0.0
    phi2 = inputs.potentials(32, 20)
    phi2[5] = np.nan
    phi2[6] = np.inf
    h, tau, W, lz, stalled = temper(phi2, 0.0, 0.5)
    assert W[5] == 0.0 and W[6] == 0.0 and np.isfinite(lz) and not stalled


# ------------------------------------------------------------------ resampling

def _brute(W, u53):
    N = len(W)
    q = [int(math.floor(w * 2 ** 53)) for w in W]
    C = np.cumsum(np.array(q, dtype=object))
    Q = C[-1]
    out = []
    for i in range(N):
        p = ((i * 2 ** 53 + u53) * Q) // (N * 2 ** 53)
        out.append(next(n for n in range(N) if C[n] > p))
    return out


@pytest.mark.parametrize("kind", ["dirichlet", "sparse", "one", "uniform"])
def test_resampling_against_brute_force(kind):
    for N, seed in ((1, 1), (7, 2), (200, 3)):
        W = inputs.weights(N, seed, kind)
        u = inputs.u53(seed)
        assert systematic(W, u) == _brute(W, u)


@pytest.mark.parametrize("kind", ["dirichlet", "sparse", "one"])
def test_resampling_selected_outputs_against_brute_force(kind):
    """systematic_at, the per-output form used on batches too large to list, against the brute
    force on every output and against systematic on a subset."""
    for N, seed in ((1, 4), (9, 5), (300, 6)):
        W = inputs.weights(N, seed, kind)
        u = inputs.u53(seed + 10)
        assert systematic_at(W, u, range(N)) == _brute(W, u)
        sub = [0, N // 3, N - 1]
        full = systematic(W, u)
        assert systematic_at(W, u, sub) == [full[i] for i in sub]


def test_resampling_counts_and_order():
    N = 500
    W = inputs.weights(N, 21)
    idx = systematic(W, inputs.u53(21))
    assert all(a <= b for a, b in zip(idx, idx[1:]))
    counts = np.bincount(idx, minlength=N)
    q = np.floor(W * 2 ** 53)
    Wt = q / q.sum()
    assert np.all(counts >= np.floor(N * Wt) - 0) and np.all(counts <= np.ceil(N * Wt))
    # float systematic resampling on the same uniform agrees away from ties
    pts = (np.arange(N) + inputs.u53(21) / 2 ** 53) / N
    ref = np.searchsorted(np.cumsum(Wt), pts, side="right")
    assert np.mean(ref == np.array(idx)) > 0.99
    assert systematic(inputs.weights(64, 0, "uniform"), inputs.u53(4)) == list(range(64))


# ------------------------------------------------------------------ whole runs

def _tiny_1d(obs, kl=2, n=16, seed_truth=0, mirror=False):
    d = dict(name="tiny", dim=1, grids=[n], kl_per_axis=kl, kr=kl, obs_den=n, obs=[[o] for o in obs],
             y=[0.0] * len(obs), sigma=1.0)
    p = Problem(d)
    xt = np.zeros(kl)
    xt[:2] = [0.8, 1.6]
    G = observe(p, solve(p, synthesize(p, xt, 64), 64), 64)
    sigma = 0.05 * np.abs(G).max()
    y = G + sigma * np.random.default_rng(1).standard_normal(G.size)
    if mirror:
        half = len(obs) // 2
        y[:half] = y[half:] = 0.5 * (G[:half] + G[half:]) + sigma * np.random.default_rng(2).standard_normal(half)
    p.y, p.sigma = y, sigma
    return p


def test_linear_gaussian_posterior_check_b():
    """Check (b): SMC on F(xi) = H xi approaches the closed-form posterior and evidence."""
    p = _tiny_1d([3, 8, 13], kl=4)
    from oracle.problem import basis_matrix
    B = basis_matrix(1, 4, 16)
    H = B[[3, 8, 13]] * p.sqrt_lam[None, :] * 0.0 + B[[3, 8, 13]]       # point values of u
    H = H * p.sqrt_lam[None, :]
    sig = 0.05
    d = H @ np.array([0.8, 1.6, -0.5, 0.3]) + sig * np.array([0.3, -1.1, 0.6])
    m_p, S_p = linear.posterior(H, d, sig)
    f = linear.phi_fn(H, d, sig)
    N = 2000
    out = smc.run(p, 16, N, M=2, n_moves=5, rho=0.5, beta0=0.3, seed=3, phi_fn=f, kr=4)
    xi = out["xi"]
    sd = np.sqrt(np.diag(S_p))
    assert np.all(np.abs(xi.mean(0) - m_p) < 6 * sd / math.sqrt(N / 3))
    assert np.all(np.abs(xi.std(0) / sd - 1) < 0.15)
    assert out["log_Z"] == pytest.approx(linear.log_evidence(H, d, sig), abs=0.15)
    assert out["taus"][-1] == 1.0


def test_bimodal_quadrature_check_d():
    """Check (d): mirrored observations make the 2-mode 1D posterior symmetric in xi_2."""
    p = _tiny_1d([4, 6, 12, 10], kl=2, mirror=True)
    from oracle.forward import phi
    f = lambda x: phi(p, x, 16)
    assert abs(f(np.array([0.4, 1.3])) - f(np.array([0.4, -1.3]))) < 1e-9 * f(np.array([0.4, 1.3]))
    mean_q, cov_q, w, grid = quadrature.moments(f, 2, pts=241)
    mass_pos = w[grid[:, 1] > 0].sum()
    assert abs(mean_q[1]) < 1e-6 and abs(mass_pos - 0.5) < 0.02
    N = 2000
    out = smc.run(p, 16, N, M=2, n_moves=6, rho=0.5, beta0=0.5, seed=4, phi_fn=f, kr=2)
    xi = out["xi"]
    assert abs(np.mean(xi[:, 1] > 0) - 0.5) < 0.08
    assert abs(xi[:, 0].mean() - mean_q[0]) < 5 * math.sqrt(cov_q[0, 0] / (N / 4))
    assert abs(np.var(xi[:, 1]) / cov_q[1, 1] - 1) < 0.15


# ------------------------------------------------------------------ gradient

@pytest.mark.parametrize("n", [16, 32])
def test_adjoint_gradient_finite_differences(problems, n):
    """Central differences (h = 1e-6, FP64) on seeded unit directions, and the Taylor remainder."""
    from oracle.adjoint import value_and_grad
    from oracle.forward import phi
    p = problems["t2"]
    xi = inputs.particles(1, p.K, 22)[0]
    f0, g = value_and_grad(p, xi, n)
    assert f0 == pytest.approx(phi(p, xi, n), rel=1e-12)
    dirs = inputs.particles(6, p.K, 23)
    for d in dirs:
        d /= np.linalg.norm(d)
        fd = (phi(p, xi + 1e-6 * d, n) - phi(p, xi - 1e-6 * d, n)) / 2e-6
        assert fd == pytest.approx(g @ d, rel=2e-6, abs=1e-6 * np.linalg.norm(g))
    d = dirs[0]
    r = [abs(phi(p, xi + e * d, n) - f0 - e * (g @ d)) for e in (1e-2, 5e-3)]
    assert 3.0 < r[0] / r[1] < 5.0
