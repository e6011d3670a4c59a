"""SMC-pCN-GM driver: the loop of Alg. 1 with the pCN-GM mutation, over the C ABI.

Per stage, in the order S^N P_{j+1} L_{j+1} of Sec. 2.2 (eq. (decidemuJN)):
  smc_temper    next increment h by ESS bisection (App. C), weights, log Z increment
  smc_resample  systematic resampling of the re-weighted cloud (Alg. 1)
  smc_gather    copy the selected rows
  mixture fit   Gaussian mixture over the active modes (stage input, see fit_mixture)
  smc_gmpcn_move  n_moves pCN-GM steps at the new temperature (Alg. 2)
  step size     beta <- 2 beta if acceptance > 0.3, beta / 2 if < 0.15 (App. C), beta <= 1
The loop ends when the cumulative temperature reaches 1.
"""
import numpy as np
import torch

from . import smc

STAGE_STRIDE = 1 << 20


def fit_mixture(X, M, seed, iters=50, var_floor=1e-3):
    """Diagonal Gaussian mixture by EM on rows of X (host, float64).

    The paper fits its mixture with the estimator of its reference [Feng2018], which it does
    not describe; this stand-in seeds the means by k-means++ and runs a fixed number of EM
    steps with a variance floor.  Returns (logw[M], mean[M][D], var[M][D]).
    """
    X = np.asarray(X, dtype=np.float64)
    N, D = X.shape
    rng = np.random.default_rng(seed)
    centers = [X[rng.integers(N)]]
    for _ in range(1, M):
        d2 = np.min(np.stack([((X - c) ** 2).sum(1) for c in centers]), axis=0)
        tot = d2.sum()
        centers.append(X[rng.choice(N, p=d2 / tot)] if tot > 0 else X[rng.integers(N)])
    mean = np.array(centers)
    var = np.tile(np.maximum(X.var(0), var_floor), (M, 1))
    logw = np.full(M, -np.log(M))
    for _ in range(iters):
        ll = logw[None, :] - 0.5 * (((X[:, None, :] - mean[None]) ** 2) / var[None] +
                                    np.log(2 * np.pi * var[None])).sum(-1)
        mx = ll.max(1, keepdims=True)
        R = np.exp(ll - mx)
        R /= R.sum(1, keepdims=True)
        Nk = R.sum(0) + 1e-300
        logw = np.log(Nk / N)
        mean = (R.T @ X) / Nk[:, None]
        var = np.maximum((R.T @ (X * X)) / Nk[:, None] - mean ** 2, var_floor)
    logw -= np.log(np.exp(logw - logw.max()).sum()) + logw.max()
    return logw, mean, var


def pcn_mixture(kr, device):
    """The single zero-mean unit-scale component: plain pCN."""
    return (torch.zeros(1, dtype=torch.float64, device=device),
            torch.zeros(1, kr, dtype=torch.float64, device=device),
            torch.ones(1, kr, dtype=torch.float64, device=device))


class SMCSampler:
    def __init__(self, problem, N, M, n_moves, ess_frac=0.5, beta0=0.2, prec=smc.SMC_FP32_REFINE, seed=0,
                 device="cuda"):
        self.p, self.N, self.M, self.n_moves = problem, int(N), int(M), int(n_moves)
        self.ess_frac, self.beta, self.prec, self.seed = ess_frac, float(beta0), prec, int(seed)
        dev = torch.device(device)
        K = problem.K
        f64 = dict(dtype=torch.float64, device=dev)
        self.xi = torch.empty(N, K, **f64)
        self.xi2 = torch.empty(N, K, **f64)
        self.phi = torch.empty(N, **f64)
        self.phi2 = torch.empty(N, **f64)
        self.G = torch.empty(N, problem.n_obs, **f64)
        self.W = torch.empty(N, **f64)
        self.tau = torch.zeros(1, **f64)
        self.tau_new = torch.zeros(1, **f64)
        self.h = torch.zeros(1, **f64)
        self.log_z = torch.zeros(1, **f64)
        self.idx = torch.empty(N, dtype=torch.int32, device=dev)
        self.n_acc = torch.empty(N, dtype=torch.int32, device=dev)
        self.flags = torch.zeros(1, dtype=torch.int32, device=dev)
        self.active = torch.tensor(problem.active, dtype=torch.long, device=dev)
        self.dev = dev
        self.stage = 0
        self.log_Z = 0.0
        self.history = []

    def initialise(self):
        p, N = self.p, self.N
        smc.smc_prior_sample(p, N, self.seed, 0, self.xi)
        smc.smc_forward_batch(p, N, self.xi, None, self.prec, self.G)
        smc.smc_potential(p, N, self.G, self.phi)

    def mixture(self):
        if self.M == 1:
            return pcn_mixture(self.p.kr, self.dev)
        X = self.xi.cpu().numpy()[:, self.p.active]
        logw, mean, var = fit_mixture(X, self.M, self.seed + self.stage)
        t = lambda a: torch.tensor(a, dtype=torch.float64, device=self.dev).contiguous()
        return t(logw), t(mean), t(var)

    def step(self):
        """One stage: temper, resample, gather, mixture, moves, step-size rule."""
        p, N = self.p, self.N
        self.stage += 1
        base = self.stage * STAGE_STRIDE
        smc.smc_temper(N, self.phi, self.tau, self.ess_frac, self.h, self.tau_new, self.W, self.log_z, self.flags)
        u53 = int(np.random.default_rng([self.seed, self.stage]).integers(0, 1 << 53))
        smc.smc_resample(N, self.W, u53, self.idx, self.flags)
        smc.smc_gather(N, p.K, self.idx, self.xi, self.phi, self.xi2, self.phi2)
        self.xi, self.xi2 = self.xi2, self.xi
        self.phi, self.phi2 = self.phi2, self.phi
        self.tau.copy_(self.tau_new)
        tau = float(self.tau.item())
        gm = self.mixture()
        smc.smc_gmpcn_move(p, N, gm, self.beta, tau, self.n_moves, self.seed, base, None, self.prec, self.xi,
                           self.phi, self.n_acc)
        rate = float(self.n_acc.cpu().numpy().sum()) / (N * max(1, self.n_moves))
        self.log_Z += float(self.log_z.item())
        self.history.append(dict(stage=self.stage, tau=tau, h=float(self.h.item()), beta=self.beta, rate=rate))
        if rate > 0.3:
            self.beta = min(1.0, 2.0 * self.beta)
        elif rate < 0.15:
            self.beta *= 0.5
        return tau

    def run(self, max_stages=500):
        self.initialise()
        for _ in range(max_stages):
            if self.step() >= 1.0:
                break
        if int(self.flags.item()) & smc.FLAG_STALL:
            raise RuntimeError("temperature bisection stalled")
        return dict(xi=self.xi, phi=self.phi, log_Z=self.log_Z, history=self.history)
