"""The paper's Example 1 (Sec. 3.1) on the GPU: a four-term L^2 likelihood with no PDE, whose
posterior is an exact four-component Gaussian mixture (oracle/example1.py).

  * smc_phi_batch against the oracle's potential (1e-12 relative);
  * pCN-GM moves with the same random numbers as the oracle's: identical accept counts,
    states and potentials to 1e-10;
  * whole SMC-GM (Alg. 3) and SMC-pCN-GM (Alg. 1 + 2) runs replayed against the oracle's runs
    from the same seed (every random number comes from the same Philox layout): temperatures,
    step sizes, accept rates, log Z and final states to rounding;
  * an SMC-pCN-GM run against the exact posterior: the mass of each mode, the mean and spread of
    each mode's own coordinate, and log Z, within Monte Carlo error (effective size N / 4).
    SMC-GM is not held to the exact posterior: Alg. 3 re-weights draws from the fitted mixture
    without correcting for the fit, and on this 64-mode problem its mode masses drift from
    run to run (the oracle's own runs show the same).
"""
import math
import sys

import numpy as np
import pytest
import torch

import inputs
from oracle import example1 as ex
from oracle.moves import GM, gmpcn_moves

pytestmark = pytest.mark.gpu
DEV = "cuda"
K = 64


def banner(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def t(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


@pytest.fixture(scope="module", autouse=True)
def _lib():
    from paper_2503_16028_amd import smc
    smc.lib()
    assert torch.cuda.is_available()


def make(N, sigma=0.1, kr=K):
    from paper_2503_16028_amd import smc
    prob = ex.problem(K=K, sigma=sigma)
    return prob, smc.L2MixProblem(K, kr, prob["alpha"], prob["c"], sigma, N)


def test_potential_parity():
    from paper_2503_16028_amd import smc
    banner("example1 potential")
    N = 1000
    prob, p = make(N)
    _, mean, var = ex.posterior(prob)
    xi = inputs.particles(N, K, 3)
    xi[:400] = mean[np.arange(400) % 4] + np.sqrt(var) * xi[:400]      # near every mode, and prior-like
    phi = torch.empty(N, dtype=torch.float64, device=DEV)
    iters = torch.full((N,), -7, dtype=torch.int32, device=DEV)
    smc.smc_phi_batch(p, N, t(xi), None, smc.SMC_FP64, phi, iters)
    ref = ex.phi(prob, xi)
    assert np.abs(phi.cpu().numpy() / ref - 1).max() <= 1e-12
    assert (iters.cpu().numpy() == 0).all()
    with pytest.raises(smc.SMCError):           # no observation operator, no grid
        smc.smc_forward_batch(p, N, t(xi), None, smc.SMC_FP64, torch.empty(N, 1, dtype=torch.float64, device=DEV))


def test_moves_parity():
    from paper_2503_16028_amd import smc
    banner("example1 pcn-gm moves")
    N, M, beta, tau, n_moves = 64, 4, 0.5, 0.7, 3
    prob, p = make(N)
    xi0 = inputs.particles(N, K, 5, 0.9)
    phi0 = ex.phi(prob, xi0)
    logw, mean, scale = inputs.mixture(M, K, 6, spread=0.5)
    gm = GM(logw, mean, scale, np.arange(K), K)
    xi, phi = t(xi0), t(phi0)
    acc = torch.empty(N, dtype=torch.int32, device=DEV)
    smc.smc_gmpcn_move(p, N, (t(logw), t(mean), t(scale)), beta, tau, n_moves, 9, 40, None, smc.SMC_FP64, xi, phi,
                       acc)
    rx, rphi, racc = gmpcn_moves(None, 0, xi0, phi0, gm, beta, tau, n_moves, 9, 40,
                                 phi_fn=lambda x: ex.phi(prob, x))
    assert np.array_equal(acc.cpu().numpy(), racc) and racc.sum() > 0
    assert np.abs(xi.cpu().numpy() - rx).max() <= 1e-10 * np.abs(rx).max()
    assert np.abs(phi.cpu().numpy() / rphi - 1).max() <= 1e-10


def _check_posterior(prob, xg, log_z, N):
    logW, mean, var = ex.posterior(prob)
    mode = ex.nearest_mode(prob, xg)
    for i, (kk, _) in enumerate(ex.CENTRES):
        w = math.exp(logW[i])
        got = np.mean(mode == i)
        assert abs(got - w) < 4 * math.sqrt(w * (1 - w) * 4.0 / N), (i, got, w)
        sel = xg[mode == i, kk]
        assert abs(sel.mean() - mean[i, kk]) < 4 * math.sqrt(var[kk] * 4.0 / max(1, sel.size)) + 0.01, (i, kk)
        assert abs(sel.std() / math.sqrt(var[kk]) - 1) < 0.15, (i, kk, sel.std(), math.sqrt(var[kk]))
    assert abs(log_z - ex.log_evidence(prob)) < 0.3


def test_smc_gm_run_replays_the_oracle_run():
    """SMC-GM (Alg. 3) on the GPU against the oracle's run from the same seed: both draw every random
    number from the same Philox layout, so the two runs agree to rounding, stage by stage."""
    from paper_2503_16028_amd import smc
    from paper_2503_16028_amd.sampler import SMCGMSampler
    from oracle import smc as osmc
    banner("example1 smc-gm replay")
    N, M, seed = 1024, 8, 11
    prob, p = make(N)
    out = SMCGMSampler(p, N, M=M, ess_frac=0.5, prec=smc.SMC_FP64, seed=seed).run()
    ref = osmc.run_gm(_Shape(), 0, N, M=M, rho=0.5, seed=seed, phi_fn=lambda x: ex.phi(prob, x), kr=K, iters=50)
    taus = [0.0] + [h["tau"] for h in out["history"]]
    assert len(taus) == len(ref["taus"]) and np.allclose(taus, ref["taus"], rtol=1e-9, atol=1e-12)
    assert out["log_Z"] == pytest.approx(ref["log_Z"], abs=1e-8)
    xg = out["xi"].cpu().numpy()
    assert np.abs(xg - ref["xi"]).max() <= 1e-7 * np.abs(ref["xi"]).max()
    assert np.abs(out["phi"].cpu().numpy() / ref["phi"] - 1).max() <= 1e-7


def test_smc_pcngm_run_replays_the_oracle_run():
    """SMC-pCN-GM (Alg. 1 with Alg. 2) on the GPU against the oracle's run from the same seed:
    the same temperatures, step sizes, accept counts and final states to rounding."""
    from paper_2503_16028_amd import smc
    from paper_2503_16028_amd.sampler import SMCSampler
    from oracle import smc as osmc
    banner("example1 smc-pcn-gm replay")
    N, M, n_moves, seed = 512, 8, 5, 12
    prob, p = make(N)
    out = SMCSampler(p, N, M=M, n_moves=n_moves, ess_frac=0.5, beta0=0.5, prec=smc.SMC_FP64, seed=seed).run()
    ref = osmc.run(_Shape(), 0, N, M=M, n_moves=n_moves, rho=0.5, beta0=0.5, seed=seed,
                   phi_fn=lambda x: ex.phi(prob, x), kr=K)
    taus = [0.0] + [h["tau"] for h in out["history"]]
    assert len(taus) == len(ref["taus"]) and np.allclose(taus, ref["taus"], rtol=1e-9, atol=1e-12)
    assert [h["beta"] for h in out["history"]] == ref["betas"]
    assert np.allclose([h["rate"] for h in out["history"]], ref["rates"], rtol=0, atol=0)
    assert out["log_Z"] == pytest.approx(ref["log_Z"], abs=1e-8)
    assert np.abs(out["xi"].cpu().numpy() - ref["xi"]).max() <= 1e-7 * np.abs(ref["xi"]).max()


def test_smc_pcngm_run_against_exact_posterior():
    """SMC-pCN-GM keeps every tempered target invariant, so its cloud must carry the exact
    posterior's mode masses, per-mode means and spreads, and its evidence."""
    from paper_2503_16028_amd import smc
    from paper_2503_16028_amd.sampler import SMCSampler
    banner("example1 smc-pcn-gm vs exact posterior")
    N = 4096
    prob, p = make(N)
    out = SMCSampler(p, N, M=8, n_moves=10, ess_frac=0.5, beta0=0.5, prec=smc.SMC_FP64, seed=12).run()
    assert out["history"][-1]["tau"] == 1.0
    _check_posterior(prob, out["xi"].cpu().numpy(), out["log_Z"], N)


class _Shape:
    """What the oracle's SMC loops read from a problem when phi_fn and kr are given."""
    K = K
