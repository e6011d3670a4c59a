"""Whole SMC runs of the GPU sampler against the oracle's posterior (GPU).

The sampler (Alg. 1 with the pCN-GM mutation, driven over the C ABI) must reproduce posterior
moments within Monte Carlo error:
  * a 1D problem with two mirrored observation pairs, whose posterior is symmetric in the
    second coordinate (two modes), against brute-force quadrature of the posterior and of the
    evidence Z;
  * a 2D problem with 2 x 2 cosine modes on the FP32+refinement path, against a stored SMC
    run of the oracle (the quadrature would need 4 dimensions).
Tolerances are stated per assertion in units of the Monte Carlo standard error.
"""
import json
import math
import sys

import numpy as np
import pytest
import torch

from conftest import golden
from oracle import quadrature
from oracle.forward import observe, phi as oracle_phi, solve
from oracle.problem import Problem as OProblem, synthesize

pytestmark = pytest.mark.gpu


def banner(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _lib():
    from paper_2503_16028_amd import smc
    smc.lib()
    assert torch.cuda.is_available()


def mirrored_1d():
    """K = 2 sine modes on 16 intervals, observations at 4, 6 and their mirrors 12, 10 with
    pair-averaged data, so Phi(xi_1, xi_2) = Phi(xi_1, -xi_2)."""
    obs = [4, 6, 12, 10]
    d = dict(name="mirrored1d", dim=1, grids=[16], kl_per_axis=2, kr=2, obs_den=16, obs=[[o] for o in obs],
             y=[0.0] * 4, sigma=1.0, f=1.0)
    p = OProblem(d)
    G = observe(p, solve(p, synthesize(p, np.array([0.8, 1.6]), 64), 64), 64)
    sigma = 0.05 * np.abs(G).max()
    noise = sigma * np.random.default_rng(2).standard_normal(2)
    y = np.concatenate([0.5 * (G[:2] + G[2:]) + noise] * 2)
    d["y"], d["sigma"] = [float(v) for v in y], float(sigma)
    return d, OProblem(d)


def test_sampler_1d_bimodal_against_quadrature():
    from paper_2503_16028_amd import smc
    from paper_2503_16028_amd.sampler import SMCSampler
    banner("sampler 1d bimodal")
    d, op = mirrored_1d()
    f = lambda x: oracle_phi(op, x, 16)
    assert abs(f(np.array([0.4, 1.3])) - f(np.array([0.4, -1.3]))) < 1e-9 * f(np.array([0.4, 1.3]))
    mean_q, cov_q, w, grid = quadrature.moments(f, 2, pts=241)
    step = grid[1, 1] - grid[0, 1]
    logp = np.array([-f(x) for x in grid]) - 0.5 * (grid ** 2).sum(1) - np.log(2 * np.pi)
    log_z_q = logp.max() + np.log(np.exp(logp - logp.max()).sum() * step * step)
    N = 4096
    p = smc.Problem(d, N, tol64=1e-13)
    s = SMCSampler(p, N, M=2, n_moves=8, ess_frac=0.5, beta0=0.5, prec=smc.SMC_FP64, seed=4)
    out = s.run()
    xi = out["xi"].cpu().numpy()
    n_eff = N / 4                                         # resampling and finite mixing
    assert abs(np.mean(xi[:, 1] > 0) - 0.5) < 4 * math.sqrt(0.25 / n_eff)
    assert abs(xi[:, 0].mean() - mean_q[0]) < 4 * math.sqrt(cov_q[0, 0] / n_eff)
    assert abs(np.var(xi[:, 1]) / cov_q[1, 1] - 1) < 4 * math.sqrt(2 / n_eff)
    assert abs(np.var(xi[:, 0]) / cov_q[0, 0] - 1) < 4 * math.sqrt(2 / n_eff)
    assert abs(out["log_Z"] - log_z_q) < 0.1
    assert out["history"][-1]["tau"] == 1.0
    assert smc.smc_status_flags(p) == 0


def test_sampler_2d_fp32_refine_against_oracle_smc():
    """Reference: tests/golden/sampler_small2d_oracle.json (the problem and the oracle's run,
    written by make_sampler_reference.py beside it)."""
    from paper_2503_16028_amd import smc
    from paper_2503_16028_amd.sampler import SMCSampler
    banner("sampler 2d fp32+refine vs oracle smc")
    ref = json.load(open(golden("sampler_small2d_oracle.json")))
    d = ref["problem"]
    N_o, N_g = ref["N"], 4096
    mo, so = np.array(ref["mean"]), np.array(ref["std"])
    p = smc.Problem(d, N_g, tol64=1e-10, tol_inner=1e-5)
    s = SMCSampler(p, N_g, M=ref["M"], n_moves=ref["n_moves"], ess_frac=ref["rho"], beta0=ref["beta0"],
                   prec=smc.SMC_FP32_REFINE, seed=7)
    out = s.run()
    xg = out["xi"].cpu().numpy()
    sd = np.sqrt(0.5 * (so ** 2 + xg.var(0)))
    se = sd * np.sqrt(4.0 / N_o + 4.0 / N_g)           # both clouds, effective size N / 4
    assert np.all(np.abs(xg.mean(0) - mo) < 4 * se), (xg.mean(0), mo, se)
    assert np.all(np.abs(xg.std(0) / so - 1) < 4 * math.sqrt(2 * (4.0 / N_o + 4.0 / N_g))), (xg.std(0), so)
    assert abs(out["log_Z"] - ref["log_Z"]) < 0.3
    assert smc.smc_status_flags(p) == 0
