"""Write the problem definitions with their synthetic data to tests/golden/.

TEST INFRASTRUCTURE ONLY: this script calls nothing but the oracle.  Run
    python -m oracle.make_problems
from the repository root.  Each file holds the problem definition (grid, prior,
observation layout, sampler settings) and the data d = F(u_true) + eps computed
by the oracle on a fine grid of 512 intervals (the paper generates its data on a
finer mesh than the inference mesh, Sec. 3.2), with sigma = noise_frac *
max|F(u_true)| (Sec. 3.2 noise rule) and seeded draws of u_true and eps.
"""
import json
import os
import sys

import numpy as np

from .forward import observe, solve
from .problem import Problem

N_FINE = 512
TRUTH_SEED = 2503
NOISE_SEED = 16028


def grid5(den, pts):
    return [[a, b] for a in pts for b in pts]


def definitions():
    c2_obs = grid5(64, [11, 21, 32, 43, 53])
    ys = [32, 48, 64, 80, 96]
    c3_obs = [[102, y] for y in ys] + [[26, y] for y in ys]
    base2 = dict(dim=2, kl_per_axis=32, kr=64, f=1.0, noise_frac=0.01)
    return [
        dict(name="c1", dim=1, grids=[64], kl_per_axis=64, kr=64, f=1.0, noise_frac=0.01,
             obs_den=64, obs=[[7], [14], [21], [28], [36], [43], [50], [57]],
             N=256, M=1, n_moves=10, ess_frac=0.5, beta0=0.2, precision="fp64",
             what="1D elliptic, 65-point grid, 64 sine modes, 8 observations, pCN"),
        dict(name="c2", grids=[64], obs_den=64, obs=c2_obs, N=1024, M=4, n_moves=20, ess_frac=0.5,
             beta0=0.2, precision="fp64", what="2D 64^2, 25 observations, 4-component GM-pCN", **base2),
        dict(name="c3", grids=[128], obs_den=128, obs=c3_obs, pairs=[[k, k + 5] for k in range(5)],
             N=4096, M=8, n_moves=20, ess_frac=0.5, beta0=0.2, precision="fp32_refine",
             what="2D 128^2, 10 observations mirrored about x=1/2, 8-component GM-pCN", **base2),
        dict(name="c4", grids=[128], obs_den=64, obs=c2_obs, N=2048, M=1, n_moves=20, ess_frac=0.5,
             beta0=0.2, precision="fp32_refine", move="pcnl",
             what="2D 128^2, 25 observations, pCN-Langevin with adjoint gradients", **base2),
        dict(name="c5", grids=[64, 128, 256], obs_den=64, obs=c2_obs, N=[4096, 3072, 1024], M=8,
             n_moves=20, ess_frac=0.5, beta0=0.2, precision="fp32_refine",
             what="2D mixed resolution 64^2/128^2/256^2, same prior and data", **base2),
        # small problems for parity tests: several tiles, ragged tails, quick oracle
        dict(name="t2", grids=[16, 32, 64], obs_den=16, obs=grid5(16, [4, 8, 12])[:9] , N=64, M=3,
             n_moves=2, ess_frac=0.5, beta0=0.3, precision="fp64", what="small 2D test problem",
             **dict(base2, kl_per_axis=8, kr=12)),
        dict(name="t1", dim=1, grids=[16, 64], kl_per_axis=8, kr=8, f=1.0, noise_frac=0.01, obs_den=16,
             obs=[[3], [8], [13]], N=64, M=1, n_moves=2, ess_frac=0.5, beta0=0.3, precision="fp64",
             what="small 1D test problem"),
    ]


def generate(d):
    d = dict(d)
    prob = Problem(dict(d, y=[0.0] * len(d["obs"]), sigma=1.0))
    rng_t = np.random.default_rng(TRUTH_SEED)
    xi_true = rng_t.standard_normal(prob.K)
    from .problem import synthesize
    U = synthesize(prob, xi_true, N_FINE)
    G = observe(prob, solve(prob, U, N_FINE), N_FINE)
    sigma = d["noise_frac"] * float(np.max(np.abs(G)))
    rng_n = np.random.default_rng(NOISE_SEED)
    if d.get("pairs"):
        y = np.empty_like(G)
        eta = rng_n.standard_normal(len(d["pairs"]))
        for (a, b), e in zip(d["pairs"], eta):
            y[a] = y[b] = 0.5 * (G[a] + G[b]) + sigma * e
    else:
        y = G + sigma * rng_n.standard_normal(G.size)
    d.update(y=y.tolist(), sigma=sigma, G_true_fine=G.tolist(), xi_true=xi_true.tolist(),
             n_fine=N_FINE, truth_seed=TRUTH_SEED, noise_seed=NOISE_SEED,
             generated_by="python -m oracle.make_problems")
    return d


def main(argv):
    out = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", "golden")
    names = set(argv[1:])
    for d in definitions():
        if names and d["name"] not in names:
            continue
        g = generate(d)
        with open(os.path.join(out, "problem_%s.json" % d["name"]), "w") as fh:
            json.dump(g, fh, indent=1)
        print(d["name"], "sigma=%.6g" % g["sigma"], flush=True)


if __name__ == "__main__":
    main(sys.argv)
