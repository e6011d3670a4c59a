"""Writes sampler_small2d_oracle.json: a small 2D problem (2 x 2 cosine modes, 16 x 16 grid,
3 x 3 observations, data from the oracle's forward map on a 64 x 64 grid) and the posterior
moments and evidence of one SMC run of the oracle on it (Alg. 1 with the pCN-GM mutation).

    python tests/golden/make_sampler_reference.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import smc as osmc  # noqa: E402
from oracle.forward import observe, solve  # noqa: E402
from oracle.problem import Problem, synthesize  # noqa: E402

N, M, N_MOVES, RHO, BETA0, SEED = 1500, 2, 6, 0.5, 0.5, 6


def small_2d():
    nodes = [4, 8, 12]
    obs = [[i, j] for j in nodes for i in nodes]
    d = dict(name="small2d", dim=2, grids=[16], kl_per_axis=2, kr=4, obs_den=16, obs=obs,
             y=[0.0] * len(obs), sigma=1.0, f=1.0)
    p = Problem(d)
    G = observe(p, solve(p, synthesize(p, np.array([0.9, -0.7, 0.5, 1.1]), 64), 64), 64)
    sigma = 0.02 * np.abs(G).max()
    y = G + sigma * np.random.default_rng(5).standard_normal(G.size)
    d["y"], d["sigma"] = [float(v) for v in y], float(sigma)
    return d


def main():
    d = small_2d()
    ref = osmc.run(Problem(d), 16, N, M=M, n_moves=N_MOVES, rho=RHO, beta0=BETA0, seed=SEED, kr=4)
    out = dict(problem=d, N=N, M=M, n_moves=N_MOVES, rho=RHO, beta0=BETA0, seed=SEED,
               mean=ref["xi"].mean(0).tolist(), std=ref["xi"].std(0).tolist(), log_Z=float(ref["log_Z"]),
               stages=len(ref["taus"]) - 1, generated_by="python tests/golden/make_sampler_reference.py")
    with open(os.path.join(HERE, "sampler_small2d_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
