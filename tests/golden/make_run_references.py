"""Writes run_<name>_oracle.json: one whole SMC-pCN-GM run (Alg. 1 with the pCN-GM mutation, Alg. 2)
of the oracle on a workload's problem, from its seed to temperature 1, in FP64 with a direct solve
per proposal.  The GPU tests replay these runs (the random numbers of both sides come from the
same Philox layout) and compare the posterior moments of the GPU's FP32-with-refinement runs.

    python tests/golden/make_run_references.py [c1 c2 c3] [--workers P]

Workloads (the problems' own fields give the grid, mixture size, moves per stage, ESS fraction
and starting step size):
  c1  1D, 64 intervals, N = 256, plain pCN (M = 1), 10 moves per stage
  c2  64^2, N = 1024, M = 4, 20 moves per stage
  c3  128^2 with the mirrored observations, M = 8, 20 moves per stage, N = 1024 (the workload's
      4096 particles would take hours of oracle solves; the GPU runs both sizes)
Stored: the temperature schedule, step sizes, acceptance rates and counts, log Z, every final
potential, the mean and standard deviation of every coordinate of the final cloud, and the full
final state of four particles.
"""
import argparse
import concurrent.futures
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import smc as osmc  # noqa: E402
from oracle.problem import Problem  # noqa: E402

RUNS = {"c1": dict(N=256, seed=0), "c2": dict(N=1024, seed=0), "c3": dict(N=1024, seed=0)}


def make(name, workers):
    d = json.load(open(os.path.join(HERE, "problem_%s.json" % name)))
    p = Problem(d)
    cfg = RUNS[name]
    N, seed = cfg["N"], cfg["seed"]
    n = d["grids"][0]
    M, n_moves, rho, beta0 = int(d["M"]), int(d["n_moves"]), float(d["ess_frac"]), float(d["beta0"])
    t0 = time.time()
    ctx = mp.get_context("fork")
    with concurrent.futures.ProcessPoolExecutor(workers, mp_context=ctx) as ex:
        ref = osmc.run(p, n, N, M=M, n_moves=n_moves, rho=rho, beta0=beta0, seed=seed, pmap=ex.map,
                       chunks=4 * workers)
    xi = ref["xi"]
    keep = [0, N // 3, (2 * N) // 3, N - 1]
    out = dict(problem=name, grid=n, N=N, M=M, n_moves=n_moves, rho=rho, beta0=beta0, seed=seed, fit_iters=50,
               var_floor=1e-3, taus=[float(v) for v in ref["taus"]], betas=[float(v) for v in ref["betas"]],
               rates=[float(v) for v in ref["rates"]], accepts=[int(v) for v in ref["n_acc"]],
               log_Z=float(ref["log_Z"]), phi=[float(v) for v in ref["phi"]],
               mean=xi.mean(0).tolist(), std=xi.std(0).tolist(), keep=keep, xi_keep=xi[keep].tolist(),
               seconds=round(time.time() - t0, 1), workers=workers,
               generated_by="python tests/golden/make_run_references.py %s" % name)
    with open(os.path.join(HERE, "run_%s_oracle.json" % name), "w") as f:
        json.dump(out, f)
    print(name, "stages", len(ref["taus"]) - 1, "log Z %.6f" % ref["log_Z"], "%.0f s" % out["seconds"], flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*", default=sorted(RUNS))
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    os.environ["OMP_NUM_THREADS"] = "1"
    for name in a.names:
        make(name, a.workers)


if __name__ == "__main__":
    main()
