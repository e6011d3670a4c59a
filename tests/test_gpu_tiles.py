"""Every tile shape of the fast-Poisson solver against the oracle, and the autotuner (GPU).

Tolerance as for the FP32+refinement forward map: 1e-7 of the largest observation.
"""
import json
import sys

import numpy as np
import pytest
import torch

import inputs
from conftest import golden
from oracle.forward import observe, solve
from oracle.problem import Problem as OProblem, synthesize

pytestmark = pytest.mark.gpu
DEV = "cuda"
CASES = [("t2", 32, 4), ("t2", 32, 8), ("c2", 64, 4), ("c2", 64, 8), ("c2", 64, 16), ("c3", 128, 16),
         ("c3", 128, 32)]


def banner(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _lib():
    from paper_2503_16028_amd import smc
    smc.lib()
    assert torch.cuda.is_available()


@pytest.mark.parametrize("name,grid,rows", CASES)
def test_tile_shape_matches_oracle(name, grid, rows):
    from paper_2503_16028_amd import smc
    banner("tile", name, grid, rows)
    d = json.load(open(golden("problem_%s.json" % name)))
    op = OProblem(d)
    N = 5
    p = smc.Problem(d, N, grids=[grid], tol64=1e-10, tol_inner=1e-5)
    assert rows in smc.smc_tile_candidates(grid)
    smc.smc_set_tile(p, 0, rows)
    assert smc.smc_get_tile(p, 0) == rows
    xi = inputs.particles(N, op.K, 50)
    G = torch.empty(N, op.n_obs, dtype=torch.float64, device=DEV)
    it = torch.empty(N, dtype=torch.int32, device=DEV)
    smc.smc_forward_batch(p, N, torch.tensor(xi, device=DEV), None, smc.SMC_FP32_REFINE, G, it)
    torch.cuda.synchronize()
    got = G.cpu().numpy()
    assert (it.cpu().numpy() < 60).all()
    for k in range(N):
        ref = observe(op, solve(op, synthesize(op, xi[k], grid), grid), grid)
        assert np.abs(got[k] - ref).max() <= 1e-7 * np.abs(ref).max()
    assert smc.smc_status_flags(p) == 0


def test_autotune_keeps_the_fastest():
    from paper_2503_16028_amd import smc
    banner("autotune 128")
    d = json.load(open(golden("problem_c3.json")))
    p = smc.Problem(d, 512, grids=[128], tol64=1e-10, tol_inner=1e-5)
    rows, ms = smc.smc_autotune(p, 0, 512, reps=2)
    assert set(ms) == set(smc.smc_tile_candidates(128))
    assert all(v > 0 for v in ms.values())
    assert rows == min(ms, key=ms.get)
    assert smc.smc_get_tile(p, 0) == rows
    with pytest.raises(smc.SMCError):
        smc.smc_set_tile(p, 0, 7)
