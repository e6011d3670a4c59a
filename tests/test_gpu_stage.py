"""The persistent stage launch (one launch for every move of a stage, each workgroup running all the
moves of a particle) against one launch per step (smc_set_stage_fusion off): the same bits for the
states, potentials and accept counts, eagerly and replayed from a captured graph; and against the
oracle on sampled particles at the metric configuration's launch.
"""
import json
import sys

import numpy as np
import pytest
import torch

import inputs
from conftest import golden
from oracle.forward import observe, potential, solve
from oracle.moves import GM, gmpcn_moves
from oracle.problem import Problem as OProblem, synthesize

pytestmark = pytest.mark.gpu
DEV = "cuda"


def banner(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def t(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def start(name, grid, N, seed):
    from paper_2503_16028_amd import smc
    d = json.load(open(golden("problem_%s.json" % name)))
    op = OProblem(d)
    p = smc.Problem(d, N, grids=[grid], tol64=1e-10, tol_inner=1e-3)
    xi = inputs.particles(N, op.K, seed, 0.8)
    G = torch.empty(N, op.n_obs, dtype=torch.float64, device=DEV)
    phi = torch.empty(N, dtype=torch.float64, device=DEV)
    smc.smc_forward_batch(p, N, t(xi), None, smc.SMC_FP32_REFINE, G)
    smc.smc_potential(p, N, G, phi)
    torch.cuda.synchronize()
    return d, op, p, xi, phi.cpu().numpy()


def moves(p, N, gm, xi0, phi0, fused, beta=0.3, tau=0.6, n_moves=3, seed=5, ctr=70):
    from paper_2503_16028_amd import smc
    smc.smc_set_stage_fusion(p, fused)
    xi, phi = t(xi0), t(phi0)
    acc = torch.empty(N, dtype=torch.int32, device=DEV)
    smc.smc_gmpcn_move(p, N, gm, beta, tau, n_moves, seed, ctr, None, smc.SMC_FP32_REFINE, xi, phi, acc)
    torch.cuda.synchronize()
    assert smc.smc_status_flags(p) == 0
    return xi, phi, acc


@pytest.mark.parametrize("name,grid,rows,N", [("c3", 128, 32, 300), ("c3", 128, 16, 130), ("c2", 64, 8, 257)])
def test_stage_launch_gives_the_bits_of_one_launch_per_step(name, grid, rows, N):
    from paper_2503_16028_amd import smc
    banner("stage launch vs per step", name, grid, rows, N)
    d, op, p, xi0, phi0 = start(name, grid, N, 81)
    smc.smc_set_tile(p, 0, rows)
    logw, mean, scale = inputs.mixture(8, op.kr, 82, spread=0.5)
    gm = (t(logw), t(mean), t(scale))
    xa, pa, aa = moves(p, N, gm, xi0, phi0, True)
    xb, pb, ab = moves(p, N, gm, xi0, phi0, False)
    assert 0 < int(aa.sum()) < 3 * N
    assert torch.equal(aa, ab) and torch.equal(pa, pb) and torch.equal(xa, xb)


def test_stage_launch_in_a_graph_replays_eager_runs():
    """A captured single-grid stage (the persistent launch, parameters read on the device) replayed
    three times with the parameters changed between replays; each replay against an eager run of one
    launch per step from the same state."""
    from paper_2503_16028_amd import smc
    banner("stage launch graph")
    N, M = 200, 4
    d, op, p, xi0, phi0 = start("c3", 128, N, 83)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        logw, mean, scale = (t(a)[None].contiguous() for a in inputs.mixture(M, op.kr, 84, spread=0.5))
        beta = t([0.3])
        tau = t([0.5])
        ctr = torch.zeros(1, dtype=torch.int64, device=DEV)
        sd = smc.stage_desc(1, logw, mean, scale, beta, tau, ctr, 9)
        xi, phi = t(xi0), t(phi0)
        acc = torch.empty(N, dtype=torch.int32, device=DEV)
        smc.smc_set_stage_fusion(p, True)        # captured as the persistent stage launch
        graph = smc.StageGraph(p, N, None, sd, 2, smc.SMC_FP32_REFINE, xi, phi, acc, s)
    for r in range(3):
        with torch.cuda.stream(s):
            beta.fill_(0.2 + 0.1 * r)
            tau.fill_(0.4 + 0.2 * r)
            ctr.fill_(1000 * (r + 1))
            before_x, before_p = xi.clone(), phi.clone()
            graph.launch(s)
        s.synchronize()
        smc.smc_set_stage_fusion(p, False)
        ex, ep = before_x.clone(), before_p.clone()
        ea = torch.empty(N, dtype=torch.int32, device=DEV)
        smc.smc_gmpcn_move(p, N, (logw[0], mean[0], scale[0]), 0.2 + 0.1 * r, 0.4 + 0.2 * r, 2, 9, 1000 * (r + 1),
                           None, smc.SMC_FP32_REFINE, ex, ep, ea)
        torch.cuda.synchronize()
        smc.smc_set_stage_fusion(p, True)
        assert torch.equal(acc, ea) and torch.equal(phi, ep) and torch.equal(xi, ex), r
    graph.close()


def test_stage_launch_at_the_metric_configuration_against_the_oracle():
    """128^2, N = 4096, M = 8, 20 moves in one launch (the benchmark's stage); 24 particles spread over
    the batch replayed by the oracle move by move."""
    from paper_2503_16028_amd import smc
    banner("stage launch 128^2 N=4096 20 moves")
    N, M, n_moves = 4096, 8, 20
    d, op, p, xi0, phi0 = start("c3", 128, N, 85)
    logw, mean, scale = inputs.mixture(M, op.kr, 86, spread=0.4)
    xi, phi, acc = moves(p, N, (t(logw), t(mean), t(scale)), xi0, phi0, True, beta=0.2, tau=0.05,
                         n_moves=n_moves, seed=3, ctr=4000)
    pick = np.linspace(0, N - 1, 24).astype(int)
    gm = GM(logw, mean, scale, op.active(), op.K)
    rphi0 = np.array([potential(observe(op, solve(op, synthesize(op, x, 128), 128), 128), op.y, op.sigma)
                      for x in xi0[pick]])                 # the oracle's own starting potentials
    rx, rphi, racc = gmpcn_moves(op, 128, xi0[pick], rphi0, gm, 0.2, 0.05, n_moves, 3, 4000, ids=pick)
    assert np.array_equal(acc.cpu().numpy()[pick], racc) and racc.sum() > 0
    assert np.abs(xi.cpu().numpy()[pick] - rx).max() <= 1e-6
    assert np.abs(phi.cpu().numpy()[pick] / rphi - 1).max() <= 1e-8
