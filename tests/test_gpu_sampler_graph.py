"""A whole tempering stage as one captured graph (smc_sampler_graph_create) against the same calls
made one by one (GPU).

The graph holds tempering, resampling, gather, the mixture fit, the moves and the step-size rule,
with the stage counter, step sizes and temperatures in device memory, so replaying it once per
stage must give the bits of the samplers' call-by-call loops: the same particles, potentials,
temperatures, steps, step sizes, acceptance rates and evidence, stage by stage.  The cases cover
one grid with the plain pCN component (M = 1) and with a fitted mixture, a run resumed after two
stages, and three samplers on three grids finishing at different stages (a finished sampler's
rows pass through later stages unchanged).
"""
import json
import sys

import numpy as np
import pytest
import torch

from conftest import golden

pytestmark = pytest.mark.gpu


def banner(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _lib():
    from paper_2503_16028_amd import smc
    smc.lib()
    assert torch.cuda.is_available()


def load(name):
    return json.load(open(golden("problem_%s.json" % name)))


def same_run(a, b, hist_a, hist_b):
    assert torch.equal(a.xi, b.xi) and torch.equal(a.phi, b.phi)
    assert a.log_Z == b.log_Z and a.beta == b.beta and a.stage == b.stage
    assert len(hist_a) == len(hist_b)
    for ha, hb in zip(hist_a, hist_b):
        assert ha == hb, (ha, hb)


@pytest.mark.parametrize("M,prec_name,grid", [(1, "fp64", 32), (3, "fp64", 32), (4, "fp32_refine", 64)])
def test_single_grid_graph_gives_the_bits_of_the_calls(M, prec_name, grid):
    from paper_2503_16028_amd import smc
    from paper_2503_16028_amd.sampler import SMCSampler
    banner("sampler graph single grid", M, prec_name, grid)
    d = load("t2")
    N, n_moves, seed = 192, 3, 11
    prec = smc.SMC_FP64 if prec_name == "fp64" else smc.SMC_FP32_REFINE
    p = smc.Problem(d, N, grids=[grid], tol64=1e-11 if prec_name == "fp64" else 1e-10, tol_inner=1e-5)
    runs = []
    for graph in (False, True):
        s = SMCSampler(p, N, M, n_moves, seed=seed, prec=prec, graph=graph)
        s.run(max_stages=60)
        torch.cuda.synchronize()
        runs.append(s)
    a, b = runs
    assert a.history[-1]["tau"] == 1.0 and len(a.history) >= 3
    same_run(a, b, a.history, b.history)
    assert int(a.flags.item()) == 0 and int(b.flags.item()) == 0
    p.close()


def test_graph_run_resumed_after_two_stages():
    """run(stop_after=2) then run() again on the graph: the counter and step size restart from the
    sampler's state, so the result is the uninterrupted call-by-call run."""
    from paper_2503_16028_amd import smc
    from paper_2503_16028_amd.sampler import SMCSampler
    banner("sampler graph resume")
    d = load("t2")
    N, M, n_moves, seed = 160, 3, 2, 4
    p = smc.Problem(d, N, grids=[32], tol64=1e-11)
    a = SMCSampler(p, N, M, n_moves, seed=seed, prec=smc.SMC_FP64)
    a.run(max_stages=60)
    b = SMCSampler(p, N, M, n_moves, seed=seed, prec=smc.SMC_FP64, graph=True)
    b.run(max_stages=60, stop_after=2)
    assert b.stage == 2
    b.run(max_stages=60)
    torch.cuda.synchronize()
    same_run(a, b, a.history, b.history)
    p.close()


def test_mixed_whole_stage_graph_gives_the_bits_of_the_calls():
    """MixedSampler with graph="stage" (one launch per stage for all three samplers) against the
    captured-moves form: identical clouds, evidence and histories; every sampler ends at
    temperature 1 and keeps its cloud from the stage it got there."""
    from paper_2503_16028_amd import smc
    from paper_2503_16028_amd.sampler import MixedSampler
    banner("mixed sampler whole-stage graph")
    d = load("c5")
    counts, M, n_moves, seed = (32, 8, 4), 4, 2, 5
    N = sum(counts)
    p = smc.Problem(d, N, grids=[64, 128, 256], tol64=6e-12, max_iter=60 * 256, max_sweeps=6)
    res = []
    for graph in (True, "stage"):
        ms = MixedSampler(p, counts, M, n_moves, prec=smc.SMC_FP64, seed=seed, graph=graph)
        ms.initialise()
        frozen, ends = {}, {}
        for _ in range(200):
            before = list(ms.running)
            left = ms.step()
            for g in before:
                if g not in ms.running:
                    r = ms.rows(g)
                    frozen[g] = (ms.xi[r].cpu().numpy().copy(), ms.phi[r].cpu().numpy().copy())
                    ends[g] = ms.stage
            if left == 0:
                break
        ms.stream.synchronize()
        if ms.whole:
            ms._collect_whole()
        out = [dict(xi=ms.xi[ms.rows(g)].cpu().numpy(), phi=ms.phi[ms.rows(g)].cpu().numpy(), log_Z=ms.log_Z[g],
                    history=ms.history[g], end=ends[g]) for g in range(3)]
        assert int(ms.flags.item()) == 0
        banner("graph", graph, "stages at which the samplers reached 1:", [ends[g] for g in range(3)])
        ms.close()
        for g in range(3):
            assert out[g]["history"][-1]["tau"] == 1.0
            assert np.array_equal(out[g]["xi"], frozen[g][0]) and np.array_equal(out[g]["phi"], frozen[g][1])
        res.append(out)
    for g in range(3):
        a, b = res[0][g], res[1][g]
        assert np.array_equal(a["xi"], b["xi"]) and np.array_equal(a["phi"], b["phi"])
        assert a["log_Z"] == b["log_Z"] and a["end"] == b["end"]
        assert a["history"] == b["history"]
    assert len({res[1][g]["end"] for g in range(3)}) > 1   # some sampler went on after another finished
    p.close()


def test_sampler_graph_rejects_bad_arguments():
    """Invalid descriptions fail with SMC_E_INVAL before any capture, leaving the stream usable."""
    from paper_2503_16028_amd import smc
    banner("sampler graph argument checks")
    d = load("t2")
    N, M = 64, 3
    p = smc.Problem(d, N, grids=[32])
    dev = torch.device("cuda:0")
    f64 = dict(dtype=torch.float64, device=dev)
    K, kr = p.K, p.kr
    R, G3, MM = N + 8, 3, 100   # room for every bad shape below, so that only the library objects
    t = dict(xi=torch.zeros(R, K, **f64), phi=torch.zeros(R, **f64), xi2=torch.zeros(R, K, **f64),
             phi2=torch.zeros(R, **f64), W=torch.zeros(R, **f64), idx=torch.zeros(R, dtype=torch.int32, device=dev),
             tau=torch.zeros(G3, **f64), tau_new=torch.zeros(G3, **f64), h=torch.zeros(G3, **f64),
             log_z=torch.zeros(G3, **f64), beta=torch.full((G3,), 0.2, **f64), logw=torch.zeros(G3, MM, **f64),
             mean=torch.zeros(G3, MM, kr, **f64), scale=torch.ones(G3, MM, kr, **f64),
             ctr=torch.zeros(1, dtype=torch.int64, device=dev), n_acc=torch.zeros(R, dtype=torch.int32, device=dev),
             record=torch.zeros(4, G3, 5, **f64))
    s = torch.cuda.Stream()

    def make(counts=(N,), M_=M, stride=1 << 20, **over):
        tt = dict(t, **over)
        return smc.SamplerGraph(p, list(counts), M_, 2, 10, 0.5, 1e-3, 1, stride, smc.SMC_FP64, tt, s, 4)

    bad = [dict(counts=(N // 2, N // 2)),            # two groups without a level map
           dict(counts=(0,)),                        # an empty group
           dict(counts=(N + 1,)),                    # more rows than the problem holds
           dict(M_=0), dict(M_=99),                  # mixture size
           dict(stride=0),                           # counter spacing
           dict(xi2=t["xi"]),                        # gather scratch aliasing the particles
           dict(level=torch.zeros(R, dtype=torch.int32, device=dev))]   # a level map on a one-grid 32^2 problem
    for kw in bad:
        with pytest.raises(smc.SMCError) as e:
            make(**kw)
        assert e.value.status == smc.SMC_E_INVAL, kw
    B = (1 << 20) + 1                                 # a group beyond the tempering step's batch
    big = dict(xi=torch.zeros(B, K, **f64), xi2=torch.zeros(B, K, **f64), phi=torch.zeros(B, **f64),
               phi2=torch.zeros(B, **f64), W=torch.zeros(B, **f64), idx=torch.zeros(B, dtype=torch.int32, device=dev),
               n_acc=torch.zeros(B, dtype=torch.int32, device=dev))
    with pytest.raises(smc.SMCError) as e:
        make(counts=(B,), **big)
    assert e.value.status == smc.SMC_E_INVAL
    del big
    g = make()                                       # the stream still captures a valid stage
    g.close()
    s.synchronize()
    p.close()


def test_whole_stage_graph_at_the_metric_configuration():
    """128^2, N = 4096, M = 8, 20 moves per stage, FP32 with refinement at the benchmark's
    tolerances: three stages as graph launches give the bits of three call-by-call stages."""
    from paper_2503_16028_amd import smc
    from paper_2503_16028_amd.sampler import SMCSampler
    banner("sampler graph metric configuration")
    d = load("c3")
    N, M, n_moves = 4096, 8, 20
    p = smc.Problem(d, N, tol64=1e-10, tol_inner=1e-3)
    runs = []
    for graph in (False, True):
        s = SMCSampler(p, N, M, n_moves, seed=2503, graph=graph)
        s.run(stop_after=3)
        torch.cuda.synchronize()
        runs.append(s)
    a, b = runs
    assert a.stage == 3
    same_run(a, b, a.history, b.history)
    assert all(0.0 < h["rate"] <= 1.0 for h in a.history)
    p.close()
