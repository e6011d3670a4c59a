"""Particles on several grids in one launch (level maps), per-group stage parameters and the
captured stage graph, against the oracle and against the single-grid calls (GPU).

Tolerances as in the single-grid parity tests: FP64 1e-10 relative, FP32+refinement 1e-7 on G
and 1e-4 on potentials; accept counts bit-exact; graph replays bit-identical to eager runs.
"""
import json
import sys

import numpy as np
import pytest
import torch

import inputs
from conftest import golden
from oracle.forward import observe, phi as oracle_phi, solve
from oracle.moves import GM, gmpcn_moves
from oracle.problem import Problem as OProblem, synthesize

pytestmark = pytest.mark.gpu
DEV = "cuda"
GRIDS = [64, 128, 256]


def banner(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def load(name):
    d = json.load(open(golden("problem_%s.json" % name)))
    return d, OProblem(d)


def t(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


@pytest.fixture(scope="module", autouse=True)
def _lib():
    from paper_2503_16028_amd import smc
    smc.lib()
    assert torch.cuda.is_available()


def mixed_problem(d, N, prec_name, **kw):
    from paper_2503_16028_amd import smc
    if prec_name == "fp64":
        return smc.Problem(d, N, grids=GRIDS, tol64=6e-12, max_iter=60 * 256, max_sweeps=6, **kw)
    return smc.Problem(d, N, grids=GRIDS, tol64=1e-10, tol_inner=1e-5, max_iter=80 * 256, **kw)


LEVELS = np.array([2, 1, 0, 0, 1, 0, 1, 0], dtype=np.int32)


@pytest.mark.parametrize("prec_name", ["fp64", "fp32_refine"])
def test_forward_levels(prec_name):
    """One call over 64^2, 128^2 and 256^2 particles (one launch per grid, each in its single-grid
    shape); each row equals the oracle on its grid, and every row equals, bit for bit, the
    single-grid launch."""
    from paper_2503_16028_amd import smc
    banner("forward levels", prec_name)
    d, op = load("c5")
    N = len(LEVELS)
    prec = smc.PRECISIONS[prec_name]
    p = mixed_problem(d, N, prec_name)
    xi = inputs.particles(N, op.K, 40)
    G = torch.empty(N, op.n_obs, dtype=torch.float64, device=DEV)
    it = torch.empty(N, dtype=torch.int32, device=DEV)
    smc.smc_forward_batch(p, N, t(xi), t(LEVELS, torch.int32), prec, G, it)
    torch.cuda.synchronize()
    got = G.cpu().numpy()
    assert (it.cpu().numpy() > 0).all()
    assert smc.smc_status_flags(p) == 0
    tol = 1e-10 if prec_name == "fp64" else 1e-7
    for k in range(N):
        n = GRIDS[LEVELS[k]]
        ref = observe(op, solve(op, synthesize(op, xi[k], n), n), n)
        assert np.abs(got[k] - ref).max() <= tol * np.abs(ref).max(), (k, n)
    for lv in (0, 1, 2):
        rows = np.nonzero(LEVELS == lv)[0]
        q = smc.Problem(d, len(rows), grids=[GRIDS[lv]], tol64=p_tol(prec_name), tol_inner=1e-5,
                        max_iter=(60 if prec_name == "fp64" else 80) * 256, max_sweeps=6 if prec_name == "fp64" else 8)
        G1 = torch.empty(len(rows), op.n_obs, dtype=torch.float64, device=DEV)
        smc.smc_forward_batch(q, len(rows), t(xi[rows]), None, prec, G1)
        torch.cuda.synchronize()
        assert np.array_equal(G1.cpu().numpy(), got[rows]), lv


@pytest.mark.parametrize("levels", [[2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1], [0, 1, 2, 0, 1, 2]])
def test_forward_levels_rows_keep_their_workspace(levels):
    """Rows of every grid in one launch, the 256^2 rows first: the FP32 scaling of an on-chip
    (64^2, 128^2) row lies inside its own row of the workspace, never inside the FP64 scaling
    of a 256^2 row solved at the same time.  Every row converges and equals, bit for bit, a
    launch of its grid alone."""
    from paper_2503_16028_amd import smc
    lv = np.array(levels, dtype=np.int32)
    banner("forward levels rows keep their workspace", levels)
    d, op = load("c5")
    N = len(lv)
    p = mixed_problem(d, N, "fp32_refine")
    xi = inputs.particles(N, op.K, 50)
    G = torch.empty(N, op.n_obs, dtype=torch.float64, device=DEV)
    it = torch.empty(N, dtype=torch.int32, device=DEV)
    smc.smc_forward_batch(p, N, t(xi), t(lv, torch.int32), smc.SMC_FP32_REFINE, G, it)
    torch.cuda.synchronize()
    assert (it.cpu().numpy() > 0).all(), it.cpu().numpy()
    assert smc.smc_status_flags(p) == 0
    got = G.cpu().numpy()
    for l in sorted(set(levels)):
        rows = np.nonzero(lv == l)[0]
        q = smc.Problem(d, len(rows), grids=GRIDS, tol64=1e-10, tol_inner=1e-5, max_iter=80 * 256)
        G1 = torch.empty(len(rows), op.n_obs, dtype=torch.float64, device=DEV)
        smc.smc_forward_batch(q, len(rows), t(xi[rows]), t(np.full(len(rows), l, np.int32), torch.int32),
                              smc.SMC_FP32_REFINE, G1)
        torch.cuda.synchronize()
        assert np.array_equal(G1.cpu().numpy(), got[rows]), l


def p_tol(prec_name):
    return 6e-12 if prec_name == "fp64" else 1e-10


def test_forward_levels_out_of_range():
    from paper_2503_16028_amd import smc
    banner("forward levels out of range")
    d, op = load("c5")
    lv = np.array([0, 5, -1, 1], dtype=np.int32)
    N = len(lv)
    p = mixed_problem(d, N, "fp32_refine")
    xi = inputs.particles(N, op.K, 41)
    G = torch.empty(N, op.n_obs, dtype=torch.float64, device=DEV)
    it = torch.empty(N, dtype=torch.int32, device=DEV)
    smc.smc_forward_batch(p, N, t(xi), t(lv, torch.int32), smc.SMC_FP32_REFINE, G, it)
    torch.cuda.synchronize()
    g, i = G.cpu().numpy(), it.cpu().numpy()
    assert np.isnan(g[1]).all() and np.isnan(g[2]).all() and i[1] == -1 and i[2] == -1
    assert np.isfinite(g[0]).all() and np.isfinite(g[3]).all() and i[0] > 0 and i[3] > 0
    assert smc.smc_status_flags(p) & smc.FLAG_BADLEVEL


def group_mixture(op, G, M, seed):
    logw, mean, scale = [], [], []
    for g in range(G):
        lw, mu, sc = inputs.mixture(M, op.kr, seed + g, spread=0.5)
        logw.append(lw), mean.append(mu), scale.append(sc)
    return np.array(logw), np.array(mean), np.array(scale)


def test_stage_per_group_matches_oracle():
    """Three samplers (one per grid), each with its own mixture, beta and tau, moved in one
    call; every particle replays the oracle's moves on its grid with its group's parameters."""
    from paper_2503_16028_amd import smc
    banner("stage per group fp64")
    d, op = load("c5")
    lv = np.array([0, 1, 0, 2, 1, 0], dtype=np.int32)
    N, M, n_moves, seed, ctr = len(lv), 3, 2, 31, 5000
    p = mixed_problem(d, N, "fp64")
    xi = inputs.particles(N, op.K, 42) * 0.3
    logw, mean, scale = group_mixture(op, 3, M, 43)
    beta = np.array([0.3, 0.2, 0.4])
    tau = np.array([1e-3, 2e-3, 5e-4])
    X, L = t(xi), t(lv, torch.int32)
    Gm = torch.empty(N, op.n_obs, dtype=torch.float64, device=DEV)
    phi = torch.empty(N, dtype=torch.float64, device=DEV)
    smc.smc_forward_batch(p, N, X, L, smc.SMC_FP64, Gm)
    smc.smc_potential(p, N, Gm, phi)
    acc = torch.empty(N, dtype=torch.int32, device=DEV)
    ctr_t = torch.tensor([ctr], dtype=torch.int64, device=DEV)
    tens = [t(logw), t(mean), t(scale), t(beta), t(tau)]
    sd = smc.stage_desc(3, *tens, ctr_t, seed)
    smc.smc_gmpcn_stage(p, N, L, sd, n_moves, smc.SMC_FP64, X, phi, acc)
    torch.cuda.synchronize()
    gx, gphi, gacc = X.cpu().numpy(), phi.cpu().numpy(), acc.cpu().numpy()
    assert smc.smc_status_flags(p) == 0
    for g in range(3):
        ids = np.nonzero(lv == g)[0]
        n = GRIDS[g]
        gm = GM(logw[g], mean[g], scale[g], op.active(), op.K)
        ph0 = np.array([oracle_phi(op, x, n) for x in xi[ids]])
        rx, rphi, racc = gmpcn_moves(op, n, xi[ids], ph0, gm, beta[g], tau[g], n_moves, seed, ctr, ids=ids)
        assert np.array_equal(gacc[ids], racc), (g, gacc[ids], racc)
        assert np.abs(gx[ids] - rx).max() <= 1e-10 * np.abs(rx).max()
        assert np.abs(gphi[ids] / rphi - 1).max() <= 1e-9
    assert 0 < gacc.sum() < N * n_moves


def test_stage_equals_scalar_move_with_levels():
    """Equal parameters in every group: smc_gmpcn_stage and smc_gmpcn_move with the same level
    map produce the same bits."""
    from paper_2503_16028_amd import smc
    banner("stage vs scalar move")
    d, op = load("c5")
    lv = np.array([1, 0, 0, 1, 0, 0, 1, 0, 0, 0], dtype=np.int32)
    N, M = len(lv), 2
    p = mixed_problem(d, N, "fp32_refine")
    xi = inputs.particles(N, op.K, 44) * 0.3
    lw, mu, sc = inputs.mixture(M, op.kr, 45, spread=0.5)
    L = t(lv, torch.int32)
    Gm = torch.empty(N, op.n_obs, dtype=torch.float64, device=DEV)
    phi0 = torch.empty(N, dtype=torch.float64, device=DEV)
    smc.smc_forward_batch(p, N, t(xi), L, smc.SMC_FP32_REFINE, Gm)
    smc.smc_potential(p, N, Gm, phi0)
    Xa, Pa, Aa = t(xi), phi0.clone(), torch.empty(N, dtype=torch.int32, device=DEV)
    smc.smc_gmpcn_move(p, N, (t(lw), t(mu), t(sc)), 0.3, 2e-3, 3, 9, 700, L, smc.SMC_FP32_REFINE, Xa, Pa, Aa)
    Xb, Pb, Ab = t(xi), phi0.clone(), torch.empty(N, dtype=torch.int32, device=DEV)
    G3 = 3
    sd = smc.stage_desc(G3, t(np.tile(lw, (G3, 1))), t(np.tile(mu, (G3, 1, 1))), t(np.tile(sc, (G3, 1, 1))),
                        t(np.full(G3, 0.3)), t(np.full(G3, 2e-3)), torch.tensor([700], dtype=torch.int64, device=DEV),
                        9)
    smc.smc_gmpcn_stage(p, N, L, sd, 3, smc.SMC_FP32_REFINE, Xb, Pb, Ab)
    torch.cuda.synchronize()
    assert torch.equal(Xa, Xb) and torch.equal(Pa, Pb) and torch.equal(Aa, Ab)
    assert 0 < Aa.sum().item()


def test_stage_bad_parameters_keep_state():
    from paper_2503_16028_amd import smc
    banner("stage bad parameters")
    d, op = load("c5")
    lv = np.array([0, 1, 0, 0], dtype=np.int32)
    N, M = len(lv), 1
    p = mixed_problem(d, N, "fp32_refine")
    xi = inputs.particles(N, op.K, 46) * 0.3
    L = t(lv, torch.int32)
    phi = torch.zeros(N, dtype=torch.float64, device=DEV)
    X = t(xi)
    acc = torch.empty(N, dtype=torch.int32, device=DEV)
    sd = smc.stage_desc(3, t(np.zeros((3, M))), t(np.zeros((3, M, op.kr))), t(np.ones((3, M, op.kr))),
                        t([0.5, 1.5, 0.5]), t([0.0, 0.0, 0.0]), torch.tensor([0], dtype=torch.int64, device=DEV), 1)
    smc.smc_gmpcn_stage(p, N, L, sd, 2, smc.SMC_FP32_REFINE, X, phi, acc)
    torch.cuda.synchronize()
    a = acc.cpu().numpy()
    assert a[1] == 0 and np.array_equal(X.cpu().numpy()[1], xi[1])
    assert (a[[0, 2, 3]] == 2).all()            # tau = 0 and Phi = 0: plain pCN accepts every move
    assert smc.smc_status_flags(p) & smc.FLAG_BADPARAM


def test_stage_graph_replays_match_eager():
    """The captured stage replayed three times, with tau, beta and the counter changed on the
    device between replays and eager work in between; each replay equals an eager run from the
    same state, bit for bit."""
    from paper_2503_16028_amd import smc
    banner("stage graph replay")
    d, op = load("c5")
    lv = np.array([1, 0, 0, 1, 0, 0, 0, 1], dtype=np.int32)
    N, M, n_moves = len(lv), 2, 2
    p = mixed_problem(d, N, "fp32_refine")
    xi = inputs.particles(N, op.K, 47) * 0.3
    logw, mean, scale = group_mixture(op, 3, M, 48)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        L = t(lv, torch.int32)
        Xg = t(xi)
        Gm = torch.empty(N, op.n_obs, dtype=torch.float64, device=DEV)
        Pg = torch.empty(N, dtype=torch.float64, device=DEV)
        smc.smc_forward_batch(p, N, Xg, L, smc.SMC_FP32_REFINE, Gm)
        smc.smc_potential(p, N, Gm, Pg)
        Ag = torch.empty(N, dtype=torch.int32, device=DEV)
        beta = t([0.3, 0.25, 0.3])
        tau = t([1e-3, 1e-3, 1e-3])
        ctr = torch.tensor([100], dtype=torch.int64, device=DEV)
        sd = smc.stage_desc(3, t(logw), t(mean), t(scale), beta, tau, ctr, 77)
        s.synchronize()
        graph = smc.StageGraph(p, N, L, sd, n_moves, smc.SMC_FP32_REFINE, Xg, Pg, Ag, s)
        Xr = torch.empty_like(Xg)
        Pr = torch.empty_like(Pg)
        Ar = torch.empty_like(Ag)
        total = 0
        for rep in range(3):
            tau.mul_(2.0)
            beta.sub_(0.05)
            ctr.add_(1 << 20)
            Xr.copy_(Xg)
            Pr.copy_(Pg)
            smc.smc_gmpcn_stage(p, N, L, sd, n_moves, smc.SMC_FP32_REFINE, Xr, Pr, Ar, s)
            graph.launch(s)
            s.synchronize()
            assert torch.equal(Xg, Xr) and torch.equal(Pg, Pr) and torch.equal(Ag, Ar), rep
            total += int(Ag.sum().item())
        graph.close()
    assert total > 0
    assert smc.smc_status_flags(p) == 0


def test_levels_converge_second_order():
    """The same xi on the three nested grids in one launch: successive differences of G and Phi
    shrink by four per halving of h, with the ratios the oracle's direct solves give."""
    from paper_2503_16028_amd import smc
    banner("levels converge second order")
    d, op = load("c5")
    xi1 = inputs.particles(2, op.K, 49)
    xi = np.repeat(xi1, 3, axis=0)
    lv = np.tile(np.arange(3, dtype=np.int32), 2)
    N = len(lv)
    p = mixed_problem(d, N, "fp32_refine")
    G = torch.empty(N, op.n_obs, dtype=torch.float64, device=DEV)
    phi = torch.empty(N, dtype=torch.float64, device=DEV)
    smc.smc_forward_batch(p, N, t(xi), t(lv, torch.int32), smc.SMC_FP32_REFINE, G)
    smc.smc_potential(p, N, G, phi)
    torch.cuda.synchronize()
    g, ph = G.cpu().numpy().reshape(2, 3, -1), phi.cpu().numpy().reshape(2, 3)
    for k in range(2):
        r = np.linalg.norm(g[k, 0] - g[k, 1]) / np.linalg.norm(g[k, 1] - g[k, 2])
        rp = (ph[k, 0] - ph[k, 1]) / (ph[k, 1] - ph[k, 2])
        ref = [observe(op, solve(op, synthesize(op, xi1[k], n), n), n) for n in GRIDS]
        rr = np.linalg.norm(ref[0] - ref[1]) / np.linalg.norm(ref[1] - ref[2])
        assert 3.8 < r < 4.2 and 3.8 < rp < 4.2, (k, r, rp)
        assert abs(r / rr - 1) < 1e-3, (k, r, rr)


def test_parked_particles_keep_their_state():
    """Level SMC_LEVEL_PARKED: a forward call gives NaN rows and iters = -1 without a flag; a stage
    leaves parked particles as they are (n_acc = 0) and gives every other particle the bits it
    gets when nothing is parked."""
    from paper_2503_16028_amd import smc
    banner("parked particles")
    d, op = load("c5")
    home = np.array([0, 1, 2, 0, 1, 0, 2, 1], dtype=np.int32)
    parked = home.copy()
    parked[[1, 2, 5]] = smc.LEVEL_PARKED
    N, M, n_moves = len(home), 2, 2
    p = mixed_problem(d, N, "fp32_refine")
    xi = inputs.particles(N, op.K, 50) * 0.3
    G = torch.empty(N, op.n_obs, dtype=torch.float64, device=DEV)
    it = torch.empty(N, dtype=torch.int32, device=DEV)
    smc.smc_status_flags(p)
    smc.smc_forward_batch(p, N, t(xi), t(parked, torch.int32), smc.SMC_FP32_REFINE, G, it)
    torch.cuda.synchronize()
    g, i = G.cpu().numpy(), it.cpu().numpy()
    assert smc.smc_status_flags(p) == 0
    assert np.isnan(g[[1, 2, 5]]).all() and (i[[1, 2, 5]] == -1).all()
    assert np.isfinite(g[parked >= 0]).all() and (i[parked >= 0] > 0).all()
    phi0 = torch.empty(N, dtype=torch.float64, device=DEV)
    smc.smc_forward_batch(p, N, t(xi), t(home, torch.int32), smc.SMC_FP32_REFINE, G)
    smc.smc_potential(p, N, G, phi0)
    logw, mean, scale = group_mixture(op, 3, M, 51)
    sd = smc.stage_desc(3, t(logw), t(mean), t(scale), t([0.3, 0.3, 0.3]), t([1e-3, 1e-3, 1e-3]),
                        torch.tensor([900], dtype=torch.int64, device=DEV), 13)
    out = []
    for lv in (home, parked):
        X, P, A = t(xi), phi0.clone(), torch.empty(N, dtype=torch.int32, device=DEV)
        smc.smc_gmpcn_stage(p, N, t(lv, torch.int32), sd, n_moves, smc.SMC_FP32_REFINE, X, P, A)
        torch.cuda.synchronize()
        out.append((X.cpu().numpy(), P.cpu().numpy(), A.cpu().numpy()))
    assert smc.smc_status_flags(p) == 0
    (xh, ph, ah), (xp, pp, ap) = out
    keep = parked >= 0
    assert np.array_equal(xh[keep], xp[keep]) and np.array_equal(ph[keep], pp[keep]) and np.array_equal(ah[keep], ap[keep])
    assert np.array_equal(xp[~keep], xi[~keep]) and np.array_equal(pp[~keep], phi0.cpu().numpy()[~keep])
    assert (ap[~keep] == 0).all() and ah[~keep].sum() > 0 and ah[keep].sum() > 0


def test_mixed_sampler_replays_the_oracle_runs():
    """Three samplers on 64^2, 128^2 and 256^2 run to temperature 1 by MixedSampler: the 64^2 and
    128^2 samplers replay the oracle's runs on their grids from the same seed (the same
    temperatures, step sizes, accept rates, log Z and final clouds); every sampler reaches 1 and
    keeps its cloud from then on; the captured and the eager stage give the same bits."""
    from paper_2503_16028_amd import smc
    from paper_2503_16028_amd.sampler import MixedSampler
    from oracle import smc as osmc
    from oracle.moves import prior_sample
    banner("mixed sampler replay fp64")
    d, op = load("c5")
    counts, M, n_moves, seed = (32, 8, 4), 4, 2, 5
    N = sum(counts)
    p = mixed_problem(d, N, "fp64")
    runs = []
    for graph in (True, False):
        ms = MixedSampler(p, counts, M, n_moves, prec=smc.SMC_FP64, seed=seed, graph=graph)
        ms.initialise()
        frozen = {}
        for _ in range(200):
            before = list(ms.running)
            left = ms.step()
            for g in before:
                if g not in ms.running:
                    r = ms.rows(g)
                    frozen[g] = (ms.xi[r].cpu().numpy().copy(), ms.phi[r].cpu().numpy().copy())
            if left == 0:
                break
        res = [dict(xi=ms.xi[ms.rows(g)].cpu().numpy(), phi=ms.phi[ms.rows(g)].cpu().numpy(), log_Z=ms.log_Z[g],
                    history=ms.history[g]) for g in range(3)]
        ms.close()
        assert smc.smc_status_flags(p) == 0 and int(ms.flags.item()) == 0
        for g in range(3):
            assert res[g]["history"][-1]["tau"] == 1.0
            assert np.array_equal(res[g]["xi"], frozen[g][0]) and np.array_equal(res[g]["phi"], frozen[g][1])
        runs.append(res)
    for g in range(3):
        assert np.array_equal(runs[0][g]["xi"], runs[1][g]["xi"]) and runs[0][g]["log_Z"] == runs[1][g]["log_Z"]
    xi_all = prior_sample(op.K, N, seed, 0)
    for g in (0, 1):
        r = slice(sum(counts[:g]), sum(counts[:g + 1]))
        ids = np.arange(N)[r]
        ref = osmc.run(op, GRIDS[g], counts[g], M=M, n_moves=n_moves, rho=0.5, beta0=0.2, seed=seed, xi0=xi_all[r],
                       ids=ids, ctr_off=g)
        out = runs[0][g]
        taus = [0.0] + [h["tau"] for h in out["history"]]
        assert len(taus) == len(ref["taus"]) and np.allclose(taus, ref["taus"], rtol=1e-9, atol=1e-12), g
        assert [h["beta"] for h in out["history"]] == ref["betas"], g
        assert np.allclose([h["rate"] for h in out["history"]], ref["rates"], rtol=0, atol=0), g
        assert out["log_Z"] == pytest.approx(ref["log_Z"], abs=1e-8)
        assert np.abs(out["xi"] - ref["xi"]).max() <= 1e-7 * np.abs(ref["xi"]).max(), g
