"""Parity of every C ABI call with the oracle on identical seeded inputs (GPU).

Tolerances, element-wise: FP64 path 1e-10 relative (the observed states are positive, so every
element has a relative error; particle coefficients, which cross zero, 1e-10 relative above 1 in
magnitude and absolute below); FP32+refinement: observations 1e-9 relative, potentials 1e-4
relative; integer work (resampling indices, accept counts) bit-exact.
"""
import json
import math
import sys

import numpy as np
import pytest
import torch

import inputs
from conftest import golden
from oracle import philox
from oracle.forward import observe, potential, solve
from oracle.moves import GM, gmpcn_moves, pcn_gm
from oracle.problem import Problem as OProblem, synthesize
from oracle.resample import systematic, systematic_at
from oracle.temper import temper

pytestmark = pytest.mark.gpu
DEV = "cuda"


def banner(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def load(name):
    d = json.load(open(golden("problem_%s.json" % name)))
    return d, OProblem(d)


def gpu_problem(d, n_max, grids=None, **kw):
    from paper_2503_16028_amd import smc
    return smc.Problem(d, n_max, grids=grids, **kw)


def t(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def oracle_G(op, xi, n):
    return np.array([observe(op, solve(op, synthesize(op, x, n), n), n) for x in xi])


@pytest.fixture(scope="module", autouse=True)
def _lib():
    from paper_2503_16028_amd import smc
    smc.lib()
    assert torch.cuda.is_available()


# ------------------------------------------------------------------ synthesis and draws

@pytest.mark.parametrize("name,grid,N", [("t2", 16, 5), ("t2", 32, 4), ("t2", 64, 3), ("c2", 64, 3), ("c3", 128, 3),
                                         ("c5", 256, 2), ("t1", 64, 4), ("c1", 64, 3)])
def test_synthesis(name, grid, N):
    from paper_2503_16028_amd import smc
    banner("synthesis", name, grid, N)
    d, op = load(name)
    p = gpu_problem(d, N, grids=[grid])
    xi = inputs.particles(N, op.K, 1)
    u = torch.empty(N, (grid + 1) ** op.dim, dtype=torch.float64, device=DEV)
    smc.smc_synthesize(p, N, t(xi), 0, u)
    torch.cuda.synchronize()
    got = u.cpu().numpy()
    for k in range(N):
        U = synthesize(op, xi[k], grid)
        ref = U.T.reshape(-1) if op.dim == 2 else U
        assert np.abs(got[k] - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())


def test_synthesis_full_batch_sampled():
    """The metric workload's launch shape (128^2, 32 x 32 modes, 4096 particles, one workgroup per
    particle): eight particles spread over the batch against the oracle's synthesis."""
    from paper_2503_16028_amd import smc
    banner("synthesis full batch 128 4096")
    d, op = load("c3")
    N = 4096
    p = gpu_problem(d, N)
    xi = inputs.particles(N, op.K, 31)
    u = torch.empty(N, 129 * 129, dtype=torch.float64, device=DEV)
    smc.smc_synthesize(p, N, t(xi), 0, u)
    torch.cuda.synchronize()
    for k in (0, 1, 255, 256, 1023, 2048, 4094, 4095):
        ref = synthesize(op, xi[k], 128).T.reshape(-1)
        got = u[k].cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max()), k


@pytest.mark.parametrize("kl,grid", [(1, 16), (5, 32), (31, 64), (17, 128)])
def test_synthesis_odd_mode_counts(kl, grid):
    """Mode counts other than the padded 32 (odd ones included): the even/odd split of the
    products and the zero padding of the coefficient tile, against the oracle's synthesis."""
    from paper_2503_16028_amd import smc
    banner("synthesis kl", kl, grid)
    d, _ = load("t2")
    d = dict(d, kl_per_axis=kl, kr=min(12, kl * kl))
    op = OProblem(d)
    N = 3
    p = gpu_problem(d, N, grids=[grid])
    xi = inputs.particles(N, op.K, 7)
    u = torch.empty(N, (grid + 1) ** 2, dtype=torch.float64, device=DEV)
    smc.smc_synthesize(p, N, t(xi), 0, u)
    torch.cuda.synchronize()
    got = u.cpu().numpy()
    for k in range(N):
        ref = synthesize(op, xi[k], grid).T.reshape(-1)
        assert np.abs(got[k] - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())


def test_prior_sample_matches_generator():
    from paper_2503_16028_amd import smc
    banner("prior sample")
    d, op = load("c3")
    N = 33
    p = gpu_problem(d, N)
    xi = torch.empty(N, op.K, dtype=torch.float64, device=DEV)
    smc.smc_prior_sample(p, N, 2503, 17, xi)
    ref = philox.normals(2503, 17, np.arange(N), op.K)
    assert np.abs(xi.cpu().numpy() - ref).max() < 1e-13


# ------------------------------------------------------------------ forward map and potential

FWD_CASES = [("t2", 16, 13), ("t2", 32, 13), ("t2", 64, 7), ("c2", 64, 5), ("c3", 128, 4), ("c5", 256, 2)]
# FP64 residual tolerance each grid can certify: evaluating f - A w in FP64 carries rounding of
# about eps |A| |w| / |f|, and |A| grows like 8 / h^2 (1e-12 relative at 128^2)
TOL64 = {16: 1e-13, 32: 1e-13, 64: 1e-13, 128: 2e-12, 256: 6e-12}


@pytest.mark.parametrize("name,grid,N", FWD_CASES)
def test_forward_fp64(name, grid, N):
    from paper_2503_16028_amd import smc
    banner("forward fp64", name, grid, N)
    d, op = load(name)
    p = gpu_problem(d, N, grids=[grid], tol64=TOL64[grid], max_iter=60 * grid, max_sweeps=6)
    xi = inputs.particles(N, op.K, 2)
    G = torch.empty(N, op.n_obs, dtype=torch.float64, device=DEV)
    it = torch.empty(N, dtype=torch.int32, device=DEV)
    smc.smc_forward_batch(p, N, t(xi), None, smc.SMC_FP64, G, it)
    torch.cuda.synchronize()
    ref = oracle_G(op, xi, grid)
    assert (it.cpu().numpy() > 0).all()
    assert (ref > 0).all()                              # observed states are positive (M-matrix, f = 1)
    err = np.abs(G.cpu().numpy() / ref - 1).max()       # element-wise relative
    print("[measured] forward fp64 %s %d: %.3g" % (name, grid, err), flush=True)
    assert err <= 1e-10
    assert smc.smc_status_flags(p) == 0


@pytest.mark.parametrize("name,grid,N", FWD_CASES)
def test_forward_fp32_refine(name, grid, N):
    from paper_2503_16028_amd import smc
    banner("forward fp32+refine", name, grid, N)
    d, op = load(name)
    p = gpu_problem(d, N, grids=[grid], tol64=1e-10, tol_inner=1e-5, max_iter=80 * grid)
    xi = inputs.particles(N, op.K, 3)
    G = torch.empty(N, op.n_obs, dtype=torch.float64, device=DEV)
    phi = torch.empty(N, dtype=torch.float64, device=DEV)
    it = torch.empty(N, dtype=torch.int32, device=DEV)
    smc.smc_forward_batch(p, N, t(xi), None, smc.SMC_FP32_REFINE, G, it)
    smc.smc_potential(p, N, G, phi)
    torch.cuda.synchronize()
    ref = oracle_G(op, xi, grid)
    err = np.abs(G.cpu().numpy() / ref - 1).max()       # element-wise relative
    print("[measured] forward fp32+refine %s %d: %.3g" % (name, grid, err), flush=True)
    assert err <= 1e-9
    if grid in (32, 64, 128, 256):                      # fast-Poisson preconditioner: grid-independent
        assert (it.cpu().numpy() < 60).all(), it
    ref_phi = potential(ref, op.y, op.sigma)
    assert np.abs(phi.cpu().numpy() / ref_phi - 1).max() <= 1e-4


@pytest.mark.parametrize("grid", [32, 64, 128, 256])
def test_fast_poisson_preconditioner(grid):
    """z = L^{-1} r up to a constant, against the same formula in FP64 (FP16 transforms: 4e-3 of
    the largest value).  The input is scaled by a power of two from its norm, so scaling r by 2^k
    scales z by exactly 2^k."""
    from paper_2503_16028_amd import smc
    banner("fast-Poisson preconditioner", grid)
    d, op = load("c5" if grid != 32 else "t2")
    p = gpu_problem(d, 3, grids=[grid])
    n = grid
    r = inputs.particles(3, n * n, 9).reshape(3, n, n)
    r[:, n - 1, :] = 0.0
    r[:, :, n - 1] = 0.0
    z = torch.empty(3, n, n, dtype=torch.float32, device=DEV)
    smc.smc_precond_apply(p, 0, 3, torch.tensor(r, dtype=torch.float32, device=DEV).contiguous(), z)
    torch.cuda.synchronize()
    a = np.arange(1, n)
    S = np.sqrt(2.0 / n) * np.sin(np.pi * np.outer(a, a) / n)
    lam = np.sin(np.pi * a / (2 * n)) ** 2
    got = z.cpu().numpy()
    tol = 4e-3
    for k in range(3):
        ref = S @ ((S @ r[k, :n - 1, :n - 1] @ S) / (lam[:, None] + lam[None, :])) @ S
        assert np.abs(got[k, :n - 1, :n - 1] - ref).max() <= tol * np.abs(ref).max()
        assert np.abs(got[k, n - 1, :]).max() == 0 and np.abs(got[k, :, n - 1]).max() == 0
    for e in (-30, 20):
        z2 = torch.empty_like(z)
        r2 = torch.tensor(np.ldexp(r, e), dtype=torch.float32, device=DEV).contiguous()
        smc.smc_precond_apply(p, 0, 3, r2, z2)
        torch.cuda.synchronize()
        assert np.array_equal(z2.cpu().numpy(), np.ldexp(got, e)), e


@pytest.mark.parametrize("name,grid,N", [("t2", 32, 9), ("c2", 64, 5), ("c3", 128, 4), ("c5", 256, 1)])
def test_forward_fp32_jacobi_only(name, grid, N):
    """The Jacobi-preconditioned FP32 path (the fast-Poisson one is the default on these grids)."""
    from paper_2503_16028_amd import smc
    banner("forward fp32+refine jacobi", name, grid, N)
    d, op = load(name)
    p = gpu_problem(d, N, grids=[grid], tol64=1e-10, tol_inner=1e-5, max_iter=80 * grid,
                    precond=smc.PRECOND_JACOBI)
    xi = inputs.particles(N, op.K, 8)
    G = torch.empty(N, op.n_obs, dtype=torch.float64, device=DEV)
    it = torch.empty(N, dtype=torch.int32, device=DEV)
    smc.smc_forward_batch(p, N, t(xi), None, smc.SMC_FP32_REFINE, G, it)
    torch.cuda.synchronize()
    ref = oracle_G(op, xi, grid)
    assert np.abs(G.cpu().numpy() / ref - 1).max() <= 1e-9
    assert (it.cpu().numpy() > 3 * grid).all()          # Jacobi needs O(n) iterations per decade


@pytest.mark.parametrize("name,grid,N", [("c3", 128, 2), ("c5", 256, 1)])
def test_forward_fp64_jacobi_only(name, grid, N):
    """The Jacobi-scaled FP64 global-memory path (the fast-Poisson one is the default)."""
    from paper_2503_16028_amd import smc
    banner("forward fp64 jacobi", name, grid, N)
    d, op = load(name)
    p = gpu_problem(d, N, grids=[grid], tol64=TOL64[grid], max_iter=60 * grid, max_sweeps=6,
                    precond=smc.PRECOND_JACOBI)
    xi = inputs.particles(N, op.K, 8)
    G = torch.empty(N, op.n_obs, dtype=torch.float64, device=DEV)
    it = torch.empty(N, dtype=torch.int32, device=DEV)
    smc.smc_forward_batch(p, N, t(xi), None, smc.SMC_FP64, G, it)
    torch.cuda.synchronize()
    ref = oracle_G(op, xi, grid)
    assert np.abs(G.cpu().numpy() / ref - 1).max() <= 1e-10
    assert (it.cpu().numpy() > 3 * grid).all()          # Jacobi needs O(n) iterations per decade
    assert smc.smc_status_flags(p) == 0


@pytest.mark.parametrize("name,grid", [("t1", 16), ("t1", 64), ("c1", 64)])
def test_forward_1d(name, grid):
    from paper_2503_16028_amd import smc
    banner("forward 1d", name, grid)
    d, op = load(name)
    N = 37
    p = gpu_problem(d, N, grids=[grid])
    xi = inputs.particles(N, op.K, 4)
    G = torch.empty(N, op.n_obs, dtype=torch.float64, device=DEV)
    smc.smc_forward_batch(p, N, t(xi), None, smc.SMC_FP64, G)
    torch.cuda.synchronize()
    ref = oracle_G(op, xi, grid)
    assert np.abs(G.cpu().numpy() / ref - 1).max() <= 1e-12


def test_potential():
    from paper_2503_16028_amd import smc
    banner("potential")
    d, op = load("c2")
    N = 300
    p = gpu_problem(d, N)
    G = 0.05 + 0.01 * inputs.particles(N, op.n_obs, 5)
    G[7, 3] = np.nan
    G[9, 0] = np.inf
    phi = torch.empty(N, dtype=torch.float64, device=DEV)
    smc.smc_potential(p, N, t(G), phi)
    ref = potential(G, op.y, op.sigma)
    got = phi.cpu().numpy()
    assert np.isinf(got[7]) and np.isinf(got[9])
    fin = np.isfinite(ref)
    assert np.abs(got[fin] / ref[fin] - 1).max() < 1e-13


def test_batch_invariance_and_determinism():
    """A particle solved alone gives the same bits as inside a batch, and runs repeat."""
    from paper_2503_16028_amd import smc
    banner("batch invariance")
    d, op = load("c2")
    N = 16
    p = gpu_problem(d, N)
    xi = t(inputs.particles(N, op.K, 6))
    G = torch.empty(N, op.n_obs, dtype=torch.float64, device=DEV)
    smc.smc_forward_batch(p, N, xi, None, smc.SMC_FP32_REFINE, G)
    G2 = torch.empty_like(G)
    smc.smc_forward_batch(p, N, xi, None, smc.SMC_FP32_REFINE, G2)
    one = torch.empty(1, op.n_obs, dtype=torch.float64, device=DEV)
    for k in (0, 5, 15):
        smc.smc_forward_batch(p, 1, xi[k:k + 1].contiguous(), None, smc.SMC_FP32_REFINE, one)
        assert torch.equal(one[0], G[k])
    assert torch.equal(G, G2)


def test_nonconvergence_is_reported_and_rejected():
    from paper_2503_16028_amd import smc
    banner("non-convergence")
    d, op = load("t2")
    N = 6
    p = gpu_problem(d, N, grids=[32], max_iter=3, max_sweeps=2)
    xi = t(inputs.particles(N, op.K, 7))
    G = torch.empty(N, op.n_obs, dtype=torch.float64, device=DEV)
    it = torch.empty(N, dtype=torch.int32, device=DEV)
    smc.smc_forward_batch(p, N, xi, None, smc.SMC_FP32_REFINE, G, it)
    assert (it.cpu().numpy() == -1).all() and torch.isnan(G).all()
    assert smc.smc_status_flags(p) & smc.FLAG_NOCONV
    phi = torch.zeros(N, dtype=torch.float64, device=DEV)
    n_acc = torch.empty(N, dtype=torch.int32, device=DEV)
    xi0 = xi.clone()
    smc.smc_gmpcn_move(p, N, (t([0.0]), t(np.zeros((1, op.kr))), t(np.ones((1, op.kr)))), 0.3, 1.0, 2, 1, 1,
                       None, smc.SMC_FP32_REFINE, xi, phi, n_acc)
    assert (n_acc.cpu().numpy() == 0).all() and torch.equal(xi, xi0)


# ------------------------------------------------------------------ moves

def _move_case(name, grid, N, M, beta, tau, n_moves, prec, seed):
    from paper_2503_16028_amd import smc
    d, op = load(name)
    tol = dict(tol64=1e-13, max_iter=60 * grid, max_sweeps=6) if prec == 0 else dict(tol64=1e-10)
    p = gpu_problem(d, N, grids=[grid], **tol)
    assert list(p.active) == list(op.active())
    xi0 = inputs.particles(N, op.K, seed, 0.8)
    phi0 = potential(oracle_G(op, xi0, grid), op.y, op.sigma)
    if M == 0:
        gm = pcn_gm(op.K, op.active())
    else:
        logw, mean, scale = inputs.mixture(M, op.kr, seed + 1, spread=0.5)
        gm = GM(logw, mean, scale, op.active(), op.K)
    xi = t(xi0)
    phi = t(phi0)
    n_acc = torch.empty(N, dtype=torch.int32, device=DEV)
    smc.smc_gmpcn_move(p, N, (t(gm.logw), t(gm.mean), t(gm.scale)), beta, tau, n_moves, seed, 1000 + seed, None,
                       prec, xi, phi, n_acc)
    torch.cuda.synchronize()
    rx, rphi, racc = gmpcn_moves(op, grid, xi0, phi0, gm, beta, tau, n_moves, seed, 1000 + seed)
    return xi.cpu().numpy(), phi.cpu().numpy(), n_acc.cpu().numpy(), rx, rphi, racc


@pytest.mark.parametrize("name,grid,N,M,beta,tau,n_moves", [
    ("t2", 32, 24, 3, 0.4, 0.7, 3),
    ("t2", 16, 40, 0, 0.5, 1.0, 2),       # plain pCN
    ("t2", 32, 16, 4, 1.0, 0.5, 2),       # beta = 1: mixture independence sampler
    ("t1", 64, 50, 0, 0.3, 1.0, 4),       # 1D pCN (the 1D workload's kernel)
    ("c2", 64, 6, 4, 0.2, 0.6, 2),
    ("t2", 32, 20, 16, 0.4, 0.7, 2),      # the most components: every lane of each half-wave sum
    ("t2", 16, 20, 1, 0.6, 0.8, 2),       # one component
])
def test_move_fp64(name, grid, N, M, beta, tau, n_moves):
    banner("move fp64", name, grid, N, M, beta, tau, n_moves)
    xi, phi, acc, rx, rphi, racc = _move_case(name, grid, N, M, beta, tau, n_moves, 0, 11)
    assert np.array_equal(acc, racc)
    assert 0 < acc.sum()
    # element-wise, relative for |xi| >= 1 and absolute below (coefficients cross zero)
    assert (np.abs(xi - rx) <= 1e-10 * np.maximum(1.0, np.abs(rx))).all()
    assert np.abs(phi / rphi - 1).max() <= 1e-10


def test_move_fp32_refine():
    banner("move fp32+refine")
    xi, phi, acc, rx, rphi, racc = _move_case("t2", 64, 12, 3, 0.3, 0.8, 2, 1, 12)
    assert np.array_equal(acc, racc)
    assert np.abs(phi / rphi - 1).max() <= 1e-4


# ------------------------------------------------------------------ tempering and resampling

@pytest.mark.parametrize("N,tau", [(1, 0.0), (7, 0.3), (1000, 0.0), (4096, 0.55), (8193, 0.2), (20000, 0.1),
                                   (1 << 20, 0.0)])
def test_temper(N, tau):
    """Past 8192 potentials the kernel streams them from memory on every pass instead of keeping
    them in registers: 8193, 20000 and 2^20 (the largest batch it takes) cover that path."""
    from paper_2503_16028_amd import smc
    banner("temper", N, tau)
    phi0 = inputs.potentials(N, 30 + N)
    if N > 10:
        phi0[3] = np.inf
        phi0[5] = np.nan
    h, tau_new, W, lz = (torch.empty(1, dtype=torch.float64, device=DEV) for _ in range(4))
    Wt = torch.empty(N, dtype=torch.float64, device=DEV)
    flags = torch.zeros(1, dtype=torch.int32, device=DEV)
    smc.smc_temper(N, t(phi0), t([tau]), 0.5, h, tau_new, Wt, lz, flags)
    rh, rtau, rW, rlz, stalled = temper(phi0, tau, 0.5)
    assert h.item() == pytest.approx(rh, rel=1e-10, abs=1e-300)
    assert tau_new.item() == pytest.approx(rtau, rel=1e-12)
    assert lz.item() == pytest.approx(rlz, rel=1e-10, abs=1e-10)
    Wg = Wt.cpu().numpy()
    pos = rW > 0
    assert np.array_equal(Wg[~pos], rW[~pos])           # non-finite potentials weigh exactly 0
    assert np.abs(Wg[pos] / rW[pos] - 1).max() <= 1e-10    # element-wise relative
    assert flags.item() == 0


def test_temper_edge_cases():
    from paper_2503_16028_amd import smc
    banner("temper edges")
    h, tau_new, lz = (torch.empty(1, dtype=torch.float64, device=DEV) for _ in range(3))
    W = torch.empty(64, dtype=torch.float64, device=DEV)
    flags = torch.zeros(1, dtype=torch.int32, device=DEV)
    smc.smc_temper(64, t(np.full(64, 3.0)), t([0.25]), 0.5, h, tau_new, W, lz, flags)
    assert h.item() == 0.75 and tau_new.item() == 1.0 and flags.item() == 0
    stall = np.full(64, 1e308)
    stall[3] = 0.0
    smc.smc_temper(64, t(stall), t([0.0]), 0.5, h, tau_new, W, lz, flags)
    assert h.item() == 0.0 and flags.item() & smc.FLAG_STALL
    flags.zero_()
    smc.smc_temper(64, t(np.full(64, np.inf)), t([0.0]), 0.5, h, tau_new, W, lz, flags)
    assert flags.item() & smc.FLAG_NONFINITE
    flags.zero_()                                     # already at temperature 1: a zero step, no stall
    smc.smc_temper(64, t(inputs.potentials(64, 80)), t([1.0]), 0.5, h, tau_new, W, lz, flags)
    assert h.item() == 0.0 and tau_new.item() == 1.0 and flags.item() == 0
    assert np.allclose(W.cpu().numpy(), 1.0 / 64, rtol=1e-14)


@pytest.mark.parametrize("N", [1, 7, 1000, 4096, 16384, 20000, 1 << 20])
@pytest.mark.parametrize("kind", ["dirichlet", "sparse", "one", "uniform"])
def test_resample_bit_exact(N, kind):
    from paper_2503_16028_amd import smc
    banner("resample", N, kind)
    W = inputs.weights(N, N + 3, kind)
    u = inputs.u53(N)
    idx = torch.empty(N, dtype=torch.int32, device=DEV)
    smc.smc_resample(N, t(W), u, idx)
    assert idx.cpu().numpy().tolist() == systematic(W, u)


def test_resample_largest_batch():
    """N = 2^24, the largest batch: 4096 outputs spread over the batch (the first and last
    included) against the oracle one by one, and every particle's copy count within one of
    N q_n / Q, the property of systematic resampling at any size."""
    from paper_2503_16028_amd import smc
    banner("resample 2^24")
    N = 1 << 24
    W = inputs.weights(N, 2024, "dirichlet")
    u = inputs.u53(N)
    idx = torch.empty(N, dtype=torch.int32, device=DEV)
    flags = torch.zeros(1, dtype=torch.int32, device=DEV)
    smc.smc_resample(N, t(W), u, idx, flags)
    got = idx.cpu().numpy()
    assert flags.item() == 0
    outs = sorted(set(np.linspace(0, N - 1, 4096).astype(np.int64).tolist()))
    assert got[outs].tolist() == systematic_at(W, u, outs)
    assert np.all(np.diff(got) >= 0)
    q = np.floor(W * 2.0 ** 53)
    expect = N * q / q.sum()
    counts = np.bincount(got, minlength=N)
    assert np.all(np.abs(counts - expect) < 1.0 + 1e-6)


@pytest.mark.parametrize("case", ["above_one", "negative", "nan", "inf", "sum_too_large", "exp_weights", "zero"])
def test_resample_rejects_weights_it_cannot_quantise(case):
    """Weights must be normalised (each in [0, 1], total at most 1 + 2N 2^-53): anything else sets
    SMC_FLAG_BADWEIGHTS and gives the identity, instead of a wrapped integer CDF."""
    from paper_2503_16028_amd import smc
    banner("resample rejects", case)
    N = 4096
    W = inputs.weights(N, 77, "dirichlet")
    if case == "above_one":
        W[100] = 1.5
    elif case == "negative":
        W[5] = -W[5]
    elif case == "nan":
        W[4095] = np.nan
    elif case == "inf":
        W[0] = np.inf
    elif case == "sum_too_large":
        W = W * (1.0 + 1e-9)
    elif case == "exp_weights":                       # exp(-h (Phi - Phi_min)) in (0, 1], not normalised
        W = np.exp(-0.01 * inputs.potentials(N, 78))
        W /= W.max()
    else:
        W[:] = 0.0
    idx = torch.empty(N, dtype=torch.int32, device=DEV)
    flags = torch.zeros(1, dtype=torch.int32, device=DEV)
    smc.smc_resample(N, t(W), inputs.u53(N), idx, flags)
    assert flags.item() == smc.FLAG_BADWEIGHTS
    assert np.array_equal(idx.cpu().numpy(), np.arange(N))


def test_resample_accepts_normalisation_rounding():
    """A total just inside the bound 1 + 2N 2^-53 is still resampled, bit-exact with the oracle."""
    from paper_2503_16028_amd import smc
    banner("resample rounding slack")
    N = 1000
    W = inputs.weights(N, 79, "dirichlet")
    W[np.argmax(W)] += N * 2.0 ** -53
    u = inputs.u53(N + 1)
    idx = torch.empty(N, dtype=torch.int32, device=DEV)
    flags = torch.zeros(1, dtype=torch.int32, device=DEV)
    smc.smc_resample(N, t(W), u, idx, flags)
    assert flags.item() == 0
    assert idx.cpu().numpy().tolist() == systematic(W, u)


def test_gather():
    from paper_2503_16028_amd import smc
    banner("gather")
    N, K = 500, 1024
    W = inputs.weights(N, 40)
    idx = torch.empty(N, dtype=torch.int32, device=DEV)
    smc.smc_resample(N, t(W), inputs.u53(40), idx)
    xi = t(inputs.particles(N, K, 41))
    phi = t(inputs.potentials(N, 42))
    xo = torch.empty_like(xi)
    po = torch.empty_like(phi)
    smc.smc_gather(N, K, idx, xi, phi, xo, po)
    ii = idx.long().cpu()
    assert torch.equal(xo.cpu(), xi.cpu()[ii]) and torch.equal(po.cpu(), phi.cpu()[ii])


# ------------------------------------------------------------------ full size, sampled

def test_full_size_metric_configuration_sampled():
    """128^2, N = 4096, FP32 + refinement at the benchmark's tolerances (inner 1e-3, outer 1e-10),
    in the launch configuration the benchmark times: one move for every particle; 64 particles
    spread over the batch replayed by the oracle."""
    from paper_2503_16028_amd import smc
    banner("full size 128^2 N=4096")
    d, op = load("c3")
    N = 4096
    p = gpu_problem(d, N, tol64=1e-10, tol_inner=1e-3)
    xi = torch.empty(N, op.K, dtype=torch.float64, device=DEV)
    smc.smc_prior_sample(p, N, 2503, 0, xi)
    G = torch.empty(N, op.n_obs, dtype=torch.float64, device=DEV)
    it = torch.empty(N, dtype=torch.int32, device=DEV)
    phi = torch.empty(N, dtype=torch.float64, device=DEV)
    smc.smc_forward_batch(p, N, xi, None, smc.SMC_FP32_REFINE, G, it)
    smc.smc_potential(p, N, G, phi)
    xi_h = philox.normals(2503, 0, np.arange(N), op.K)   # the oracle's own draws of the same counters
    assert np.abs(xi.cpu().numpy() - xi_h).max() < 1e-13
    phi_h = phi.cpu().numpy()
    assert (it.cpu().numpy() > 0).all() and np.isfinite(phi_h).all()
    pick = sorted(set(np.linspace(0, N - 1, 62).astype(int).tolist()) | {1, 777})
    ref = potential(oracle_G(op, xi_h[pick], 128), op.y, op.sigma)
    assert np.abs(phi_h[pick] / ref - 1).max() <= 1e-4
    logw, mean, scale = inputs.mixture(8, op.kr, 43, spread=0.5)
    n_acc = torch.empty(N, dtype=torch.int32, device=DEV)
    smc.smc_gmpcn_move(p, N, (t(logw), t(mean), t(scale)), 0.2, 0.05, 1, 9, 500, None, smc.SMC_FP32_REFINE, xi,
                       phi, n_acc)
    gm = GM(logw, mean, scale, op.active(), op.K)
    rx, rphi, racc = gmpcn_moves(op, 128, xi_h[pick], ref, gm, 0.2, 0.05, 1, 9, 500, ids=pick)   # oracle's own Phi
    assert np.array_equal(n_acc.cpu().numpy()[pick], racc)
    assert np.abs(xi.cpu().numpy()[pick] - rx).max() <= 1e-6
    assert np.abs(phi.cpu().numpy()[pick] / rphi - 1).max() <= 1e-4


def test_batch_with_offsets_beyond_2_31_elements():
    """128^2 with N = 131072 (about 190 GB of workspace): the node fields of particles past
    129050 start beyond element 2^31 of their arrays (131071 x 16641 = 2.18e9), so an offset kept
    in 32 bits anywhere on the path would wrap.  Prior draw, forward map, potential and one pCN-GM
    move for the whole batch; particles at both ends replayed by the oracle."""
    from paper_2503_16028_amd import smc
    banner("batch offsets beyond 2^31: 128^2 N=131072")
    d, op = load("c3")
    N = 131072
    pick = [0, 65535, 129049, 129051, 131070, 131071]
    assert pick[-1] * 129 * 129 > 2 ** 31
    p = gpu_problem(d, N, tol64=1e-10, tol_inner=1e-3)
    xi = torch.empty(N, op.K, dtype=torch.float64, device=DEV)
    smc.smc_prior_sample(p, N, 2503, 0, xi)
    G = torch.empty(N, op.n_obs, dtype=torch.float64, device=DEV)
    it = torch.empty(N, dtype=torch.int32, device=DEV)
    phi = torch.empty(N, dtype=torch.float64, device=DEV)
    smc.smc_forward_batch(p, N, xi, None, smc.SMC_FP32_REFINE, G, it)
    smc.smc_potential(p, N, G, phi)
    torch.cuda.synchronize()
    xi_h = philox.normals(2503, 0, np.array(pick), op.K)
    assert np.abs(xi[pick].cpu().numpy() - xi_h).max() < 1e-13
    assert (it.cpu().numpy() > 0).all()
    ref = potential(oracle_G(op, xi_h, 128), op.y, op.sigma)
    assert np.abs(phi[pick].cpu().numpy() / ref - 1).max() <= 1e-4
    logw, mean, scale = inputs.mixture(8, op.kr, 43, spread=0.5)
    n_acc = torch.empty(N, dtype=torch.int32, device=DEV)
    smc.smc_gmpcn_move(p, N, (t(logw), t(mean), t(scale)), 0.2, 0.05, 1, 9, 500, None, smc.SMC_FP32_REFINE, xi,
                       phi, n_acc)
    gm = GM(logw, mean, scale, op.active(), op.K)
    rx, rphi, racc = gmpcn_moves(op, 128, xi_h, ref, gm, 0.2, 0.05, 1, 9, 500, ids=pick)
    assert np.array_equal(n_acc[pick].cpu().numpy(), racc)
    assert np.abs(xi[pick].cpu().numpy() - rx).max() <= 1e-6
    assert np.abs(phi[pick].cpu().numpy() / rphi - 1).max() <= 1e-4
    assert smc.smc_status_flags(p) == 0
    del xi, G, it, phi, n_acc
    p.close()
    torch.cuda.empty_cache()


def test_global_solver_vectors_beyond_2_31_elements():
    """256^2 with N = 4800: the global-memory solver's CG vectors (7 x 65536 values per particle)
    of particles past 4681 start beyond element 2^31 of their array.  Forward map of the batch
    (FP32 with refinement), particles at both ends against the oracle."""
    from paper_2503_16028_amd import smc
    banner("global solver vectors beyond 2^31: 256^2 N=4800")
    d, op = load("c5")
    N = 4800
    pick = [0, 4681, 4799]
    assert pick[-1] * 7 * 256 * 256 > 2 ** 31
    p = gpu_problem(d, N, grids=[256], tol64=1e-10, tol_inner=1e-3)
    xi = torch.empty(N, op.K, dtype=torch.float64, device=DEV)
    smc.smc_prior_sample(p, N, 77, 0, xi)
    G = torch.empty(N, op.n_obs, dtype=torch.float64, device=DEV)
    it = torch.empty(N, dtype=torch.int32, device=DEV)
    smc.smc_forward_batch(p, N, xi, None, smc.SMC_FP32_REFINE, G, it)
    torch.cuda.synchronize()
    assert (it.cpu().numpy() > 0).all()
    xi_h = philox.normals(77, 0, np.array(pick), op.K)
    assert np.abs(xi[pick].cpu().numpy() - xi_h).max() < 1e-13
    ref = oracle_G(op, xi_h, 256)
    assert np.abs(G[pick].cpu().numpy() / ref - 1).max() <= 1e-9
    assert smc.smc_status_flags(p) == 0
    del xi, G, it
    p.close()
    torch.cuda.empty_cache()
