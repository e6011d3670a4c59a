"""Adjoint gradient, forward-state checkpointing, the potential's autograd function and the
pCN-Langevin move against the oracle (GPU).

Tolerances: gradients on the FP64 path within 1e-10 of the largest oracle component, on the
FP32+refinement path within 1e-8 (both solves are refined to the FP64 tolerance; the components
span many orders of magnitude, sqrt(lambda_k) falling like 1/k^2, so the error is measured against
the largest); potentials 1e-10 relative (FP64); accept counts bit-exact.
"""
import json
import sys

import numpy as np
import pytest
import torch

import inputs
from conftest import golden
from oracle.adjoint import value_and_grad
from oracle.forward import phi as oracle_phi, solve
from oracle.moves import pcnl_moves
from oracle.problem import Problem as OProblem, synthesize

pytestmark = pytest.mark.gpu
DEV = "cuda"
TOL64 = {16: 1e-13, 32: 1e-13, 64: 1e-13, 128: 2e-12, 256: 6e-12}


def banner(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def load(name):
    d = json.load(open(golden("problem_%s.json" % name)))
    return d, OProblem(d)


def t(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def fp64_problem(d, N, grid):
    from paper_2503_16028_amd import smc
    return smc.Problem(d, N, grids=[grid], tol64=TOL64[grid], max_iter=60 * grid, max_sweeps=6)


@pytest.fixture(scope="module", autouse=True)
def _lib():
    from paper_2503_16028_amd import smc
    smc.lib()
    assert torch.cuda.is_available()


def gpu_value_and_grad(p, xi, prec, w=None):
    from paper_2503_16028_amd import smc
    N = xi.shape[0]
    phi = torch.empty(N, dtype=torch.float64, device=DEV)
    g = torch.empty(N, p.K, dtype=torch.float64, device=DEV)
    it = torch.empty(N, dtype=torch.int32, device=DEV)
    smc.smc_value_and_grad(p, N, xi, prec, w, phi, g, it)
    torch.cuda.synchronize()
    return phi.cpu().numpy(), g.cpu().numpy(), it.cpu().numpy()


GRAD_CASES = [("t2", 16, 4), ("t2", 32, 4), ("t2", 64, 3), ("c4", 128, 3), ("c5", 256, 1)]


@pytest.mark.parametrize("name,grid,N", GRAD_CASES)
def test_value_and_grad_fp64(name, grid, N):
    from paper_2503_16028_amd import smc
    banner("value_and_grad fp64", name, grid, N)
    d, op = load(name)
    p = fp64_problem(d, N, grid)
    xi = inputs.particles(N, op.K, 21)
    phi, g, it = gpu_value_and_grad(p, t(xi), smc.SMC_FP64)
    assert (it > 0).all(), it
    for k in range(N):
        rphi, rg = value_and_grad(op, xi[k], grid)
        assert abs(phi[k] / rphi - 1) <= 1e-10
        assert np.abs(g[k] - rg).max() <= 1e-10 * np.abs(rg).max(), (k, np.abs(g[k] - rg).max(), np.abs(rg).max())
    assert smc.smc_status_flags(p) == 0


@pytest.mark.parametrize("kl,grid", [(5, 64), (31, 32)])
def test_value_and_grad_odd_mode_counts(kl, grid):
    """The gradient's contraction with mode counts other than 32 (the even/odd split of its first
    product and the masked output), FP64, against the oracle's adjoint gradient."""
    from paper_2503_16028_amd import smc
    banner("value_and_grad kl", kl, grid)
    d, _ = load("t2")
    d = dict(d, kl_per_axis=kl, kr=min(12, kl * kl))
    op = OProblem(d)
    N = 2
    p = fp64_problem(d, N, grid)
    xi = inputs.particles(N, op.K, 23)
    phi, g, it = gpu_value_and_grad(p, t(xi), smc.SMC_FP64)
    assert (it > 0).all(), it
    for k in range(N):
        rphi, rg = value_and_grad(op, xi[k], grid)
        assert abs(phi[k] / rphi - 1) <= 1e-10
        assert np.abs(g[k] - rg).max() <= 1e-10 * np.abs(rg).max()


@pytest.mark.parametrize("name,grid,N", [("t2", 32, 4), ("t2", 64, 3), ("c4", 128, 3)])
def test_value_and_grad_fp32_refine(name, grid, N):
    from paper_2503_16028_amd import smc
    banner("value_and_grad fp32+refine", name, grid, N)
    d, op = load(name)
    p = smc.Problem(d, N, grids=[grid], tol64=1e-10, tol_inner=1e-5, max_iter=80 * grid)
    xi = inputs.particles(N, op.K, 22)
    phi, g, it = gpu_value_and_grad(p, t(xi), smc.SMC_FP32_REFINE)
    assert (it > 0).all() and (it < 200).all(), it     # two fast-Poisson-preconditioned solves
    for k in range(N):
        rphi, rg = value_and_grad(op, xi[k], grid)
        assert abs(phi[k] / rphi - 1) <= 1e-4
        assert np.abs(g[k] - rg).max() <= 1e-8 * np.abs(rg).max()


@pytest.mark.parametrize("name,grid", [("t2", 32), ("c4", 128)])
def test_gradient_central_differences(name, grid):
    """g . d against (Phi(xi + h d) - Phi(xi - h d)) / 2h, h = 1e-6, 16 seeded unit directions,
    with Phi from the library's FP64 forward solves; at 128^2 on the pCN-Langevin workload's
    problem.  The difference quotient carries the potentials' own error, at most 2e-12 relative
    on these grids (3e-13 measured at 128^2), amplified by Phi / h: the bound allows that on top
    of 1e-6 of the largest directional derivative."""
    from paper_2503_16028_amd import smc
    banner("central differences 16 directions", name, grid)
    d, op = load(name)
    D = 16
    p = fp64_problem(d, 2 * D + 1, grid)
    x0 = inputs.particles(1, op.K, 23)[0]
    dirs = inputs.particles(D, op.K, 24)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    h = 1e-6
    X = np.concatenate([x0[None], x0 + h * dirs, x0 - h * dirs])
    G = torch.empty(len(X), op.n_obs, dtype=torch.float64, device=DEV)
    phi = torch.empty(len(X), dtype=torch.float64, device=DEV)
    smc.smc_forward_batch(p, len(X), t(X), None, smc.SMC_FP64, G)
    smc.smc_potential(p, len(X), G, phi)
    _, g, _ = gpu_value_and_grad(p, t(x0[None]), smc.SMC_FP64)
    ph = phi.cpu().numpy()
    fd = (ph[1:D + 1] - ph[D + 1:]) / (2 * h)
    an = dirs @ g[0]
    err = np.abs(fd - an).max()
    print("[measured] central differences %s %d: max |fd - g.d| %.3g, max |g.d| %.3g, Phi %.4g" %
          (name, grid, err, np.abs(an).max(), ph[0]), flush=True)
    assert err <= 1e-6 * np.abs(an).max() + 2 * 2e-12 * ph[0] / (2 * h), (fd, an)


def test_value_and_grad_c4_full_size_sampled():
    """The pCN-Langevin workload's launch (128^2, N = 2048, FP32 + refinement at the benchmark's
    tolerances): potentials and gradients of 8 particles spread over the batch against the oracle."""
    from paper_2503_16028_amd import smc
    banner("value_and_grad c4 full size")
    d, op = load("c4")
    N = 2048
    p = smc.Problem(d, N, tol64=1e-10, tol_inner=1e-3)
    xi = inputs.particles(N, op.K, 32)
    phi, g, it = gpu_value_and_grad(p, t(xi), smc.SMC_FP32_REFINE)
    assert (it > 0).all() and smc.smc_status_flags(p) == 0
    for k in np.linspace(0, N - 1, 8).astype(int):
        rphi, rg = value_and_grad(op, xi[k], 128)
        assert abs(phi[k] / rphi - 1) <= 1e-4
        assert np.abs(g[k] - rg).max() <= 1e-8 * np.abs(rg).max()


def test_value_and_grad_crowded_column():
    """Seven observations in one column within one thread's strip of 32 rows (more point sources
    than the adjoint's residual pass keeps in its per-strip list), beside three elsewhere: the
    128^2 FP32+refinement gradient of two particles against the oracle."""
    from paper_2503_16028_amd import smc
    banner("value_and_grad crowded column")
    d, _ = load("c4")
    d = dict(d)
    d["obs"] = [[32, y] for y in range(17, 24)] + [[11, 11], [43, 53], [53, 21]]
    d["y"] = [0.03 + 0.001 * k for k in range(len(d["obs"]))]
    d.pop("G_true_fine", None)
    op = OProblem(d)
    N = 2
    p = smc.Problem(d, N, tol64=1e-10, tol_inner=1e-3)
    xi = inputs.particles(N, op.K, 33)
    phi, g, it = gpu_value_and_grad(p, t(xi), smc.SMC_FP32_REFINE)
    assert (it > 0).all() and smc.smc_status_flags(p) == 0
    for k in range(N):
        rphi, rg = value_and_grad(op, xi[k], 128)
        assert abs(phi[k] / rphi - 1) <= 1e-4
        assert np.abs(g[k] - rg).max() <= 1e-8 * np.abs(rg).max()


def test_gradient_taylor_remainder():
    """|Phi(xi + e d) - Phi(xi) - e g.d| falls as e^2."""
    from paper_2503_16028_amd import smc
    banner("taylor remainder")
    d, op = load("t2")
    grid = 32
    p = fp64_problem(d, 8, grid)
    x0 = inputs.particles(1, op.K, 25)[0] * 0.3
    dv = inputs.particles(1, op.K, 26)[0]
    dv /= np.linalg.norm(dv)
    eps = np.array([4e-2, 2e-2, 1e-2, 5e-3])
    X = np.concatenate([x0[None], x0 + eps[:, None] * dv])
    G = torch.empty(len(X), op.n_obs, dtype=torch.float64, device=DEV)
    phi = torch.empty(len(X), dtype=torch.float64, device=DEV)
    smc.smc_forward_batch(p, len(X), t(X), None, smc.SMC_FP64, G)
    smc.smc_potential(p, len(X), G, phi)
    _, g, _ = gpu_value_and_grad(p, t(x0[None]), smc.SMC_FP64)
    ph = phi.cpu().numpy()
    rem = np.abs(ph[1:] - ph[0] - eps * (g[0] @ dv))
    ratios = rem[:-1] / rem[1:]
    assert (ratios > 3.0).all() and (ratios < 5.0).all(), ratios


@pytest.mark.parametrize("prec_name", ["fp64", "fp32_refine"])
def test_forward_state_checkpoint(prec_name):
    """smc_forward_state keeps the oracle's forward solution; the gradient from the kept state
    equals, bit for bit, the gradient that solves the forward problem itself."""
    from paper_2503_16028_amd import smc
    prec = smc.PRECISIONS[prec_name]
    banner("forward state checkpoint", prec_name)
    d, op = load("c4")
    grid, N = 64, 5
    p = smc.Problem(d, N, grids=[grid], tol64=1e-12, tol_inner=1e-5, max_iter=60 * grid, max_sweeps=8)
    xi = inputs.particles(N, op.K, 27)
    w = torch.zeros(N, grid * grid, dtype=torch.float64, device=DEV)
    G = torch.empty(N, op.n_obs, dtype=torch.float64, device=DEV)
    smc.smc_forward_state(p, N, t(xi), prec, G, w)
    torch.cuda.synchronize()
    W = w.cpu().numpy().reshape(N, grid, grid)
    for k in range(N):
        ref = solve(op, synthesize(op, xi[k], grid), grid)[1:grid, 1:grid].T    # [y][x] interior
        assert np.abs(W[k, :grid - 1, :grid - 1] - ref).max() <= 1e-9 * np.abs(ref).max()
        assert np.abs(W[k, grid - 1, :]).max() == 0 and np.abs(W[k, :, grid - 1]).max() == 0
    phi_a, g_a, _ = gpu_value_and_grad(p, t(xi), prec)
    phi_b, g_b, _ = gpu_value_and_grad(p, t(xi), prec, w=w)
    assert np.array_equal(phi_a, phi_b)
    assert np.array_equal(g_a, g_b)


@pytest.mark.parametrize("mode", ["state", "recompute"])
def test_autograd_potential(mode):
    """backward of sum(c * Phi) is c * dPhi/dxi; chunks of n_max particles; both checkpoint modes
    give the same bits."""
    from paper_2503_16028_amd import autodiff, smc
    banner("autograd", mode)
    d, op = load("t2")
    grid, N = 32, 7
    p = smc.Problem(d, 3, grids=[grid], tol64=1e-12, max_iter=60 * grid)   # n_max 3 < N: chunked
    xi = inputs.particles(N, op.K, 28)
    c = inputs.particles(1, N, 29)[0]
    x = t(xi).requires_grad_(True)
    phi = autodiff.potential(p, x, smc.SMC_FP64, checkpoint=mode)
    (phi * t(c)).sum().backward()
    torch.cuda.synchronize()
    got = x.grad.cpu().numpy()
    for k in range(N):
        rphi, rg = value_and_grad(op, xi[k], grid)
        assert abs(phi[k].item() / rphi - 1) <= 1e-10
        assert np.abs(got[k] - c[k] * rg).max() <= 1e-8 * np.abs(c[k] * rg).max()
    x2 = t(xi).requires_grad_(True)
    other = "recompute" if mode == "state" else "state"
    (autodiff.potential(p, x2, smc.SMC_FP64, checkpoint=other) * t(c)).sum().backward()
    assert torch.equal(x.grad, x2.grad)


@pytest.mark.parametrize("grid,N,beta,n_moves", [(16, 6, 0.3, 3), (32, 4, 0.3, 2)])
def test_pcnl_move_fp64(grid, N, beta, n_moves):
    """pCN-Langevin moves: the same proposals, decisions and states as the oracle's."""
    from paper_2503_16028_amd import smc
    banner("pcnl fp64", grid, N, beta, n_moves)
    d, op = load("t2")
    p = fp64_problem(d, N, grid)
    xi = inputs.particles(N, op.K, 30) * 0.5
    vg = [value_and_grad(op, x, grid) for x in xi]
    phi0 = np.array([v[0] for v in vg])
    g0 = np.array([v[1] for v in vg])
    tau = float(min(1.0, 2.0 / np.median(phi0)))
    seed, ctr = 99, 1000
    rx, rphi, rg, racc = pcnl_moves(beta, tau, xi, phi0, g0, n_moves, seed, ctr,
                                    lambda v: value_and_grad(op, v, grid))
    X = t(xi)
    phi = torch.empty(N, dtype=torch.float64, device=DEV)
    g = torch.empty(N, op.K, dtype=torch.float64, device=DEV)
    smc.smc_value_and_grad(p, N, X, smc.SMC_FP64, None, phi, g)
    acc = torch.empty(N, dtype=torch.int32, device=DEV)
    smc.smc_pcnl_move(p, N, beta, tau, n_moves, seed, ctr, smc.SMC_FP64, X, phi, g, acc)
    torch.cuda.synchronize()
    assert np.array_equal(acc.cpu().numpy(), racc), (acc.cpu().numpy(), racc)
    assert 0 < racc.sum() < N * n_moves                     # some moves accepted, some rejected
    assert np.abs(X.cpu().numpy() - rx).max() <= 1e-9 * np.abs(rx).max()
    assert np.abs(phi.cpu().numpy() / rphi - 1).max() <= 1e-9
    assert np.abs(g.cpu().numpy() - rg).max() <= 1e-7 * np.abs(rg).max()


def test_pcnl_move_fp32_refine_128_sampled():
    """The 128^2 pCN-Langevin workload shape (FP32+refinement): 2 moves of 256 particles,
    three particles replayed by the oracle."""
    from paper_2503_16028_amd import smc
    banner("pcnl fp32+refine 128 sampled")
    d, op = load("c4")
    grid, N, beta, n_moves = 128, 256, 0.2, 2
    p = smc.Problem(d, N, grids=[grid], tol64=1e-10, tol_inner=1e-5)
    xi = inputs.particles(N, op.K, 31) * 0.5
    X = t(xi)
    phi = torch.empty(N, dtype=torch.float64, device=DEV)
    g = torch.empty(N, op.K, dtype=torch.float64, device=DEV)
    smc.smc_value_and_grad(p, N, X, smc.SMC_FP32_REFINE, None, phi, g)
    torch.cuda.synchronize()
    picks = (0, 101, 255)
    ref0 = {k: value_and_grad(op, xi[k], grid) for k in picks}       # the oracle's own starting points
    tau = float(min(1.0, 2.0 / np.median([ref0[k][0] for k in picks])))
    acc = torch.empty(N, dtype=torch.int32, device=DEV)
    smc.smc_pcnl_move(p, N, beta, tau, n_moves, 5, 77, smc.SMC_FP32_REFINE, X, phi, g, acc)
    torch.cuda.synchronize()
    assert smc.smc_status_flags(p) == 0
    got_acc, got_x, got_phi = acc.cpu().numpy(), X.cpu().numpy(), phi.cpu().numpy()
    assert 0 < got_acc.sum() < N * n_moves
    for k in picks:
        rphi0, rg0 = ref0[k]
        rx, rphi, _, racc = pcnl_moves(beta, tau, xi[k:k + 1], np.array([rphi0]), rg0[None], n_moves, 5, 77,
                                       lambda v: value_and_grad(op, v, grid), ids=[k])
        assert got_acc[k] == racc[0]
        assert np.abs(got_x[k] - rx[0]).max() <= 1e-6 * np.abs(rx[0]).max()
        assert abs(got_phi[k] / rphi[0] - 1) <= 1e-4
