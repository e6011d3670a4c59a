"""Pins of the oracle's generator, prior basis and forward map (CPU only)."""
import math

import numpy as np
import pytest
import scipy.fft
import scipy.stats

from conftest import golden
from oracle import philox
from oracle.forward import darcy_matrix_2d, forward, observe, potential, solve, solve_1d, solve_2d
from oracle.problem import Problem, active_modes, basis_matrix, eigenvalues, reflect_x, synthesize


# ------------------------------------------------------------------ generator

def test_philox_known_answers():
    rows = [l.split() for l in open(golden("philox_kat.txt")) if l.strip() and not l.startswith("#")]
    for r in rows:
        v = [int(x, 16) for x in r]
        out = philox.philox4x32_10(np.array(v[:4]), np.array(v[4:6]))
        assert [int(w) for w in out] == v[6:]


def test_normals_are_standard():
    z = philox.normals(seed=7, ctr=3, particles=np.arange(64), K=1024).reshape(-1)
    assert abs(z.mean()) < 4.0 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 4.0 * math.sqrt(2.0 / z.size)
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-3


def test_draw_layout_independent_streams():
    a = philox.normals(1, 5, [0, 1], 8)
    b = philox.normals(1, 6, [0, 1], 8)
    c = philox.normals(2, 5, [0, 1], 8)
    assert not np.allclose(a, b) and not np.allclose(a, c) and not np.allclose(a[0], a[1])
    # particle ids address rows independently of which other rows are drawn
    assert np.array_equal(philox.normals(1, 5, [1], 8)[0], a[1])
    u1, u2 = philox.move_uniforms(3, 9, np.arange(4096))
    assert 0 <= u1.min() and u1.max() < 1 and abs(u2.mean() - 0.5) < 0.02


# ------------------------------------------------------------------ prior basis

def _mode(prob, idx):
    xi = np.zeros(prob.K)
    xi[idx] = 1.0 / prob.sqrt_lam[idx]
    return xi


@pytest.mark.parametrize("k,l", [(0, 0), (1, 0), (0, 3), (2, 5), (7, 1)])
def test_kl_2d_eigenpairs(k, l):
    """(I - Delta) phi_kl = lambda_kl^{-1/2} phi_kl with Neumann walls: the prior (I - Delta)^{-2}."""
    prob = Problem(dict(name="x", dim=2, grids=[64], kl_per_axis=8, obs_den=1, obs=[]))
    errs = []
    for n in (32, 64, 128):
        U = synthesize(prob, _mode(prob, k * 8 + l), n)
        h = 1.0 / n
        lap = (U[2:, 1:-1] + U[:-2, 1:-1] + U[1:-1, 2:] + U[1:-1, :-2] - 4 * U[1:-1, 1:-1]) / h ** 2
        res = (U[1:-1, 1:-1] - lap) - prob.lam[k * 8 + l] ** -0.5 * U[1:-1, 1:-1]
        errs.append(np.abs(res).max() / prob.lam[k * 8 + l] ** -0.5)
        # Neumann walls: one-sided normal derivative is O(h)
        assert np.abs(U[1, :] - U[0, :]).max() / h < 10 * (1 + k * k) * h
    assert errs[-1] < 5e-3 * (1 + k * k + l * l)
    if k + l > 0:
        assert 3.5 < errs[0] / errs[1] < 4.5          # second order in h
    # x varies with the first index k, y with the second index l
    U = synthesize(prob, _mode(prob, k * 8 + l), 64)
    x = np.arange(65) / 64
    ck = 1.0 if k == 0 else math.sqrt(2)
    cl = 1.0 if l == 0 else math.sqrt(2)
    assert np.allclose(U[:, 5], ck * np.cos(k * math.pi * x) * cl * math.cos(l * math.pi * 5 / 64), atol=1e-12)


def test_kl_2d_orthonormal():
    prob = Problem(dict(name="x", dim=2, grids=[64], kl_per_axis=6, obs_den=1, obs=[]))
    n = 240
    wts = np.full(n + 1, 1.0 / n)
    wts[0] = wts[-1] = 0.5 / n
    W2 = np.outer(wts, wts)
    F = np.stack([synthesize(prob, _mode(prob, i), n) for i in range(prob.K)])
    gram = np.einsum("aij,bij,ij->ab", F, F, W2)
    assert np.abs(gram - np.eye(prob.K)).max() < 1e-10


def test_kl_1d_eigenpairs():
    prob = Problem(dict(name="x", dim=1, grids=[64], kl_per_axis=8, obs_den=1, obs=[]))
    for k in (1, 3, 8):
        U = synthesize(prob, _mode(prob, k - 1), 256)
        h = 1 / 256
        lap = (U[2:] - 2 * U[1:-1] + U[:-2]) / h ** 2
        res = U[1:-1] - lap - prob.lam[k - 1] ** -0.5 * U[1:-1]
        assert np.abs(res).max() < 2e-3 * prob.lam[k - 1] ** -0.5 * np.abs(U).max()
        assert abs(U[0]) < 1e-15 and abs(U[-1]) < 1e-12
        assert abs(np.sum(U[:-1] ** 2) / 256 - 1.0) < 1e-10


def test_active_modes_are_the_largest():
    lam = eigenvalues(2, 32)
    act = active_modes(lam, 64)
    rest = np.setdiff1d(np.arange(lam.size), act)
    assert lam[act].min() >= lam[rest].max()
    assert list(act[:5]) == [0, 1, 32, 33, 2]          # (0,0) (0,1) (1,0) (1,1) (0,2)


def test_synthesis_matches_mode_sum():
    prob = Problem(dict(name="x", dim=2, grids=[16], kl_per_axis=5, obs_den=1, obs=[]))
    xi = np.random.default_rng(3).standard_normal(prob.K)
    U = synthesize(prob, xi, 16)
    for (i, j) in [(0, 0), (3, 11), (16, 7)]:
        x, y = i / 16, j / 16
        s = 0.0
        for k in range(5):
            for l in range(5):
                c = (1 if k == 0 else math.sqrt(2)) * (1 if l == 0 else math.sqrt(2))
                s += math.sqrt(prob.lam[k * 5 + l]) * xi[k * 5 + l] * c * math.cos(k * math.pi * x) * math.cos(l * math.pi * y)
        assert abs(U[i, j] - s) < 1e-13


# ------------------------------------------------------------------ forward map

@pytest.mark.parametrize("n", [16, 64])
def test_constant_field_matches_dst(n):
    """u = c makes A = e^c L_h; invert L_h by the DST-I diagonalisation."""
    c = 0.37
    prob = Problem(dict(name="x", dim=2, grids=[n], kl_per_axis=4, obs_den=1, obs=[]))
    xi = np.zeros(prob.K)
    xi[0] = c                                       # lambda_00 = 1, phi_00 = 1
    W = solve_2d(synthesize(prob, xi, n), n, 1.0)
    m = n - 1
    h = 1.0 / n
    p = np.arange(1, n)
    mu = 4.0 / h ** 2 * (np.sin(p * np.pi * h / 2) ** 2)
    F = scipy.fft.dstn(np.ones((m, m)), type=1)
    ref = math.exp(-c) * scipy.fft.idstn(F / (mu[:, None] + mu[None, :]), type=1)
    assert np.abs(W[1:n, 1:n] - ref).max() < 1e-13 * np.abs(ref).max() * n


def test_manufactured_solution_second_order():
    """u = 0.3 cos(pi x) cos(2 pi y), w = sin(pi x) sin(pi y), f = -div(e^u grad w)."""
    errs = []
    for n in (16, 32, 64):
        x = np.arange(n + 1) / n
        X, Y = np.meshgrid(x, x, indexing="ij")
        u = 0.3 * np.cos(np.pi * X) * np.cos(2 * np.pi * Y)
        ux = -0.3 * np.pi * np.sin(np.pi * X) * np.cos(2 * np.pi * Y)
        uy = -0.6 * np.pi * np.cos(np.pi * X) * np.sin(2 * np.pi * Y)
        w = np.sin(np.pi * X) * np.sin(np.pi * Y)
        wx = np.pi * np.cos(np.pi * X) * np.sin(np.pi * Y)
        wy = np.pi * np.sin(np.pi * X) * np.cos(np.pi * Y)
        lap = -2 * np.pi ** 2 * w
        f = -np.exp(u) * (ux * wx + uy * wy + lap)
        W = solve_2d(u, n, f)
        errs.append(np.abs(W - w).max())
    assert errs[-1] < 2e-3
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_1d_closed_form():
    """Flux F_{i+1/2} = F_{1/2} - i h f and w_{i+1} = w_i + h F_{i+1/2} / a_{i+1/2}."""
    n = 64
    U = 0.5 * np.sin(7 * np.arange(n + 1) / n) + 0.2
    W = solve_1d(U, n, 1.0)
    h = 1.0 / n
    a = [math.exp(0.5 * (U[i] + U[i + 1])) for i in range(n)]
    F0 = sum(i * h / a[i] for i in range(n)) / sum(1.0 / a[i] for i in range(n))
    w = [0.0]
    for i in range(n):
        w.append(w[-1] + h * (F0 - i * h) / a[i])
    assert abs(w[-1]) < 1e-15
    assert np.abs(W - np.array(w)).max() < 1e-14


def test_operator_symmetric_positive():
    n = 12
    U = np.random.default_rng(0).standard_normal((n + 1, n + 1)) * 0.3
    A = darcy_matrix_2d(U, n).toarray()
    assert np.abs(A - A.T).max() == 0.0
    assert np.linalg.eigvalsh(A).min() > 0


def test_fixture_data_consistent(problems):
    """Stored noise-free values are F(u_true) on the fine grid; sigma follows the 1% rule."""
    for name in ("c1", "t2"):
        p = problems[name]
        G = forward(p, np.array(p.d["xi_true"]), p.d["n_fine"])
        assert np.allclose(G, p.d["G_true_fine"], rtol=1e-12, atol=0)
        assert abs(p.sigma - 0.01 * np.abs(G).max()) < 1e-15


def test_potential_definition():
    G = np.array([[1.0, 2.0], [np.nan, 0.0]])
    out = potential(G, [0.5, 1.0], 0.5)
    assert out[0] == pytest.approx((0.25 + 1.0) / 0.5) and out[1] == np.inf


def test_mirror_symmetry_c3(problems):
    """Mirrored nodes with pair-averaged data make Phi invariant under x -> 1 - x."""
    p = problems["c3"]
    from oracle.forward import phi
    xi = np.random.default_rng(5).standard_normal(p.K)
    a = phi(p, xi, 128)
    b = phi(p, reflect_x(p, xi), 128)
    assert abs(a - b) <= 1e-9 * abs(a)
    xt = np.array(p.d["xi_true"])
    # the truth field is asymmetric, so xi_true and its mirror image are two distinct
    # points of equal potential: the posterior has two mirror modes
    assert np.linalg.norm(xt - reflect_x(p, xt)) > 1.0
    assert abs(phi(p, xt, 128) - phi(p, reflect_x(p, xt), 128)) <= 1e-9 * phi(p, xt, 128)


def test_nested_grids_converge_second_order(problems):
    """The three grids of the mixed-resolution runs nest (h = 1/64, 1/128, 1/256), so the same xi
    gives the same field at every shared node and the observations sit on nodes of each grid.
    The five-point flux discretisation is second order: successive differences of G and of Phi
    shrink by four per halving of h (Sec. 3.2 compares the resolutions by this)."""
    from oracle.forward import phi
    p = problems["c5"]
    rng = np.random.default_rng(11)
    for _ in range(2):
        xi = rng.standard_normal(p.K)
        G = [forward(p, xi, n) for n in (64, 128, 256)]
        r = np.linalg.norm(G[0] - G[1]) / np.linalg.norm(G[1] - G[2])
        ph = [phi(p, xi, n) for n in (64, 128, 256)]
        rp = (ph[0] - ph[1]) / (ph[1] - ph[2])
        assert 3.8 < r < 4.2 and 3.8 < rp < 4.2, (r, rp)
        assert np.linalg.norm(G[1] - G[2]) < 1e-3 * np.linalg.norm(G[2])
