"""smc_gm_fit_noalloc (the mixture fit on the library's static workspace, for callers that cannot
allocate) against smc_gm_fit (the same fit on a problem's workspace), through the C ABI.

Two calls in a row on one device, the second with fewer particles, components and coordinates, so
the second runs on what the first left in the shared array; each must give the bits the
problem-based call gives (the same kernels in the same order), and sizes beyond the static
array's are refused before anything runs.
"""
import sys

import numpy as np
import pytest
import torch

import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda"


def banner(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def fit_both(p, xi, active, M, iters, seed, ctr):
    from paper_2503_16028_amd import smc
    N, K = xi.shape
    kr = active.numel()
    outs = []
    for which in ("problem", "noalloc"):
        logw = torch.full((M,), np.nan, dtype=torch.float64, device=DEV)
        mean = torch.full((M, kr), np.nan, dtype=torch.float64, device=DEV)
        scale = torch.full((M, kr), np.nan, dtype=torch.float64, device=DEV)
        centers = torch.full((M,), -1, dtype=torch.int32, device=DEV)
        if which == "problem":
            smc.smc_gm_fit(p, N, xi, M, iters, 1e-3, seed, ctr, logw, mean, scale, centers)
        else:
            smc.smc_gm_fit_noalloc(N, K, active, xi, M, iters, 1e-3, seed, ctr, logw, mean, scale, centers)
        torch.cuda.synchronize()
        outs.append([a.cpu().numpy() for a in (centers, logw, mean, scale)])
    return outs


def test_noalloc_fit_matches_problem_fit_twice():
    from paper_2503_16028_amd import smc
    N1 = 20000
    c = np.zeros((1, 1024))
    p = smc.L2MixProblem(1024, 64, 0.01, c, 0.1, N1)   # a problem with no grid: only the fit's workspace
    active = torch.tensor(np.asarray(p.active, dtype=np.int32), device=DEV)
    cases = [(N1, 8, 50, 3, 1 << 20), (777, 5, 20, 4, 7)]
    for N, M, iters, seed, ctr in cases:
        banner("noalloc fit", N, M, iters)
        X, *_ = inputs.clusters(N, p.kr, M, seed, sep=3.0)
        xi = inputs.particles(N, p.K, seed + 10)
        xi[:, np.asarray(p.active)] = X
        xt = torch.tensor(xi, dtype=torch.float64, device=DEV)
        (c0, w0, m0, s0), (c1, w1, m1, s1) = fit_both(p, xt, active, M, iters, seed, ctr)
        assert (c0 >= 0).all() and np.isfinite(m0).all()
        assert np.array_equal(c0, c1)
        for a, b in ((w0, w1), (m0, m1), (s0, s1)):
            assert np.array_equal(a, b)
    # a different coordinate list (the first 12 modes) with no centres output, on a fresh shape
    banner("noalloc fit, 12 coordinates")
    N, M = 513, 3
    xi = torch.tensor(inputs.particles(N, p.K, 99), dtype=torch.float64, device=DEV)
    act12 = torch.arange(12, dtype=torch.int32, device=DEV)
    lw = torch.empty(M, dtype=torch.float64, device=DEV)
    mn = torch.empty(M, 12, dtype=torch.float64, device=DEV)
    sc = torch.empty(M, 12, dtype=torch.float64, device=DEV)
    smc.smc_gm_fit_noalloc(N, p.K, act12, xi, M, 10, 1e-3, 5, 9, lw, mn, sc)
    torch.cuda.synchronize()
    assert np.isfinite(mn.cpu().numpy()).all() and (sc.cpu().numpy() >= 1e-3).all()
    assert abs(np.exp(lw.cpu().numpy()).sum() - 1.0) < 1e-12


def test_noalloc_fit_refuses_sizes_beyond_the_static_workspace():
    from paper_2503_16028_amd import smc
    banner("noalloc fit limits")
    big = smc.smc_gm_fit_noalloc_max() + 1
    assert smc.smc_gm_fit_noalloc_max() == 32768
    lib = smc.lib()
    import ctypes
    v = ctypes.c_void_p(8)
    assert lib.smc_gm_fit_noalloc(big, 1024, 64, v, v, 8, 10, 1e-3, 0, 0, v, v, v, None, None) == -1
    assert b"static workspace" in lib.smc_last_error()
    assert lib.smc_gm_fit_noalloc(100, 1024, 65, v, v, 8, 10, 1e-3, 0, 0, v, v, v, None, None) == -1
    assert lib.smc_gm_fit_noalloc(100, 1024, 64, v, v, 17, 10, 1e-3, 0, 0, v, v, v, None, None) == -1
