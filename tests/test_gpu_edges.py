"""Edge cases of the boundary on the device: empty batches and rejected arguments (GPU).

The header's contract: N = 0 is a valid empty batch for the problem calls and the gather (nothing
is launched, no output changes); smc_temper and smc_resample need N >= 1; an invalid argument
returns SMC_E_INVAL with nothing launched and no output touched.  Every output below is filled
with a sentinel first and compared bit for bit afterwards.
"""
import json
import sys

import numpy as np
import pytest
import torch

import inputs
from conftest import golden

pytestmark = pytest.mark.gpu
DEV = "cuda"
SENT = 12345.678


def banner(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def t(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


@pytest.fixture(scope="module")
def setup():
    from paper_2503_16028_amd import smc
    d = json.load(open(golden("problem_t2.json")))
    N = 8
    p = smc.Problem(d, N, grids=[32])
    xi = t(inputs.particles(N, p.K, 71))
    M, kr = 2, p.kr
    gm = (t(np.log([0.4, 0.6])), t(inputs.particles(M, kr, 72, 0.3)), t(np.full((M, kr), 0.8)))
    return smc, d, p, N, xi, gm


def filled(*shape, dtype=torch.float64):
    return torch.full(shape, SENT if dtype == torch.float64 else 777, dtype=dtype, device=DEV)


def same(a, b):
    return torch.equal(a, b)


def test_empty_batches_touch_nothing(setup):
    smc, d, p, N, xi, gm = setup
    banner("empty batches")
    G = filled(N, p.n_obs)
    phi = filled(N)
    it = filled(N, dtype=torch.int32)
    acc = filled(N, dtype=torch.int32)
    grad = filled(N, p.K)
    x0 = xi.clone()
    smc.smc_forward_batch(p, 0, xi, None, smc.SMC_FP32_REFINE, G, it)
    smc.smc_potential(p, 0, G, phi)
    smc.smc_gmpcn_move(p, 0, gm, 0.3, 0.5, 2, 1, 2, None, smc.SMC_FP64, xi, phi, acc)
    smc.smc_gm_draw(p, 0, gm, 1, 3, None, smc.SMC_FP64, xi, phi, it)
    smc.smc_value_and_grad(p, 0, xi, smc.SMC_FP64, None, phi, grad, it)
    idx = torch.arange(N, dtype=torch.int32, device=DEV)
    out = filled(N, p.K)
    smc.smc_gather(0, p.K, idx, xi, None, out, None)
    torch.cuda.synchronize()
    assert smc.smc_status_flags(p) == 0
    assert same(G, filled(N, p.n_obs)) and same(phi, filled(N)) and same(grad, filled(N, p.K))
    assert same(it, filled(N, dtype=torch.int32)) and same(acc, filled(N, dtype=torch.int32))
    assert same(xi, x0) and same(out, filled(N, p.K))


def test_invalid_arguments_leave_outputs_alone(setup):
    smc, d, p, N, xi, gm = setup
    banner("invalid arguments")
    G = filled(N, p.n_obs)
    phi = filled(N)
    acc = filled(N, dtype=torch.int32)
    x0 = xi.clone()
    big = N + 1
    xb = t(inputs.particles(big, p.K, 73))
    Gb, phib = filled(big, p.n_obs), filled(big)

    def rejected(fn):
        with pytest.raises(smc.SMCError) as e:
            fn()
        assert e.value.status == smc.SMC_E_INVAL, e.value

    rejected(lambda: smc.smc_forward_batch(p, big, xb, None, smc.SMC_FP32_REFINE, Gb))    # N > n_max
    rejected(lambda: smc.smc_forward_batch(p, N, xi, None, 7, G))                         # unknown precision
    rejected(lambda: smc.smc_potential(p, -1, G, phi))
    for beta, tau in ((0.0, 0.5), (1.5, 0.5), (0.3, -0.1), (0.3, 1.5)):                   # out of range
        rejected(lambda: smc.smc_gmpcn_move(p, N, gm, beta, tau, 1, 1, 2, None, smc.SMC_FP64, xi, phi, acc))
    h, tn, lz = filled(1), filled(1), filled(1)
    W = filled(N)
    rejected(lambda: smc.smc_temper(0, phi, t([0.0]), 0.5, h, tn, W, lz))                 # N >= 1
    rejected(lambda: smc.smc_temper(N, phi, t([0.0]), 1.0, h, tn, W, lz))                 # ess_frac in (0, 1)
    idx = filled(N, dtype=torch.int32)
    rejected(lambda: smc.smc_resample(N, t(np.full(N, 1.0 / N)), 1 << 53, idx))           # u53 < 2^53
    rejected(lambda: smc.smc_resample(0, t(np.full(N, 1.0 / N)), 5, idx))
    rejected(lambda: smc.smc_gather(N, p.K, t(np.arange(N), torch.int32), xi, None, xi, None))   # aliasing
    torch.cuda.synchronize()
    assert smc.smc_status_flags(p) == 0
    assert same(G, filled(N, p.n_obs)) and same(phi, filled(N)) and same(acc, filled(N, dtype=torch.int32))
    assert same(Gb, filled(big, p.n_obs)) and same(phib, filled(big))
    assert same(h, filled(1)) and same(tn, filled(1)) and same(lz, filled(1)) and same(W, filled(N))
    assert same(idx, filled(N, dtype=torch.int32)) and same(xi, x0)


def test_single_particle_batches_match_the_full_batch(setup):
    """N = 1 (one workgroup, ragged against every tile) gives each particle the bits it gets in
    the batch of 8, for the forward map at 32^2 in both precisions."""
    smc, d, p, N, xi, gm = setup
    banner("single-particle batches")
    for prec in (smc.SMC_FP64, smc.SMC_FP32_REFINE):
        G = torch.empty(N, p.n_obs, dtype=torch.float64, device=DEV)
        smc.smc_forward_batch(p, N, xi, None, prec, G)
        for k in (0, 5, 7):
            g1 = torch.empty(1, p.n_obs, dtype=torch.float64, device=DEV)
            smc.smc_forward_batch(p, 1, xi[k:k + 1].contiguous(), None, prec, g1)
            torch.cuda.synchronize()
            assert torch.equal(g1[0], G[k]), (prec, k)
