"""The C ABI library builds, loads and exports what include/smc.h declares (CPU only).

No call here reaches the device: the only calls made are ones whose host-side validation
rejects the arguments before anything is launched.
"""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "smc.h")


@pytest.fixture(scope="module")
def libsmc():
    from paper_2503_16028_amd import build, smc
    if not os.path.exists(smc.LIB_PATH):
        build.build()
    return smc.lib()


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|void|uint64_t|const char\*)\s+(smc_\w+)\s*\(", text, re.M)))


def test_header_declares_the_calls():
    names = declared()
    for n in ("smc_prior_sample", "smc_forward_batch", "smc_potential", "smc_gmpcn_move", "smc_temper",
              "smc_resample"):
        assert n in names


def test_every_declared_symbol_is_exported(libsmc):
    from paper_2503_16028_amd import smc
    for n in declared():
        assert hasattr(libsmc, n), n
    assert sorted(declared()) == smc.EXPORTED


def test_host_validation_rejects_without_launching(libsmc):
    from paper_2503_16028_amd import smc
    c_vp = ctypes.c_void_p
    null = c_vp()
    assert libsmc.smc_temper(0, null, null, 0.5, null, null, null, null, null, null) == -1
    assert b"N must be" in libsmc.smc_last_error()
    assert libsmc.smc_temper(4, c_vp(8), c_vp(8), 1.5, c_vp(8), c_vp(8), c_vp(8), c_vp(8), null, null) == -1
    assert libsmc.smc_resample((1 << 24) + 1, c_vp(8), 0, c_vp(8), null, null) == -1
    assert libsmc.smc_resample(4, c_vp(8), 1 << 53, c_vp(8), null, null) == -1
    assert libsmc.smc_gather(4, 8, c_vp(8), c_vp(16), null, c_vp(16), null, null) == -1   # aliasing
    assert libsmc.smc_problem_create(None, None) == -1
    d = smc.ProblemDesc()
    d.dim = 3
    h = c_vp()
    assert libsmc.smc_problem_create(ctypes.byref(d), ctypes.byref(h)) == -1
    assert b"dim" in libsmc.smc_last_error()
    d.dim, d.n_levels = 2, 1
    d.grid_n[0] = 100                                          # not a power of two
    assert libsmc.smc_problem_create(ctypes.byref(d), ctypes.byref(h)) == -1
    assert libsmc.smc_problem_info(None, None, None, None) == -1


def test_observation_must_be_a_node(libsmc):
    from paper_2503_16028_amd import smc
    d = smc.ProblemDesc()
    d.dim, d.n_levels, d.kl, d.kr, d.n_obs, d.obs_den = 2, 1, 8, 8, 1, 128
    d.grid_n[0] = 64
    obs = (ctypes.c_int32 * 2)(3, 64)                         # 3/128 is not a node of the 64 grid
    y = (ctypes.c_double * 1)(0.1)
    d.obs_num, d.y, d.sigma, d.f, d.n_max = obs, y, 0.01, 1.0, 4
    d.tol64, d.tol_inner, d.max_iter, d.max_sweeps = 1e-10, 1e-5, 100, 4
    h = ctypes.c_void_p()
    assert libsmc.smc_problem_create(ctypes.byref(d), ctypes.byref(h)) == -1
    assert b"not a node" in libsmc.smc_last_error()


def test_checkpoint_policy():
    """'auto' keeps the FP64 forward states (8 n^2 bytes per particle) only when they fit."""
    from paper_2503_16028_amd.autodiff import choose_checkpoint
    assert choose_checkpoint("auto", 2048, 128, 2048 * 128 * 128 * 8) == "state"
    assert choose_checkpoint("auto", 2048, 128, 2048 * 128 * 128 * 8 - 1) == "recompute"
    assert choose_checkpoint("state", 10 ** 9, 256, 0) == "state"
    assert choose_checkpoint("recompute", 1, 16, 1 << 40) == "recompute"
    with pytest.raises(ValueError):
        choose_checkpoint("keep", 1, 16, 0)


def test_tile_candidates():
    """Every fast-Poisson tile shape fits one workgroup and the transform's wave tiling
    (16 x 16 output tiles shared evenly by the waves, whole strips of S per wave)."""
    from paper_2503_16028_amd import smc
    for n in (32, 64, 128):
        cands = smc.smc_tile_candidates(n)
        assert len(cands) >= 2 and len(set(cands)) == len(cands)
        for rows in cands:
            threads = n * n // rows
            waves = threads // 64
            nb = n // 16
            assert n % rows == 0 and threads % 64 == 0 and threads <= 1024
            assert (nb * nb) % waves == 0 and waves % nb == 0
    assert smc.smc_tile_candidates(256) == [0]
    with pytest.raises(smc.SMCError):
        smc.smc_tile_candidates(16)


def test_host_philox_matches_the_oracle_generator(libsmc):
    """smc_philox_u53 (host arithmetic) against the oracle's Philox4x32-10 and its 53-bit integer."""
    from oracle import gmfit, philox
    from oracle.smc import RESAMPLE_BLOCK, resample_u53
    from paper_2503_16028_amd import smc
    for seed, ctr in [(0, 0), (3, 1 << 20), (2 ** 40 + 7, 5 << 20), (2 ** 64 - 1, 2 ** 63 + 5)]:
        assert smc.smc_philox_u53(seed, ctr, RESAMPLE_BLOCK, 0) == resample_u53(seed, ctr)
        for m in (0, 1, 15):
            assert smc.smc_philox_u53(seed, ctr, gmfit.KMPP_BLOCK, m) == gmfit.kmpp_u53(seed, ctr, m)
        w = philox.philox4x32_10([5, 9, ctr & philox.MASK32, ctr >> 32], philox._key(seed))
        assert smc.smc_philox_u53(seed, ctr, 5, 9) == (int(w[0]) >> 5) * (1 << 26) + (int(w[1]) >> 6)


def test_binding_constants_match_the_header():
    """Status codes, precisions, flag bits and the parked level of the binding are the header's."""
    from paper_2503_16028_amd import smc
    text = open(HEADER).read()
    defs = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define SMC_(\w+) \(?(-?\d+)\)?", text)}
    for name in ("NOCONV", "STALL", "NONFINITE", "BADWEIGHTS", "BADLEVEL", "BADPARAM"):
        assert getattr(smc, "FLAG_" + name) == defs["FLAG_" + name], name
    assert smc.LEVEL_PARKED == defs["LEVEL_PARKED"]
    enums = {m.group(1): int(m.group(2)) for m in re.finditer(r"\b(SMC_\w+)\s*=\s*(-?\d+)", text)}
    assert smc.SMC_OK == enums["SMC_OK"]
    assert smc.SMC_FP64 == enums["SMC_FP64"] and smc.SMC_FP32_REFINE == enums["SMC_FP32_REFINE"]
    assert smc.PRECOND_AUTO == defs["PRECOND_AUTO"] and smc.PRECOND_JACOBI == defs["PRECOND_JACOBI"]
