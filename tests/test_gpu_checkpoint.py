"""Checkpoint and resume of the samplers' state between stages (GPU).

Every random number of a stage is keyed by (seed, stage, move, particle), so a run saved after
some stages and restored into a new sampler must end with the same bits as the run never
interrupted: particles, potentials, evidence and the per-stage history.
"""
import json
import sys

import pytest
import torch

from conftest import golden

pytestmark = pytest.mark.gpu


def banner(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("kind", ["SMCSampler", "SMCGMSampler"])
def test_resume_gives_the_uninterrupted_run(kind, tmp_path):
    from paper_2503_16028_amd import smc, sampler
    banner("checkpoint resume", kind)
    d = json.load(open(golden("problem_t2.json")))
    N = 512
    p = smc.Problem(d, N, grids=[32], tol64=1e-10, tol_inner=1e-3)
    cls = getattr(sampler, kind)
    make = (lambda: cls(p, N, M=2, n_moves=3, prec=smc.SMC_FP32_REFINE, seed=3)) if kind == "SMCSampler" else \
        (lambda: cls(p, N, M=2, prec=smc.SMC_FP32_REFINE, seed=3))
    ref = make().run()
    ref_xi, ref_phi = ref["xi"].clone(), ref["phi"].clone()
    assert len(ref["history"]) >= 3
    first = make()
    first.run(stop_after=2)
    assert first.stage == 2 and float(first.tau.item()) < 1.0
    path = str(tmp_path / "state.pt")
    first.save(path)
    second = make()
    second.load(path)
    out = second.run()
    assert torch.equal(out["xi"], ref_xi) and torch.equal(out["phi"], ref_phi)
    assert out["log_Z"] == ref["log_Z"] and out["history"] == ref["history"]
    assert smc.smc_status_flags(p) == 0


def test_checkpoint_of_another_configuration_is_refused(tmp_path):
    from paper_2503_16028_amd import smc
    from paper_2503_16028_amd.sampler import SMCSampler
    banner("checkpoint config mismatch")
    d = json.load(open(golden("problem_t2.json")))
    p = smc.Problem(d, 64, grids=[32])
    a = SMCSampler(p, 64, M=2, n_moves=1, seed=1)
    a.initialise()
    path = str(tmp_path / "a.pt")
    a.save(path)
    b = SMCSampler(p, 64, M=2, n_moves=1, seed=2)
    with pytest.raises(ValueError):
        b.load(path)
