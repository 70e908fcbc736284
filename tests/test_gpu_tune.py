"""The autotuner on the GPU: every candidate it may pick agrees with the
default path, the chosen configuration reproduces it, the options are restored
afterwards, and the cache answers the second call."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import paper_2603_15964_amd as lmep
import workloads
from paper_2603_15964_amd import tune

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _batch(problems, states):
    b = lmep.Batch(problems, device=DEV)
    w = b.empty_weights()
    u0 = b.pack(states)
    if any(p.get("nonlin") != "burgers_frozen" for p in problems):
        b.build_weights(w, u0)
    return b, w, u0


@pytest.mark.parametrize("name", ["ac_subset", "burgers", "chebyshev", "mixed"])
def test_tune_choice_reproduces_default(name, tmp_path):
    print("case: tune", name, flush=True)
    if name == "ac_subset":
        ps, us = workloads.allen_cahn_batch(count=24, n_min=512, n_max=8000)
    elif name == "burgers":
        p, u = workloads.burgers(N=20000)
        ps, us = [p], [u]
    elif name == "chebyshev":
        ps, us = workloads.allen_cahn_chebyshev_batch(count=64)
    else:
        ps, us = workloads.allen_cahn_batch(count=6, n_min=512, n_max=4000)
        c, cu = workloads.allen_cahn_chebyshev_batch(count=5)
        ps, us = ps + c, us + cu
    b, w, u0 = _batch(ps, us)
    before = [lmep.lmep_get_option(o) for o in (lmep.LMEP_OPT_FUSE_FROZEN, lmep.LMEP_OPT_STEPS_PER_LAUNCH,
                                                  lmep.LMEP_OPT_APPLY_TILE)]
    path = str(tmp_path / "tune.json")
    r = tune.tune(b, w, u0, steps=16, cache_path=path)
    after = [lmep.lmep_get_option(o) for o in (lmep.LMEP_OPT_FUSE_FROZEN, lmep.LMEP_OPT_STEPS_PER_LAUNCH,
                                                 lmep.LMEP_OPT_APPLY_TILE)]
    assert before == after and not r.from_cache and r.ms_per_step > 0
    ref = b.step(w, u0, 16, 0)
    with tune.use(r.choice) as flags:
        got = b.step(w, u0, 16, flags)
    torch.cuda.synchronize()
    scale = float(torch.max(torch.abs(ref)))
    assert float(torch.max(torch.abs(got - ref))) <= 1e-12 * scale
    r2 = tune.tune(b, w, u0, steps=16, cache_path=path)
    assert r2.from_cache and r2.choice == r.choice
