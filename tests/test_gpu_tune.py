"""The autotuner on the GPU: every candidate it may pick agrees with the
default path, the chosen configuration reproduces it and matches the oracle,
the options are restored afterwards, and the cache answers the second call;
the frozen-velocity region sizes it tries give the same bits."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
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


@pytest.mark.parametrize("name", ["ac_subset", "burgers", "chebyshev", "mixed", "upwind_mixed"])
def test_tune_choice_reproduces_default(name, tmp_path):
    print("case: tune", name, flush=True)
    if name == "ac_subset":
        ps, us = workloads.allen_cahn_batch(count=24, n_min=512, n_max=8000)
    elif name == "burgers":
        p, u = workloads.burgers(N=20000)
        ps, us = [p], [u]
    elif name == "chebyshev":
        ps, us = workloads.allen_cahn_chebyshev_batch(count=64)
    elif name == "mixed":
        ps, us = workloads.allen_cahn_batch(count=6, n_min=512, n_max=4000)
        c, cu = workloads.allen_cahn_chebyshev_batch(count=5)
        ps, us = ps + c, us + cu
    else:  # one-sided stationary and frozen-velocity instances together
        ps, us = workloads.allen_cahn_batch(count=4, n_min=512, n_max=4000)
        ps = [dict(p, window="upwind", c=0.5 * p["h"] / p["dt"] * (p["n"] - 1)) for p in ps]
        q, qu = workloads.burgers_upwind(N=3000)
        ps, us = ps + [q], us + [qu]
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
    # the chosen configuration against the oracle, instance by instance
    outs = b.unpack(got)
    for k, (p, u) in enumerate(zip(ps, us)):
        want = oracle.run(p, u, 16)
        err = np.max(np.abs(outs[k] - want)) / max(np.max(np.abs(want)), 1e-300)
        assert err <= 1e-10, (k, r.choice.describe(), err)


def test_taylor_region_sizes_give_the_same_bits():
    """LMEP_OPT_TAYLOR_REGION (the positions a block of the frozen-velocity
    multi-step kernel stages) changes the launch shape, not the values."""
    print("case: taylor region", flush=True)
    probs = [workloads.burgers(N=9000, n=7)[0], workloads.burgers_upwind(N=5000)[0]]
    states = [workloads.burgers(N=9000, n=7)[1], workloads.burgers_upwind(N=5000)[1]]
    b, w, u0 = _batch(probs, states)
    outs = []
    for reg in (0, 128, 256, 448, 512):
        lmep.lmep_set_option(lmep.LMEP_OPT_TAYLOR_REGION, reg)
        try:
            outs.append(b.step(w, u0, 13, lmep.LMEP_F_PERSISTENT))
        finally:
            lmep.lmep_set_option(lmep.LMEP_OPT_TAYLOR_REGION, 0)
    torch.cuda.synchronize()
    for k in range(1, len(outs)):
        assert torch.equal(outs[k], outs[0]), k
