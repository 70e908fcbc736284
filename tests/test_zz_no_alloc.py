"""lmep_step_noalloc: lmep_step with its scratch in the library's static
per-device array, called through the C ABI, against lmep_step on the same
inputs (same kernels, so the same bits) and against the oracle (1e-10 of the
state's max norm), on two calls in a row, the second with a smaller batch, so
the second call must overwrite what the first left in the shared array."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import paper_2603_15964_amd as lmep
import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _case(*a):
    print("case:", *a, flush=True)


def _stream():
    return torch.cuda.current_stream(torch.device(DEV)).cuda_stream


def _both(problems, states, steps, flags):
    """(lmep_step result, lmep_step_noalloc result) as host arrays per instance."""
    b = lmep.Batch(problems, device=DEV)
    w = b.empty_weights()
    u0 = b.pack(states)
    if not all(p.get("nonlin") == "burgers_frozen" for p in problems):
        b.build_weights(w, u0)
    ref = b.step(w, u0, steps, flags)
    got = b.empty_state()
    lmep.lmep_step_noalloc(b.structs, b.count, w.data_ptr(), u0.data_ptr(), got.data_ptr(), steps, flags, _stream())
    torch.cuda.synchronize()
    return b.unpack(ref), b.unpack(got)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _first_call():
    """Frozen-velocity Burgers (Dirichlet, n = 7, several tiles and a ragged
    last one) batched with an Allen-Cahn instance (periodic, n = 9), 12 steps
    at 8 steps per launch: two launches, the second a partial one."""
    pb, ub = workloads.burgers(N=20001, n=7)
    pa = workloads.make_problem(N=7000, n=9, bc="periodic", h=2.0 / 7000, dt=0.5 * (2.0 / 7000) ** 2 / 1e-4,
                                nu=1e-4, scheme="etd1", nonlin="allen_cahn", nl_coef=1.0)
    ua = workloads.rng(7).uniform(-0.1, 0.1, size=7000)
    return [pb, pa], [ub, ua], 12, lmep.LMEP_F_PERSISTENT


def _second_call():
    """A smaller batch: one periodic KdV instance (n = 9, ETD2RK), one step per
    launch."""
    p, u0 = workloads.kdv(N=4096, n=9, tau=0.05)
    return [p], [u0], 5, 0


def test_two_calls_in_a_row_match_lmep_step_and_oracle():
    for name, (probs, states, steps, flags) in (("first", _first_call()), ("second, smaller", _second_call())):
        _case("noalloc", name, [int(p["N"]) for p in probs], steps, hex(flags))
        ref, got = _both(probs, states, steps, flags)
        for k, (p, u0) in enumerate(zip(probs, states)):
            assert np.array_equal(ref[k], got[k]), (name, k)
            want = oracle.run(p, u0, steps)
            assert _rel(got[k], want) <= 1e-10, (name, k, _rel(got[k], want))


def test_rejects_other_flags():
    _case("noalloc rejects LMEP_F_GRAPH")
    probs, states, steps, _ = _second_call()
    b = lmep.Batch(probs, device=DEV)
    w, u0, out = b.empty_weights(), b.pack(states), b.empty_state()
    with pytest.raises(lmep.LmepError) as e:
        lmep.lmep_step_noalloc(b.structs, b.count, w.data_ptr(), u0.data_ptr(), out.data_ptr(), 1,
                               lmep.LMEP_F_GRAPH, _stream())
    assert e.value.code == lmep.LMEP_ERR_ARG
