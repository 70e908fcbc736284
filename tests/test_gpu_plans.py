"""Plans (lmep_plan_*): the same results, bit for bit, as the plain entry
points they stand for; graphs captured once and replayed on later calls;
per-plan option values that leave the process-wide ones alone; a plan used
from a stream other than the one its tables were uploaded on; and the
per-kernel timings of a profiled call."""
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


def _mixed_batch():
    """Frozen-velocity Burgers (Dirichlet), Allen-Cahn (periodic, n = 9) and
    KdV (periodic, ETD2RK): three build/apply variants in one batch."""
    pb, ub = workloads.burgers(N=3001, n=7)
    pa = workloads.make_problem(N=2500, n=9, bc="periodic", h=2.0 / 2500, dt=0.5 * (2.0 / 2500) ** 2 / 1e-4,
                                nu=1e-4, scheme="etd1", nonlin="allen_cahn", nl_coef=1.0)
    ua = workloads.rng(11).uniform(-0.1, 0.1, size=2500)
    pk, uk = workloads.kdv(N=2048, n=9, tau=0.05)
    return [pb, pa, pk], [ub, ua, uk]


def _run(batch, states, steps, flags):
    w = batch.empty_weights()
    u0 = batch.pack(states)
    if not all(p.get("nonlin") == "burgers_frozen" for p in batch.problems):
        batch.build_weights(w, u0)
    out = batch.step(w, u0, steps, flags)
    torch.cuda.synchronize()
    return batch.unpack(out)


@pytest.mark.parametrize("flags", [0, lmep.LMEP_F_GRAPH])
def test_plan_step_equals_plain_step(flags):
    _case("plan vs plain lmep_step", hex(flags))
    probs, states = _mixed_batch()
    got = _run(lmep.Batch(probs, device=DEV), states, 9, flags)
    ref = _run(lmep.Batch(probs, device=DEV, use_plans=False), states, 9, flags)
    for g, r in zip(got, ref):
        assert np.array_equal(g, r)


def test_plan_adjoint_equals_plain_adjoint_and_oracle():
    _case("plan vs plain lmep_adjoint_step")
    p, _, u0s = workloads.burgers_adjoint_batch(batch=3, N=900)
    lams = [workloads.rng(30 + k).normal(size=900) for k in range(3)]
    outs = []
    for use in (True, False):
        b = lmep.Batch([p] * 3, device=DEV, use_plans=use)
        lk, g = b.adjoint_step(b.pack(u0s), b.pack(lams))
        lk, g = b.adjoint_step(b.pack(u0s), lk, grad=g)  # a second call on the same plan
        torch.cuda.synchronize()
        outs.append((b.unpack(lk), g.cpu().numpy()))
    for a, r in zip(outs[0][0], outs[1][0]):
        assert np.array_equal(a, r)
    assert np.array_equal(outs[0][1], outs[1][1])
    want, wg = oracle.adjoint_step(p, u0s[0], lams[0])
    want, wg2 = oracle.adjoint_step(p, u0s[0], want)
    rel = np.max(np.abs(outs[0][0][0] - want)) / np.max(np.abs(want))
    assert rel <= 1e-10


def test_graph_replays_match_eager_with_work_between():
    """The plan keeps the graph of each (weights, input, output, steps) and
    replays it; every replay, with eager work and synchronisations between,
    equals the eager result."""
    _case("plan graph replays")
    probs, states = _mixed_batch()
    b = lmep.Batch(probs, device=DEV)
    w = b.empty_weights()
    u0 = b.pack(states)
    b.build_weights(w, u0)
    eager = b.step(w, u0, 6, 0)
    torch.cuda.synchronize()
    out = b.empty_state()
    for rep in range(4):
        out.fill_(float("nan"))
        b.step(w, u0, 6, lmep.LMEP_F_GRAPH, u_out=out)
        scratch = b.step(w, u0, 2, 0)  # eager work on the same plan between replays
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
        assert torch.isfinite(scratch).all()
    h = b.plan(lmep.OP_STEP, 0)
    assert h  # one plan served every call above


def test_plan_options_override_process_values():
    """A plan made with its own steps-per-launch gives the same bits as the
    process-wide default (multi-step launches equal one-step ones) and leaves
    the process-wide value untouched."""
    _case("per-plan options")
    p, u0 = workloads.burgers(N=5000, n=7)
    b = lmep.Batch([p], device=DEV)
    before = lmep.lmep_get_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH)
    outs = []
    for kb in (2, 8):
        nbytes = lmep.lmep_scratch_bytes(b.structs, 1, lmep.OP_STEP)
        scratch = torch.empty(nbytes, dtype=torch.uint8, device=DEV)
        h = lmep.lmep_plan_create(b.structs, 1, lmep.OP_STEP, lmep.LMEP_F_PERSISTENT,
                                  {lmep.LMEP_OPT_STEPS_PER_LAUNCH: kb}, scratch.data_ptr(), nbytes, _stream())
        try:
            u = b.pack(u0)
            out = b.empty_state()
            w = b.empty_weights()
            lmep.lmep_plan_step(h, w.data_ptr(), u.data_ptr(), out.data_ptr(), 11, lmep.LMEP_F_PERSISTENT, _stream())
            torch.cuda.synchronize()
            outs.append(out.cpu().numpy())
        finally:
            lmep.lmep_plan_destroy(h)
    assert lmep.lmep_get_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH) == before
    assert np.array_equal(outs[0], outs[1])
    want = oracle.run(p, u0, 11)
    assert np.max(np.abs(outs[1] - want)) / np.max(np.abs(want)) <= 1e-10


def test_plan_used_on_another_stream():
    """Tables uploaded on one stream, the step run on another: the step waits
    for the upload on the device."""
    _case("plan on a second stream")
    probs, states = _mixed_batch()
    b = lmep.Batch(probs, device=DEV)
    w = b.empty_weights()
    u0 = b.pack(states)
    b.build_weights(w, u0)
    ref = b.step(w, u0, 5, 0)
    torch.cuda.synchronize()
    b2 = lmep.Batch(probs, device=DEV)
    nbytes = lmep.lmep_scratch_bytes(b2.structs, b2.count, lmep.OP_STEP)
    scratch = torch.empty(nbytes, dtype=torch.uint8, device=DEV)
    h = lmep.lmep_plan_create(b2.structs, b2.count, lmep.OP_STEP, 0, None, scratch.data_ptr(), nbytes, _stream())
    side = torch.cuda.Stream(device=DEV)
    out = b2.empty_state()
    try:
        with torch.cuda.stream(side):
            lmep.lmep_plan_step(h, w.data_ptr(), u0.data_ptr(), out.data_ptr(), 5, 0, side.cuda_stream)
        side.synchronize()
    finally:
        lmep.lmep_plan_destroy(h)
    assert torch.equal(out, ref)


def test_profiled_call_names_its_kernels():
    _case("per-kernel profile")
    probs, states = _mixed_batch()
    b = lmep.Batch(probs, device=DEV)
    w = b.empty_weights()
    u0 = b.pack(states)
    b.build_weights(w, u0)
    ref = b.step(w, u0, 3, 0)
    got = b.step(w, u0, 3, lmep.LMEP_F_PROFILE)
    torch.cuda.synchronize()
    assert torch.equal(ref, got)
    ks = {name: (ms, n) for name, ms, n in lmep.lmep_profile_kernels()}
    assert "build_taylor_kernel<7,true>" in ks
    assert "apply_kernel<9,1,3,false,256>" in ks
    assert "apply_kernel<9,2,2,false,256>" in ks
    for name, (ms, n) in ks.items():
        assert n == 3 and ms > 0.0, name
    prof = lmep.lmep_profile_last()
    assert prof["build_launches"] == 3 and prof["apply_launches"] == 6


def test_single_kernel_steps_share_one_event_span():
    """A step that runs one kernel: one pair of events spans its back-to-back
    launches, reported with their count."""
    _case("one event span")
    p, u0 = workloads.burgers(N=4000, n=7)
    b = lmep.Batch([p], device=DEV)
    w = b.empty_weights()
    u = b.pack(u0)
    ref = b.step(w, u, 20, lmep.LMEP_F_PERSISTENT)
    got = b.step(w, u, 20, lmep.LMEP_F_PERSISTENT | lmep.LMEP_F_PROFILE)
    torch.cuda.synchronize()
    assert torch.equal(ref, got)
    ks = lmep.lmep_profile_kernels()
    kb = lmep.lmep_get_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH)
    assert len(ks) == 1 and ks[0][0] == "taylor_stepk_kernel<7>"
    assert ks[0][2] == -(-20 // kb) and ks[0][1] > 0.0
