"""Multi-step launches (LMEP_F_PERSISTENT) against the one-step path and the oracle.

Each block of the multi-step kernel advances its tile of nodes up to 1, 2, 4, 8 or 16
steps in LDS, recomputing a halo instead of exchanging it.  It forms every
value with the same expression as the one-step kernel, so the two paths must
agree bit for bit; both are also checked against the CPU oracle (1e-10
relative, FP64).  Cases cover every boundary type, scheme and nonlinearity
with stationary weights, step counts that are not multiples of the launch
depth, grids much smaller than the halo, uneven batches, graph capture, and
the full-size Allen-Cahn batch and KdV grid in the benchmark's configuration.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import paper_2603_15964_amd as lmep
import workloads
from workloads import make_problem

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
PERSIST = lmep.LMEP_F_PERSISTENT


def _print_case(*a):
    print("case:", *a, flush=True)


def state_rel_err(got, want):
    return float(np.max(np.abs(got - want)) / np.max(np.abs(want)))


class _Depth:
    """Set the steps per launch for the duration of a test."""

    def __init__(self, kb):
        self.kb = kb

    def __enter__(self):
        self.old = lmep.lmep_get_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH)
        lmep.lmep_set_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH, self.kb)

    def __exit__(self, *exc):
        lmep.lmep_set_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH, self.old)


def run_both(problems, states, steps, kb, extra_flags=0):
    """(one-step result, multi-step result) on the same weights and input."""
    b = lmep.Batch(problems, device=DEV)
    w = b.empty_weights()
    u0 = b.pack(states)
    b.build_weights(w, u0)
    ref = b.step(w, u0, steps, 0)
    with _Depth(kb):
        out = b.step(w, u0, steps, PERSIST | extra_flags)
    torch.cuda.synchronize()
    return b.unpack(ref), b.unpack(out)


def _ac(N, n, bc, scheme="etd1", seed=5, mu=0.5):
    h = 2.0 / (N if bc == "periodic" else N - 1)
    p = make_problem(N=N, n=n, bc=bc, h=h, nu=1e-4, dt=mu * h * h / 1e-4, scheme=scheme, nonlin="allen_cahn",
                     nl_coef=1.0)
    return p, np.random.default_rng(seed).uniform(-0.1, 0.1, N)


def _kdv(N, bc, scheme="etd2rk", n=9):
    p, u0 = workloads.kdv(N=N, tau=0.05, n=n)
    return dict(p, bc=bc, scheme=scheme), u0


CASES = [
    ("adv-diff periodic CFL1 n5 linear", lambda: workloads.advection_diffusion(cfl=1.0)),
    ("adv-diff dirichlet n7 linear", lambda: (make_problem(N=5000, n=7, bc="dirichlet", h=0.01, dt=0.005, c=0.8,
                                                           nu=0.002, scheme="linear", bc_left=0.2, bc_right=-0.1),
                                              np.cos(np.linspace(0, 30, 5000)))),
    ("adv-diff neumann n11 etd1 no N", lambda: (make_problem(N=4100, n=11, bc="neumann", h=0.01, dt=0.004, c=0.5,
                                                             nu=0.003, scheme="etd1"),
                                                np.sin(np.linspace(0, 20, 4100)))),
    ("adv-diff periodic n13 etd2rk no N", lambda: (make_problem(N=3000, n=13, bc="periodic", h=0.01, dt=0.004,
                                                                c=-0.6, nu=0.003, scheme="etd2rk"),
                                                   np.sin(np.linspace(0, 2 * np.pi * 7, 3000, endpoint=False)))),
    ("allen-cahn periodic n5 etd1", lambda: _ac(5000, 5, "periodic")),
    ("allen-cahn neumann n11 etd1", lambda: _ac(6000, 11, "neumann")),
    ("allen-cahn neumann n9 etd2rk", lambda: _ac(4500, 9, "neumann", "etd2rk")),
    # mu = 0.1: at 0.5 the one-sided n=7 end rows amplify (the oracle grows 100x in 19 steps)
    ("allen-cahn dirichlet n7 etd2rk react", lambda: (dict(_ac(4200, 7, "dirichlet", "etd2rk", mu=0.1)[0],
                                                           react=-0.3, bc_left=0.05, bc_right=-0.05),
                                                      _ac(4200, 7, "dirichlet", "etd2rk", mu=0.1)[1])),
    ("kdv periodic n9 etd2rk", lambda: _kdv(4096, "periodic")),
    ("kdv periodic n9 etd1", lambda: _kdv(4096, "periodic", "etd1")),
    ("kdv neumann n9 etd2rk", lambda: _kdv(5000, "neumann")),
    ("kdv dirichlet n7 etd2rk", lambda: (dict(_kdv(4500, "dirichlet", n=7)[0], bc_left=0.1),
                                         _kdv(4500, "dirichlet", n=7)[1])),
    ("kdv periodic n15 etd1", lambda: _kdv(4096, "periodic", "etd1", n=15)),
]


@pytest.mark.parametrize("kb", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_multistep_matches_one_step_and_oracle(name, make, kb):
    _print_case("multistep", name, "kb", kb)
    p, u0 = make()
    steps = 19  # not a multiple of the launch depth
    ref, got = run_both([p], [u0], steps, kb)
    assert np.array_equal(ref[0], got[0]), np.max(np.abs(ref[0] - got[0]))
    assert state_rel_err(got[0], oracle.run(p, u0, steps)) <= 1e-10


def _kdv_small(N, n, bc, scheme, h=0.5, dt=2e-3):
    x = np.arange(N) * h
    p = make_problem(N=N, n=n, bc=bc, h=h, dt=dt, delta=1.0, scheme=scheme, nonlin="kdv", nl_coef=6.0)
    return p, 0.5 * np.cos(2 * np.pi * x / (N * h)) + 0.2


TINY = [
    ("periodic N=n=9 kdv", lambda: _kdv_small(9, 9, "periodic", "etd2rk")),
    ("periodic N=16 n=15 kdv", lambda: _kdv_small(16, 15, "periodic", "etd1")),
    ("neumann N=n=9 (halo wider than the grid)", lambda: (
        make_problem(N=9, n=9, bc="neumann", h=0.25, nu=0.05, dt=0.05, c=0.3, scheme="etd1", nonlin="allen_cahn",
                     nl_coef=1.0), np.random.default_rng(5).uniform(-0.5, 0.5, 9))),
    ("neumann N=40 n=9 kdv", lambda: _kdv_small(40, 9, "neumann", "etd2rk")),
    ("dirichlet N=n=7", lambda: (make_problem(N=7, n=7, bc="dirichlet", h=0.1, dt=0.01, c=0.4, nu=0.05,
                                              scheme="etd1", nonlin="allen_cahn", nl_coef=1.0, bc_left=0.3),
                                 np.linspace(0.3, 0.0, 7))),
    ("dirichlet N=11 n=9 kdv", lambda: _kdv_small(11, 9, "dirichlet", "etd2rk")),
]


@pytest.mark.parametrize("name,make", TINY, ids=[c[0] for c in TINY])
def test_multistep_tiny_grids(name, make):
    _print_case("multistep tiny", name)
    p, u0 = make()
    steps = 13
    ref, got = run_both([p], [u0], steps, 8)
    assert np.array_equal(ref[0], got[0])
    want = oracle.run(p, u0, steps)
    assert np.max(np.abs(got[0] - want)) <= 1e-10 * max(1.0, np.max(np.abs(want)))


def test_multistep_uneven_batch_and_graph():
    """An uneven batch of every nonlinearity and boundary; graph capture of the
    multi-step loop replays to the same bits as the eager multi-step loop."""
    _print_case("multistep uneven batch + graph")
    probs, states = [], []
    for k, (N, n, bc, sch) in enumerate([(2047, 5, "periodic", "etd1"), (2049, 7, "neumann", "etd1"),
                                         (6000, 9, "periodic", "etd1"), (513, 11, "neumann", "etd1"),
                                         (4097, 9, "neumann", "etd2rk")]):
        p, u = _ac(N, n, bc, sch, seed=10 + k)
        probs.append(p)
        states.append(u)
    p, u = _kdv(3000, "periodic")
    probs.append(p)
    states.append(u)
    p, u = workloads.advection_diffusion(N=700, cfl=1.0)
    probs.append(p)
    states.append(u)
    steps = 21
    ref, got = run_both(probs, states, steps, 8)
    _, graphed = run_both(probs, states, steps, 8, extra_flags=lmep.LMEP_F_GRAPH)
    for k, (p, u0) in enumerate(zip(probs, states)):
        assert np.array_equal(ref[k], got[k]), k
        assert np.array_equal(graphed[k], got[k]), k
        assert state_rel_err(got[k], oracle.run(p, u0, steps)) <= 1e-10, k


def test_multistep_rejects_uncovered_frozen_weights():
    """Frozen velocity runs several steps per launch only through the
    finite-Taylor multi-step kernel (Dirichlet or periodic grids); a Neumann
    instance is refused."""
    _print_case("multistep rejects frozen neumann")
    p, u0 = workloads.burgers(N=512)
    p = dict(p, bc="neumann")
    b = lmep.Batch([p], device=DEV)
    w = b.empty_weights()
    with pytest.raises(lmep.LmepError) as e:
        b.step(w, b.pack([u0]), 3, PERSIST)
    assert e.value.code == lmep.LMEP_ERR_UNSUPPORTED


# ---------------------------------------------------------- full size ----
@pytest.mark.parametrize("kb,merge", [(8, 0), (16, 1)])
def test_full_size_allen_cahn_batch(kb, merge):
    """The 4096-instance Allen-Cahn batch (sum N ~ 1.35e8), at 8 steps per
    launch with a launch per stencil size and in the benchmark's launch
    configuration (16 steps per launch, every size in one launch, the
    unit-coefficient kernel): 16 steps equal the one-step path bit for bit
    everywhere; four instances (smallest, largest, two others) match the
    oracle."""
    _print_case("full size allen-cahn batch multistep", kb, merge)
    probs, states = workloads.allen_cahn_batch()
    steps = 16
    lmep.lmep_set_option(lmep.LMEP_OPT_MERGE_GROUPS, merge)
    try:
        ref, got = run_both(probs, states, steps, kb, lmep.LMEP_F_PROFILE)
        names = [k[0] for k in lmep.lmep_profile_kernels()]
    finally:
        lmep.lmep_set_option(lmep.LMEP_OPT_MERGE_GROUPS, 0)
    if merge:
        assert names == ["stepk_mixed_kernel<1,4,16>"], names
    for k in range(len(probs)):
        if not np.array_equal(ref[k], got[k]):
            raise AssertionError(f"instance {k} differs: {np.max(np.abs(ref[k] - got[k]))}")
    sizes = np.array([p["N"] for p in probs])
    for k in {int(np.argmin(sizes)), int(np.argmax(sizes)), 17, 2049}:
        assert state_rel_err(got[k], oracle.run(probs[k], states[k], steps)) <= 1e-10, k


def test_full_size_kdv_multistep():
    _print_case("full size kdv multistep")
    p, u0 = workloads.kdv()
    steps = 10
    ref, got = run_both([p], [u0], steps, 8)
    assert np.array_equal(ref[0], got[0])
    assert state_rel_err(got[0], oracle.run(p, u0, steps)) <= 1e-10


@pytest.mark.parametrize("kb", [8, 16])
@pytest.mark.parametrize("kind", ["allen_cahn_etd1", "allen_cahn_etd2rk_g07", "allen_cahn_mixed_g", "kdv_etd2rk",
                                  "linear_dirichlet"])
def test_merged_stencil_sizes_equal_separate_launches(kind, kb):
    """LMEP_OPT_MERGE_GROUPS: instances of several stencil sizes in one
    launch (largest n first) give the separate launches' result bit for bit,
    and that launch is the one that runs; Allen-Cahn launches whose every
    instance has coefficient 1 take the kernel without the product by g
    (nonlinearity code 4), others the general one (code 3)."""
    _print_case("merged sizes", kind, kb)
    probs, states = [], []
    for k, (n, N) in enumerate([(5, 3000), (11, 2600), (7, 4100), (9, 2049), (11, 700), (3, 1500), (15, 2100)]):
        if kind == "allen_cahn_etd1":
            p, u = _ac(N, n, "periodic" if k % 2 else "neumann", "etd1")
        elif kind == "allen_cahn_etd2rk_g07":
            if n > 13:  # ETD2RK builds n + 2 <= 16
                continue
            # clamped Dirichlet windows of n >= 7 need a small diffusion number
            p, u = _ac(N, n, "periodic" if k % 2 else "dirichlet", "etd2rk", mu=0.1)
            p = dict(p, nl_coef=0.7)
        elif kind == "allen_cahn_mixed_g":  # one instance with g != 1: the general kernel
            p, u = _ac(N, n, "neumann", "etd1")
            if k == 3:
                p = dict(p, nl_coef=1.5)
        elif kind == "kdv_etd2rk":
            if n > 13:
                continue
            p, u = _kdv(N, "periodic", n=n)
        else:
            h = 1.0 / N
            p = make_problem(N=N, n=n, bc="dirichlet", h=h, dt=0.2 * h * h / 1e-3, nu=1e-3, c=0.3 * 1e-3 / h,
                             scheme="linear", bc_left=0.2, bc_right=-0.1)
            u = np.cos(np.linspace(0.0, 3.0, N))
            u[0], u[-1] = 0.2, -0.1
        probs.append(p)
        states.append(u)
    saved = lmep.lmep_get_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH)
    lmep.lmep_set_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH, kb)
    try:
        outs = []
        for merge in (0, 1):
            lmep.lmep_set_option(lmep.LMEP_OPT_MERGE_GROUPS, merge)
            b = lmep.Batch(probs, device=DEV)
            w = b.empty_weights()
            u0 = b.pack(states)
            b.build_weights(w, u0)
            outs.append(b.step(w, u0, 2 * kb + 3, lmep.LMEP_F_PERSISTENT | lmep.LMEP_F_PROFILE))
            names = [k[0] for k in lmep.lmep_profile_kernels()]
            torch.cuda.synchronize()
            if merge:
                assert any(x.startswith("stepk_mixed_kernel<") for x in names), names
                assert not any(x.startswith("stepk_kernel<") for x in names), names
                if kind.startswith("allen_cahn"):
                    code = 4 if kind == "allen_cahn_etd1" else 3
                    assert f"stepk_mixed_kernel<{1 if 'etd1' in kind or 'mixed' in kind else 2},{code},{kb}>" in names, names
    finally:
        lmep.lmep_set_option(lmep.LMEP_OPT_MERGE_GROUPS, 0)
        lmep.lmep_set_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH, saved)
    assert bool(torch.isfinite(outs[0]).all())
    assert torch.equal(outs[0], outs[1])
    got = lmep.Batch(probs, device=DEV).unpack(outs[1])
    for k, (p, u) in enumerate(zip(probs, states)):
        assert state_rel_err(got[k], oracle.run(p, u, 2 * kb + 3)) <= 1e-10, k
