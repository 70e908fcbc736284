"""GPU parity of the finite-Taylor weight build for frozen-velocity Burgers.

The default exponential method (LMEP_EXP_AUTO) builds the per-node weights of
frozen-velocity instances from the finite Taylor series of e^{q(D)} (the
window operator is a polynomial in the nilpotent first-derivative matrix).
These tests hold that kernel to the oracle at the same bars as the Pade path:
weights 1e-12 relative per harvested row, one step 1e-13 and final states
1e-10 relative to the state's max norm; batched and graph-replayed launches
must equal single eager launches bit for bit.  They cover the wavefront-uniform
path (interior nodes), the per-lane path (Dirichlet edge rows, one-sided
windows changing side), ragged last tiles, instances smaller than a tile,
dispersion, and the Pade fallback for a reaction term.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import paper_2603_15964_amd as lmep
import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _print_case(*a):
    print("case:", *a, flush=True)


def _rel_rows(got, want):
    """got, want [kind, k, N]: max over (kind, node) of the row's inf-norm error over its inf norm."""
    num = np.max(np.abs(got - want), axis=1)
    den = np.max(np.abs(want), axis=1)
    return float(np.max(num / den))


def _state_err(got, want):
    return float(np.max(np.abs(got - want)) / np.max(np.abs(want)))


class _method:
    def __init__(self, value):
        self.value = value

    def __enter__(self):
        self.saved = lmep.lmep_get_option(lmep.LMEP_OPT_EXP_METHOD)
        lmep.lmep_set_option(lmep.LMEP_OPT_EXP_METHOD, self.value)

    def __exit__(self, *exc):
        lmep.lmep_set_option(lmep.LMEP_OPT_EXP_METHOD, self.saved)
        return False


def _weights(problems, states):
    b = lmep.Batch(problems, device=DEV)
    w = b.empty_weights()
    b.build_weights(w, b.pack(states))
    torch.cuda.synchronize()
    return b.unpack_weights(w)


def _run(problems, states, steps, flags=0):
    b = lmep.Batch(problems, device=DEV)
    w = b.empty_weights()
    out = b.step(w, b.pack(states), steps, flags)
    torch.cuda.synchronize()
    return b.unpack(out)


def _problem(N, n, bc="dirichlet", window="centred", cfl=1.0, mu=0.15, tau=0.0, seed=0, rough=False):
    """Frozen-velocity Burgers instance with a velocity field of peak CFL `cfl`
    (smooth Fourier modes, or seeded noise with `rough`), diffusion number mu
    and dispersion number tau."""
    rng = np.random.default_rng(workloads.BASE_SEED + 40 + seed)
    h, dt = 0.05, 0.01
    x = np.arange(N) / N
    if rough:
        u = rng.uniform(-1.0, 1.0, N)
    else:
        u = sum(rng.normal(0, 1.0 / k) * np.sin(2 * np.pi * k * x + rng.uniform(0, 2 * np.pi)) for k in range(1, 5))
    u = u / np.max(np.abs(u)) * cfl * h / dt
    p = workloads.make_problem(N=N, n=n, bc=bc, h=h, dt=dt, nu=mu * h * h / dt, delta=tau * h ** 3 / dt,
                               scheme="etd1", nonlin="burgers_frozen", nl_coef=1.0, window=window)
    if bc == "dirichlet":
        u[0] = u[-1] = 0.0
    return p, u


WEIGHT_CASES = []
for n in (3, 5, 7, 9, 11, 13, 15):
    cfl = 2.0 if n <= 9 else 1.0
    WEIGHT_CASES.append((n, "dirichlet", "centred", cfl, False))
    WEIGHT_CASES.append((n, "periodic", "centred", cfl, True))
WEIGHT_CASES += [(7, "neumann", "centred", 1.5, False), (5, "dirichlet", "upwind", 1.5, False),
                 (7, "periodic", "upwind", 2.5, False), (7, "periodic", "upwind", 2.0, True),
                 (9, "dirichlet", "upwind", 2.0, True)]


@pytest.mark.parametrize("n,bc,window,cfl,rough", WEIGHT_CASES)
def test_taylor_weights_match_oracle(n, bc, window, cfl, rough):
    """Per-node weights (W0, W1) of the finite-Taylor build against the
    oracle's Pade exponentials, on a ragged grid (N = 3 tiles + 37 nodes)."""
    _print_case("taylor weights", n, bc, window, cfl, rough)
    N = 3 * 256 + 37
    p, u = _problem(N, n, bc, window, cfl=cfl, rough=rough, seed=n)
    got = _weights([p], [u])[0]
    want = np.transpose(oracle.build_weights(p, u), (1, 2, 0))
    assert got.shape == want.shape
    assert _rel_rows(got, want) <= 1e-12


def test_taylor_weights_with_dispersion():
    """A dispersive term (delta != 0) enters the moment recursion."""
    _print_case("taylor weights dispersion")
    for n in (5, 9):
        p, u = _problem(600, n, "periodic", cfl=1.0, mu=0.1, tau=0.05, seed=100 + n)
        got = _weights([p], [u])[0]
        want = np.transpose(oracle.build_weights(p, u), (1, 2, 0))
        assert _rel_rows(got, want) <= 1e-12


def test_taylor_and_pade_weights_agree():
    """The two exponential methods agree to 1e-12 per row through the C ABI."""
    _print_case("taylor vs pade weights")
    p, u = workloads.burgers(N=4000, n=7)
    tay = _weights([p], [u])[0]
    with _method(lmep.LMEP_EXP_PADE):
        pad = _weights([p], [u])[0]
    assert _rel_rows(tay, pad) <= 1e-12


@pytest.mark.parametrize("N,n,bc", [(7, 7, "dirichlet"), (9, 9, "periodic"), (5, 5, "neumann"), (255, 5, "dirichlet"),
                                    (257, 7, "periodic"), (256, 3, "neumann")])
def test_taylor_small_and_ragged_instances(N, n, bc):
    """Instances of at most one or two tiles, down to N = n: weights and one
    fused step (1e-13) against the oracle."""
    _print_case("taylor small", N, n, bc)
    p, u = _problem(N, n, bc, cfl=1.0, seed=N)
    got = _weights([p], [u])[0]
    want = np.transpose(oracle.build_weights(p, u), (1, 2, 0))
    assert _rel_rows(got, want) <= 1e-12
    one = _run([p], [u], 1)[0]
    assert _state_err(one, oracle.run(p, u, 1)) <= 1e-13


@pytest.mark.parametrize("bc,window", [("dirichlet", "centred"), ("periodic", "centred"), ("neumann", "centred"),
                                       ("periodic", "upwind"), ("dirichlet", "upwind")])
def test_taylor_fused_steps_match_oracle(bc, window):
    """Fused build-and-apply: one step to 1e-13, ten steps to 1e-10."""
    _print_case("taylor fused steps", bc, window)
    n = 7 if window == "centred" else 5
    p, u = _problem(1500, n, bc, window, cfl=1.0 if window == "centred" else 1.5, seed=7)
    one = _run([p], [u], 1)[0]
    assert _state_err(one, oracle.run(p, u, 1)) <= 1e-13
    ten = _run([p], [u], 10)[0]
    assert _state_err(ten, oracle.run(p, u, 10)) <= 1e-10


def test_taylor_fused_unfused_and_pade_agree():
    """Fused Taylor step, build-then-apply Taylor step and the Pade paths agree
    to rounding over five steps."""
    _print_case("taylor fused/unfused/pade")
    p, u = workloads.burgers(N=5000, n=7)
    fused = _run([p], [u], 5)[0]
    lmep.lmep_set_option(lmep.LMEP_OPT_FUSE_FROZEN, 0)
    try:
        pair = _run([p], [u], 5)[0]
    finally:
        lmep.lmep_set_option(lmep.LMEP_OPT_FUSE_FROZEN, 1)
    with _method(lmep.LMEP_EXP_PADE):
        pade = _run([p], [u], 5)[0]
    assert _state_err(fused, pair) <= 1e-13
    assert _state_err(fused, pade) <= 1e-13


def test_taylor_batch_equals_single_and_graph_equals_eager():
    """Uneven batch (tile -> instance map) equals single-instance launches, and
    graph replay equals eager launches, bit for bit; a reaction-term instance
    in the same batch takes the Pade path and still matches the oracle."""
    _print_case("taylor batch/graph")
    cases = [_problem(3000, 7, "dirichlet", seed=1), _problem(700, 5, "periodic", seed=2),
             _problem(256, 9, "neumann", seed=3), _problem(1000, 7, "periodic", "upwind", cfl=1.5, seed=4),
             _problem(513, 7, "dirichlet", seed=5)]
    probs = [c[0] for c in cases]
    states = [c[1] for c in cases]
    probs[4] = dict(probs[4], react=-0.3)
    batched = _run(probs, states, 4)
    graph = _run(probs, states, 4, flags=lmep.LMEP_F_GRAPH)
    for k, (p, u) in enumerate(zip(probs, states)):
        single = _run([p], [u], 4)[0]
        assert np.array_equal(batched[k], single), k
        assert np.array_equal(graph[k], single), k
        assert _state_err(single, oracle.run(p, u, 4)) <= 1e-10, k


@pytest.mark.parametrize("persistent", [False, True])
def test_equal_instances_batch_equals_single(persistent):
    """Instances with equal work (each block then finds its instance by a
    division instead of a search): each instance of the batch equals its own
    single-instance run bit for bit, one step per launch and at 8 per launch."""
    _print_case("equal-instance batch", persistent)
    cases = [_problem(2500, 7, "dirichlet", seed=10 + k) for k in range(3)]
    probs = [c[0] for c in cases]
    states = [c[1] for c in cases]
    flags = lmep.LMEP_F_PERSISTENT if persistent else 0
    saved = lmep.lmep_get_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH)
    _set_kb(8)
    try:
        batched = _run(probs, states, 11, flags=flags)
        for k, (p, u) in enumerate(zip(probs, states)):
            assert np.array_equal(batched[k], _run([p], [u], 11, flags=flags)[0]), k
    finally:
        _set_kb(saved)
    assert _state_err(batched[1], oracle.run(probs[1], states[1], 11)) <= 1e-10


def test_taylor_counts_nodes_without_squarings():
    """LMEP_F_COUNT: a Taylor-built node counts as one matrix, no squarings."""
    _print_case("taylor counters")
    p, u = workloads.burgers(N=1000, n=7)
    _run([p], [u], 3, flags=lmep.LMEP_F_COUNT)
    prof = lmep.lmep_profile_last()
    assert prof["matrices"] == 3 * 1000 and prof["squarings"] == 0
    with _method(lmep.LMEP_EXP_PADE):
        _run([p], [u], 3, flags=lmep.LMEP_F_COUNT)
        prof = lmep.lmep_profile_last()
    assert prof["matrices"] == 3 * 1000


def _set_kb(kb):
    lmep.lmep_set_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH, kb)


# groups under 2^20 nodes stage half-size regions (n <= 9 at 8 steps per launch); the
# 1.1M-node cases take the full ones
MULTI_CASES = [(7, "dirichlet", 3000), (7, "periodic", 2000), (3, "dirichlet", 700), (9, "periodic", 513),
               (15, "dirichlet", 1200), (5, "dirichlet", 5), (9, "periodic", 9), (11, "periodic", 300),
               (7, "dirichlet", 1100001), (9, "periodic", 1100000)]


@pytest.mark.parametrize("n,bc,N", MULTI_CASES)
def test_taylor_multistep_equals_one_step(n, bc, N):
    """LMEP_F_PERSISTENT for frozen velocity: 1, 2, 4 or 8 fused steps per
    launch (11 steps, so the last launch is short) equal the one-step fused
    kernel bit for bit, including instances smaller than the halo."""
    _print_case("taylor multistep", n, bc, N)
    p, u = _problem(N, n, bc, cfl=1.0, seed=200 + n)
    want = _run([p], [u], 11)[0]
    saved = lmep.lmep_get_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH)
    try:
        for kb in (1, 2, 4, 8):
            _set_kb(kb)
            got = _run([p], [u], 11, flags=lmep.LMEP_F_PERSISTENT)[0]
            assert np.array_equal(got, want), kb
    finally:
        _set_kb(saved)


def test_taylor_multistep_batch_graph_and_oracle():
    """Uneven frozen-velocity batch at 8 steps per launch: equals the one-step
    path per instance, graph replay equals eager, and 20 steps match the
    oracle to 1e-10; a high-Courant-number instance exercises shifted
    expansions inside the staged region."""
    _print_case("taylor multistep batch")
    cases = [_problem(4000, 7, "dirichlet", seed=301), _problem(777, 9, "periodic", seed=302),
             _problem(300, 7, "dirichlet", cfl=1.5, seed=303), _problem(2048, 7, "periodic", cfl=1.2, rough=True,
                                                                       seed=304)]
    probs = [c[0] for c in cases]
    states = [c[1] for c in cases]
    one = _run(probs, states, 20)
    saved = lmep.lmep_get_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH)
    try:
        _set_kb(8)
        multi = _run(probs, states, 20, flags=lmep.LMEP_F_PERSISTENT)
        graph = _run(probs, states, 20, flags=lmep.LMEP_F_PERSISTENT | lmep.LMEP_F_GRAPH)
    finally:
        _set_kb(saved)
    for k, (p, u) in enumerate(zip(probs, states)):
        assert np.array_equal(multi[k], one[k]), k
        assert np.array_equal(graph[k], one[k]), k
        assert _state_err(multi[k], oracle.run(p, u, 20)) <= 1e-10, k


# frozen upwind stencils are stable only for small n (n = 9 blows up on these fields)
UPWIND_MULTI = [(5, "periodic", 2000, 1.5), (7, "dirichlet", 3000, 1.5), (5, "periodic", 700, 2.0),
                (3, "dirichlet", 700, 1.0), (7, "periodic", 1100000, 1.5)]


@pytest.mark.parametrize("n,bc,N,cfl", UPWIND_MULTI)
def test_taylor_multistep_upwind_equals_one_step(n, bc, N, cfl):
    """One-sided windows under LMEP_F_PERSISTENT (halo 2 (n - 1) per step):
    1, 2, 4 and 8 steps per launch equal the one-step fused kernel bit for
    bit over 11 steps."""
    _print_case("taylor multistep upwind", n, bc, N, cfl)
    p, u = _problem(N, n, bc, "upwind", cfl=cfl, seed=400 + n)
    want = _run([p], [u], 11)[0]
    assert np.all(np.isfinite(want))
    saved = lmep.lmep_get_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH)
    try:
        for kb in (1, 2, 4, 8):
            _set_kb(kb)
            got = _run([p], [u], 11, flags=lmep.LMEP_F_PERSISTENT)[0]
            assert np.array_equal(got, want), kb
    finally:
        _set_kb(saved)


def test_taylor_multistep_upwind_workload_and_oracle():
    """The upwind Burgers workload (N = 65536, n = 7, CFL 3.5) at 8 steps per
    launch: equal to the one-step path, and 5 steps match the oracle."""
    _print_case("taylor multistep upwind workload")
    p, u = workloads.burgers_upwind()
    one = _run([p], [u], 16)[0]
    saved = lmep.lmep_get_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH)
    try:
        _set_kb(8)
        multi = _run([p], [u], 16, flags=lmep.LMEP_F_PERSISTENT)[0]
        five = _run([p], [u], 5, flags=lmep.LMEP_F_PERSISTENT)[0]
    finally:
        _set_kb(saved)
    assert np.array_equal(multi, one)
    assert _state_err(five, oracle.run(p, u, 5)) <= 1e-10


def test_taylor_multistep_mixed_windows_speed_and_dispersion():
    """One frozen-velocity group at 4 steps per launch holding centred and
    one-sided instances (per-instance tiles), a background speed c and a
    dispersive term: equal to the one-step path instance by instance."""
    _print_case("taylor multistep mixed")
    a, ua = _problem(1500, 5, "periodic", "centred", cfl=1.0, tau=0.02, seed=501)
    b, ub = _problem(900, 5, "dirichlet", "upwind", cfl=1.2, seed=502)
    c, uc = _problem(2000, 5, "periodic", "upwind", cfl=1.0, seed=503)
    a = dict(a, c=0.4)
    probs, states = [a, b, c], [ua, ub, uc]
    one = _run(probs, states, 9)
    saved = lmep.lmep_get_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH)
    try:
        _set_kb(4)
        multi = _run(probs, states, 9, flags=lmep.LMEP_F_PERSISTENT)
    finally:
        _set_kb(saved)
    for k in range(3):
        assert np.all(np.isfinite(one[k])), k
        assert np.array_equal(multi[k], one[k]), k
    assert _state_err(one[0], oracle.run(a, ua, 9)) <= 1e-10
