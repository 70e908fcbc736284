"""Several steps per launch (LMEP_F_PERSISTENT) with stationary weights on
one-sided (upwind) windows (Sec. 4.1): the multi-step kernel keeps its whole
halo upstream of the tile.  Bit for bit the one-step path at 1, 2, 4, 8 and 16
steps per launch, for both flow directions, every boundary type, the
pointwise and derivative nonlinearities, ragged last tiles and the last tile
of a Dirichlet or Neumann instance that would start next to the end (it is
moved back to end at node N - 1); within 1e-10 of the oracle.  Also the
centred kernel on such a last tile, and small one-sided instances held whole
by one block."""
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
REGION = 2048


def _case(*a):
    print("case:", *a, flush=True)


def _tile(n, scheme, nonlin, kb):
    apps = (2 if scheme == "etd2rk" and nonlin != "none" else 1) * (2 if scheme != "linear" and nonlin == "kdv" else 1)
    return REGION - 2 * kb * apps * ((n - 1) // 2)


def _run(probs, states, steps, flags, kb=None):
    saved = lmep.lmep_get_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH)
    if kb is not None:
        lmep.lmep_set_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH, kb)
    try:
        b = lmep.Batch(probs, device=DEV)
        w = b.empty_weights()
        u0 = b.pack(states)
        b.build_weights(w, u0)
        out = b.step(w, u0, steps, flags)
        torch.cuda.synchronize()
        return b.unpack(out)
    finally:
        lmep.lmep_set_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH, saved)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _courant(n, bc, sgn):
    """The middle of the one-sided band, (n - 1) / 2; 1 on Dirichlet grids,
    where the clamped windows at the inflow end extrapolate for any larger
    Courant number and the run blows up (the oracle's too)."""
    return sgn * (1.0 if bc == "dirichlet" else (n - 1) / 2)


def _problem(N, n, bc, scheme, nonlin, cfl, seed):
    """Advection at Courant number cfl (its sign the flow direction), with a
    little diffusion; Allen-Cahn or KdV-form nonlinearity as asked."""
    h = 1.0 / N
    dt = abs(cfl) * h
    g = {"none": 0.0, "allen_cahn": 1.0, "kdv": 1e-3}[nonlin]
    p = make_problem(N=N, n=n, bc=bc, h=h, dt=dt, c=np.sign(cfl) * 1.0, nu=2e-3 * h, scheme=scheme, nonlin=nonlin,
                     nl_coef=g, window="upwind", bc_left=0.1 if bc == "dirichlet" else 0.0,
                     bc_right=-0.2 if bc == "dirichlet" else 0.0)
    x = h * np.arange(N)
    u = 0.5 * np.sin(2 * np.pi * x) + 0.2 * np.cos(6 * np.pi * x) + 0.01 * workloads.rng(seed).normal(size=N)
    if bc == "dirichlet":
        u[0], u[-1] = p["bc_left"], p["bc_right"]
    return p, u


CASES = []
for n, scheme, nonlin in [(9, "linear", "none"), (5, "etd1", "allen_cahn"), (15, "etd1", "none"),
                          (7, "etd2rk", "allen_cahn"), (9, "etd1", "kdv"), (5, "etd2rk", "kdv")]:
    for bc in ("periodic", "dirichlet", "neumann"):
        for sgn in (1, -1):
            CASES.append((n, scheme, nonlin, bc, sgn))


@pytest.mark.parametrize("n,scheme,nonlin,bc,sgn", CASES)
def test_upwind_multistep_equals_one_step(n, scheme, nonlin, bc, sgn):
    """Instances whose last tile is ragged (N = 2 tiles + 1000) or starts
    next to the end (N = tile + 2) at 8 steps per launch: 1, 2, 4, 8 and 16 steps
    per launch equal one step per launch bit for bit over 11 steps."""
    cfl = _courant(n, bc, sgn)
    _case("upwind multistep", n, scheme, nonlin, bc, sgn)
    t8 = _tile(n, scheme, nonlin, 8)
    probs, states = zip(*[_problem(N, n, bc, scheme, nonlin, cfl, seed=N + n) for N in (2 * t8 + 1000, t8 + 2)])
    want = _run(list(probs), list(states), 11, 0)
    for k, wv in enumerate(want):
        assert np.all(np.isfinite(wv)), k
    for kb in (1, 2, 4, 8, 16):
        got = _run(list(probs), list(states), 11, lmep.LMEP_F_PERSISTENT, kb)
        for k, (g, wv) in enumerate(zip(got, want)):
            assert np.array_equal(g, wv), (kb, k)


@pytest.mark.parametrize("n,scheme,nonlin,bc,sgn", [(9, "linear", "none", "dirichlet", 1),
                                                    (7, "etd2rk", "allen_cahn", "neumann", -1),
                                                    (15, "etd1", "none", "periodic", 1),
                                                    (9, "etd1", "kdv", "periodic", -1)])
def test_upwind_multistep_matches_oracle(n, scheme, nonlin, bc, sgn):
    _case("upwind multistep vs oracle", n, scheme, nonlin, bc, sgn)
    p, u0 = _problem(3000, n, bc, scheme, nonlin, _courant(n, bc, sgn), seed=7 * n)
    got = _run([p], [u0], 20, lmep.LMEP_F_PERSISTENT, 8)[0]
    want = oracle.run(p, u0, 20)
    assert np.all(np.isfinite(want)) and _rel(got, want) <= 1e-10


@pytest.mark.parametrize("kb", [1, 8])
@pytest.mark.parametrize("scheme,nonlin", [("linear", "none"), ("etd1", "allen_cahn")])
def test_centred_last_tile_next_to_dirichlet_end(kb, scheme, nonlin):
    """Centred windows, Dirichlet ends, n = 15: an instance whose last tile
    would start two nodes before the end (N = tile + 2) gives the one-step
    result bit for bit (the clamped window of node N - 2 reaches n - 1 nodes
    inwards, beyond such a tile's halo)."""
    n = 15
    _case("centred last tile", kb, scheme, nonlin)
    N = _tile(n, scheme, nonlin, kb) + 2
    h = 1.0 / N
    nu = 1e-3
    p = make_problem(N=N, n=n, bc="dirichlet", h=h, dt=0.1 * h * h / nu, nu=nu, c=0.4 * nu / h, scheme=scheme,
                     nonlin=nonlin, nl_coef=1.0 if nonlin != "none" else 0.0, bc_left=0.3, bc_right=-0.4)
    x = np.linspace(0.0, 1.0, N)
    u0 = np.cos(3 * x) + 0.05 * workloads.rng(N).normal(size=N)
    u0[0], u0[-1] = 0.3, -0.4
    want = _run([p], [u0], 9, 0)[0]
    got = _run([p], [u0], 9, lmep.LMEP_F_PERSISTENT, kb)[0]
    assert np.array_equal(got, want)
    assert _rel(got, oracle.run(p, u0, 9)) <= 1e-10


@pytest.mark.parametrize("bc", ["periodic", "dirichlet", "neumann"])
def test_small_upwind_instances_whole_per_block(bc):
    """One-sided instances of at most 512 nodes: all steps in one launch of
    the resident kernel, equal to the one-step path, within 1e-10 of the
    oracle."""
    _case("small upwind resident", bc)
    probs, states = zip(*[_problem(N, n, bc, "etd1", "allen_cahn", _courant(n, bc, s), seed=N)
                          for N, n, s in ((300, 7, 1), (512, 7, 1), (40, 9, -1))])
    one = _run(list(probs), list(states), 17, 0)
    res = _run(list(probs), list(states), 17, lmep.LMEP_F_PERSISTENT)
    for k, (a, b) in enumerate(zip(one, res)):
        assert np.array_equal(a, b), k
        assert _rel(b, oracle.run(probs[k], states[k], 17)) <= 1e-10, k


def test_upwind_multistep_kernel_names():
    """The profiled names of the one-sided kernels (side 1: c > 0, 2: c < 0)."""
    _case("upwind kernel names")
    t8 = _tile(9, "etd1", "allen_cahn", 8)
    probs, states = zip(*[_problem(3 * t8, 9, "periodic", "etd1", "allen_cahn", s * 4.0, seed=3) for s in (1, -1)])
    b = lmep.Batch(list(probs), device=DEV)
    w = b.empty_weights()
    u0 = b.pack(list(states))
    b.build_weights(w, u0)
    saved = lmep.lmep_get_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH)
    lmep.lmep_set_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH, 8)
    try:
        b.step(w, u0, 16, lmep.LMEP_F_PERSISTENT | lmep.LMEP_F_PROFILE)
    finally:
        lmep.lmep_set_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH, saved)
    torch.cuda.synchronize()
    names = sorted(k[0] for k in lmep.lmep_profile_kernels())
    assert names == ["stepk_upwind_kernel<9,1,3,8,1>", "stepk_upwind_kernel<9,1,3,8,2>"], names
