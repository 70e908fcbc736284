"""Whole small uniform-grid instances per block (LMEP_F_PERSISTENT with
stationary weights and at most 512 nodes per instance of a kernel group): all
steps of a call in one launch, bit for bit the one-step path, and within
1e-10 of the oracle.  Covers every boundary type, the pointwise schemes,
stencils from 3 to 15 points, instances of n and of 512 nodes, a group one
node too large for it (the tiled multi-step kernel instead), and the
advection-diffusion workload (N = 256, n = 5) over its 100 steps."""
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


def _case(*a):
    print("case:", *a, flush=True)


def _run(probs, states, steps, flags):
    b = lmep.Batch(probs, device=DEV)
    w = b.empty_weights()
    u0 = b.pack(states)
    b.build_weights(w, u0)
    out = b.step(w, u0, steps, flags)
    torch.cuda.synchronize()
    return b.unpack(out)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _state(p, seed):
    N = int(p["N"])
    x = np.linspace(0.0, 1.0, N)
    u = 0.6 * np.sin(2 * np.pi * x) + 0.05 * workloads.rng(seed).normal(size=N)
    if p["bc"] == "dirichlet":
        u[0], u[-1] = p["bc_left"], p["bc_right"]
    return u


def _diffusion(N, n, bc, scheme, nonlin="none", c=0.0, **kw):
    h = 1.0 / N
    nu = 1e-3
    return make_problem(N=N, n=n, bc=bc, h=h, dt=0.2 * h * h / nu, c=c, nu=nu, scheme=scheme, nonlin=nonlin,
                        nl_coef=1.0 if nonlin != "none" else 0.0, **kw)


CASES = [
    ("periodic linear n5 N256 advection", _diffusion(256, 5, "periodic", "linear", c=0.5)),
    ("neumann etd1 AC n7 N100", _diffusion(100, 7, "neumann", "etd1", "allen_cahn")),
    ("dirichlet etd2rk AC n9 N512", _diffusion(512, 9, "dirichlet", "etd2rk", "allen_cahn", bc_left=0.2,
                                               bc_right=-0.1)),
    ("periodic etd2rk none n13 N13", _diffusion(13, 13, "periodic", "etd2rk")),
    ("neumann linear n3 N3", _diffusion(3, 3, "neumann", "linear", c=0.3)),
    ("dirichlet etd1 AC n15 N40", _diffusion(40, 15, "dirichlet", "etd1", "allen_cahn")),
]


@pytest.mark.parametrize("name,p", CASES, ids=[c[0] for c in CASES])
def test_resident_uniform_equals_one_step_and_oracle(name, p):
    _case("resident uniform", name)
    u0 = _state(p, 5)
    steps = 23
    one = _run([p], [u0], steps, 0)[0]
    res = _run([p], [u0], steps, lmep.LMEP_F_PERSISTENT)[0]
    assert np.array_equal(one, res)
    want = oracle.run(p, u0, steps)
    assert _rel(res, want) <= 1e-10, _rel(res, want)


def test_mixed_batch_resident_tiled_and_frozen():
    """A resident group, a group one node too large for it (tiled multi-step
    kernel) and a frozen-velocity instance in one persistent call."""
    _case("mixed resident batch")
    probs = [_diffusion(300, 7, "periodic", "etd1", "allen_cahn"),
             _diffusion(200, 7, "periodic", "etd1", "allen_cahn"),
             _diffusion(513, 9, "neumann", "etd1", "allen_cahn"),
             workloads.burgers(N=700, n=7)[0]]
    states = [_state(p, 10 + k) for k, p in enumerate(probs[:3])] + [workloads.burgers(N=700, n=7)[1]]
    steps = 19
    one = _run(probs, states, steps, 0)
    res = _run(probs, states, steps, lmep.LMEP_F_PERSISTENT)
    for k, (a, b) in enumerate(zip(one, res)):
        assert np.array_equal(a, b), k
    for k, (p, u0) in enumerate(zip(probs, states)):
        want = oracle.run(p, u0, steps)
        assert _rel(res[k], want) <= 1e-10, k


def test_advection_diffusion_workload_in_one_launch():
    """The workload's 100 steps as one launch: equal to the one-step path at
    its literal Courant number 2 (which amplifies the highest modes, so only
    the two GPU paths are compared there) and within 1e-10 of the oracle at
    Courant number 1 and, without diffusion, at 2 (an exact shift)."""
    _case("advection-diffusion workload")
    p, u0 = workloads.advection_diffusion()
    one = _run([p], [u0], 100, 0)[0]
    res = _run([p], [u0], 100, lmep.LMEP_F_PERSISTENT)[0]
    assert np.array_equal(one, res)
    b = lmep.Batch([p], device=DEV)
    w = b.empty_weights()
    b.build_weights(w, b.pack(u0))
    b.step(w, b.pack(u0), 100, lmep.LMEP_F_PERSISTENT | lmep.LMEP_F_PROFILE)
    ks = lmep.lmep_profile_kernels()
    assert [k[0] for k in ks] == ["resident_kernel<5,0,0,true>"] and ks[0][2] == 1
    for q in (workloads.advection_diffusion(cfl=1.0)[0], workloads.advection_diffusion(nu=0.0)[0]):
        got = _run([q], [u0], 100, lmep.LMEP_F_PERSISTENT)[0]
        assert _rel(got, oracle.run(q, u0, 100)) <= 1e-10
