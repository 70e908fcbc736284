"""GPU parity of ETDRK4 (weights from the (n+3)-order augmented matrix at dt
and the (n+1)-order one at dt/2 -- in 16-lane DPP rows up to order 16, by the
LDS build beyond, up to the paper's n = 19 -- four-stage update) with the CPU
oracle.

Weights: 1e-12 relative per harvested row, all six kinds and every stencil
row.  States: 1e-10 relative after several steps, for every boundary type and
nonlinearity, one step per launch and several; the launch depths must agree
bit for bit.  The paper-shaped Burgers run and the full-size throughput
configuration are checked as well.
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


def _case(*a):
    print("case:", *a, flush=True)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _run(problems, states, steps, kb=None):
    b = lmep.Batch(problems, device=DEV)
    w = b.empty_weights()
    u0 = b.pack(states)
    b.build_weights(w, u0)
    flags = 0
    old = lmep.lmep_get_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH)
    if kb is not None:
        lmep.lmep_set_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH, kb)
        flags = lmep.LMEP_F_PERSISTENT
    try:
        out = b.step(w, u0, steps, flags)
        torch.cuda.synchronize()
    finally:
        lmep.lmep_set_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH, old)
    return b.unpack(out)


@pytest.mark.parametrize("n", [3, 5, 7, 9, 11, 13, 15, 17, 19])
def test_weights_all_rows(n):
    _case("etdrk4 weights", n)
    p = make_problem(N=n, n=n, bc="dirichlet", h=0.3, dt=0.07, c=0.9, nu=0.04, delta=0.001, react=-0.2,
                     scheme="etdrk4", nonlin="allen_cahn", nl_coef=1.0)
    b = lmep.Batch([p], device=DEV)
    w = b.empty_weights()
    b.build_weights(w, None)
    torch.cuda.synchronize()
    got = b.unpack_weights(w)[0]  # [kind, r, k]
    want = np.transpose(oracle.build_weights(p), (1, 0, 2))
    for kind in range(6):
        num = np.max(np.abs(got[kind] - want[kind]), axis=-1)
        den = np.max(np.abs(want[kind]), axis=-1)
        assert np.max(num / den) <= 1e-12, kind


def _ac(N, n, bc, mu=0.3, seed=3):
    h = 2.0 / (N if bc == "periodic" else N - 1)
    p = make_problem(N=N, n=n, bc=bc, h=h, nu=1e-4, dt=mu * h * h / 1e-4, scheme="etdrk4", nonlin="allen_cahn",
                     nl_coef=1.0)
    return p, np.random.default_rng(seed).uniform(-0.3, 0.3, N)


def _kdv(N, n, bc, h=0.5, dt=2e-3):
    x = np.arange(N) * h
    p = make_problem(N=N, n=n, bc=bc, h=h, dt=dt, delta=1.0, scheme="etdrk4", nonlin="kdv", nl_coef=6.0)
    return p, 0.5 * np.cos(2 * np.pi * x / (N * h)) + 0.2


CASES = [
    ("allen-cahn periodic n5", lambda: _ac(3000, 5, "periodic")),
    ("allen-cahn neumann n11", lambda: _ac(4100, 11, "neumann")),
    ("allen-cahn dirichlet n7", lambda: (dict(_ac(2500, 7, "dirichlet", mu=0.1)[0], bc_left=0.05, bc_right=-0.05),
                                         _ac(2500, 7, "dirichlet", mu=0.1)[1])),
    ("kdv periodic n9", lambda: _kdv(2048, 9, "periodic")),
    ("kdv neumann n13", lambda: _kdv(3000, 13, "neumann")),
    ("kdv dirichlet n9", lambda: (dict(_kdv(2600, 9, "dirichlet")[0], bc_left=0.7, bc_right=0.7),
                                  _kdv(2600, 9, "dirichlet")[1])),
    ("no nonlinearity dirichlet n13", lambda: (make_problem(N=2200, n=13, bc="dirichlet", h=0.05, dt=0.01, c=0.7,
                                                            nu=0.02, delta=1e-5, scheme="etdrk4", bc_left=0.2),
                                               np.cos(np.linspace(0, 9, 2200)))),
    ("paper burgers N1024 n13", lambda: workloads.burgers_etdrk4(N=1024, n=13)),
    ("paper burgers N1024 n19", lambda: workloads.burgers_etdrk4(N=1024, n=19)),
    ("allen-cahn neumann n17", lambda: _ac(3000, 17, "neumann")),
    ("kdv periodic n19", lambda: _kdv(2048, 19, "periodic")),
    ("allen-cahn dirichlet n15", lambda: (dict(_ac(2500, 15, "dirichlet", mu=0.1)[0], bc_left=0.05,
                                               bc_right=-0.05), _ac(2500, 15, "dirichlet", mu=0.1)[1])),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_matches_oracle_every_depth(name, make):
    _case("etdrk4 run", name)
    p, u0 = make()
    steps = 11
    want = oracle.run(p, u0, steps)
    one = _run([p], [u0], steps)[0]
    assert _rel(one, want) <= 1e-10
    for kb in (1, 2, 4, 8):
        assert np.array_equal(_run([p], [u0], steps, kb=kb)[0], one), kb


def test_tiny_grids():
    _case("etdrk4 tiny grids")
    cases = [_kdv(9, 9, "periodic"), _kdv(13, 13, "neumann"), _kdv(11, 9, "dirichlet"),
             (make_problem(N=7, n=7, bc="neumann", h=0.25, nu=0.05, dt=0.05, c=0.3, scheme="etdrk4",
                           nonlin="allen_cahn", nl_coef=1.0), np.random.default_rng(5).uniform(-0.5, 0.5, 7))]
    for p, u0 in cases:
        want = oracle.run(p, u0, 9)
        got = _run([p], [u0], 9, kb=8)[0]
        assert np.max(np.abs(got - want)) <= 1e-10 * max(1.0, np.max(np.abs(want))), (p["N"], p["bc"])


def test_mixed_batch_with_other_schemes():
    """ETDRK4 instances in one call with ETD1 / ETD2RK / frozen-velocity ones."""
    _case("etdrk4 mixed batch")
    probs, states = [], []
    for mk in (lambda: _ac(1500, 9, "periodic"), lambda: _kdv(1200, 7, "periodic"),
               lambda: workloads.burgers(N=900), lambda: workloads.kdv(N=1024, tau=0.05),
               lambda: workloads.allen_cahn_batch(count=1, n_min=800, n_max=800)):
        p, u = mk()
        if isinstance(p, list):
            p, u = p[0], u[0]
        probs.append(p)
        states.append(u)
    got = _run(probs, states, 6)
    for p, u0, g in zip(probs, states, got):
        assert _rel(g, oracle.run(p, u0, 6)) <= 1e-10, (p["scheme"], p["N"])


def test_full_size_paper_burgers():
    """The throughput configuration (N = 2^20, n = 19, 8 steps per launch):
    16 steps equal the one-step path bit for bit and the oracle to 1e-10."""
    _case("etdrk4 full size")
    p, u0 = workloads.burgers_etdrk4()
    steps = 16
    one = _run([p], [u0], steps)[0]
    assert np.array_equal(_run([p], [u0], steps, kb=8)[0], one)
    assert _rel(one, oracle.run(p, u0, steps)) <= 1e-10


def test_fourth_order_at_n19():
    """The paper's stencil on the GPU: periodic diffusion + Allen-Cahn (N = 64,
    n = 19) against the semi-discrete system integrated to 1e-13; the errors
    at T = 1 fall by 2^4 per halving of dt."""
    from scipy.integrate import solve_ivp
    _case("etdrk4 order at n = 19")
    N, n, nu, g, T = 64, 19, 0.02, 1.0, 1.0
    h = 2 * np.pi / N
    x = np.arange(N) * h
    u0 = 0.4 * np.sin(x) + 0.1
    D = oracle.fd_matrices(n, h)
    R = (n - 1) // 2
    A = np.zeros((N, N))
    for i in range(N):
        for k in range(n):
            A[i, (i - R + k) % N] += nu * D[1][R][k]
    ref = solve_ivp(lambda t, u: A @ u + g * (u - u ** 3), (0, T), u0, method="DOP853", rtol=1e-13,
                    atol=1e-15).y[:, -1]
    errs = []
    for m in (8, 16, 32, 64):
        p = make_problem(N=N, n=n, bc="periodic", h=h, dt=T / m, nu=nu, scheme="etdrk4", nonlin="allen_cahn",
                         nl_coef=g)
        errs.append(np.max(np.abs(_run([p], [u0], m, kb=8)[0] - ref)))
    slopes = [np.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert all(abs(s - 4.0) <= 0.3 for s in slopes), (errs, slopes)
