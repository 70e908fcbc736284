"""Pins of the oracle's hand-written adjoint (reverse step of LINEAR / ETD1).

The forward map is analytic in the state and the coefficients (the exponential
is a terminating series, the nonlinearities are polynomials), so complex-step
derivatives Im f(x + i e) / e are exact to rounding and independent of the
adjoint code.  Central finite differences are checked too, at their own
noise level.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from workloads import make_problem

CS = 1e-30  # complex-step size


def _cases():
    return [
        ("burgers_dirichlet", make_problem(N=40, n=9, bc="dirichlet", h=0.02, dt=0.008, nu=5e-3, scheme="etd1",
                                           nonlin="burgers_frozen", nl_coef=1.0)),
        ("burgers_dirichlet_n7_c", make_problem(N=33, n=7, bc="dirichlet", h=0.04, dt=0.01, c=0.3, nu=1e-2,
                                                scheme="etd1", nonlin="burgers_frozen", nl_coef=1.0)),
        ("burgers_periodic", make_problem(N=36, n=5, bc="periodic", h=0.05, dt=0.01, nu=2e-2, scheme="etd1",
                                          nonlin="burgers_frozen", nl_coef=1.0)),
        ("allen_cahn_neumann", make_problem(N=30, n=7, bc="neumann", h=0.05, dt=0.1, nu=1e-3, scheme="etd1",
                                            nonlin="allen_cahn", nl_coef=1.0)),
        ("adv_diff_periodic", make_problem(N=32, n=5, bc="periodic", h=0.2, dt=0.15, c=1.0, nu=0.01, delta=1e-4,
                                           scheme="linear")),
        ("adv_diff_dirichlet", make_problem(N=25, n=7, bc="dirichlet", h=0.2, dt=0.05, c=0.4, nu=0.02,
                                            scheme="linear", bc_left=0.3, bc_right=-0.2)),
    ]


def _state(p, seed):
    N = p["N"]
    x = np.linspace(0, 1, N)
    g = np.random.default_rng(seed)
    u = 0.8 * np.sin(np.pi * x) + 0.1 * g.normal(size=N)
    if p["bc"] == "dirichlet":
        u[0], u[-1] = p["bc_left"], p["bc_right"]
    return u


@pytest.mark.parametrize("name,p", _cases())
def test_adjoint_step_dot_product(name, p):
    """<J x, y> = <x, J^T y>: J x by complex step of one forward step, J^T y by the adjoint."""
    u = _state(p, 1)
    g = np.random.default_rng(2)
    for _ in range(3):
        x, y = g.normal(size=p["N"]), g.normal(size=p["N"])
        Jx = oracle.run_complex(p, u, CS * x, 1).imag / CS
        JTy, _ = oracle.adjoint_step(p, u, y)
        a, b = np.dot(Jx, y), np.dot(x, JTy)
        assert abs(a - b) <= 1e-13 * (np.linalg.norm(Jx) * np.linalg.norm(y) + 1e-300), (a, b)


@pytest.mark.parametrize("name,p", _cases())
def test_adjoint_step_parameter_gradients(name, p):
    """d<y, step(u)>/d(nu, c, delta) from the adjoint equals the complex step."""
    u = _state(p, 3)
    y = np.random.default_rng(4).normal(size=p["N"])
    _, grad = oracle.adjoint_step(p, u, y)
    for k, key in enumerate(("nu_im", "c_im", "delta_im")):
        d = np.dot(y, oracle.run_complex(p, u, None, 1, **{key: CS}).imag / CS)
        assert abs(grad[k] - d) <= 1e-12 * max(1.0, abs(d)), (key, grad[k], d)


@pytest.mark.parametrize("name,p", _cases()[:4])
def test_adjoint_run_matches_complex_step(name, p):
    """Gradient of 0.5 ||u(T) - target||^2 over several steps w.r.t. u0 and (nu, c, delta)."""
    steps = 6
    u0 = _state(p, 5)
    target = oracle.run(dict(p, nu=p["nu"] * 1.1), u0, steps)
    loss, gu, grad = oracle.adjoint_run(p, u0, target, steps)
    uT = oracle.run(p, u0, steps)
    assert abs(loss - 0.5 * np.sum((uT - target) ** 2)) <= 1e-15 * max(1.0, loss)

    def dloss(**kw):
        z = oracle.run_complex(p, u0, kw.pop("u0_im", None), steps, **kw)
        return np.sum((z.real - target) * z.imag) / CS  # d/de of 0.5 sum (u - t)^2

    for k, key in enumerate(("nu_im", "c_im", "delta_im")):
        d = dloss(**{key: CS})
        assert abs(grad[k] - d) <= 1e-11 * max(abs(d), 1e-12 * np.max(np.abs(grad))), (key, grad[k], d)
    g = np.random.default_rng(6)
    for _ in range(3):
        v = g.normal(size=p["N"])
        d = dloss(u0_im=CS * v)
        assert abs(np.dot(gu, v) - d) <= 1e-11 * max(1e-300, np.linalg.norm(gu) * np.linalg.norm(v))


def test_adjoint_central_differences_and_zero_at_target():
    """Central FD (h = 1e-6) agrees at FD accuracy; the gradient vanishes when
    the target is the forward solution itself (nu = nu_target)."""
    p = _cases()[0][1]
    steps = 5
    u0 = _state(p, 7)
    target = oracle.run(dict(p, nu=p["nu"] * 1.1), u0, steps)
    _, _, grad = oracle.adjoint_run(p, u0, target, steps)
    hfd = 1e-6

    def L(nu):
        return 0.5 * np.sum((oracle.run(dict(p, nu=nu), u0, steps) - target) ** 2)

    fd = (L(p["nu"] + hfd) - L(p["nu"] - hfd)) / (2 * hfd)
    assert abs(fd - grad[0]) <= 1e-5 * abs(grad[0])
    same = oracle.run(p, u0, steps)
    loss0, gu0, grad0 = oracle.adjoint_run(p, u0, same, steps)
    assert loss0 == 0.0 and np.all(gu0 == 0.0) and np.all(grad0 == 0.0)
