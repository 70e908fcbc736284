"""Pins of the oracle's one-sided (upwind) windows, the fully one-sided
stencils of Sec. 4.1: the window of node i ends at i when its advection speed
is positive and starts at i when it is negative (centred at zero speed), moved
inside the grid next to Dirichlet ends.  Checked against facts independent of
the oracle's code:

* the selection rule itself (integer arithmetic);
* Thm 1 on the shifted window: pure-advection weights are the Lagrange basis
  at the departure point x_i - c dt, for any Courant number;
* Lagrangian Courant numbers up to n - 1 give an exact shift;
* the paper's stability statement: |G| <= 1 at CFL (n+1)/2 - sigma, inside
  the band where the departure point sits in the window's central cells, and
  growth outside it;
* the frozen-velocity case picks each node's side from its own velocity.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from workloads import make_problem


@pytest.mark.parametrize("n", [3, 5, 9, 15])
def test_selection_rule(n):
    N = 40
    for bc in ("periodic", "neumann", "dirichlet"):
        for c, pref in ((1.3, -(n - 1)), (-0.7, 0), (0.0, -(n - 1) // 2)):
            p = make_problem(N=N, n=n, bc=bc, h=0.1, dt=0.01, c=c, scheme="linear", window="upwind")
            for i in range(N):
                o = oracle.window_offset(p, i)
                want = pref if bc != "dirichlet" else min(max(pref, -i), N - n - i)
                assert o == want, (bc, c, i, o, want)
    # centred windows are unchanged by the option's existence
    p = make_problem(N=N, n=n, bc="periodic", h=0.1, dt=0.01, c=1.0, scheme="linear")
    assert all(oracle.window_offset(p, i) == -(n - 1) // 2 for i in range(N))


@pytest.mark.parametrize("n,cfl", [(5, 0.7), (7, 2.5), (9, 4.3), (11, 5.5), (13, 6.5), (15, 7.9)])
def test_theorem1_on_upwind_window(n, cfl):
    """W0 of the harvest row n-1 (c > 0) is the Lagrange basis of the window
    x_{i-n+1} .. x_i evaluated at the departure point x_i - c dt.  The series
    of the most one-sided rows cancels by up to ~1e10 at large n and CFL, which
    is why the oracle carries one-sided windows in binary128."""
    h, c = 0.2, 1.1
    dt = cfl * h / c
    p = make_problem(N=n, n=n, bc="dirichlet", h=h, dt=dt, c=c, scheme="linear", window="upwind")
    w0 = oracle.build_weights(p)[n - 1, 0]  # node n-1 harvests row n-1
    x = h * np.arange(n)
    t = x[-1] - c * dt
    lag = np.array([np.prod([(t - x[l]) / (x[k] - x[l]) for l in range(n) if l != k]) for k in range(n)])
    assert np.max(np.abs(w0 - lag)) <= 1e-13 * max(1.0, np.max(np.abs(lag)))


@pytest.mark.parametrize("n", [5, 7, 9, 13, 15])
def test_lagrangian_courant_numbers_shift_exactly(n):
    N = 60
    u0 = np.random.default_rng(7).normal(size=N)
    for cfl in range(1, n):
        p = make_problem(N=N, n=n, bc="periodic", h=1.0, dt=float(cfl), c=1.0, scheme="linear", window="upwind")
        assert np.max(np.abs(oracle.run(p, u0, 1) - np.roll(u0, cfl))) <= 1e-13 * n, cfl
        q = dict(p, c=-1.0)
        assert np.max(np.abs(oracle.run(q, u0, 1) - np.roll(u0, -cfl))) <= 1e-13 * n, cfl


def _gmax(n, cfl):
    p = make_problem(N=n, n=n, bc="dirichlet", h=1.0, dt=cfl, c=1.0, scheme="linear", window="upwind")
    row = oracle.build_weights(p)[n - 1, 0]
    th = np.linspace(0, np.pi, 2001)
    ks = np.arange(n) - (n - 1)
    return np.max(np.abs(np.exp(1j * np.outer(th, ks)) @ row))


@pytest.mark.parametrize("n", [3, 5, 7, 9, 11, 13, 15])
def test_stable_band_reaches_half_the_stencil(n):
    """Sec. 4.1 runs one-sided stencils at Courant numbers (n+1)/2 - sigma,
    sigma in {0, 1/2}, and reports them stable, so the stable Courant number
    grows linearly with n.  Independently of the oracle, a one-sided
    interpolation stencil is stable exactly while the departure point lies in
    the window's central cells, CFL in [(n-3)/2, (n+1)/2] (and at the integers,
    where the update is an exact shift); the amplification factor of the
    harvested row must show that band and the growth outside it."""
    for cfl in (max(0.5, (n - 3) / 2), (n - 2) / 2, (n - 1) / 2, n / 2, (n + 1) / 2, 1.0):
        assert _gmax(n, cfl) <= 1.0 + 1e-12, cfl
    if n >= 5:
        assert _gmax(n, 0.5) > 1.2  # departure point next to the window's end
        assert _gmax(n, (n + 2) / 2) > 1.0 + 1e-6
        assert _gmax(n, n - 1.5) > 1.2


def test_frozen_velocity_picks_side_per_node():
    """Burgers with upwind windows: node i's stencil lies on the side its own
    velocity comes from; with n = 7 and every local Courant number inside the
    stable band (3.15 .. 3.85) a periodic run stays bounded for 60 steps, where
    the centred stencil at the same step blows up within 20.  (The explicitly
    treated frozen-velocity remainder limits how long such runs stay bounded
    at larger n; the linear part alone is stable in the whole band.)"""
    N, n = 240, 7
    h, nu = 0.04, 1e-3
    x = h * np.arange(N)
    for sgn in (1.0, -1.0):
        u0 = sgn * (1.0 + 0.1 * np.sin(2 * np.pi * x / (h * N)))
        p = make_problem(N=N, n=n, bc="periodic", h=h, dt=3.5 * h, nu=nu, scheme="etd1", nonlin="burgers_frozen",
                         nl_coef=1.0, window="upwind")
        for i in (0, 60, 120, 180):
            assert oracle.window_offset(p, i, a=u0[i]) == (-(n - 1) if sgn > 0 else 0)
        u = oracle.run(p, u0, 60)
        assert np.all(np.isfinite(u)) and 0.85 <= np.min(np.abs(u)) and np.max(np.abs(u)) <= 1.15
        uc = oracle.run(dict(p, window="centred"), u0, 20)
        assert not np.all(np.isfinite(uc)) or np.max(np.abs(uc)) > 10.0


@pytest.mark.parametrize("cfl", [0.3, 1.0, 1.7])
def test_three_point_upwind_row_is_beam_warming(cfl):
    """Example 1: the last row of the three-point stencil is the second-order
    upwind (Beam-Warming) update
      u+_i = u_i - nu/2 (3 u_i - 4 u_{i-1} + u_{i-2}) + nu^2/2 (u_i - 2 u_{i-1} + u_{i-2})."""
    p = make_problem(N=3, n=3, bc="dirichlet", h=0.5, dt=cfl * 0.5 / 2.0, c=2.0, scheme="linear", window="upwind")
    w = oracle.build_weights(p)[2, 0]
    want = [-cfl / 2 + cfl ** 2 / 2, 2 * cfl - cfl ** 2, 1 - 1.5 * cfl + cfl ** 2 / 2]
    assert np.max(np.abs(w - want)) <= 1e-15
