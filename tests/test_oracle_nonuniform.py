"""Pins of the oracle's non-uniform grids (Sec. 4.3.3: on a Chebyshev grid
every node has its own local operator, harvested once).  Checked against facts
independent of the oracle's code:

* the differentiation matrices on arbitrary nodes differentiate polynomials of
  degree < n exactly (numpy's polynomial derivatives);
* uniform coordinates reproduce the uniform-grid path;
* Thm 1 on a non-uniform window: pure-advection weights are the Lagrange basis
  at the departure point x_i - c dt;
* diffusion: the harvested rows applied to x^k give the heat flow of x^k and
  its time integral in closed form (the exponential of a nilpotent operator
  acting on polynomials of degree < n is exact);
* the paper's Chebyshev Allen-Cahn run keeps its Dirichlet values, stays
  bounded, and ETD1 converges at first order in time;
* unsupported combinations are refused.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from workloads import make_problem


def _cheb(N):
    return -np.cos(np.pi * np.arange(N) / (N - 1))


@pytest.mark.parametrize("n", [3, 5, 9, 15, 21])
def test_fd_on_nodes_is_exact_on_polynomials(n):
    rng = np.random.default_rng(n)
    x = np.sort(rng.uniform(-1.0, 1.0, n))
    x[0], x[-1] = -1.0, 1.0
    D1, D2, D3 = oracle.fd_nodes(x)
    for k in range(n):
        c = np.zeros(k + 1)
        c[k] = 1.0
        for m, D in enumerate((D1, D2, D3), start=1):
            want = np.polynomial.polynomial.polyval(x, np.polynomial.polynomial.polyder(c, m)) if k >= m else 0 * x
            # rounding of the products D @ x^k: a few ulps of ||D||_inf (random
            # nodes come close together, which makes the matrices large)
            tol = 4e-16 * np.max(np.sum(np.abs(D), axis=1)) + 1e-13 * max(1.0, np.max(np.abs(want)))
            assert np.max(np.abs(D @ x ** k - want)) <= tol, (k, m)


@pytest.mark.parametrize("scheme", ["linear", "etd1", "etd2rk", "etdrk4"])
def test_uniform_coordinates_reproduce_uniform_path(scheme):
    N, n, h = 40, 7, 0.05
    common = dict(N=N, n=n, bc="dirichlet", h=h, dt=0.004, c=0.6, nu=0.02, delta=1e-5, scheme=scheme,
                  nonlin="none" if scheme == "linear" else "allen_cahn", nl_coef=1.0, bc_left=0.3,
                  bc_right=-0.2)
    pu = make_problem(**common)
    px = make_problem(x=h * np.arange(N), **common)
    wu, wx = oracle.build_weights(pu), oracle.build_weights(px)
    assert np.max(np.abs(wu - wx)) <= 1e-13 * np.max(np.abs(wu))
    u0 = np.cos(np.linspace(0, 3, N))
    assert np.max(np.abs(oracle.run(pu, u0, 5) - oracle.run(px, u0, 5))) <= 1e-13


def _lagrange(xs, t):
    return np.array([np.prod([(t - xs[l]) / (xs[k] - xs[l]) for l in range(len(xs)) if l != k])
                     for k in range(len(xs))])


@pytest.mark.parametrize("n,i", [(5, 1), (9, 4), (13, 20), (21, 0), (21, 31)])
def test_theorem1_on_chebyshev_window(n, i):
    N, c, dt = 64, 1.3, 0.004
    x = _cheb(N)
    p = make_problem(N=N, n=n, bc="dirichlet", h=2.0 / (N - 1), dt=dt, c=c, scheme="linear", x=x)
    o = oracle.window_offset(p, i)
    w0 = oracle.build_weights(p)[i, 0]
    lag = _lagrange(x[i + o:i + o + n] - x[i], -c * dt)
    assert np.max(np.abs(w0 - lag)) <= 1e-12 * max(1.0, np.max(np.abs(lag)))


@pytest.mark.parametrize("n,i", [(7, 3), (11, 0), (21, 10), (21, 50)])
def test_heat_flow_of_polynomials(n, i):
    """e^{dt nu d2} x^k = sum_j (nu dt)^j k! / (j! (k-2j)!) x^(k-2j), and
    dt phi1 gives its integral over [0, dt]; coordinates relative to x_i."""
    N, nu, dt = 64, 1e-4, 0.01
    x = _cheb(N)
    p = make_problem(N=N, n=n, bc="dirichlet", h=2.0 / (N - 1), dt=dt, nu=nu, scheme="etd1",
                     nonlin="allen_cahn", nl_coef=1.0, x=x)
    o = oracle.window_offset(p, i)
    w = oracle.build_weights(p)[i]
    xs = x[i + o:i + o + n] - x[i]
    for k in range(n):
        flow = sum((nu * dt) ** j * math.factorial(k) / (math.factorial(j) * math.factorial(k - 2 * j))
                   * (0.0 ** (k - 2 * j)) for j in range(k // 2 + 1))
        integ = sum(nu ** j * dt ** (j + 1) / (j + 1) * math.factorial(k) / (math.factorial(j) *
                    math.factorial(k - 2 * j)) * (0.0 ** (k - 2 * j)) for j in range(k // 2 + 1))
        vals = xs ** k
        scale = max(1.0, np.sum(np.abs(w[0] * vals)))
        assert abs(w[0] @ vals - flow) <= 1e-13 * scale, k
        assert abs(w[1] @ vals - integ) <= 1e-13 * max(dt, np.sum(np.abs(w[1] * vals))), k


def _paper_ac(dt, N=64, n=21):
    x = _cheb(N)
    u0 = 0.53 * x + 0.47 * np.sin(-1.5 * np.pi * x)
    p = make_problem(N=N, n=n, bc="dirichlet", h=2.0 / (N - 1), dt=dt, nu=1e-4, scheme="etd1",
                     nonlin="allen_cahn", nl_coef=1.0, bc_left=-1.0, bc_right=1.0, x=x)
    return p, u0


def test_chebyshev_allen_cahn_run():
    """Sec. 4.3.3's run (N = 64, n = 21, Dirichlet -1 / 1) to t = 70: the ends
    hold, the state separates into phases near -1 and +1 and stays bounded."""
    p, u0 = _paper_ac(0.01)
    u = oracle.run(p, u0, 7000)
    assert u[0] == -1.0 and u[-1] == 1.0
    assert np.max(np.abs(u)) <= 1.02
    assert np.sum(np.abs(np.abs(u) - 1.0) < 0.05) >= 50


def test_paper_chebyshev_run_literal_coefficient():
    """The run as printed (nu = eps = 0.01) to t = 70 at dt = 1e-4: the same
    phase separation; at dt = 3e-4 the local scheme on this grid blows up."""
    import workloads
    p, u0 = workloads.allen_cahn_chebyshev()
    u = oracle.run(p, u0, 700000)
    assert u[0] == -1.0 and u[-1] == 1.0 and np.max(np.abs(u)) <= 1.02
    assert np.sum(np.abs(np.abs(u) - 1.0) < 0.05) >= 40
    q, _ = workloads.allen_cahn_chebyshev(dt=3e-4)
    bad = oracle.run(q, u0, 7000)
    assert not np.all(np.isfinite(bad)) or np.max(np.abs(bad)) > 10.0


def test_chebyshev_etd1_first_order_in_time():
    T = 1.0
    ref = oracle.run(_paper_ac(T / 3200)[0], _paper_ac(0.01)[1], 3200)
    errs = []
    for m in (100, 200, 400):
        p, u0 = _paper_ac(T / m)
        errs.append(np.max(np.abs(oracle.run(p, u0, m) - ref)))
    slopes = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert all(0.8 <= s <= 1.2 for s in slopes), (errs, slopes)


def test_unsupported_combinations_are_refused():
    p, u0 = _paper_ac(0.01)
    for bad in (dict(bc="periodic"), dict(window="upwind"), dict(nonlin="kdv", scheme="etd2rk"),
                dict(x=np.r_[p["x"][:10], p["x"][9], p["x"][11:]])):
        with pytest.raises(ValueError):
            oracle.run(dict(p, **bad), u0, 1)
    with pytest.raises(ValueError):
        oracle.adjoint_step(dict(p, scheme="etd1"), u0, u0)
