"""Pins of the oracle's nonlinear terms against closed forms that do not use its code.

Two terms reach the benchmark paths through the oracle and are pinned here:

* the frozen-velocity Burgers remainder N^(i)_j = -g (u_j - u_i) (du/dx)_j that
  node i applies through its phi1 row (ETD-s of Sec. 3 with the node's own
  velocity frozen into its local operator; Burgers of Sec. 4.3.1);
* the KdV term N = -(g/2) d/dx(u^2) (Sec. 4.3.2, conservative form of -g u u_x)
  inside the Cox-Matthews ETD2RK stages.

The closed forms rest on Thm 1's mechanism, that the window matrices act
exactly on polynomials of degree below n.  D1 maps the window values of a
polynomial f to those of f', and D2 = D1^2, D3 = D1^3 (full-stencil rows).  So
for data that is polynomial on every window involved, exp(s L) acts on the
values as the continuous semigroup exp(s A) with A = -a d/dx + nu d2/dx2 -
delta d3/dx3 acts on f.  On polynomials that semigroup is a finite sum:
(exp(s A) f)(x) = sum_k s^k/k! (A^k f)(x).  The phi rows are time integrals of it:
dt phi1(dt A) f = sum_k dt^(k+1)/(k+1)! A^k f and dt phi2(dt A) f =
sum_k dt^(k+1)/(k+2)! A^k f.  The expected values below come from that
continuous operator in exact rational arithmetic.  They use no difference
matrix, window rule or exponential of the oracle.

A sign, a factor or an index error in either term (N_j built from u_j alone,
(u_i - u_j), the derivative at i instead of j, a lost 1/2) changes these values
at first order in the perturbation.  The KdV soliton run then ties the
oracle's sign conventions to the equation itself: a right-moving
(c/2) sech^2 solitary wave of u_t + 6 u u_x + u_xxx = 0 must travel at speed c.
"""
from __future__ import annotations

import math
from fractions import Fraction as F

import numpy as np
import pytest

import oracle
from workloads import make_problem


# ---------------------------------------------------------------------------
# exact polynomial algebra: coefficient lists, lowest degree first
def _trim(p):
    p = list(p)
    while len(p) > 1 and p[-1] == 0:
        p.pop()
    return p


def _add(p, q):
    r = [F(0)] * max(len(p), len(q))
    for k, v in enumerate(p):
        r[k] += v
    for k, v in enumerate(q):
        r[k] += v
    return _trim(r)


def _scale(p, s):
    return _trim([s * v for v in p])


def _mul(p, q):
    r = [F(0)] * (len(p) + len(q) - 1)
    for a, x in enumerate(p):
        for b, y in enumerate(q):
            r[a + b] += x * y
    return _trim(r)


def _deriv(p, m=1):
    for _ in range(m):
        p = _trim([k * p[k] for k in range(1, len(p))] or [F(0)])
    return p


def _at(p, x):
    return sum(v * x ** k for k, v in enumerate(p))


def _apply_A(f, a, nu, delta):
    """A f = -a f' + nu f'' - delta f''' (the symbol of the local operator)."""
    return _add(_add(_scale(_deriv(f, 1), -a), _scale(_deriv(f, 2), nu)), _scale(_deriv(f, 3), -delta))


def _series(f, x, dt, a, nu, delta, shift):
    """sum_k dt^(k + shift) / (k + shift)! (A^k f)(x): shift 0 gives exp(dt A) f,
    shift 1 gives dt phi1(dt A) f.  Terminates because A lowers the degree."""
    total, g, k = F(0), list(f), 0
    while any(v != 0 for v in g):
        total += dt ** (k + shift) / math.factorial(k + shift) * _at(g, x)
        g = _apply_A(g, a, nu, delta)
        k += 1
    return total


def _series_phi2(f, x, dt, a, nu, delta):
    """dt phi2(dt A) f at x = sum_k dt^(k+1) / (k+2)! (A^k f)(x)."""
    total, g, k = F(0), list(f), 0
    while any(v != 0 for v in g):
        total += dt ** (k + 1) / math.factorial(k + 2) * _at(g, x)
        g = _apply_A(g, a, nu, delta)
        k += 1
    return total


def _values(p, xs):
    return np.array([float(_at(p, x)) for x in xs])


# ---------------------------------------------------------------------------
# frozen-velocity Burgers (ETD1)
def _burgers_closed_form(poly, N, h, dt, c, nu, g, i):
    """One frozen-velocity ETD1 step at node i of polynomial data u = poly:
    exp(dt A_i) u + dt phi1(dt A_i) q_i at x_i, with A_i advecting at the frozen
    speed c + g u_i and q_i(x) = -g (u(x) - u_i) u'(x)."""
    xi = i * h
    ui = _at(poly, xi)
    a = c + g * ui
    q = _scale(_mul(_add(poly, [-ui]), _deriv(poly)), -g)
    return _series(poly, xi, dt, a, nu, F(0), 0) + _series(q, xi, dt, a, nu, F(0), 1)


BURGERS_CASES = [
    # (name, n, N, h, dt, c, nu, g, polynomial coefficients (lowest first), window)
    ("linear_nu0", 7, 24, F(1, 8), F(1, 32), F(0), F(0), F(1), [F(3, 10), F(-2, 5)], "centred"),
    ("quadratic", 7, 24, F(1, 8), F(1, 32), F(0), F(1, 100), F(1), [F(1, 5), F(-3, 10), F(1, 8)], "centred"),
    ("cubic_speed_coef", 7, 22, F(1, 8), F(1, 64), F(1, 4), F(1, 50), F(3, 2),
     [F(-1, 10), F(2, 5), F(-1, 4), F(1, 16)], "centred"),
    ("quadratic_n5", 5, 20, F(1, 4), F(1, 16), F(0), F(1, 40), F(1), [F(1, 2), F(-1, 4), F(1, 20)], "centred"),
    ("quadratic_n9_upwind", 9, 26, F(1, 8), F(1, 32), F(1, 2), F(1, 200), F(1), [F(1, 5), F(1, 5), F(-1, 10)],
     "upwind"),
]


@pytest.mark.parametrize("case", BURGERS_CASES, ids=[c[0] for c in BURGERS_CASES])
def test_burgers_frozen_step_closed_form(case):
    """Every updated node of a Dirichlet grid (interior, clamped edge rows and,
    for upwind windows, per-node sides) equals the continuous closed form.
    Needs deg(u) <= (n - 1) / 2 so that the remainder (degree 2 deg(u) - 1) is
    still exact on every window."""
    name, n, N, h, dt, c, nu, g, poly, window = case
    assert 2 * (len(poly) - 1) - 1 < n
    xs = [j * h for j in range(N)]
    u0 = _values(poly, xs)
    p = make_problem(N=N, n=n, bc="dirichlet", h=float(h), dt=float(dt), c=float(c), nu=float(nu), scheme="etd1",
                     nonlin="burgers_frozen", nl_coef=float(g), bc_left=float(u0[0]), bc_right=float(u0[-1]),
                     window=window)
    got = oracle.run(p, u0, 1)
    want = np.array([float(_burgers_closed_form(poly, N, h, dt, c, nu, g, i)) for i in range(1, N - 1)])
    scale = np.max(np.abs(want))
    err = np.max(np.abs(got[1:-1] - want)) / scale
    assert err <= 2e-14, (name, err)
    assert got[0] == u0[0] and got[-1] == u0[-1]


def test_burgers_linear_data_two_term_form_and_local_error():
    """nu = 0, linear data u = alpha x + beta: Thm 1 (the exponential row is
    Lagrange interpolation at the departure point x_i - u_i dt) and the phi1 row
    of the linear remainder -alpha^2 (x - x_i) give
    u+_i = u_i (1 - alpha dt + alpha^2 dt^2 / 2).  The exact solution of
    u_t + u u_x = 0 is u_i / (1 + alpha t), so the local error is
    +alpha^2 u_i dt^2 / 2 + O(dt^3); a remainder of the wrong sign would give
    -alpha^2 u_i dt^2 / 2 in the first and 3/2 alpha^2 u_i dt^2 in the second."""
    alpha, beta, h, N = -0.4, 0.3, 0.125, 24
    x = h * np.arange(N)
    u0 = alpha * x + beta
    for dt in (1.0 / 32, 1.0 / 64, 1.0 / 128):
        p = make_problem(N=N, n=7, bc="dirichlet", h=h, dt=dt, nu=0.0, scheme="etd1", nonlin="burgers_frozen",
                         nl_coef=1.0, bc_left=u0[0], bc_right=u0[-1])
        got = oracle.run(p, u0, 1)[1:-1]
        ui = u0[1:-1]
        assert np.max(np.abs(got - ui * (1 - alpha * dt + 0.5 * alpha ** 2 * dt ** 2))) <= 1e-15
        exact = ui / (1 + alpha * dt)
        lead = 0.5 * alpha ** 2 * ui * dt ** 2   # exact - got to leading order
        rel = (exact - got) / lead
        assert np.all(np.abs(rel - 1.0) <= 2.5 * abs(alpha) * dt), (dt, rel.min(), rel.max())


def test_burgers_frozen_converges_to_semi_discrete_system():
    """Several steps on a smooth periodic problem converge at first order in dt
    to the semi-discrete advective Burgers system u_i' = -g u_i (D1 u)_i +
    nu (D2 u)_i: at node i the frozen split's remainder N^(i)_i vanishes, so
    this is what ETD1 integrates.  D1 and D2 here are the classical centred
    difference weights (exact rationals from the polynomial fit), written
    independently of the oracle."""
    from scipy.integrate import solve_ivp
    N, n, nu, g = 48, 5, 0.02, 1.0
    h = 2 * math.pi / N
    x = h * np.arange(N)
    u0 = 0.6 + 0.3 * np.sin(x) + 0.1 * np.cos(2 * x)
    d1 = np.array([1 / 12, -2 / 3, 0.0, 2 / 3, -1 / 12]) / h
    d2 = np.array([-1 / 12, 4 / 3, -5 / 2, 4 / 3, -1 / 12]) / h ** 2

    def rhs(_, u):
        win = np.stack([np.roll(u, 2 - k) for k in range(5)])  # win[k][i] = u[i + k - 2]
        return -g * u * (d1 @ win) + nu * (d2 @ win)

    T = 0.4
    ref = solve_ivp(rhs, (0, T), u0, method="DOP853", rtol=1e-13, atol=1e-13).y[:, -1]
    errs = []
    for steps in (20, 40, 80):
        p = make_problem(N=N, n=n, bc="periodic", h=h, dt=T / steps, nu=nu, scheme="etd1",
                         nonlin="burgers_frozen", nl_coef=g)
        errs.append(np.max(np.abs(oracle.run(p, u0, steps) - ref)))
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert all(0.9 <= r <= 1.15 for r in rates), (errs, rates)


# ---------------------------------------------------------------------------
# KdV (ETD2RK, Cox-Matthews)
def _kdv_closed_form(poly, h, dt, c, nu, delta, g, i):
    """One ETD2RK step at node i for polynomial data, N(v) = -(g/2) (v^2)':
    a = exp(dt A) u + dt phi1(dt A) N(u);  u+ = a + dt phi2(dt A) (N(a) - N(u)),
    all at x_i; a is formed as a polynomial (the stage is exact everywhere on
    the windows involved)."""
    xi = i * h

    def Nf(v):
        return _scale(_deriv(_mul(v, v)), -g / 2)

    Nu = Nf(poly)
    # a as a polynomial: exp(dt A) and dt phi1(dt A) map polynomials to polynomials
    a_poly = [F(0)]
    for f, shift in ((poly, 0), (Nu, 1)):
        gk, k = list(f), 0
        while any(v != 0 for v in gk):
            a_poly = _add(a_poly, _scale(gk, dt ** (k + shift) / math.factorial(k + shift)))
            gk = _apply_A(gk, c, nu, delta)
            k += 1
    diff = _add(Nf(a_poly), _scale(Nu, F(-1)))
    return _at(a_poly, xi) + _series_phi2(diff, xi, dt, c, nu, delta)


KDV_CASES = [
    # (name, n, N, h, dt, c, nu, delta, g, polynomial)
    ("kdv6_quadratic", 9, 30, F(1, 8), F(1, 1024), F(0), F(0), F(1), F(6), [F(1, 5), F(-3, 10), F(1, 4)]),
    ("kdv1_with_adv_diff", 9, 30, F(1, 8), F(1, 128), F(1, 3), F(1, 20), F(1, 2), F(1), [F(-1, 5), F(2, 5), F(-1, 8)]),
    ("kdv6_linear_n7", 7, 24, F(1, 8), F(1, 1024), F(0), F(0), F(1), F(6), [F(1, 2), F(-1, 3)]),
]


@pytest.mark.parametrize("case", KDV_CASES, ids=[c[0] for c in KDV_CASES])
def test_kdv_etd2rk_step_closed_form(case):
    """Interior nodes whose windows, and their windows' windows, avoid the held
    Dirichlet end nodes (i in [n, N-1-n]) equal the continuous closed form.
    Needs 4 deg(u) - 2 < n so that a^2 stays exact on every window."""
    name, n, N, h, dt, c, nu, delta, g, poly = case
    d = len(poly) - 1
    assert 2 * (2 * d - 1) < n
    xs = [j * h for j in range(N)]
    u0 = _values(poly, xs)
    p = make_problem(N=N, n=n, bc="dirichlet", h=float(h), dt=float(dt), c=float(c), nu=float(nu),
                     delta=float(delta), scheme="etd2rk", nonlin="kdv", nl_coef=float(g),
                     bc_left=float(u0[0]), bc_right=float(u0[-1]))
    got = oracle.run(p, u0, 1)
    idx = list(range(n, N - n))
    want = np.array([float(_kdv_closed_form(poly, h, dt, c, nu, delta, g, i)) for i in idx])
    err = np.max(np.abs(got[idx] - want)) / np.max(np.abs(want))
    assert err <= 2e-14, (name, err)


def _soliton(x, cs, x0, L):
    out = np.zeros_like(x)
    for s in (-L, 0.0, L):
        out += 0.5 * cs / np.cosh(0.5 * math.sqrt(cs) * (x - x0 - s)) ** 2
    return out


def test_kdv_soliton_travels_at_its_speed():
    """(c/2) sech^2(sqrt(c)(x - x0 - c t)/2) solves u_t + 6 u u_x + u_xxx = 0.
    The oracle's periodic ETD2RK run must follow it: the error against the
    translated wave falls as the stencil grows, and the best run is close to
    it; an opposite sign of either term moves the wave the wrong way or not at
    all (error of the wave's own size)."""
    L, N, cs, x0 = 30.0, 300, 2.0, 10.0
    h = L / N
    x = h * np.arange(N)
    dt = 0.05 * h ** 3
    steps = 4000
    T = steps * dt
    u0 = _soliton(x, cs, x0, L)
    want = _soliton(x, cs, x0 + cs * T, L)
    errs = {}
    for n in (5, 7, 9):
        p = make_problem(N=N, n=n, bc="periodic", h=h, dt=dt, delta=1.0, scheme="etd2rk", nonlin="kdv", nl_coef=6.0)
        errs[n] = np.max(np.abs(oracle.run(p, u0, steps) - want))
    assert errs[9] < errs[7] < errs[5], errs
    assert errs[9] <= 2e-4 * np.max(u0), errs
    # the wave moved by c T (a few grid cells), not by zero or backwards
    assert np.max(np.abs(u0 - want)) > 50 * errs[9]
