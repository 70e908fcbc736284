"""Pins of the oracle's ETDRK4 (Sec. 3, ETDRK4 stages a, b, c and the final
update with alpha, beta, gamma; weights harvested from the augmented local
matrix of Sec. 3.1) against facts independent of the oracle's code:

* L = 0 reduces the scheme to classical fourth-order Runge-Kutta;
* N = 0 reduces it to the linear propagator (LINEAR scheme);
* the six harvested rows sum to 1, dt/2, 1, dt/6, dt/3, dt/6 (phi_j(0) = 1/j!
  and L annihilates constants);
* the rows equal the corresponding columns of scipy's exponential of the
  compact augmented matrix at dt/2 and at dt;
* the global error against a tight integration of the semi-discrete system
  u' = A u + N(u) falls at order 4 (and ETD2RK at order 2) on a resolved
  problem, the paper's fourth-order claim before the spatial floor;
* Dirichlet end nodes keep their values.
"""
from __future__ import annotations

import mpmath
import numpy as np
import pytest
import scipy.linalg
from scipy.integrate import solve_ivp

import oracle
from workloads import make_problem


def _rk4(f, u, dt):
    k1 = f(u)
    k2 = f(u + 0.5 * dt * k1)
    k3 = f(u + 0.5 * dt * k2)
    k4 = f(u + dt * k3)
    return u + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)


@pytest.mark.parametrize("n", [5, 9, 13, 19])
def test_zero_operator_is_classical_rk4(n):
    N, dt, g = 40, 0.07, 1.7
    p = make_problem(N=N, n=n, bc="periodic", h=0.1, dt=dt, scheme="etdrk4", nonlin="allen_cahn", nl_coef=g)
    u0 = np.random.default_rng(11).uniform(-0.6, 0.6, N)
    want = u0.copy()
    for _ in range(3):
        want = _rk4(lambda v: g * (v - v ** 3), want, dt)
    assert np.max(np.abs(oracle.run(p, u0, 3) - want)) <= 1e-15


@pytest.mark.parametrize("bc", ["periodic", "dirichlet", "neumann"])
def test_without_nonlinearity_is_the_linear_propagator(bc):
    common = dict(N=50, n=9, bc=bc, h=0.05, dt=0.01, c=0.7, nu=0.02, delta=1e-5, bc_left=0.2, bc_right=-0.1)
    u0 = np.cos(np.linspace(0, 4, 50))
    a = oracle.run(make_problem(scheme="etdrk4", nonlin="none", **common), u0, 4)
    b = oracle.run(make_problem(scheme="linear", **common), u0, 4)
    assert np.max(np.abs(a - b)) <= 1e-14


@pytest.mark.parametrize("n", [3, 5, 7, 9, 11, 13, 15, 17, 19])
def test_row_sums(n):
    dt = 0.13
    p = make_problem(N=n, n=n, bc="dirichlet", h=0.3, dt=dt, c=0.9, nu=0.04, delta=0.001, scheme="etdrk4",
                     nonlin="allen_cahn", nl_coef=1.0)
    w = oracle.build_weights(p)  # [node = harvest row, kind, k]
    want = [1.0, dt / 2, 1.0, dt / 6, dt / 3, dt / 6]
    for r in range(n):
        s = max(1.0, np.sum(np.abs(w[r, 0])))
        for kind in range(6):
            assert abs(w[r, kind].sum() - want[kind]) <= 1e-14 * s, (r, kind)


@pytest.mark.parametrize("n", [5, 9, 13, 19])
def test_rows_match_exponential_of_compact_matrices(n):
    """Half-step rows from expm of dt/2 [[L^T, e_r], [0, 0]]; full-step rows from
    expm of dt [[L^T, e_r, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1], [0, 0, 0, 0]], whose
    columns n, n+1, n+2 are dt phi1, dt^2 phi2, dt^3 phi3 applied to e_r."""
    h, dt = 0.2, 0.09
    D = oracle.fd_matrices(n, h)
    L = -0.6 * D[0] + 0.05 * D[1] - 0.001 * D[2]
    p = make_problem(N=n, n=n, bc="dirichlet", h=h, dt=dt, c=0.6, nu=0.05, delta=0.001, scheme="etdrk4",
                     nonlin="allen_cahn", nl_coef=1.0)
    w = oracle.build_weights(p)
    # FP64 expm is accurate enough up to n = 13; the n = 19 edge rows carry
    # large one-sided weights, so there the reference is a 40-digit expm of a
    # few rows (both edges, the centre)
    wide = n > 13

    def expm(M):
        if not wide:
            return scipy.linalg.expm(M)
        mpmath.mp.dps = 40
        return np.array(mpmath.expm(mpmath.matrix(M.tolist())).tolist(), dtype=float)

    for r in ((0, 1, n // 2, n - 2, n - 1) if wide else range(n)):
        Mh = np.zeros((n + 1, n + 1))
        Mh[:n, :n] = L.T
        Mh[r, n] = 1.0
        Eh = expm(0.5 * dt * Mh)
        Mf = np.zeros((n + 3, n + 3))
        Mf[:n, :n] = L.T
        Mf[r, n] = 1.0
        Mf[n, n + 1] = 1.0
        Mf[n + 1, n + 2] = 1.0
        Ef = expm(dt * Mf)
        phi1, phi2, phi3 = Ef[:n, n] / dt, Ef[:n, n + 1] / dt ** 2, Ef[:n, n + 2] / dt ** 3
        ref = [Eh[:n, r], Eh[:n, n], Ef[:n, r], dt * (phi1 - 3 * phi2 + 4 * phi3), dt * (2 * phi2 - 4 * phi3),
               dt * (4 * phi3 - phi2)]
        for kind in range(6):
            err = np.max(np.abs(w[r, kind] - ref[kind]))
            assert err <= 1e-13 * max(1.0, np.max(np.abs(ref[kind]))), (r, kind, err)


@pytest.mark.parametrize("n", [13, 19])
def test_fourth_order_in_time(n):
    """Periodic diffusion + Allen-Cahn, resolved (N = 64; n = 13, and the
    paper's n = 19): errors at T = 1 against the semi-discrete system
    integrated to 1e-13 fall by 2^4 per halving of dt for ETDRK4 and by 2^2
    for ETD2RK."""
    N, nu, g, T = 64, 0.02, 1.0, 1.0
    h = 2 * np.pi / N
    x = np.arange(N) * h
    u0 = 0.4 * np.sin(x) + 0.1
    D = oracle.fd_matrices(n, h)
    R = (n - 1) // 2
    row = nu * D[1][R]
    A = np.zeros((N, N))
    for i in range(N):
        for k in range(n):
            A[i, (i - R + k) % N] += row[k]
    ref = solve_ivp(lambda t, u: A @ u + g * (u - u ** 3), (0, T), u0, method="DOP853", rtol=1e-13,
                    atol=1e-15).y[:, -1]
    for scheme, order in (("etdrk4", 4.0), ("etd2rk", 2.0)):
        errs = []
        for m in (8, 16, 32, 64):
            p = make_problem(N=N, n=n, bc="periodic", h=h, dt=T / m, nu=nu, scheme=scheme, nonlin="allen_cahn",
                             nl_coef=g)
            errs.append(np.max(np.abs(oracle.run(p, u0, m) - ref)))
        slopes = [np.log2(errs[i] / errs[i + 1]) for i in range(3)]
        assert all(abs(s - order) <= 0.3 for s in slopes), (scheme, errs, slopes)


def test_dirichlet_ends_are_held():
    p = make_problem(N=40, n=7, bc="dirichlet", h=0.05, dt=0.002, c=0.3, nu=0.05, scheme="etdrk4",
                     nonlin="allen_cahn", nl_coef=1.0, bc_left=-1.0, bc_right=1.0)
    u0 = np.tanh(np.linspace(-2, 2, 40))
    u0[0], u0[-1] = -1.0, 1.0
    u = oracle.run(p, u0, 5)
    assert u[0] == -1.0 and u[-1] == 1.0
