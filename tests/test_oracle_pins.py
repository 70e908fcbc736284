"""Pins of the CPU oracle against facts the paper and mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints (tests/golden/), closed forms (Lagrange interpolation, Taylor
coefficients of scalar functions), exact rational arithmetic, library routines
(scipy / mpmath matrix exponentials), invariants, and complex-step
derivatives.  None of them re-types the oracle's own formula.
"""
from __future__ import annotations

import math
import os
from fractions import Fraction

import mpmath
import numpy as np
import pytest
import scipy.linalg

import oracle
from workloads import make_problem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            label, idx, exprs = [s.strip() for s in line.split("|")]
            rows.append((label, int(idx), [e.strip() for e in exprs.split(";")]))
    return rows


def _eval(expr, **vars_):
    return eval(expr, {"__builtins__": {}}, vars_)  # fixture expressions in nu / mu only


# ------------------------------------------------------------------ P1 ----
def test_printed_first_derivative_matrix():
    """D3^(1) printed in Example 1 (Sec. 2.2)."""
    with open(os.path.join(GOLDEN, "example1_D3_first_derivative.txt")) as f:
        rows = [[float(Fraction(t)) for t in l.split()] for l in f if l.strip() and not l.startswith("#")]
    for h in (1.0, 0.25, 3.0):
        D1, _, _ = oracle.fd_matrices(3, h)
        assert np.array_equal(D1 * h, np.array(rows))


def _exact_fd_row(xs, a, m):
    """Exact rational weights w with sum_k w_k x_k^q = d^m/dx^m x^q at x_a, q < n."""
    n = len(xs)
    A = [[Fraction(xs[k]) ** q for k in range(n)] for q in range(n)]
    b = [Fraction(math.factorial(q), math.factorial(q - m)) * Fraction(xs[a]) ** (q - m) if q >= m else Fraction(0)
         for q in range(n)]
    M = [A[q] + [b[q]] for q in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col] / M[col][col]
                M[r] = [M[r][c] - f * M[col][c] for c in range(n + 1)]
    return [M[k][n] / M[k][k] for k in range(n)]


@pytest.mark.parametrize("n", [3, 5, 7, 9, 11])
def test_fd_matrices_exact_rationals(n):
    """Every row of D^(1..3) equals the exact polynomial-exact weights (Sec. 2.1 step 1)."""
    xs = [Fraction(2 * k - (n - 1), 2) for k in range(n)]
    D = oracle.fd_matrices(n, 1.0)
    for m in (1, 2, 3):
        for a in range(n):
            exact = np.array([float(v) for v in _exact_fd_row(xs, a, m)])
            scale = max(1.0, np.max(np.abs(exact)))
            assert np.max(np.abs(D[m - 1][a] - exact)) <= 4e-15 * scale


@pytest.mark.parametrize("n", [3, 5, 9, 13, 15])
def test_fd_polynomial_exactness(n):
    """D^(m) differentiates every polynomial of degree < n exactly (Thm 1 proof)."""
    h = 0.37
    D = oracle.fd_matrices(n, h)
    x = h * (np.arange(n) - (n - 1) / 2)
    for m in (1, 2, 3):
        for q in range(n):
            want = np.zeros(n) if q < m else (math.factorial(q) / math.factorial(q - m)) * x ** (q - m)
            got = D[m - 1] @ x ** q
            scale = max(1.0, np.max(np.abs(want)), np.max(np.abs(D[m - 1])) * np.max(np.abs(x ** q)))
            assert np.max(np.abs(got - want)) <= 1e-13 * scale


# ------------------------------------------------------------------ P2 ----
@pytest.mark.parametrize("nu", [Fraction(3, 10), Fraction(-7, 8), Fraction(1, 3), Fraction(5, 2)])
def test_example1_lax_wendroff_beam_warming(nu):
    """Rows of exp(nu h D3^(1)) printed in Example 1 (Sec. 2.2)."""
    D1, _, _ = oracle.fd_matrices(3, 1.0)
    for label, r, exprs in _golden_rows("example1_advective_rows.txt"):
        want = np.array([float(_eval(e, nu=nu)) for e in exprs])
        w0, *_ = oracle.augmented_row(D1, float(nu), r, 0)
        assert np.max(np.abs(w0 - want)) <= 2e-15 * max(1.0, np.max(np.abs(want))), label
        # the same row through the problem API: a u_x with a = -nu (h = dt = 1)
        p = make_problem(N=3, n=3, bc="dirichlet", h=1.0, dt=1.0, c=-float(nu), scheme="linear")
        w = oracle.build_weights(p)
        node = {0: 0, 1: 1, 2: 2}[r]
        assert np.max(np.abs(w[node, 0] - want)) <= 2e-15 * max(1.0, np.max(np.abs(want))), label


# ------------------------------------------------------------------ P3 ----
@pytest.mark.parametrize("mu", [Fraction(1, 10), Fraction(1, 4), Fraction(2, 3), Fraction(3, 2)])
def test_example2_ftcs_and_five_point(mu):
    """Centre rows of exp(mu h^2 D_n^(2)) printed in Example 2 (Sec. 2.3)."""
    for label, n, exprs in _golden_rows("example2_diffusive_rows.txt"):
        want = np.array([float(_eval(e, mu=mu)) for e in exprs])
        for h in (1.0, 0.1):
            _, D2, _ = oracle.fd_matrices(n, h)
            w0, *_ = oracle.augmented_row(D2, float(mu) * h * h, (n - 1) // 2, 0)
            assert np.max(np.abs(w0 - want)) <= 4e-15 * max(1.0, np.max(np.abs(want))), (label, h)


# ------------------------------------------------------------------ P4 ----
@pytest.mark.parametrize("n", [3, 5, 7, 9, 11, 13])
def test_theorem1_lagrange_weights_at_departure_point(n):
    """Pure advection: each row of exp(-c dt D) is the Lagrange basis at x_r - c dt (Thm 1)."""
    h = 0.5
    x = h * (np.arange(n) - (n - 1) / 2)
    for cfl in (0.37, 1.0, 2.5, -1.8, 4.6):
        c, dt = math.copysign(1.3, cfl), abs(cfl) * h / 1.3
        # a Dirichlet grid of exactly n nodes: node r harvests row r of the one window
        w = oracle.build_weights(make_problem(N=n, n=n, bc="dirichlet", h=h, dt=dt, c=c, scheme="linear"))
        for r in range(n):
            t = x[r] - c * dt
            lag = np.array([np.prod([(t - x[l]) / (x[k] - x[l]) for l in range(n) if l != k]) for k in range(n)])
            # the series cancels more on edge rows at large shifts: 1e-14 up to |CFL| 2.5, 1e-13 beyond
            tol = 1e-14 if abs(cfl) <= 2.5 else 1e-13
            assert np.max(np.abs(w[r, 0] - lag)) <= tol * max(1.0, np.sum(np.abs(lag))), (cfl, r)


def test_integer_cfl_is_an_exact_shift():
    """Lagrangian CFL: the harvested stencil is a pure shift (Sec. 4.1 error floor)."""
    for n in (5, 9, 13):
        p = make_problem(N=64, n=n, bc="periodic", h=1.0, dt=2.0, c=1.0, scheme="linear")
        u0 = np.random.default_rng(3).normal(size=64)
        u1 = oracle.run(p, u0, 1)
        assert np.max(np.abs(u1 - np.roll(u0, 2))) <= 1e-14 * np.max(np.abs(u0)) * n


# ------------------------------------------------------------------ P5 ----
def _series(coeffs, nterms):
    return [Fraction(c) for c in coeffs] + [Fraction(0)] * (nterms - len(coeffs))


def _mul(a, b, n):
    return [sum((a[i] * b[k - i] for i in range(k + 1)), Fraction(0)) for k in range(n)]


def _phi_series(q, j, n):
    """Taylor coefficients (in z) of phi_j(q(z)) for q(0) = 0, truncated at z^n,
    from phi_j(x) = sum_k x^k / (k + j)!."""
    out = [Fraction(0)] * n
    power = [Fraction(1)] + [Fraction(0)] * (n - 1)
    for k in range(n):
        f = Fraction(1, math.factorial(k + j))
        out = [o + f * pw for o, pw in zip(out, power)]
        power = _mul(power, q, n)
    return out


@pytest.mark.parametrize("n,p,o", [(5, 2, -1), (5, 2, -2), (7, 1, -3), (7, 1, 0), (9, 2, -4), (3, 1, -2),
                                   (7, 3, -3), (9, 3, -2), (5, 3, 0)])
def test_theorem2_moments(n, p, o):
    """Exact evolution of the interpolant (Thm 2): applied to (x - x_i)^q, q < n,
    W0 returns q! [z^q] e^{dt P(z)}, W1 returns q! [z^q] dt phi1(dt P(z)), W2
    q! [z^q] dt phi2(dt P(z)) and W3 q! [z^q] dt phi3(dt P(z)), with
    P(z) = -c z + nu z^2 - delta z^3 the symbol."""
    h, dt, c, nu, de = Fraction(3, 10), Fraction(7, 100), Fraction(13, 10), Fraction(1, 20), Fraction(1, 1000)
    D = oracle.fd_matrices(n, float(h))
    L = -float(c) * D[0] + float(nu) * D[1] - float(de) * D[2]
    r = -o
    W = oracle.augmented_row(L, float(dt), r, p)
    q_ser = _series([0, -c * dt, nu * dt, -de * dt], n)
    targets = [_phi_series(q_ser, j, n) for j in range(4)]
    for j in (1, 2, 3):
        targets[j] = [dt * t for t in targets[j]]
    xrel = [(k - r) * h for k in range(n)]
    for kind in range(p + 1):
        for q in range(n):
            want = math.factorial(q) * targets[kind][q]
            got = sum(W[kind][k] * float(xrel[k]) ** q for k in range(n))
            assert abs(got - float(want)) <= 1e-13 * max(1.0, abs(float(want))) * 10 ** (q // 3), (kind, q)


# ------------------------------------------------------------------ P6 ----
@pytest.mark.parametrize("n", [3, 5, 7, 9, 11, 13])
def test_row_sums(n):
    """L annihilates constants: rows of e^{dt L}, dt phi1, dt phi2, dt phi3 sum to
    1, dt, dt/2, dt/6 (phi_j(0) = 1/j!)."""
    D = oracle.fd_matrices(n, 0.2)
    L = -0.9 * D[0] + 0.03 * D[1] - 0.0004 * D[2]
    dt = 0.11
    for r in range(n):
        w0, w1, w2, w3 = oracle.augmented_row(L, dt, r, 3)
        s = max(1.0, np.sum(np.abs(w0)))
        assert abs(w0.sum() - 1.0) <= 1e-14 * s
        assert abs(w1.sum() - dt) <= 1e-14 * s
        assert abs(w2.sum() - dt / 2) <= 1e-14 * s
        assert abs(w3.sum() - dt / 6) <= 1e-14 * s


# ------------------------------------------------------------------ P7 ----
@pytest.mark.parametrize("n,p", [(5, 1), (5, 2), (7, 1), (9, 2), (11, 1), (5, 3), (9, 3), (13, 3)])
def test_block_form_equals_compact_form(n, p):
    """First block row of the paper's block exponential (Sec. 3.1) equals the
    harvest from the compact matrix dt [[L^T, e_r, 0], [0, 0, 1], [0, 0, 0]],
    exponentiated by scipy's Pade scaling-and-squaring; the block matrix's lower
    block rows are [0, I, dt I, ...] (checked on the full block matrix)."""
    D = oracle.fd_matrices(n, 0.5)
    L = -0.8 * D[0] + 0.06 * D[1] - 0.002 * D[2]
    dt = 0.09
    m = n + p
    for r in range(n):
        M = np.zeros((m, m))
        M[:n, :n] = L.T
        M[r, n] = 1.0
        for b in range(1, p):
            M[n + b - 1, n + b] = 1.0
        E = scipy.linalg.expm(dt * M)
        W = oracle.augmented_row(L, dt, r, p)
        ref = [E[:n, r], E[:n, n]] + [E[:n, n + b] / dt ** b for b in range(1, p)]
        for kind in range(p + 1):
            assert np.max(np.abs(W[kind] - ref[kind])) <= 1e-13 * max(1.0, np.max(np.abs(ref[kind])))
    s = p + 1
    A = np.zeros((s * n, s * n))
    A[:n, :n] = L
    for b in range(s - 1):
        A[b * n:(b + 1) * n, (b + 1) * n:(b + 2) * n] = np.eye(n)
    E = scipy.linalg.expm(dt * A)
    assert np.allclose(E[n:2 * n, n:2 * n], np.eye(n), atol=1e-14)
    if s == 3:
        assert np.allclose(E[n:2 * n, 2 * n:], dt * np.eye(n), atol=1e-14)
        assert np.allclose(E[2 * n:, 2 * n:], np.eye(n), atol=1e-14)
    if s == 4:  # second block row [0, I, dt I, dt^2/2 I] (Sec. 3, augmented matrix)
        assert np.allclose(E[n:2 * n, 2 * n:3 * n], dt * np.eye(n), atol=1e-14)
        assert np.allclose(E[n:2 * n, 3 * n:], dt * dt / 2 * np.eye(n), atol=1e-14)


# ------------------------------------------------------------------ P8 ----
def _mp_block_row(L, dt, r, p, dps=50):
    mpmath.mp.dps = dps
    n = L.shape[0]
    s = p + 1
    A = mpmath.zeros(s * n, s * n)
    for a in range(n):
        for b in range(n):
            A[a, b] = mpmath.mpf(float(L[a, b])) * mpmath.mpf(dt)
    for blk in range(s - 1):
        for a in range(n):
            A[blk * n + a, (blk + 1) * n + a] = mpmath.mpf(dt)
    E = mpmath.expm(A)
    out = [np.array([float(E[r, k * n + j]) for j in range(n)]) for k in range(s)]
    if p == 2:
        out[2] = out[2] / dt
    return out


CONFIG_OPERATORS = [
    # (n, p, h, dt, c, nu, delta, harvested rows): shapes of the five workloads
    (5, 0, 2 * math.pi / 256, 2 * (2 * math.pi / 256), 1.0, 1e-3, 0.0, [2]),           # advection-diffusion CFL 2
    (7, 1, 0.04, 0.02, 1.8, 1e-2, 0.0, [1, 2, 3]),                                     # Burgers, edge + centre rows
    (9, 2, 200 / 2 ** 20, (4 / math.pi ** 3) * (200 / 2 ** 20) ** 3, 0.0, 0.0, 1.0, [4]),  # KdV
    (11, 1, 2 / 512, 0.5 * (2 / 512) ** 2 / 1e-4, 0.0, 1e-4, 0.0, [5]),                # Allen-Cahn n=11
    (9, 1, 0.02, 0.01, 1.5, 5e-3, 0.0, [1, 4]),                                        # adjoint Burgers
]


@pytest.mark.parametrize("case", CONFIG_OPERATORS)
def test_exponential_vs_50_digit_reference(case):
    """fact (c): the FP64 terminating series against a 50-digit exponential of
    the same (FP64) block matrix, on every workload's operator and rows."""
    n, p, h, dt, c, nu, de, rows = case
    D = oracle.fd_matrices(n, h)
    L = -c * D[0] + nu * D[1] - de * D[2]
    for r in rows:
        W = oracle.augmented_row(L, dt, r, p)
        ref = _mp_block_row(L, dt, r, p)
        for kind in range(p + 1):
            err = np.max(np.abs(W[kind] - ref[kind])) / np.max(np.abs(ref[kind]))
            assert err <= 2e-14, (r, kind, err)


# ------------------------------------------------------------------ P9 ----
def _phi_scalar(j, z):
    """phi_j(z) by the recursion phi_{j+1} = (phi_j - 1/j!)/z (Sec. 3), exact in mpmath."""
    mpmath.mp.dps = 60
    z = mpmath.mpf(z)
    f = mpmath.e ** z
    for k in range(j):
        f = (f - mpmath.mpf(1) / mpmath.factorial(k)) / z
    return float(f)


@pytest.mark.parametrize("z", [-3.0, -0.4, 0.05, 0.7, 2.0])
def test_one_node_stencil_gives_scalar_phi(z):
    """n = 1: the augmented row reduces to e^z, dt phi1(z), dt phi2(z), dt phi3(z)
    with z = react dt."""
    dt = 0.25
    L = np.array([[z / dt]])
    W = oracle.augmented_row(L, dt, 0, 3, nilpotent=False)
    assert abs(W[0][0] - math.exp(z)) <= 1e-15 * math.exp(abs(z))
    assert abs(W[1][0] - dt * _phi_scalar(1, z)) <= 2e-15 * dt * math.exp(abs(z))
    assert abs(W[2][0] - dt * _phi_scalar(2, z)) <= 2e-15 * dt * math.exp(abs(z))
    assert abs(W[3][0] - dt * _phi_scalar(3, z)) <= 2e-15 * dt * math.exp(abs(z))


def test_reaction_factor_theorem2():
    """L = c0 I + K: e^{dt L} = e^{c0 dt} e^{dt K} (Thm 2 proof)."""
    n, dt, c0 = 7, 0.13, -0.8
    D = oracle.fd_matrices(n, 0.3)
    K = -0.5 * D[0] + 0.02 * D[1]
    for r in (0, 3, 6):
        a, *_ = oracle.augmented_row(K + c0 * np.eye(n), dt, r, 0, nilpotent=False)
        b, *_ = oracle.augmented_row(K, dt, r, 0)
        assert np.max(np.abs(a - math.exp(c0 * dt) * b)) <= 1e-14 * np.max(np.abs(b))


# ------------------------------------------------------------------ P10 ---
@pytest.mark.parametrize("n", [5, 9, 13])
def test_fourier_mode_amplification(n):
    """fact (d): a periodic Fourier mode is multiplied by G(theta) = sum_k w_k
    e^{i (k - r) theta} in one step, and G approaches the exact symbol factor
    e^{dt P(i theta / h)} on resolved modes as n grows (Sec. 4.1, 4.2)."""
    N, h, c, nu, dt = 32, 0.2, 1.0, 0.01, 0.1
    p = make_problem(N=N, n=n, bc="periodic", h=h, dt=dt, c=c, nu=nu, scheme="linear")
    w = oracle.build_weights(p)[0, 0]
    r = (n - 1) // 2
    j = np.arange(N)
    for mode in (1, 3, 7):
        th = 2 * math.pi * mode / N
        G = np.sum(w * np.exp(1j * (np.arange(n) - r) * th))
        u = np.cos(th * j) + 0.0
        v = np.sin(th * j)
        ur, vr = oracle.run(p, u, 1), oracle.run(p, v, 1)
        got = ur + 1j * vr
        assert np.max(np.abs(got - G * np.exp(1j * th * j))) <= 1e-14


def test_fourier_trend_with_stencil_size():
    N, h, c, nu, dt = 32, 0.2, 1.0, 0.01, 0.1
    errs = []
    for n in (3, 5, 7, 9, 11):
        p = make_problem(N=N, n=n, bc="periodic", h=h, dt=dt, c=c, nu=nu, scheme="linear")
        w = oracle.build_weights(p)[0, 0]
        r = (n - 1) // 2
        th = 2 * math.pi * 2 / N
        G = np.sum(w * np.exp(1j * (np.arange(n) - r) * th))
        k = th / h
        exact = np.exp(dt * (-c * 1j * k - nu * k * k))
        errs.append(abs(G - exact))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs


def test_global_exponential_trend():
    """Tiny periodic grid: the dense global exponential of the n-point periodic
    FD matrix and the LMEP step agree on a resolved mode, ever closer as n grows
    (the dense propagator the method avoids, Sec. 2)."""
    N, h, c, nu, dt = 24, 0.25, 1.0, 0.02, 0.15
    j = np.arange(N)
    u = np.sin(2 * math.pi * j / N) + 0.5 * np.cos(4 * math.pi * j / N)
    errs = []
    for n in (3, 5, 7, 9):
        D = oracle.fd_matrices(n, h)
        r = (n - 1) // 2
        G = np.zeros((N, N))
        for i in range(N):
            for k in range(n):
                G[i, (i + k - r) % N] += -c * D[0][r, k] + nu * D[1][r, k]
        glob = scipy.linalg.expm(dt * G) @ u
        p = make_problem(N=N, n=n, bc="periodic", h=h, dt=dt, c=c, nu=nu, scheme="linear")
        errs.append(np.max(np.abs(oracle.run(p, u, 1) - glob)))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs


# ------------------------------------------------------------------ P12 ---
def test_periodic_mass_conservation():
    rng = np.random.default_rng(5)
    u0 = rng.normal(size=200)
    for p in (make_problem(N=200, n=7, bc="periodic", h=0.1, dt=0.05, c=1.2, nu=0.01, scheme="linear"),
              make_problem(N=200, n=9, bc="periodic", h=0.1, dt=0.05 * 0.1 ** 3, delta=1.0, scheme="etd2rk",
                           nonlin="kdv", nl_coef=6.0)):
        u1 = oracle.run(p, u0, 5)
        assert abs(u1.sum() - u0.sum()) <= 1e-12 * np.sum(np.abs(u0))


def test_neumann_equals_mirrored_periodic():
    N = 40
    rng = np.random.default_rng(6)
    u0 = rng.uniform(-0.1, 0.1, N)
    for n in (5, 9):
        pn = make_problem(N=N, n=n, bc="neumann", h=0.05, dt=0.5 * 0.05 ** 2 / 1e-2, nu=1e-2, scheme="etd1",
                          nonlin="allen_cahn", nl_coef=1.0)
        pp = dict(pn, N=2 * (N - 1), bc="periodic")
        mirrored = np.concatenate([u0, u0[-2:0:-1]])
        a = oracle.run(pn, u0, 3)
        b = oracle.run(pp, mirrored, 3)[:N]
        assert np.max(np.abs(a - b)) <= 1e-15


# ------------------------------------------------------------------ P13 ---
def test_zero_operator_reduces_to_euler_and_heun():
    N = 30
    u0 = np.random.default_rng(7).uniform(-0.5, 0.5, N)
    dt = 0.1
    p1 = make_problem(N=N, n=5, bc="periodic", h=0.1, dt=dt, scheme="etd1", nonlin="allen_cahn", nl_coef=1.0)
    f = lambda v: v - v ** 3
    assert np.max(np.abs(oracle.run(p1, u0, 1) - (u0 + dt * f(u0)))) <= 1e-16
    p2 = dict(p1, scheme="etd2rk")
    a = u0 + dt * f(u0)
    assert np.max(np.abs(oracle.run(p2, u0, 1) - (a + dt / 2 * (f(a) - f(u0))))) <= 1e-16


def test_temporal_orders():
    """ETD1 is first order, ETD2RK second order in dt (Sec. 3), on a smooth
    Allen-Cahn problem against a fine-step ETD2RK reference."""
    N, h, T = 64, 2 * math.pi / 64, 0.4
    x = h * np.arange(N)
    u0 = 0.5 * np.sin(x) + 0.2 * np.cos(2 * x)
    base = make_problem(N=N, n=9, bc="periodic", h=h, dt=1.0, nu=0.05, scheme="etd2rk", nonlin="allen_cahn",
                        nl_coef=1.0)
    ref = oracle.run(dict(base, dt=T / 1600), u0, 1600)
    for scheme, order in (("etd1", 1), ("etd2rk", 2)):
        errs = []
        for steps in (10, 20, 40):
            errs.append(np.max(np.abs(oracle.run(dict(base, scheme=scheme, dt=T / steps), u0, steps) - ref)))
        slopes = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
        assert all(abs(s - order) < 0.25 for s in slopes), (scheme, slopes)


# ------------------------------------------------------------------ a1 ----
def test_windows_are_in_domain_and_harvest_own_row():
    for N, n in ((9, 9), (10, 5), (40, 7), (41, 11)):
        p = make_problem(N=N, n=n, bc="dirichlet", h=1.0, dt=1.0)
        for i in range(N):
            o = oracle.window_offset(p, i)
            assert 0 <= i + o and i + o + n - 1 <= N - 1
            assert 0 <= -o <= n - 1
            # the n nearest nodes: centred unless an end forces a shift
            want = max(-i, min(-(n - 1) // 2, N - n - i))
            assert o == want
        pp = dict(p, bc="periodic")
        assert all(oracle.window_offset(pp, i) == -(n - 1) // 2 for i in range(N))


# ------------------------------------------------------- nilpotent D ----
@pytest.mark.parametrize("n", [3, 5, 7, 9, 11, 13, 15])
def test_window_operator_is_polynomial_in_nilpotent_first_derivative(n):
    """The stencil's derivative matrices are those of the degree n - 1
    interpolant (Sec. 2.1 step 1): D2 = D1^2, D3 = D1^3 and D1^n = 0, so every
    local operator -c D1 + nu D2 - delta D3 is a polynomial in a nilpotent
    matrix and its exponential a finite Taylor sum (the premise of the
    finite-Taylor weight build for frozen-velocity instances)."""
    h = 0.61
    D1, D2, D3 = oracle.fd_matrices(n, h)
    s1 = np.max(np.abs(D1))
    assert np.max(np.abs(D1 @ D1 - D2)) <= 1e-13 * s1 ** 2 * n
    assert np.max(np.abs(D1 @ D1 @ D1 - D3)) <= 1e-13 * s1 ** 3 * n ** 2
    P = np.eye(n)
    for _ in range(n):
        P = P @ D1
    assert np.max(np.abs(P)) <= 1e-12 * s1 ** n * n ** (n - 1)
    # and the degree n - 1 power does not vanish (index exactly n)
    Q = np.linalg.matrix_power(D1 * h, n - 1)
    assert np.max(np.abs(Q)) >= 0.5
