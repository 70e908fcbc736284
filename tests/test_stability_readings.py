"""Von Neumann / spectral-radius scans behind the time-step readings.

The paper fixes no time step for the throughput workloads, and some literal
settings amplify rounding without bound.  These scans, made with the oracle's
harvested weights, record which readings are stable (amplification factor
|G(theta)| of the periodic stencil, or spectral radius of the assembled banded
step matrix for Dirichlet grids), in the manner of the paper's spectral
footprints (Sec. 4.1) and stability boundary (Sec. 4.2, Remark on stability).
"""
from __future__ import annotations

import math

import numpy as np

import oracle
from workloads import make_problem


def max_amplification(p):
    n = p["n"]
    w = oracle.build_weights(dict(p, N=max(p["N"], n), bc="periodic", scheme="linear", nonlin="none"))[0, 0]
    r = (n - 1) // 2
    th = np.linspace(0.0, math.pi, 4001)
    G = np.exp(1j * np.outer(th, np.arange(n) - r)) @ w
    return float(np.max(np.abs(G))), float(np.abs(G[-1]))


def test_advection_diffusion_literal_cfl2_is_unstable_cfl1_is_not():
    h = 2 * math.pi / 256
    lit = make_problem(N=256, n=5, bc="periodic", h=h, dt=2 * h, c=1.0, nu=1e-3)
    gmax, gpi = max_amplification(lit)
    assert abs(gpi - 3.226) < 2e-3 and gmax == gpi          # |G(pi)| = 1 + 26.67 mu + 8 mu^2
    gmax1, _ = max_amplification(dict(lit, dt=h))
    assert gmax1 <= 1.0 + 1e-12
    pure, _ = max_amplification(dict(lit, nu=0.0))           # CFL 2, nu = 0: exact shift
    assert abs(pure - 1.0) <= 1e-12


def test_kdv_dispersive_readings():
    h = 200 / 2 ** 20
    base = make_problem(N=1024, n=9, bc="periodic", h=h, delta=1.0, dt=1.0)
    lit, _ = max_amplification(dict(base, dt=4.0 * h ** 3))
    assert lit > 1000.0                                       # literal dt/h^3 = 4: |G| ~ 1023
    g129, _ = max_amplification(dict(base, dt=(4 / math.pi ** 3) * h ** 3))
    g05, _ = max_amplification(dict(base, dt=0.05 * h ** 3))
    assert 5e-3 < g129 - 1 < 7e-3                             # growth ~1.5e5 over 2000 steps
    assert 2e-4 < g05 - 1 < 3e-4                              # growth ~1.7 over 2000 steps


def test_allen_cahn_diffusion_number_half_is_stable_for_all_stencils():
    for n in (5, 7, 9, 11):
        p = make_problem(N=512, n=n, bc="periodic", h=2 / 512, nu=1e-4, dt=0.5 * (2 / 512) ** 2 / 1e-4)
        g, _ = max_amplification(p)
        assert g <= 1.0 + 1e-12, n


def _dirichlet_step_matrix(p, velocity):
    """Assembled banded matrix of the LINEAR part with frozen velocity field."""
    N, n = p["N"], p["n"]
    w = oracle.build_weights(dict(p, scheme="etd1", nonlin="burgers_frozen", nl_coef=1.0), velocity)
    A = np.zeros((N, N))
    for i in range(1, N - 1):
        o = oracle.window_offset(p, i)
        A[i, i + o:i + o + n] = w[i, 0]
    return A


def test_burgers_dirichlet_reading_is_stable():
    """Velocity vanishing at the walls, CFL <= 1, mu <= 0.25: spectral radius < 1."""
    for n in (7, 9):
        N, nu = 48, 1e-2
        h = 4 * nu
        dt = min(h / 1.0, 0.25 * h * h / nu)
        x = np.linspace(0, 1, N)
        p = make_problem(N=N, n=n, bc="dirichlet", h=h, dt=dt, nu=nu)
        A = _dirichlet_step_matrix(p, np.sin(math.pi * x))
        rho = np.max(np.abs(np.linalg.eigvals(A)))
        assert rho < 1.0, (n, rho)


def test_burgers_literal_cfl8_is_unstable():
    """CFL 8 with a centred n = 7 stencil amplifies (the reading of the paper's 'CFL up to 8')."""
    h = 0.04
    p = make_problem(N=256, n=7, bc="periodic", h=h, c=1.0, nu=1e-2, dt=8 * h)
    g, _ = max_amplification(p)
    assert g > 10.0
