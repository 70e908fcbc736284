"""Seeded synthetic workloads shaped like the paper's benchmark runs.

This module holds input generation only (random initial states, grid sizes,
stencil sizes and the derived time steps).  It contains none of the method's
arithmetic, so both the HIP path and the CPU oracle can take their inputs from
it.  Every generator uses numpy's PCG64 with a fixed seed.

Problems are plain dicts with the keys

    N, n, bc, h, dt, c, nu, delta, react, scheme, nonlin, nl_coef,
    bc_left, bc_right, window

describing  u_t = -c u_x + nu u_xx - delta u_xxx + react u + N(u)  on a uniform
grid of N nodes with spacing h (Sec. 2: grid of N points, stencil size n,
time step dt, coefficients of the coupled operator, boundary handling).

The five workloads stand in for the paper's experiments (Sec. 4: coupled
advection-diffusion, Burgers, KdV, Allen-Cahn); the paper ships no data, so
every input is synthetic.
"""
from __future__ import annotations

import math

import numpy as np

BASE_SEED = 1000


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def make_problem(**kw) -> dict:
    p = dict(N=0, n=5, bc="periodic", h=1.0, dt=1.0, c=0.0, nu=0.0, delta=0.0, react=0.0,
             scheme="linear", nonlin="none", nl_coef=0.0, bc_left=0.0, bc_right=0.0, window="centred", x=None)
    unknown = set(kw) - set(p)
    if unknown:
        raise KeyError(f"unknown problem keys {sorted(unknown)}")
    p.update(kw)
    return p


def stencil_p(scheme: str) -> int:
    """Highest phi-function a scheme uses (p; its augmented local matrix has order n + p)."""
    return {"linear": 0, "etd1": 1, "etd2rk": 2, "etdrk4": 3}[scheme]


# ---------------------------------------------------------------- C1 ------
def advection_diffusion(N: int = 256, cfl: float = 2.0, n: int = 5, c: float = 1.0, nu: float = 1e-3,
                        seed: int = BASE_SEED + 0):
    """Periodic u_t + c u_x = nu u_xx on [0, 2pi): periodised Gaussian (centre
    U[1,5], width 0.3) plus four sine modes with N(0, 0.1) amplitudes."""
    L = 2.0 * math.pi
    h = L / N
    x = h * np.arange(N)
    g = rng(seed)
    xc = g.uniform(1.0, 5.0)
    a = g.normal(0.0, math.sqrt(0.1), 4)
    u0 = sum(np.exp(-((x - xc - s) ** 2) / (2 * 0.3 ** 2)) for s in (-L, 0.0, L))
    for k in range(1, 5):
        u0 = u0 + a[k - 1] * np.sin(k * x)
    p = make_problem(N=N, n=n, bc="periodic", h=h, dt=cfl * h / c, c=c, nu=nu, scheme="linear")
    return p, u0


# ---------------------------------------------------------------- C2 ------
def _dirichlet_modes(g: np.random.Generator, x: np.ndarray, length: float, modes: int = 8) -> np.ndarray:
    a = g.normal(0.0, 1.0, modes) / np.arange(1, modes + 1)  # N(0, 1/k^2)
    return sum(a[k - 1] * np.sin(k * math.pi * x / length) for k in range(1, modes + 1))


def burgers(N: int = 65536, n: int = 7, nu: float = 1e-2, cfl: float = 1.0, mu: float = 0.25,
            seed: int = BASE_SEED + 1):
    """Viscous Burgers u_t + u u_x = nu u_xx on [0, (N-1)h], h = 4 nu, with
    Dirichlet u = 0 ends; frozen-velocity ETD1.  u0 = sum of 8 sine modes with
    N(0, 1/k^2) amplitudes.  dt = min(cfl h / max|u0|, mu h^2 / nu)."""
    h = 4.0 * nu
    length = (N - 1) * h
    x = h * np.arange(N)
    u0 = _dirichlet_modes(rng(seed), x, length)
    dt = min(cfl * h / float(np.max(np.abs(u0))), mu * h * h / nu)
    p = make_problem(N=N, n=n, bc="dirichlet", h=h, dt=dt, nu=nu, scheme="etd1",
                     nonlin="burgers_frozen", nl_coef=1.0)
    return p, u0


# ---------------------------------------------------------------- C3 ------
def kdv(N: int = 2 ** 20, n: int = 9, tau: float = 4.0 / math.pi ** 3, length: float = 200.0,
        seed: int = BASE_SEED + 2):
    """Periodic KdV u_t + 6 u u_x + u_xxx = 0 on [0, 200): two solitons
    (c/2) sech^2(sqrt(c)(x - x0)/2), c ~ U[1,4], x0 ~ U[0,200); ETD2RK;
    dt = tau h^3 (dispersive number tau = dt/h^3)."""
    h = length / N
    x = h * np.arange(N)
    g = rng(seed)
    cs = g.uniform(1.0, 4.0, 2)
    x0 = g.uniform(0.0, length, 2)
    u0 = np.zeros(N)
    for cc, xx in zip(cs, x0):
        for s in (-length, 0.0, length):
            u0 += 0.5 * cc / np.cosh(0.5 * math.sqrt(cc) * (x - xx - s)) ** 2
    p = make_problem(N=N, n=n, bc="periodic", h=h, dt=tau * h ** 3, delta=1.0, scheme="etd2rk",
                     nonlin="kdv", nl_coef=6.0)
    return p, u0


# ---------------------------------------------------------------- C4 ------
def allen_cahn_batch(count: int = 4096, n_min: int = 512, n_max: int = 65536, stencils=(5, 7, 9, 11),
                     eps2: float = 1e-4, mu: float = 0.5, seed: int = BASE_SEED + 3):
    """Independent 1-D Allen-Cahn instances u_t = eps^2 u_xx + u - u^3 on
    [-1, 1]: N_k ~ U{n_min..n_max}, n_k from `stencils`, periodic or Neumann
    with probability 1/2 each, dt_k = mu h_k^2 / eps^2, ETD1, u0 ~ U[-0.1, 0.1]."""
    g = rng(seed)
    Ns = g.integers(n_min, n_max + 1, count)
    ns = g.choice(np.asarray(stencils), count)
    bcs = g.integers(0, 2, count)
    probs, states = [], []
    for N, n, b in zip(Ns, ns, bcs):
        N, n = int(N), int(n)
        bc = "periodic" if b == 0 else "neumann"
        h = 2.0 / N if bc == "periodic" else 2.0 / (N - 1)
        probs.append(make_problem(N=N, n=n, bc=bc, h=h, dt=mu * h * h / eps2, nu=eps2, scheme="etd1",
                                  nonlin="allen_cahn", nl_coef=1.0))
        states.append(g.uniform(-0.1, 0.1, N))
    return probs, states


# ---------------------------------------------------------------- C5 ------
def burgers_adjoint_batch(batch: int = 64, N: int = 262144, n: int = 9, nu: float = 5e-3,
                          nu_factor: float = 1.1, cfl: float = 1.0, mu: float = 0.25,
                          seed: int = BASE_SEED + 4):
    """Batch of viscous-Burgers trajectories for the adjoint workload: the C2
    recipe with h = 4 nu, trajectory b seeded with seed + b, one common dt.
    Returns (problem, target_problem, u0 list); the target problem uses
    nu * nu_factor on the same grid and dt."""
    h = 4.0 * nu
    length = (N - 1) * h
    x = h * np.arange(N)
    u0s = [_dirichlet_modes(rng(seed + b), x, length) for b in range(batch)]
    umax = max(float(np.max(np.abs(u))) for u in u0s)
    dt = min(cfl * h / umax, mu * h * h / nu)
    p = make_problem(N=N, n=n, bc="dirichlet", h=h, dt=dt, nu=nu, scheme="etd1",
                     nonlin="burgers_frozen", nl_coef=1.0)
    pt = dict(p, nu=nu * nu_factor)
    return p, pt, u0s


# ------------------------------------------------- ETDRK4 (next row) ------
def burgers_etdrk4(N: int = 2 ** 20, n: int = 19, nu: float = 0.03, mu: float = 0.5):
    """The paper's own Burgers run (Sec. 4.3.1) at a throughput size: periodic
    [-pi, pi), nu = 0.03, u0 = exp(-10 sin^2(x/2)), stationary L = nu D2 and
    N = -u u_x in the conservative form -(1/2) d/dx(u^2) (the KdV-form term with
    coefficient 1), ETDRK4 with the paper's n = 19; dt = mu h^2 / nu.
    Deterministic, no seed."""
    h = 2.0 * math.pi / N
    x = -math.pi + h * np.arange(N)
    u0 = np.exp(-10.0 * np.sin(x / 2.0) ** 2)
    p = make_problem(N=N, n=n, bc="periodic", h=h, dt=mu * h * h / nu, nu=nu, scheme="etdrk4", nonlin="kdv",
                     nl_coef=1.0)
    return p, u0


# --------------------------------------------- upwind windows (next row) --
def burgers_upwind(N: int = 65536, n: int = 7, nu: float = 2.5e-3, cfl: float = 3.5, modes: int = 8,
                   seed: int = BASE_SEED + 5, amp: float = 0.1):
    """Viscous Burgers at high Courant number on fully one-sided stencils
    (Sec. 4.1 runs them at CFL (n+1)/2 - sigma): periodic, h = 16 nu (cell
    Peclet number 16, so the diffusion number cfl/16 stays inside the
    one-sided rows' stable range), u0 = 1 + 0.1 p(x) / max|p| with p a sum of 8
    sine modes, amplitudes N(0, 1/k^2), phases U[0, 2pi); dt = cfl h / mean(u0),
    so every node's Courant number lies in [0.9, 1.1] * cfl (amp = 0.1), inside
    the stable band [(n-3)/2, (n+1)/2].  Frozen-velocity ETD1 with
    window="upwind".  (For n >= 13 the explicit frozen-velocity term amplifies
    grid-scale perturbations unless amp is small.)"""
    h = 16.0 * nu
    length = N * h
    x = h * np.arange(N)
    g = rng(seed)
    a = g.normal(0.0, 1.0, modes) / np.arange(1, modes + 1)
    ph = g.uniform(0.0, 2.0 * math.pi, modes)
    pert = sum(a[k - 1] * np.sin(2.0 * math.pi * k * x / length + ph[k - 1]) for k in range(1, modes + 1))
    u0 = 1.0 + amp * pert / float(np.max(np.abs(pert)))
    p = make_problem(N=N, n=n, bc="periodic", h=h, dt=cfl * h / float(np.mean(u0)), nu=nu, scheme="etd1",
                     nonlin="burgers_frozen", nl_coef=1.0, window="upwind")
    return p, u0


def upwind_advection(n: int = 15, N: int = 2 ** 20, sigma: float = 0.5, modes: int = 8,
                     seed: int = BASE_SEED + 7):
    """Linear advection u_t + u_x = 0 on fully one-sided stencils at the
    Courant numbers of Sec. 4.1's efficiency runs, nu = (n+1)/2 - sigma
    (sigma = 1/2: departure points half-way between nodes): periodic [0, 1),
    u0 a sum of 8 sine modes with amplitudes N(0, 1/k^2) and phases U[0, 2pi).
    dt = nu h grows with n, so a fixed final time takes fewer steps."""
    h = 1.0 / N
    x = h * np.arange(N)
    g = rng(seed)
    a = g.normal(0.0, 1.0, modes) / np.arange(1, modes + 1)
    ph = g.uniform(0.0, 2.0 * math.pi, modes)
    u0 = sum(a[k - 1] * np.sin(2.0 * math.pi * k * x + ph[k - 1]) for k in range(1, modes + 1))
    cfl = (n + 1) / 2 - sigma
    p = make_problem(N=N, n=n, bc="periodic", h=h, dt=cfl * h, c=1.0, scheme="linear", window="upwind")
    return p, u0


# ---------------------------------------- Chebyshev grids (next row) -----
def chebyshev(N: int) -> np.ndarray:
    """Chebyshev points of the second kind on [-1, 1], increasing."""
    return -np.cos(np.pi * np.arange(N) / (N - 1))


def allen_cahn_chebyshev(N: int = 64, n: int = 21, nu: float = 0.01, dt: float = 1e-4):
    """The paper's Allen-Cahn run (Sec. 4.3.3): u_t = nu u_xx + u - u^3 on a
    Chebyshev grid on [-1, 1], Dirichlet u(-1) = -1, u(1) = 1,
    u0 = 0.53 x + 0.47 sin(-1.5 pi x), ETD1 with per-node stationary weights.
    nu = eps = 0.01 as printed there; on this grid the local scheme is stable
    for dt <= 2e-4 (3e-4 blows up), so dt = 1e-4, the step of the paper's
    reference solution (t = 70 in 700,000 steps).  Deterministic."""
    x = chebyshev(N)
    u0 = 0.53 * x + 0.47 * np.sin(-1.5 * math.pi * x)
    p = make_problem(N=N, n=n, bc="dirichlet", h=2.0 / (N - 1), dt=dt, nu=nu, scheme="etd1",
                     nonlin="allen_cahn", nl_coef=1.0, bc_left=-1.0, bc_right=1.0, x=x)
    return p, u0


def allen_cahn_chebyshev_batch(count: int = 8192, N: int = 64, n: int = 21, nu_range=(0.005, 0.01),
                               dt: float = 1e-4, seed: int = BASE_SEED + 6):
    """A batch of the paper's Chebyshev Allen-Cahn instance: nu ~ U[0.005, 0.01]
    per instance and u0 = the paper's profile + N(0, 0.01^2) noise at the
    interior nodes; every instance carries its own copy of the grid."""
    g = rng(seed)
    probs, states = [], []
    for _ in range(count):
        p, u0 = allen_cahn_chebyshev(N=N, n=n, nu=float(g.uniform(*nu_range)), dt=dt)
        u0 = u0.copy()
        u0[1:-1] += g.normal(0.0, 0.01, N - 2)
        probs.append(p)
        states.append(u0)
    return probs, states


STEPS = {"advection_diffusion": 100, "burgers": 1000, "kdv": 2000, "allen_cahn_batch": 500,
         "burgers_adjoint_batch": 500, "burgers_etdrk4": 1000, "burgers_upwind": 1000,
         "allen_cahn_chebyshev": 700000, "allen_cahn_chebyshev_batch": 500}
