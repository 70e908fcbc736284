"""The reverse step and the checkpointed gradient at the adjoint workload's own
size: 64 viscous-Burgers trajectories of N = 262144 nodes, n = 9, frozen-velocity
ETD1, in the launch configuration the benchmark times (the whole batch in one
lmep_adjoint_step call per step).

* Two reverse steps of the whole batch, compared for trajectories 0 and 63 with
  the oracle's reverse steps: λ_k to 1e-10, and the accumulated (∂ν, ∂c, ∂δ)
  to 1e-10 or to the FP64 noise floor of the component, whichever is larger.
  The oracle's inputs are its own: its forward states and its own λ chain.

  The noise floor: on this grid the state is so smooth that a node's
  ν-derivative term is a stencil sum of O(dt/h^2) weights times O(1) values
  that cancels to O(dt |u_xx|), and the δ term cancels far more (O(dt/h^3)
  weights); summed over 262144 nodes, a component's value is fixed by the FP64
  inputs only to within sigma, the change of the oracle's own exact result
  when u and λ are perturbed by one unit in the last place with random signs
  (RMS over two draws).  An FP64 evaluation rounds about 4n^2 intermediate
  values per node at that same scale, which under the usual random-rounding
  model adds sqrt(4n^2) = 18 times sigma; the bound allows 64 sigma.  For ∂c
  this floor is about 1e-10 of the value, for ∂ν about 1e-7, and ∂δ (δ = 0
  here) is below FP64 resolution altogether.
* The full run -- 500 steps, a checkpoint every 50, loss against the state
  the same u0 reaches with ν·1.1 -- whose gradient in ν and along seeded
  smooth directions of u0 must match central differences (h = 1e-6) of the
  same loss.  This compares the library with itself (the oracle cannot run 500
  steps of 16.8M nodes in a test); it checks that checkpointing, recomputation
  and the reverse steps differentiate the forward path that actually ran.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import paper_2603_15964_amd as lmep
from paper_2603_15964_amd import autograd as lad
import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _case(*a):
    print("case:", *a, flush=True)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def test_reverse_steps_at_full_size_match_oracle():
    p, _, u0s = workloads.burgers_adjoint_batch()
    B, N = len(u0s), int(p["N"])
    checked = (0, B - 1)
    _case("C5 reverse steps", B, N)
    # forward states u^1, u^2 of the checked trajectories from the oracle; the
    # other trajectories take their own u0 (any state of the recipe will do)
    ora_states = {b: [u0s[b]] for b in checked}
    for b in checked:
        for _ in range(2):
            ora_states[b].append(oracle.run(p, ora_states[b][-1], 1))
    g = workloads.rng(77)
    lam_top = [g.normal(size=N) for _ in range(B)]
    batch = lmep.Batch([p] * B, device=DEV)
    lam = batch.pack(lam_top)
    grad = torch.zeros(3 * B, dtype=torch.float64, device=DEV)
    ora_lam = {b: lam_top[b] for b in checked}
    ora_grad = {b: np.zeros(3) for b in checked}
    floor = {b: np.zeros(3) for b in checked}
    ulp = 2.0 ** -52
    for k in (1, 0):
        states = [ora_states[b][k] if b in checked else u0s[b] for b in range(B)]
        lam, grad = batch.adjoint_step(batch.pack(states), lam, grad=grad)
        torch.cuda.synchronize()
        got = batch.unpack(lam)
        gg = grad.cpu().numpy().reshape(B, 3)
        for b in checked:
            u_k, lam_in = ora_states[b][k], ora_lam[b]
            ora_lam[b], dg = oracle.adjoint_step(p, u_k, lam_in)
            ora_grad[b] += dg
            draws = []
            for d in range(2):
                sg = np.where(workloads.rng(1000 * k + 10 * b + d).random((2, N)) < 0.5, -1.0, 1.0)
                _, dgp = oracle.adjoint_step(p, u_k * (1 + ulp * sg[0]), lam_in * (1 + ulp * sg[1]))
                draws.append((dgp - dg) ** 2)
            floor[b] += 64.0 * np.sqrt(np.mean(draws, axis=0))
            e = _rel(got[b], ora_lam[b])
            print(f"  step {k} trajectory {b}: lambda rel err {e:.2e}; gradient err "
                  f"{np.abs(gg[b] - ora_grad[b])} floor {floor[b]} value {ora_grad[b]}", flush=True)
            assert e <= 1e-10, (k, b, e)
            for c in range(3):
                bound = max(1e-10 * abs(ora_grad[b][c]), floor[b][c])
                assert abs(gg[b][c] - ora_grad[b][c]) <= bound, (k, b, c, gg[b][c], ora_grad[b][c], bound)


def test_full_run_gradient_matches_central_differences():
    """Loss 0.5 ||u(500) - target||^2 over the whole batch.  The central
    differences carry an O(h^2) truncation error and a rounding error of about
    eps * ||u(T) - target||_1 / h; at these magnitudes both stay far below the
    1e-5 relative bound."""
    p, pt, u0s = workloads.burgers_adjoint_batch()
    B = len(u0s)
    steps, every, hfd = 500, 50, 1e-6
    _case("C5 full-run gradient vs central differences", B, p["N"], steps, every)
    batch = lmep.Batch([p] * B, device=DEV)
    tbatch = lmep.Batch([pt] * B, device=DEV)
    u0 = batch.pack(u0s)
    with torch.no_grad():
        target = lad.solve(tbatch, u0, steps, checkpoint_every=steps)

    def loss_at(nu_shift=0.0, du=None):
        b = batch if nu_shift == 0.0 else lmep.Batch([dict(p, nu=p["nu"] + nu_shift)] * B, device=DEV)
        x0 = u0 if du is None else u0 + du
        with torch.no_grad():
            uT = lad.solve(b, x0, steps, checkpoint_every=steps)
        return 0.5 * float(torch.sum((uT - target) ** 2))

    x = u0.clone().requires_grad_(True)
    nu = torch.full((B,), p["nu"], dtype=torch.float64, device=DEV, requires_grad=True)
    uT = lad.solve(batch, x, steps, nu=nu, checkpoint_every=every)
    loss = 0.5 * torch.sum((uT - target) ** 2)
    loss.backward()
    gnu = float(nu.grad.sum())
    fd_nu = (loss_at(hfd) - loss_at(-hfd)) / (2 * hfd)
    print(f"  d loss / d nu: {gnu:.12e} (FD {fd_nu:.12e})", flush=True)
    assert abs(gnu - fd_nu) <= 1e-5 * abs(fd_nu)
    # seeded random directions in the span of the recipe's eight sine modes per
    # trajectory (zero at the held Dirichlet ends).  A direction spread over
    # all 16.8M nodes with independent entries would project the smooth
    # gradient onto it sqrt(N) times more weakly, and its differences (2h
    # times a derivative near 1e-12) would fall to the level of the rounding
    # the 500 forward steps leave in the loss.
    N = int(p["N"])
    xs = np.arange(N) / (N - 1)
    modes = np.stack([np.sin(k * np.pi * xs) for k in range(1, 9)])
    g = workloads.rng(1234)
    for j in range(2):
        d = np.concatenate([g.normal(size=8) @ modes for _ in range(B)])
        d = torch.from_numpy(d / np.linalg.norm(d)).to(DEV)
        gd = float(torch.dot(x.grad, d))
        fd = (loss_at(du=hfd * d) - loss_at(du=-hfd * d)) / (2 * hfd)
        print(f"  direction {j}: {gd:.12e} (FD {fd:.12e})", flush=True)
        assert abs(gd - fd) <= 1e-5 * abs(fd)
