"""Differentiable LMEP time stepping: torch.autograd.Function over the C ABI.

Forward: ``lmep_step`` over ``steps`` steps, keeping the state every
``checkpoint_every`` steps (by default every step when all states fit in half
the free device memory, which on a 288 GB GPU is the common case, so nothing
is recomputed).  Backward: for each segment, last first, the states of the
segment are recomputed from its checkpoint one step at a time and
``lmep_adjoint_step`` (derivative of every node's weights -- by the finite
Taylor series where it applies, else by the block-triangular Pade exponential
-- plus the transposed banded apply) is applied backwards through them.  The result is the gradient with respect to
the initial state and to the per-instance coefficients nu, c and delta.

Only the bookkeeping (which state to recompute, which adjoint to pass on)
happens here; every derivative is computed by the library's kernels.
"""
from __future__ import annotations

import math

import torch

from . import Batch


class _Solve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, nu, c, delta, batch: Batch, steps: int, checkpoint_every: int):
        values = torch.stack([nu, c, delta], dim=1).detach().cpu().tolist()
        probs = [dict(p, nu=float(vn), c=float(vc), delta=float(vd)) for p, (vn, vc, vd) in zip(batch.problems, values)]
        b = Batch(probs, device=batch.device)
        w = b.empty_weights()
        stationary = any(p.get("nonlin") != "burgers_frozen" for p in b.problems)
        if stationary:
            b.build_weights(w, u0)
        ck = [u0.detach().clone()]
        u = u0.detach()
        done = 0
        while done < steps:
            k = min(checkpoint_every, steps - done)
            u = b.step(w, u, k)
            done += k
            if done < steps:
                ck.append(u.clone())
        ctx.b, ctx.w, ctx.ck = b, w, ck
        ctx.steps, ctx.every, ctx.stationary = steps, checkpoint_every, stationary
        return u

    @staticmethod
    def backward(ctx, grad_out):
        b, w, ck = ctx.b, ctx.w, ctx.ck
        lam = grad_out.detach().contiguous().clone()
        grad = torch.zeros(3 * b.count, dtype=torch.float64, device=b.device)
        nseg = len(ck)
        for seg in range(nseg - 1, -1, -1):
            first = seg * ctx.every
            k = min(ctx.every, ctx.steps - first)
            states = [ck[seg]]
            for _ in range(k - 1):  # recompute u^{first+1} .. u^{first+k-1}
                states.append(b.step(w, states[-1], 1))
            for st in range(k - 1, -1, -1):
                lam, grad = b.adjoint_step(states[st], lam, grad=grad)
        g = grad.view(b.count, 3)
        return lam, g[:, 0].clone(), g[:, 1].clone(), g[:, 2].clone(), None, None, None


def checkpoint_interval(steps: int, state_bytes: int, free_bytes: int, budget: float = 0.5) -> int:
    """Checkpoint interval: 1 (keep every state, no recomputation in the
    backward pass) when all `steps` states fit in `budget` of the free device
    memory, else ceil(sqrt(steps)), which keeps about 2 sqrt(steps) states
    alive (the checkpoints plus one recomputed segment)."""
    steps = max(1, int(steps))
    if steps * state_bytes <= budget * free_bytes:
        return 1
    return math.isqrt(steps - 1) + 1


def auto_checkpoint_every(batch: Batch, steps: int) -> int:
    """checkpoint_interval() for this batch on its device's free memory now."""
    free, _ = torch.cuda.mem_get_info(torch.device(batch.device))
    return checkpoint_interval(steps, batch.state_size * 8, free)


def solve(batch: Batch, u0: torch.Tensor, steps: int, nu=None, c=None, delta=None, checkpoint_every=None):
    """Advance the batch `steps` steps from the packed state u0, differentiably.

    nu, c, delta are optional per-instance tensors (shape [count]); when
    omitted, the batch's own coefficients are used (with zero gradient).
    checkpoint_every=None picks the interval by auto_checkpoint_every().
    """
    dev = batch.device
    if checkpoint_every is None:
        checkpoint_every = auto_checkpoint_every(batch, steps)

    def coef(x, key):
        if x is not None:
            return x
        return torch.tensor([float(p.get(key, 0.0)) for p in batch.problems], dtype=torch.float64, device=dev)

    return _Solve.apply(u0, coef(nu, "nu"), coef(c, "c"), coef(delta, "delta"), batch, int(steps),
                        int(checkpoint_every))
