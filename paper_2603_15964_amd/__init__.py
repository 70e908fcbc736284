"""LMEP hot path on AMD Instinct MI355X (gfx950).

The Local Matrix Exponential Propagator builds, for every grid node, the
exponential of a small local operator on the node's stencil (plus the
augmented matrix that yields the ETD phi-weights), harvests the node's row,
and applies the harvested rows as a banded stencil each time step.  All of
that runs in the HIP kernels of ``liblmep.so``; this package only marshals
arguments through the C ABI of ``include/lmep.h``.  PyTorch provides device
memory and streams.

``Batch`` packs a list of problem dicts (keys as in ``workloads``) into flat
device buffers and calls the entry points: ``lmep_build_weights``, and
``lmep_step`` / ``lmep_adjoint_step`` through plans (``lmep_plan_*``) that it
keeps per operation and option values, each with its own scratch buffer, so
repeated calls enqueue kernels only; ``use_plans=False`` calls the plain entry
points instead.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._native import (  # noqa: F401  (re-exported names of the C ABI)
    EXPORTED, LIB_PATH, LMEP_BC_DIRICHLET, LMEP_BC_NEUMANN, LMEP_BC_PERIODIC, LMEP_ERR_ARG, LMEP_ERR_DEVICE,
    LMEP_ERR_NONFINITE, LMEP_ERR_SCRATCH, LMEP_ERR_UNSUPPORTED, LMEP_ETD1, LMEP_ETD2RK, LMEP_ETDRK4, LMEP_EXP_AUTO,
    LMEP_EXP_PADE, LMEP_F_CHECK_FINITE, LMEP_F_COUNT, LMEP_F_GRAPH, LMEP_F_PERSISTENT, LMEP_F_PROFILE, LMEP_LINEAR,
    LMEP_NL_ALLEN_CAHN, LMEP_NL_BURGERS_FROZEN, LMEP_NL_KDV, LMEP_NL_NONE, LMEP_OK, LMEP_OPT_APPLY_TILE,
    LMEP_OPT_EXP_METHOD, LMEP_OPT_FUSE_FROZEN, LMEP_OPT_PROFILE_ADJOINT, LMEP_OPT_STEPS_PER_LAUNCH,
    LMEP_OPT_TAYLOR_REGION, LMEP_OPT_MERGE_GROUPS, LMEP_WIN_CENTRED,
    LMEP_WIN_UPWIND, OP_ADJOINT, OP_BUILD, OP_STEP, LmepError, library, lmep_adjoint_step, lmep_build_weights,
    lmep_get_option, lmep_last_error, lmep_problem, lmep_profile_last, lmep_scratch_bytes, lmep_set_option, lmep_step,
    lmep_step_noalloc, lmep_weight_count, problem_array, to_struct, LMEP_NOALLOC_SCRATCH_BYTES, lmep_plan_create,
    lmep_plan_step, lmep_plan_adjoint_step, lmep_plan_destroy, lmep_profile_kernels, option_generation)

_OPTIONS = (LMEP_OPT_STEPS_PER_LAUNCH, LMEP_OPT_PROFILE_ADJOINT, LMEP_OPT_FUSE_FROZEN, LMEP_OPT_APPLY_TILE,
            LMEP_OPT_EXP_METHOD, LMEP_OPT_TAYLOR_REGION, LMEP_OPT_MERGE_GROUPS)

_KINDS = {"linear": 1, "etd1": 2, "etd2rk": 3, "etdrk4": 6}


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class Batch:
    """A batch of independent LMEP instances packed into flat FP64 buffers.

    Instance k's state occupies ``[state_off[k], state_off[k] + N_k)`` of every
    state tensor and its weights ``[weight_off[k], ...)`` of the weight tensor
    (layouts in include/lmep.h).
    """

    def __init__(self, problems, device="cuda:0", use_plans: bool = True):
        self.use_plans = use_plans
        self._plans = {}
        self.problems = [dict(p) for p in problems]
        self.device = torch.device(device)
        self.count = len(self.problems)
        so, wo = 0, 0
        self.state_off, self.weight_off, self.weight_len = [], [], []
        # coordinates of the non-uniform grids, packed into one device tensor
        xs = [np.asarray(p["x"], dtype=np.float64) for p in self.problems if p.get("x") is not None]
        for p, x in zip([p for p in self.problems if p.get("x") is not None], xs):
            assert x.shape == (int(p["N"]),)
        self._coords = torch.from_numpy(np.concatenate(xs)).to(self.device) if xs else None
        xo = 0
        structs = []
        for p in self.problems:
            x_ptr = None
            if p.get("x") is not None:
                x_ptr = self._coords.data_ptr() + 8 * xo
                xo += int(p["N"])
            s = to_struct(p, so, wo, x_ptr)
            wl = lmep_weight_count(s)
            structs.append(s)
            self.state_off.append(so)
            self.weight_off.append(wo)
            self.weight_len.append(wl)
            so += int(p["N"])
            wo += (wl + 31) // 32 * 32
        self.structs = problem_array(structs)
        self.state_size = so
        self.weight_size = wo
        self._scratch = {}

    def __del__(self):
        self.release_plans()

    def release_plans(self):
        """Destroy the cached plans (their scratch tensors go with them)."""
        plans, self._plans = getattr(self, "_plans", {}), {}
        for handle, _ in plans.values():
            try:
                lmep_plan_destroy(handle)
            except Exception:  # noqa: BLE001 -- interpreter shutdown
                pass

    def plan(self, op: int, flags: int = 0) -> int:
        """The cached plan of op (OP_STEP or OP_ADJOINT) for the current
        process-wide option values; LMEP_F_PERSISTENT in flags selects the
        multi-step step plan."""
        persistent = int(flags) & LMEP_F_PERSISTENT if op == OP_STEP else 0
        gen = option_generation()
        if getattr(self, "_opts_gen", None) != gen:
            self._opts = tuple(lmep_get_option(o) for o in _OPTIONS)
            self._opts_gen = gen
        key = (op, persistent, self._opts)
        if key not in self._plans:
            nbytes = lmep_scratch_bytes(self.structs, self.count, op)
            t = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            assert t.data_ptr() % 256 == 0
            h = lmep_plan_create(self.structs, self.count, op, persistent, None, t.data_ptr(), nbytes,
                                 _stream_handle(self.device))
            self._plans[key] = (h, t)
        return self._plans[key][0]

    # ------------------------------------------------------------ buffers --
    def scratch(self, op: int):
        if op not in self._scratch:
            nbytes = lmep_scratch_bytes(self.structs, self.count, op)
            t = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            assert t.data_ptr() % 256 == 0
            self._scratch[op] = t
        t = self._scratch[op]
        return t.data_ptr(), t.numel()

    def empty_state(self) -> torch.Tensor:
        return torch.empty(self.state_size, dtype=torch.float64, device=self.device)

    def empty_weights(self) -> torch.Tensor:
        return torch.zeros(self.weight_size, dtype=torch.float64, device=self.device)

    def pack(self, states) -> torch.Tensor:
        if self.count == 1 and isinstance(states, np.ndarray):
            states = [states]
        flat = np.concatenate([np.asarray(s, dtype=np.float64) for s in states])
        assert flat.size == self.state_size
        return torch.from_numpy(flat).to(self.device)

    def unpack(self, t: torch.Tensor):
        a = t.detach().cpu().numpy()
        return [a[o:o + int(p["N"])].copy() for o, p in zip(self.state_off, self.problems)]

    def unpack_weights(self, w: torch.Tensor):
        """Per instance: [kind, k, N] (frozen velocity, non-uniform grid) or [kind, r, k] (stationary)."""
        a = w.detach().cpu().numpy()
        out = []
        for o, l, p in zip(self.weight_off, self.weight_len, self.problems):
            kinds, n = _KINDS[p["scheme"]], int(p["n"])
            last = int(p["N"]) if (p.get("nonlin") == "burgers_frozen" or p.get("x") is not None) else n
            out.append(a[o:o + l].reshape(kinds, n, last).copy())
        return out

    # ------------------------------------------------------- entry points --
    def build_weights(self, w: torch.Tensor, u: torch.Tensor = None) -> torch.Tensor:
        sp, sb = self.scratch(OP_BUILD)
        lmep_build_weights(self.structs, self.count, u.data_ptr() if u is not None else None, w.data_ptr(), sp, sb,
                           _stream_handle(self.device))
        return w

    def step(self, w: torch.Tensor, u_in: torch.Tensor, n_steps: int, flags: int = 0,
             u_out: torch.Tensor = None) -> torch.Tensor:
        if u_out is None:
            u_out = self.empty_state()
        if self.use_plans:
            lmep_plan_step(self.plan(OP_STEP, flags), w.data_ptr(), u_in.data_ptr(), u_out.data_ptr(), int(n_steps),
                           int(flags), _stream_handle(self.device))
            return u_out
        sp, sb = self.scratch(OP_STEP)
        lmep_step(self.structs, self.count, w.data_ptr(), u_in.data_ptr(), u_out.data_ptr(), int(n_steps),
                  int(flags), sp, sb, _stream_handle(self.device))
        return u_out

    def adjoint_step(self, u_k: torch.Tensor, lam_next: torch.Tensor, lam_k: torch.Tensor = None,
                     grad: torch.Tensor = None):
        if lam_k is None:
            lam_k = self.empty_state()
        if grad is None:
            grad = torch.zeros(3 * self.count, dtype=torch.float64, device=self.device)
        if self.use_plans:
            lmep_plan_adjoint_step(self.plan(OP_ADJOINT), u_k.data_ptr(), lam_next.data_ptr(), lam_k.data_ptr(),
                                   grad.data_ptr(), _stream_handle(self.device))
            return lam_k, grad
        sp, sb = self.scratch(OP_ADJOINT)
        lmep_adjoint_step(self.structs, self.count, u_k.data_ptr(), lam_next.data_ptr(), lam_k.data_ptr(),
                          grad.data_ptr(), sp, sb, _stream_handle(self.device))
        return lam_k, grad


__all__ = ["Batch", "LmepError", "lmep_problem", "lmep_build_weights", "lmep_step", "lmep_adjoint_step",
           "lmep_plan_create", "lmep_plan_step", "lmep_plan_adjoint_step", "lmep_plan_destroy",
           "lmep_profile_kernels",
           "lmep_step_noalloc", "lmep_scratch_bytes", "lmep_weight_count", "lmep_last_error", "lmep_profile_last", "lmep_set_option",
           "lmep_get_option", "library"]
