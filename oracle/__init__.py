"""CPU oracle for the LMEP hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It wraps the plain C oracle
(``lmep_oracle.c``), which shares no code with the HIP library.  Problems are
plain dicts (see ``workloads``) with the keys

    N, n, bc, h, dt, c, nu, delta, react, scheme, nonlin, nl_coef,
    bc_left, bc_right, window (optional: "centred" or "upwind"),
    x (optional: node coordinates of a non-uniform grid, increasing; Dirichlet)

using the string names ``bc in {"periodic", "dirichlet", "neumann"}``,
``scheme in {"linear", "etd1", "etd2rk", "etdrk4"}`` and
``nonlin in {"none", "burgers_frozen", "kdv", "allen_cahn"}``.

Every function cites the passage of the paper it follows; all arithmetic is
FP64 (long double where the C source says so).  Parity unpinned: none.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_lmep_oracle.so")

BC = {"periodic": 0, "dirichlet": 1, "neumann": 2}
SCHEME = {"linear": 0, "etd1": 1, "etd2rk": 2, "etdrk4": 3}
NONLIN = {"none": 0, "burgers_frozen": 1, "kdv": 2, "allen_cahn": 3}
WINDOW = {"centred": 0, "upwind": 1}
P_OF_SCHEME = {"linear": 0, "etd1": 1, "etd2rk": 2, "etdrk4": 3}
# weight rows stored per node (ETDRK4: E(dt/2), (dt/2)phi1(dt/2), E(dt), dt*alpha, dt*beta, dt*gamma)
KINDS_OF_SCHEME = {"linear": 1, "etd1": 2, "etd2rk": 3, "etdrk4": 6}


class _Prob(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int64), ("n", ctypes.c_int32), ("bc", ctypes.c_int32),
        ("h", ctypes.c_double), ("dt", ctypes.c_double),
        ("c", ctypes.c_double), ("nu", ctypes.c_double), ("delta", ctypes.c_double),
        ("react", ctypes.c_double),
        ("scheme", ctypes.c_int32), ("nonlin", ctypes.c_int32),
        ("nl_coef", ctypes.c_double), ("bc_left", ctypes.c_double), ("bc_right", ctypes.c_double),
        ("window", ctypes.c_int32),
        ("x", ctypes.c_void_p),
    ]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(_SO)
        P = ctypes.POINTER(_Prob)
        lib.ora_fd_matrices.argtypes = [ctypes.c_int, ctypes.c_double, _D, _D, _D]
        lib.ora_fd_nodes.argtypes = [ctypes.c_int, _D, _D, _D, _D]
        lib.ora_window_offset.argtypes = [P, ctypes.c_int64, ctypes.c_double]
        lib.ora_window_offset.restype = ctypes.c_int64
        lib.ora_augmented_row.argtypes = [ctypes.c_int, ctypes.c_int, _D, ctypes.c_double, ctypes.c_int,
                                          ctypes.c_int, _D]
        lib.ora_augmented_row_z.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_double,
                                            ctypes.c_int, ctypes.c_void_p]
        lib.ora_build_weights.argtypes = [P, _D, _D]
        lib.ora_run.argtypes = [P, _D, ctypes.c_int64, _D]
        lib.ora_run_z.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D, _D,
                                  ctypes.c_int64, _D, _D]
        lib.ora_adjoint_step.argtypes = [P, _D, _D, _D, _D]
        lib.ora_adjoint_run.argtypes = [P, _D, _D, ctypes.c_int64, _D, _D, _D]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _prob(p: dict) -> _Prob:
    x = p.get("x")
    xa = None
    if x is not None:
        xa = _f64(x)
        if xa.shape != (int(p["N"]),):
            raise ValueError("x must hold N node coordinates")
    pr = _Prob(int(p["N"]), int(p["n"]), BC[p["bc"]], float(p["h"]), float(p["dt"]),
               float(p.get("c", 0.0)), float(p.get("nu", 0.0)), float(p.get("delta", 0.0)),
               float(p.get("react", 0.0)), SCHEME[p["scheme"]], NONLIN[p.get("nonlin", "none")],
               float(p.get("nl_coef", 0.0)), float(p.get("bc_left", 0.0)), float(p.get("bc_right", 0.0)),
               WINDOW[p.get("window", "centred")], xa.ctypes.data if xa is not None else None)
    pr._keep = xa  # the coordinates must outlive the call
    return pr


def fd_matrices(n: int, h: float = 1.0):
    """Differentiation matrices D1, D2, D3 on a uniform n-point stencil (Sec. 2.1 step 1)."""
    D = [np.zeros((n, n)) for _ in range(3)]
    if _load().ora_fd_matrices(n, h, *[_ptr(d) for d in D]):
        raise ValueError("bad stencil")
    return D


def fd_nodes(x):
    """Differentiation matrices (D1, D2, D3) on the given nodes (step a2 on a
    non-uniform stencil)."""
    x = _f64(x)
    n = x.shape[0]
    D = [np.zeros((n, n)) for _ in range(3)]
    if _load().ora_fd_nodes(n, _ptr(x), _ptr(D[0]), _ptr(D[1]), _ptr(D[2])):
        raise ValueError("bad nodes")
    return D


def window_offset(p: dict, i: int, a: float = None) -> int:
    """Offset o of node i's stencil for a node with advection speed a (default:
    the problem's c): centred, or fully one-sided against the flow for
    window="upwind" (Sec. 4.1); edge rows next to Dirichlet ends (Sec. 2.1 step 3)."""
    pr = _prob(p)
    speed = float(p.get("c", 0.0)) if a is None else float(a)
    return int(_load().ora_window_offset(ctypes.byref(pr), int(i), speed))


def augmented_row(L, dt: float, r: int, p: int, nilpotent: bool = True):
    """Row r of the first block row of exp(dt * Atilde) (Sec. 3.1 steps 1-2).

    Returns (W0, W1, W2, W3) = rows r of e^{dt L}, dt phi1(dt L),
    dt phi2(dt L), dt phi3(dt L); entries beyond p are None.
    """
    L = _f64(L)
    n = L.shape[0]
    out = np.zeros(4 * n)
    if _load().ora_augmented_row(n, p, _ptr(L), dt, r, 1 if nilpotent else 0, _ptr(out)):
        raise ValueError("bad arguments")
    return tuple(out[k * n:(k + 1) * n].copy() if k <= p else None for k in range(4))


def augmented_row_complex(L, dt: float, r: int, p: int):
    """Complex version of augmented_row (terminating series; complex-step checks)."""
    L = np.ascontiguousarray(L, dtype=np.complex128)
    n = L.shape[0]
    out = np.zeros(4 * n, dtype=np.complex128)
    if _load().ora_augmented_row_z(n, p, L.ctypes.data, dt, r, out.ctypes.data):
        raise ValueError("bad arguments")
    return tuple(out[k * n:(k + 1) * n].copy() if k <= p else None for k in range(4))


def build_weights(p: dict, u=None) -> np.ndarray:
    """Weights of every node, shape [N, kinds, n] (steps a1-a6); kinds = 1 + p,
    or 6 for ETDRK4 (KINDS_OF_SCHEME)."""
    N, n, q = int(p["N"]), int(p["n"]), KINDS_OF_SCHEME[p["scheme"]]
    w = np.zeros((N, q, n))
    uu = _f64(u) if u is not None else None
    pr = _prob(p)
    if _load().ora_build_weights(ctypes.byref(pr), _ptr(uu) if uu is not None else None, _ptr(w)):
        raise ValueError("oracle rejected the problem")
    return w


def run(p: dict, u0, steps: int) -> np.ndarray:
    """Advance `steps` LMEP steps from u0 (steps a1-a9)."""
    u0 = _f64(u0)
    out = np.zeros_like(u0)
    pr = _prob(p)
    if _load().ora_run(ctypes.byref(pr), _ptr(u0), int(steps), _ptr(out)):
        raise ValueError("oracle rejected the problem")
    return out


def run_complex(p: dict, u0_re, u0_im, steps: int, c_im=0.0, nu_im=0.0, delta_im=0.0):
    """Forward run with complex perturbations (for complex-step derivatives)."""
    u0_re = _f64(u0_re)
    u0_im = _f64(u0_im if u0_im is not None else np.zeros_like(u0_re))
    re, im = np.zeros_like(u0_re), np.zeros_like(u0_re)
    pr = _prob(p)
    if _load().ora_run_z(ctypes.byref(pr), c_im, nu_im, delta_im, _ptr(u0_re), _ptr(u0_im), int(steps),
                         _ptr(re), _ptr(im)):
        raise ValueError("oracle rejected the problem")
    return re + 1j * im


def adjoint_step(p: dict, u, lam):
    """Reverse of one LINEAR/ETD1 step (step a10): (lam_k, [dnu, dc, ddelta])."""
    u, lam = _f64(u), _f64(lam)
    out = np.zeros_like(u)
    grad = np.zeros(3)
    pr = _prob(p)
    if _load().ora_adjoint_step(ctypes.byref(pr), _ptr(u), _ptr(lam), _ptr(out), _ptr(grad)):
        raise ValueError("oracle rejected the problem")
    return out, grad


def adjoint_run(p: dict, u0, target, steps: int):
    """Loss 0.5*||u(T) - target||^2 and its gradient w.r.t. u0 and (nu, c, delta)."""
    u0, target = _f64(u0), _f64(target)
    loss = np.zeros(1)
    gu = np.zeros_like(u0)
    grad = np.zeros(3)
    pr = _prob(p)
    if _load().ora_adjoint_run(ctypes.byref(pr), _ptr(u0), _ptr(target), int(steps), _ptr(loss), _ptr(gu),
                               _ptr(grad)):
        raise ValueError("oracle rejected the problem")
    return float(loss[0]), gu, grad
