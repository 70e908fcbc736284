"""ctypes binding of liblmep.so (the C ABI declared in include/lmep.h).

Argument marshalling only: the functions here pack problem records, pass
device pointers and the stream, and turn negative status codes into
exceptions.  Every step of the method runs in the library's HIP kernels.
Importing this module fails if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblmep.so")

LMEP_OK = 0
LMEP_ERR_ARG = -1
LMEP_ERR_UNSUPPORTED = -2
LMEP_ERR_DEVICE = -3
LMEP_ERR_NONFINITE = -4
LMEP_ERR_SCRATCH = -5

LMEP_BC_PERIODIC, LMEP_BC_DIRICHLET, LMEP_BC_NEUMANN = 0, 1, 2
LMEP_LINEAR, LMEP_ETD1, LMEP_ETD2RK, LMEP_ETDRK4 = 0, 1, 2, 3
LMEP_NL_NONE, LMEP_NL_BURGERS_FROZEN, LMEP_NL_KDV, LMEP_NL_ALLEN_CAHN = 0, 1, 2, 3
LMEP_WIN_CENTRED, LMEP_WIN_UPWIND = 0, 1
LMEP_F_GRAPH, LMEP_F_PERSISTENT, LMEP_F_CHECK_FINITE, LMEP_F_PROFILE, LMEP_F_COUNT = 0x1, 0x2, 0x4, 0x8, 0x10

OP_BUILD, OP_STEP, OP_ADJOINT = 0, 1, 2

BC_NAMES = {"periodic": LMEP_BC_PERIODIC, "dirichlet": LMEP_BC_DIRICHLET, "neumann": LMEP_BC_NEUMANN}
SCHEME_NAMES = {"linear": LMEP_LINEAR, "etd1": LMEP_ETD1, "etd2rk": LMEP_ETD2RK, "etdrk4": LMEP_ETDRK4}
NONLIN_NAMES = {"none": LMEP_NL_NONE, "burgers_frozen": LMEP_NL_BURGERS_FROZEN, "kdv": LMEP_NL_KDV,
                "allen_cahn": LMEP_NL_ALLEN_CAHN}
WINDOW_NAMES = {"centred": LMEP_WIN_CENTRED, "upwind": LMEP_WIN_UPWIND}


class lmep_problem(ctypes.Structure):
    """Mirror of the C struct lmep_problem."""
    _fields_ = [
        ("N", ctypes.c_int64), ("n", ctypes.c_int32), ("bc", ctypes.c_int32),
        ("h", ctypes.c_double), ("dt", ctypes.c_double), ("c", ctypes.c_double), ("nu", ctypes.c_double),
        ("delta", ctypes.c_double), ("react", ctypes.c_double),
        ("scheme", ctypes.c_int32), ("nonlin", ctypes.c_int32),
        ("nl_coef", ctypes.c_double), ("bc_left", ctypes.c_double), ("bc_right", ctypes.c_double),
        ("state_off", ctypes.c_int64), ("weight_off", ctypes.c_int64),
        ("window", ctypes.c_int32),
        ("x", ctypes.c_void_p),
    ]


class LmepError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"liblmep status {code}: {message}")
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                      "(the HIP library is required; there is no fallback)")
_lib = ctypes.CDLL(LIB_PATH)

_P = ctypes.POINTER(lmep_problem)
_V = ctypes.c_void_p
_lib.lmep_weight_count.argtypes = [_P]
_lib.lmep_weight_count.restype = ctypes.c_int64
_lib.lmep_scratch_bytes.argtypes = [_P, ctypes.c_int32, ctypes.c_int32]
_lib.lmep_scratch_bytes.restype = ctypes.c_size_t
_lib.lmep_build_weights.argtypes = [_P, ctypes.c_int32, _V, _V, _V, ctypes.c_size_t, _V]
_lib.lmep_step.argtypes = [_P, ctypes.c_int32, _V, _V, _V, ctypes.c_int32, ctypes.c_uint32, _V, ctypes.c_size_t, _V]
_lib.lmep_step_noalloc.argtypes = [_P, ctypes.c_int32, _V, _V, _V, ctypes.c_int32, ctypes.c_uint32, _V]
_lib.lmep_adjoint_step.argtypes = [_P, ctypes.c_int32, _V, _V, _V, _V, _V, ctypes.c_size_t, _V]
_lib.lmep_plan_create.argtypes = [ctypes.POINTER(_V), _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32,
                                  ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, _V, ctypes.c_size_t, _V]
_lib.lmep_plan_step.argtypes = [_V, _V, _V, _V, ctypes.c_int32, ctypes.c_uint32, _V]
_lib.lmep_plan_adjoint_step.argtypes = [_V, _V, _V, _V, _V, _V]
_lib.lmep_plan_destroy.argtypes = [_V]
_lib.lmep_profile_kernel.argtypes = [ctypes.c_int32, ctypes.c_char_p, ctypes.c_size_t,
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]
_lib.lmep_profile_kernel.restype = ctypes.c_int32
_lib.lmep_profile_last.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
_lib.lmep_last_error.restype = ctypes.c_char_p
_lib.lmep_set_option.argtypes = [ctypes.c_int32, ctypes.c_int32]
_lib.lmep_get_option.argtypes = [ctypes.c_int32]
_lib.lmep_get_option.restype = ctypes.c_int32

EXPORTED = ("lmep_weight_count", "lmep_scratch_bytes", "lmep_build_weights", "lmep_step", "lmep_step_noalloc",
            "lmep_adjoint_step", "lmep_plan_create", "lmep_plan_step", "lmep_plan_adjoint_step", "lmep_plan_destroy",
            "lmep_profile_last", "lmep_profile_kernel", "lmep_last_error", "lmep_set_option", "lmep_get_option")
LMEP_NOALLOC_SCRATCH_BYTES = 64 << 20
LMEP_OPT_STEPS_PER_LAUNCH = 1
LMEP_OPT_PROFILE_ADJOINT = 2
LMEP_OPT_FUSE_FROZEN = 3
LMEP_OPT_APPLY_TILE = 4
LMEP_OPT_EXP_METHOD = 5
LMEP_OPT_TAYLOR_REGION = 6
LMEP_OPT_MERGE_GROUPS = 7
LMEP_EXP_AUTO = 0
LMEP_EXP_PADE = 1


def library() -> ctypes.CDLL:
    return _lib


def lmep_last_error() -> str:
    return (_lib.lmep_last_error() or b"").decode()


def _check(rc: int) -> int:
    if rc < 0:
        raise LmepError(rc, lmep_last_error())
    return rc


def problem_array(problems):
    """ctypes array of lmep_problem from a sequence of lmep_problem or dicts."""
    arr = (lmep_problem * len(problems))()
    for k, p in enumerate(problems):
        arr[k] = p if isinstance(p, lmep_problem) else to_struct(p)
    return arr


def to_struct(p: dict, state_off: int = None, weight_off: int = None, x_ptr: int = None) -> lmep_problem:
    """Problem dict -> C struct.  A non-uniform grid (key "x") needs the device
    address of its coordinates in x_ptr; without one the host array's address
    stands in (enough for the host-side counting and checks, never for a
    build)."""
    x = p.get("x")
    if x is not None and x_ptr is None:
        x_ptr = x.ctypes.data if hasattr(x, "ctypes") else int(x.data_ptr())
    s = lmep_problem(
        int(p["N"]), int(p["n"]), BC_NAMES[p["bc"]], float(p["h"]), float(p["dt"]), float(p.get("c", 0.0)),
        float(p.get("nu", 0.0)), float(p.get("delta", 0.0)), float(p.get("react", 0.0)),
        SCHEME_NAMES[p["scheme"]], NONLIN_NAMES[p.get("nonlin", "none")], float(p.get("nl_coef", 0.0)),
        float(p.get("bc_left", 0.0)), float(p.get("bc_right", 0.0)),
        int(p.get("state_off", 0) if state_off is None else state_off),
        int(p.get("weight_off", 0) if weight_off is None else weight_off),
        WINDOW_NAMES[p.get("window", "centred")], x_ptr if x is not None else None)
    s._keep = x
    return s


def lmep_weight_count(prob: lmep_problem) -> int:
    return _check(_lib.lmep_weight_count(ctypes.byref(prob)))


def lmep_scratch_bytes(probs, count: int, op: int) -> int:
    n = _lib.lmep_scratch_bytes(probs, count, op)
    if n == 0:
        raise LmepError(LMEP_ERR_ARG, lmep_last_error())
    return n


def lmep_build_weights(probs, count, d_u, d_w, d_scratch, scratch_bytes, stream) -> None:
    _check(_lib.lmep_build_weights(probs, count, d_u, d_w, d_scratch, scratch_bytes, stream))


def lmep_step(probs, count, d_w, d_u_in, d_u_out, n_steps, flags, d_scratch, scratch_bytes, stream) -> None:
    _check(_lib.lmep_step(probs, count, d_w, d_u_in, d_u_out, n_steps, flags, d_scratch, scratch_bytes, stream))


def lmep_step_noalloc(probs, count, d_w, d_u_in, d_u_out, n_steps, flags, stream) -> None:
    _check(_lib.lmep_step_noalloc(probs, count, d_w, d_u_in, d_u_out, n_steps, flags, stream))


def lmep_adjoint_step(probs, count, d_u_k, d_lambda_next, d_lambda_k, d_grad, d_scratch, scratch_bytes,
                      stream) -> None:
    _check(_lib.lmep_adjoint_step(probs, count, d_u_k, d_lambda_next, d_lambda_k, d_grad, d_scratch,
                                  scratch_bytes, stream))


def lmep_plan_create(probs, count, op, flags, options, d_scratch, scratch_bytes, stream) -> int:
    """options: dict {LMEP_OPT_*: value} overriding the process-wide values for
    this plan.  Returns the plan handle (an integer)."""
    pairs = [int(v) for kv in sorted((options or {}).items()) for v in kv]
    arr = (ctypes.c_int32 * max(1, len(pairs)))(*pairs)
    h = _V()
    _check(_lib.lmep_plan_create(ctypes.byref(h), probs, count, op, flags, arr if pairs else None, len(pairs) // 2,
                                 d_scratch, scratch_bytes, stream))
    return h.value


def lmep_plan_step(plan, d_w, d_u_in, d_u_out, n_steps, flags, stream) -> None:
    _check(_lib.lmep_plan_step(plan, d_w, d_u_in, d_u_out, n_steps, flags, stream))


def lmep_plan_adjoint_step(plan, d_u_k, d_lambda_next, d_lambda_k, d_grad, stream) -> None:
    _check(_lib.lmep_plan_adjoint_step(plan, d_u_k, d_lambda_next, d_lambda_k, d_grad, stream))


def lmep_plan_destroy(plan) -> None:
    _check(_lib.lmep_plan_destroy(plan))


def lmep_profile_kernels() -> list:
    """[(name, ms, launches)] of every kernel the last timed call launched."""
    out = []
    count = _lib.lmep_profile_kernel(-1, None, 0, None, None)
    for k in range(count):
        name = ctypes.create_string_buffer(128)
        ms, n = ctypes.c_double(), ctypes.c_int32()
        _lib.lmep_profile_kernel(k, name, 128, ctypes.byref(ms), ctypes.byref(n))
        out.append((name.value.decode(), ms.value, n.value))
    return out


def lmep_profile_last() -> dict:
    b, a = ctypes.c_double(), ctypes.c_double()
    nb, na = ctypes.c_int32(), ctypes.c_int32()
    m, sq = ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.lmep_profile_last(ctypes.byref(b), ctypes.byref(nb), ctypes.byref(a), ctypes.byref(na),
                                  ctypes.byref(m), ctypes.byref(sq)))
    return dict(build_ms=b.value, build_launches=nb.value, apply_ms=a.value, apply_launches=na.value,
                matrices=m.value, squarings=sq.value)


_option_generation = [0]


def lmep_set_option(option: int, value: int) -> None:
    _check(_lib.lmep_set_option(int(option), int(value)))
    _option_generation[0] += 1


def option_generation() -> int:
    """Count of lmep_set_option calls made through this module (lets callers
    cache the process-wide option values between changes)."""
    return _option_generation[0]


def lmep_get_option(option: int) -> int:
    return _check(_lib.lmep_get_option(int(option)))
