"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/lmep.h declares, and rejects invalid arguments
before touching the device."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

import paper_2603_15964_amd as lmep
import workloads

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "lmep.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lmep_[a-z_]+)\s*\(", text)))


def test_header_symbols_are_exported():
    lib = ctypes.CDLL(lmep.LIB_PATH)
    names = _declared()
    assert {"lmep_build_weights", "lmep_step", "lmep_adjoint_step"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(lmep.EXPORTED)


def _structs(**over):
    p, _ = workloads.burgers(N=64, n=7)
    p.update(over)
    return lmep.problem_array([p])


@pytest.mark.parametrize("over,code", [
    (dict(n=4), lmep.LMEP_ERR_ARG),
    (dict(n=1), lmep.LMEP_ERR_ARG),
    (dict(n=17), lmep.LMEP_ERR_ARG),
    (dict(N=5), lmep.LMEP_ERR_ARG),
    (dict(h=0.0), lmep.LMEP_ERR_ARG),
    (dict(dt=-1.0), lmep.LMEP_ERR_ARG),
    (dict(dt=float("nan")), lmep.LMEP_ERR_ARG),
    (dict(nu=float("inf")), lmep.LMEP_ERR_ARG),
    (dict(scheme="etd2rk"), lmep.LMEP_ERR_UNSUPPORTED),   # frozen velocity needs ETD1
    (dict(n=15, nonlin="kdv", scheme="etd2rk"), lmep.LMEP_ERR_UNSUPPORTED),  # n + p = 17
])
def test_invalid_problems_rejected_before_any_device_work(over, code):
    s = _structs(**over)
    rc = lmep.library().lmep_step(s, 1, ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(4096), 1, 0,
                                  ctypes.c_void_p(256), 1 << 30, None)
    assert rc == code, lmep.lmep_last_error()
    assert lmep.lmep_last_error()


def test_bad_enums_and_flags():
    s = _structs()
    s[0].bc = 7
    assert lmep.library().lmep_build_weights(s, 1, None, ctypes.c_void_p(8), None, 0, None) == lmep.LMEP_ERR_ARG
    s = _structs()
    rc = lmep.library().lmep_step(s, 1, ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(1 << 20), 1, 0x100,
                                  ctypes.c_void_p(256), 1 << 30, None)
    assert rc == lmep.LMEP_ERR_ARG and "flag" in lmep.lmep_last_error()
    rc = lmep.library().lmep_step(s, 1, ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(1 << 20), 0, 0,
                                  ctypes.c_void_p(256), 1 << 30, None)
    assert rc == lmep.LMEP_ERR_ARG


def test_scratch_and_overlap_checks():
    s = _structs()
    need = lmep.lmep_scratch_bytes(s, 1, lmep.OP_STEP)
    assert need > 0
    rc = lmep.library().lmep_step(s, 1, ctypes.c_void_p(8), ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 24), 1, 0,
                                  ctypes.c_void_p(256), need - 1, None)
    assert rc == lmep.LMEP_ERR_SCRATCH
    rc = lmep.library().lmep_step(s, 1, ctypes.c_void_p(8), ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 20), 1, 0,
                                  ctypes.c_void_p(256), need, None)
    assert rc == lmep.LMEP_ERR_ARG and "overlap" in lmep.lmep_last_error()
    rc = lmep.library().lmep_step(s, 1, ctypes.c_void_p(8), ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 24), 1, 0,
                                  ctypes.c_void_p(260), need, None)
    assert rc == lmep.LMEP_ERR_ARG and "aligned" in lmep.lmep_last_error()
    # two instances whose states overlap
    p, _ = workloads.burgers(N=64, n=7)
    a = lmep.problem_array([lmep.to_struct(p, 0, 0), lmep.to_struct(p, 10, 5000)])
    rc = lmep.library().lmep_build_weights(a, 2, ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(256),
                                           1 << 30, None)
    assert rc == lmep.LMEP_ERR_ARG and "overlap" in lmep.lmep_last_error()


def test_weight_counts_and_batch_packing():
    p, _ = workloads.burgers(N=100, n=7)
    assert lmep.lmep_weight_count(lmep.to_struct(p)) == 2 * 7 * 100
    q, _ = workloads.kdv(N=64, n=9)
    assert lmep.lmep_weight_count(lmep.to_struct(q)) == 3 * 9 * 9
    probs, _ = workloads.allen_cahn_batch(count=5, n_min=20, n_max=40)
    b = lmep.Batch(probs, device="cpu")
    assert b.state_size == sum(x["N"] for x in probs)
    assert all(o % 32 == 0 for o in b.weight_off)
    assert lmep.lmep_scratch_bytes(b.structs, b.count, lmep.OP_BUILD) > 0


def test_multistep_flag_and_option():
    """LMEP_F_PERSISTENT is refused before any device work for frozen-velocity
    instances the multi-step finite-Taylor kernel does not cover (Neumann
    grids, a reaction term, the Pade method); the steps-per-launch option
    accepts 1, 2, 4, 8 and 16 only."""
    lib = lmep.library()
    for over in (dict(bc="neumann"), dict(react=0.5)):
        s = _structs(**over)  # frozen-velocity Burgers
        rc = lib.lmep_step(s, 1, ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(4096), 5,
                           lmep.LMEP_F_PERSISTENT, ctypes.c_void_p(256), 1 << 30, None)
        assert rc == lmep.LMEP_ERR_UNSUPPORTED, (over, lmep.lmep_last_error())
    lmep.lmep_set_option(lmep.LMEP_OPT_EXP_METHOD, lmep.LMEP_EXP_PADE)
    try:
        rc = lib.lmep_step(_structs(), 1, ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(4096), 5,
                           lmep.LMEP_F_PERSISTENT, ctypes.c_void_p(256), 1 << 30, None)
        assert rc == lmep.LMEP_ERR_UNSUPPORTED, lmep.lmep_last_error()
    finally:
        lmep.lmep_set_option(lmep.LMEP_OPT_EXP_METHOD, lmep.LMEP_EXP_AUTO)
    opt = lmep.LMEP_OPT_STEPS_PER_LAUNCH
    assert lmep.lmep_get_option(opt) == 8
    for bad in (0, 3, 5, 32, -8):
        with pytest.raises(lmep.LmepError):
            lmep.lmep_set_option(opt, bad)
    with pytest.raises(lmep.LmepError):
        lmep.lmep_set_option(99, 8)
    with pytest.raises(lmep.LmepError):
        lmep.lmep_get_option(99)
    try:
        lmep.lmep_set_option(opt, 4)
        assert lmep.lmep_get_option(opt) == 4
    finally:
        lmep.lmep_set_option(opt, 8)


def test_taylor_region_option():
    """LMEP_OPT_TAYLOR_REGION takes 0 or a multiple of 64 in [128, 512]."""
    opt = lmep.LMEP_OPT_TAYLOR_REGION
    assert lmep.lmep_get_option(opt) == 0
    for bad in (-64, 64, 100, 576, 1024):
        with pytest.raises(lmep.LmepError):
            lmep.lmep_set_option(opt, bad)
    try:
        for good in (128, 320, 512):
            lmep.lmep_set_option(opt, good)
            assert lmep.lmep_get_option(opt) == good
    finally:
        lmep.lmep_set_option(opt, 0)


def test_merge_groups_option():
    """LMEP_OPT_MERGE_GROUPS takes 0 (default) or 1."""
    opt = lmep.LMEP_OPT_MERGE_GROUPS
    assert lmep.lmep_get_option(opt) == 0
    for bad in (-1, 2):
        with pytest.raises(lmep.LmepError):
            lmep.lmep_set_option(opt, bad)
    try:
        lmep.lmep_set_option(opt, 1)
        assert lmep.lmep_get_option(opt) == 1
    finally:
        lmep.lmep_set_option(opt, 0)


def test_exp_method_option():
    """LMEP_OPT_EXP_METHOD takes LMEP_EXP_AUTO (default) or LMEP_EXP_PADE."""
    opt = lmep.LMEP_OPT_EXP_METHOD
    assert lmep.lmep_get_option(opt) == lmep.LMEP_EXP_AUTO
    for bad in (-1, 2, 7):
        with pytest.raises(lmep.LmepError):
            lmep.lmep_set_option(opt, bad)
    try:
        lmep.lmep_set_option(opt, lmep.LMEP_EXP_PADE)
        assert lmep.lmep_get_option(opt) == lmep.LMEP_EXP_PADE
    finally:
        lmep.lmep_set_option(opt, lmep.LMEP_EXP_AUTO)
    assert lmep.lmep_get_option(opt) == lmep.LMEP_EXP_AUTO


def test_window_field_checks():
    """The window field: unknown values are ARG; upwind windows are refused
    with ETDRK4 and by the reverse step before any device work.  The Python
    mirror has the C layout (window at byte 112)."""
    assert lmep.lmep_problem.window.offset == 112 and lmep.lmep_problem.x.offset == 120
    assert ctypes.sizeof(lmep.lmep_problem) == 128
    lib = lmep.library()
    s = _structs()
    s[0].window = 2
    assert lib.lmep_build_weights(s, 1, ctypes.c_void_p(8), ctypes.c_void_p(8), None, 0, None) == lmep.LMEP_ERR_ARG
    assert "window" in lmep.lmep_last_error()
    rk4 = dict(N=64, n=9, bc="periodic", h=0.1, dt=0.01, nu=0.1, scheme="etdrk4", nonlin="allen_cahn",
               nl_coef=1.0, window="upwind")
    assert lmep.lmep_weight_count(lmep.to_struct(dict(rk4, window="centred"))) == 6 * 9 * 9
    s = lmep.problem_array([rk4])
    rc = lib.lmep_step(s, 1, ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(4096), 1, 0,
                       ctypes.c_void_p(256), 1 << 30, None)
    assert rc == lmep.LMEP_ERR_UNSUPPORTED, lmep.lmep_last_error()
    s = _structs(window="upwind")
    rc = lib.lmep_adjoint_step(s, 1, ctypes.c_void_p(8), ctypes.c_void_p(4096), ctypes.c_void_p(1 << 20),
                               ctypes.c_void_p(1 << 24), ctypes.c_void_p(256), 1 << 30, None)
    assert rc == lmep.LMEP_ERR_UNSUPPORTED, lmep.lmep_last_error()


def test_nonuniform_checks():
    """Non-uniform grids: per-node weight counts, refusals before any device
    work (periodic ends, upwind windows, ETDRK4, KdV, the reverse step, and
    multi-step launches beyond 512 nodes)."""
    import workloads
    lib = lmep.library()
    p, _ = workloads.allen_cahn_chebyshev()
    assert lmep.lmep_weight_count(lmep.to_struct(p)) == 2 * 21 * 64
    big = dict(p, N=600, x=workloads.chebyshev(600))
    for bad in (dict(bc="periodic"), dict(window="upwind"), dict(scheme="etdrk4"), dict(nonlin="kdv")):
        s = lmep.problem_array([dict(p, **bad)])
        rc = lib.lmep_step(s, 1, ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(4096), 1, 0,
                           ctypes.c_void_p(256), 1 << 30, None)
        assert rc == lmep.LMEP_ERR_UNSUPPORTED, (bad, lmep.lmep_last_error())
    s = lmep.problem_array([dict(p, n=27)])
    assert lib.lmep_build_weights(s, 1, None, ctypes.c_void_p(8), ctypes.c_void_p(256), 1 << 30, None) == \
        lmep.LMEP_ERR_ARG
    s = lmep.problem_array([big])
    rc = lib.lmep_step(s, 1, ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(1 << 20), 4,
                       lmep.LMEP_F_PERSISTENT, ctypes.c_void_p(256), 1 << 30, None)
    assert rc == lmep.LMEP_ERR_UNSUPPORTED and "512" in lmep.lmep_last_error()
    s = lmep.problem_array([p])
    rc = lib.lmep_adjoint_step(s, 1, ctypes.c_void_p(8), ctypes.c_void_p(4096), ctypes.c_void_p(1 << 20),
                               ctypes.c_void_p(1 << 24), ctypes.c_void_p(256), 1 << 30, None)
    assert rc == lmep.LMEP_ERR_UNSUPPORTED


def test_noalloc_step_checks_before_device_work():
    """lmep_step_noalloc rejects flags other than LMEP_F_PERSISTENT and batches
    whose scratch exceeds its static array, before touching a device."""
    s = _structs()
    rc = lmep.library().lmep_step_noalloc(s, 1, ctypes.c_void_p(8), ctypes.c_void_p(1 << 20),
                                          ctypes.c_void_p(1 << 24), 1, lmep.LMEP_F_GRAPH, None)
    assert rc == lmep.LMEP_ERR_ARG and "LMEP_F_PERSISTENT" in lmep.lmep_last_error()
    big = lmep.problem_array([workloads.make_problem(N=9 << 20, n=5, bc="periodic", h=1e-3, dt=1e-4, c=1.0,
                                                     scheme="linear")])
    assert lmep.lmep_scratch_bytes(big, 1, lmep.OP_STEP) > lmep.LMEP_NOALLOC_SCRATCH_BYTES
    rc = lmep.library().lmep_step_noalloc(big, 1, ctypes.c_void_p(8), ctypes.c_void_p(1 << 40),
                                          ctypes.c_void_p(1 << 41), 1, 0, None)
    assert rc == lmep.LMEP_ERR_SCRATCH and "static array" in lmep.lmep_last_error()
