"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point include/ecodp.h declares, validates arguments before it
touches a device, and reports a missing device as DP_EDEVICE."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2104_01284_amd import _lib as L
from paper_2104_01284_amd import instances as ins
from paper_2104_01284_amd.api import _Desc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.SO_PATH):
        from paper_2104_01284_amd import build
        build.build()
    return L.load(require_torch=False)


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ecodp.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*\**\s*(dp_\w+)\s*\(", src, re.M)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTS)


def test_status_strings(lib):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.dp_status_string(code)
    assert lib.dp_status_string(-99) == b"unknown status"


def build_rc(lib, inst, n=1, flags=0, kernel=0, tile=(0, 0, 0, 0)):
    d = _Desc(inst)
    arr = (L.DpProblemDesc * n)(*([d.d] * n))
    opt = L.DpOptions()
    opt.flags = flags
    opt.kernel = kernel
    for q in range(4):
        opt.tile[q] = tile[q]
    h = C.c_void_p()
    rc = lib.dp_build_problem(arr, n, C.byref(opt), 0, C.byref(h))
    if rc == 0:
        lib.dp_destroy(h)
    return rc


def last_error(lib):
    buf = C.create_string_buffer(512)
    lib.dp_last_error(buf, 512)
    return buf.value.decode()


@pytest.mark.parametrize("mutate,needle", [
    (lambda x: x.__setitem__("ds", float("nan")), "ds"),
    (lambda x: x.__setitem__("v_grid", (0.0, 20.0, 1)), "speed grid"),
    (lambda x: x.__setitem__("soc_grid", (0.7, 0.4, 11)), "SoC grid"),
    (lambda x: x.__setitem__("t_grid", (0.0, -1.0, 31)), "time grid"),
    (lambda x: x.__setitem__("lights", [(0, 60.0, 25.0, 10.0)]), "light"),
    (lambda x: x.__setitem__("lights", [(50, 60.0, 25.0, 10.0)]), "light"),
    (lambda x: x.__setitem__("lights", [(10, 60.0, 70.0, 10.0)]), "red"),
    (lambda x: x.__setitem__("lights", [(10, 60.0, 25.0, 0.0), (10, 50.0, 20.0, 0.0)]), "two lights"),
    (lambda x: x.__setitem__("theta", [0.0, 0.7, 0.01, 0.5, 5000.0]), "theta"),
    (lambda x: x["konst"].__setitem__(13, 0.0), "constants"),
    (lambda x: x.__setitem__("soc0", 0.9), "x0"),
    (lambda x: x.__setitem__("te_grid", (0.0, 150.0, 4000)), "controls"),
    (lambda x: x.__setitem__("t_grid", (0.0, 90.0, 2000)), "n_t"),
])
def test_validation_before_device(lib, mutate, needle):
    inst = ins.plain()
    inst["konst"] = list(inst["konst"])
    mutate(inst)
    rc = build_rc(lib, inst)
    assert rc in (L.DP_EINVAL, L.DP_EUNSUPPORTED)
    assert needle in last_error(lib)


def test_nan_grade_rejected(lib):
    inst = ins.plain()
    inst["grade"] = np.array(inst["grade"])
    inst["grade"][7] = np.nan
    assert build_rc(lib, inst) == L.DP_EINVAL
    assert "grade[7]" in last_error(lib)


def test_null_arguments(lib):
    h = C.c_void_p()
    assert lib.dp_build_problem(None, 1, None, 0, C.byref(h)) == L.DP_EINVAL
    assert lib.dp_build_problem(None, 1, None, 0, None) == L.DP_EINVAL
    assert lib.dp_solve(None, None, None, None, None, None, None) == L.DP_EINVAL
    assert lib.dp_solve_static(None, None, None, None, None, None) == L.DP_EINVAL
    assert lib.dp_rollout(None, None, None, None, None, None) == L.DP_EINVAL
    assert lib.dp_adjoint(None, None, None, None, None, None, None) == L.DP_EINVAL
    assert lib.dp_adjoint_grade(None, None, None, None, None, None, None, None) == L.DP_EINVAL
    assert lib.dp_adjoint_spat(None, None, None, None, None, None, None, None) == L.DP_EINVAL
    assert lib.dp_set_state(None, 0, 1.0, 0.5, 0.0, None) == L.DP_EINVAL
    n = (C.c_int64 * 1)()
    assert lib.dp_executed_evaluations(None, n, None) == L.DP_EINVAL
    assert lib.dp_device_check(None, None) == L.DP_EINVAL
    a = C.c_size_t()
    assert lib.dp_workspace_size(None, C.byref(a), None, None) == L.DP_EINVAL
    lib.dp_destroy(None)
    assert lib.dp_loop_create(None, 20, 80.0, 40, None, 0, C.byref(h)) == L.DP_EINVAL
    assert lib.dp_loop_step(None, None) == L.DP_EINVAL
    assert lib.dp_loop_get_totals(None, None) == L.DP_EINVAL
    lib.dp_loop_destroy(None)


@pytest.mark.parametrize("args,needle", [
    ((0, 80.0, 40, 0), "horizon"),
    ((20, 0.0, 40, 0), "time grid"),
    ((20, 80.0, 1, 0), "time grid"),
    ((20, 80.0, 40, L.DP_GRAPH), "DP_TIMING"),
])
def test_loop_validated_before_device(lib, args, needle):
    """dp_loop_create rejects a bad horizon, time grid or option flag before
    it touches a device."""
    d = _Desc(ins.mpc_route(seed=9, length_m=600.0, n_lights=2))
    horizon, t_f, n_t, flags = args
    opt = L.DpOptions()
    opt.flags = flags
    h = C.c_void_p()
    assert lib.dp_loop_create(C.byref(d.d), horizon, t_f, n_t, C.byref(opt), 0, C.byref(h)) == L.DP_EINVAL
    assert needle in last_error(lib)
    assert not h.value


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="a GPU device node is present")
def test_no_device_is_edevice(lib):
    assert build_rc(lib, ins.plain()) == L.DP_EDEVICE


@pytest.mark.parametrize("kw,needle", [
    (dict(flags=64), "flags"),
    (dict(kernel=4), "kernel"),
    (dict(flags=6), "exclude"),
    (dict(kernel=-1), "kernel"),
    (dict(tile=(5, 0, 0, 0)), "tile[0]"),
    (dict(tile=(0, 17, 0, 0)), "tile[1]"),
    (dict(tile=(0, 0, 33, 0)), "tile[2]"),
    (dict(tile=(0, 0, 0, 1)), "tile[3]"),
])
def test_options_validated_before_device(lib, kw, needle):
    assert build_rc(lib, ins.plain(), **kw) == L.DP_EINVAL
    assert needle in last_error(lib)


def test_per_instance_options_validated(lib):
    d = _Desc(ins.plain())
    arr = (L.DpProblemDesc * 2)(d.d, d.d)
    io = np.array([[2, 8, 0, 0], [2, 5, 0, 0]], dtype=np.int32)
    opt = L.DpOptions()
    opt.inst_opt = io.ctypes.data_as(C.POINTER(C.c_int32))
    h = C.c_void_p()
    assert lib.dp_build_problem(arr, 2, C.byref(opt), 0, C.byref(h)) == L.DP_EINVAL
    assert "instance 1" in last_error(lib) and "tile[0]" in last_error(lib)


def test_terminal_from_values_validated_before_device(lib):
    """dp_terminal_from_values rejects bad grids, shifts, J_inf, NULL and
    overlapping buffers on the host, before any launch."""
    buf = (C.c_float * 64)()
    other = (C.c_float * 64)()
    src, dst = C.cast(buf, C.c_void_p), C.cast(other, C.c_void_p)
    f = lib.dp_terminal_from_values
    ok = dict(n_v=2, n_soc=2, n_t_src=4, t_f_src=10.0, t_shift=0.0, n_t_dst=3, t_f_dst=5.0, J_inf=1e4)

    def call(s=src, d=dst, **kw):
        a = dict(ok, **kw)
        return f(s, a["n_v"], a["n_soc"], a["n_t_src"], a["t_f_src"], a["t_shift"], a["n_t_dst"], a["t_f_dst"],
                 a["J_inf"], d, None)
    assert call(s=None) == L.DP_EINVAL
    assert call(d=None) == L.DP_EINVAL
    assert call(n_t_src=1) == L.DP_EINVAL
    assert call(n_t_dst=1) == L.DP_EINVAL
    assert call(n_v=0) == L.DP_EINVAL
    assert call(t_shift=-1.0) == L.DP_EINVAL
    assert call(t_f_src=float("nan")) == L.DP_EINVAL
    assert call(t_f_dst=0.0) == L.DP_EINVAL
    assert call(J_inf=0.0) == L.DP_EINVAL
    assert call(d=C.c_void_p(src.value + 8)) == L.DP_EINVAL     # overlapping
    msg = C.create_string_buffer(256)
    lib.dp_last_error(msg, 256)
    assert b"overlap" in msg.value


def test_device_terminal_flag_needs_device_memory(lib):
    inst = ins.plain()
    inst["terminal_V"] = np.zeros((21, 11, 31), dtype=np.float32)
    d = _Desc(inst)
    d.d.flags |= L.DP_TERMINAL_DEVICE                       # a host pointer with the device flag
    h = C.c_void_p()
    rc = lib.dp_build_problem(C.byref(d.d), 1, None, 0, C.byref(h))
    assert rc in (L.DP_EINVAL, L.DP_EDEVICE)
    d.d.terminal_V = None
    assert lib.dp_build_problem(C.byref(d.d), 1, None, 0, C.byref(h)) == L.DP_EINVAL


def test_negative_host_terminal_values_rejected(lib):
    """Costs are non-negative (the sweep's running minimum relies on it): a
    host terminal_V with a negative value fails the build before any device
    use; zeros and NaN (a J_inf node) pass the check."""
    inst = ins.plain()
    tv = np.zeros((21, 11, 31), dtype=np.float32)
    tv[3, 4, 5] = np.nan
    tv[7, 2, 30] = -1.0e-3
    inst["terminal_V"] = tv
    d = _Desc(inst)
    h = C.c_void_p()
    assert lib.dp_build_problem(C.byref(d.d), 1, None, 0, C.byref(h)) == L.DP_EINVAL
    msg = C.create_string_buffer(256)
    lib.dp_last_error(msg, 256)
    assert b"negative" in msg.value and b"terminal_V" in msg.value
