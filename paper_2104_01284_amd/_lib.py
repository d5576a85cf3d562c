"""ctypes declarations of the ecodp C ABI (include/ecodp.h).

Argument marshalling only: every step of the solver runs in libecodp.so.  The
library is loaded after torch so that both share torch's HIP runtime; there is
no fallback: a missing or unbuildable library raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "libecodp.so")

DP_OK, DP_EINVAL, DP_ENOMEM, DP_EDEVICE, DP_EINFEASIBLE, DP_ESTATE, DP_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
DP_WAIT_AT_RED = 1
DP_TERMINAL_DEVICE = 2
DP_STORE_ALL_V = 1
DP_TIMING = 2
DP_GRAPH = 4
DP_ROUNDS = 8
DP_STALL_TEST = 16
DP_ADJOINT_WIDE = 32

EXPORTS = ("dp_build_problem", "dp_workspace_size", "dp_instance_info_get", "dp_solve", "dp_solve_static",
           "dp_stage", "dp_set_state", "dp_terminal_from_values", "dp_rollout", "dp_adjoint", "dp_adjoint_grade",
           "dp_adjoint_spat", "dp_executed_evaluations", "dp_device_check", "dp_sweep_time", "dp_destroy",
           "dp_loop_create", "dp_loop_step", "dp_loop_get_totals", "dp_loop_destroy",
           "dp_status_string", "dp_last_error")


class DpProblemDesc(C.Structure):
    _fields_ = [
        ("n_stages", C.c_int32), ("ds", C.c_double),
        ("grade", C.POINTER(C.c_double)), ("v_max", C.POINTER(C.c_double)),
        ("n_lights", C.c_int32), ("light_stage", C.POINTER(C.c_int32)),
        ("light_cycle", C.POINTER(C.c_double)), ("light_red", C.POINTER(C.c_double)),
        ("light_offset", C.POINTER(C.c_double)),
        ("t0_abs", C.c_double), ("v0", C.c_double), ("soc0", C.c_double),
        ("v_lo", C.c_double), ("v_hi", C.c_double), ("n_v", C.c_int32),
        ("soc_lo", C.c_double), ("soc_hi", C.c_double), ("n_soc", C.c_int32),
        ("t_f", C.c_double), ("n_t", C.c_int32),
        ("te_lo", C.c_double), ("te_hi", C.c_double), ("n_te", C.c_int32),
        ("tm_lo", C.c_double), ("tm_hi", C.c_double), ("n_tm", C.c_int32),
        ("theta", C.c_double * 5), ("konst", C.c_double * 16), ("fuel", C.c_double * 6),
        ("terminal_V", C.POINTER(C.c_float)),
        ("flags", C.c_uint32),
        ("light_yellow", C.POINTER(C.c_double)),
    ]


class DpOptions(C.Structure):
    _fields_ = [("flags", C.c_uint32), ("kernel", C.c_int32), ("tile", C.c_int32 * 4),
                ("inst_opt", C.POINTER(C.c_int32))]


class DpInstanceInfo(C.Structure):
    _fields_ = [("n_stages", C.c_int32), ("n_v", C.c_int32), ("n_soc", C.c_int32), ("n_t", C.c_int32),
                ("n_u", C.c_int32), ("J_offset", C.c_size_t), ("pi_offset", C.c_size_t),
                ("traj_offset", C.c_size_t), ("slab_elems", C.c_size_t), ("evaluations", C.c_int64),
                ("sweep_kernel", C.c_int32), ("sweep_tile", C.c_int32), ("sweep_split", C.c_int32),
                ("sweep_grid", C.c_int32), ("soc_shift", C.c_int32), ("sweep_persistent", C.c_int32)]


class DpLoopRow(C.Structure):
    _fields_ = [("stage", C.c_int32), ("t_abs", C.c_double), ("v", C.c_double), ("soc", C.c_double),
                ("wait_s", C.c_double), ("horizon", C.c_int32), ("evaluations", C.c_int64), ("V0", C.c_float),
                ("u0", C.c_int32), ("v1", C.c_double), ("soc1", C.c_double), ("dt", C.c_double),
                ("fuel_g", C.c_double), ("cost", C.c_double), ("violations", C.c_int32), ("status", C.c_int32)]


class DpLoopTotals(C.Structure):
    _fields_ = [("stage", C.c_int32), ("t_abs", C.c_double), ("v", C.c_double), ("soc", C.c_double),
                ("fuel_g", C.c_double), ("cost", C.c_double), ("wait_s", C.c_double),
                ("violations", C.c_int32), ("status", C.c_int32), ("steps", C.c_int32),
                ("offline_ms", C.c_double), ("sweep_ms", C.c_double), ("sweep_launches", C.c_int32)]


_lib = None


def load(require_torch: bool = True):
    """Load libecodp.so (built in-tree by ``paper_2104_01284_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if require_torch:
        import torch  # noqa: F401  (load torch's HIP runtime first)
    if not os.path.exists(SO_PATH):
        raise ImportError(f"{SO_PATH} is missing: build it with python -m paper_2104_01284_amd.build")
    lib = C.CDLL(SO_PATH)
    vp, sz = C.c_void_p, C.c_size_t
    lib.dp_build_problem.argtypes = [C.POINTER(DpProblemDesc), C.c_int32, C.POINTER(DpOptions), C.c_int,
                                     C.POINTER(vp)]
    lib.dp_workspace_size.argtypes = [vp, C.POINTER(sz), C.POINTER(sz), C.POINTER(sz)]
    lib.dp_instance_info_get.argtypes = [vp, C.c_int32, C.POINTER(DpInstanceInfo)]
    lib.dp_solve.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.dp_solve_static.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.dp_stage.argtypes = [vp, C.c_int32, C.c_int32, vp, vp, vp, vp, vp]
    lib.dp_set_state.argtypes = [vp, C.c_int32, C.c_double, C.c_double, C.c_double, vp]
    lib.dp_terminal_from_values.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                            C.c_int32, C.c_double, C.c_double, vp, vp]
    lib.dp_rollout.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.dp_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.dp_adjoint_grade.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.dp_adjoint_spat.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.dp_executed_evaluations.argtypes = [vp, C.POINTER(C.c_int64), vp]
    lib.dp_device_check.argtypes = [vp, vp]
    lib.dp_sweep_time.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int32)]
    lib.dp_destroy.argtypes = [vp]
    lib.dp_destroy.restype = None
    lib.dp_loop_create.argtypes = [C.POINTER(DpProblemDesc), C.c_int32, C.c_double, C.c_int32,
                                   C.POINTER(DpOptions), C.c_int32, C.POINTER(vp)]
    lib.dp_loop_step.argtypes = [vp, C.POINTER(DpLoopRow)]
    lib.dp_loop_get_totals.argtypes = [vp, C.POINTER(DpLoopTotals)]
    lib.dp_loop_destroy.argtypes = [vp]
    lib.dp_loop_destroy.restype = None
    lib.dp_status_string.argtypes = [C.c_int]
    lib.dp_status_string.restype = C.c_char_p
    lib.dp_last_error.argtypes = [C.c_char_p, sz]
    _lib = lib
    return lib


class DPError(RuntimeError):
    def __init__(self, code: int, where: str):
        lib = load(require_torch=False)
        buf = C.create_string_buffer(512)
        lib.dp_last_error(buf, 512)
        super().__init__(f"{where}: {lib.dp_status_string(code).decode()} ({code}): {buf.value.decode()}")
        self.code = code


def check(rc: int, where: str):
    if rc != DP_OK:
        raise DPError(rc, where)
