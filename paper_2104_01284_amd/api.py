"""Python API over the ecodp C ABI.

Argument marshalling and device-buffer management with torch only; all
computation runs in libecodp.so on the GPU.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class _Desc:
    """An instance dict marshalled into dp_problem_desc (keeps arrays alive)."""

    def __init__(self, inst: dict):
        N = int(inst["N"])
        self.grade = np.ascontiguousarray(inst["grade"], dtype=np.float64)
        self.vmax = np.ascontiguousarray(inst["vmax"], dtype=np.float64)
        if self.grade.shape != (N,) or self.vmax.shape != (N + 1,):
            raise ValueError("grade must have N and vmax N+1 entries")
        lights = inst["lights"]
        self.ls = np.array([x[0] for x in lights], dtype=np.int32)
        self.lc = np.array([x[1] for x in lights], dtype=np.float64)
        self.lr = np.array([x[2] for x in lights], dtype=np.float64)
        self.lo = np.array([x[3] for x in lights], dtype=np.float64)
        # an optional fifth entry: the yellow duration before red (three-phase signals)
        self.ly = np.array([x[4] if len(x) > 4 else 0.0 for x in lights], dtype=np.float64)
        tv = inst.get("terminal_V")
        self.term_dev = None
        self.term = None
        if tv is not None and getattr(tv, "is_cuda", False):
            # a device table (e.g. from terminal_from_values): copied device to device at build
            import torch
            if tv.dtype != torch.float32 or not tv.is_contiguous():
                raise ValueError("a device terminal_V must be a contiguous float32 tensor")
            self.term_dev = tv
        elif tv is not None:
            self.term = np.ascontiguousarray(tv, dtype=np.float32).ravel()
        d = L.DpProblemDesc()
        d.n_stages = N
        d.ds = inst["ds"]
        d.grade = _dptr(self.grade)
        d.v_max = _dptr(self.vmax)
        d.n_lights = len(lights)
        d.light_stage = self.ls.ctypes.data_as(C.POINTER(C.c_int32))
        d.light_cycle = _dptr(self.lc)
        d.light_red = _dptr(self.lr)
        d.light_offset = _dptr(self.lo)
        d.light_yellow = _dptr(self.ly) if any(len(x) > 4 for x in lights) else None
        d.t0_abs, d.v0, d.soc0 = inst["t0_abs"], inst["v0"], inst["soc0"]
        d.v_lo, d.v_hi, d.n_v = inst["v_grid"]
        d.soc_lo, d.soc_hi, d.n_soc = inst["soc_grid"]
        t_lo, d.t_f, d.n_t = inst["t_grid"]
        if t_lo != 0.0:
            raise ValueError("the travel-time grid starts at 0")
        d.te_lo, d.te_hi, d.n_te = inst["te_grid"]
        d.tm_lo, d.tm_hi, d.n_tm = inst["tm_grid"]
        for q in range(5):
            d.theta[q] = inst["theta"][q]
        for q, x in enumerate(inst["konst"]):
            d.konst[q] = x
        for q in range(6):
            d.fuel[q] = inst["fuel"][q]
        d.flags = int(inst.get("flags", L.DP_WAIT_AT_RED))
        if self.term_dev is not None:
            d.terminal_V = C.cast(C.c_void_p(self.term_dev.data_ptr()), C.POINTER(C.c_float))
            d.flags |= L.DP_TERMINAL_DEVICE
        else:
            d.terminal_V = None if self.term is None else self.term.ctypes.data_as(C.POINTER(C.c_float))
        self.d = d


def terminal_from_values(src, t_f_src: float, t_shift: float, n_t: int, t_f: float, J_inf: float):
    """Terminal table of a horizon starting at clock t_shift of a longer solve
    (dp_terminal_from_values): src is a device float32 value slab
    [n_v, n_soc, n_t_src] on the time grid [0, t_f_src]; returns a new device
    float32 tensor [n_v, n_soc, n_t] on [0, t_f], enqueued on the current
    stream.  Pass it as the horizon's terminal_V (with w_soc = 0)."""
    import torch
    if not (src.is_cuda and src.dtype == torch.float32 and src.dim() == 3 and src.is_contiguous()):
        raise ValueError("src must be a contiguous float32 CUDA tensor [n_v, n_soc, n_t_src]")
    n_v, n_s, n_src = src.shape
    dst = torch.empty((n_v, n_s, int(n_t)), dtype=torch.float32, device=src.device)
    lib = L.load()
    stream = C.c_void_p(torch.cuda.current_stream(src.device).cuda_stream)
    L.check(lib.dp_terminal_from_values(C.c_void_p(src.data_ptr()), n_v, n_s, n_src, float(t_f_src), float(t_shift),
                                        int(n_t), float(t_f), float(J_inf), C.c_void_p(dst.data_ptr()), stream),
            "dp_terminal_from_values")
    return dst


class Plan:
    """A set of receding-horizon problems built into one dp_plan.

    ``Plan(instances, store_all=False, timing=False, device=0)`` validates the
    instances and uploads their parameter blocks; ``solve()`` runs the backward
    recursion of every instance on the current torch stream, several instances
    in one persistent sweep (or, with ``rounds=True``, in rounds of one stage
    each).
    ``graph=True`` records the solve once into a HIP graph and replays it on
    later calls; ``stall_test=True`` sets the persistent sweep's test hook
    (its bounded wait gives up and raises the device error word).
    """

    def __init__(self, instances, store_all: bool = False, timing: bool = False, device: int = 0,
                 sweep_tile: int = 0, kernel: int = 0, split: int = 0, wg_per_cu: int = 0,
                 graph: bool = False, inst_opts=None, rounds: bool = False, stall_test: bool = False,
                 adjoint_wide: bool = False):
        import torch
        self.torch = torch
        if isinstance(instances, dict):
            instances = [instances]
        self.instances = list(instances)
        self.lib = L.load()
        self._descs = [_Desc(x) for x in self.instances]
        arr = (L.DpProblemDesc * len(self._descs))(*[x.d for x in self._descs])
        opt = L.DpOptions()
        opt.flags = (L.DP_STORE_ALL_V if store_all else 0) | (L.DP_TIMING if timing else 0) | \
            (L.DP_GRAPH if graph else 0) | (L.DP_ROUNDS if rounds else 0) | (L.DP_STALL_TEST if stall_test else 0) | \
            (L.DP_ADJOINT_WIDE if adjoint_wide else 0)
        opt.tile[0] = int(sweep_tile)
        opt.tile[1] = int(split)
        opt.tile[2] = int(wg_per_cu)
        opt.kernel = int(kernel)   # 0 automatic, 1 simple per-node sweep, 2 grouped LDS sweep
        if inst_opts is not None:
            # per instance (kernel, tile, split, wg_per_cu); 0 = the plan-wide value
            io = np.zeros((len(self.instances), 4), dtype=np.int32)
            for b, o in enumerate(inst_opts):
                if o is not None:
                    io[b, :len(o)] = o
            self._inst_opts = np.ascontiguousarray(io)
            opt.inst_opt = self._inst_opts.ctypes.data_as(C.POINTER(C.c_int32))
        self.store_all = store_all
        self.device = device
        h = C.c_void_p()
        L.check(self.lib.dp_build_problem(arr, len(self._descs), C.byref(opt), device, C.byref(h)),
                "dp_build_problem")
        self._h = h
        bJ, bP, bS = C.c_size_t(), C.c_size_t(), C.c_size_t()
        L.check(self.lib.dp_workspace_size(h, C.byref(bJ), C.byref(bP), C.byref(bS)), "dp_workspace_size")
        self.bytes = (bJ.value, bP.value, bS.value)
        self.info = []
        for b in range(len(self._descs)):
            info = L.DpInstanceInfo()
            L.check(self.lib.dp_instance_info_get(h, b, C.byref(info)), "dp_instance_info_get")
            self.info.append(info)
        self.n = len(self._descs)
        dev = torch.device("cuda", device)
        self.J = torch.empty(max(1, bJ.value), dtype=torch.uint8, device=dev)
        self.pi = torch.empty(max(1, bP.value), dtype=torch.uint8, device=dev)
        self.scratch = torch.empty(max(1, bS.value), dtype=torch.uint8, device=dev)
        self.V0 = torch.empty(self.n, dtype=torch.float32, device=dev)
        self.u0 = torch.empty(self.n, dtype=torch.int16, device=dev)
        self._rows = sum(int(i.n_stages) + 1 for i in self.info)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self.lib.dp_destroy(h)
            self._h = None

    def _stream(self):
        return C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    # ------------------------------------------------------------- solve --
    def solve(self):
        """Enqueue the backward recursion of every instance; returns (V0, u0) device tensors."""
        L.check(self.lib.dp_solve(self._h, C.c_void_p(self.J.data_ptr()), C.c_void_p(self.pi.data_ptr()),
                                  C.c_void_p(self.scratch.data_ptr()), C.c_void_p(self.V0.data_ptr()),
                                  C.c_void_p(self.u0.data_ptr()), self._stream()), "dp_solve")
        return self.V0, self.u0

    def solve_static(self):
        """dp_solve on the library's own scratch (dp_solve_static: no device
        allocation; calls on one device must not overlap); returns (V0, u0)."""
        L.check(self.lib.dp_solve_static(self._h, C.c_void_p(self.J.data_ptr()), C.c_void_p(self.pi.data_ptr()),
                                         C.c_void_p(self.V0.data_ptr()), C.c_void_p(self.u0.data_ptr()),
                                         self._stream()), "dp_solve_static")
        return self.V0, self.u0

    def slab_shape(self, b=0):
        i = self.info[b]
        return (int(i.n_v), int(i.n_soc), int(i.n_t))

    def value(self, b: int, k: int):
        """Device view of J_k of instance b (stored stages only)."""
        i = self.info[b]
        S = int(i.slab_elems)
        idx = k if self.store_all else (k & 1)
        base = int(i.J_offset) // 4 + idx * S
        return self.J.view(self.torch.float32)[base:base + S].view(self.slab_shape(b))

    def values(self, b: int):
        """Device view of J_0..J_N of instance b (requires store_all)."""
        assert self.store_all
        i = self.info[b]
        S = int(i.slab_elems)
        base = int(i.J_offset) // 4
        return self.J.view(self.torch.float32)[base:base + (int(i.n_stages) + 1) * S].view(
            (int(i.n_stages) + 1,) + self.slab_shape(b))

    def policy(self, b: int, k: int | None = None):
        i = self.info[b]
        S = int(i.slab_elems)
        base = int(i.pi_offset) // 2
        allp = self.pi.view(self.torch.int16)[base:base + int(i.n_stages) * S].view(
            (int(i.n_stages),) + self.slab_shape(b))
        return allp if k is None else allp[k]

    # -------------------------------------------------------------- stage --
    def stage(self, b: int, k: int, J_next):
        """One backward step from a caller J_{k+1} (device float32 slab)."""
        torch = self.torch
        J_next = J_next.contiguous().to(torch.float32)
        assert tuple(J_next.shape) == self.slab_shape(b)
        J_out = torch.empty_like(J_next)
        pi_out = torch.empty(J_next.shape, dtype=torch.int16, device=J_next.device)
        L.check(self.lib.dp_stage(self._h, b, k, C.c_void_p(J_next.data_ptr()), C.c_void_p(J_out.data_ptr()),
                                  C.c_void_p(pi_out.data_ptr()), C.c_void_p(self.scratch.data_ptr()),
                                  self._stream()), "dp_stage")
        return J_out, pi_out

    # ---------------------------------------------------------- set_state --
    def set_state(self, b: int, v0: float, soc0: float, t0_abs: float):
        """Move instance b to a new x0 = (v0, soc0) at absolute clock t0_abs
        (receding horizon); ordered on the current stream before later calls."""
        L.check(self.lib.dp_set_state(self._h, int(b), float(v0), float(soc0), float(t0_abs), self._stream()),
                "dp_set_state")
        inst = dict(self.instances[b])
        inst["v0"], inst["soc0"], inst["t0_abs"] = float(v0), float(soc0), float(t0_abs)
        self.instances[b] = inst

    # ------------------------------------------------------------ rollout --
    def rollout(self):
        """Forward rollout of every instance: (list of [N+1, 8] traj tensors, status [n, 2])."""
        torch = self.torch
        traj = torch.empty(self._rows * 8, dtype=torch.float64, device=self.V0.device)
        status = torch.empty(2 * self.n, dtype=torch.int32, device=self.V0.device)
        L.check(self.lib.dp_rollout(self._h, C.c_void_p(self.pi.data_ptr()), C.c_void_p(self.u0.data_ptr()),
                                    C.c_void_p(traj.data_ptr()), C.c_void_p(status.data_ptr()), self._stream()),
                "dp_rollout")
        out = []
        for i in self.info:
            o = int(i.traj_offset)
            out.append(traj[o:o + (int(i.n_stages) + 1) * 8].view(int(i.n_stages) + 1, 8))
        return out, status.view(self.n, 2)

    # ------------------------------------------------------------ adjoint --
    def adjoint(self):
        """dV_0/dtheta (FP64 [n, 5]) with the stored policy held fixed."""
        torch = self.torch
        grad = torch.empty(5 * self.n, dtype=torch.float64, device=self.V0.device)
        L.check(self.lib.dp_adjoint(self._h, C.c_void_p(self.J.data_ptr()), C.c_void_p(self.pi.data_ptr()),
                                    C.c_void_p(self.u0.data_ptr()), C.c_void_p(self.scratch.data_ptr()),
                                    C.c_void_p(grad.data_ptr()), self._stream()), "dp_adjoint")
        return grad.view(self.n, 5)

    def adjoint_grade(self):
        """dV_0/dtheta (FP64 [n, 5]) and dV_0/dG_k for the grade of every step
        (FP64, one [N_b] tensor per instance), the stored policy held fixed."""
        torch = self.torch
        grad = torch.empty(5 * self.n, dtype=torch.float64, device=self.V0.device)
        Ns = [int(i.n_stages) for i in self.info]
        dg = torch.empty(sum(Ns), dtype=torch.float64, device=self.V0.device)
        L.check(self.lib.dp_adjoint_grade(self._h, C.c_void_p(self.J.data_ptr()), C.c_void_p(self.pi.data_ptr()),
                                          C.c_void_p(self.u0.data_ptr()), C.c_void_p(self.scratch.data_ptr()),
                                          C.c_void_p(grad.data_ptr()), C.c_void_p(dg.data_ptr()), self._stream()),
                "dp_adjoint_grade")
        return grad.view(self.n, 5), list(dg.split(Ns))

    def adjoint_spat(self):
        """dV_0/dtheta (FP64 [n, 5]) and dV_0 with respect to the offset, red
        time and cycle of every signal (FP64, one [n_lights_b, 3] tensor per
        instance, signals in the order of the instance's ``lights``), the
        stored policy held fixed."""
        torch = self.torch
        grad = torch.empty(5 * self.n, dtype=torch.float64, device=self.V0.device)
        nl = [len(x.ls) for x in self._descs]
        ds = torch.empty(max(1, 3 * sum(nl)), dtype=torch.float64, device=self.V0.device)
        L.check(self.lib.dp_adjoint_spat(self._h, C.c_void_p(self.J.data_ptr()), C.c_void_p(self.pi.data_ptr()),
                                         C.c_void_p(self.u0.data_ptr()), C.c_void_p(self.scratch.data_ptr()),
                                         C.c_void_p(grad.data_ptr()), C.c_void_p(ds.data_ptr()), self._stream()),
                "dp_adjoint_spat")
        return grad.view(self.n, 5), [x.view(-1, 3) for x in ds[:3 * sum(nl)].split([3 * n for n in nl])]

    def sweep_time(self):
        ms, n = C.c_double(), C.c_int32()
        L.check(self.lib.dp_sweep_time(self._h, C.byref(ms), C.byref(n)), "dp_sweep_time")
        return ms.value, n.value

    def evaluations(self) -> int:
        """Dense state-control evaluations of one solve of every instance."""
        return int(sum(int(i.evaluations) for i in self.info))

    def executed_evaluations(self):
        """Evaluations the state sweep executed per instance since the last
        solve began (synchronises the current stream)."""
        out = (C.c_int64 * self.n)()
        L.check(self.lib.dp_executed_evaluations(self._h, out, self._stream()), "dp_executed_evaluations")
        return [int(x) for x in out]

    def device_check(self):
        """Raise DPError if a kernel set the plan's device error word
        (synchronises the current stream)."""
        L.check(self.lib.dp_device_check(self._h, self._stream()), "dp_device_check")
