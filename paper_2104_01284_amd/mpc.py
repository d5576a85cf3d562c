"""Closed-loop receding-horizon eco-driving controller (Sec. V) on the HIP library.

The paper runs its DP as a model-predictive controller: at every step the
horizon problem of Eq. 6 is solved from the measured state, the first control
u_0* is applied to the vehicle, and the horizon moves on.  Its terminal cost
is the value function of an offline DP over the whole route (Sec. III, after
Eq. 9), and Table I reports the solver time of these re-solves.

The loop lives in libecodp.so (``dp_loop_create`` / ``dp_loop_step``): it
solves the full route once, keeps one plan per horizon length for the whole
drive and moves it along the route in place, and per step does the stop-line
wait at a red signal (Eq. 5c, Eq. 8), the horizon's terminal table from the
full-route values, the recorded solve, the FP64 rollout whose first step is
the plant step (Eq. 1-2, 5a-b), and the speed-limit and red-crossing checks.
This module marshals the route, times each step on the host clock and
collects the rows.
"""
from __future__ import annotations

import ctypes as C
import gc
import statistics
import time

from . import _lib as L
from . import instances as ins
from .api import _Desc


class ClosedLoop:
    """The receding-horizon controller along one route (see the module doc).

    ``route`` is a full-route instance (``instances.mpc_route``); the horizon
    has ``horizon`` steps on the time grid [0, t_f] x n_t and shares the
    route's speed and SoC grids.  ``plan_kw``: ``timing`` (sum the sweep
    launch times with events instead of replaying recorded graphs),
    ``kernel`` and ``sweep_tile`` for the horizon plans.
    """

    def __init__(self, route: dict, horizon: int = ins.MPC_HORIZON, t_f: float = ins.MPC_T_F,
                 n_t: int = ins.MPC_N_T, device: int = 0, plan_kw: dict | None = None):
        import torch
        self.torch = torch
        self.lib = L.load()
        self.route = route
        kw = dict(plan_kw or {})
        o = L.DpOptions()
        o.flags = L.DP_TIMING if kw.pop("timing", False) else 0
        o.kernel = int(kw.pop("kernel", 0) or 0)
        o.tile[0] = int(kw.pop("sweep_tile", 0) or 0)
        if kw:
            raise ValueError(f"unknown plan options {sorted(kw)}")
        self._desc = _Desc(route)
        torch.cuda.init()
        h = C.c_void_p()
        L.check(self.lib.dp_loop_create(C.byref(self._desc.d), int(horizon), float(t_f), int(n_t), C.byref(o),
                                        int(device), C.byref(h)), "dp_loop_create")
        self._h = h
        self.offline_ms = self.totals().offline_ms

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self.lib.dp_loop_destroy(h)
            self._h = None

    def totals(self) -> L.DpLoopTotals:
        t = L.DpLoopTotals()
        L.check(self.lib.dp_loop_get_totals(self._h, C.byref(t)), "dp_loop_get_totals")
        return t

    def run(self, steps: int | None = None) -> dict:
        """Drive ``steps`` stages (default: to the end of the route).  Returns
        per-step rows (stage, clock, state, V_0, u_0*, latency) and trip totals;
        ``status`` is 0, or DP_EINFEASIBLE (-4) when no admissible control
        exists or the state leaves the SoC grid."""
        N_route = int(self.route["N"])
        steps = N_route if steps is None else min(int(steps), N_route)
        rows = []
        evals = 0
        row = L.DpLoopRow()
        # a full garbage collection scans every object torch has created and
        # takes tens of milliseconds: the existing heap leaves the
        # collector's view for the loop, so a step pays only for its own objects
        gc.collect()
        gc.freeze()
        try:
            for _ in range(steps):
                if self.totals().stage >= N_route:
                    break
                t0 = time.perf_counter()
                L.check(self.lib.dp_loop_step(self._h, C.byref(row)), "dp_loop_step")
                lat_ms = (time.perf_counter() - t0) * 1e3
                evals += int(row.evaluations)
                rows.append({"s": row.stage, "t_abs": row.t_abs, "v": row.v, "soc": row.soc, "V0": float(row.V0),
                             "u0": int(row.u0), "latency_ms": lat_ms, "wait_s": row.wait_s,
                             "violations": int(row.violations)})
                if row.status != L.DP_OK:
                    break
        finally:
            gc.unfreeze()
        t = self.totals()
        lat = [x["latency_ms"] for x in rows]
        return {
            "steps": rows, "stage": t.stage, "v": t.v, "soc": t.soc, "t_abs": t.t_abs,
            "fuel_g": t.fuel_g, "cost": t.cost, "wait_s": t.wait_s, "violations": t.violations,
            "status": t.status,
            "latency_ms": {"mean": statistics.mean(lat) if lat else None,
                           "var": statistics.pvariance(lat) if len(lat) > 1 else 0.0,
                           "max": max(lat) if lat else None,
                           "argmax_step": lat.index(max(lat)) if lat else None,
                           "median": statistics.median(lat) if lat else None},
            "offline_ms": self.offline_ms, "evals": evals, "sweep_ms": t.sweep_ms,
            "sweep_launches": t.sweep_launches,
        }
