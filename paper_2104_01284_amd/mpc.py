"""Closed-loop receding-horizon eco-driving controller (Sec. V) on the HIP library.

The paper runs its DP as a model-predictive controller: at every step the
horizon problem of Eq. 6 is solved from the measured state, the first control
u_0* is applied to the vehicle, and the horizon moves on.  Its terminal cost
is the value function of an offline DP over the whole route (Sec. III, after
Eq. 9), and Table I reports the solver time of these re-solves.

``ClosedLoop(route)`` solves the full route once on the GPU (``store_all``),
then ``run()`` steps along it: per stage s it

1. lets a vehicle stopped at the stop line of a red signal wait for green
   (Eq. 5c, Eq. 8);
2. builds the horizon problem of the next N = min(20, N_route - s) steps
   (``instances.mpc_window``) with the current state and clock;
3. derives its terminal table from the full-route value slab J_{s+N} on the
   GPU (``dp_terminal_from_values``), handed to the plan as a device table;
4. builds the plan, solves it, and runs the FP64 rollout, whose first step
   is the plant step under u_0* (Eq. 1-2, 5a-b);
5. reads the next state back and advances the clock.

Every numerical step runs in libecodp.so; this module only orders the calls,
moves the state between steps and keeps the statistics.
"""
from __future__ import annotations

import gc
import math
import statistics
import time

from . import instances as ins
from .api import Plan, terminal_from_values


def _red_wait(lights, stage, t_abs):
    """Seconds until green for a vehicle stopped at the signal of ``stage``
    (two-phase SPaT of Eq. 8: red iff (t - O) mod C < R); 0 when green or
    when the stage has no signal."""
    for (L, Cy, R, O) in lights:
        if L == stage:
            ph = (t_abs - O) % Cy
            return R - ph if ph < R else 0.0
    return 0.0


class ClosedLoop:
    """The receding-horizon controller along one route (see the module doc).

    ``route`` is a full-route instance (``instances.mpc_route``); the horizon
    has ``horizon`` steps on the time grid [0, t_f] x n_t and shares the
    route's speed and SoC grids.  ``plan_kw`` goes to every horizon ``Plan``.
    """

    def __init__(self, route: dict, horizon: int = ins.MPC_HORIZON, t_f: float = ins.MPC_T_F,
                 n_t: int = ins.MPC_N_T, device: int = 0, plan_kw: dict | None = None):
        import torch
        self.torch = torch
        self.route = route
        self.horizon, self.t_f, self.n_t = int(horizon), float(t_f), int(n_t)
        self.device = device
        self.plan_kw = dict(plan_kw or {})
        t0 = time.perf_counter()
        self.full = Plan([route], store_all=True, device=device)
        self.full.solve()
        self.J_full = self.full.values(0)          # device [N + 1, n_v, n_soc, n_t_route]
        torch.cuda.synchronize(device)
        self.offline_ms = (time.perf_counter() - t0) * 1e3

    def run(self, steps: int | None = None) -> dict:
        """Drive ``steps`` stages (default: to the end of the route).  Returns
        per-step rows (stage, clock, state, V_0, u_0*, latency) and trip totals;
        ``status`` is 0, or DP_EINFEASIBLE (-4) when no admissible control
        exists or the state leaves the SoC grid."""
        torch = self.torch
        r = self.route
        N_route = int(r["N"])
        steps = N_route if steps is None else min(int(steps), N_route)
        t_f_route = float(r["t_grid"][1])
        J_inf = float(r["konst"][13])
        s_lo, s_hi = r["soc_grid"][0], r["soc_grid"][1]
        s, t_abs, v, soc = 0, float(r["t0_abs"]), float(r["v0"]), float(r["soc0"])
        fuel = cost = 0.0
        wait_s = 0.0
        violations = 0
        rows = []
        status = 0
        evals = 0
        sweep_ms, launches = 0.0, 0
        timing = bool(self.plan_kw.get("timing"))
        stream = torch.cuda.current_stream(self.device)
        # a full garbage collection scans every object torch has created and
        # takes tens of milliseconds: the existing heap leaves the
        # collector's view for the loop, so a step pays only for its own objects
        gc.collect()
        gc.freeze()
        try:
            for _ in range(steps):
                t_start = time.perf_counter()
                if v == 0.0:
                    tau = _red_wait(r["lights"], s, t_abs)
                    t_abs += tau
                    wait_s += tau
                    cost += r["theta"][3] * tau
                win = ins.mpc_window(r, s, t_abs, v, soc, self.horizon, self.t_f, self.n_t)
                N = int(win["N"])
                win["terminal_V"] = terminal_from_values(self.J_full[s + N], t_f_route, t_abs - float(r["t0_abs"]),
                                                         self.n_t, self.t_f, J_inf)
                stream.synchronize()                    # the plan copies the table at build
                plan = Plan([win], device=self.device, **self.plan_kw)
                V0, u0 = plan.solve()
                traj, _ = plan.rollout()
                # rows 0 and 1: the applied control and the plant step (the rollout's
                # own status covers its whole open-loop horizon, of which only the
                # first step is applied here)
                head = traj[0][:2].cpu()
                lat_ms = (time.perf_counter() - t_start) * 1e3
                evals += ins.evaluations(win)
                if timing:
                    ms, n = plan.sweep_time()
                    sweep_ms += ms
                    launches += n
                V0h = float(V0.cpu()[0])
                u = int(head[0, 3])
                rows.append({"s": s, "t_abs": t_abs, "v": v, "soc": soc, "V0": V0h, "u0": u, "latency_ms": lat_ms})
                v1, soc1, dt = float(head[1, 0]), float(head[1, 1]), float(head[1, 2])
                if u < 0 or not (math.isfinite(v1) and math.isfinite(soc1) and math.isfinite(dt)):
                    status = -4                         # no admissible control from this state
                    break
                fuel += float(head[1, 6])
                cost += float(head[1, 7])
                s += 1
                v, soc, t_abs = v1, soc1, t_abs + dt
                if s < N_route:
                    if v > float(r["vmax"][s]):
                        violations += 1
                    if v > 0.0 and _red_wait(r["lights"], s, t_abs) > 0.0:
                        violations += 1                 # crossing a signal during red
                if not (s_lo <= soc <= s_hi):
                    status = -4
                    break
        finally:
            gc.unfreeze()
        lat = [x["latency_ms"] for x in rows]
        return {
            "steps": rows, "stage": s, "v": v, "soc": soc, "t_abs": t_abs,
            "fuel_g": fuel, "cost": cost, "wait_s": wait_s, "violations": violations, "status": status,
            "latency_ms": {"mean": statistics.mean(lat) if lat else None,
                           "var": statistics.pvariance(lat) if len(lat) > 1 else 0.0,
                           "max": max(lat) if lat else None,
                           "argmax_step": lat.index(max(lat)) if lat else None,
                           "median": statistics.median(lat) if lat else None},
            "offline_ms": self.offline_ms, "evals": evals, "sweep_ms": sweep_ms, "sweep_launches": launches,
        }
