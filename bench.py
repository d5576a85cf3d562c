#!/usr/bin/env python
"""Benchmark of the eco-driving DP hot path on one MI355X.

One step = one pass of the whole path over one synthetic problem: the
backward recursion with stage tables, state sweeps, signal handling and the
exact root step (dp_solve), the FP64 policy rollout (dp_rollout) and the
fixed-policy adjoint (dp_adjoint).  Inputs are resident in HBM before the
timed region.  Prints one JSON line.  The batched workload times the
256-instance solve alone (one HIP-graph replay per step); the mpc workload
times closed-loop receding-horizon steps along a long route (one horizon
re-solve from the measured state per step).

  python bench.py [--gpus 1] [--steps K] [--warmup W]
                  [--workload large|realistic|plain|paper|batched|mpc] [--kernel K] [--tile T] [--split S]

The default workload is the large fine-grid solve (3 km, 300 stages,
201x81x401 states, 41x21 controls).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOPS_PER_EVAL = 24          # canonical FP32 work of one state-control evaluation
FP32_PEAK_TFLOPS = 157.3     # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2 (packed) x 2.4 GHz
HBM_PEAK_BPS = 8.0e12        # MI355X HBM3E
ALG_BYTES_PER_STATE = 10     # per state and stage: read J_{k+1} 4, write J_k 4, write pi_k 2
DESCR = {
    "realistic": "realistic_2km: 200 stages x 101x41x201 states x 41x21 controls, 4 signals, +-3% grade",
    "large": "large_3km: 300 stages x 201x81x401 states x 41x21 controls, 8 signals, +-3% grade",
    "plain": "plain_500m: 50 stages x 21x11x31 states x 11x11 controls, 1 signal",
    "paper": "paper_shape: 20 stages x 35x26x40 states x 23x30 controls, 1 signal",
    "batched": "batched_256: 256 heterogeneous solves, 50-200 stages, (41-101)x(21-41)x(61-201) states, "
               "(21-41)x(11-21) controls, one HIP graph per solve",
    "mpc": "mpc_3km: closed-loop receding horizon along a 3 km route (300 stages, 8 signals); per step one "
           "20-stage horizon of 35x26x40 states x 23x30 controls with its terminal cost from an offline "
           "full-route DP, solved from the measured state, u_0* applied to the FP64 plant",
}


PROFILE_NAME = {"realistic": "realistic_2km", "large": "large_3km", "plain": "plain_500m", "paper": "paper_shape"}


def cpu_baseline(inst, budget_s: float):
    """The FP64 oracle's backward stages from J_N, timed on all host threads
    until the budget is spent (at least one stage), then one more stage on one
    thread when that fits the budget at the measured rate."""
    import oracle
    I = oracle.Instance(inst)
    J = oracle.terminal(I)
    cores = oracle.num_threads()
    t0 = time.perf_counter()
    done = 0
    k = inst["N"] - 1
    while k >= 0:
        J, _, _ = oracle.stage(I, k, J)
        done += 1
        k -= 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    evals = done * I.S * I.n_u
    out = {"value": evals / dt, "unit": "state-control evals/s", "cores": cores, "kind": "oracle",
           "sample": f"{done} backward stages (k={inst['N'] - 1}..{inst['N'] - done}) of {inst['name']} "
                     f"from J_N, FP64, {evals:.3e} evaluations in {dt:.1f} s on {cores} threads"}
    # one more stage on one thread, when it fits the budget at the measured rate
    if cores > 1 and dt / done * cores <= 1.5 * budget_s:
        oracle.set_num_threads(1)
        t1 = time.perf_counter()
        oracle.stage(I, max(k, 0), J)
        dt1 = time.perf_counter() - t1
        oracle.set_num_threads(cores)
        out["value_1core"] = I.S * I.n_u / dt1
        out["sample"] += f"; one more stage on 1 thread in {dt1:.1f} s"
    return out


def sweep_pitch(n_t):
    """LDS row pitch of the grouped sweep (its PITCH template argument): the
    time nodes plus one padding column, rounded up to 32."""
    return (n_t + 1 + 31) // 32 * 32


def measured_traffic(workload, kernel_name, split):
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary
    of this workload, if it was measured on the current sweep source, the
    same kernel instance and the same number of control slices; else None."""
    import re
    from paper_2104_01284_amd.profiling import sweep_source_hash
    path = os.path.join(ROOT, "profiles", f"sweep_{PROFILE_NAME.get(workload, workload)}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"traffic_bytes_per_launch=(\S+) sweep_source=(\S+) split=(\S+)", text)
    if (not m or m.group(2) != sweep_source_hash() or m.group(3) != str(split)
            or kernel_name not in text.split("\n")[0]):
        return None
    return float(m.group(1))


def cpu_baseline_mpc(route, budget_s: float):
    """The FP64 oracle solving horizon problems of the route (stage 0, 1, ...
    from the route's start state, zero terminal table: the work does not
    depend on the values) on all host threads until the budget is spent."""
    import numpy as np
    import oracle
    from paper_2104_01284_amd import instances
    cores = oracle.num_threads()
    t0 = time.perf_counter()
    done = evals = 0
    while True:
        w = instances.mpc_window(route, done, 0.0, route["v0"], route["soc0"])
        w["terminal_V"] = np.zeros((w["v_grid"][2], w["soc_grid"][2], w["t_grid"][2]))
        oracle.solve(w)
        done += 1
        evals += instances.evaluations(w)
        if time.perf_counter() - t0 >= budget_s or done >= route["N"]:
            break
    dt = time.perf_counter() - t0
    return {"value": evals / dt, "unit": "state-control evals/s", "cores": cores, "kind": "oracle",
            "ms_per_horizon": dt * 1e3 / done,
            "sample": f"{done} horizon solves (stages 0..{done - 1} of {route['name']}), FP64, "
                      f"{evals:.3e} evaluations in {dt:.1f} s on {cores} threads"}


def bench_mpc(args):
    """Closed-loop receding horizon: ``warmup`` untimed steps from the route
    start, then ``steps`` timed steps of a fresh loop from the route start."""
    import torch
    from paper_2104_01284_amd import instances
    from paper_2104_01284_amd.mpc import ClosedLoop
    route = instances.mpc_route()
    print(f"[bench] workload {DESCR['mpc']}", file=sys.stderr, flush=True)
    if args.warmup:
        ClosedLoop(route).run(args.warmup)
    # the timed drive replays each step's recorded solve; the sweep launches
    # are timed with events on a separate drive of the same route
    loop = ClosedLoop(route)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = loop.run(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    k = len(res["steps"])
    del loop
    tres = ClosedLoop(route, plan_kw={"timing": True}).run(min(k, 40))
    achieved = FLOPS_PER_EVAL * tres["evals"] / (tres["sweep_ms"] * 1e-3) / 1e12 if tres["sweep_ms"] else None
    out = {
        "metric": "state-control evals/s and full-horizon solve ms (FP32 vs FP64 oracle, 1e-4 rel V_0)",
        "value": res["evals"] / wall, "unit": "state-control evals/s",
        "n_gpus": 1, "steps": k, "warmup": args.warmup, "ms_per_step": wall * 1e3 / max(1, k),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": DESCR["mpc"], "route_stages": int(route["N"]), "horizon": instances.MPC_HORIZON,
                   "step": "dp_loop_step: signal wait + in-place horizon update + terminal table + recorded "
                           "dp_solve + dp_rollout + D2H of the plant step"},
        "mpc": {"latency_ms": res["latency_ms"], "fuel_g": res["fuel_g"], "trip_s": res["t_abs"],
                "cost": res["cost"], "wait_s": res["wait_s"], "violations": res["violations"],
                "status": res["status"], "stages_driven": res["stage"], "offline_full_route_ms": res["offline_ms"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_PEAK_TFLOPS if achieved else None, "traffic": None,
                     "kernel": "state sweep", "avg_launch_ms": tres["sweep_ms"] / max(1, tres["sweep_launches"]),
                     "launches": tres["sweep_launches"], "timed_steps": len(tres["steps"])},
    }
    if not args.no_cpu_baseline:
        print("[bench] oracle CPU baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline_mpc(route, args.cpu_budget)
        out["cpu_baseline"]["host"] = platform.processor() or platform.machine()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default per workload: plain 1000, paper 200, realistic 50, batched 10, large 5)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large", choices=sorted(DESCR))
    ap.add_argument("--tile", type=int, default=0, help="SoC rows per sweep workgroup (4, 8, 16; 0 automatic)")
    ap.add_argument("--split", type=int, default=0, help="control slices per node tile (0 automatic)")
    ap.add_argument("--wg-per-cu", type=int, default=0, help="resident sweep workgroups per CU (0 automatic)")
    ap.add_argument("--kernel", type=int, default=0, help="sweep variant (0 automatic, 1 simple, 2 grouped)")
    ap.add_argument("--rounds", action="store_true",
                    help="batched workload: rounds of launches instead of the persistent sweep")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the library's own sweep configuration instead of the autotuner's")
    ap.add_argument("--mpc-repeats", type=int, default=20,
                    help="receding-horizon latency repeats after the timed steps (0 skips)")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = {"plain": 1000, "paper": 200, "realistic": 50, "batched": 10, "large": 5,
                      "mpc": 300}[args.workload]
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the solver has no multi-GPU path (asked for {args.gpus}); "
              f"run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2104_01284_amd import instances
    from paper_2104_01284_amd.api import Plan

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_MiB": args.copy_calibration, "copies": 3,
                          "expected_fetch_KiB_per_copy": args.copy_calibration * 1024,
                          "expected_write_KiB_per_copy": args.copy_calibration * 1024}))
        return
    if args.workload == "mpc":
        bench_mpc(args)
        return
    batched = args.workload == "batched"
    insts = instances.batched(256) if batched else [instances.make(args.workload)]
    inst = insts[0]
    print(f"[bench] workload {DESCR[args.workload]}", file=sys.stderr, flush=True)
    opts = dict(sweep_tile=args.tile, split=args.split, wg_per_cu=args.wg_per_cu, kernel=args.kernel,
                rounds=args.rounds)
    tuned = None
    if not args.no_tune and not (args.kernel or args.tile):
        from paper_2104_01284_amd.autotune import tuned_batch_options, tuned_options
        t0 = time.perf_counter()
        # a batch: one SoC tile for all, by whole-batch solves
        tuned = tuned_batch_options(insts, verbose=True) if batched else tuned_options(insts, verbose=True)
        print(f"[bench] sweep autotune {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        opts["inst_opts"] = tuned
    if batched:
        # the batch is timed as recorded HIP-graph solves; the sweep launches
        # are timed with events in a separate pass of an identical plan
        plan = Plan(insts, store_all=False, graph=True, **opts)
        tplan = Plan(insts, store_all=False, timing=True, **opts)
        tplan.solve()
        torch.cuda.synchronize()
        tplan.sweep_time()
        tplan.solve()
        torch.cuda.synchronize()
        sweep_ms, launches = tplan.sweep_time()
        del tplan
    else:
        plan = Plan(insts, store_all=True, timing=True, **opts)
    evals = plan.evaluations()
    info = plan.info[0]
    persistent = bool(info.sweep_persistent)

    def step():
        plan.solve()
        if not batched:
            plan.rollout()
            plan.adjoint()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if not batched:
        plan.sweep_time()                   # discard warm-up sweep events

    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q in range(args.steps):
        ev[q][0].record(stream)
        plan.solve()
        ev[q][1].record(stream)
        if not batched:
            plan.rollout()
            ev[q][2].record(stream)
            plan.adjoint()
            ev[q][3].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if not batched:
        sweep_ms, launches = plan.sweep_time()
        sweep_ms /= args.steps
        launches //= args.steps
    executed = sum(plan.executed_evaluations())      # of the last solve
    plan.device_check()
    solve_ms = [e[0].elapsed_time(e[1]) for e in ev]
    parts = {}
    if not batched:
        roll = [e[1].elapsed_time(e[2]) for e in ev]
        adj = [e[2].elapsed_time(e[3]) for e in ev]
        parts = {"rollout_ms": statistics.mean(roll), "rollout_us_per_stage": 1e3 * statistics.mean(roll) / inst["N"],
                 "adjoint_ms": statistics.mean(adj), "adjoint_us_per_stage": 1e3 * statistics.mean(adj) / inst["N"]}
    ms_per_step = wall * 1e3 / args.steps
    V0 = float(plan.V0.cpu()[0])

    # end-to-end receding-horizon latency on host clocks: upload of a moved
    # x0 and signal clock (dp_set_state), the recorded solve, and the copy of
    # V_0 and u_0* back to the host; the plan build is outside
    mpc = None
    if not batched and args.mpc_repeats > 0:
        import numpy as np
        g = Plan(insts, store_all=False, graph=True, **opts)
        rng = np.random.default_rng(11)
        vlo, vhi, _ = inst["v_grid"]
        slo, shi, _ = inst["soc_grid"]

        def mpc_step(q):
            v0 = float(np.clip(inst["v0"] + rng.uniform(-0.5, 0.5), vlo, vhi))
            s0 = float(np.clip(inst["soc0"] + rng.uniform(-0.01, 0.01), slo, shi))
            t = time.perf_counter()
            g.set_state(0, v0, s0, inst["t0_abs"] + 0.5 * q)
            g.solve()
            V, u = g.V0.cpu(), g.u0.cpu()
            assert V.numel() == 1 and u.numel() == 1
            return (time.perf_counter() - t) * 1e3

        for q in range(3):
            mpc_step(q)
        lat = [mpc_step(q) for q in range(args.mpc_repeats)]
        mpc = {"mean": statistics.mean(lat), "var": statistics.pvariance(lat), "max": max(lat),
               "median": statistics.median(lat), "repeats": len(lat),
               "what": "host wall time: dp_set_state (H2D of x0 and signal tables) + recorded dp_solve + "
                       "D2H of V_0 and u_0*"}
        del g

    # sweep-kernel roofline over one solve: all state-control evaluations of
    # the solve at the canonical FP32 work per evaluation, over the summed
    # duration of its sweep launches.  A persistent batch runs its kernel
    # classes side by side for the whole solve: its interval is the recorded
    # solve as replayed in the timed steps (stage tables, terminal and roots
    # included, so an upper bound on the sweep's own time); the eager timing
    # pass, whose launches are not recorded, is reported beside it
    eager_interval_ms = None
    if batched and persistent:
        eager_interval_ms = sweep_ms / max(1, launches)
        sweep_ms, launches = statistics.mean(solve_ms), 1
    avg_launch_ms = sweep_ms / max(1, launches)
    achieved = FLOPS_PER_EVAL * evals / (sweep_ms * 1e-3) / 1e12
    achieved_exec = FLOPS_PER_EVAL * executed / (sweep_ms * 1e-3) / 1e12
    traffic = None if batched else measured_traffic(
        args.workload, f"k_sweep_lds<{int(info.sweep_tile)}, {sweep_pitch(int(info.n_t))}>", int(info.sweep_split))
    states = sum(int(i.slab_elems) * int(i.n_stages) for i in plan.info)   # state-stages of one solve
    alg_bytes = ALG_BYTES_PER_STATE * states / max(1, launches)
    out = {
        "metric": "state-control evals/s and full-horizon solve ms (FP32 vs FP64 oracle, 1e-4 rel V_0)",
        "value": evals / (ms_per_step * 1e-3),
        "unit": "state-control evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": DESCR[args.workload], "evaluations_per_solve": evals,
                   "step": "dp_solve (HIP graph)" if batched else "dp_solve + dp_rollout + dp_adjoint",
                   "sweep": {"kernel": int(info.sweep_kernel),
                             "tile": int(info.sweep_tile), "autotuned": tuned is not None,
                             "split": int(info.sweep_split), "grid": int(info.sweep_grid),
                             "soc_shift": int(info.soc_shift)}},
        "solve_ms": {"mean": statistics.mean(solve_ms),
                     "var": statistics.pvariance(solve_ms) if len(solve_ms) > 1 else 0.0,
                     "max": max(solve_ms), "median": statistics.median(solve_ms)},
        "solve_evals_per_s": evals / (statistics.mean(solve_ms) * 1e-3),
        **parts,
        "mpc_latency_ms": mpc,
        "V0": V0,
        "V0_all_mean": float(plan.V0.double().mean().cpu()) if batched else V0,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_PEAK_TFLOPS,
                     "traffic": traffic,
                     "traffic_unit": "HBM bytes per sweep launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "kernel": ("persistent state sweep (one launch per kernel class, side by side; "
                                "one interval per recorded solve, tables and roots included)"
                                if persistent else "state sweep"),
                     "avg_launch_ms": avg_launch_ms, "launches_per_solve": launches,
                     **({"eager_interval_ms": eager_interval_ms} if eager_interval_ms is not None else {}),
                     "flops_per_launch": FLOPS_PER_EVAL * evals / max(1, launches),
                     "executed_evaluations_per_solve": executed,
                     "executed_over_dense": executed / evals,
                     "frac_executed": achieved_exec / FP32_PEAK_TFLOPS,
                     "hbm": {"algorithmic_bytes_per_launch": alg_bytes,
                             "algorithmic_frac": alg_bytes / (avg_launch_ms * 1e-3) / HBM_PEAK_BPS,
                             "measured_bytes_per_launch": traffic,
                             "measured_frac": (traffic / (avg_launch_ms * 1e-3) / HBM_PEAK_BPS
                                               if traffic else None),
                             "peak_GBps": HBM_PEAK_BPS / 1e9}},
    }
    # errors of this solve's results against the stored FP64 oracle results
    # of the same instance (digest-checked; null when none are stored)
    from paper_2104_01284_amd.profiling import golden_report, load_golden
    g = None if batched else load_golden(args.workload, inst)
    out["V0_rel_err_vs_oracle"] = None
    if batched:
        from paper_2104_01284_amd.profiling import batch_golden_report
        rep_ = batch_golden_report(insts, plan.V0.cpu().tolist(), plan.u0.cpu().tolist())
        if rep_ is not None:
            out["V0_rel_err_vs_oracle"] = rep_["V0_max_rel_err"]
            out["errors_vs_fp64_oracle"] = rep_
    if g is not None:
        trajs, _ = plan.rollout()
        grad = plan.adjoint()
        rep_ = golden_report(g, V0, plan.values(0), plan.policy(0), trajs[0], grad[0].cpu().tolist())
        out["V0_rel_err_vs_oracle"] = rep_["V0_rel_err"]
        out["errors_vs_fp64_oracle"] = rep_
    if not args.no_cpu_baseline:
        print("[bench] oracle CPU baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_budget)
        out["cpu_baseline"]["host"] = platform.processor() or platform.machine()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
