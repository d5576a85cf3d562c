#!/usr/bin/env python
"""Benchmark of the eco-driving DP hot path on one MI355X.

One step = one pass of the whole path over one synthetic problem: the
backward recursion with stage tables, state sweeps, signal handling and the
exact root step (dp_solve), the FP64 policy rollout (dp_rollout) and the
fixed-policy adjoint (dp_adjoint).  Inputs are resident in HBM before the
timed region.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload realistic|large|plain|paper]
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
DESCR = {
    "realistic": "realistic_2km: 200 stages x 101x41x201 states x 41x21 controls, 4 signals, +-3% grade",
    "large": "large_3km: 300 stages x 201x81x401 states x 41x21 controls, 8 signals, +-3% grade",
    "plain": "plain_500m: 50 stages x 21x11x31 states x 11x11 controls, 1 signal",
    "paper": "paper_shape: 20 stages x 35x26x40 states x 23x30 controls, 1 signal",
}


def cpu_baseline(inst, budget_s: float):
    """The FP64 oracle's backward stages from J_N, timed on the host cores
    until the budget is spent (at least one stage)."""
    import oracle
    I = oracle.Instance(inst)
    J = oracle.terminal(I)
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
    return {"value": evals / dt, "unit": "state-control evals/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{done} backward stages (k={inst['N'] - 1}..{inst['N'] - done}) of {inst['name']} "
                      f"from J_N, FP64, {evals:.3e} evaluations in {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="realistic", choices=sorted(DESCR))
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for {args.gpus}); "
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
    inst = instances.make(args.workload)
    print(f"[bench] workload {DESCR[args.workload]}", file=sys.stderr, flush=True)
    plan = Plan([inst], store_all=True, timing=True)
    evals = plan.evaluations()
    info = plan.info[0]
    evals_per_stage = int(info.slab_elems) * int(info.n_u)

    def step():
        plan.solve()
        plan.rollout()
        plan.adjoint()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.sweep_time()                       # discard warm-up sweep events

    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q in range(args.steps):
        ev[q][0].record(stream)
        plan.solve()
        ev[q][1].record(stream)
        plan.rollout()
        plan.adjoint()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sweep_ms, launches = plan.sweep_time()
    solve_ms = [a.elapsed_time(b) for a, b in ev]
    ms_per_step = wall * 1e3 / args.steps
    V0 = float(plan.V0.cpu()[0])

    avg_launch_ms = sweep_ms / max(1, launches)
    achieved = FLOPS_PER_EVAL * evals_per_stage / (avg_launch_ms * 1e-3) / 1e12
    out = {
        "metric": "state-control evals/s and full-horizon solve ms (FP32 vs FP64 oracle, 1e-4 rel V_0)",
        "value": evals / (ms_per_step * 1e-3),
        "unit": "state-control evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": DESCR[args.workload], "evaluations_per_solve": evals,
                   "step": "dp_solve + dp_rollout + dp_adjoint"},
        "solve_ms": {"mean": statistics.mean(solve_ms),
                     "var": statistics.pvariance(solve_ms) if len(solve_ms) > 1 else 0.0,
                     "max": max(solve_ms), "median": statistics.median(solve_ms)},
        "solve_evals_per_s": evals / (statistics.mean(solve_ms) * 1e-3),
        "V0": V0,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_PEAK_TFLOPS, "traffic": None,
                     "kernel": "state sweep", "avg_launch_ms": avg_launch_ms, "launches": launches,
                     "flops_per_launch": FLOPS_PER_EVAL * evals_per_stage},
    }
    gold = os.path.join(ROOT, "tests", "golden", f"{args.workload}_oracle.json")
    if os.path.exists(gold):
        with open(gold) as f:
            g = json.load(f)
        out["V0_rel_err_vs_oracle"] = abs(V0 - g["V0"]) / abs(g["V0"])
    if not args.no_cpu_baseline:
        print("[bench] oracle CPU baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_budget)
        out["cpu_baseline"]["host"] = platform.processor() or platform.machine()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
