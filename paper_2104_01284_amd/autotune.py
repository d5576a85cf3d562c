"""Autotuner of the grouped state sweep.

For one problem shape it times the candidate sweep configurations (SoC rows
per workgroup of the grouped sweep) on a few stages of the instance and
keeps the fastest.  The number of control slices stays with the
library, which picks it per round of a batch.  Results are cached per
(device, shape) in a JSON file, so a shape is timed once per machine.

  opts = tuned_options(instances)          # one (kernel, tile, split, wg) per instance
  plan = Plan(instances, inst_opts=opts)
"""
from __future__ import annotations

import json
import os
import sys

# (kernel, SoC rows per workgroup) of the grouped sweep
CANDIDATES = ((2, 16), (2, 8), (2, 4))


def default_cache_path() -> str:
    return os.environ.get("ECODP_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "ecodp", "sweep_tune.json"))


def shape_key(inst: dict, device_name: str) -> str:
    n_v, n_s, n_t = (int(inst[g][2]) for g in ("v_grid", "soc_grid", "t_grid"))
    n_u = int(inst["te_grid"][2]) * int(inst["tm_grid"][2])
    return f"{device_name}|v{n_v}|s{n_s}|t{n_t}|u{n_u}|N{int(inst['N'])}"


def _time_config(inst, kernel, tile, stages, repeats, device, full):
    """Milliseconds of one configuration: a whole solve (full) or the sweep
    launches of the isolated stages `stages` from a zero J_{k+1} (timing does
    not depend on the values)."""
    import torch
    from .api import Plan
    plan = Plan([inst], timing=True, kernel=kernel, sweep_tile=tile, device=device)
    info = plan.info[0]
    if int(info.sweep_kernel) != kernel or int(info.sweep_tile) != tile:
        return None
    if full:
        # whole solves: the stage tables of the next round run beside the
        # sweep, so the solve time (not the sweep launches alone) decides
        plan.solve()                                  # warm-up
        torch.cuda.synchronize(device)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(repeats):
            plan.solve()
        b.record()
        torch.cuda.synchronize(device)
        return a.elapsed_time(b) / repeats
    Jn = torch.zeros(plan.slab_shape(0), dtype=torch.float32, device=f"cuda:{device}")
    for k in stages:                                  # warm-up
        plan.stage(0, k, Jn)
    torch.cuda.synchronize(device)
    plan.sweep_time()
    for _ in range(repeats):
        for k in stages:
            plan.stage(0, k, Jn)
    torch.cuda.synchronize(device)
    ms, _ = plan.sweep_time()
    return ms / repeats


def tune(inst: dict, device: int = 0, repeats: int = 2, candidates=CANDIDATES, full: bool = False) -> dict:
    """Time every candidate on `inst`: its whole solve when `full`, else three
    of its stages.  Returns the fastest as {"kernel", "tile", "ms", "all"}."""
    N = int(inst["N"])
    stages = sorted({N - 1, N // 2, min(1, N - 1)})
    n_s = int(inst["soc_grid"][2])
    results = {}
    for kernel, tile in candidates:
        if tile > n_s and tile > 4:
            continue
        r = _time_config(inst, kernel, tile, stages, repeats, device, full)
        if r is not None:
            results[f"{kernel}/{tile}"] = r
    if not results:
        return {"kernel": 0, "tile": 0, "ms": None, "all": {}}
    best = min(results, key=results.get)
    kernel, tile = (int(x) for x in best.split("/"))
    return {"kernel": kernel, "tile": tile, "ms": results[best], "all": results}


def tuned_options(instances, device: int = 0, cache_path: str | None = None, verbose: bool = False,
                  full: bool | None = None):
    """Per-instance (kernel, tile, split, wg_per_cu) for Plan(inst_opts=...),
    timing each shape not yet in the cache: by whole solves for a single
    instance (unless `full` is False), by sampled stages for a batch."""
    if full is None:
        full = len(instances) == 1
    import torch
    path = cache_path or default_cache_path()
    cache = {}
    if os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    name = torch.cuda.get_device_name(device)
    out, dirty = [], False
    for inst in instances:
        key = shape_key(inst, name)
        if key not in cache:
            cache[key] = tune(inst, device, full=full)
            dirty = True
            if verbose:
                print(f"[autotune] {key}: {cache[key]}", file=sys.stderr, flush=True)
        c = cache[key]
        out.append((int(c["kernel"]), int(c["tile"]), 0, 0))
    if dirty:
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            tmp = path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
            os.replace(tmp, path)
        except OSError:
            pass
    return out


# SoC tiles a batch is timed with (one tile for every instance, so that the
# persistent sweep runs one kernel class per workgroup size)
BATCH_TILES = (8, 4)


def batch_key(instances, device_name: str) -> str:
    import hashlib
    shapes = "|".join(shape_key(inst, "") for inst in instances)
    return f"{device_name}|batch{len(instances)}|{hashlib.sha256(shapes.encode()).hexdigest()[:16]}"


def tune_batch(instances, device: int = 0, tiles=BATCH_TILES, repeats: int = 2) -> dict:
    """Whole solves of the batch with every instance on one SoC tile, replayed
    as recorded graphs the way a batch is solved; after two untimed solves of
    every candidate, the candidates are timed in turn `repeats` times and each
    keeps its fastest solve (so that clock ramp-up or a one-off stall does not
    land on whichever candidate happens to run first).  Returns the fastest
    as {"tile", "ms", "all"}."""
    import torch
    from .api import Plan
    plans = {t: Plan(instances, sweep_tile=t, graph=True, device=device) for t in tiles}
    for plan in plans.values():
        for _ in range(2):
            plan.solve()
    torch.cuda.synchronize(device)
    results = {}
    for _ in range(repeats):
        for t, plan in plans.items():
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            plan.solve()
            b.record()
            torch.cuda.synchronize(device)
            ms = a.elapsed_time(b)
            results[str(t)] = min(ms, results.get(str(t), ms))
    del plans
    torch.cuda.empty_cache()
    best = min(results, key=results.get)
    return {"tile": int(best), "ms": results[best], "all": results}


def tuned_batch_options(instances, device: int = 0, cache_path: str | None = None, verbose: bool = False):
    """Per-instance options of a batch: the SoC tile whose whole-batch solve
    was fastest (timed once per (device, batch of shapes), then cached)."""
    import torch
    path = cache_path or default_cache_path()
    cache = {}
    if os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    key = batch_key(instances, torch.cuda.get_device_name(device))
    if key not in cache:
        cache[key] = tune_batch(instances, device)
        if verbose:
            print(f"[autotune] {key}: {cache[key]}", file=sys.stderr, flush=True)
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            tmp = path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
            os.replace(tmp, path)
        except OSError:
            pass
    tile = int(cache[key]["tile"])
    return [(0, tile, 0, 0)] * len(instances)
