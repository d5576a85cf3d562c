"""Summaries of rocprofv3 output.

  python -m paper_2104_01284_amd.profiling trace <run_results.db>
      per-kernel table of a kernel trace: calls, total/avg/min/max duration,
      register and LDS use, launch shape;
  python -m paper_2104_01284_amd.profiling pmc <run_results.db> [kernel-substring]
      per-kernel average of every collected counter (per dispatch).
  python -m paper_2104_01284_amd.profiling traffic <fetch.db> <write.db> <copy_fetch.db> <copy_write.db>
                                                   <copy_MiB> <kernel-substring>
      HBM bytes per dispatch of a kernel from FETCH_SIZE and WRITE_SIZE (KiB
      per dispatch), each scaled by what the same counter reads for a plain
      device copy of copy_MiB MiB; prints a summary whose last line is
      machine-readable.

It also reads the stored FP64 oracle results of the parity goldens
(load_golden, golden_report) for the per-result errors the benchmark reports.
"""
import hashlib
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def trace(path, title=""):
    db = sqlite3.connect(path)
    rows = db.execute(
        "select name, count(*), sum(duration), avg(duration), min(duration), max(duration), "
        "max(vgpr_count), max(accum_vgpr_count), max(sgpr_count), max(lds_size), max(scratch_size), "
        "max(workgroup_x), max(grid_x), max(grid_y) "
        "from kernels group by name order by sum(duration) desc").fetchall()
    total = sum(r[2] for r in rows)
    if title:
        print(title)
    print(f"{'kernel':60s} {'calls':>6s} {'total_ms':>10s} {'pct':>6s} {'avg_us':>10s} {'min_us':>10s} "
          f"{'max_us':>10s} {'vgpr':>5s} {'agpr':>5s} {'sgpr':>5s} {'lds':>6s} {'scr':>5s} {'wg':>5s} {'grid':>12s}")
    for r in rows:
        name = r[0].split("(")[0][:60]
        print(f"{name:60s} {r[1]:6d} {r[2] / 1e6:10.3f} {100.0 * r[2] / total:6.2f} {r[3] / 1e3:10.2f} "
              f"{r[4] / 1e3:10.2f} {r[5] / 1e3:10.2f} {r[6]:5d} {r[7]:5d} {r[8]:5d} {r[9]:6d} {r[10]:5d} "
              f"{r[11]:5d} {str(r[12]) + 'x' + str(r[13]):>12s}")


def pmc(path, needle=""):
    db = sqlite3.connect(path)
    tabs = [r[0] for r in db.execute("select name from sqlite_master where type in ('table','view')")]
    if "counters_collection" in tabs:
        rows = db.execute("select kernel_name, counter_name, count(*), avg(value), sum(value) "
                          "from counters_collection group by kernel_name, counter_name").fetchall()
    else:
        rows = db.execute(
            "select k.name, p.counter_name, count(*), avg(p.value), sum(p.value) from pmc_events p "
            "join kernels k on k.dispatch_id = p.dispatch_id group by k.name, p.counter_name").fetchall()
    for name, cn, cnt, avg, tot in sorted(rows):
        if needle and needle not in name:
            continue
        print(f"{name.split('(')[0][:50]:50s} {cn:28s} dispatches={cnt:6d} avg={avg:16.1f} total={tot:18.1f}")


def _counter_rows(path, counter):
    db = sqlite3.connect(path)
    tabs = [r[0] for r in db.execute("select name from sqlite_master where type in ('table','view')")]
    if "counters_collection" in tabs:
        q = ("select kernel_name, avg(value), count(*) from counters_collection where counter_name = ? "
             "group by kernel_name")
    else:
        q = ("select k.name, avg(p.value), count(*) from pmc_events p join kernels k "
             "on k.dispatch_id = p.dispatch_id where p.counter_name = ? group by k.name")
    return db.execute(q, (counter,)).fetchall()


def sweep_source_hash():
    """SHA-256 of the grouped-sweep source; a stored traffic figure is valid
    only for the kernel it was measured on."""
    with open(os.path.join(HERE, "csrc", "dp_sweep.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic(fetch_db, write_db, copy_fetch_db, copy_write_db, copy_mib, needle, split="?"):
    """Copy-calibrated HBM bytes per launch of the kernels matching `needle`;
    `split` is the number of control slices of the profiled run (the byte
    count depends on it)."""
    copy_kib = float(copy_mib) * 1024.0

    def copy_factor(db, counter):
        rows = [r for r in _counter_rows(db, counter) if "opy" in r[0] or "elementwise" in r[0]]
        big = max(rows, key=lambda r: r[1])
        return copy_kib / big[1], big

    ff, frow = copy_factor(copy_fetch_db, "FETCH_SIZE")
    fw, wrow = copy_factor(copy_write_db, "WRITE_SIZE")
    f = [r for r in _counter_rows(fetch_db, "FETCH_SIZE") if needle in r[0]]
    w = [r for r in _counter_rows(write_db, "WRITE_SIZE") if needle in r[0]]
    print(f"copy calibration ({copy_mib} MiB): FETCH_SIZE {frow[1]:.1f} KiB -> factor {ff:.3f}; "
          f"WRITE_SIZE {wrow[1]:.1f} KiB -> factor {fw:.3f}  [{frow[0].split('(')[0][:60]}]")
    tot = 0.0
    for (name, fk, n) in f:
        wk = dict((r[0], r[1]) for r in w).get(name, 0.0)
        b = (fk * ff + wk * fw) * 1024.0
        tot = max(tot, b)
        print(f"{name.split('(')[0][:60]:60s} dispatches={n:5d} FETCH={fk:12.1f} KiB WRITE={wk:12.1f} KiB "
              f"-> HBM bytes/dispatch {b:.4e}")
    print(f"traffic_bytes_per_launch={tot:.6e} sweep_source={sweep_source_hash()} split={split}")


GOLDEN_DIR = os.path.join(os.path.dirname(HERE), "tests", "golden")


def load_golden(name, inst):
    """Stored FP64 oracle results of workload `name` (written by
    tests/golden/make_golden.py), or None when there are none or their
    instance digest differs from `inst`'s (stale for today's generator)."""
    import json
    from . import instances
    path = os.path.join(GOLDEN_DIR, f"{name}_oracle.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        g = json.load(f)
    return g if g.get("digest") == instances.digest(inst) else None


def batch_golden_report(insts, V0, u0):
    """V_0 and u_0 of the batch members with stored FP64 oracle results
    (tests/golden/batched_oracle.json, each member digest-checked against
    `insts`) against those results; None when the file is missing."""
    import json
    from . import instances
    path = os.path.join(GOLDEN_DIR, "batched_oracle.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        g = json.load(f)
    errs, mism, stale = [], 0, 0
    for m in g["members"]:
        b = int(m["member"])
        if b >= len(insts) or instances.digest(insts[b]) != m["digest"]:
            stale += 1
            continue
        errs.append(abs(float(V0[b]) - m["V0"]) / abs(m["V0"]))
        mism += int(int(u0[b]) != int(m["u0"]))
    return {"members": len(errs), "stale_members": stale,
            "V0_max_rel_err": max(errs) if errs else None, "u0_mismatch": mism}


def _rel(a, b):
    return abs(a - b) / max(1.0, abs(b))


def golden_report(g, V0, J_all=None, pi_all=None, traj=None, grad=None, band=1e-4):
    """Errors of one solve's results against stored FP64 oracle results `g`.

    V0: the solve's V_0.  J_all [N+1, n_v, n_soc, n_t] and pi_all [N, ...]:
    its stored values and policy (device tensors), compared at the stored
    sample nodes: J relative error (to max(1, |J_64|)); policy mismatches,
    counted all together, where the FP64 gap between the best and second-best
    candidate is at least 1e-6 (the absolute reading) or 1e-6 max(1, |J_64|)
    (the relative reading) or `band` max(1, |J_64|); and the FP64 regret
    Q_64(u) - J_64 of every mismatching choice u from the stored near-tie
    list (a choice outside it regrets more than the list's bound).  traj:
    the rollout rows [N+1, 8] (fuel and time of the last row against the
    oracle's rollout of its own policy); grad: dV_0/dtheta [5] against the
    oracle's adjoint on its own solve."""
    out = {"V0_rel_err": abs(float(V0) - g["V0"]) / abs(g["V0"])}
    if J_all is not None and g.get("samples"):
        import torch
        s = g["samples"]
        idx = [torch.as_tensor([row[q] for row in s], device=J_all.device) for q in range(4)]
        Jg = J_all[idx[0], idx[1], idx[2], idx[3]].double().cpu().tolist()
        pg = pi_all[idx[0], idx[1], idx[2], idx[3]].cpu().tolist()
        jerr = 0.0
        mism = lit = relr = inband = beyond = 0
        regret = regret_rel = 0.0
        lim = g.get("near_tie", 1e-3)
        for row, Jv, pv in zip(s, Jg, pg):
            _, _, _, _, J64, p64, q2, ties = row
            jerr = max(jerr, _rel(Jv, J64))
            if pv == p64:
                continue
            mism += 1
            gap = q2 - J64
            sc = max(1.0, abs(J64))
            lit += gap >= 1e-6
            relr += gap >= 1e-6 * sc
            inband += gap >= band * sc
            q = dict((u, Q) for u, Q in ties).get(pv)
            if q is None:
                beyond += 1
                regret_rel = max(regret_rel, lim)
            else:
                regret = max(regret, q - J64)
                regret_rel = max(regret_rel, (q - J64) / sc)
        out["samples"] = {"nodes": len(s), "J_max_rel_err": jerr, "policy_mismatch": mism,
                          "mismatch_gap_ge_1e-6_abs": lit, "mismatch_gap_ge_1e-6_rel": relr,
                          f"mismatch_gap_ge_{band:g}_rel": inband, "choice_outside_near_tie_list": beyond,
                          "max_regret": regret, "max_regret_rel": regret_rel}
    if traj is not None and "rollout" in g:
        t = traj[-1].double().cpu().tolist()
        r = g["rollout"]
        out["rollout"] = {"fuel_rel_err": abs(t[6] - r["fuel_g"]) / abs(r["fuel_g"]),
                          "time_rel_err": abs(t[2] - r["time_s"]) / abs(r["time_s"]),
                          "cost_rel_err": abs(t[7] - r["cost"]) / abs(r["cost"])}
    if grad is not None and "grad" in g:
        gg = [float(x) for x in grad]
        out["grad_rel_err"] = [abs(a - b) / abs(b) if b else abs(a) for a, b in zip(gg, g["grad"])]
    return out


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(sys.argv[2], " ".join(sys.argv[3:]))
    elif sys.argv[1] == "pmc":
        pmc(sys.argv[2], sys.argv[3] if len(sys.argv) > 3 else "")
    elif sys.argv[1] == "traffic":
        traffic(*sys.argv[2:9])
    else:
        trace(sys.argv[1])
