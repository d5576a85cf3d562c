"""Summaries of rocprofv3 output.

  python -m paper_2104_01284_amd.profiling trace <run_results.db>
      per-kernel table of a kernel trace: calls, total/avg/min/max duration,
      register and LDS use, launch shape;
  python -m paper_2104_01284_amd.profiling pmc <run_results.db> [kernel-substring]
      per-kernel average of every collected counter (per dispatch).
"""
import sqlite3
import sys


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


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(sys.argv[2], " ".join(sys.argv[3:]))
    elif sys.argv[1] == "pmc":
        pmc(sys.argv[2], sys.argv[3] if len(sys.argv) > 3 else "")
    else:
        trace(sys.argv[1])
