"""Write the stored oracle values used by the GPU parity tests at full size.

Calls only the FP64 oracle and the seeded instance generator.  Run from the
repository root:  python tests/golden/make_golden.py [realistic]
The 2 km instance takes several minutes on 8 host cores.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2104_01284_amd import instances as ins  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def instance_digest(inst):
    h = hashlib.sha256()
    for k in sorted(inst):
        v = inst[k]
        if isinstance(v, np.ndarray):
            h.update(k.encode() + v.tobytes())
        else:
            h.update(k.encode() + repr(v).encode())
    return h.hexdigest()[:16]


def make(name, stages_to_sample=(0, 1, 50, 100, 150, 199), per_stage=256, seed=123):
    inst = ins.make(name)
    t = time.time()
    r = oracle.solve(inst, q2=True)
    dt = time.time() - t
    ro = oracle.rollout(inst, r["pi"], r["u0"])
    rng = np.random.default_rng(seed)
    nv, ns, nt = inst["v_grid"][2], inst["soc_grid"][2], inst["t_grid"][2]
    samples = []
    for k in stages_to_sample:
        if k >= inst["N"]:
            continue
        for _ in range(per_stage):
            i, j, m = int(rng.integers(0, nv)), int(rng.integers(0, ns)), int(rng.integers(0, nt))
            samples.append([k, i, j, m, float(r["J"][k, i, j, m]), int(r["pi"][k, i, j, m]),
                            float(r["q2"][k, i, j, m])])
    out = {
        "source": "oracle.solve (FP64) on paper_2104_01284_amd.instances." + name,
        "instance": inst["name"], "digest": instance_digest(inst),
        "V0": r["V0"], "u0": r["u0"],
        "J_inf": ins.J_INF,
        "rollout": {"status": ro["status"], "violations": ro["violations"],
                    "fuel_g": float(ro["traj"][-1, 6]), "time_s": float(ro["traj"][-1, 2]),
                    "cost": float(ro["traj"][-1, 7])},
        "oracle_seconds": dt, "oracle_threads": oracle.num_threads(),
        "evaluations": ins.evaluations(inst),
        "samples": samples,
    }
    path = os.path.join(HERE, f"{name}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path}: V0={r['V0']:.6f} u0={r['u0']} in {dt:.1f}s")


if __name__ == "__main__":
    for name in (sys.argv[1:] or ["realistic"]):
        make(name)
