"""Write the stored oracle values used by the GPU parity tests at full size.

Calls only the FP64 oracle and the seeded instance generator.  Run from the
repository root:  python tests/golden/make_golden.py [realistic] [large] [batched]
The 2 km instance takes about ten minutes on 6 host threads, the 3 km one
(1.7e12 evaluations, about 20 GB of host memory for the stored values and
policy) about two hours.

Each file holds, for the named instance:
  * the instance digest (instance_digest below), which the tests and the
    benchmark check before using any stored value;
  * V_0 and u_0* (Eq. 6), the FP64 rollout totals of the oracle's own policy
    and the oracle's fixed-policy gradient dV_0/dtheta on its own solve;
  * sampled nodes (k, i, j, m) of a few stages with J_k, pi_k, the
    second-best candidate value q2 and the near-tie list: every control whose
    FP64 candidate value lies within NEAR_TIE max(1, |J_k|) of the best, as
    (u, Q) pairs, so the FP64 regret of any admissible choice there can be
    read off without the oracle.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from paper_2104_01284_amd import instances as ins  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
NEAR_TIE = 1e-3

STAGES = {
    "realistic": (0, 1, 50, 100, 150, 199),
    "large": (0, 1, 75, 150, 225, 299),
}


def instance_digest(inst):
    return ins.digest(inst)


def near_ties(I, k, Jn, i, j, m, J, n_u):
    """Controls whose FP64 candidate is within NEAR_TIE max(1, |J|) of the best."""
    import oracle
    if J >= ins.J_INF:
        return []
    lim = J + NEAR_TIE * max(1.0, abs(J))
    out = []
    for u in list(range(n_u)) + [-2]:
        q = oracle.node_q(I, k, Jn, i, j, m, u)
        if q <= lim:
            out.append([u, q])
    return out


def make(name, per_stage=256, seed=123):
    import oracle
    inst = ins.make(name)
    I = oracle.Instance(inst)
    t = time.time()
    r = oracle.solve(I)
    dt = time.time() - t
    print(f"{name}: solve {dt:.1f} s, V0={r['V0']:.9f} u0={r['u0']}", flush=True)
    ro = oracle.rollout(I, r["pi"], r["u0"])
    ad = oracle.adjoint(I, r["J"], r["pi"], r["u0"])
    rng = np.random.default_rng(seed)
    nv, ns, nt = I.shape
    samples = []
    for k in STAGES[name]:
        if k >= inst["N"]:
            continue
        Jn = r["J"][k + 1]
        for _ in range(per_stage):
            i, j, m = int(rng.integers(0, nv)), int(rng.integers(0, ns)), int(rng.integers(0, nt))
            J, pi, q2 = oracle.node(I, k, Jn, i, j, m)
            assert J == r["J"][k, i, j, m] and pi == r["pi"][k, i, j, m]
            samples.append([k, i, j, m, J, pi, q2, near_ties(I, k, Jn, i, j, m, J, I.n_u)])
    out = {
        "source": "oracle.solve (FP64) on paper_2104_01284_amd.instances." + name,
        "instance": inst["name"], "digest": instance_digest(inst),
        "V0": r["V0"], "u0": r["u0"],
        "J_inf": ins.J_INF,
        "rollout": {"status": ro["status"], "violations": ro["violations"],
                    "fuel_g": float(ro["traj"][-1, 6]), "time_s": float(ro["traj"][-1, 2]),
                    "cost": float(ro["traj"][-1, 7])},
        "grad": [float(x) for x in ad["grad"]],
        "oracle_seconds": dt, "oracle_threads": oracle.num_threads(),
        "evaluations": ins.evaluations(inst),
        "near_tie": NEAR_TIE,
        "sample_fields": ["k", "i", "j", "m", "J", "pi", "q2", "near_ties [[u, Q64], ...]"],
        "samples": samples,
    }
    path = os.path.join(HERE, f"{name}_oracle.json")
    with open(path + ".tmp", "w") as f:
        json.dump(out, f, indent=0)
    os.replace(path + ".tmp", path)
    print(f"wrote {path}: V0={r['V0']:.6f} u0={r['u0']} in {dt:.1f}s", flush=True)


def batch_subset(n=256):
    """Stratified members of the 256-instance batch: the smallest and the
    largest by evaluations, and every 16th."""
    work = sorted((ins.evaluations(ins.batched_member(b)), b) for b in range(n))
    return sorted({work[0][1], work[-1][1]} | set(range(0, n, 16)))


def make_batched():
    """V_0, u_0* and the second-best root candidate of the stratified batch
    members (FP64 oracle)."""
    import oracle
    rows = []
    t = time.time()
    for b in batch_subset():
        inst = ins.batched_member(b)
        r = oracle.solve(inst)
        # the second-best root candidate: where it is within the FP32
        # tolerance of V_0, another u_0 is an admissible answer
        _, _, q2 = oracle.root(inst, r["J"][1])
        rows.append({"member": b, "instance": inst["name"], "digest": instance_digest(inst),
                     "V0": r["V0"], "u0": r["u0"], "q2_root": q2, "evaluations": ins.evaluations(inst)})
        print(f"batched member {b}: V0={r['V0']:.9f} u0={r['u0']} q2={q2:.9f}", flush=True)
        del r
    out = {"source": "oracle.solve (FP64) on paper_2104_01284_amd.instances.batched_member(b)",
           "members": rows, "oracle_seconds": time.time() - t, "oracle_threads": oracle.num_threads()}
    path = os.path.join(HERE, "batched_oracle.json")
    with open(path + ".tmp", "w") as f:
        json.dump(out, f, indent=1)
    os.replace(path + ".tmp", path)
    print(f"wrote {path}", flush=True)


def load(name):
    """The stored file for instance `name` if its digest matches today's
    generator, else None (reads JSON only)."""
    path = os.path.join(HERE, f"{name}_oracle.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        g = json.load(f)
    if g.get("digest") != instance_digest(ins.make(name)):
        return None
    return g


if __name__ == "__main__":
    for name in (sys.argv[1:] or ["realistic"]):
        if name == "batched":
            make_batched()
        else:
            make(name)
