"""Model-fidelity variants of the oracle (CPU): the speed-dependent torque
limits of Eq. 7e-f as power caps, and stop signs as a zero route speed limit
(Eq. 7a), pinned against closed forms."""
import numpy as np

import oracle
from paper_2104_01284_amd import instances as ins

ST_TORQUE = 16


def test_power_caps_closed_form():
    base = ins.plain()
    inst = ins.with_torque_limits(base, 20000.0, 8000.0)
    rw, ig = inst["konst"][2], inst["konst"][3]
    v = 20.0
    w = v * ig / rw                                   # crank speed, 200 rad/s
    te = np.linspace(*inst["te_grid"][:2], inst["te_grid"][2])
    tm = np.linspace(*inst["tm_grid"][:2], inst["tm_grid"][2])
    for a in range(len(te)):
        for b in range(len(tm)):
            st, _ = oracle.transition(inst, 0, v, 0.55, a, b)
            over = te[a] * w > 20000.0 or abs(tm[b]) * w > 8000.0
            assert bool(st & ST_TORQUE) == over, (a, b, te[a], tm[b])
    # at low speed the caps do not bind on the control grid
    for a in range(len(te)):
        for b in range(len(tm)):
            st, _ = oracle.transition(inst, 0, 4.0, 0.55, a, b)
            assert not st & ST_TORQUE


def test_zero_caps_change_nothing():
    base = ins.plain()
    same = ins.with_torque_limits(base, 0.0, 0.0)
    for v in (0.0, 3.0, 12.5, 20.0):
        for a in (0, 5, 10):
            for b in (0, 4, 10):
                s0, o0 = oracle.transition(base, 3, v, 0.5, a, b)
                s1, o1 = oracle.transition(same, 3, v, 0.5, a, b)
                assert s0 == s1
                assert np.array_equal(list(o0.values()), list(o1.values()), equal_nan=True)
    assert oracle.solve(base)["V0"] == oracle.solve(same)["V0"]


def test_stop_sign_forces_rest():
    inst = ins.plain_fidelity()
    k = inst["stop_signs"][0]
    r = oracle.solve(inst)
    Jinf = inst["konst"][13]
    assert np.all(r["J"][k][1:] == Jinf)              # every moving node at the sign is infeasible
    assert np.any(r["J"][k][0] < Jinf)
    ro = oracle.rollout(inst, r["pi"], r["u0"])
    assert ro["status"] == 0
    assert ro["traj"][k, 0] == 0.0                     # the vehicle is at rest at the sign
    assert ro["traj"][k + 1, 0] > 0.0                  # and leaves it
    # the controls of the rollout respect the caps at their step's speed
    rw, ig = inst["konst"][2], inst["konst"][3]
    for row in ro["traj"][:-1]:
        if row[3] >= 0:
            w = row[0] * ig / rw
            assert row[4] * w <= 20000.0 + 1e-9 and abs(row[5]) * w <= 8000.0 + 1e-9
    # the sign costs time: the unconstrained instance is at least as cheap
    free = oracle.solve(ins.plain())
    assert free["V0"] <= r["V0"]
