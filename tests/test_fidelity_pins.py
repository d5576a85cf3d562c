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


def test_yellow_rule_closed_form():
    """Three-phase signal (Sec. III): at the signal stage a node in yellow
    (phase x in [C - Y, C)) must stop, as in red, exactly when the time since
    yellow began exceeds v / (2 b), b = -a_min: the vehicle was farther from
    the stop line than its critical braking distance v^2 / (2 b) when yellow
    began; otherwise yellow is green and the node keeps the two-phase value.
    A vehicle at rest in yellow waits until green, C - x + R, its value w_t tau
    plus the next stage lerped at t_m + tau.  Red nodes and every other stage
    are unchanged; a zero yellow reproduces the two-phase solve exactly."""
    import math
    base = ins.plain()
    inst = ins.with_yellow(base, 8.0)
    r0 = oracle.solve(base)
    r = oracle.solve(inst)
    k, C, R, O, Y = inst["lights"][0]
    b = -inst["konst"][10]
    Jinf = inst["konst"][13]
    wt = inst["theta"][3]
    v = np.linspace(*inst["v_grid"][:2], inst["v_grid"][2])
    t = np.linspace(*inst["t_grid"][:2], inst["t_grid"][2])
    ht = t[1] - t[0]
    nt = len(t)
    assert np.array_equal(r["J"][k + 1:], r0["J"][k + 1:])
    blocked = green = 0
    for m in range(nt):
        x = (inst["t0_abs"] + t[m] - O) % C
        if x < R or x < C - Y:
            assert np.array_equal(r["J"][k, :, :, m], r0["J"][k, :, :, m]), m
            continue
        since = x - (C - Y)
        for i in range(len(v)):
            if v[i] > 0.0 and since > v[i] / (2.0 * b):
                blocked += 1
                assert np.all(r["J"][k, i, :, m] == Jinf) and np.all(r["pi"][k, i, :, m] == -1), (m, i)
            elif v[i] > 0.0:
                green += 1
                assert np.array_equal(r["J"][k, i, :, m], r0["J"][k, i, :, m]), (m, i)
            else:
                tau = (C - x) + R
                rt = m + tau / ht
                for j in range(inst["soc_grid"][2]):
                    if rt > nt - 1:
                        assert r["J"][k, 0, j, m] == Jinf
                        continue
                    c = min(int(math.floor(rt)), nt - 2)
                    f = rt - c
                    want = wt * tau + (1 - f) * r["J"][k + 1, 0, j, c] + f * r["J"][k + 1, 0, j, c + 1]
                    assert r["J"][k, 0, j, m] == min(want, Jinf) or abs(r["J"][k, 0, j, m] - want) <= 1e-12 * want
    assert blocked > 20 and green > 20
    same = oracle.solve(ins.with_yellow(base, 0.0))
    assert np.array_equal(same["J"], r0["J"]) and np.array_equal(same["pi"], r0["pi"])


def test_red_wait_in_yellow():
    """The closed loop's stop-line wait: to the end of red in red; in yellow,
    for a vehicle at rest, to the end of the red that follows."""
    inst = ins.with_yellow(ins.plain(), 8.0)
    k, C, R, O, Y = inst["lights"][0]
    assert oracle.red_wait(inst, k, O + 5.0) == R - 5.0          # red
    assert oracle.red_wait(inst, k, O + 30.0) == 0.0              # green
    x = C - Y + 3.0                                              # 3 s into yellow
    assert oracle.red_wait(inst, k, O + x) == (C - x) + R
    assert oracle.red_wait(inst, k, O + C - Y) == 0.0             # the instant yellow begins
