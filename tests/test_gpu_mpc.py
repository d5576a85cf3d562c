"""GPU: the receding-horizon state update (dp_set_state).

Moving x0 and the signal clock on an existing plan must give exactly the
solve of a plan built for the moved instance (same FP64 signal tables, same
kernels), in eager mode and on the replay of a recorded solve; the rollout
follows the moved state."""
import sys

import numpy as np
import pytest

import oracle
from paper_2104_01284_amd import instances as ins

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-mpc]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    return T


def Plan(*a, **k):
    from paper_2104_01284_amd.api import Plan as P
    return P(*a, **k)


def moved(inst, v0, soc0, t0):
    x = dict(inst)
    x["v0"], x["soc0"], x["t0_abs"] = v0, soc0, t0
    return x


CASES = [
    (ins.plain, (7.3, 0.61, 23.5)),
    (lambda: ins.tiny(seed=301, N=9, n_v=9, n_s=7, n_t=67, n_e=5, n_m=5, light=True, t_f=90.0), (3.1, 0.47, 41.0)),
]


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_set_state_equals_fresh_plan(torch, case, graph):
    make, (v0, soc0, t0) = CASES[case]
    inst = make()
    plan = Plan([inst], store_all=not graph, graph=graph)
    plan.solve()
    torch.cuda.synchronize()
    say(inst["name"], "graph", graph, "move to", v0, soc0, t0)
    plan.set_state(0, v0, soc0, t0)
    V0, u0 = plan.solve()
    torch.cuda.synchronize()
    fresh = Plan([moved(inst, v0, soc0, t0)], store_all=not graph)
    Vf, uf = fresh.solve()
    torch.cuda.synchronize()
    assert float(V0[0]) == float(Vf[0]) and int(u0[0]) == int(uf[0])
    assert torch.equal(plan.policy(0), fresh.policy(0))
    if not graph:
        assert torch.equal(plan.values(0), fresh.values(0))
    r = oracle.solve(moved(inst, v0, soc0, t0))
    assert abs(float(V0[0]) - r["V0"]) <= 1e-4 * abs(r["V0"])


def test_rollout_follows_moved_state(torch):
    """After dp_set_state the rollout starts from the moved state: with the
    oracle's solve of the moved instance loaded into the plan, the GPU
    rollout equals the oracle's."""
    inst = ins.plain()
    plan = Plan([inst], store_all=True)
    plan.solve()
    plan.set_state(0, 8.2, 0.52, 11.0)
    plan.solve()
    r = oracle.solve(moved(inst, 8.2, 0.52, 11.0))
    plan.policy(0).copy_(torch.from_numpy(r["pi"]).cuda())
    plan.u0.fill_(int(r["u0"]))
    trajs, status = plan.rollout()
    torch.cuda.synchronize()
    ro = oracle.rollout(moved(inst, 8.2, 0.52, 11.0), r["pi"], r["u0"])
    st = status.cpu().numpy()[0]
    assert st[0] == ro["status"] and st[1] == ro["violations"]
    tg = trajs[0].cpu().numpy()
    both = np.isfinite(ro["traj"])
    np.testing.assert_allclose(tg[both], ro["traj"][both], rtol=1e-9, atol=1e-9)


def test_set_state_rejects_outside_grid(torch):
    from paper_2104_01284_amd import _lib as L
    plan = Plan([ins.plain()])
    with pytest.raises(L.DPError):
        plan.set_state(0, 5.0, 0.95, 0.0)
    with pytest.raises(L.DPError):
        plan.set_state(0, float("nan"), 0.5, 0.0)
    assert plan.lib.dp_set_state(plan._h, 3, 5.0, 0.5, 0.0, None) == L.DP_EINVAL


# ------------------------------------------------- closed loop (Sec. V) --

def test_terminal_from_values_matches_oracle(torch):
    """The horizon's terminal table from a full-route value slab (Sec. III
    after Eq. 9): the kernel against the oracle's interpolation on the same
    seeded FP32 slab, exactly after the one FP32 rounding."""
    from paper_2104_01284_amd.api import terminal_from_values
    rng = np.random.default_rng(77)
    n_v, n_s, n_src, t_f_src = 35, 26, 104, 211.3
    J = rng.uniform(0.0, 300.0, (n_v, n_s, n_src)).astype(np.float32)
    J[rng.random(J.shape) < 0.05] = 1.0e4          # some infeasible nodes
    for shift in (0.0, 37.7, 150.0, 230.0):
        say("terminal shift", shift)
        dev = terminal_from_values(torch.from_numpy(J).cuda(), t_f_src, shift, 40, 80.0, 1.0e4)
        torch.cuda.synchronize()
        ref = oracle.window_terminal(J.astype(np.float64), t_f_src, shift, 40, 80.0, 1.0e4).astype(np.float32)
        assert np.array_equal(dev.cpu().numpy(), ref), shift


def test_device_terminal_equals_host_terminal(torch):
    inst = ins.paper_shape()
    rng = np.random.default_rng(78)
    tv = rng.uniform(0.0, 40.0, (35, 26, 40)).astype(np.float32)
    a = dict(inst, terminal_V=tv)
    b = dict(inst, terminal_V=torch.from_numpy(tv).cuda())
    pa, pb = Plan([a], store_all=True), Plan([b], store_all=True)
    Va, _ = pa.solve()
    Vb, _ = pb.solve()
    torch.cuda.synchronize()
    assert float(Va[0]) == float(Vb[0])
    assert torch.equal(pa.values(0), pb.values(0)) and torch.equal(pa.policy(0), pb.policy(0))


@pytest.mark.parametrize("yellow", [0.0, 3.0])
def test_closed_loop_matches_oracle(torch, yellow):
    """Twelve steps of the receding-horizon controller on a 600 m route with
    the paper's horizon grid (two-phase signals, and three-phase with a 3 s
    yellow): the GPU loop (FP32 values, FP64 plant) and the oracle's loop
    (FP64 throughout), each with its own full-route DP for the terminal cost.
    Per step V_0 within 1e-4, the same u_0* (a differing choice must be a near
    tie at the root, after which the loops may part), and the plant states
    within 1e-9."""
    from paper_2104_01284_amd.mpc import ClosedLoop
    route = ins.mpc_route(seed=9, length_m=600.0, n_lights=2)
    if yellow:
        route = ins.with_yellow(route, yellow)
    steps = 12
    say("closed loop on", route["name"], "N", route["N"], "lights", route["lights"])
    loop = ClosedLoop(route).run(steps)
    ref = oracle.closed_loop(route, steps, ins.MPC_HORIZON, ins.MPC_T_F, ins.MPC_N_T, ins.mpc_window)
    assert loop["status"] == 0 and ref["status"] == 0
    for g, o in zip(loop["steps"], ref["steps"]):
        assert g["s"] == o["s"]
        for key in ("v", "soc", "t_abs"):
            assert abs(g[key] - o[key]) <= 1e-9 * max(1.0, abs(o[key])), (g["s"], key, g[key], o[key])
        assert abs(g["V0"] - o["V0"]) <= 1e-4 * abs(o["V0"]), (g["s"], g["V0"], o["V0"])
        if g["u0"] != o["u0"]:
            assert o["q2"] - o["V0"] < 1e-4 * max(1.0, abs(o["V0"])), (g["s"], g["u0"], o["u0"])
            say("u0 differs at a near tie, stage", g["s"])
            break
    else:
        assert len(loop["steps"]) == len(ref["steps"]) == steps
        assert loop["fuel_g"] == pytest.approx(ref["fuel"], rel=1e-9)
    lat = loop["latency_ms"]
    say("latency ms mean %.3f max %.3f" % (lat["mean"], lat["max"]))


def test_closed_loop_drives_to_route_end(torch):
    """The library loop (dp_loop) over a whole 300 m route with a signal:
    every horizon length 20 .. 1 of its kept plans is used (the window
    shrinks over the last 19 stages), against the oracle's loop step by step
    (V_0 within 1e-4, the same u_0* unless a root near tie, plant states within
    1e-9); past the last stage dp_loop_step reports DP_ESTATE."""
    import ctypes as C
    from paper_2104_01284_amd import _lib as L
    from paper_2104_01284_amd.mpc import ClosedLoop
    route = ins.mpc_route(seed=5, length_m=300.0, n_lights=1)
    loop = ClosedLoop(route)
    res = loop.run()
    say("route end: stage", res["stage"], "status", res["status"], "fuel", res["fuel_g"], "wait", res["wait_s"])
    ref = oracle.closed_loop(route, int(route["N"]), ins.MPC_HORIZON, ins.MPC_T_F, ins.MPC_N_T, ins.mpc_window)
    assert res["status"] == 0 and ref["status"] == 0
    parted = False
    for g, o in zip(res["steps"], ref["steps"]):
        assert g["s"] == o["s"]
        for key in ("v", "soc", "t_abs"):
            assert abs(g[key] - o[key]) <= 1e-9 * max(1.0, abs(o[key])), (g["s"], key, g[key], o[key])
        assert abs(g["V0"] - o["V0"]) <= 1e-4 * abs(o["V0"]), (g["s"], g["V0"], o["V0"])
        if g["u0"] != o["u0"]:
            assert o["q2"] - o["V0"] < 1e-4 * max(1.0, abs(o["V0"])), (g["s"], g["u0"], o["u0"])
            parted = True
            break
    if not parted:
        assert res["stage"] == int(route["N"]) and len(res["steps"]) == int(route["N"])
        assert res["fuel_g"] == pytest.approx(ref["fuel"], rel=1e-9)
        row = L.DpLoopRow()
        assert loop.lib.dp_loop_step(loop._h, C.byref(row)) == L.DP_ESTATE


def test_negative_device_terminal_value_reported(torch):
    """A device terminal_V cannot be checked on the host: a negative value
    sets the plan's device error word, which dp_device_check reports (costs
    must be non-negative); the word is cleared by the report."""
    inst = ins.plain()
    tv = np.zeros((21, 11, 31), dtype=np.float32)
    tv[5, 5, 10] = -2.0
    from paper_2104_01284_amd._lib import DPError
    plan = Plan([dict(inst, terminal_V=torch.from_numpy(tv).cuda())], store_all=True)
    plan.solve()
    with pytest.raises(DPError) as e:
        plan.device_check()
    assert "negative" in str(e.value)
    plan.device_check()
    ok = Plan([dict(inst, terminal_V=torch.from_numpy(np.abs(tv)).cuda())], store_all=True)
    ok.solve()
    ok.device_check()
