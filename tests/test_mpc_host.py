"""Closed-loop receding horizon (Sec. V), host side: the horizon window cut
from a route, the oracle's terminal table from a full-route value slab
(Sec. III after Eq. 9), and the oracle's closed loop, pinned against closed
forms and against the full-route solve itself."""
import numpy as np
import pytest

import oracle
from paper_2104_01284_amd import instances as ins


def small_route(seed=21, N=12, n_t=13, t_f=36.0, lights=((4, 40.0, 15.0, 3.0), (9, 50.0, 20.0, 11.0))):
    r = ins.mpc_route(seed=seed, length_m=10.0 * N, n_lights=0)
    r["t_grid"] = (0.0, t_f, n_t)
    r["lights"] = [tuple(x) for x in lights]
    r["v_grid"] = (0.0, 20.0, 9)
    r["soc_grid"] = (0.4, 0.7, 7)
    r["te_grid"] = (0.0, 150.0, 5)
    r["tm_grid"] = (-100.0, 100.0, 5)
    r["v0"] = 6.0
    r["vmax"] = np.full(N + 1, 20.0)
    return r


def test_window_cut_from_route():
    r = ins.mpc_route(seed=3, length_m=600.0, n_lights=3)
    s = 17
    w = ins.mpc_window(r, s, 42.5, 7.0, 0.5)
    N = w["N"]
    assert N == ins.MPC_HORIZON
    assert np.array_equal(w["grade"], r["grade"][s:s + N])
    assert np.array_equal(w["vmax"], r["vmax"][s:s + N + 1])
    expect = [(L - s, C, R, O) for (L, C, R, O) in r["lights"] if s < L < s + N]
    assert w["lights"] == expect
    assert all(1 <= x[0] <= N - 1 for x in w["lights"])
    assert (w["t0_abs"], w["v0"], w["soc0"]) == (42.5, 7.0, 0.5)
    assert w["t_grid"] == (0.0, ins.MPC_T_F, ins.MPC_N_T)
    assert w["theta"][4] == 0.0 and w["theta"][:4] == r["theta"][:4]
    assert r["theta"][4] > 0.0                       # the route keeps its terminal SoC weight
    # the last horizons shrink to the end of the route
    w_end = ins.mpc_window(r, r["N"] - 5, 0.0, 5.0, 0.5)
    assert w_end["N"] == 5 and len(w_end["vmax"]) == 6
    with pytest.raises(ValueError):
        ins.mpc_window(r, r["N"], 0.0, 5.0, 0.5)


def test_route_time_grid_has_horizon_step():
    r = ins.mpc_route(seed=4, length_m=3000.0, n_lights=8)
    h_route = r["t_grid"][1] / (r["t_grid"][2] - 1)
    assert abs(h_route - ins.MPC_T_F / (ins.MPC_N_T - 1)) < 1e-12
    assert r["t_grid"][1] >= 3.5 * r["N"] - 1e-9
    assert len(r["lights"]) == 8 and r["N"] == 300


def test_window_terminal_identity_on_same_grid():
    rng = np.random.default_rng(5)
    J = rng.uniform(0.0, 50.0, (3, 4, 9))
    out = oracle.window_terminal(J, 16.0, 0.0, 9, 16.0, 1.0e4)
    assert np.array_equal(out, J)


def test_window_terminal_exact_for_linear_time_and_jinf_past_end():
    # a value linear in time is reproduced exactly (up to rounding) at any shift
    n_src, t_f_src = 21, 40.0
    t = np.linspace(0.0, t_f_src, n_src)
    a = np.array([[3.0, 5.0], [7.0, 11.0]])
    b = np.array([[0.5, 0.25], [1.5, 2.0]])
    J = a[:, :, None] + b[:, :, None] * t[None, None, :]
    shift, n_t, t_f = 27.3, 9, 24.0
    out = oracle.window_terminal(J, t_f_src, shift, n_t, t_f, 1.0e4)
    tt = shift + np.linspace(0.0, t_f, n_t)
    for m in range(n_t):
        if tt[m] <= t_f_src:
            assert np.allclose(out[:, :, m], a + b * tt[m], rtol=1e-13, atol=1e-12)
        else:
            assert np.all(out[:, :, m] == 1.0e4)
    assert np.any(tt > t_f_src) and np.any(tt <= t_f_src)
    # capped at J_inf
    capped = oracle.window_terminal(J * 1.0e4, t_f_src, 0.0, 5, 10.0, 1.0e4)
    assert capped.max() == 1.0e4


def test_red_wait_closed_form():
    r = {"lights": [(5, 60.0, 25.0, 10.0)]}
    assert oracle.red_wait(r, 4, 12.0) == 0.0            # no signal at stage 4
    assert oracle.red_wait(r, 5, 12.0) == pytest.approx(23.0)   # phase 2 of a 25 s red
    assert oracle.red_wait(r, 5, 40.0) == 0.0            # green (phase 30)
    assert oracle.red_wait(r, 5, 70.0 + 60.0) == pytest.approx(25.0)


def test_closed_loop_first_horizon_is_the_full_route_problem():
    # with a horizon covering the whole route and the route's own time grid,
    # the first horizon problem is the route problem: same V_0 and u_0
    r = small_route()
    t_f, n_t = r["t_grid"][1], r["t_grid"][2]
    full = oracle.solve(r)
    loop = oracle.closed_loop(r, 1, r["N"], t_f, n_t, ins.mpc_window)
    st = loop["steps"][0]
    assert st["V0"] == pytest.approx(full["V0"], rel=1e-12, abs=1e-12)
    assert st["u0"] == full["u0"]


def test_closed_loop_follows_its_own_controls():
    # the loop's plant steps are the one-step model under each u_0*, and the
    # clock only moves forward
    r = small_route()
    loop = oracle.closed_loop(r, 6, 5, 20.0, 11, ins.mpc_window)
    rows = loop["steps"]
    assert loop["status"] == 0 and len(rows) == 6
    for a_, b_ in zip(rows[:-1], rows[1:]):
        assert b_["s"] == a_["s"] + 1 and b_["t_abs"] > a_["t_abs"]
        w = ins.mpc_window(r, a_["s"], a_["t_abs"], a_["v"], a_["soc"], 5, 20.0, 11)
        a, b = divmod(a_["u0"], int(w["tm_grid"][2]))
        st, o = oracle.transition(w, 0, a_["v"], a_["soc"], a, b)
        assert st & 4 == 0
        assert b_["v"] == pytest.approx(o["v1"], rel=1e-14, abs=1e-14)
        assert b_["soc"] == pytest.approx(a_["soc"] - o["dt"] * o["I_bat"] / r["konst"][6], rel=1e-14)
