"""Seeded synthetic problem instances for the receding-horizon eco-driving DP.

This module only draws numbers: route data (grade, speed limits, signal
timing), grids, control grids, vehicle parameters and fuel-map coefficients.
It holds none of the method's arithmetic (no dynamics, no costs, no
interpolation), so both the FP64 CPU oracle and the HIP library read the same
instance without sharing any computation.

An instance is a plain dict of Python scalars, lists and numpy arrays.  The
field meanings follow the problem statement of the paper (Sec. III):

* ``N`` stages of ``ds`` metres (Eq. 2 distance step); stage ``k`` sits at
  distance ``k*ds``; the transition k -> k+1 uses ``grade[k]``.
* ``vmax[k]`` (length N+1) is the route speed limit at stage ``k`` (Eq. 7a).
* ``lights`` is a list of ``(stage, cycle, red, offset)``: red at absolute time
  ``tau`` iff ``(tau - offset) mod cycle`` lies in ``[0, red)`` (two-phase SPaT,
  yellow counted as green, Sec. III).
* grids are uniform with inclusive end points: ``(lo, hi, n)``; the travel-time
  grid is ``[0, t_f]`` relative to the horizon start, ``t0_abs`` is the
  absolute clock at the horizon start.
* ``theta`` = (M, CdA, Crr, w_t, w_soc); ``konst`` = the fixed vehicle and
  battery constants listed in ``KONST_NAMES``; ``fuel`` = q0..q5 coefficients
  of the synthetic fuel-rate polynomial in (speed, engine torque).

The paper's routes, SPaT logs and calibrated powertrain maps are not public;
the recipes below keep the structure the paper describes (10 m steps, signals
every few hundred metres, two-phase SPaT, piecewise-constant grade) and the
grid sizes of the workloads the method is measured on.
"""
from __future__ import annotations

import copy
import hashlib

import numpy as np

KONST_NAMES = ("g", "rho_air", "r_w", "i_g", "eta_dl", "eta_m", "C_nom",
               "Voc0", "Voc1", "R_bat", "a_min", "a_max", "xi_ref", "J_inf",
               "P_eng_max", "P_bsg_max")

# Cost given to infeasible states and state-control pairs: orders of magnitude
# above a stage cost (about 1 g per 10 m step) and above any feasible total.
J_INF = 1.0e4
THETA_NAMES = ("M", "CdA", "Crr", "w_t", "w_soc")

WAIT_AT_RED = 1  # option flag bit: a stopped vehicle may wait out a red phase (Eq. 5c)


def default_konst(xi_ref: float) -> list:
    """Vehicle/battery constants of the synthetic 48 V mild hybrid; the last
    two are the engine and BSG power caps of the speed-dependent torque
    limits (Eq. 7e-f), 0 = none."""
    return [9.81, 1.2, 0.30, 3.0, 0.95, 0.90, 28800.0, 42.0, 12.0, 0.1,
            -2.5, 2.0, float(xi_ref), J_INF, 0.0, 0.0]


def draw_fuel(rng: np.random.Generator) -> list:
    """Seeded coefficients q0..q5 of the fuel-rate polynomial (g/s)."""
    lo = np.array([0.10, 0.005, 0.005, 0.0, 1e-4, 0.0])
    hi = np.array([0.20, 0.015, 0.009, 2e-4, 3e-4, 1e-5])
    return [float(x) for x in lo + (hi - lo) * rng.random(6)]


def _piecewise(rng, n, seg_lo, seg_hi, draw):
    out = np.empty(n)
    k = 0
    while k < n:
        L = int(rng.integers(seg_lo, seg_hi + 1))
        out[k:k + L] = draw()
        k += L
    return out


def _lights(rng, N, count, lo, hi, min_gap):
    """Distinct signal stages in [lo, hi] at least ``min_gap`` apart."""
    stages = []
    tries = 0
    while len(stages) < count:
        tries += 1
        s = int(rng.integers(lo, hi + 1))
        if all(abs(s - o) >= min_gap for o in stages):
            stages.append(s)
        if tries > 10000:  # relax the gap for short horizons
            min_gap = max(1, min_gap // 2)
            tries = 0
    stages.sort()
    out = []
    for s in stages:
        C = float(rng.uniform(50.0, 90.0))
        R = float(C * rng.uniform(0.35, 0.55))
        O = float(rng.uniform(0.0, C))
        out.append((s, C, R, O))
    return out


def _base(name, seed, N, ds, grade, vmax, lights, t0_abs, v0, soc0,
          vgrid, sgrid, tgrid, egrid, mgrid, theta, fuel, wait=True):
    return {
        "name": name, "seed": int(seed),
        "N": int(N), "ds": float(ds),
        "grade": np.asarray(grade, dtype=np.float64),
        "vmax": np.asarray(vmax, dtype=np.float64),
        "lights": [tuple(x) for x in lights],
        "t0_abs": float(t0_abs), "v0": float(v0), "soc0": float(soc0),
        "v_grid": tuple(vgrid), "soc_grid": tuple(sgrid), "t_grid": tuple(tgrid),
        "te_grid": tuple(egrid), "tm_grid": tuple(mgrid),
        "theta": [float(x) for x in theta],
        "konst": default_konst(soc0),
        "fuel": list(fuel),
        "terminal_V": None,
        "flags": WAIT_AT_RED if wait else 0,
    }


THETA0 = (1600.0, 0.7, 0.01, 0.5, 5000.0)


def plain(seed: int = 1) -> dict:
    """500 m flat route, 50 stages, one signal at 300 m (C=60 s, R=25 s,
    offset 10 s); grids 21x11x31 states, 11x11 controls."""
    rng = np.random.default_rng(seed)
    N = 50
    return _base("plain_500m", seed, N, 10.0, np.zeros(N), np.full(N + 1, 20.0),
                 [(30, 60.0, 25.0, 10.0)], 0.0, 10.0, 0.55,
                 (0.0, 20.0, 21), (0.4, 0.7, 11), (0.0, 90.0, 31),
                 (0.0, 150.0, 11), (-100.0, 100.0, 11), THETA0, draw_fuel(rng))


def _route(rng, N, n_lights, vtop):
    grade = _piecewise(rng, N, 10, 50, lambda: rng.uniform(-0.03, 0.03))
    limits = [vtop, 0.8 * vtop, 0.6 * vtop]
    vmax = _piecewise(rng, N + 1, 40, 120, lambda: limits[int(rng.integers(0, 3))])
    lights = _lights(rng, N, n_lights, max(1, N // 20), N - max(1, N // 20),
                     max(2, N // 10))
    return grade, vmax, lights


def realistic(seed: int = 2) -> dict:
    """2 km route, 200 stages, 4 signals, +-3 % piecewise-constant grade;
    grids 101x41x201 states, 41x21 controls."""
    rng = np.random.default_rng(seed)
    N = 200
    fuel = draw_fuel(rng)
    grade, vmax, lights = _route(rng, N, 4, 25.0)
    v0 = rng.uniform(5.0, 15.0)
    soc0 = rng.uniform(0.45, 0.65)
    t0 = rng.uniform(0.0, 90.0)
    return _base("realistic_2km", seed, N, 10.0, grade, vmax, lights, t0, v0, soc0,
                 (0.0, 25.0, 101), (0.3, 0.8, 41), (0.0, 240.0, 201),
                 (0.0, 150.0, 41), (-100.0, 100.0, 21), THETA0, fuel)


def large(seed: int = 5) -> dict:
    """3 km route, 300 stages, 8 signals; grids 201x81x401 states (6.5 M per
    stage), 41x21 controls."""
    rng = np.random.default_rng(seed)
    N = 300
    fuel = draw_fuel(rng)
    grade, vmax, lights = _route(rng, N, 8, 30.0)
    v0 = rng.uniform(5.0, 15.0)
    soc0 = rng.uniform(0.45, 0.65)
    t0 = rng.uniform(0.0, 90.0)
    return _base("large_3km", seed, N, 10.0, grade, vmax, lights, t0, v0, soc0,
                 (0.0, 30.0, 201), (0.3, 0.8, 81), (0.0, 360.0, 401),
                 (0.0, 150.0, 41), (-100.0, 100.0, 21), THETA0, fuel)


def batched_member(b: int, base_seed: int = 3000) -> dict:
    """One receding-horizon solve of the heterogeneous batch: horizon 50-200
    stages, grids v 41-101, SoC 21-41, t 61-201 points, controls 21-41 x
    11-21 (odd, so 0 Nm is on the motor grid)."""
    seed = base_seed + b
    rng = np.random.default_rng(seed)
    N = int(rng.integers(50, 201))
    fuel = draw_fuel(rng)
    n_l = max(1, int(round(N * 10.0 / 500.0)))
    grade, vmax, lights = _route(rng, N, n_l, 25.0)
    n_v = int(rng.integers(41, 102))
    n_s = int(rng.integers(21, 42))
    n_t = int(rng.integers(61, 202))
    t_f = max(90.0, 0.12 * N * 10.0)
    n_e = int(rng.integers(21, 42))
    n_m = 2 * int(rng.integers(5, 11)) + 1
    v0 = rng.uniform(0.0, 15.0)
    soc0 = rng.uniform(0.4, 0.7)
    t0 = rng.uniform(0.0, 120.0)
    return _base(f"batch_{b}", seed, N, 10.0, grade, vmax, lights, t0, v0, soc0,
                 (0.0, 25.0, n_v), (0.3, 0.8, n_s), (0.0, t_f, n_t),
                 (0.0, 150.0, n_e), (-100.0, 100.0, n_m), THETA0, fuel)


def batched(n: int = 256, base_seed: int = 3000) -> list:
    return [batched_member(b, base_seed) for b in range(n)]


def paper_shape(seed: int = 7) -> dict:
    """The grid of the paper's own measurement (Sec. IV): 20 steps of 10 m,
    35x26x40 states, 23x30 controls, one signal."""
    rng = np.random.default_rng(seed)
    N = 20
    fuel = draw_fuel(rng)
    light = (12, 60.0, 25.0, float(rng.uniform(0.0, 60.0)))
    return _base("paper_shape", seed, N, 10.0, np.zeros(N), np.full(N + 1, 25.0),
                 [light], 0.0, 10.0, 0.55,
                 (0.0, 25.0, 35), (0.3, 0.8, 26), (0.0, 80.0, 40),
                 (0.0, 150.0, 23), (-100.0, 100.0, 30), THETA0, fuel)


def tiny(seed: int = 11, N: int = 6, n_v: int = 7, n_s: int = 5, n_t: int = 9,
         n_e: int = 3, n_m: int = 3, light: bool = True, flat: bool = False,
         t_f: float | None = None, wait: bool = True) -> dict:
    """Small random instance for exhaustive checks."""
    rng = np.random.default_rng(seed)
    fuel = draw_fuel(rng)
    grade = np.zeros(N) if flat else rng.uniform(-0.03, 0.03, N)
    vmax = np.full(N + 1, 20.0)
    if t_f is None:
        t_f = 1.8 * N * 10.0 / 8.0
    lights = []
    if light and N >= 3:
        k = int(rng.integers(1, N))
        C = float(rng.uniform(20.0, 40.0))
        lights = [(k, C, float(C * rng.uniform(0.3, 0.5)), float(rng.uniform(0, C)))]
    v0 = float(rng.uniform(4.0, 12.0))
    soc0 = float(rng.uniform(0.45, 0.6))
    return _base(f"tiny_{seed}", seed, N, 10.0, grade, vmax, lights,
                 float(rng.uniform(0, 30)), v0, soc0,
                 (0.0, 20.0, n_v), (0.3, 0.8, n_s), (0.0, t_f, n_t),
                 (0.0, 150.0, n_e), (-100.0, 100.0, n_m), THETA0, fuel, wait)


WORKLOADS = {
    "plain": plain,
    "realistic": realistic,
    "large": large,
    "paper": paper_shape,
}


# Horizon of the closed-loop controller on the paper's own grid (Sec. IV):
# 20 steps of 10 m, t_f = 80 s over 40 time nodes.
MPC_HORIZON = 20
MPC_T_F = 80.0
MPC_N_T = 40


def mpc_route(seed: int = 8, length_m: float = 3000.0, n_lights: int = 8) -> dict:
    """A long route for the closed-loop receding-horizon controller (Sec. V):
    ``length_m`` at 10 m steps, ``n_lights`` signals, +-3 % piecewise grade,
    speed limits {25, 20, 15} m/s.  Its grids are those of the paper-shaped
    horizon (35 speed x 26 SoC nodes, 23 x 30 controls); its time grid spans
    the whole trip [0, 3.5 s per 10 m] with the horizon's time step, so that the
    offline full-route DP that supplies the horizons' terminal cost (Sec. III
    after Eq. 9) lives on the same state grid."""
    rng = np.random.default_rng(seed)
    N = int(round(length_m / 10.0))
    grade, vmax, lights = _route(rng, N, n_lights, 25.0)
    h_t = MPC_T_F / (MPC_N_T - 1)
    n_t = int(np.ceil(3.5 * N / h_t)) + 1
    if n_t > 1024:
        raise ValueError("route too long for a 1024-node trip time grid")
    return _base("mpc_route", seed, N, 10.0, grade, vmax, lights, 0.0, 0.0, 0.55,
                 (0.0, 25.0, 35), (0.3, 0.8, 26), (0.0, h_t * (n_t - 1), n_t),
                 (0.0, 150.0, 23), (-100.0, 100.0, 30), THETA0, draw_fuel(rng))


def mpc_window(route: dict, s: int, t_abs: float, v: float, soc: float, horizon: int = MPC_HORIZON,
               t_f: float = MPC_T_F, n_t: int = MPC_N_T) -> dict:
    """The horizon problem of the closed loop at stage ``s`` of ``route``
    (Eq. 6 with the window s .. s+N): the next N = min(horizon, N_route - s)
    steps of the route's grade, speed limits and signals (signals strictly
    inside the window, re-indexed from s), the current state (v, soc) at
    absolute clock ``t_abs``, the horizon time grid [0, t_f] x n_t, and
    w_soc = 0: the terminal cost comes in as ``terminal_V``, taken from the
    full-route solve (the caller fills it)."""
    N = min(int(horizon), int(route["N"]) - int(s))
    if N < 1:
        raise ValueError("no steps left on the route")
    out = copy.deepcopy({k: v_ for k, v_ in route.items() if k != "terminal_V"})
    out["name"] = f"{route['name']}@{s}"
    out["N"] = N
    out["grade"] = np.array(route["grade"][s:s + N], dtype=np.float64)
    out["vmax"] = np.array(route["vmax"][s:s + N + 1], dtype=np.float64)
    out["lights"] = [(x[0] - s,) + tuple(x[1:]) for x in route["lights"] if s < x[0] < s + N]
    out["t0_abs"] = float(t_abs)
    out["v0"] = float(v)
    out["soc0"] = float(soc)
    out["t_grid"] = (0.0, float(t_f), int(n_t))
    theta = list(route["theta"])
    theta[4] = 0.0
    out["theta"] = theta
    out["terminal_V"] = None
    return out


def with_torque_limits(inst: dict, p_eng: float, p_bsg: float) -> dict:
    """The instance with speed-dependent torque limits (Eq. 7e-f) given as
    engine and BSG power caps [W]: T_eng <= p_eng / omega(v) and
    |T_bsg| <= p_bsg / omega(v) at the crank speed of the step's initial
    speed."""
    out = copy.deepcopy(inst)
    out["konst"] = list(out["konst"]) + [0.0] * (16 - len(out["konst"]))
    out["konst"][14] = float(p_eng)
    out["konst"][15] = float(p_bsg)
    return out


def with_yellow(inst: dict, yellow: float) -> dict:
    """The instance with a yellow phase of ``yellow`` seconds before every
    red (three-phase signals, Sec. III): a light becomes (stage, C, R, O, Y),
    yellow for (t_abs - O) mod C in [C - Y, C)."""
    out = copy.deepcopy(inst)
    lights = []
    for light in out["lights"]:
        L, C, R, O = light[:4]
        if not 0.0 <= yellow <= C - R:
            raise ValueError("the yellow phase must fit between green and red")
        lights.append((L, C, R, O, float(yellow)))
    out["lights"] = lights
    return out


def plain_yellow(seed: int = 1) -> dict:
    """The 500 m instance with an 8 s yellow before the signal's red."""
    return with_yellow(plain(seed), 8.0)


def with_stop_signs(inst: dict, stages) -> dict:
    """The instance with stop signs at the given stages: the route speed
    limit there is 0 (Eq. 7a), so the vehicle must be at rest at the sign."""
    out = copy.deepcopy(inst)
    vmax = np.array(out["vmax"], dtype=np.float64)
    for k in stages:
        if not 1 <= int(k) <= int(out["N"]) - 1:
            raise ValueError("a stop sign must sit at a stage in [1, N-1]")
        vmax[int(k)] = 0.0
    out["vmax"] = vmax
    out["stop_signs"] = [int(k) for k in stages]
    return out


def plain_fidelity(seed: int = 1) -> dict:
    """The 500 m instance with a stop sign at 150 m and engine/BSG power caps
    of 20 kW and 8 kW (the caps bind above about 13 m/s and 8 m/s)."""
    return with_stop_signs(with_torque_limits(plain(seed), 20000.0, 8000.0), [15])


def make(name: str, **kw) -> dict:
    return WORKLOADS[name](**kw)


def with_theta(inst: dict, theta) -> dict:
    out = copy.deepcopy(inst)
    out["theta"] = [float(x) for x in theta]
    return out


def value_slab(inst: dict, seed: int) -> np.ndarray:
    """A seeded stand-in for a next-stage value slab J_{k+1} [n_v, n_soc, n_t]
    (FP32): a bowl in speed and SoC, a ramp in time, small noise, J_INF at the
    latest 15 % of the time nodes and on one speed row.  Both the oracle and
    the library can then be fed the same J_{k+1} for an isolated stage at any
    grid size."""
    rng = np.random.default_rng(seed)
    n_v, n_s, n_t = inst["v_grid"][2], inst["soc_grid"][2], inst["t_grid"][2]
    v = np.linspace(0.0, 1.0, n_v)[:, None, None]
    x = np.linspace(0.0, 1.0, n_s)[None, :, None]
    t = np.linspace(0.0, 1.0, n_t)[None, None, :]
    a, bv, bs, ct = rng.uniform(20, 60), rng.uniform(10, 40), rng.uniform(50, 200), rng.uniform(5, 40)
    v0, x0 = rng.uniform(0.3, 0.7), rng.uniform(0.3, 0.7)
    J = a + bv * (v - v0) ** 2 + bs * (x - x0) ** 2 + ct * t + rng.uniform(0.0, 0.5, (n_v, n_s, n_t))
    J[:, :, int(np.ceil(0.85 * n_t)):] = J_INF
    J[int(rng.integers(0, n_v)), :, :] = J_INF
    return J.astype(np.float32)


def evaluations(inst: dict) -> int:
    """Dense state-control evaluations of one full backward sweep: every grid
    node of every stage 0..N-1 times every control pair (Sec. IV counts the
    innermost loop this way)."""
    states = inst["v_grid"][2] * inst["soc_grid"][2] * inst["t_grid"][2]
    return int(inst["N"]) * states * inst["te_grid"][2] * inst["tm_grid"][2]


def digest(inst: dict) -> str:
    """Short content hash of an instance (every field, in key order): stored
    values written from an instance carry it, and a reader compares it with
    the hash of today's generator output before using them."""
    h = hashlib.sha256()
    for k in sorted(inst):
        v = inst[k]
        if isinstance(v, np.ndarray):
            h.update(k.encode() + v.tobytes())
        else:
            h.update(k.encode() + repr(v).encode())
    return h.hexdigest()[:16]
