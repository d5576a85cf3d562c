"""FP64 CPU oracle of the eco-driving dynamic program (test infrastructure).

TEST INFRASTRUCTURE ONLY: ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` import this package; the product library
never does.  It is a plain C implementation (``oracle.c``) of the paper's
equations (Sec. III) and its serial nested-loop DP (Sec. IV), wrapped here with
ctypes and numpy.  It shares no code with the HIP library: the only common
input is the instance dict of ``paper_2104_01284_amd.instances``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compile ``oracle.c`` with gcc (FP64, no fast-math, no FMA contraction, OpenMP)."""
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
           "-Wall", "-shared", "-o", _SO + ".tmp", os.path.join(_HERE, "oracle.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


class OrInst(C.Structure):
    _fields_ = [
        ("N", C.c_int32), ("ds", C.c_double),
        ("grade", C.POINTER(C.c_double)), ("vmax", C.POINTER(C.c_double)),
        ("n_lights", C.c_int32), ("l_stage", C.POINTER(C.c_int32)),
        ("l_cycle", C.POINTER(C.c_double)), ("l_red", C.POINTER(C.c_double)),
        ("l_off", C.POINTER(C.c_double)),
        ("t0_abs", C.c_double), ("v0", C.c_double), ("soc0", C.c_double),
        ("v_lo", C.c_double), ("v_hi", C.c_double), ("n_v", C.c_int32),
        ("s_lo", C.c_double), ("s_hi", C.c_double), ("n_s", C.c_int32),
        ("t_f", C.c_double), ("n_t", C.c_int32),
        ("e_lo", C.c_double), ("e_hi", C.c_double), ("n_e", C.c_int32),
        ("m_lo", C.c_double), ("m_hi", C.c_double), ("n_m", C.c_int32),
        ("theta", C.c_double * 5), ("konst", C.c_double * 16), ("fuel", C.c_double * 6),
        ("terminal_V", C.POINTER(C.c_double)),
        ("wait_at_red", C.c_int32),
        ("l_yel", C.POINTER(C.c_double)),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = C.CDLL(_SO)
    P = C.POINTER
    d, i16, i32 = P(C.c_double), P(C.c_int16), P(C.c_int32)
    ins = P(OrInst)
    lib.or_transition.argtypes = [ins, C.c_int, C.c_double, C.c_double, C.c_int, C.c_int, d]
    lib.or_interp.argtypes = [ins, d, C.c_double, C.c_double, C.c_double]
    lib.or_interp.restype = C.c_double
    lib.or_stage.argtypes = [ins, C.c_int, d, d, i16, d]
    lib.or_node_q.argtypes = [ins, C.c_int, d, C.c_int, C.c_int, C.c_int, C.c_int]
    lib.or_node_q.restype = C.c_double
    lib.or_node.argtypes = [ins, C.c_int, d, C.c_int, C.c_int, C.c_int, d, i32, d]
    lib.or_terminal.argtypes = [ins, d]
    lib.or_root.argtypes = [ins, d, d, i32, d]
    lib.or_solve.argtypes = [ins, d, i16, d, d, i32]
    lib.or_rollout.argtypes = [ins, i16, C.c_int32, d, i32]
    lib.or_policy_lookup.argtypes = [ins, i16, C.c_double, C.c_double, C.c_double, i32]
    lib.or_tangent.argtypes = [ins, d, i16, C.c_int32, d]
    lib.or_adjoint.argtypes = [ins, d, i16, C.c_int32, d, d, d, d, d, d, d, d, d]
    lib.or_count_evals.argtypes = [ins]
    lib.or_count_evals.restype = C.c_int64
    lib.or_num_threads.restype = C.c_int
    lib.or_set_num_threads.argtypes = [C.c_int]
    lib.or_set_num_threads.restype = None
    _lib = lib
    return lib


def _ptr(a, ct):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ct))


class Instance:
    """An instance dict marshalled into the oracle's own C struct (it keeps
    the numpy buffers alive)."""

    def __init__(self, inst: dict):
        self.inst = inst
        N = int(inst["N"])
        self.N = N
        self.grade = np.ascontiguousarray(inst["grade"], dtype=np.float64)
        self.vmax = np.ascontiguousarray(inst["vmax"], dtype=np.float64)
        assert self.grade.shape == (N,) and self.vmax.shape == (N + 1,)
        L = inst["lights"]
        self.l_stage = np.array([x[0] for x in L], dtype=np.int32)
        self.l_cycle = np.array([x[1] for x in L], dtype=np.float64)
        self.l_red = np.array([x[2] for x in L], dtype=np.float64)
        self.l_off = np.array([x[3] for x in L], dtype=np.float64)
        # an optional fifth entry: the yellow duration before red (Sec. III)
        self.l_yel = np.array([x[4] if len(x) > 4 else 0.0 for x in L], dtype=np.float64)
        tv = inst.get("terminal_V")
        self.term = None if tv is None else np.ascontiguousarray(tv, dtype=np.float64).ravel()
        s = OrInst()
        s.N = N
        s.ds = inst["ds"]
        s.grade = _ptr(self.grade, C.c_double)
        s.vmax = _ptr(self.vmax, C.c_double)
        s.n_lights = len(L)
        s.l_stage = _ptr(self.l_stage, C.c_int32)
        s.l_cycle = _ptr(self.l_cycle, C.c_double)
        s.l_red = _ptr(self.l_red, C.c_double)
        s.l_off = _ptr(self.l_off, C.c_double)
        s.l_yel = _ptr(self.l_yel, C.c_double)
        s.t0_abs, s.v0, s.soc0 = inst["t0_abs"], inst["v0"], inst["soc0"]
        s.v_lo, s.v_hi, s.n_v = inst["v_grid"]
        s.s_lo, s.s_hi, s.n_s = inst["soc_grid"]
        t_lo, s.t_f, s.n_t = inst["t_grid"]
        assert t_lo == 0.0
        s.e_lo, s.e_hi, s.n_e = inst["te_grid"]
        s.m_lo, s.m_hi, s.n_m = inst["tm_grid"]
        for q in range(5):
            s.theta[q] = inst["theta"][q]
        for q, x in enumerate(inst["konst"]):
            s.konst[q] = x
        for q in range(6):
            s.fuel[q] = inst["fuel"][q]
        s.terminal_V = _ptr(self.term, C.c_double)
        s.wait_at_red = 1 if (inst.get("flags", 1) & 1) else 0
        self.s = s
        self.shape = (int(s.n_v), int(s.n_s), int(s.n_t))
        self.S = int(s.n_v) * int(s.n_s) * int(s.n_t)
        self.n_u = int(s.n_e) * int(s.n_m)

    @property
    def ref(self):
        return C.byref(self.s)


def _as_inst(inst):
    return inst if isinstance(inst, Instance) else Instance(inst)


def transition(inst, k, v, xi, a, b):
    """Continuous one-step model: (status, dict of v1, dt, cost, acc, P_bat, I_bat, mf, q)."""
    I = _as_inst(inst)
    out = np.zeros(8)
    st = _load().or_transition(I.ref, int(k), float(v), float(xi), int(a), int(b), _ptr(out, C.c_double))
    keys = ("v1", "dt", "cost", "acc", "P_bat", "I_bat", "mf", "q")
    return st, dict(zip(keys, out.tolist()))


def interp(inst, J, rv, rs, rt):
    I = _as_inst(inst)
    J = np.ascontiguousarray(J, dtype=np.float64)
    return _load().or_interp(I.ref, _ptr(J, C.c_double), float(rv), float(rs), float(rt))


def terminal(inst):
    I = _as_inst(inst)
    JN = np.empty(I.S)
    _load().or_terminal(I.ref, _ptr(JN, C.c_double))
    return JN.reshape(I.shape)


def stage(inst, k, Jn):
    """One backward step from a given J_{k+1}: (J_k, pi_k, second-best q2_k)."""
    I = _as_inst(inst)
    Jn = np.ascontiguousarray(Jn, dtype=np.float64).ravel()
    Jk = np.empty(I.S)
    pik = np.empty(I.S, dtype=np.int16)
    q2 = np.empty(I.S)
    _load().or_stage(I.ref, int(k), _ptr(Jn, C.c_double), _ptr(Jk, C.c_double),
                     _ptr(pik, C.c_int16), _ptr(q2, C.c_double))
    return Jk.reshape(I.shape), pik.reshape(I.shape), q2.reshape(I.shape)


def node_q(inst, k, Jn, i, j, m, u):
    I = _as_inst(inst)
    Jn = np.ascontiguousarray(Jn, dtype=np.float64).ravel()
    return _load().or_node_q(I.ref, int(k), _ptr(Jn, C.c_double), int(i), int(j), int(m), int(u))


def node(inst, k, Jn, i, j, m):
    """One node of the backward step from J_{k+1}: (J_k, pi_k, second best)."""
    I = _as_inst(inst)
    Jn = np.ascontiguousarray(Jn, dtype=np.float64).ravel()
    J = C.c_double()
    pi = C.c_int32()
    q2 = C.c_double()
    _load().or_node(I.ref, int(k), _ptr(Jn, C.c_double), int(i), int(j), int(m),
                    C.byref(J), C.byref(pi), C.byref(q2))
    return J.value, pi.value, q2.value


def root(inst, J1):
    I = _as_inst(inst)
    J1 = np.ascontiguousarray(J1, dtype=np.float64).ravel()
    V0 = C.c_double()
    u0 = C.c_int32()
    q2 = C.c_double()
    _load().or_root(I.ref, _ptr(J1, C.c_double), C.byref(V0), C.byref(u0), C.byref(q2))
    return V0.value, u0.value, q2.value


def solve(inst, q2=False):
    """Full backward recursion: dict(J [(N+1), n_v, n_s, n_t], pi [N, ...], V0, u0, q2)."""
    I = _as_inst(inst)
    N = I.N
    J = np.empty((N + 1) * I.S)
    pi = np.empty(N * I.S, dtype=np.int16)
    Q2 = np.empty(N * I.S) if q2 else None
    V0 = C.c_double()
    u0 = C.c_int32()
    _load().or_solve(I.ref, _ptr(J, C.c_double), _ptr(pi, C.c_int16), _ptr(Q2, C.c_double),
                     C.byref(V0), C.byref(u0))
    out = {"J": J.reshape((N + 1,) + I.shape), "pi": pi.reshape((N,) + I.shape),
           "V0": V0.value, "u0": u0.value}
    if q2:
        out["q2"] = Q2.reshape((N,) + I.shape)
    return out


def rollout(inst, pi, u0):
    I = _as_inst(inst)
    pi = np.ascontiguousarray(pi, dtype=np.int16).ravel()
    traj = np.empty((I.N + 1) * 8)
    viol = C.c_int32()
    st = _load().or_rollout(I.ref, _ptr(pi, C.c_int16), int(u0), _ptr(traj, C.c_double), C.byref(viol))
    return {"status": st, "violations": viol.value, "traj": traj.reshape(I.N + 1, 8)}


def policy_lookup(inst, pik, v, xi, t):
    """The rollout's control at the off-grid state (v, xi, t) from one
    stage's policy slab: (u, out_of_grid)."""
    I = _as_inst(inst)
    pik = np.ascontiguousarray(pik, dtype=np.int16).ravel()
    assert pik.size == I.S
    oog = C.c_int32()
    u = _load().or_policy_lookup(I.ref, _ptr(pik, C.c_int16), float(v), float(xi), float(t), C.byref(oog))
    return int(u), int(oog.value)


def tangent(inst, J, pi, u0):
    I = _as_inst(inst)
    J = np.ascontiguousarray(J, dtype=np.float64).ravel()
    pi = np.ascontiguousarray(pi, dtype=np.int16).ravel()
    g = np.empty(5)
    _load().or_tangent(I.ref, _ptr(J, C.c_double), _ptr(pi, C.c_int16), int(u0), _ptr(g, C.c_double))
    return g


def adjoint(inst, J, pi, u0, want_rho=False):
    I = _as_inst(inst)
    J = np.ascontiguousarray(J, dtype=np.float64).ravel()
    pi = np.ascontiguousarray(pi, dtype=np.int16).ravel()
    g = np.empty(5)
    rs = np.empty(I.N + 1)
    ab = np.empty(I.N + 1)
    ec = np.empty(I.N + 1)
    et = C.c_double()
    ep = C.c_double()
    rho = np.empty((I.N + 1) * I.S) if want_rho else None
    dg = np.empty(I.N)
    nl = len(I.l_stage)
    ds = np.empty(3 * max(1, nl))
    _load().or_adjoint(I.ref, _ptr(J, C.c_double), _ptr(pi, C.c_int16), int(u0), _ptr(g, C.c_double),
                       _ptr(rs, C.c_double), _ptr(ab, C.c_double), _ptr(ec, C.c_double), C.byref(et), C.byref(ep),
                       _ptr(rho, C.c_double), _ptr(dg, C.c_double), _ptr(ds, C.c_double))
    out = {"grad": g, "rho_sum": rs, "absorbed": ab, "exp_cost": ec, "exp_time": et.value, "exp_socpen": ep.value,
           "dgrade": dg, "dspat": ds[:3 * nl].reshape(nl, 3)}
    if want_rho:
        out["rho"] = rho.reshape((I.N + 1,) + I.shape)
    return out


def window_terminal(J_slab, t_f_src, t_shift, n_t, t_f, J_inf):
    """Terminal cost of a horizon that starts at clock ``t_shift`` of a longer
    solve (Sec. III after Eq. 9: the value function of an offline full-route
    DP serves as the horizon's terminal cost).  ``J_slab`` [n_v, n_s, n_src]
    is that solve's value at the horizon's last stage on the time grid
    [0, t_f_src]; the result [n_v, n_s, n_t] on [0, t_f] is the piecewise-linear
    interpolation in time at t_shift + m t_f / (n_t - 1), J_inf past
    t_f_src, capped at J_inf.  Plain FP64."""
    J = np.asarray(J_slab, dtype=np.float64)
    n_src = J.shape[2]
    h_src = t_f_src / (n_src - 1)
    h = t_f / (n_t - 1)
    out = np.full(J.shape[:2] + (n_t,), float(J_inf))
    for m in range(n_t):
        r = (t_shift + m * h) / h_src
        if r > n_src - 1:
            continue
        c = min(int(np.floor(r)), n_src - 2)
        f = r - c
        out[:, :, m] = np.minimum((1.0 - f) * J[:, :, c] + f * J[:, :, c + 1], J_inf)
    return out


def red_wait(inst_route, stage, t_abs):
    """Wait of a vehicle stopped at the stop line of the signal at ``stage``
    until green (Eq. 5c, Eq. 8): to the end of red, or in yellow (the optional
    fifth light entry: its duration before red) to the end of the red that
    follows, since a vehicle at rest is never inside its braking distance
    after yellow began; 0 if there is no signal or it is green."""
    for light in inst_route["lights"]:
        L, Cy, R, O = light[:4]
        Y = light[4] if len(light) > 4 else 0.0
        if L == stage:
            ph = (t_abs - O) % Cy
            if ph < R:
                return R - ph
            if Y > 0.0 and ph >= Cy - Y and ph - (Cy - Y) > 0.0:
                return (Cy - ph) + R
            return 0.0
    return 0.0


def closed_loop(route, steps, horizon, t_f, n_t, window):
    """The receding-horizon controller of Sec. V on ``route``: an offline
    full-route DP gives the terminal cost; at every stage s the horizon
    problem (``window(route, s, t_abs, v, soc)``, from the instance
    generators) is solved with that terminal cost, its first control u_0* is
    applied to the FP64 plant model (the same one-step model, Eq. 1-2, 5a-b),
    the vehicle moves one step, and a vehicle stopped at a red signal first
    waits for green.  Returns per step (s, t_abs, v, soc, V0, u0, q2 at the
    root) and the trip totals."""
    full = solve(route)
    Jfull = full["J"]
    t_f_src = route["t_grid"][1]
    J_inf = route["konst"][13]
    wt = route["theta"][3]
    s, t_abs, v, soc = 0, route["t0_abs"], route["v0"], route["soc0"]
    fuel = cost = 0.0
    rows = []
    status = 0
    for _ in range(steps):
        if s >= route["N"]:
            break
        if v == 0.0:
            tau = red_wait(route, s, t_abs)
            t_abs += tau
            cost += wt * tau
        win = window(route, s, t_abs, v, soc, horizon, t_f, n_t)
        N = win["N"]
        win["terminal_V"] = window_terminal(Jfull[s + N], t_f_src, t_abs - route["t0_abs"], n_t, t_f, J_inf)
        I = Instance(win)
        r = solve(I)
        V0, u0, q2 = root(I, r["J"][1])
        rows.append({"s": s, "t_abs": t_abs, "v": v, "soc": soc, "V0": V0, "u0": u0, "q2": q2})
        if u0 < 0:
            status = -4
            break
        a, b = divmod(u0, int(win["tm_grid"][2]))
        st, o = transition(I, 0, v, soc, a, b)
        if st & (4 | 8):      # the vehicle cannot move, or no battery current exists
            status = -4
            break
        fuel += o["mf"] * o["dt"]
        cost += o["cost"]
        soc = soc - o["dt"] * o["I_bat"] / route["konst"][6]
        v = o["v1"]
        t_abs += o["dt"]
        s += 1
    return {"steps": rows, "fuel": fuel, "cost": cost, "t_abs": t_abs, "stage": s, "v": v, "soc": soc,
            "status": status}


def count_evals(inst):
    return int(_load().or_count_evals(_as_inst(inst).ref))


def num_threads():
    return int(_load().or_num_threads())


def set_num_threads(n):
    """Threads of the oracle's parallel loops from now on (for timing)."""
    _load().or_set_num_threads(int(n))
