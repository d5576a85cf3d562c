"""Planted mistakes in the FP64 oracle, each caught by a pin.

Every case below edits one expression of ``oracle/oracle.c`` (a plausible
slip: a sign, a dropped term, a transposed operand, a wrong comparison),
builds that copy into a separate library on the CPU and runs the named pins
of ``tests/test_oracle_pins.py`` (and ``tests/test_fidelity_pins.py``) against
it; at least one of them must fail.
The oracle in the repository is not touched.
"""
import contextlib
import os
import subprocess

import pytest

import oracle
import test_fidelity_pins as fpins
import test_oracle_pins as pins
from paper_2104_01284_amd import instances as ins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")


def _fd_mass_small():
    inst = ins.tiny(seed=31, N=4, n_v=9, n_s=7, n_t=13, n_e=4, n_m=3, light=False, t_f=40.0)
    pins.tangent_adjoint_fd_identities(inst, [0])


# (name, text in oracle.c, replacement, pins that must catch it)
MUTANTS = [
    ("grade sign", "(Crr * p->cosa + p->sina)", "(Crr * p->cosa - p->sina)",
     [pins.test_downhill_energy_conservation]),
    ("dropped drag", "+ 0.5 * K[K_RHO] * CdA * v * v;", ";",
     [pins.test_aero_drag_work]),
    ("transposed interpolation operand",
     "double acc = 0.0;\n    for (int a = 0; a < 2; a++) {\n        double wa = a ? v.f : 1.0 - v.f;",
     "double acc = 0.0;\n    for (int a = 0; a < 2; a++) {\n        double wa = a ? 1.0 - v.f : v.f;",
     [pins.test_interp_reproduces_multilinear]),
    ("SoC sign", "double rs = rs0 - (p->dt * o.Ib)", "double rs = rs0 + (p->dt * o.Ib)",
     [pins.test_single_stage_bruteforce_linear_terminal, pins.test_markov_policy_bruteforce]),
    ("tie-break", "if (Q < best) { second = best; best = Q; bu = u; }\n                        else",
     "if (Q <= best) { second = best; best = Q; bu = u; }\n                        else",
     [pins.test_tie_break_lowest_control_index]),
    ("wait time", "*tau = R - x;", "*tau = x;",
     [pins.test_red_phase_invariant_and_wait]),
    ("half-open red", "if (x < R) {", "if (x <= R) {",
     [pins.test_red_phase_half_open]),
    ("fuel coefficient", "q[4] * v * Te", "q[4] * Te",
     [pins.test_fuel_map_monomials]),
    ("dq/dM sign", "dq[T_M] = 2.0 * ds * (-g *", "dq[T_M] = 2.0 * ds * (g *",
     [_fd_mass_small]),
    ("motor efficiency", "p->Pb = Pm >= 0.0 ? Pm / K[K_ETAM] : Pm * K[K_ETAM];",
     "p->Pb = Pm >= 0.0 ? Pm * K[K_ETAM] : Pm * K[K_ETAM];",
     [pins.test_battery_equivalent_circuit]),
    ("root SoC coordinate", "const double rs0 = (I->soc0 - I->s_lo) / h.hs;\n        for (int u = 0",
     "const double rs0 = (I->soc0 - I->s_lo) / h.hs + 0.5;\n        for (int u = 0",
     [pins.test_single_stage_bruteforce_linear_terminal]),
    ("time fraction", "    x.f = delta - fl;\n", "    x.f = 1.0 - (delta - fl);\n",
     [pins.test_markov_policy_bruteforce, pins.test_openloop_bruteforce_refinement]),
    ("rollout tie rule", "if (w > bw || (w == bw && nidx < bn))", "if (w >= bw)",
     [pins.test_rollout_policy_lookup_nearest_corner]),
    ("yellow braking time", "if (since > v / (2.0 * -I->konst[K_AMIN])) {", "if (since > v / (-I->konst[K_AMIN])) {",
     [fpins.test_yellow_rule_closed_form]),
    ("yellow wait", "*tau = (C - x) + R;", "*tau = (C - x);",
     [fpins.test_yellow_rule_closed_form]),
]


@contextlib.contextmanager
def _oracle_library(path):
    saved = (oracle._lib, oracle._SO)
    oracle._lib, oracle._SO = None, path
    try:
        yield
    finally:
        oracle._lib, oracle._SO = saved


@pytest.mark.parametrize("name,old,new,catchers", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, name, old, new, catchers):
    src = open(SRC).read()
    assert src.count(old) == 1, (name, src.count(old))
    mut = tmp_path / "oracle_mutant.c"
    mut.write_text(src.replace(old, new))
    so = str(tmp_path / "liboracle_mutant.so")
    subprocess.run(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                    "-I", os.path.dirname(SRC), "-o", so, str(mut), "-lm"], check=True)
    caught = []
    with _oracle_library(so):
        for pin in catchers:
            try:
                pin()
            except AssertionError:
                caught.append(pin.__name__)
    assert caught, f"planted mistake '{name}' passed {[p.__name__ for p in catchers]}"
