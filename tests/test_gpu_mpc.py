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
    inst = ins.plain()
    plan = Plan([inst], store_all=True)
    plan.solve()
    plan.set_state(0, 8.2, 0.52, 11.0)
    plan.solve()
    trajs, status = plan.rollout()
    torch.cuda.synchronize()
    pi = plan.policy(0).cpu().numpy()
    u0 = int(plan.u0.cpu()[0])
    ro = oracle.rollout(moved(inst, 8.2, 0.52, 11.0), pi, u0)
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
