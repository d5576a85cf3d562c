"""GPU: the batched solve (the persistent multi-instance sweep, and rounds of
one stage each), its HIP-graph replay and per-instance sweep configurations.

A batch must reproduce every instance's single solve bit for bit: each node's
candidates are computed by the same arithmetic whatever the batch, the
control slices are combined first-minimum in visit order (the persistent
sweep takes no slices: one pass keeps the same first minimum), and exact FP32
minima do not depend on the order the work items run in.  Against the FP64
oracle the tolerances of the single-instance parity tests apply.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2104_01284_amd import instances as ins

pytestmark = pytest.mark.gpu
REL_J = 4e-6
REL_GAP = 1e-6


def say(*a):
    print("[gpu-batched]", *a, flush=True)
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


def small_batch():
    """Heterogeneous horizons, grids, control sets and signal layouts."""
    out = [ins.plain()]
    out.append(ins.tiny(seed=201, N=9, n_v=9, n_s=7, n_t=67, n_e=5, n_m=5, light=True, t_f=90.0))
    out.append(ins.tiny(seed=202, N=3, n_v=5, n_s=4, n_t=20, n_e=3, n_m=3, light=False, t_f=30.0))
    out.append(ins.tiny(seed=203, N=12, n_v=13, n_s=6, n_t=130, n_e=4, n_m=3, light=True, t_f=150.0, wait=False))
    out.append(ins.tiny(seed=204, N=6, n_v=11, n_s=17, n_t=200, n_e=7, n_m=5, light=True, t_f=100.0))
    out.append(ins.tiny(seed=205, N=10, n_v=8, n_s=5, n_t=33, n_e=3, n_m=3, light=False, t_f=60.0))
    return out


def smallest_members(n, pool=64):
    cand = [(ins.evaluations(ins.batched_member(b)), b) for b in range(pool)]
    return [ins.batched_member(b) for _, b in sorted(cand)[:n]]


def solve_single(torch, inst, **kw):
    one = Plan([inst], store_all=True, **kw)
    V0, u0 = one.solve()
    torch.cuda.synchronize()
    return one, float(V0[0]), int(u0[0])


def assert_batch_equals_single(torch, big, insts, **kw):
    for b, inst in enumerate(insts):
        one, V, u = solve_single(torch, inst, **kw)
        assert float(big.V0[b]) == V and int(big.u0[b]) == u, (b, inst["name"])
        if big.store_all:
            assert torch.equal(big.values(b), one.values(0)), (b, inst["name"])
        assert torch.equal(big.policy(b), one.policy(0)), (b, inst["name"])


@pytest.mark.parametrize("kernel,rounds", [(1, False), (2, False), (2, True)])
def test_batch_equals_single_solves(torch, kernel, rounds):
    """The batch in one persistent sweep (the default) and in rounds of
    launches, against every instance's single solve."""
    insts = small_batch()
    say("batch of", len(insts), "kernel", kernel, "rounds", rounds)
    big = Plan(insts, store_all=True, kernel=kernel, rounds=rounds)
    big.solve()
    torch.cuda.synchronize()
    big.device_check()
    assert_batch_equals_single(torch, big, insts, kernel=kernel)


def test_persistent_wait_gives_up_on_stall(torch):
    """The persistent sweep's bounded wait, forced from the host: with the
    test hook every queue's first job waits for a count nothing reaches; the
    wait gives up after its poll limit, every workgroup leaves, the device
    error word is set and dp_device_check reports it; a plan without the hook
    then solves normally."""
    from paper_2104_01284_amd._lib import DPError
    insts = small_batch()
    bad = Plan(insts, store_all=True, stall_test=True)
    bad.solve()
    torch.cuda.synchronize()
    with pytest.raises(DPError) as e:
        bad.device_check()
    assert "gave up" in str(e.value)
    bad.device_check()                  # the word was cleared
    good = Plan(insts, store_all=True)
    good.solve()
    torch.cuda.synchronize()
    good.device_check()
    assert_batch_equals_single(torch, good, insts)


def test_batch_against_oracle(torch):
    insts = small_batch()
    big = Plan(insts, store_all=True)
    V0, u0 = big.solve()
    torch.cuda.synchronize()
    for b, inst in enumerate(insts):
        r = oracle.solve(inst)
        say("batch member", b, inst["name"], "V0 gpu", float(V0[b]), "oracle", r["V0"])
        assert abs(float(V0[b]) - r["V0"]) <= 1e-4 * abs(r["V0"])


def test_per_instance_tiles_in_one_batch(torch):
    """Instances with different SoC tiles (one sweep launch per kernel class
    and round, run side by side) against their single solves and the oracle."""
    insts = small_batch()
    tiles = [4, 8, 16, 4, 8, 16]
    opts = [(2, t, 0, 0) for t in tiles]
    big = Plan(insts, store_all=True, inst_opts=opts)
    for b, t in enumerate(tiles):
        n_s = int(insts[b]["soc_grid"][2])
        if n_s >= t:
            assert int(big.info[b].sweep_tile) == t, (b, t)
    big.solve()
    torch.cuda.synchronize()
    for b, inst in enumerate(insts):
        one, V, u = solve_single(torch, inst, sweep_tile=tiles[b])
        assert float(big.V0[b]) == V and int(big.u0[b]) == u, b
        assert torch.equal(big.values(b), one.values(0)), b
        assert torch.equal(big.policy(b), one.policy(0)), b
    # the isolated stage of a batch member on caller slabs, against the oracle
    inst = insts[4]
    r = oracle.solve(inst)
    for k in range(inst["N"]):
        say("batch member isolated stage", inst["name"], k)
        Jn32 = r["J"][k + 1].astype(np.float32)
        Jo, po, q2 = oracle.stage(inst, k, Jn32.astype(np.float64))
        Jg, pg = big.stage(4, k, torch.from_numpy(Jn32).cuda())
        torch.cuda.synchronize()
        Jg, pg = Jg.cpu().numpy().astype(np.float64), pg.cpu().numpy()
        err = np.abs(Jg - Jo) / np.maximum(1.0, np.abs(Jo))
        assert err.max() <= REL_J, (k, float(err.max()))
        mism = pg != po
        bad = mism & ~((q2 - Jo) < REL_GAP * np.maximum(1.0, np.abs(Jo)))
        assert int(bad.sum()) == 0, (k, int(bad.sum()))


def test_graph_replays_match_eager(torch):
    """Every replay of the recorded solve equals the eager solve, with eager
    work and synchronisation between the replays."""
    insts = small_batch()
    eager = Plan(insts, store_all=True)
    eager.solve()
    torch.cuda.synchronize()
    g = Plan(insts, store_all=True, graph=True)
    for rep in range(4):
        say("graph replay", rep)
        g.J.fill_(0xFF)
        g.pi.fill_(0x7F)
        g.V0.fill_(-1.0)
        V0, u0 = g.solve()
        x = torch.randn(1 << 16, device="cuda").sum()     # unrelated eager work
        torch.cuda.synchronize()
        assert torch.isfinite(x)
        assert torch.equal(V0, eager.V0) and torch.equal(u0, eager.u0), rep
        for b in range(len(insts)):
            assert torch.equal(g.values(b), eager.values(b)), (rep, b)
            assert torch.equal(g.policy(b), eager.policy(b)), (rep, b)
        eager.solve()                                   # eager solve between replays
        torch.cuda.synchronize()


def test_graph_rerecorded_when_buffers_change(torch):
    insts = small_batch()[:3]
    g = Plan(insts, store_all=True, graph=True)
    g.solve()
    torch.cuda.synchronize()
    V_first = g.V0.clone()
    g.J = torch.empty_like(g.J)
    g.pi = torch.empty_like(g.pi)
    g.V0 = torch.empty_like(g.V0)
    g.solve()
    torch.cuda.synchronize()
    assert torch.equal(g.V0, V_first)


def test_batched_members_against_oracle_and_single(torch):
    """Members of the heterogeneous batch workload (the smallest of the first
    64), solved together with the graph, against the oracle's V_0 and against
    their single solves."""
    insts = smallest_members(6)
    say("batched members", [x["name"] for x in insts])
    big = Plan(insts, store_all=False, graph=True)
    V0, u0 = big.solve()
    torch.cuda.synchronize()
    assert_batch_equals_single(torch, big, insts)
    for b, inst in enumerate(insts[:3]):
        r = oracle.solve(inst)
        say("member", inst["name"], "V0 gpu", float(V0[b]), "oracle", r["V0"])
        assert abs(float(V0[b]) - r["V0"]) <= 1e-4 * abs(r["V0"])


def test_full_batch_sampled(torch):
    """The full 256-instance batch in the launch configuration the benchmark
    times: every member against its single solve bit for bit (V_0, u_0*, J_0,
    pi_0), and stage 0 of a stratified subset (smallest, largest, every 16th)
    in the batch's configuration from seeded J_1 slabs, on sampled nodes
    against the oracle fed the same slab."""
    insts = ins.batched(256)
    say("full batch: 256 instances")
    big = Plan(insts, store_all=False, graph=True)
    big.solve()
    torch.cuda.synchronize()
    for b, inst in enumerate(insts):
        one = Plan([inst], store_all=False)
        one.solve()
        torch.cuda.synchronize()
        assert float(big.V0[b]) == float(one.V0[0]) and int(big.u0[b]) == int(one.u0[0]), b
        assert torch.equal(big.value(b, 0), one.value(0, 0)), b
        assert torch.equal(big.policy(b, 0), one.policy(0, 0)), b
        del one
    say("all 256 members equal their single solves")
    work = sorted((ins.evaluations(x), b) for b, x in enumerate(insts))
    strat = sorted({work[0][1], work[-1][1]} | set(range(0, 256, 16)))
    rng = np.random.default_rng(17)
    for b in strat:
        inst = insts[b]
        I = oracle.Instance(inst)
        shp = big.slab_shape(b)
        # stage 0 of the member in the batch's configuration from a seeded J_1
        J1 = ins.value_slab(inst, 5000 + b)
        J0, p0 = big.stage(b, 0, torch.from_numpy(J1).cuda())
        torch.cuda.synchronize()
        J0, p0 = J0.cpu().numpy().astype(np.float64), p0.cpu().numpy()
        J1_64 = J1.astype(np.float64).ravel()
        say("member", b, inst["name"], "shape", shp, "N", inst["N"])
        for _ in range(40):
            i, j, m = (int(rng.integers(0, n)) for n in shp)
            Jo, po, q2 = oracle.node(I, 0, J1_64, i, j, m)
            assert abs(J0[i, j, m] - Jo) <= REL_J * max(1.0, abs(Jo)), (b, i, j, m, J0[i, j, m], Jo)
            if p0[i, j, m] != po:
                assert q2 - Jo < REL_GAP * max(1.0, abs(Jo)), (b, i, j, m)


def test_full_batch_against_stored_oracle_and_rollouts(torch):
    """The full 256-instance batch as the benchmark times it (persistent
    sweep, HIP graph) against the stored FP64 oracle results of its
    stratified subset (tests/golden/batched_oracle.json, each member
    digest-checked): V_0 within 1e-4 relative, and u_0* equal to the oracle's
    unless the oracle's second-best root candidate is within 1e-4 max(1, |V_0|)
    of V_0.  Then the batch's rollouts (one launch, one wave per instance)
    against each subset member's single-plan rollout, bit for bit."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "batched_oracle.json")
    with open(path) as f:
        g = json.load(f)
    insts = ins.batched(256)
    big = Plan(insts, store_all=False, graph=True)
    assert all(int(i.sweep_persistent) == 1 for i in big.info)
    V0, u0 = big.solve()
    torch.cuda.synchronize()
    big.device_check()
    checked = 0
    for m in g["members"]:
        b = int(m["member"])
        assert ins.digest(insts[b]) == m["digest"], b      # the stored results are of today's generator
        rel = abs(float(V0[b]) - m["V0"]) / abs(m["V0"])
        say("member", b, "V0 gpu", float(V0[b]), "oracle", m["V0"], "rel", rel, "u0", int(u0[b]), m["u0"])
        assert rel <= 1e-4, b
        if int(u0[b]) != int(m["u0"]):
            assert "q2_root" in m and m["q2_root"] - m["V0"] < 1e-4 * max(1.0, abs(m["V0"])), b
        checked += 1
    assert checked == len(g["members"]) >= 16
    trajs, status = big.rollout()
    torch.cuda.synchronize()
    for m in g["members"]:
        b = int(m["member"])
        one = Plan([insts[b]], store_all=False)
        one.solve()
        t1, s1 = one.rollout()
        torch.cuda.synchronize()
        a, c = trajs[b], t1[0]
        same = (a == c) | (torch.isnan(a) & torch.isnan(c))     # the last row's control fields are NaN
        assert bool(same.all()), b
        assert torch.equal(status[b], s1[0]), b
        del one
