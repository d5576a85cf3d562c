"""GPU: dp_solve_static, the solve that allocates nothing (its kernels use a
scratch array the library holds on the device), called through the C ABI,
against dp_solve on the same instance: V_0, u_0*, every value slab and every
policy slab bit for bit (the same kernels on the same inputs).  Two calls in
a row, the second on a smaller instance, so the second runs on the contents
the first left in the shared array; and a plan whose scratch exceeds the
array is refused before anything is enqueued."""
import ctypes as C
import sys

import pytest

from paper_2104_01284_amd import _lib as L
from paper_2104_01284_amd import instances as ins

pytestmark = pytest.mark.gpu
STATIC_BYTES = 64 << 20        # DP_STATIC_SCRATCH_BYTES


def say(*a):
    print("[gpu-no-alloc]", *a, flush=True)
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


def solve_static_abi(torch, plan):
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return plan.lib.dp_solve_static(plan._h, C.c_void_p(plan.J.data_ptr()), C.c_void_p(plan.pi.data_ptr()),
                                    C.c_void_p(plan.V0.data_ptr()), C.c_void_p(plan.u0.data_ptr()), stream)


def test_solve_static_matches_solve(torch):
    cases = [ins.paper_shape(), ins.plain()]          # the second smaller than the first
    for inst in cases:
        say("instance", inst["name"])
        ref = Plan([inst], store_all=True)
        ref.solve()
        st = Plan([inst], store_all=True)
        assert st.bytes[2] <= STATIC_BYTES, st.bytes
        st.J.fill_(0xFF)                              # NaN values, policy -1: nothing carried over
        st.pi.fill_(0xFF)
        st.V0.fill_(-1.0)
        assert solve_static_abi(torch, st) == L.DP_OK
        torch.cuda.synchronize()
        assert torch.equal(st.V0, ref.V0) and torch.equal(st.u0, ref.u0), inst["name"]
        assert torch.equal(st.values(0), ref.values(0)), inst["name"]
        assert torch.equal(st.policy(0), ref.policy(0)), inst["name"]
        assert st.executed_evaluations() == ref.executed_evaluations()
        st.device_check()


def test_solve_static_refuses_large_scratch(torch):
    plan = Plan([ins.realistic()], store_all=False)
    assert plan.bytes[2] > STATIC_BYTES
    plan.V0.fill_(-7.0)
    assert solve_static_abi(torch, plan) == L.DP_EUNSUPPORTED
    buf = C.create_string_buffer(256)
    plan.lib.dp_last_error(buf, 256)
    assert b"static scratch" in buf.value
    torch.cuda.synchronize()
    assert float(plan.V0[0]) == -7.0                  # nothing was enqueued
