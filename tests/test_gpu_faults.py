"""Allocation failures forced from the host (slrx_fault_alloc, the allocator's
fault-injection hook): every call whose device allocation fails returns
SLRX_ENOMEM, leaves the objects it touched usable, and the device memory in use
returns to where it was once everything is destroyed.  Every kernel still runs
normally: the hook fails the allocation call itself, before any launch."""
import numpy as np
import pytest

import workload
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

slrx = pytest.importorskip("paper_1704_04511_amd")
torch = pytest.importorskip("torch")


def arm(n):
    slrx.lib().slrx_fault_alloc(n)


def free_bytes():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


@pytest.fixture(autouse=True)
def disarm():
    yield
    arm(-1)


def small(seed=130, N1=3, N2=3, M=2, **kw):
    return workload.make_problem(seed=seed, P=32, Q=32, T=6, K=1, R=4, N1=N1, N2=N2, M=M, n_irls=3, n_cg=4, **kw)


def run(pb, prm):
    T, P, Q = pb.b.shape
    with slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, prm) as pl:
        pl.set_kspace(pb.b)
        pl.set_mask(pb.S)
        pl.run()
        pl.sync()
        return pl.images()


def test_plan_coils_and_direct_buffers_fail_cleanly():
    pb = small()
    T, P, Q = pb.b.shape
    prm = slrx.make_params(lam=pb.lam, n_irls=3, n_cg=4)
    ref = run(pb, prm)
    base = free_bytes()
    say("fault: plan arena")
    arm(0)
    with pytest.raises(slrx.SlrxError) as e:
        slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, prm)
    assert e.value.name == "SLRX_ENOMEM"
    say("fault: coil buffers")
    with slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, prm) as pl:
        pl.set_kspace(pb.b)
        pl.set_mask(pb.S)
        arm(0)
        with pytest.raises(slrx.SlrxError) as e:
            pl.set_coils(np.ones((2, P, Q), np.complex64), np.zeros((2, T, P, Q), np.complex64))
        assert e.value.name == "SLRX_ENOMEM"
        pl.run()  # the plan is still the single-channel plan it was
        pl.sync()
        np.testing.assert_array_equal(pl.images(), ref)
    say("fault: IRLS-direct buffers")
    dprm = slrx.make_params(lam=pb.lam, n_irls=3, n_cg=4, direct=True)
    dref = run(pb, dprm)
    with slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, dprm) as pl:
        pl.set_kspace(pb.b)
        pl.set_mask(pb.S)
        arm(0)
        with pytest.raises(slrx.SlrxError) as e:
            pl.run()
        assert e.value.name == "SLRX_ENOMEM"
        pl.run()
        pl.sync()
        np.testing.assert_array_equal(pl.images(), dref)
    assert abs(free_bytes() - base) <= 8 << 20


def test_batch_buffers_fail_cleanly():
    """A filter size no other test uses, so the batched eigen-decomposition's buffers
    for it are allocated here: the batch fails with SLRX_ENOMEM and every plan in it
    runs normally afterwards."""
    pbs = [small(seed=131 + i, N1=7, N2=1, M=1) for i in range(2)]
    refs = [run(pb, slrx.make_params(lam=pb.lam, n_irls=3, n_cg=4)) for pb in pbs]
    plans = []
    try:
        for pb in pbs:
            T, P, Q = pb.b.shape
            pl = slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, slrx.make_params(lam=pb.lam, n_irls=3, n_cg=4))
            pl.set_kspace(pb.b)
            pl.set_mask(pb.S)
            plans.append(pl)
        say("fault: batched eigen-decomposition buffers")
        arm(0)
        with pytest.raises(slrx.SlrxError) as e:
            slrx.run_batch(plans)
        assert e.value.name == "SLRX_ENOMEM"
        arm(-1)
        slrx.run_batch(plans)
        for pl, ref in zip(plans, refs):
            np.testing.assert_array_equal(pl.images(), ref)
    finally:
        for pl in plans:
            pl.close()


def test_server_request_whose_plan_cannot_be_allocated():
    pb = small(seed=133)
    T, P, Q = pb.b.shape
    prm = slrx.make_params(lam=pb.lam, n_irls=3, n_cg=4)
    ref = run(pb, prm)
    srv = slrx.Server(1 << 30)
    try:
        say("fault: a served request's plan")
        arm(0)
        t1 = srv.submit_data(pb.b, pb.S, pb.N1, pb.N2, pb.M, prm)
        with pytest.raises(slrx.SlrxError) as e:
            srv.wait(t1)
        assert e.value.name == "SLRX_ENOMEM"
        t2 = srv.submit_data(pb.b, pb.S, pb.N1, pb.N2, pb.M, prm)
        srv.wait(t2)
        np.testing.assert_array_equal(srv.fetch(t2, pb.b.shape), ref)
    finally:
        srv.close()
