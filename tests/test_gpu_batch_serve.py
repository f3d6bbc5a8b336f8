"""Batch and serving on the GPU.  A problem's result in a lock-step batch or in
the server equals, bit for bit, its result as a batch of one and as a plain
single-plan run (the batched eigen-decomposition kernels treat every problem
with the single-problem arithmetic, every other kernel works on the problem's
own buffers with fixed-order reductions); it agrees with the FP64 oracle to
the parity tolerance; admission never exceeds the HBM budget."""
import time

import numpy as np
import pytest

import oracle
import workload
from tests.gpu_util import nrmse, say

pytestmark = pytest.mark.gpu

slrx = pytest.importorskip("paper_1704_04511_amd")

# small uneven slices in the style of the batch workload (filter 9x9x5, odd radices)
SPECS = [
    dict(seed=201, P=96, Q=96, T=8, K=1, R=4, N1=9, N2=9, M=5),
    dict(seed=202, P=128, Q=128, T=12, K=2, R=6, N1=9, N2=9, M=5),
    dict(seed=203, P=160, Q=160, T=8, K=2, R=8, N1=9, N2=9, M=5),
    dict(seed=204, P=64, Q=64, T=16, K=1, R=4, N1=5, N2=5, M=3),
    dict(seed=205, P=192, Q=192, T=8, K=1, R=6, N1=9, N2=9, M=5),
    # Gram size 676: a group of its own
    dict(seed=206, P=64, Q=64, T=8, K=1, R=4, N1=13, N2=13, M=4),
]
N_IRLS, N_CG = 3, 6


def problems():
    return [workload.make_problem(n_irls=N_IRLS, n_cg=N_CG, name=f"slice{i}", **s) for i, s in enumerate(SPECS)]


def plan_for(pb):
    T, P, Q = pb.b.shape
    pl = slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, slrx.make_params(lam=pb.lam, n_irls=N_IRLS, n_cg=N_CG))
    pl.set_kspace(pb.b)
    pl.set_mask(pb.S)
    return pl


def alone(pb):
    """The problem as a batch of one."""
    with plan_for(pb) as pl:
        slrx.run_batch([pl])
        return pl.images()


def single_run(pb):
    """The problem through slrx_run."""
    with plan_for(pb) as pl:
        pl.run()
        pl.sync()
        return pl.images()


def test_batch_equals_alone_and_oracle():
    pbs = problems()
    say(f"batch of {len(pbs)} uneven slices")
    ref = [alone(pb) for pb in pbs]
    plans = [plan_for(pb) for pb in pbs]
    try:
        slrx.run_batch(plans)
        out = [pl.images() for pl in plans]
        st = [pl.stats() for pl in plans]
    finally:
        for pl in plans:
            pl.close()
    for i, (a, b) in enumerate(zip(out, ref)):
        np.testing.assert_array_equal(a, b, err_msg=f"slice {i}")
        assert st[i]["n_irls"] == N_IRLS
    for i, pb in enumerate(pbs):
        np.testing.assert_array_equal(out[i], single_run(pb), err_msg=f"slice {i} vs a single run")
    for i in (0, 5):
        pb = pbs[i]
        ora = oracle.irls(pb.b, pb.S, pb.N1, pb.N2, pb.M, pb.lam, N_IRLS, N_CG)
        say(f"slice {i} vs oracle: {nrmse(out[i], ora):.3e}")
        assert nrmse(out[i], ora) < 1e-4


def test_batch_of_the_32_slice_draw_at_full_counts():
    """The batch workload itself: 32 slices of uneven sizes (96..256 squared, 8..20
    echoes), filter 9x9x5, 15 outer x 10 CG iterations, in one lock-step batch.  Every
    slice equals its plain single-plan run bit for bit; the smallest and the median-sized
    slice match the FP64 oracle at the full counts."""
    specs = workload.batch_specs(32, seed=11)
    pbs = [workload.make_problem(name=f"slice{j}", **sp) for j, sp in enumerate(specs)]
    assert all((pb.n_irls, pb.n_cg) == (15, 10) for pb in pbs)
    say("batch of the 32-slice draw, 15 x 10")
    plans = []
    try:
        for pb in pbs:
            T, P, Q = pb.b.shape
            pl = slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, slrx.make_params(lam=pb.lam, n_irls=15, n_cg=10))
            pl.set_kspace(pb.b)
            pl.set_mask(pb.S)
            plans.append(pl)
        slrx.run_batch(plans)
        out = [pl.images() for pl in plans]
    finally:
        for pl in plans:
            pl.close()
    say("32-slice draw: single-plan runs")
    for i, pb in enumerate(pbs):
        T, P, Q = pb.b.shape
        with slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, slrx.make_params(lam=pb.lam, n_irls=15, n_cg=10)) as pl:
            pl.set_kspace(pb.b)
            pl.set_mask(pb.S)
            pl.run()
            pl.sync()
            np.testing.assert_array_equal(out[i], pl.images(), err_msg=f"slice {i} ({pb.b.shape})")
    sizes = [pb.b.size for pb in pbs]
    order = np.argsort(sizes, kind="stable")
    for i in (int(order[0]), int(order[len(order) // 2])):
        pb = pbs[i]
        say(f"32-slice draw: slice {i} {pb.b.shape} vs the oracle")
        ora = oracle.irls(pb.b, pb.S, pb.N1, pb.N2, pb.M, pb.lam, 15, 10)
        e = nrmse(out[i], ora)
        print(f"  slice {i} {pb.b.shape}: NRMSE vs oracle {e:.3e}", flush=True)
        assert e < 1e-4


def test_batch_with_uneven_iteration_counts():
    pbs = problems()[:3]
    n_irls = [1, 3, 2]
    say("batch with iteration counts " + str(n_irls))
    ref, plans = [], []
    for pb, n in zip(pbs, n_irls):
        T, P, Q = pb.b.shape
        prm = slrx.make_params(lam=pb.lam, n_irls=n, n_cg=N_CG)
        with slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, prm) as pl:
            pl.set_kspace(pb.b)
            pl.set_mask(pb.S)
            slrx.run_batch([pl])
            ref.append(pl.images())
        pl = slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, prm)
        pl.set_kspace(pb.b)
        pl.set_mask(pb.S)
        plans.append(pl)
    try:
        slrx.run_batch(plans)
        for i, pl in enumerate(plans):
            np.testing.assert_array_equal(pl.images(), ref[i], err_msg=f"slice {i}")
            assert pl.stats()["n_irls"] == n_irls[i]
    finally:
        for pl in plans:
            pl.close()


def test_server_mix_equals_alone_within_budget():
    pbs = problems()
    say(f"server with {len(pbs)} requests")
    ref = [alone(pb) for pb in pbs]
    fps = [slrx.footprint(slrx.Dims(pb.b.shape[1], pb.b.shape[2], pb.b.shape[0], pb.N1, pb.N2, pb.M))
           for pb in pbs]
    budget = int(max(fps) * 2.2)  # at most two of the larger requests at a time
    srv = slrx.Server(budget, max_slots=3)
    try:
        tickets = []
        for pb in pbs:
            prm = slrx.make_params(lam=pb.lam, n_irls=N_IRLS, n_cg=N_CG)
            tickets.append(srv.submit_data(pb.b, pb.S, pb.N1, pb.N2, pb.M, prm))
        peak = 0
        deadline = time.time() + 120.0
        while not all(srv.poll(t) for t in tickets):
            used, _ = srv.usage()
            peak = max(peak, used)
            assert time.time() < deadline, "server did not finish within 120 s"
            time.sleep(0.002)
        infos = [srv.info(t) for t in tickets]
        out = [srv.fetch(t, pb.b.shape) for t, pb in zip(tickets, pbs)]
        assert srv.usage()[0] <= budget  # idle plans kept for reuse
        # a second round reuses the idle plans and gives the same results
        again = []
        for pb in pbs:
            prm = slrx.make_params(lam=pb.lam, n_irls=N_IRLS, n_cg=N_CG)
            t = srv.submit_data(pb.b, pb.S, pb.N1, pb.N2, pb.M, prm)
            srv.wait(t)
            again.append(srv.fetch(t, pb.b.shape))
    finally:
        srv.close()
    assert peak <= budget
    # from the admission intervals: the running footprint never exceeded the budget
    events = sorted([(i["t_admit"], f) for i, f in zip(infos, fps)] + [(i["t_done"], -f) for i, f in zip(infos, fps)])
    run = 0
    for _, df in events:
        run += df
        assert run <= budget
    # requests submitted together overlapped on the device (continuous batching, not a queue)
    spans = [(i["t_admit"], i["t_done"]) for i in infos]
    overlap = any(a0 < b1 and b0 < a1 for k, (a0, a1) in enumerate(spans) for (b0, b1) in spans[k + 1:])
    assert overlap
    for i, (a, b, c) in enumerate(zip(out, ref, again)):
        np.testing.assert_array_equal(a, b, err_msg=f"request {i}")
        np.testing.assert_array_equal(c, b, err_msg=f"request {i} on a reused plan")


def test_server_mix_with_a_full_size_request():
    """The serving mix at its stated counts: one 256x256x20 request (15x15x5, 20 x 15)
    among three slices of the batch workload (9x9x5, 15 x 10), submitted together.
    Each served result equals its single-plan batch run bit for bit (the full-size
    request's single run is pinned to the oracle at these counts elsewhere), and
    the large request overlaps the small ones on the device."""
    pbs = [workload.make_problem(seed=3, P=256, Q=256, T=20, K=2, R=8, N1=15, N2=15, M=5, n_irls=20, n_cg=15,
                                 phase=True, name="c3-size")]
    pbs += [workload.make_problem(n_irls=15, n_cg=10, name=f"slice{i}", **s) for i, s in enumerate(SPECS[:3])]
    say("server mix with a 256x256x20 request at 20 x 15 and three slices at 15 x 10")
    refs = []
    for pb in pbs:
        T, P, Q = pb.b.shape
        with slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M,
                       slrx.make_params(lam=pb.lam, n_irls=pb.n_irls, n_cg=pb.n_cg)) as pl:
            pl.set_kspace(pb.b)
            pl.set_mask(pb.S)
            slrx.run_batch([pl])
            refs.append(pl.images())
    srv = slrx.Server(8 << 30, max_slots=4)
    try:
        tickets = [srv.submit_data(pb.b, pb.S, pb.N1, pb.N2, pb.M,
                                   slrx.make_params(lam=pb.lam, n_irls=pb.n_irls, n_cg=pb.n_cg)) for pb in pbs]
        for t in tickets:
            srv.wait(t)
        infos = [srv.info(t) for t in tickets]
        out = [srv.fetch(t, pb.b.shape) for t, pb in zip(tickets, pbs)]
    finally:
        srv.close()
    for i, (a, b) in enumerate(zip(out, refs)):
        np.testing.assert_array_equal(a, b, err_msg=f"request {i} ({pbs[i].name})")
    big = infos[0]
    assert any(i["t_admit"] < big["t_done"] and big["t_admit"] < i["t_done"] for i in infos[1:])


def test_server_rejects_request_larger_than_budget():
    pb = problems()[1]
    srv = slrx.Server(1 << 20, max_slots=1)
    try:
        with pytest.raises(slrx.SlrxError) as ei:
            srv.submit_data(pb.b, pb.S, pb.N1, pb.N2, pb.M, slrx.make_params(n_irls=1, n_cg=1))
        assert ei.value.name == "SLRX_ENOMEM"
    finally:
        srv.close()


def _long_problem(seed=301):
    """A request that keeps the device busy for a while (about 0.2 s)."""
    return workload.make_problem(seed=seed, P=256, Q=256, T=20, K=2, R=8, N1=15, N2=15, M=5,
                                 n_irls=20, n_cg=15, name="long")


def test_server_budget_bounds_device_memory():
    """The budget covers the engine's eigen-decomposition buffers too: what the server
    reports never exceeds it, and neither does the device memory it actually holds
    (hipMemGetInfo), beyond a small runtime allowance for streams and events."""
    import torch
    pbs = problems()
    say(f"server device memory within the budget, {len(pbs)} requests x 2")
    dims = [slrx.Dims(pb.b.shape[1], pb.b.shape[2], pb.b.shape[0], pb.N1, pb.N2, pb.M) for pb in pbs]
    fps = [slrx.footprint(d) for d in dims]
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    budget = int(max(fps) * 2.5)
    srv = slrx.Server(budget, max_slots=4)
    slack = 64 << 20
    try:
        tickets = []
        for rep in range(2):
            for pb in pbs:
                prm = slrx.make_params(lam=pb.lam, n_irls=N_IRLS, n_cg=N_CG)
                tickets.append(srv.submit_data(pb.b, pb.S, pb.N1, pb.N2, pb.M, prm))
        peak_srv, peak_dev = 0, 0
        deadline = time.time() + 180.0
        while not all(srv.poll(t) for t in tickets):
            peak_srv = max(peak_srv, srv.usage()[0])
            free, _ = torch.cuda.mem_get_info()
            peak_dev = max(peak_dev, free0 - free)
            assert time.time() < deadline, "server did not finish within 180 s"
            time.sleep(0.002)
        infos = [srv.info(t) for t in tickets]
        for t in tickets:
            srv.wait(t)
    finally:
        srv.close()
    say(f"budget {budget >> 20} MiB: server peak {peak_srv >> 20} MiB, device peak {peak_dev >> 20} MiB")
    assert peak_srv <= budget
    assert peak_dev <= budget + slack
    # every request is charged more than its plan: its share of the engine buffers
    for i, f in zip(infos, fps * 2):
        assert i["bytes"] > f


def test_server_rejects_a_plan_already_queued():
    pb = _long_problem()
    T, P, Q = pb.b.shape
    say("server: the same plan submitted twice")
    srv = slrx.Server(8 << 30, max_slots=2)
    pl = slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, slrx.make_params(lam=pb.lam, n_irls=pb.n_irls, n_cg=pb.n_cg))
    try:
        pl.set_kspace(pb.b)
        pl.set_mask(pb.S)
        t = srv.submit(pl)
        with pytest.raises(slrx.SlrxError) as ei:
            srv.submit(pl)
        assert ei.value.name == "SLRX_EBUSY"
        srv.wait(t)
        t2 = srv.submit(pl)  # free again once done
        srv.wait(t2)
    finally:
        srv.close()
        pl.close()


def test_server_cancel_and_queue_timeout():
    pb = _long_problem()
    small = problems()[0]
    say("server: cancel a queued request, time out another")
    srv = slrx.Server(8 << 30, max_slots=1)
    try:
        prm = slrx.make_params(lam=pb.lam, n_irls=pb.n_irls, n_cg=pb.n_cg)
        sp = slrx.make_params(lam=small.lam, n_irls=N_IRLS, n_cg=N_CG)
        ta = srv.submit_data(pb.b, pb.S, pb.N1, pb.N2, pb.M, prm)
        tb = srv.submit_data(small.b, small.S, small.N1, small.N2, small.M, sp)
        srv.cancel(tb)
        with pytest.raises(slrx.SlrxError) as ei:
            srv.wait(tb)
        assert ei.value.name == "SLRX_ECANCELED"
        srv.set_queue_timeout(0.02)
        tc = srv.submit_data(small.b, small.S, small.N1, small.N2, small.M, sp)
        with pytest.raises(slrx.SlrxError) as ei:
            srv.wait(tc)
        assert ei.value.name == "SLRX_ETIMEDOUT"
        srv.set_queue_timeout(0.0)
        assert srv.wait_for(ta, 60.0)
        with pytest.raises(slrx.SlrxError) as ei:
            srv.cancel(ta)  # finished
        assert ei.value.name == "SLRX_ESTATE"
        td = srv.submit_data(small.b, small.S, small.N1, small.N2, small.M, sp)
        srv.wait(td)
        np.testing.assert_array_equal(srv.fetch(td, small.b.shape), alone(small))
    finally:
        srv.close()


def test_server_destroy_releases_waiting_threads():
    import threading
    pb = _long_problem()
    small = problems()[0]
    say("server destroyed while a thread waits on a queued request")
    srv = slrx.Server(8 << 30, max_slots=1)
    ta = srv.submit_data(pb.b, pb.S, pb.N1, pb.N2, pb.M, slrx.make_params(lam=pb.lam, n_irls=4, n_cg=15))
    tb = srv.submit_data(small.b, small.S, small.N1, small.N2, small.M,
                         slrx.make_params(lam=small.lam, n_irls=N_IRLS, n_cg=N_CG))
    result = {}

    def waiter():
        try:
            srv.wait(tb)
            result["status"] = "SLRX_OK"
        except slrx.SlrxError as e:
            result["status"] = e.name

    th = threading.Thread(target=waiter)
    th.start()
    time.sleep(0.01)
    srv.close()  # cancels tb, lets ta finish, waits for the waiter to leave
    th.join(timeout=60)
    assert not th.is_alive()
    assert result.get("status") in ("SLRX_ECANCELED", "SLRX_OK")
