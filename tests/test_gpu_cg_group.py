"""Grouped CG launches in lock-step batches (slrx_set_cg_grouping): one launch per
CG pass for every single-channel problem of a step that shares the tap count M
and the CG count, across frame sizes and counts.  Every problem's result equals,
bit for bit, its result with per-problem CG launches and its plain single-plan
run; problems that cannot be grouped (coil data, IRLS-direct) and problems of
other M or n_cg take their own launches in the same batch; the online choice
between the two strategies (the default) gives the same bits again."""
import numpy as np
import pytest

import workload
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

slrx = pytest.importorskip("paper_1704_04511_amd")


def specs():
    mk = workload.make_problem
    return [
        (mk(seed=301, P=96, Q=96, T=8, K=1, R=4, N1=5, N2=5, M=3, n_irls=4, n_cg=5), {}),
        (mk(seed=302, P=64, Q=128, T=12, K=2, R=4, N1=5, N2=5, M=3, n_irls=4, n_cg=5), {}),
        (mk(seed=303, P=160, Q=32, T=5, K=1, R=4, N1=3, N2=5, M=3, n_irls=3, n_cg=5), dict(giraf=True)),
        (mk(seed=304, P=32, Q=32, T=8, K=1, R=4, N1=1, N2=1, M=3, n_irls=4, n_cg=5), dict(voxel=True)),
        (mk(seed=305, P=64, Q=64, T=8, K=1, R=4, N1=5, N2=5, M=3, n_irls=4, n_cg=0), {}),
        (mk(seed=306, P=64, Q=64, T=10, K=2, R=4, N1=5, N2=5, M=4, n_irls=4, n_cg=5), {}),
        (mk(seed=307, P=32, Q=32, T=6, K=1, R=4, N1=3, N2=3, M=2, n_irls=3, n_cg=4), dict(direct=True)),
        (mk(seed=308, P=256, Q=256, T=8, K=1, R=8, N1=5, N2=5, M=3, n_irls=2, n_cg=5), {}),
    ]


def plan_of(pb, kw):
    T, P, Q = pb.b.shape
    pl = slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M,
                   slrx.make_params(lam=pb.lam, n_irls=pb.n_irls, n_cg=pb.n_cg, **kw))
    pl.set_kspace(pb.b)
    pl.set_mask(pb.S)
    return pl


def run_batch(items, mode, repeats=1):
    slrx.set_cg_grouping(mode)
    plans = [plan_of(pb, kw) for pb, kw in items]
    try:
        for _ in range(repeats):
            slrx.run_batch(plans)
        return [pl.images() for pl in plans]
    finally:
        slrx.set_cg_grouping(-1)
        for pl in plans:
            pl.close()


def test_grouped_cg_equals_per_problem_and_single_runs():
    items = specs()
    say("batch, CG per problem")
    per = run_batch(items, 0)
    say("batch, grouped CG")
    grp = run_batch(items, 1, repeats=2)
    say("batch, tuned CG strategy (several runs)")
    tuned = run_batch(items, -1, repeats=4)
    for i, (pb, kw) in enumerate(items):
        np.testing.assert_array_equal(grp[i], per[i], err_msg=f"problem {i} {pb.b.shape} {kw}")
        np.testing.assert_array_equal(tuned[i], per[i], err_msg=f"problem {i} (tuned)")
        with plan_of(pb, kw) as pl:
            pl.run()
            pl.sync()
            np.testing.assert_array_equal(pl.images(), per[i], err_msg=f"problem {i} vs a single run")


def test_grouped_cg_with_a_coil_problem_in_the_batch():
    mc = workload.make_mc_problem(seed=309, P=32, Q=32, T=8, K=2, R=4, ncoils=3, N1=3, N2=3, M=2, n_irls=3, n_cg=4)
    pbs = [workload.make_problem(seed=310 + i, P=32, Q=32, T=8, K=1, R=4, N1=3, N2=3, M=2, n_irls=3, n_cg=4)
           for i in range(2)]
    say("grouped CG batch with a coil problem")
    out = {}
    for mode in (0, 1):
        slrx.set_cg_grouping(mode)
        plans = []
        try:
            pl = slrx.Plan(32, 32, 8, 3, 3, 2, slrx.make_params(lam=mc.lam, n_irls=3, n_cg=4))
            pl.set_mask(mc.S)
            pl.set_coils(mc.coils, mc.b)
            plans.append(pl)
            for pb in pbs:
                plans.append(plan_of(pb, {}))
            slrx.run_batch(plans)
            out[mode] = [p.images() for p in plans]
        finally:
            slrx.set_cg_grouping(-1)
            for p in plans:
                p.close()
    for a, b in zip(out[0], out[1]):
        np.testing.assert_array_equal(a, b)
