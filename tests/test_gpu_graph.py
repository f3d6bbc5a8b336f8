"""The CG body replayed from a captured HIP graph equals the same kernels
launched one by one (SLRX_FLAG_NO_GRAPH), bit for bit, on every replay: every
outer iteration replays the graph with the plan's own eager work (Gram matrix,
eigen-decomposition, weights) in between, runs are repeated, a parameter change
forces a new capture, and coil plans take the same path; lock-step batches
(which launch one by one) still give the bits of a plan run alone."""
import numpy as np
import pytest

import workload
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

slrx = pytest.importorskip("paper_1704_04511_amd")


def run(pb, no_graph, lam=None, n_cg=None, repeats=1):
    T, P, Q = pb.b.shape
    prm = slrx.make_params(lam=pb.lam if lam is None else lam, n_irls=pb.n_irls,
                           n_cg=pb.n_cg if n_cg is None else n_cg, no_graph=no_graph)
    out = []
    with slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, prm) as pl:
        pl.set_kspace(pb.b)
        pl.set_mask(pb.S)
        for _ in range(repeats):
            pl.run()
            pl.sync()
            out.append(pl.images())
    return out


def test_graph_replays_equal_direct_launches():
    pb = workload.config_problem("c1", n_irls=6)
    say("cg graph vs direct, c1 x 3 runs")
    direct = run(pb, True)[0]
    for i, img in enumerate(run(pb, False, repeats=3)):
        np.testing.assert_array_equal(img, direct, err_msg=f"run {i}")


def test_graph_recaptured_after_parameter_change():
    pb = workload.config_problem("c1", n_irls=3)
    T, P, Q = pb.b.shape
    say("cg graph recapture on set_params")
    with slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, slrx.make_params(lam=pb.lam, n_irls=3, n_cg=6)) as pl:
        pl.set_kspace(pb.b)
        pl.set_mask(pb.S)
        pl.run()
        pl.sync()
        pl.set_params(slrx.make_params(lam=2 * pb.lam, n_irls=3, n_cg=9))
        pl.run()
        pl.sync()
        got = pl.images()
    np.testing.assert_array_equal(got, run(pb, True, lam=2 * pb.lam, n_cg=9)[0])


def test_graph_with_coils_and_in_a_batch():
    say("cg graph: coil plan and batch")
    mc = workload.make_mc_problem(seed=71, P=32, Q=32, T=8, K=2, R=4, ncoils=3, N1=3, N2=3, M=2, n_irls=3, n_cg=5)
    nc, T, P, Q = mc.b.shape
    res = []
    for no_graph in (True, False):
        with slrx.Plan(P, Q, T, 3, 3, 2, slrx.make_params(lam=mc.lam, n_irls=3, n_cg=5, no_graph=no_graph)) as pl:
            pl.set_mask(mc.S)
            pl.set_coils(mc.coils, mc.b)
            pl.run()
            pl.sync()
            res.append(pl.images())
    np.testing.assert_array_equal(res[0], res[1])
    pbs = [workload.make_problem(seed=72 + i, P=64, Q=64, T=8, K=1, R=4, N1=5, N2=5, M=3, n_irls=3, n_cg=6)
           for i in range(3)]
    ref = [run(pb, True)[0] for pb in pbs]
    plans = []
    for pb in pbs:
        pl = slrx.Plan(64, 64, 8, 5, 5, 3, slrx.make_params(lam=pb.lam, n_irls=3, n_cg=6))
        pl.set_kspace(pb.b)
        pl.set_mask(pb.S)
        plans.append(pl)
    try:
        for rep in range(2):
            slrx.run_batch(plans)
            for i, pl in enumerate(plans):
                np.testing.assert_array_equal(pl.images(), ref[i], err_msg=f"slice {i}, batch run {rep}")
    finally:
        for pl in plans:
            pl.close()
