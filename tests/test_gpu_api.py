"""C-ABI behaviour on the GPU beyond the numerics of one run: changing the
filter support of a plan (smaller, then back to its capacity), batches that mix
the library eigensolver with the own chain, batches on a caller's stream,
state errors and non-finite input."""
import numpy as np
import pytest
import torch

import oracle
import workload
from tests.gpu_util import nrmse, say

pytestmark = pytest.mark.gpu

slrx = pytest.importorskip("paper_1704_04511_amd")

N_IRLS, N_CG = 3, 6


def problem(seed=301, N1=5, N2=5, M=3):
    return workload.make_problem(seed=seed, P=64, Q=64, T=8, K=1, R=4, N1=N1, N2=N2, M=M, n_irls=N_IRLS,
                                 n_cg=N_CG, name="api")


def new_plan(pb, N1=None, N2=None, M=None, lib_eigh=False):
    T, P, Q = pb.b.shape
    pl = slrx.Plan(P, Q, T, N1 or pb.N1, N2 or pb.N2, M or pb.M,
                   slrx.make_params(lam=pb.lam, n_irls=N_IRLS, n_cg=N_CG, lib_eigh=lib_eigh))
    pl.set_kspace(pb.b)
    pl.set_mask(pb.S)
    return pl


def run_images(pl):
    pl.run()
    pl.sync()
    return pl.images()


def test_set_filter_shrinks_and_restores():
    pb = problem()
    say("set_filter 5x5x3 -> 3x3x2 -> 5x5x3")
    with new_plan(pb) as pl:
        full = run_images(pl)
        pl.set_filter(3, 3, 2)
        small = run_images(pl)
        ref_small = oracle.irls(pb.b, pb.S, 3, 3, 2, pb.lam, N_IRLS, N_CG)
        assert nrmse(small, ref_small) < 1e-4
        pl.set_filter(5, 5, 3)
        again = run_images(pl)
        np.testing.assert_array_equal(again, full)
        with pytest.raises(slrx.SlrxError) as ei:
            pl.set_filter(7, 5, 3)  # beyond the capacity the plan was created with
        assert ei.value.name == "SLRX_EINVAL"
    ref_full = oracle.irls(pb.b, pb.S, 5, 5, 3, pb.lam, N_IRLS, N_CG)
    assert nrmse(full, ref_full) < 1e-4


def test_batch_mixing_library_and_own_eigensolver():
    pbs = [problem(seed=311), problem(seed=312), problem(seed=313, N1=3, N2=3, M=2)]
    say("batch with one library-eigensolver plan")
    refs = []
    for i, pb in enumerate(pbs):
        with new_plan(pb, lib_eigh=(i == 1)) as pl:
            refs.append(run_images(pl))
    plans = [new_plan(pb, lib_eigh=(i == 1)) for i, pb in enumerate(pbs)]
    try:
        slrx.run_batch(plans)
        for i, pl in enumerate(plans):
            np.testing.assert_array_equal(pl.images(), refs[i], err_msg=f"plan {i}")
    finally:
        for pl in plans:
            pl.close()
    # the two eigensolvers agree to the parity tolerance
    assert nrmse(refs[1], oracle.irls(pbs[1].b, pbs[1].S, 5, 5, 3, pbs[1].lam, N_IRLS, N_CG)) < 1e-4


def test_batch_on_caller_stream_runs_plans_in_turn():
    pbs = [problem(seed=321), problem(seed=322)]
    say("batch on a caller stream")
    refs = []
    for pb in pbs:
        with new_plan(pb) as pl:
            refs.append(run_images(pl))
    plans = [new_plan(pb) for pb in pbs]
    stream = torch.cuda.Stream()
    try:
        slrx.run_batch(plans, stream=stream.cuda_stream)
        for i, pl in enumerate(plans):
            np.testing.assert_array_equal(pl.images(), refs[i], err_msg=f"plan {i}")
    finally:
        for pl in plans:
            pl.close()


def test_state_errors():
    pb = problem(seed=331)
    T, P, Q = pb.b.shape
    with slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, slrx.make_params(lam=pb.lam, n_irls=1, n_cg=1)) as pl:
        with pytest.raises(slrx.SlrxError) as ei:
            pl.run()  # no k-space or mask yet
        assert ei.value.name == "SLRX_ESTATE"
        with pytest.raises(slrx.SlrxError) as ei:
            pl.images()  # nothing has run
        assert ei.value.name == "SLRX_ENOTREADY"
        pl.set_kspace(pb.b)
        pl.set_mask(pb.S)
        pl.run()
        pl.sync()
        assert pl.stats()["n_irls"] == 1


def test_non_finite_input_is_reported_and_the_plan_recovers():
    """A NaN in the sampled k-space makes every Gram entry non-finite; the Gram
    pass writes zeros in their place (the eigen-decomposition only sees finite
    input) and the run reports SLRX_ENUMERIC.  With good data the same plan runs
    again; in a batch the other plans are unaffected."""
    say("non-finite input")
    pb = problem(seed=311)
    bad = pb.b.copy()
    t, r, c = np.argwhere(pb.S)[0]
    bad[t, r, c] = np.nan
    with new_plan(pb) as ref_plan:
        ref = run_images(ref_plan)
    with new_plan(pb) as pl:
        pl.set_kspace(bad)
        pl.run()
        with pytest.raises(slrx.SlrxError) as ei:
            pl.sync()
        assert ei.value.name == "SLRX_ENUMERIC"
        pl.set_kspace(pb.b)
        assert np.array_equal(run_images(pl), ref)
    good, poisoned = new_plan(pb), new_plan(pb)
    poisoned.set_kspace(bad)
    try:
        slrx.run_batch([good, poisoned], sync=False)
        good.sync()
        with pytest.raises(slrx.SlrxError) as ei:
            poisoned.sync()
        assert ei.value.name == "SLRX_ENUMERIC"
        assert np.array_equal(good.images(), ref)
    finally:
        good.close()
        poisoned.close()


def test_zero_data_reconstructs_zero():
    """All-zero data: R = 0 and eps = 0 make the weights infinite, and the CG stop
    rule (NaN or non-positive <r,r>) keeps the iterate at zero."""
    say("zero data")
    pb = problem(seed=312)
    with new_plan(pb) as pl:
        pl.set_kspace(np.zeros_like(pb.b))
        img = run_images(pl)
    assert np.array_equal(img, np.zeros_like(img))
