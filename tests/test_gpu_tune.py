"""The online tuner of launch configurations: while it tries the candidate
workgroup budgets of the tridiagonalisation on the first decompositions of a
shape, then the row access policy (cached or nontemporal) for the chosen
budget, and after it has chosen, results stay the same bit for bit (neither the
row split among workgroups nor the cache policy enters the arithmetic); it
settles on both choices for the batch shape; and with SLRX_TUNE_CACHE set the
choices are written to that file."""
import os

import numpy as np
import pytest

import workload
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

slrx = pytest.importorskip("paper_1704_04511_amd")


def test_tuned_batches_are_bitwise_stable_and_settle(tmp_path):
    os.environ["SLRX_TUNE_CACHE"] = str(tmp_path / "tune.txt")
    # five problems of Gram size 6*6*3 = 108: a shape no other test uses
    pbs = [workload.make_problem(seed=90 + i, P=64, Q=64, T=8, K=1, R=4, N1=6, N2=6, M=3, n_irls=2, n_cg=4)
           for i in range(5)]
    plans = []
    for pb in pbs:
        pl = slrx.Plan(64, 64, 8, 6, 6, 3, slrx.make_params(lam=pb.lam, n_irls=2, n_cg=4))
        pl.set_kspace(pb.b)
        pl.set_mask(pb.S)
        plans.append(pl)
    try:
        ref = None
        for rep in range(12):
            slrx.run_batch(plans)
            imgs = [pl.images() for pl in plans]
            if ref is None:
                ref = imgs
            for i, (a, b) in enumerate(zip(imgs, ref)):
                np.testing.assert_array_equal(a, b, err_msg=f"slice {i}, batch {rep}")
        budget = int(slrx.lib().slrx_tri_workgroup_budget(108, 5))
        say(f"tuned workgroup budget for 5 x 108: {budget}")
        assert budget in (256, 512, 1024, 2048, 4096)
        rows = [[int(x) for x in ln.split()] for ln in (tmp_path / "tune.txt").read_text().splitlines()]
        # device kind a b c ncand chosen
        budget_rows = [r for r in rows if r[1] == 1 and r[2:4] == [108, 5]]
        access_rows = [r for r in rows if r[1] == 3 and r[2:4] == [108, 5]]
        assert len(budget_rows) == 1 and len(access_rows) == 1, rows
        assert access_rows[0][4] == budget_rows[0][6] and access_rows[0][5:] in ([2, 0], [2, 1])
    finally:
        os.environ.pop("SLRX_TUNE_CACHE", None)
        for pl in plans:
            pl.close()
