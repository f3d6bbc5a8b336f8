"""Edge cases at the limits of the supported sizes and degenerate inputs, against
the FP64 oracle (bars as in test_gpu_irls: relative image NRMSE <= 1e-4 over all
frames and per frame, the eps / lambda_max trace within 1e-5):

* the largest filter the eigensolver chain takes (19 x 19 x 8, s = 2888 of 3000),
  two outer iterations;
* the largest frame count with the largest tap count (T = 32, M = 8);
* a single frame (T = 1, M = 1: no echo structure left, the penalty is joint
  sparsity of one image);
* an all-zero sampling mask (nothing measured: the reconstruction is zero).
"""
import numpy as np
import pytest

import oracle
import workload
from tests.gpu_util import nrmse, say

pytestmark = pytest.mark.gpu

slrx = pytest.importorskip("paper_1704_04511_amd")


def check(pb):
    T, P, Q = pb.b.shape
    prm = slrx.make_params(lam=pb.lam, n_irls=pb.n_irls, n_cg=pb.n_cg)
    with slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, prm) as pl:
        pl.set_kspace(pb.b)
        pl.set_mask(pb.S)
        pl.run()
        pl.sync()
        img, st = pl.images(), pl.stats()
    tr = {}
    ref = oracle.irls(pb.b, pb.S, pb.N1, pb.N2, pb.M, pb.lam, pb.n_irls, pb.n_cg, trace=tr)
    e = nrmse(img, ref)
    per_frame = [nrmse(img[t], ref[t]) for t in range(T)]
    print(f"  NRMSE vs oracle {e:.3e}, worst frame {max(per_frame):.3e}", flush=True)
    assert e <= 1e-4 and max(per_frame) <= 1e-4, (e, per_frame)
    n = len(tr["eps"])
    np.testing.assert_allclose(st["eps"][:n], tr["eps"], rtol=1e-5)
    np.testing.assert_allclose(st["lambda_max"][:n], tr["lambda_max"], rtol=1e-5)


def test_largest_filter():
    pb = workload.make_problem(seed=140, P=64, Q=64, T=16, K=2, R=4, N1=19, N2=19, M=8, n_irls=2, n_cg=5)
    say("largest filter 19x19x8 (s = 2888), 64x64x16, 2 x 5")
    check(pb)


def test_largest_frame_and_tap_counts():
    pb = workload.make_problem(seed=141, P=16, Q=16, T=32, K=2, R=4, N1=3, N2=3, M=8, n_irls=4, n_cg=6)
    say("T = 32, M = 8 at 16x16, 3x3x8, 4 x 6")
    check(pb)


def test_single_frame():
    pb = workload.make_problem(seed=142, P=32, Q=32, T=1, K=1, R=2, N1=5, N2=5, M=1, n_irls=4, n_cg=6)
    say("T = 1, M = 1 at 32x32, 5x5x1, 4 x 6")
    check(pb)


def test_all_zero_mask_reconstructs_zero():
    pb = workload.make_problem(seed=143, P=32, Q=32, T=6, K=1, R=4, N1=3, N2=3, M=2, n_irls=3, n_cg=4)
    T, P, Q = pb.b.shape
    say("all-zero sampling mask")
    with slrx.Plan(P, Q, T, 3, 3, 2, slrx.make_params(lam=pb.lam, n_irls=3, n_cg=4)) as pl:
        pl.set_kspace(pb.b)
        pl.set_mask(np.zeros((T, P, Q), np.uint8))
        pl.run()
        pl.sync()
        img = pl.images()
    assert np.array_equal(img, np.zeros_like(img))
