"""GPU parity of IRLS-direct (SLRX_FLAG_DIRECT: the method without the FFT-based
approximations, Sec. IV / Fig. 2; the lifting linear in all three dimensions,
both sub-problems on the explicit lifted matrix) against the FP64 oracle.

Bar as for the main method: relative image NRMSE <= 1e-4 over all frames and for
every frame alone, the eps / lambda_max trace within 1e-5 relative.  The GPU's
Gram matrix is formed in complex128 from the complex64 iterate, the CG operator's
lifted matrix and its product with H in complex64 (FP32 GEMM over s terms), the
adjoint summed in FP64.
"""
import numpy as np
import pytest

import oracle
import workload
from tests.gpu_util import nrmse, say

pytestmark = pytest.mark.gpu

slrx = pytest.importorskip("paper_1704_04511_amd")

TOL = 1e-4


def prm(pb, n_irls=None, n_cg=None):
    return slrx.make_params(lam=pb.lam, n_irls=n_irls or pb.n_irls, n_cg=pb.n_cg if n_cg is None else n_cg, p=pb.p,
                            gamma=pb.gamma, eps0_frac=pb.eps0_frac, direct=True)


def run_gpu(pb, n_irls=None, n_cg=None):
    T, P, Q = pb.b.shape
    with slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, prm(pb, n_irls, n_cg)) as pl:
        pl.set_kspace(pb.b)
        pl.set_mask(pb.S)
        pl.run()
        pl.sync()
        return pl.images(), pl.stats()


def check(pb, n_irls=None, n_cg=None):
    img, st = run_gpu(pb, n_irls, n_cg)
    tr = {}
    ref = oracle.irls_direct(pb.b, pb.S, pb.N1, pb.N2, pb.M, pb.lam, n_irls or pb.n_irls,
                             pb.n_cg if n_cg is None else n_cg, p=pb.p, gamma=pb.gamma, eps0_frac=pb.eps0_frac,
                             trace=tr)
    e = nrmse(img, ref)
    per_frame = [nrmse(img[t], ref[t]) for t in range(ref.shape[0])]
    print(f"  NRMSE vs oracle {e:.3e}, worst frame {max(per_frame):.3e}; vs truth gpu {nrmse(img, pb.truth):.4f} "
          f"oracle {nrmse(ref, pb.truth):.4f}", flush=True)
    assert e <= TOL, e
    assert max(per_frame) <= TOL, per_frame
    n = len(tr["eps"])
    assert st["n_irls"] == n
    np.testing.assert_allclose(st["eps"][:n], tr["eps"], rtol=1e-5)
    np.testing.assert_allclose(st["lambda_max"][:n], tr["lambda_max"], rtol=1e-5)
    return img


def test_direct_small():
    pb = workload.make_problem(seed=110, P=32, Q=32, T=6, K=1, R=4, N1=3, N2=3, M=2, n_irls=4, n_cg=8)
    say("direct 32x32x6 3x3x2 4x8")
    check(pb)


def test_direct_even_filter_uneven_frame():
    pb = workload.make_problem(seed=111, P=96, Q=64, T=7, K=2, R=4, N1=4, N2=3, M=3, n_irls=3, n_cg=6, phase=True)
    say("direct 96x64x7 4x3x3 3x6")
    check(pb)


def test_direct_c1_full_counts():
    """The 64x64x8 workload (5x5x3 filter) at its stated 15 x 10 iterations."""
    pb = workload.config_problem("c1")
    say(f"direct c1 {pb.b.shape} 5x5x3 {pb.n_irls}x{pb.n_cg}")
    check(pb)


def test_direct_alone_equals_batch_and_rejections():
    pb = workload.make_problem(seed=112, P=32, Q=32, T=6, K=1, R=4, N1=3, N2=3, M=2, n_irls=3, n_cg=4)
    say("direct plan in a batch; rejected calls")
    img, _ = run_gpu(pb)
    T, P, Q = pb.b.shape
    with slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, prm(pb)) as pl:
        pl.set_kspace(pb.b)
        pl.set_mask(pb.S)
        slrx.run_batch([pl])
        np.testing.assert_array_equal(pl.images(), img)
        with pytest.raises(slrx.SlrxError):
            pl.step_gram()
        with pytest.raises(slrx.SlrxError):
            pl.set_coils(np.ones((2, P, Q), np.complex64), np.zeros((2, T, P, Q), np.complex64))
        srv = slrx.Server(1 << 30)
        try:
            with pytest.raises(slrx.SlrxError):
                srv.submit(pl)
        finally:
            srv.close()
