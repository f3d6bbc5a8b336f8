"""End-to-end GPU parity of the IRLS reconstruction against the FP64 oracle.

Bar: relative image NRMSE ||x_gpu - x_oracle|| / ||x_oracle|| <= 1e-4 over all
frames after the fixed iteration counts (FP32 data path vs FP64 oracle), with
the eps / lambda_max trace of every outer iteration within 1e-5 relative.
"""
import numpy as np
import pytest

import oracle
import workload
from tests.gpu_util import crandn, nrmse, say

pytestmark = pytest.mark.gpu

slrx = pytest.importorskip("paper_1704_04511_amd")

TOL = 1e-4


def run_gpu(pb, n_irls=None, n_cg=None, timing=False):
    T, P, Q = pb.b.shape
    prm = slrx.make_params(lam=pb.lam, n_irls=n_irls or pb.n_irls, n_cg=pb.n_cg if n_cg is None else n_cg,
                           p=pb.p, gamma=pb.gamma, eps0_frac=pb.eps0_frac, timing=timing)
    with slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, prm) as pl:
        pl.set_kspace(pb.b)
        pl.set_mask(pb.S)
        pl.run()
        pl.sync()
        return pl.images(), pl.stats()


def run_oracle(pb, n_irls=None, n_cg=None):
    tr = {}
    img = oracle.irls(pb.b, pb.S, pb.N1, pb.N2, pb.M, pb.lam, n_irls or pb.n_irls,
                      pb.n_cg if n_cg is None else n_cg, p=pb.p, gamma=pb.gamma,
                      eps0_frac=pb.eps0_frac, trace=tr)
    return img, tr


def check(pb, n_irls=None, n_cg=None, tol=TOL):
    say(f"irls {pb.name} {pb.b.shape} filter {pb.N1}x{pb.N2}x{pb.M} n_irls={n_irls} n_cg={n_cg}")
    img, st = run_gpu(pb, n_irls, n_cg)
    ref, tr = run_oracle(pb, n_irls, n_cg)
    e = nrmse(img, ref)
    per_frame = [nrmse(img[t], ref[t]) for t in range(ref.shape[0])]
    print(f"  NRMSE vs oracle {e:.3e} (worst frame {max(per_frame):.3e}); vs truth gpu "
          f"{nrmse(img, pb.truth):.4f} oracle {nrmse(ref, pb.truth):.4f}")
    assert e <= tol, e
    assert max(per_frame) <= tol, per_frame
    n = len(tr["eps"])
    np.testing.assert_allclose(st["eps"][:n], tr["eps"], rtol=1e-5)
    np.testing.assert_allclose(st["lambda_max"][:n], tr["lambda_max"], rtol=1e-5)
    return e


def test_c1_full_counts():
    check(workload.config_problem("c1"))


def test_c1_library_eigensolver_path():
    # the reference path (rocSOLVER zheevd for the whole decomposition) agrees too
    pb = workload.config_problem("c1")
    say("irls c1 with SLRX_FLAG_LIBEIGH")
    T, P, Q = pb.b.shape
    prm = slrx.make_params(lam=pb.lam, n_irls=pb.n_irls, n_cg=pb.n_cg, lib_eigh=True)
    with slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, prm) as pl:
        pl.set_kspace(pb.b)
        pl.set_mask(pb.S)
        pl.run()
        pl.sync()
        img = pl.images()
    ref, _ = run_oracle(pb)
    assert nrmse(img, ref) <= TOL


def test_c2_three_outer_iterations():
    check(workload.config_problem("c2"), n_irls=3)


def test_c3_one_outer_iteration():
    check(workload.config_problem("c3"), n_irls=1)


@pytest.mark.parametrize("P,Q,T,N1,N2,M", [(96, 96, 8, 9, 9, 5), (160, 160, 12, 9, 9, 5), (192, 192, 8, 9, 9, 5)])
def test_odd_radix_batch_shapes(P, Q, T, N1, N2, M):
    pb = workload.make_problem(seed=77 + P, P=P, Q=Q, T=T, K=2, R=6, N1=N1, N2=N2, M=M,
                               n_irls=2, n_cg=10, name=f"odd{P}")
    check(pb)


def test_scalar_filter_closed_form():
    # Filter 1x1x1: x^(n) = S b / (1 + lam alpha_n), alpha_n = (||x^(n-1)||^2 + eps_{n-1})^(p/2-1).
    say("scalar filter closed form")
    rng = np.random.default_rng(9)
    T, P, Q = 6, 16, 32
    S = (rng.random((T, P, Q)) < 0.5).astype(np.uint8)
    b = (S * crandn(rng, T, P, Q)).astype(np.complex64)
    lam, p, n_irls = 2.0, 0.6, 5
    prm = slrx.make_params(lam=lam, n_irls=n_irls, n_cg=3, p=p)
    with slrx.Plan(P, Q, T, 1, 1, 1, prm) as pl:
        pl.set_kspace(b)
        pl.set_mask(S)
        pl.run()
        pl.sync()
        img = pl.images()
    x = b.astype(np.complex128)
    eps = np.linalg.norm(x) ** 2 / 100
    for _ in range(n_irls):
        al = (np.linalg.norm(x) ** 2 + eps) ** (p / 2 - 1)
        x = b / (1 + lam * al)
        eps /= 1.4
    assert nrmse(img, np.fft.ifft2(x, norm="ortho")) < 1e-4


def test_lambda_zero_returns_zero_filled():
    say("lambda = 0")
    rng = np.random.default_rng(10)
    T, P, Q = 5, 32, 32
    S = (rng.random((T, P, Q)) < 0.3).astype(np.uint8)
    b = crandn(rng, T, P, Q).astype(np.complex64)
    prm = slrx.make_params(lam=0.0, n_irls=2, n_cg=4)
    with slrx.Plan(P, Q, T, 3, 3, 2, prm) as pl:
        pl.set_kspace(b)
        pl.set_mask(S)
        pl.run()
        pl.sync()
        img = pl.images()
    ref = np.fft.ifft2(S * b.astype(np.complex128), norm="ortho")
    assert nrmse(img, ref) < 1e-6


def test_kspace_output_and_repeat_run_deterministic():
    pb = workload.config_problem("c1", n_irls=2)
    say("kspace + determinism c1")
    T, P, Q = pb.b.shape
    prm = slrx.make_params(lam=pb.lam, n_irls=2, n_cg=10)
    with slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, prm) as pl:
        pl.set_kspace(pb.b)
        pl.set_mask(pb.S)
        pl.run()
        pl.sync()
        img1 = pl.images()
        k1 = pl.kspace()
        pl.run()
        pl.sync()
        img2 = pl.images()
    np.testing.assert_array_equal(img1, img2)
    assert nrmse(k1, np.fft.fft2(img1.astype(np.complex128), norm="ortho")) < 1e-6
