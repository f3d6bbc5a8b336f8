"""End-to-end GPU parity at the stated iteration counts of the 128x128x16 (15 x 10)
and 256x256x20 (20 x 15) workloads, and the weight update on the Gram matrix of
a late iterate, where epsilon has fallen to lambda_max / 100 / 1.4^19 and the
Gram matrix is close to rank deficient (Algorithm 1; Sec. III.B, III.C).

Bars (FP32 data path vs the FP64 oracle):
  * images: relative NRMSE <= 1e-4 over all frames and for every frame alone;
  * the eps / lambda_max trace of every outer iteration within 1e-5 relative;
  * eigenvalues at the late iterate: the GPU forms the Gram matrix from FP32
    images (relative rounding delta ~ 1e-6 after the 2-D transform), so each
    eigenvalue may move by |d lambda_i| <= 2 delta sqrt(lambda_i lambda_max)
    + delta^2 lambda_max (first-order perturbation of T^H T by T^H dT + dT^H T);
    the test bounds d lambda_i / (lambda_i + eps), the relative change of the
    quantity the weights are a power of, by that bound over (lambda_i + eps);
  * H and the masks E: alpha_i = (lambda_i + eps)^(p/2-1) inherits
    (1 - p/2) times that relative change, H and E are sums dominated by the
    largest alpha_i, so their relative error is bounded by (1 - p/2) times the
    largest relative eigenvalue change, with a factor 2 for the eigenvector
    mixing inside clusters of near-null eigenvalues.
"""
import numpy as np
import pytest

import oracle
import workload
from tests.gpu_util import masks_to_pairs, nrmse, pairs, say

pytestmark = pytest.mark.gpu

slrx = pytest.importorskip("paper_1704_04511_amd")

TOL = 1e-4
DELTA = 1e-6  # relative rounding of the FP32 images the GPU forms the Gram matrix from


def gpu_run(pb):
    T, P, Q = pb.b.shape
    prm = slrx.make_params(lam=pb.lam, n_irls=pb.n_irls, n_cg=pb.n_cg, p=pb.p, gamma=pb.gamma,
                           eps0_frac=pb.eps0_frac)
    with slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, prm) as pl:
        pl.set_kspace(pb.b)
        pl.set_mask(pb.S)
        pl.run()
        pl.sync()
        return pl.images(), pl.stats()


def oracle_run(pb):
    tr = {}
    xk = oracle.irls(pb.b, pb.S, pb.N1, pb.N2, pb.M, pb.lam, pb.n_irls, pb.n_cg, p=pb.p, gamma=pb.gamma,
                     eps0_frac=pb.eps0_frac, trace=tr, return_kspace=True)
    return xk, oracle.idft2(xk), tr


def check_images(name, img, st, ref, tr):
    e = nrmse(img, ref)
    per_frame = [nrmse(img[t], ref[t]) for t in range(ref.shape[0])]
    print(f"  {name}: NRMSE vs oracle {e:.3e}, worst frame {max(per_frame):.3e} "
          f"(frame {int(np.argmax(per_frame))})", flush=True)
    assert e <= TOL, e
    assert max(per_frame) <= TOL, per_frame
    n = len(tr["eps"])
    assert st["n_irls"] == n
    np.testing.assert_allclose(st["eps"][:n], tr["eps"], rtol=1e-5)
    np.testing.assert_allclose(st["lambda_max"][:n], tr["lambda_max"], rtol=1e-5)


@pytest.fixture(scope="module")
def c3_oracle():
    pb = workload.config_problem("c3")
    say(f"oracle c3 {pb.b.shape} 15x15x5 {pb.n_irls}x{pb.n_cg} (FP64, host)")
    return pb, *oracle_run(pb)


def test_c2_full_counts():
    pb = workload.config_problem("c2")
    assert (pb.n_irls, pb.n_cg) == (15, 10)
    say(f"irls c2 {pb.b.shape} 9x9x5 {pb.n_irls}x{pb.n_cg}")
    img, st = gpu_run(pb)
    _, ref, tr = oracle_run(pb)
    check_images("c2", img, st, ref, tr)


def test_c3_full_counts(c3_oracle):
    pb, _, ref, tr = c3_oracle
    assert (pb.n_irls, pb.n_cg) == (20, 15)
    say(f"irls c3 {pb.b.shape} 15x15x5 {pb.n_irls}x{pb.n_cg}")
    img, st = gpu_run(pb)
    check_images("c3", img, st, ref, tr)


def test_weights_at_late_iterate(c3_oracle):
    """The weight update on the Gram matrix of the oracle's final iterate, at the
    epsilon of the last outer iteration: eigenvalues (the smallest ones relative to
    lambda + eps), H and every mask plane."""
    pb, xk, _, tr = c3_oracle
    T, P, Q = pb.b.shape
    N1, N2, M = pb.N1, pb.N2, pb.M
    eps = tr["eps"][-1]
    R = oracle.gram(xk, N1, N2, M)
    lam_ref, U, alpha = oracle.eig_weights(R, eps, pb.p)
    lmax = lam_ref.max()
    say(f"weights at the late iterate: eps = lambda_max / {lmax / eps:.3g}")
    with slrx.Plan(P, Q, T, N1, N2, M, slrx.make_params(lam=pb.lam, n_irls=1, n_cg=1)) as pl:
        pl.set_kspace(pb.b)
        pl.set_mask(pb.S)
        pl.set_init(xk.astype(np.complex64))
        lam, H, E = pl.step_weights(eps)
    lp = np.maximum(lam_ref, 0.0)
    bound = 2 * DELTA * np.sqrt(lp * lmax) + DELTA ** 2 * lmax
    rel = np.abs(lam - lam_ref) / (lp + eps)
    rel_bound = bound / (lp + eps)
    k = 64
    print(f"  smallest {k}: max rel change {rel[:k].max():.3e} (bound {rel_bound[:k].max():.3e}); "
          f"all: {rel.max():.3e}; lambda_min/lambda_max {lam_ref[0] / lmax:.2e}", flush=True)
    assert np.all(np.abs(lam - lam_ref) <= bound), np.max(np.abs(lam - lam_ref) / bound)
    tol_w = 2 * (1 - pb.p / 2) * rel_bound.max()
    H_ref = oracle.weight_matrix(U, alpha)
    eH = nrmse(H, H_ref)
    E_ref = oracle.penalty_masks(U, alpha, N1, N2, M, P, Q)
    eE = [nrmse(E[w], E_ref[m, mp]) for w, (m, mp) in enumerate(pairs(M))]
    print(f"  H NRMSE {eH:.3e}, worst mask plane {max(eE):.3e}, bar {tol_w:.3e}", flush=True)
    assert eH <= tol_w
    assert max(eE) <= tol_w
    # and the masks land in the CG unchanged: the stored planes are the complex64 rounding
    assert nrmse(E, masks_to_pairs(E_ref)) <= tol_w
