"""GPU parity of the GIRAF variant (SLRX_FLAG_GIRAF: the lifting circular along
the parameter axis as well as in space, the approximation the paper compares
with in Sec. IV / Fig. 3) against the FP64 oracle with ``circ_t=True``.

Same bars as the hybrid steps: the Gram (FP64 accumulation of FP32 images),
the normal operator with one and several coils, and whole reconstructions.
"""
import numpy as np
import pytest

import oracle
import workload
from tests.gpu_util import crandn, masks_to_pairs, nrmse, pairs_to_masks, say

pytestmark = pytest.mark.gpu

slrx = pytest.importorskip("paper_1704_04511_amd")

# (T, P, Q, N1, N2, M): T = M (one circular window per shift), T < 2M-1, the
# largest frame and tap counts, odd radices, a 256 x 256 frame.
SHAPES = [
    (5, 16, 16, 3, 3, 2),
    (6, 16, 16, 2, 2, 6),
    (4, 16, 16, 2, 2, 3),
    (32, 16, 16, 2, 2, 8),
    (6, 32, 96, 4, 5, 3),
    (20, 256, 256, 15, 15, 5),
]


def _plan(T, P, Q, N1, N2, M, lam=1e-2, n_irls=1, n_cg=1):
    return slrx.Plan(P, Q, T, N1, N2, M, slrx.make_params(lam=lam, n_irls=n_irls, n_cg=n_cg, giraf=True))


@pytest.mark.parametrize("shape", SHAPES)
def test_circular_gram_matches_oracle(shape):
    T, P, Q, N1, N2, M = shape
    say(f"giraf gram {shape}")
    rng = np.random.default_rng(81)
    x = crandn(rng, T, P, Q).astype(np.complex64)
    with _plan(*shape) as pl:
        pl.set_kspace(x)
        pl.set_mask(np.ones((T, P, Q), np.uint8))
        R = pl.step_gram()
    R_ref = oracle.gram(x.astype(np.complex128), N1, N2, M, circ_t=True)
    assert np.linalg.norm(R - R_ref) / np.linalg.norm(R_ref) < 2e-6


def _weights(x, N1, N2, M, P, Q):
    R = oracle.gram(x.astype(np.complex128), N1, N2, M, circ_t=True)
    ev, U, alpha = oracle.eig_weights(R, 0.05 * np.linalg.eigvalsh(R).max(), 0.6)
    return masks_to_pairs(oracle.penalty_masks(U, alpha, N1, N2, M, P, Q))


@pytest.mark.parametrize("shape", SHAPES)
def test_circular_normal_operator_matches_oracle(shape):
    T, P, Q, N1, N2, M = shape
    say(f"giraf apply {shape}")
    rng = np.random.default_rng(82)
    x = crandn(rng, T, P, Q).astype(np.complex64)
    S = (rng.random((T, P, Q)) < 0.4).astype(np.uint8)
    Ew = _weights(x, N1, N2, M, P, Q)
    v = crandn(rng, T, P, Q).astype(np.complex64)
    lam = 0.7 / np.abs(Ew).max()
    with _plan(*shape, lam=lam) as pl:
        pl.set_kspace(x)
        pl.set_mask(S)
        out = pl.step_apply(Ew, v)
    ref = oracle.normal_apply(v.astype(np.complex128), S, pairs_to_masks(Ew, M), lam, circ_t=True)
    assert nrmse(out, ref) < 2e-6


@pytest.mark.parametrize("shape", [SHAPES[0], SHAPES[2], SHAPES[4]])
def test_circular_coil_operator_matches_oracle(shape):
    T, P, Q, N1, N2, M = shape
    say(f"giraf coil apply {shape}")
    rng = np.random.default_rng(83)
    x = crandn(rng, T, P, Q).astype(np.complex64)
    S = (rng.random((T, P, Q)) < 0.4).astype(np.uint8)
    C = workload.make_coils(rng, P, Q, 3)
    b = crandn(rng, 3, T, P, Q).astype(np.complex64)
    Ew = _weights(x, N1, N2, M, P, Q)
    v = crandn(rng, T, P, Q).astype(np.complex64)
    lam = 0.7 / np.abs(Ew).max()
    with _plan(*shape, lam=lam) as pl:
        pl.set_mask(S)
        pl.set_coils(C, b)
        out = pl.step_apply(Ew, v)
    ref = oracle.coil_normal(v.astype(np.complex128), S.astype(np.float64), C.astype(np.complex128),
                             pairs_to_masks(Ew, M), lam, circ_t=True)
    assert nrmse(out, ref) < 5e-6


@pytest.mark.parametrize("seed,P,T,M", [(84, 32, 8, 2), (85, 64, 12, 3), (86, 32, 4, 3)])
def test_circular_reconstruction_matches_oracle(seed, P, T, M):
    say(f"giraf recon seed={seed} P={P} T={T} M={M}")
    pb = workload.make_problem(seed=seed, P=P, Q=P, T=T, K=2, R=4, N1=3, N2=3, M=M, n_irls=4, n_cg=6)
    with slrx.Plan(P, P, T, 3, 3, M, slrx.make_params(lam=pb.lam, n_irls=4, n_cg=6, giraf=True)) as pl:
        pl.set_kspace(pb.b)
        pl.set_mask(pb.S)
        pl.run()
        pl.sync()
        img = pl.images()
    ref = oracle.irls(pb.b, pb.S, 3, 3, M, pb.lam, 4, 6, circ_t=True)
    err = nrmse(img, ref)
    say(f"giraf recon NRMSE vs oracle {err:.3e}")
    assert err <= 1e-4


def test_giraf_plans_in_a_batch_equal_their_single_runs():
    say("giraf batch")
    pbs = [workload.make_problem(seed=87 + j, P=32, Q=32, T=8, K=1, R=3, N1=3, N2=3, M=2, n_irls=3, n_cg=4)
           for j in range(2)]
    mk = lambda g: slrx.make_params(lam=1e-3, n_irls=3, n_cg=4, giraf=g)
    single = []
    for pb in pbs:
        with slrx.Plan(32, 32, 8, 3, 3, 2, mk(True)) as pl:
            pl.set_kspace(pb.b)
            pl.set_mask(pb.S)
            pl.run()
            pl.sync()
            single.append(pl.images())
    plans = []
    for j, pb in enumerate(pbs + pbs[:1]):  # two GIRAF plans and one hybrid plan of equal s
        pl = slrx.Plan(32, 32, 8, 3, 3, 2, mk(j < 2))
        pl.set_kspace(pb.b)
        pl.set_mask(pb.S)
        plans.append(pl)
    try:
        slrx.run_batch(plans)
        for pl, ref in zip(plans[:2], single):
            assert np.array_equal(pl.images(), ref)
        assert not np.array_equal(plans[2].images(), single[0])  # the hybrid differs
    finally:
        for pl in plans:
            pl.close()
