"""GPU parity of the multichannel data term (Sec. II.A, eq. ``measurement_ij``).

The normal operator, CG solves and whole reconstructions with coil
sensitivities are compared with the FP64 oracle on the same seeded inputs
(relative Frobenius bars from FP32 rounding of the forward half of the coil
path; its adjoint half runs in FP64); one coil of constant phase at lam = 1e-3
must match the oracle and the single-channel plan; the 12-coil workload must
match the oracle at its stated counts; coil plans in a lock-step batch must
equal their single runs bit for bit; and the entry point checks its
arguments.
"""
import ctypes

import numpy as np
import pytest

import oracle
import workload
from tests.gpu_util import crandn, masks_to_pairs, nrmse, pairs_to_masks, say

pytestmark = pytest.mark.gpu

slrx = pytest.importorskip("paper_1704_04511_amd")

# (T, P, Q, N1, N2, M, ncoils): odd radices in both directions, the largest
# frame count with the largest tap count, T < 2M-1 (no Toeplitz part), the
# largest coil count, the multichannel workload's frame and coil count, and
# the largest frame.
COIL_SHAPES = [
    (5, 16, 16, 3, 3, 2, 1),
    (6, 32, 96, 4, 5, 3, 3),
    (4, 160, 32, 3, 2, 4, 2),
    (32, 16, 16, 2, 2, 8, 4),
    (4, 16, 16, 2, 2, 3, 2),
    (3, 8, 8, 1, 1, 1, 32),
    (12, 128, 128, 9, 9, 5, 12),
    (20, 256, 256, 15, 15, 5, 4),
]


def coil_problem(seed, T, P, Q, nc, frac=0.4):
    rng = np.random.default_rng(seed)
    x = crandn(rng, T, P, Q).astype(np.complex64)
    S = (rng.random((T, P, Q)) < frac).astype(np.uint8)
    C = workload.make_coils(rng, P, Q, nc) if nc > 1 else np.full((1, P, Q), np.exp(0.4j), np.complex64)
    b = crandn(rng, nc, T, P, Q).astype(np.complex64)
    return rng, x, S, C, b


def weights(x, N1, N2, M, P, Q, frac):
    R = oracle.gram(x.astype(np.complex128), N1, N2, M)
    ev, U, alpha = oracle.eig_weights(R, frac * np.linalg.eigvalsh(R).max(), 0.6)
    return masks_to_pairs(oracle.penalty_masks(U, alpha, N1, N2, M, P, Q))


@pytest.mark.parametrize("dominant", ["penalty", "data"])
@pytest.mark.parametrize("shape", COIL_SHAPES)
def test_coil_normal_operator_matches_oracle(shape, dominant):
    T, P, Q, N1, N2, M, nc = shape
    say(f"coil apply {shape} {dominant}")
    rng, x, S, C, b = coil_problem(31, T, P, Q, nc)
    Ew = weights(x, N1, N2, M, P, Q, 0.05)
    v = crandn(rng, T, P, Q).astype(np.complex64)
    lam = (0.7 if dominant == "penalty" else 1e-3) / np.abs(Ew).max()
    with slrx.Plan(P, Q, T, N1, N2, M, slrx.make_params(lam=lam, n_irls=1, n_cg=1)) as pl:
        pl.set_mask(S)
        pl.set_coils(C, b)
        out = pl.step_apply(Ew, v)
    ref = oracle.coil_normal(v.astype(np.complex128), S.astype(np.float64), C.astype(np.complex128),
                             pairs_to_masks(Ew, M), lam)
    assert nrmse(out, ref) < 5e-6


@pytest.mark.parametrize("shape", COIL_SHAPES[:5])
def test_coil_cg_matches_oracle(shape):
    T, P, Q, N1, N2, M, nc = shape
    say(f"coil cg {shape}")
    rng, x, S, C, b = coil_problem(32, T, P, Q, nc, frac=0.5)
    Ew = weights(x, N1, N2, M, P, Q, 0.02)
    lam = 0.5 / np.abs(Ew).max()
    Sd, Cd = S.astype(np.float64), C.astype(np.complex128)
    rhs = oracle.coil_adjoint(Sd[None] * b.astype(np.complex128), Sd, Cd)
    for n_cg in (0, 1, 4):
        with slrx.Plan(P, Q, T, N1, N2, M, slrx.make_params(lam=lam, n_irls=1, n_cg=1)) as pl:
            pl.set_mask(S)
            pl.set_coils(C, b)
            pl.step_cg(Ew, n_cg)
            xk_gpu = pl.kspace()
        xk = oracle.cg(lambda v: oracle.coil_normal(v, Sd, Cd, pairs_to_masks(Ew, M), lam), rhs, rhs, n_cg)
        assert nrmse(xk_gpu, xk) < 1e-5, n_cg


def _mc(seed, P=32, Q=32, T=8, nc=4, n_irls=4, n_cg=6):
    return workload.make_mc_problem(seed=seed, P=P, Q=Q, T=T, K=2, R=4, ncoils=nc, N1=3, N2=3, M=2,
                                    n_irls=n_irls, n_cg=n_cg)


def _plan(pb):
    T, P, Q = pb.b.shape[1:]
    pl = slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M,
                   slrx.make_params(lam=pb.lam, n_irls=pb.n_irls, n_cg=pb.n_cg, p=pb.p))
    pl.set_mask(pb.S)
    pl.set_coils(pb.coils, pb.b)
    return pl


@pytest.mark.parametrize("seed,P,nc", [(41, 32, 4), (42, 64, 8), (43, 96, 3)])
def test_coil_reconstruction_matches_oracle(seed, P, nc):
    say(f"coil recon seed={seed} P={P} nc={nc}")
    pb = _mc(seed, P=P, Q=P, nc=nc)
    with _plan(pb) as pl:
        pl.run()
        pl.sync()
        img = pl.images()
    ref = oracle.irls(pb.b, pb.S, pb.N1, pb.N2, pb.M, pb.lam, pb.n_irls, pb.n_cg, p=pb.p, coils=pb.coils)
    err = nrmse(img, ref)
    say(f"coil recon NRMSE vs oracle {err:.3e}")
    assert err <= 1e-4


def test_single_coil_of_constant_phase_matches_oracle_and_single_channel_plan():
    """One coil of constant phase is the single-channel model (the data term is
    exactly S): at the workloads' lam = 1e-3 the operator is only of size lam in
    the unsampled k-space, so rounding spread there by the adjoint half of the
    coil data term would show up at ~1e-4; in complex128 it does not.  Checked
    against the FP64 oracle with coil maps (bar 1e-4, every frame) and against
    the single-channel plan, which applies S exactly (bar 1e-5)."""
    say("single coil of constant phase, lam = 1e-3")
    pb = workload.make_problem(seed=44, P=32, Q=32, T=8, K=1, R=3, N1=3, N2=3, M=2, n_irls=6, n_cg=8,
                               lam=1e-3)
    ph = np.complex64(np.exp(0.9j))
    C = np.full((1, 32, 32), ph, np.complex64)
    bc = (pb.b * ph)[None]
    prm = slrx.make_params(lam=pb.lam, n_irls=pb.n_irls, n_cg=pb.n_cg)
    with slrx.Plan(32, 32, 8, 3, 3, 2, prm) as a, slrx.Plan(32, 32, 8, 3, 3, 2, prm) as c:
        a.set_kspace(pb.b)
        a.set_mask(pb.S)
        c.set_mask(pb.S)
        c.set_coils(C, bc)
        for pl in (a, c):
            pl.run()
            pl.sync()
        img_c, img_a = c.images(), a.images()
    ref = oracle.irls(bc, pb.S, 3, 3, 2, pb.lam, pb.n_irls, pb.n_cg, p=pb.p, coils=C)
    e_ora = nrmse(img_c, ref)
    e_frames = max(nrmse(img_c[t], ref[t]) for t in range(ref.shape[0]))
    e_single = nrmse(img_c, img_a)
    say(f"single coil: vs oracle {e_ora:.3e} (worst frame {e_frames:.3e}), vs single-channel plan {e_single:.3e}")
    assert e_ora <= 1e-4 and e_frames <= 1e-4
    assert e_single < 1e-5


def test_mc_workload_full_counts_matches_oracle():
    """The 12-coil workload (128x128 x 12 echoes, R = 8, filter 9x9x5, lam = 1e-3,
    15 x 10) against the FP64 oracle: bar 1e-4 over all frames and per frame, and
    the eps / lambda_max trace."""
    pb = workload.config_problem("mc")
    nc, T, P, Q = pb.b.shape
    say(f"mc workload {nc} coils {T}x{P}x{Q} {pb.N1}x{pb.N2}x{pb.M} {pb.n_irls}x{pb.n_cg}")
    with _plan(pb) as pl:
        pl.run()
        pl.sync()
        img = pl.images()
        st = pl.stats()
    tr = {}
    ref = oracle.irls(pb.b, pb.S, pb.N1, pb.N2, pb.M, pb.lam, pb.n_irls, pb.n_cg, p=pb.p, coils=pb.coils, trace=tr)
    e = nrmse(img, ref)
    e_frames = max(nrmse(img[t], ref[t]) for t in range(T))
    say(f"mc workload NRMSE vs oracle {e:.3e} (worst frame {e_frames:.3e})")
    assert e <= 1e-4 and e_frames <= 1e-4
    n = len(tr["eps"])
    np.testing.assert_allclose(st["eps"][:n], tr["eps"], rtol=1e-5)
    np.testing.assert_allclose(st["lambda_max"][:n], tr["lambda_max"], rtol=1e-5)


def test_coil_plans_in_a_batch_equal_their_single_runs():
    say("coil batch")
    pbs = [_mc(51, nc=3), _mc(52, P=64, Q=64, nc=5, n_irls=3)]
    single = []
    for pb in pbs:
        with _plan(pb) as pl:
            pl.run()
            pl.sync()
            single.append(pl.images())
    sc = workload.make_problem(seed=53, P=32, Q=32, T=8, K=1, R=3, N1=3, N2=3, M=2, n_irls=3, n_cg=5)
    plans = [_plan(pb) for pb in pbs]
    p3 = slrx.Plan(32, 32, 8, 3, 3, 2, slrx.make_params(lam=sc.lam, n_irls=sc.n_irls, n_cg=sc.n_cg))
    p3.set_kspace(sc.b)
    p3.set_mask(sc.S)
    try:
        slrx.run_batch(plans + [p3])
        for pl, ref in zip(plans, single):
            assert np.array_equal(pl.images(), ref)
    finally:
        for pl in plans + [p3]:
            pl.close()


def test_device_inputs_equal_host_inputs_and_reset():
    import torch
    say("coil device inputs")
    pb = _mc(61, nc=3, n_irls=2)
    with _plan(pb) as a:
        a.run()
        a.sync()
        ref = a.images()
    T, P, Q = pb.b.shape[1:]
    with slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M,
                   slrx.make_params(lam=pb.lam, n_irls=pb.n_irls, n_cg=pb.n_cg, p=pb.p)) as pl:
        pl.set_mask(pb.S)
        pl.set_coils(torch.from_numpy(pb.coils).cuda(), torch.from_numpy(pb.b).cuda())
        pl.run()
        pl.sync()
        assert np.array_equal(pl.images(), ref)
        # back to the single-channel model: k-space is required again
        pl.set_coils(None, None)
        with pytest.raises(slrx.SlrxError):
            pl.run()


def test_set_coils_rejects_bad_arguments():
    say("coil argument checks")
    with slrx.Plan(16, 16, 4, 2, 2, 2) as pl:
        lib = slrx.lib()
        C = np.zeros((33, 16, 16), np.complex64)
        b = np.zeros((33, 4, 16, 16), np.complex64)
        ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        assert lib.slrx_set_coils(pl.handle, 33, ptr(C), ptr(b), slrx.SLRX_MEM_HOST) == -1
        assert lib.slrx_set_coils(pl.handle, -1, ptr(C), ptr(b), slrx.SLRX_MEM_HOST) == -1
        assert lib.slrx_set_coils(pl.handle, 2, None, ptr(b), slrx.SLRX_MEM_HOST) == -1
        assert lib.slrx_set_coils(pl.handle, 2, ptr(C), None, slrx.SLRX_MEM_HOST) == -1
        assert lib.slrx_set_coils(pl.handle, 2, ptr(C), ptr(b), 7) == -1
        assert lib.slrx_set_coils(pl.handle, 0, None, None, slrx.SLRX_MEM_HOST) == 0
