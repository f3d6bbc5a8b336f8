"""GPU parity of each step of the IRLS hot path against the FP64 oracle.

Each test drives one entry point of the C ABI (through the thin binding) on
seeded inputs and compares element by element with the oracle on the same
inputs.  FP32 data path (complex64 FFTs, CG, penalty) and FP64 Gram /
eigen-decomposition / filter product: the bars below are relative Frobenius
errors derived from FP32 rounding (~6e-8 per operation, grown by the FFT
length and the conditioning of the step).
"""
import numpy as np
import pytest

import oracle
import workload
from tests.gpu_util import crandn, masks_to_pairs, nrmse, pairs, pairs_to_masks, say

pytestmark = pytest.mark.gpu

slrx = pytest.importorskip("paper_1704_04511_amd")

# (T, P, Q, N1, N2, M): several tiles, odd radices (96 = 16*3*2, 160 = 16*5*2,
# 192 = 16*4*3), even/odd filters, M = 1 and M = T, the largest frame count
# (T = 32) with the largest tap count (M = 8), one-wide filters (N1 = 1 or N2 = 1)
# on the spectral lag-sum route.
STEP_SHAPES = [
    (5, 16, 16, 3, 3, 2),
    (32, 16, 16, 2, 2, 8),
    (8, 64, 64, 5, 5, 3),
    (6, 32, 96, 4, 5, 3),
    (4, 160, 32, 3, 2, 4),
    (3, 192, 16, 2, 3, 1),
    (12, 8, 8, 1, 1, 1),
    (16, 128, 128, 9, 9, 5),
    (6, 16, 16, 2, 1, 1),
    (6, 16, 16, 1, 1, 3),
    (4, 32, 32, 1, 18, 1),
    (4, 32, 32, 16, 1, 2),
    (20, 256, 256, 15, 15, 5),
]


def problem(seed, T, P, Q, frac=0.4):
    rng = np.random.default_rng(seed)
    x = crandn(rng, T, P, Q).astype(np.complex64)
    S = (rng.random((T, P, Q)) < frac).astype(np.uint8)
    return rng, x, S


def make_plan(T, P, Q, N1, N2, M, lam=1e-2, n_irls=1, n_cg=5):
    return slrx.Plan(P, Q, T, N1, N2, M, slrx.make_params(lam=lam, n_irls=n_irls, n_cg=n_cg))


@pytest.mark.parametrize("shape", STEP_SHAPES)
def test_gram_matches_oracle(shape):
    T, P, Q, N1, N2, M = shape
    say(f"gram {shape}")
    rng, x, _ = problem(1, T, P, Q)
    S = np.ones((T, P, Q), np.uint8)
    with make_plan(*shape) as pl:
        pl.set_kspace(x)
        pl.set_mask(S)
        R = pl.step_gram()
    R_ref = oracle.gram(x.astype(np.complex128), N1, N2, M)
    err = np.linalg.norm(R - R_ref) / np.linalg.norm(R_ref)
    assert err < 2e-6, err
    assert np.abs(R - R.conj().T).max() <= 1e-12 * np.abs(R).max()
    # every (m, m') block on its own scale, so that no block hides under the global norm
    NN = N1 * N2
    for m in range(M):
        for mp in range(M):
            blk = (slice(m * NN, (m + 1) * NN), slice(mp * NN, (mp + 1) * NN))
            assert np.abs(R[blk] - R_ref[blk]).max() <= 1e-5 * np.abs(R_ref[blk]).max(), (m, mp)


@pytest.mark.parametrize("shape", STEP_SHAPES)
def test_weights_and_masks_match_oracle(shape):
    T, P, Q, N1, N2, M = shape
    say(f"weights {shape}")
    rng, x, _ = problem(2, T, P, Q)
    S = np.ones((T, P, Q), np.uint8)
    R_ref = oracle.gram(x.astype(np.complex128), N1, N2, M)
    lam_ref = np.linalg.eigvalsh(R_ref)
    eps = 0.01 * lam_ref.max()
    with make_plan(*shape) as pl:
        pl.set_kspace(x)
        pl.set_mask(S)
        lam, H, E = pl.step_weights(eps)
    assert np.abs(lam - lam_ref).max() < 2e-6 * lam_ref.max()
    # each eigenvalue relative to itself (the small ones set the largest weights): a
    # perturbation dR of the Gram matrix moves lambda_i by at most ||dR|| ~ 1e-7 lambda_max
    assert np.all(np.abs(lam - lam_ref) <= 1e-5 * lam_ref + 2e-7 * lam_ref.max())
    ev, U, alpha = oracle.eig_weights(R_ref, eps, 0.6)
    H_ref = oracle.weight_matrix(U, alpha)
    assert nrmse(H, H_ref) < 2e-5
    E_ref = oracle.penalty_masks(U, alpha, N1, N2, M, P, Q)
    for w, (m, mp) in enumerate(pairs(M)):
        assert nrmse(E[w], E_ref[m, mp]) < 2e-5, (m, mp)


@pytest.mark.parametrize("shape", [(8, 64, 64, 16, 18, 8), (8, 64, 64, 19, 19, 8), (8, 64, 64, 15, 25, 8)])
def test_weights_at_the_largest_filters(shape):
    """Gram sizes 2304, 2888 and 3000 (the largest the own eigensolver chain takes):
    the tridiagonalisation's long-column kernel instances (more than 2048 entries per
    column) against the oracle's eigenvalues, H and masks."""
    T, P, Q, N1, N2, M = shape
    say(f"weights, large filter {shape}")
    rng, x, _ = problem(7, T, P, Q)
    R_ref = oracle.gram(x.astype(np.complex128), N1, N2, M)
    lam_ref = np.linalg.eigvalsh(R_ref)
    eps = 0.01 * lam_ref.max()
    with make_plan(*shape) as pl:
        pl.set_kspace(x)
        pl.set_mask(np.ones((T, P, Q), np.uint8))
        lam, H, E = pl.step_weights(eps)
    assert np.all(np.abs(lam - lam_ref) <= 1e-5 * lam_ref + 2e-7 * lam_ref.max())
    ev, U, alpha = oracle.eig_weights(R_ref, eps, 0.6)
    assert nrmse(H, oracle.weight_matrix(U, alpha)) < 2e-5
    E_ref = oracle.penalty_masks(U, alpha, N1, N2, M, P, Q)
    for w, (m, mp) in enumerate(pairs(M)):
        assert nrmse(E[w], E_ref[m, mp]) < 2e-5, (m, mp)


@pytest.mark.parametrize("shape", [(4, 32, 32, 5, 19, 1), (8, 32, 32, 4, 4, 6), (4, 16, 128, 1, 97, 1),
                                   (4, 32, 32, 7, 7, 2), (4, 64, 64, 1, 43, 3), (4, 64, 64, 2, 43, 3)])
def test_weights_around_the_last_columns_kernel(shape):
    """Gram sizes 95, 96, 97, 98, 129 and 258: the tridiagonalisation's last 96
    columns run in one register-resident workgroup, so 95 and 96 never launch a
    column kernel, 97 and 98 hand one or two columns' pending update to it, 129
    hands it 33, and 258 crosses from two vector entries per thread to one in the
    column launches."""
    T, P, Q, N1, N2, M = shape
    say(f"weights around the last-columns kernel {shape} (s = {N1 * N2 * M})")
    rng, x, _ = problem(11, T, P, Q)
    R_ref = oracle.gram(x.astype(np.complex128), N1, N2, M)
    lam_ref = np.linalg.eigvalsh(R_ref)
    eps = 0.01 * lam_ref.max()
    with make_plan(*shape) as pl:
        pl.set_kspace(x)
        pl.set_mask(np.ones((T, P, Q), np.uint8))
        lam, H, E = pl.step_weights(eps)
    assert np.all(np.abs(lam - lam_ref) <= 1e-5 * lam_ref + 2e-7 * lam_ref.max())
    ev, U, alpha = oracle.eig_weights(R_ref, eps, 0.6)
    assert nrmse(H, oracle.weight_matrix(U, alpha)) < 2e-5
    E_ref = oracle.penalty_masks(U, alpha, N1, N2, M, P, Q)
    for w, (m, mp) in enumerate(pairs(M)):
        assert nrmse(E[w], E_ref[m, mp]) < 2e-5, (m, mp)


def masks_from_H(H, N1, N2, M, P, Q):
    """Masks straight from H: the lag sums w_{m',m}[a' - a] of the (m', m) block, then
    E(r) = sum_Delta w[Delta] e^{+2 pi i (Delta1 r1 / P + Delta2 r2 / Q)} (FP64)."""
    NN, L1, L2 = N1 * N2, 2 * N1 - 1, 2 * N2 - 1
    a1, a2 = np.divmod(np.arange(NN), N2)
    d1 = (a1[:, None] - a1[None, :] + N1 - 1).ravel()  # row a', column a
    d2 = (a2[:, None] - a2[None, :] + N2 - 1).ravel()
    F1 = np.exp(2j * np.pi * np.outer(np.arange(P), np.arange(L1) - (N1 - 1)) / P)
    F2 = np.exp(2j * np.pi * np.outer(np.arange(Q), np.arange(L2) - (N2 - 1)) / Q)
    out = []
    for m, mp in pairs(M):
        w = np.zeros((L1, L2), np.complex128)
        np.add.at(w, (d1, d2), H[mp * NN:(mp + 1) * NN, m * NN:(m + 1) * NN].ravel())
        out.append(F1 @ w @ F2.T)
    return np.stack(out)


@pytest.mark.parametrize("shape", STEP_SHAPES[:-1])
def test_masks_agree_with_the_returned_filter_matrix(shape):
    """The masks of one weights step (from the filter spectra where the shape allows,
    else from H's diagonal sums) against masks synthesised on the host from the H the
    same call returns: two routes to the same quantity, FP64 up to the FP32 store."""
    T, P, Q, N1, N2, M = shape
    say(f"masks vs H {shape}")
    rng, x, _ = problem(6, T, P, Q)
    lam_max = np.linalg.eigvalsh(oracle.gram(x.astype(np.complex128), N1, N2, M)).max()
    with make_plan(*shape) as pl:
        pl.set_kspace(x)
        pl.set_mask(np.ones((T, P, Q), np.uint8))
        lam, H, E = pl.step_weights(0.01 * lam_max)
    ref = masks_from_H(H, N1, N2, M, P, Q)
    assert nrmse(E, ref) < 2e-6


@pytest.mark.parametrize("shape", STEP_SHAPES)
def test_normal_operator_matches_oracle(shape):
    T, P, Q, N1, N2, M = shape
    say(f"apply {shape}")
    rng, x, S = problem(3, T, P, Q)
    R = oracle.gram(x.astype(np.complex128), N1, N2, M)
    ev, U, alpha = oracle.eig_weights(R, 0.05 * np.linalg.eigvalsh(R).max(), 0.6)
    E = oracle.penalty_masks(U, alpha, N1, N2, M, P, Q)
    Ew = masks_to_pairs(E)
    v = crandn(rng, T, P, Q).astype(np.complex64)
    lam = 0.7 / np.abs(E).max()
    with make_plan(*shape, lam=lam) as pl:
        pl.set_kspace(x)
        pl.set_mask(S)
        out = pl.step_apply(Ew, v)
    ref = oracle.normal_apply(v.astype(np.complex128), S, pairs_to_masks(Ew, M), lam)
    assert nrmse(out, ref) < 2e-6
    assert max(nrmse(out[t], ref[t]) for t in range(T)) < 4e-6  # every frame on its own


@pytest.mark.parametrize("shape", STEP_SHAPES[:5])
def test_cg_matches_oracle(shape):
    T, P, Q, N1, N2, M = shape
    say(f"cg {shape}")
    rng, x, S = problem(4, T, P, Q, frac=0.5)
    b = (S * x).astype(np.complex64)
    R = oracle.gram(b.astype(np.complex128), N1, N2, M)
    ev, U, alpha = oracle.eig_weights(R, 0.02 * np.linalg.eigvalsh(R).max(), 0.6)
    E = oracle.penalty_masks(U, alpha, N1, N2, M, P, Q)
    Ew = masks_to_pairs(E)
    lam = 0.5 / np.abs(E).max()
    for n_cg in (0, 1, 3, 12):
        with make_plan(*shape, lam=lam) as pl:
            pl.set_kspace(b)
            pl.set_mask(S)
            pl.step_cg(Ew, n_cg)
            img = pl.images()
        Sd = S.astype(np.float64)
        xk = oracle.cg(lambda v: oracle.normal_apply(v, Sd, pairs_to_masks(Ew, M), lam),
                       Sd * b, Sd * b.astype(np.complex128), n_cg)
        ref = oracle.idft2(xk)
        assert nrmse(img, ref) < 1e-5, n_cg
        assert max(nrmse(img[t], ref[t]) for t in range(T)) < 2e-5, n_cg  # every frame on its own


def test_fft_roundtrip_and_kspace_output():
    # with E = 0 and a full mask the operator is the identity through F^H then F
    T, P, Q, N1, N2, M = 4, 96, 160, 3, 3, 2
    say("fft roundtrip 96x160")
    rng, x, _ = problem(5, T, P, Q)
    S = np.ones((T, P, Q), np.uint8)
    Ew = np.zeros((3, P, Q), np.complex64)
    with make_plan(T, P, Q, N1, N2, M) as pl:
        pl.set_kspace(x)
        pl.set_mask(S)
        out = pl.step_apply(Ew, x)
    assert nrmse(out, x) < 1e-6
