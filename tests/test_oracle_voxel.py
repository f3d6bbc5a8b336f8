"""Pins of the oracle's HLR-Voxel functions (the pixel-wise Hankel low-rank prior of
Sec. II.E, eq. ``eq: MORASA-objective``, solved by IRLS as the paper does in Sec. IV):

* the per-pixel Gram matrices against the explicitly built per-pixel Toeplitz
  matrices (brute force);
* the penalty through the per-pixel masks against sum_r ||T_r H_r^(1/2)||_F^2 with
  H_r a fractional matrix power computed by Schur-Pade (an independent route; pins
  the conjugation of the masks);
* the annihilation property per pixel: a noiseless sum of K damped exponentials
  with pixel-dependent decays gives G_r of rank K (M - K zero eigenvalues);
* a one-pixel image, where the 3-D lifting with a 1 x 1 x M filter is the
  pixel's own Toeplitz matrix: irls_voxel equals the main irls outer iteration by
  outer iteration.
"""
import numpy as np
import pytest
import scipy.linalg

import oracle


def series(rng, T, P, Q, K=2, noise=0.0):
    """rho_t(r) = sum_k a_k(r) beta_k(r)^t, pixel-dependent amplitudes and decays."""
    a = rng.standard_normal((K, P, Q)) + 1j * rng.standard_normal((K, P, Q))
    # well separated frequencies (component k near 1.5 k rad), so K components stay of rank K
    phase = 1.5 * np.arange(K)[:, None, None] + rng.uniform(-0.3, 0.3, (K, P, Q))
    beta = rng.uniform(0.6, 0.95, (K, P, Q)) * np.exp(1j * phase)
    t = np.arange(T)[:, None, None, None]
    rho = (a[None] * beta[None] ** t).sum(axis=1)
    rho = rho + noise * (rng.standard_normal(rho.shape) + 1j * rng.standard_normal(rho.shape))
    return oracle.dft2(rho)


def test_voxel_gram_equals_explicit_toeplitz_gram():
    rng = np.random.default_rng(1)
    xhat = series(rng, 7, 3, 4, noise=0.3)
    M = 3
    Tm = oracle.voxel_lift(xhat, M)
    G = oracle.voxel_gram(xhat, M)
    ref = np.einsum("pqnm,pqnk->pqmk", np.conj(Tm), Tm)
    assert np.abs(G - ref).max() <= 1e-13 * np.abs(ref).max()
    # and each Toeplitz matrix holds the pixel's series: row n, column m is rho_{n-m}
    rho = oracle.idft2(xhat)
    assert np.allclose(Tm[1, 2, :, 0], rho[M - 1:, 1, 2]) and np.allclose(Tm[1, 2, :, M - 1], rho[:7 - M + 1, 1, 2])


@pytest.mark.parametrize("p", [0.6, 1.0])
def test_voxel_penalty_equals_schatten_weighted_toeplitz_norms(p):
    rng = np.random.default_rng(2)
    xhat = series(rng, 8, 3, 3, noise=0.1)
    M, eps = 3, 0.05
    E, lmax = oracle.voxel_masks(xhat, M, eps, p)
    rho = oracle.idft2(xhat)
    J = oracle.penalty_value(rho, E)
    Tm = oracle.voxel_lift(xhat, M)
    ref = 0.0
    for r1 in range(3):
        for r2 in range(3):
            T_r = Tm[r1, r2]
            H = scipy.linalg.fractional_matrix_power(T_r.conj().T @ T_r + eps * np.eye(M), p / 2 - 1)
            ref += np.linalg.norm(T_r @ scipy.linalg.sqrtm(H), "fro") ** 2
    assert abs(J - ref) <= 1e-10 * abs(ref)
    assert np.isclose(lmax, max(np.linalg.eigvalsh(Tm[i, j].conj().T @ Tm[i, j]).max()
                                for i in range(3) for j in range(3)))


def test_voxel_gram_of_k_exponentials_has_rank_k():
    rng = np.random.default_rng(3)
    M, K = 5, 2
    G = oracle.voxel_gram(series(rng, 12, 4, 4, K=K), M)
    ev = np.linalg.eigvalsh(G)                      # per pixel, ascending
    assert np.all(ev[..., : M - K] <= 1e-10 * ev[..., -1:])
    assert np.all(ev[..., M - K] > 1e-6 * ev[..., -1])


def test_one_pixel_voxel_irls_equals_main_irls_with_1x1xM_filter():
    rng = np.random.default_rng(4)
    T, M = 10, 3
    xhat = series(rng, T, 1, 1, noise=0.05)
    S = (rng.random((T, 1, 1)) < 0.7).astype(np.float64)
    S[0] = 1.0
    b = S * xhat
    tr_v, tr_m = {}, {}
    a = oracle.irls_voxel(b, S, M, 0.3, 5, 4, trace=tr_v)
    ref = oracle.irls(b, S, 1, 1, M, 0.3, 5, 4, trace=tr_m)
    assert np.abs(a - ref).max() <= 1e-10 * np.abs(ref).max()
    np.testing.assert_allclose(tr_v["eps"], tr_m["eps"], rtol=1e-12)
    np.testing.assert_allclose(tr_v["lambda_max"], tr_m["lambda_max"], rtol=1e-12)


def test_voxel_eps_schedule_over_several_pixels():
    """eps^(0) is a hundredth of the largest eigenvalue over every pixel's Toeplitz
    Gram matrix of the zero-filled data (Sec. III.C), divided by 1.4 per iteration."""
    rng = np.random.default_rng(5)
    T, P, Q, M = 8, 3, 2, 3
    xhat = series(rng, T, P, Q, noise=0.1)
    S = (rng.random((T, P, Q)) < 0.6).astype(np.float64)
    b = S * xhat
    tr = {}
    oracle.irls_voxel(b, S, M, 0.2, 3, 2, trace=tr)
    Tm = oracle.voxel_lift(b, M)
    top = max(np.linalg.svd(Tm[i, j], compute_uv=False)[0] ** 2 for i in range(P) for j in range(Q))
    assert np.isclose(tr["lambda_max"][0], top, rtol=1e-12)
    np.testing.assert_allclose(tr["eps"], [top / 100 / 1.4 ** k for k in range(3)], rtol=1e-12)


def test_one_pixel_voxel_irls_with_coils_equals_main_irls():
    """The multichannel least-squares step (Sec. II.A) under the pixel-wise prior: on a
    one-pixel image it is the main loop's with the 1 x 1 x M filter and the same coils."""
    rng = np.random.default_rng(6)
    T, M, nc = 9, 3, 3
    xhat = series(rng, T, 1, 1, noise=0.05)
    C = rng.standard_normal((nc, 1, 1)) + 1j * rng.standard_normal((nc, 1, 1))
    S = (rng.random((T, 1, 1)) < 0.7).astype(np.float64)
    S[0] = 1.0
    b = oracle.coil_forward(xhat, S, C)
    a = oracle.irls_voxel(b, S, M, 0.3, 4, 4, coils=C)
    ref = oracle.irls(b, S, 1, 1, M, 0.3, 4, 4, coils=C)
    assert np.abs(a - ref).max() <= 1e-10 * np.abs(ref).max()
