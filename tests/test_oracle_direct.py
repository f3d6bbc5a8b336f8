"""Pins of the oracle's IRLS-direct functions (the method without the FFT-based
approximations that the paper compares with in Sec. IV and Fig. 2: linear
convolutions in all three dimensions, both sub-problems on the explicit lifting):

* the linear lifting against SciPy's 3-D convolution in 'valid' mode of the
  centred k-space with the filter (an independent library routine);
* the adjoint against the definition of the adjoint (inner products);
* k-space that vanishes within N - 1 samples of the borders of the centred grid:
  every circular shift that is not a linear one then reads only zeros, so the Gram
  matrix and the normal operator equal those of the (separately pinned) circular
  lifting of the main method;
* the IRLS loop against a dense implementation that builds the operator's matrix
  from the lifting's matrix and solves it exactly;
* eps^(0) from the largest singular value of the explicit lifting.
"""
import numpy as np
import pytest
import scipy.signal

import oracle


def crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("T,P,Q,N1,N2,M", [(5, 8, 6, 3, 2, 2), (4, 6, 8, 2, 3, 3), (6, 8, 8, 1, 1, 4)])
def test_linear_lifting_is_a_valid_convolution(T, P, Q, N1, N2, M):
    rng = np.random.default_rng(T * 100 + N1 * 10 + N2)
    x = crandn(rng, T, P, Q)
    u = crandn(rng, M * N1 * N2)
    X = oracle.lift_linear(x, N1, N2, M)
    assert X.shape == ((T - M + 1) * (P - N1 + 1) * (Q - N2 + 1), M * N1 * N2)
    xc = np.fft.fftshift(x, axes=(1, 2))
    a1, a2 = oracle.filter_offsets(N1, N2)
    K = np.zeros((M, N1, N2), complex)
    for m in range(M):
        for ia in range(N1 * N2):
            K[m, a1[ia] - a1.min(), a2[ia] - a2.min()] = u[m * N1 * N2 + ia]
    ref = scipy.signal.convolve(xc, K, mode="valid")
    np.testing.assert_allclose(X @ u, ref.ravel(), atol=1e-12 * np.abs(ref).max())


def test_linear_lifting_adjoint():
    rng = np.random.default_rng(7)
    T, P, Q, N1, N2, M = 5, 8, 8, 3, 3, 2
    x = crandn(rng, T, P, Q)
    X = oracle.lift_linear(x, N1, N2, M)
    Y = crandn(rng, *X.shape)
    lhs = np.vdot(X, Y)
    rhs = np.vdot(x, oracle.lift_linear_adjoint(Y, T, P, Q, N1, N2, M))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def banded(rng, T, P, Q, N1, N2):
    """k-space (DFT order) whose centred grid is zero within N - 1 samples of every border."""
    xc = np.zeros((T, P, Q), complex)
    xc[:, N1 - 1:P - N1 + 1, N2 - 1:Q - N2 + 1] = crandn(rng, T, P - 2 * N1 + 2, Q - 2 * N2 + 2)
    return np.fft.ifftshift(xc, axes=(1, 2))


def test_banded_kspace_linear_equals_circular():
    rng = np.random.default_rng(8)
    T, P, Q, N1, N2, M = 5, 12, 10, 3, 2, 2
    x = banded(rng, T, P, Q, N1, N2)
    np.testing.assert_allclose(oracle.gram_direct(x, N1, N2, M), oracle.gram(x, N1, N2, M), atol=1e-10)
    s = M * N1 * N2
    U, _ = np.linalg.qr(crandn(rng, s, s))
    alpha = rng.uniform(0.2, 3.0, s)
    H = oracle.weight_matrix(U, alpha)
    E = oracle.penalty_masks(U, alpha, N1, N2, M, P, Q)
    S = (rng.random((T, P, Q)) < 0.5).astype(float)
    v = banded(rng, T, P, Q, N1, N2)
    a = oracle.direct_normal_apply(v, S, H, 0.7, N1, N2, M)
    b = oracle.normal_apply(v, S, E, 0.7)
    np.testing.assert_allclose(a, b, atol=1e-10 * np.abs(b).max())


def lifting_matrix(T, P, Q, N1, N2, M):
    """The matrix of vec(lift_linear(x)) (row-major) as a function of vec(x)."""
    cols = []
    for k in range(T * P * Q):
        e = np.zeros(T * P * Q, complex)
        e[k] = 1.0
        cols.append(oracle.lift_linear(e.reshape(T, P, Q), N1, N2, M).ravel())
    return np.stack(cols, axis=1)


def test_irls_direct_equals_dense_solves():
    rng = np.random.default_rng(9)
    T, P, Q, N1, N2, M = 4, 6, 6, 2, 2, 2
    S = (rng.random((T, P, Q)) < 0.6).astype(float)
    b = S * crandn(rng, T, P, Q)
    lam, n_irls = 0.05, 3
    L = lifting_matrix(T, P, Q, N1, N2, M)
    m, s = L.shape[0] // (M * N1 * N2), M * N1 * N2
    x = b.copy()
    eps = None
    for _ in range(n_irls):
        X = (L @ x.ravel()).reshape(m, s)
        lamR, U = np.linalg.eigh(X.conj().T @ X)
        if eps is None:
            eps = 0.01 * lamR.max()
        H = (U * ((np.maximum(lamR, 0) + eps) ** (0.6 / 2 - 1))[None]) @ U.conj().T
        N = np.diag(S.ravel()) + lam * L.conj().T @ np.kron(np.eye(m), H.T) @ L
        x = np.linalg.solve(N, b.ravel()).reshape(T, P, Q)
        eps /= 1.4
    ref = np.fft.ifft2(x, norm="ortho")
    out = oracle.irls_direct(b, S, N1, N2, M, lam, n_irls, 300)
    np.testing.assert_allclose(out, ref, atol=1e-8 * np.abs(ref).max())


def test_irls_direct_eps_schedule():
    rng = np.random.default_rng(10)
    T, P, Q, N1, N2, M = 5, 8, 8, 3, 3, 2
    S = (rng.random((T, P, Q)) < 0.6).astype(float)
    b = S * crandn(rng, T, P, Q)
    tr = {}
    oracle.irls_direct(b, S, N1, N2, M, 0.1, 3, 2, trace=tr)
    top = np.linalg.svd(oracle.lift_linear(b, N1, N2, M), compute_uv=False)[0] ** 2
    assert np.isclose(tr["lambda_max"][0], top, rtol=1e-12)
    np.testing.assert_allclose(tr["eps"], [top / 100 / 1.4 ** k for k in range(3)], rtol=1e-12)
