"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: an
explicitly built DFT matrix, a brute-force convolution, the explicitly built
lifted matrix, closed forms for traces and null-space dimensions, a library
fractional matrix power, dense linear solves and explicit Krylov minimisers,
and closed-form special cases of the whole IRLS loop.  A plausible mistake in
the oracle (a dropped term, a wrong sign or index, a conjugated or transposed
operand) breaks at least one of them.
"""
import numpy as np
import pytest
import scipy.linalg

import oracle


def crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def dft_matrix(N):
    k = np.arange(N)
    return np.exp(-2j * np.pi * np.outer(k, k) / N) / np.sqrt(N)


# ------------------------------------------------------------------ DFT (F)
@pytest.mark.parametrize("P,Q", [(2, 3), (4, 4), (5, 6), (8, 12), (15, 10), (16, 16), (6, 96)])
def test_dft_matches_naive_matrix(P, Q):
    rng = np.random.default_rng(P * 100 + Q)
    a = crandn(rng, 3, P, Q)
    ref = np.einsum("kp,tpq,lq->tkl", dft_matrix(P), a, dft_matrix(Q))
    np.testing.assert_allclose(oracle.dft2(a), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    # inverse and Parseval (unitary F)
    np.testing.assert_allclose(oracle.idft2(oracle.dft2(a)), a, atol=1e-12)
    assert abs(np.linalg.norm(oracle.dft2(a)) - np.linalg.norm(a)) < 1e-11 * np.linalg.norm(a)


# ------------------------------------------------------------ lifting T(x)
def brute_conv(x, d, N1, N2, M):
    """y[n, w] = sum_{m, a} x_{n-m}[(w - a) mod (P, Q)] d[m, a], n = M-1..T-1 (loops)."""
    T, P, Q = x.shape
    a1, a2 = oracle.filter_offsets(N1, N2)
    y = np.zeros((T - M + 1, P, Q), complex)
    for n in range(M - 1, T):
        for w1 in range(P):
            for w2 in range(Q):
                acc = 0j
                for m in range(M):
                    for ia in range(N1 * N2):
                        acc += x[n - m, (w1 - a1[ia]) % P, (w2 - a2[ia]) % Q] * d[m * N1 * N2 + ia]
                y[n - M + 1, w1, w2] = acc
    return y


def fft_conv(x, d, N1, N2, M):
    """Same convolution by the convolution theorem: circular in space, valid in n."""
    T, P, Q = x.shape
    a1, a2 = oracle.filter_offsets(N1, N2)
    y = np.zeros((T - M + 1, P, Q), complex)
    for m in range(M):
        frame = np.zeros((P, Q), complex)
        np.add.at(frame, (a1 % P, a2 % Q), d[m * N1 * N2:(m + 1) * N1 * N2])
        Df = np.fft.fft2(frame)
        for n in range(M - 1, T):
            y[n - M + 1] += np.fft.ifft2(np.fft.fft2(x[n - m]) * Df)
    return y


@pytest.mark.parametrize("T,P,Q,N1,N2,M", [(5, 8, 6, 3, 3, 2), (4, 5, 7, 2, 3, 3), (3, 4, 4, 1, 1, 1), (6, 6, 6, 4, 2, 6)])
def test_lift_is_hybrid_convolution(T, P, Q, N1, N2, M):
    rng = np.random.default_rng(7)
    x = crandn(rng, T, P, Q)
    d = crandn(rng, N1 * N2 * M)
    L = oracle.lift(x, N1, N2, M)
    assert L.shape == ((T - M + 1) * P * Q, N1 * N2 * M)
    y = (L @ d).reshape(T - M + 1, P, Q)
    np.testing.assert_allclose(y, brute_conv(x, d, N1, N2, M), atol=1e-12)
    np.testing.assert_allclose(y, fft_conv(x, d, N1, N2, M), atol=1e-11)


# -------------------------------------------------------------------- Gram
GRAM_SHAPES = [(5, 8, 6, 3, 3, 2), (4, 5, 7, 2, 3, 3), (6, 6, 6, 4, 2, 6), (3, 4, 4, 1, 1, 1),
               (5, 4, 4, 4, 4, 2), (7, 9, 5, 5, 3, 4)]


@pytest.mark.parametrize("T,P,Q,N1,N2,M", GRAM_SHAPES)
def test_gram_fft_equals_explicit(T, P, Q, N1, N2, M):
    rng = np.random.default_rng(11)
    x = crandn(rng, T, P, Q)
    L = oracle.lift(x, N1, N2, M)
    R_ref = L.conj().T @ L
    R = oracle.gram(x, N1, N2, M)
    np.testing.assert_allclose(R, R_ref, rtol=0, atol=1e-12 * np.abs(R_ref).max())


@pytest.mark.parametrize("T,P,Q,N1,N2,M", GRAM_SHAPES)
def test_gram_trace_hermitian_psd(T, P, Q, N1, N2, M):
    rng = np.random.default_rng(13)
    x = crandn(rng, T, P, Q)
    R = oracle.gram(x, N1, N2, M)
    tr = N1 * N2 * sum(np.linalg.norm(x[n - m]) ** 2 for m in range(M) for n in range(M - 1, T))
    assert abs(np.trace(R).real - tr) < 1e-11 * tr
    assert np.abs(R - R.conj().T).max() < 1e-12 * np.abs(R).max()
    ev = np.linalg.eigvalsh(R)
    assert ev.min() > -1e-12 * ev.max()


def exp_series(rng, T, P, Q, betas):
    """rho_t(r) = sum_k a_k(r) beta_k(r)^t with generic complex amplitudes."""
    img = np.zeros((T, P, Q), complex)
    t = np.arange(T)[:, None, None]
    for beta in betas:
        a = crandn(rng, P, Q)
        img += a[None] * np.asarray(beta)[None] ** t if np.ndim(beta) else a[None] * beta ** t
    return img


@pytest.mark.parametrize("K,expect", [(1, 27), (2, 18)])
def test_nullity_constant_exponentials(K, expect):
    # Sec. II.C: filters d = c (x) e annihilate the data; with space-invariant
    # beta_k the null space of T has dimension N1 N2 (M - K) exactly.
    rng = np.random.default_rng(3 + K)
    T, P, Q, N1, N2, M = 8, 8, 8, 3, 3, 4
    img = exp_series(rng, T, P, Q, [0.9, 0.55][:K])
    R = oracle.gram(oracle.dft2(img), N1, N2, M)
    ev = np.linalg.eigvalsh(R)
    nullity = int(np.sum(ev < 1e-10 * ev.max()))
    assert nullity == expect == N1 * N2 * (M - K)


def test_nullity_bandlimited_parameter():
    # beta(r) = 0.8 + 0.1 cos(2 pi r1/P): minimal filter support 3 x 1 x 2, so
    # |Lambda:Theta| = (N1-2) N2 (M-1) null vectors (Sec. II.C bounds).
    rng = np.random.default_rng(5)
    T, P, Q, N1, N2, M = 8, 12, 12, 5, 5, 3
    r1 = np.arange(P)[:, None] * np.ones((1, Q))
    beta = 0.8 + 0.1 * np.cos(2 * np.pi * r1 / P)
    img = crandn(rng, P, Q)[None] * beta[None] ** np.arange(T)[:, None, None]
    R = oracle.gram(oracle.dft2(img), N1, N2, M)
    ev = np.linalg.eigvalsh(R)
    nullity = int(np.sum(ev < 1e-10 * ev.max()))
    bound = (N1 - 2) * N2 * (M - 1)
    assert nullity >= bound
    assert nullity == bound  # generic amplitudes: no extra null vectors


def test_noise_lifts_null_space():
    rng = np.random.default_rng(6)
    T, P, Q, N1, N2, M = 8, 8, 8, 3, 3, 4
    x = oracle.dft2(exp_series(rng, T, P, Q, [0.9]))
    x += 1e-3 * np.abs(x).max() * crandn(rng, *x.shape)
    ev = np.linalg.eigvalsh(oracle.gram(x, N1, N2, M))
    assert int(np.sum(ev < 1e-10 * ev.max())) == 0


# ----------------------------------------------------------------- weights
def test_weight_matrix_is_fractional_power():
    # H = (R + eps I)^(p/2 - 1) (eq. weight-update); check H (R + eps I)^(1 - p/2) = I
    # with the fractional power from a Schur-Pade library routine.
    rng = np.random.default_rng(8)
    x = crandn(rng, 5, 6, 6)
    R = oracle.gram(x, 3, 3, 2)
    eps = 1e-3 * np.linalg.eigvalsh(R).max()
    for p in (0.6, 0.7, 1.0, 0.0):
        lam, U, alpha = oracle.eig_weights(R, eps, p)
        H = oracle.weight_matrix(U, alpha)
        F = scipy.linalg.fractional_matrix_power(R + eps * np.eye(len(R)), 1 - p / 2)
        np.testing.assert_allclose(H @ F, np.eye(len(R)), atol=1e-9)


def test_schatten_identity():
    # ||Y||_p = (1/p) Tr[(Y^H Y)^(p/2)] = (1/p) ||Y H^(1/2)||_F^2 (eq. irls_identity)
    rng = np.random.default_rng(9)
    x = crandn(rng, 5, 6, 6)
    Y = oracle.lift(x, 3, 3, 2)
    sv = np.linalg.svd(Y, compute_uv=False)
    p = 0.6
    lam, U, alpha = oracle.eig_weights(Y.conj().T @ Y, 0.0, p)
    H = oracle.weight_matrix(U, alpha)
    lhs = np.sum(sv ** p) / p
    rhs = np.trace(Y @ H @ Y.conj().T).real / p
    assert abs(lhs - rhs) < 1e-9 * lhs


# ------------------------------------------------------------------- masks
MASK_SHAPES = [(6, 8, 6, 3, 3, 2), (5, 5, 7, 2, 3, 3), (4, 6, 6, 4, 4, 1), (6, 6, 6, 4, 2, 6)]


@pytest.mark.parametrize("T,P,Q,N1,N2,M", MASK_SHAPES)
def test_penalty_masks_equal_explicit_filter_norms(T, P, Q, N1, N2, M):
    # J(x) = sum_i alpha_i ||T(x) u_i||^2 (eq. ls_update with h^(i) = sqrt(alpha_i) u_i^*)
    rng = np.random.default_rng(21)
    x0 = crandn(rng, T, P, Q)
    x = crandn(rng, T, P, Q)
    R = oracle.gram(x0, N1, N2, M)
    lam, U, alpha = oracle.eig_weights(R, 0.05 * np.linalg.eigvalsh(R).max(), 0.6)
    E = oracle.penalty_masks(U, alpha, N1, N2, M, P, Q, chunk=7)
    L = oracle.lift(x, N1, N2, M)
    J_ref = float(np.sum(alpha * np.linalg.norm(L @ U, axis=0) ** 2))
    J = oracle.penalty_value(oracle.idft2(x), E)
    assert abs(J - J_ref) < 1e-10 * J_ref
    # per-pixel masks are Hermitian PSD
    Er = np.moveaxis(E.reshape(M, M, -1), -1, 0)
    assert np.abs(Er - np.conj(np.swapaxes(Er, 1, 2))).max() < 1e-10 * np.abs(Er).max()
    assert np.linalg.eigvalsh(Er).min() > -1e-10 * np.abs(Er).max()


@pytest.mark.parametrize("T,P,Q,N1,N2,M", MASK_SHAPES)
def test_penalty_masks_equal_weight_matrix_diagonal_sums(T, P, Q, N1, N2, M):
    # Second, independent route: E_r[m,m'] = sum_Delta w_{m',m}[Delta] e^{+2 pi i Delta.r},
    # w_{m',m}[Delta] = sum_{a' - a = Delta} H[(m',a'),(m,a)], H = U diag(alpha) U^H.
    rng = np.random.default_rng(22)
    R = oracle.gram(crandn(rng, T, P, Q), N1, N2, M)
    lam, U, alpha = oracle.eig_weights(R, 0.02 * np.linalg.eigvalsh(R).max(), 0.7)
    E = oracle.penalty_masks(U, alpha, N1, N2, M, P, Q)
    H = (U * alpha) @ U.conj().T
    a1, a2 = oracle.filter_offsets(N1, N2)
    NN = N1 * N2
    r1 = np.arange(P)[:, None]
    r2 = np.arange(Q)[None, :]
    for m in range(M):
        for mp in range(M):
            acc = np.zeros((P, Q), complex)
            for ia in range(NN):          # a  (column side, tap m)
                for ib in range(NN):      # a' (row side, tap m')
                    d1 = a1[ib] - a1[ia]
                    d2 = a2[ib] - a2[ia]
                    acc += H[mp * NN + ib, m * NN + ia] * np.exp(2j * np.pi * (d1 * r1 / P + d2 * r2 / Q))
            np.testing.assert_allclose(E[m, mp], acc, atol=1e-10 * np.abs(E).max())


# ---------------------------------------------------------------- operator
def tiny_system(seed=31, T=5, P=6, Q=6, N1=3, N2=3, M=2, lam=0.3):
    rng = np.random.default_rng(seed)
    x0 = crandn(rng, T, P, Q)
    S = (rng.random((T, P, Q)) < 0.4).astype(float)
    R = oracle.gram(x0, N1, N2, M)
    ev, U, alpha = oracle.eig_weights(R, 0.05 * np.linalg.eigvalsh(R).max(), 0.6)
    E = oracle.penalty_masks(U, alpha, N1, N2, M, P, Q)
    return rng, S, U, alpha, E, lam, (T, P, Q, N1, N2, M)


def test_normal_operator_adjoint_and_quadratic_form():
    rng, S, U, alpha, E, lam, (T, P, Q, N1, N2, M) = tiny_system()
    A = lambda v: oracle.normal_apply(v, S, E, lam)
    u = crandn(rng, T, P, Q)
    v = crandn(rng, T, P, Q)
    lhs = np.vdot(A(u), v)
    rhs = np.vdot(u, A(v))
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)
    # <x, A x> = ||S x||^2 + lam sum_i alpha_i ||T(x) u_i||^2
    q = np.vdot(u, A(u))
    L = oracle.lift(u, N1, N2, M)
    ref = np.linalg.norm(S * u) ** 2 + lam * np.sum(alpha * np.linalg.norm(L @ U, axis=0) ** 2)
    assert abs(q.imag) < 1e-10 * abs(q) and abs(q.real - ref) < 1e-10 * ref


def explicit_normal_matrix(S, U, alpha, lam, dims):
    """N = diag(S) + lam sum_i alpha_i L_i^H L_i with L_i x = T(x) u_i, built column by column."""
    T, P, Q, N1, N2, M = dims
    n = T * P * Q
    cols = []
    for j in range(n):
        e = np.zeros(n, complex)
        e[j] = 1
        cols.append(oracle.lift(e.reshape(T, P, Q), N1, N2, M) @ U)
    Ls = np.stack(cols, axis=-1)  # (rows, s, n): Ls[:, i, :] = L_i
    N = np.diag(S.ravel().astype(complex))
    for i in range(U.shape[1]):
        Li = Ls[:, i, :]
        N += lam * alpha[i] * (Li.conj().T @ Li)
    return N


def test_normal_operator_equals_explicit_matrix():
    rng, S, U, alpha, E, lam, dims = tiny_system(T=4, P=4, Q=4, N1=2, N2=3, M=2)
    N = explicit_normal_matrix(S, U, alpha, lam, dims)
    v = crandn(rng, *dims[:3])
    np.testing.assert_allclose(oracle.normal_apply(v, S, E, lam).ravel(), N @ v.ravel(), atol=1e-10)


def test_cg_reaches_dense_solve_and_krylov_minimiser():
    rng, S, U, alpha, E, lam, dims = tiny_system(T=4, P=4, Q=4, N1=2, N2=3, M=2, lam=0.5)
    N = explicit_normal_matrix(S, U, alpha, lam, dims)
    b = S * crandn(rng, *dims[:3])
    x0 = crandn(rng, *dims[:3])
    A = lambda v: oracle.normal_apply(v, S, E, lam)
    xs = np.linalg.solve(N, b.ravel())
    x_cg = oracle.cg(A, b, x0, 400)
    np.testing.assert_allclose(x_cg.ravel(), xs, atol=1e-8 * np.abs(xs).max())
    # k steps of CG minimise the N-norm error over x0 + K_k(N, r0)
    r0 = b.ravel() - N @ x0.ravel()
    for k in (1, 2, 3, 5):
        K = np.stack([np.linalg.matrix_power(N, j) @ r0 for j in range(k)], axis=1)
        V, _ = np.linalg.qr(K)
        y = np.linalg.solve(V.conj().T @ N @ V, V.conj().T @ r0)
        x_ref = x0.ravel() + V @ y
        x_k = oracle.cg(A, b, x0, k).ravel()
        np.testing.assert_allclose(x_k, x_ref, atol=1e-8 * np.abs(x_ref).max())


# -------------------------------------------------------------- whole loop
def test_irls_scalar_filter_closed_form():
    # Filter 1x1x1 (s = 1): R = ||x||^2, E = alpha, G = alpha I, so each LS step
    # gives x = S b / (1 + lam alpha_n), alpha_n = (||x^(n-1)||^2 + eps_{n-1})^(p/2-1),
    # eps_0 = ||x^(0)||^2/100, eps_n = eps_{n-1}/1.4.
    rng = np.random.default_rng(41)
    T, P, Q = 4, 6, 5
    S = (rng.random((T, P, Q)) < 0.5).astype(np.uint8)
    b = S * crandn(rng, T, P, Q)
    lam, p, n_irls = 2.0, 0.6, 6
    img = oracle.irls(b, S, 1, 1, 1, lam, n_irls, 3, p=p)
    x = b.copy()
    eps = np.linalg.norm(x) ** 2 / 100
    for _ in range(n_irls):
        al = (np.linalg.norm(x) ** 2 + eps) ** (p / 2 - 1)
        x = b / (1 + lam * al)
        eps /= 1.4
    np.testing.assert_allclose(img, np.fft.ifft2(x, norm="ortho"), atol=1e-12)


def test_irls_lambda_zero_keeps_zero_filled():
    rng = np.random.default_rng(42)
    T, P, Q = 5, 8, 8
    S = (rng.random((T, P, Q)) < 0.5).astype(np.uint8)
    b = crandn(rng, T, P, Q)
    img = oracle.irls(b, S, 3, 3, 2, 0.0, 3, 5)
    np.testing.assert_array_equal(img, np.fft.ifft2(S * b, norm="ortho"))


def test_irls_full_sampling_noiseless_bias_is_order_lambda():
    # Exact recovery reading: with every sample observed and no noise the
    # penalty only biases the fit, by O(lam).
    rng = np.random.default_rng(43)
    T, P, Q = 8, 12, 12
    img = exp_series(rng, T, P, Q, [0.85])
    b = oracle.dft2(img)
    S = np.ones((T, P, Q), np.uint8)
    errs = []
    for lam in (1e-2, 1e-3, 1e-4):
        out = oracle.irls(b, S, 3, 3, 2, lam, 3, 20)
        errs.append(np.linalg.norm(out - img) / np.linalg.norm(img))
    for e0, e1 in zip(errs, errs[1:]):
        assert 0.05 < e1 / e0 < 0.2, errs
    assert errs[-1] < 1e-3


def irls_explicit(b, S, N1, N2, M, lam, n_irls, p=0.6, gamma=1.4, eps0_frac=0.01):
    """IRLS with explicit matrices: explicit T(x)^H T(x), dense eigh, dense normal solve."""
    T, P, Q = b.shape
    b = S * b
    x = b.copy()
    eps = None
    for _ in range(n_irls):
        L = oracle.lift(x, N1, N2, M)
        lamR, U = np.linalg.eigh(L.conj().T @ L)
        if eps is None:
            eps = eps0_frac * lamR.max()
        alpha = (np.maximum(lamR, 0) + eps) ** (p / 2 - 1)
        N = explicit_normal_matrix(S, U, alpha, lam, (T, P, Q, N1, N2, M))
        x = np.linalg.solve(N, b.ravel()).reshape(T, P, Q)
        eps /= gamma
    return np.fft.ifft2(x, norm="ortho")


def test_irls_equals_explicit_matrix_irls():
    rng = np.random.default_rng(44)
    T, P, Q, N1, N2, M = 4, 4, 4, 2, 2, 2
    img = exp_series(rng, T, P, Q, [0.8])
    S = (rng.random((T, P, Q)) < 0.6).astype(np.uint8)
    b = S * (oracle.dft2(img) + 0.01 * crandn(rng, T, P, Q))
    ref = irls_explicit(b, S, N1, N2, M, 0.05, 3)
    out = oracle.irls(b, S, N1, N2, M, 0.05, 3, 300)
    np.testing.assert_allclose(out, ref, atol=1e-8 * np.abs(ref).max())
