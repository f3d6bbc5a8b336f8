"""Pins of the oracle's GIRAF variant (``circ_t``): the lifting circular along the
parameter axis as well as in space, the approximation the paper compares its
hybrid lifting with (Sec. IV, Fig. 3).

Independent routes: the FFT Gram against the explicit circular lifting; the
block-circulant structure that a lifting circular in n must give; the
penalty's commutation with a circular frame shift (which the hybrid lifting
breaks); the penalty value against the explicit sum of weighted filter norms.
"""
import numpy as np
import pytest

import oracle


def crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


SHAPES = [(5, 8, 6, 3, 3, 2), (4, 5, 7, 2, 3, 3), (6, 6, 6, 4, 2, 6), (3, 4, 4, 1, 1, 1), (7, 4, 5, 2, 2, 4)]


@pytest.mark.parametrize("T,P,Q,N1,N2,M", SHAPES)
def test_circular_gram_equals_explicit_circular_lifting(T, P, Q, N1, N2, M):
    rng = np.random.default_rng(31)
    x = crandn(rng, T, P, Q)
    L = oracle.lift(x, N1, N2, M, circ_t=True)
    assert L.shape == (T * P * Q, N1 * N2 * M)
    R_ref = L.conj().T @ L
    R = oracle.gram(x, N1, N2, M, circ_t=True)
    np.testing.assert_allclose(R, R_ref, rtol=0, atol=1e-12 * np.abs(R_ref).max())


@pytest.mark.parametrize("T,P,Q,N1,N2,M", SHAPES)
def test_circular_gram_is_block_circulant_in_the_taps(T, P, Q, N1, N2, M):
    rng = np.random.default_rng(32)
    R = oracle.gram(crandn(rng, T, P, Q), N1, N2, M, circ_t=True)
    NN = N1 * N2
    blk = lambda m, mp: R[m * NN:(m + 1) * NN, mp * NN:(mp + 1) * NN]
    for m in range(M - 1):
        for mp in range(M - 1):
            np.testing.assert_allclose(blk(m + 1, mp + 1), blk(m, mp), rtol=0, atol=1e-11 * np.abs(R).max())


def _masks(rng, T, P, Q, N1, N2, M, circ_t):
    R = oracle.gram(crandn(rng, T, P, Q), N1, N2, M, circ_t=circ_t)
    lam, U, alpha = oracle.eig_weights(R, 0.05 * np.linalg.eigvalsh(R).max(), 0.6)
    return U, alpha, oracle.penalty_masks(U, alpha, N1, N2, M, P, Q, chunk=7)


@pytest.mark.parametrize("T,P,Q,N1,N2,M", SHAPES)
def test_circular_penalty_commutes_with_a_frame_shift(T, P, Q, N1, N2, M):
    rng = np.random.default_rng(33)
    _, _, E = _masks(rng, T, P, Q, N1, N2, M, True)
    rho = crandn(rng, T, P, Q)
    g = oracle.penalty_apply(rho, E, circ_t=True)
    g_shift = oracle.penalty_apply(np.roll(rho, 1, axis=0), E, circ_t=True)
    np.testing.assert_allclose(g_shift, np.roll(g, 1, axis=0), rtol=0, atol=1e-12 * np.abs(g).max())
    if 1 < M < T:  # the hybrid (linear in n) penalty does not (with M = T its one window covers every frame)
        h = oracle.penalty_apply(rho, E)
        h_shift = oracle.penalty_apply(np.roll(rho, 1, axis=0), E)
        assert np.abs(h_shift - np.roll(h, 1, axis=0)).max() > 1e-3 * np.abs(h).max()


@pytest.mark.parametrize("T,P,Q,N1,N2,M", SHAPES)
def test_circular_penalty_value_equals_explicit_filter_norms(T, P, Q, N1, N2, M):
    rng = np.random.default_rng(34)
    U, alpha, E = _masks(rng, T, P, Q, N1, N2, M, True)
    x = crandn(rng, T, P, Q)
    L = oracle.lift(x, N1, N2, M, circ_t=True)
    J_ref = float(np.sum(alpha * np.linalg.norm(L @ U, axis=0) ** 2))
    J = oracle.penalty_value(oracle.idft2(x), E, circ_t=True)
    assert abs(J - J_ref) < 1e-10 * J_ref
