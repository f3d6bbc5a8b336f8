"""Pins of the oracle's multichannel data term (Sec. II.A, eq. ``measurement_ij``).

Each check comes from outside the code under test: the adjoint identity, an
explicit matrix built from 1-D DFT matrices (no FFT routine), the identity
that full sampling with normalised sensitivities must give, the special case
of a single coil of constant phase (the single-channel operator S o x), and
the single-channel reconstruction it must then reproduce.
"""
import numpy as np
import pytest

import oracle
import workload

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _rand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _dft_matrix(n):
    k = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(k, k) / n) / np.sqrt(n)


def test_coil_forward_adjoint_identity():
    rng = np.random.default_rng(5)
    Nc, T, P, Q = 3, 4, 6, 8
    x = _rand(rng, T, P, Q)
    y = _rand(rng, Nc, T, P, Q)
    S = (rng.random((T, P, Q)) < 0.4).astype(np.float64)
    C = _rand(rng, Nc, P, Q)
    lhs = np.vdot(oracle.coil_forward(x, S, C), y)
    rhs = np.vdot(x, oracle.coil_adjoint(y, S, C))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_coil_normal_against_explicit_matrices():
    """A^H A x with A_j = diag(S_t) F diag(C_j) F^H per frame, F = kron(F_P, F_Q)."""
    rng = np.random.default_rng(6)
    Nc, T, P, Q = 2, 2, 3, 4
    x = _rand(rng, T, P, Q)
    S = (rng.random((T, P, Q)) < 0.5).astype(np.float64)
    C = _rand(rng, Nc, P, Q)
    F = np.kron(_dft_matrix(P), _dft_matrix(Q))  # row-major vectorised frames
    out = np.zeros((T, P * Q), dtype=np.complex128)
    for t in range(T):
        for j in range(Nc):
            A = np.diag(S[t].ravel()) @ F @ np.diag(C[j].ravel()) @ F.conj().T
            out[t] += A.conj().T @ (A @ x[t].ravel())
    E0 = np.zeros((1, 1, P, Q), dtype=np.complex128)
    got = oracle.coil_normal(x, S, C, E0, 0.0)
    np.testing.assert_allclose(got.reshape(T, -1), out, rtol=0, atol=1e-12 * np.abs(out).max())


def test_full_sampling_with_normalised_coils_is_identity():
    rng = np.random.default_rng(7)
    T, P, Q = 3, 16, 16
    C = workload.make_coils(rng, P, Q, 5).astype(np.complex128)
    C /= np.sqrt((np.abs(C) ** 2).sum(axis=0, keepdims=True))
    x = _rand(rng, T, P, Q)
    S = np.ones((T, P, Q))
    got = oracle.coil_adjoint(oracle.coil_forward(x, S, C), S, C)
    np.testing.assert_allclose(got, x, rtol=0, atol=1e-12 * np.abs(x).max())


def test_single_coil_of_constant_phase_is_the_masking_operator():
    rng = np.random.default_rng(8)
    T, P, Q, M = 5, 8, 8, 2
    x = _rand(rng, T, P, Q)
    S = (rng.random((T, P, Q)) < 0.3).astype(np.float64)
    C = np.full((1, P, Q), np.exp(0.7j))
    E = _rand(rng, M, M, P, Q)
    E = 0.5 * (E + np.conj(np.swapaxes(E, 0, 1)))  # Hermitian per pixel
    got = oracle.coil_normal(x, S, C, E, 0.3)
    np.testing.assert_allclose(got - 0.3 * oracle.dft2(oracle.penalty_apply(oracle.idft2(x), E)), S * x,
                               rtol=0, atol=1e-12 * np.abs(x).max())


def test_irls_single_coil_of_constant_phase_reproduces_single_channel():
    pb = workload.make_problem(seed=21, P=16, Q=16, T=6, K=1, R=3, N1=3, N2=3, M=2, n_irls=3, n_cg=4)
    ph = np.exp(-1.1j)
    C = np.full((1, 16, 16), ph, dtype=np.complex128)
    b1 = (pb.b.astype(np.complex128) * ph)[None]  # the same data seen through the coil
    ref = oracle.irls(pb.b, pb.S, pb.N1, pb.N2, pb.M, pb.lam, pb.n_irls, pb.n_cg, return_kspace=True)
    got = oracle.irls(b1, pb.S, pb.N1, pb.N2, pb.M, pb.lam, pb.n_irls, pb.n_cg, return_kspace=True, coils=C)
    assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)


def test_irls_multichannel_recovers_a_noiseless_fully_sampled_series():
    """Full sampling, no noise, normalised coils: A^H b is the data itself and the
    reconstruction stays within O(lam) of it (the single-channel exact-recovery reading)."""
    rng = np.random.default_rng(9)
    T, P, Q = 6, 16, 16
    img, _, _ = workload.make_images(rng, P, Q, T, 1, False)
    C = workload.make_coils(rng, P, Q, 4).astype(np.complex128)
    C /= np.sqrt((np.abs(C) ** 2).sum(axis=0, keepdims=True))
    S = np.ones((T, P, Q), dtype=np.uint8)
    b = np.stack([oracle.dft2(C[j][None] * img) for j in range(4)])
    out = oracle.irls(b, S, 3, 3, 2, 1e-4, 2, 5, coils=C)
    assert np.linalg.norm(out - img) <= 1e-2 * np.linalg.norm(img)

