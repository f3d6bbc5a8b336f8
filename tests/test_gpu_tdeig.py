"""Divide-and-conquer eigensolver of the real symmetric tridiagonal (the middle
stage of the Gram eigen-decomposition) against its definition: T Z = Z diag(lam)
with Z orthogonal, and the eigenvalues of LAPACK's tridiagonal solver.  The
matrices exercise the solver's branches: random, zero couplings (merges
without a rank-one term), nearly equal diagonals (deflation by rotation),
repeated blocks, Wilkinson's matrix, a clustered Gram-like spectrum, a
rank-deficient Gram-like spectrum at the full 1125 size and a graded
diagonal."""
import numpy as np
import pytest
import scipy.linalg

from tests.gpu_util import say

pytestmark = pytest.mark.gpu

slrx = pytest.importorskip("paper_1704_04511_amd")

# plan shapes giving the tridiagonal size s = N1 N2 M
SIZES = {1: (8, 8, 8, 1, 1, 1), 2: (8, 8, 8, 2, 1, 1), 3: (8, 8, 8, 3, 1, 1), 7: (8, 8, 8, 7, 1, 1),
         64: (8, 8, 8, 8, 8, 1), 200: (8, 8, 8, 5, 5, 8), 1125: (16, 16, 8, 15, 15, 5),
         3000: (16, 32, 8, 15, 25, 8)}


def matrices(n, rng):
    out = {"random": (rng.standard_normal(n), rng.standard_normal(n - 1))}
    if n >= 3:
        e = rng.standard_normal(n - 1)
        e[rng.random(n - 1) < 0.2] = 0.0
        out["zero couplings"] = (rng.standard_normal(n), e)
        out["close diagonals"] = (np.ones(n) + 1e-15 * rng.standard_normal(n), 1e-9 * rng.standard_normal(n - 1))
        blk = np.repeat(np.arange(1.0, 4.0), (n + 2) // 3)[:n]
        e = np.where(np.arange(n - 1) % max(n // 3, 1) == max(n // 3, 1) - 1, 0.0, 1e-8)
        out["repeated blocks"] = (blk, e)
        out["graded"] = (10.0 ** (-12.0 * np.arange(n) / n), 1e-3 * 10.0 ** (-12.0 * np.arange(n - 1) / n))
    if n % 2 == 1 and n >= 3:
        h = (n - 1) // 2
        out["wilkinson"] = (np.abs(np.arange(-h, h + 1)).astype(float), np.ones(n - 1))
    if 64 <= n <= 200:
        X = rng.standard_normal((n, 8 * n))
        Tm = scipy.linalg.hessenberg(X @ X.T)
        out["clustered gram"] = (np.diag(Tm).copy(), np.diag(Tm, 1).copy())
    if n == 1125:
        # rank n/3 plus a 1e-12 floor: two thirds of the spectrum in a tight cluster, as in
        # the Gram matrices of late IRLS iterations (long deflation chains, bitonic sort)
        X = rng.standard_normal((n, n // 3))
        Tm = scipy.linalg.hessenberg(X @ X.T + 1e-12 * np.eye(n))
        out["low-rank gram"] = (np.diag(Tm).copy(), np.diag(Tm, 1).copy())
    return out


def tri_matmul(D, E, Z):
    """T Z for the tridiagonal T = (D, E), in O(n^2)."""
    out = D[:, None] * Z
    if len(E):
        out[:-1] += E[:, None] * Z[1:]
        out[1:] += E[:, None] * Z[:-1]
    return out


@pytest.mark.parametrize("n", sorted(SIZES))
def test_tdeig_matches_definition(n):
    P, Q, T, N1, N2, M = SIZES[n]
    rng = np.random.default_rng(n)
    with slrx.Plan(P, Q, T, N1, N2, M, slrx.make_params(lam=1e-3, n_irls=1, n_cg=1)) as pl:
        assert pl.s == n
        for name, (D, E) in matrices(n, rng).items():
            say(f"tdeig n={n} {name}")
            lam, Z = pl.step_tdeig(D, E)
            assert np.all(Z.imag == 0.0)
            Z = Z.real
            nrm = max(np.abs(D).max() + (2 * np.abs(E).max() if n > 1 else 0.0), 1e-300)
            ref = scipy.linalg.eigh_tridiagonal(D, E, eigvals_only=True) if n > 1 else D.copy()
            assert np.all(np.diff(lam) >= 0.0), name
            assert np.abs(lam - ref).max() <= 1e-13 * n * nrm, name
            assert np.linalg.norm(tri_matmul(D, E, Z) - Z * lam) <= 1e-13 * n * nrm, name
            # orthogonality: a block of columns against all, and Z^T Z g = g for random g
            cols = rng.choice(n, size=min(n, 64), replace=False)
            G = Z[:, cols].T @ Z
            G[np.arange(len(cols)), cols] -= 1.0
            assert np.abs(G).max() <= 1e-13 * n, name
            g = rng.standard_normal((n, 4))
            assert np.abs(Z.T @ (Z @ g) - g).max() <= 1e-13 * n * np.abs(g).max(), name
