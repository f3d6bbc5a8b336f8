"""FP64 CPU oracle of the IRLS structured low-rank recovery of damped exponentials.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  The product
(``libslrx`` and its Python binding) never calls it and shares no code with it.

Every function follows the paper (Balachandrasekaran, Magnotta, Jacob,
"Recovery of damped exponentials using structured low rank matrix
completion", arXiv 1704.04511) step by step, in complex128, using NumPy's
FFT and LAPACK ``eigh`` as library primitives.  Conventions (readings of the
paper where it is silent, listed again in the design notes):

* ``xhat`` (the paper's rho-hat) is k-space, complex ``[T][P][Q]``, DC at
  ``[0, 0]``.  ``F`` is the unitary 2-D DFT (the matrix F of the measurement
  model, Sec. II.A); images are ``rho_t = F^-1 xhat_t``.
* Filter support Lambda = Lambda_s x {0..M-1}; Lambda_s holds the centred
  offsets a = (a1, a2), a1 in [-floor(N1/2), N1-1-floor(N1/2)] (same for a2).
  Lifted columns are ordered (m, a), m-major, a row-major.
* Hybrid lifting (Sec. III.A, the approximation of eq. ``Toeplitz -
  circ_rep``): T(xhat)[(n, w), (m, a)] = xhat_{n-m}[(w - a) mod (P, Q)] for
  n = M-1..T-1 and all w, i.e. T(xhat) d is a 3-D convolution that is linear
  (valid) along the parameter axis and circular in space.
* The Gram matrix is R = T^H T (s x s, the filter side); its eigenvectors are
  the filters (Sec. III.B, eq. ``eq:gram matrix``).
* Per least-squares step the objective is ||S xhat - b||^2 + lam J(xhat) with
  J = sum_i alpha_i ||T(xhat) u_i||^2; lam = 2/(mu p) relative to eq.
  ``eq:x-update``.
* epsilon^(0) = eps0_frac * lambda_max of the first Gram matrix, and after each
  least-squares step epsilon <- epsilon / gamma (Sec. III.C); negative
  round-off eigenvalues are clamped to zero before adding epsilon.
* CG is warm-started from the current iterate, runs exactly ``n_cg``
  iterations and stops early only on an exactly zero residual or curvature.
* Multichannel data (Sec. II.A, eq. ``measurement_ij``): coil j of frame i
  measures S_i F C_j F^* xhat_i, with C_j a pointwise image-domain
  sensitivity shared by all frames and S_i shared by all coils.  The data
  term is then sum_ij ||S_i F C_j F^* xhat_i - b_ij||^2, its normal operator
  sum_j F C_j^* F^* S F C_j F^*, and the initial iterate the zero-filled coil
  combination A^H b (which is S o b for one coil of ones).
"""
from __future__ import annotations

import numpy as np
import scipy.fft

__all__ = [
    "dft2", "idft2", "filter_offsets", "pair_index", "lift", "gram",
    "eig_weights", "weight_matrix", "filter_spectra", "penalty_masks",
    "penalty_apply", "penalty_value", "normal_apply", "coil_forward", "coil_adjoint",
    "coil_normal", "cg", "irls", "t2_fit", "voxel_lift", "voxel_gram", "voxel_weights", "voxel_masks",
    "irls_voxel", "linear_rows", "lift_linear", "lift_linear_adjoint", "gram_direct",
    "direct_normal_apply", "irls_direct",
]


# ---------------------------------------------------------------- transforms
def dft2(a: np.ndarray) -> np.ndarray:
    """Unitary 2-D DFT over the last two axes (F in Sec. II.A, eq. ``measurement_ij``)."""
    return np.fft.fft2(a, norm="ortho")


def idft2(a: np.ndarray) -> np.ndarray:
    """Inverse unitary 2-D DFT (F^* in Sec. II.A; Q^* = I (x) F^* in Sec. III.A)."""
    return np.fft.ifft2(a, norm="ortho")


# ------------------------------------------------------------ index helpers
def filter_offsets(N1: int, N2: int) -> tuple[np.ndarray, np.ndarray]:
    """Spatial support Lambda_s of one filter frame (Sec. II.C, N1 x N2), centred, row-major."""
    a1 = np.arange(N1) - N1 // 2
    a2 = np.arange(N2) - N2 // 2
    A1, A2 = np.meshgrid(a1, a2, indexing="ij")
    return A1.ravel(), A2.ravel()


def pair_index(M: int) -> list[tuple[int, int]]:
    """Tap pairs (m, m') with m <= m', in row-major order of the upper triangle."""
    return [(m, mp) for m in range(M) for mp in range(m, M)]


# ------------------------------------------------------------------ lifting
def lift(xhat: np.ndarray, N1: int, N2: int, M: int, circ_t: bool = False) -> np.ndarray:
    """Explicit lifted matrix T(xhat) in C^{(k P Q) x s} (Sec. II.B, eq. ``annihil-compact``).

    Rows (n, w) for n = M-1..T-1 (k = T-M+1 valid shifts along the parameter
    axis) and w in Z_P x Z_Q; columns (m, a).  Circular in space per the
    hybrid approximation of Sec. III.A.  With ``circ_t`` (the GIRAF
    approximation, circular along the parameter axis too): all k = T rows
    n = 0..T-1, frame index (n - m) mod T.  Tiny inputs only.
    """
    T, P, Q = xhat.shape
    a1, a2 = filter_offsets(N1, N2)
    NN = N1 * N2
    n0 = 0 if circ_t else M - 1
    k = T - n0
    w1, w2 = np.meshgrid(np.arange(P), np.arange(Q), indexing="ij")
    out = np.zeros((k * P * Q, M * NN), dtype=np.complex128)
    for n in range(n0, T):
        rows = slice((n - n0) * P * Q, (n - n0 + 1) * P * Q)
        for m in range(M):
            for ia in range(NN):
                vals = xhat[(n - m) % T][(w1 - a1[ia]) % P, (w2 - a2[ia]) % Q]
                out[rows, m * NN + ia] = vals.ravel()
    return out


# -------------------------------------------------------------- Gram matrix
def gram(xhat: np.ndarray, N1: int, N2: int, M: int, circ_t: bool = False) -> np.ndarray:
    """Gram matrix R = T(xhat)^H T(xhat) by FFT autocorrelation (Sec. III.B).

    Block (m, m') of R (eq. ``eq:block-expression for R``) sums, over the
    k valid parameter shifts, products of Toeplitz blocks; each product is read
    from g = F_u(conj(rho_i) o rho_j) with a sliding N1 x N2 window over the
    (2N1-1) x (2N2-1) lag neighbourhood (eq. ``eq:P_ij modified``).  Here
    R[(m,a),(m',a')] = sum_{n=M-1}^{T-1} F_u(conj(rho_{n-m}) rho_{n-m'})[a - a'],
    F_u the unnormalised forward DFT.  All M^2 blocks are formed directly.
    ``circ_t``: the sum runs over n = 0..T-1 with frame indices mod T.
    """
    T, P, Q = xhat.shape
    rho = idft2(xhat)
    a1, a2 = filter_offsets(N1, N2)
    NN = N1 * N2
    d1 = (a1[:, None] - a1[None, :]) % P
    d2 = (a2[:, None] - a2[None, :]) % Q
    R = np.empty((M * NN, M * NN), dtype=np.complex128)
    for m in range(M):
        for mp in range(M):
            c = np.zeros((P, Q), dtype=np.complex128)
            for n in range(0 if circ_t else M - 1, T):
                c += np.conj(rho[(n - m) % T]) * rho[(n - mp) % T]
            g = np.fft.fft2(c)
            R[m * NN:(m + 1) * NN, mp * NN:(mp + 1) * NN] = g[d1, d2]
    return R


# ---------------------------------------------------------- weight update
def eig_weights(R: np.ndarray, eps: float, p: float):
    """Eigen-decomposition of R and IRLS weights (Sec. III.B, Algorithm 1 step 1).

    alpha_i = (lambda_i + eps)^(p/2 - 1), with lambda_i clamped at 0.
    Returns (lambda ascending, U, alpha).
    """
    lam, U = np.linalg.eigh(R)
    alpha = (np.maximum(lam, 0.0) + eps) ** (p / 2.0 - 1.0)
    return lam, U, alpha


def weight_matrix(U: np.ndarray, alpha: np.ndarray) -> np.ndarray:
    """H = U (Lambda + eps I)^(p/2-1) U^* (Sec. III.B, weight update eq. ``eq:weight-update``)."""
    return (U * alpha[None, :]) @ U.conj().T


def filter_spectra(u: np.ndarray, N1: int, N2: int, M: int, P: int, Q: int) -> np.ndarray:
    """mu_m(r) = sum_{a in Lambda_s} u[(m, a)] e^{+2 pi i (a1 r1/P + a2 r2/Q)}.

    The diagonal of D_l in eq. ``eq:circ_fft``: the transform of the zero-padded
    filter frame (Sec. III.A).  ``u`` has shape (..., s); result (..., M, P, Q).
    """
    a1, a2 = filter_offsets(N1, N2)
    NN = N1 * N2
    lead = u.shape[:-1]
    frames = np.zeros(lead + (M, P, Q), dtype=np.complex128)
    uu = u.reshape(lead + (M, NN))
    frames[..., a1 % P, a2 % Q] = uu
    # e^{+2 pi i a r / N} summed over a = unnormalised inverse DFT
    return scipy.fft.ifft2(frames, workers=-1) * (P * Q)


def penalty_masks(U: np.ndarray, alpha: np.ndarray, N1: int, N2: int, M: int,
                  P: int, Q: int, chunk: int = 64) -> np.ndarray:
    """Per-pixel M x M penalty masks E_r (Sec. III.A; G precompute after eq. ``eq:grad_ls``).

    E_r[m, m'] = sum_i alpha_i conj(mu^(i)_m(r)) mu^(i)_m'(r): the summed
    (cross) power spectra of the weighted filters h^(i) = sqrt(alpha_i) u_i,
    one filter at a time.  E_r is Hermitian, so the pairs m > m' are the
    conjugates of m < m'.  Returned as complex128 [M][M][P][Q].
    """
    s = U.shape[1]
    E = np.zeros((M, M, P * Q), dtype=np.complex128)
    for i0 in range(0, s, chunk):
        i1 = min(s, i0 + chunk)
        mu = filter_spectra(U[:, i0:i1].T, N1, N2, M, P, Q)      # (c, M, P, Q)
        mu *= np.sqrt(alpha[i0:i1])[:, None, None, None]
        mu = mu.reshape(i1 - i0, M, P * Q)
        cmu = np.conj(mu)
        for m in range(M):
            for mp in range(m, M):
                E[m, mp] += np.einsum("ir,ir->r", cmu[:, m], mu[:, mp])
    for m in range(M):
        for mp in range(m):
            E[m, mp] = np.conj(E[mp, m])
    return E.reshape(M, M, P, Q)


def penalty_apply(rho: np.ndarray, E: np.ndarray, circ_t: bool = False) -> np.ndarray:
    """Image-domain penalty operator G (Sec. III.A, eq. ``eq:grad_ls``).

    J = sum_{n=M-1}^{T-1} sum_r z^H E_r z with z_m = rho_{n-m}(r); returns
    dJ/d conj(rho): (G rho)_{n-m} += sum_m' E[m, m'] rho_{n-m'}.  ``circ_t``:
    n = 0..T-1 and frame indices mod T.
    """
    M = E.shape[0]
    T = rho.shape[0]
    out = np.zeros_like(rho, dtype=np.complex128)
    for n in range(0 if circ_t else M - 1, T):
        for m in range(M):
            for mp in range(M):
                out[(n - m) % T] += E[m, mp] * rho[(n - mp) % T]
    return out


def penalty_value(rho: np.ndarray, E: np.ndarray, circ_t: bool = False) -> float:
    """J(rho) = <rho, G rho> (real by construction)."""
    return float(np.vdot(rho, penalty_apply(rho, E, circ_t)).real)


def normal_apply(xhat: np.ndarray, S: np.ndarray, E: np.ndarray, lam: float, circ_t: bool = False) -> np.ndarray:
    """Normal operator of eq. ``eq:grad_ls``: S o xhat + lam F G F^* xhat (A = S, single coil)."""
    return S * xhat + lam * dft2(penalty_apply(idft2(xhat), E, circ_t))


# ------------------------------------------------------------ multichannel
def coil_forward(xhat: np.ndarray, S: np.ndarray, C: np.ndarray) -> np.ndarray:
    """A xhat of eq. ``measurement_ij``: b_ij = S_i F C_j F^* xhat_i, shape [Nc][T][P][Q]."""
    rho = idft2(xhat)
    return np.stack([S * dft2(C[j][None] * rho) for j in range(C.shape[0])])


def coil_adjoint(b: np.ndarray, S: np.ndarray, C: np.ndarray) -> np.ndarray:
    """A^H b = sum_j F C_j^* F^* (S o b_j) (the adjoint of ``coil_forward``)."""
    acc = np.zeros(b.shape[1:], dtype=np.complex128)
    for j in range(C.shape[0]):
        acc += np.conj(C[j])[None] * idft2(S * b[j])
    return dft2(acc)


def coil_normal(xhat: np.ndarray, S: np.ndarray, C: np.ndarray, E: np.ndarray, lam: float,
                circ_t: bool = False) -> np.ndarray:
    """Normal operator with the multichannel data term: A^H A xhat + lam F G F^* xhat."""
    rho = idft2(xhat)
    acc = lam * penalty_apply(rho, E, circ_t)
    for j in range(C.shape[0]):
        acc = acc + np.conj(C[j])[None] * idft2(S * dft2(C[j][None] * rho))
    return dft2(acc)


# ----------------------------------------------------------------------- CG
def cg(apply, rhs: np.ndarray, x0: np.ndarray, n_iter: int, trace: list | None = None) -> np.ndarray:
    """Conjugate gradients (Algorithm 1 step 2), warm start, exactly ``n_iter`` iterations."""
    x = x0.astype(np.complex128).copy()
    r = rhs - apply(x)
    p = r.copy()
    rr = float(np.vdot(r, r).real)
    if trace is not None:
        trace.append(rr)
    for _ in range(n_iter):
        if rr == 0.0:
            break
        q = apply(p)
        pq = float(np.vdot(p, q).real)
        if pq <= 0.0:
            break
        a = rr / pq
        x += a * p
        r -= a * q
        rr_new = float(np.vdot(r, r).real)
        p = r + (rr_new / rr) * p
        rr = rr_new
        if trace is not None:
            trace.append(rr)
    return x


# --------------------------------------------------------------------- IRLS
def irls(b: np.ndarray, S: np.ndarray, N1: int, N2: int, M: int, lam: float,
         n_irls: int, n_cg: int, p: float = 0.6, gamma: float = 1.4,
         eps0_frac: float = 0.01, x0: np.ndarray | None = None,
         trace: dict | None = None, return_kspace: bool = False,
         coils: np.ndarray | None = None, circ_t: bool = False) -> np.ndarray:
    """Algorithm 1: alternate the weight update and the CG least-squares step.

    Step 1 (Sec. III.B): Gram matrix by FFT autocorrelation, eigen-decomposition,
    weights alpha_i = (lambda_i + eps)^(p/2-1) and masks E.  Step 2 (Sec. III.A):
    a few CG iterations on (S + lam F G F^*) xhat = S o b.  Then eps <- eps/gamma
    (Sec. III.C).  Returns the images F^-1 xhat (or xhat with ``return_kspace``).

    With ``coils`` (sensitivities C, [Nc][P][Q]) the data b is [Nc][T][P][Q] and
    the least-squares step uses the multichannel model of Sec. II.A:
    (A^H A + lam F G F^*) xhat = A^H b, starting from A^H b.

    ``circ_t``: the GIRAF approximation the paper compares against (Sec. IV,
    Fig. 3), circular along the parameter axis as well as in space.
    """
    S = S.astype(np.float64)
    if coils is None:
        b = S * b.astype(np.complex128)
        normal = lambda v, E: normal_apply(v, S, E, lam, circ_t)
    else:
        C = coils.astype(np.complex128)
        b = coil_adjoint(S[None] * b.astype(np.complex128), S, C)
        normal = lambda v, E: coil_normal(v, S, C, E, lam, circ_t)
    T, P, Q = b.shape
    x = b.copy() if x0 is None else x0.astype(np.complex128).copy()
    eps = None
    for _ in range(n_irls):
        R = gram(x, N1, N2, M, circ_t)
        lamR, U = np.linalg.eigh(R)
        if eps is None:
            eps = eps0_frac * float(lamR.max())
        alpha = (np.maximum(lamR, 0.0) + eps) ** (p / 2.0 - 1.0)
        E = penalty_masks(U, alpha, N1, N2, M, P, Q)
        cg_trace = [] if trace is not None else None
        x = cg(lambda v: normal(v, E), b, x, n_cg, cg_trace)
        if trace is not None:
            trace.setdefault("eps", []).append(eps)
            trace.setdefault("lambda_max", []).append(float(lamR.max()))
            trace.setdefault("cg_rr", []).append(cg_trace)
        eps = eps / gamma
    return x if return_kspace else idft2(x)


# ------------------------------------------- IRLS-direct (Sec. IV, Fig. 2)
def linear_rows(P: int, Q: int, N1: int, N2: int) -> tuple[np.ndarray, np.ndarray]:
    """Valid shifts w of the linear lifting: the N1 x N2 support w - a stays inside the
    P x Q grid (centred k-space coordinates), row-major.  (P-N1+1)(Q-N2+1) of them."""
    a1, a2 = filter_offsets(N1, N2)
    w1 = np.arange(a1.max(), P + a1.min())
    w2 = np.arange(a2.max(), Q + a2.min())
    W1, W2 = np.meshgrid(w1, w2, indexing="ij")
    return W1.ravel(), W2.ravel()


def lift_linear(xhat: np.ndarray, N1: int, N2: int, M: int) -> np.ndarray:
    """The lifted matrix without the circular approximation (the IRLS-direct method the
    paper compares with in Sec. IV / Fig. 2): linear convolutions in all three
    dimensions.  k-space is taken in centred order (DC at index (P/2, Q/2), i.e.
    fftshift of the DFT order); rows (n, w) for n = M-1..T-1 and the valid shifts w of
    ``linear_rows``, columns (m, a) as in ``lift``; entry xc[n-m][w - a].
    Shape ((T-M+1)(P-N1+1)(Q-N2+1), s)."""
    T, P, Q = xhat.shape
    xc = np.fft.fftshift(xhat, axes=(1, 2))
    a1, a2 = filter_offsets(N1, N2)
    w1, w2 = linear_rows(P, Q, N1, N2)
    NN, nw = N1 * N2, w1.size
    out = np.zeros(((T - M + 1) * nw, M * NN), dtype=np.complex128)
    for n in range(M - 1, T):
        rows = slice((n - M + 1) * nw, (n - M + 2) * nw)
        for m in range(M):
            for ia in range(NN):
                out[rows, m * NN + ia] = xc[n - m][w1 - a1[ia], w2 - a2[ia]]
    return out


def lift_linear_adjoint(Y: np.ndarray, T: int, P: int, Q: int, N1: int, N2: int, M: int) -> np.ndarray:
    """Adjoint of ``lift_linear`` (Frobenius inner product): every entry of Y is added
    back to the k-space sample it was read from.  Returns [T][P][Q] in DFT order."""
    a1, a2 = filter_offsets(N1, N2)
    w1, w2 = linear_rows(P, Q, N1, N2)
    NN, nw = N1 * N2, w1.size
    xc = np.zeros((T, P, Q), dtype=np.complex128)
    for n in range(M - 1, T):
        rows = slice((n - M + 1) * nw, (n - M + 2) * nw)
        for m in range(M):
            for ia in range(NN):
                np.add.at(xc[n - m], (w1 - a1[ia], w2 - a2[ia]), Y[rows, m * NN + ia])
    return np.fft.ifftshift(xc, axes=(1, 2))


def gram_direct(xhat: np.ndarray, N1: int, N2: int, M: int) -> np.ndarray:
    """R = T^H T of the linear lifting, formed from the explicit matrix."""
    X = lift_linear(xhat, N1, N2, M)
    return X.conj().T @ X


def direct_normal_apply(v: np.ndarray, S: np.ndarray, H: np.ndarray, lam: float,
                        N1: int, N2: int, M: int) -> np.ndarray:
    """S o v + lam T^*(T(v) H): the normal operator of the least-squares step with the
    penalty tr(T(v) H T(v)^H) = sum_i alpha_i ||T(v) u_i||^2 of the linear lifting."""
    T, P, Q = v.shape
    return S * v + lam * lift_linear_adjoint(lift_linear(v, N1, N2, M) @ H, T, P, Q, N1, N2, M)


def irls_direct(b: np.ndarray, S: np.ndarray, N1: int, N2: int, M: int, lam: float,
                n_irls: int, n_cg: int, p: float = 0.6, gamma: float = 1.4,
                eps0_frac: float = 0.01, trace: dict | None = None,
                return_kspace: bool = False) -> np.ndarray:
    """IRLS-direct: Algorithm 1 with both sub-problems solved on the explicit linear
    lifting, without the FFT-based approximations (Sec. IV): R = T^H T from the explicit
    matrix, H = U (Lambda + eps I)^(p/2-1) U^H, n_cg CG iterations with
    ``direct_normal_apply``, the same eps schedule as ``irls``."""
    S = S.astype(np.float64)
    b = S * b.astype(np.complex128)
    x = b.copy()
    eps = None
    for _ in range(n_irls):
        R = gram_direct(x, N1, N2, M)
        lamR, U, _ = eig_weights(R, 1.0, p)
        if eps is None:
            eps = eps0_frac * float(lamR.max())
        alpha = (np.maximum(lamR, 0.0) + eps) ** (p / 2.0 - 1.0)
        H = weight_matrix(U, alpha)
        cg_trace = [] if trace is not None else None
        x = cg(lambda v: direct_normal_apply(v, S, H, lam, N1, N2, M), b, x, n_cg, cg_trace)
        if trace is not None:
            trace.setdefault("eps", []).append(eps)
            trace.setdefault("lambda_max", []).append(float(lamR.max()))
            trace.setdefault("cg_rr", []).append(cg_trace)
        eps = eps / gamma
    return x if return_kspace else idft2(x)


# ------------------------------------------------ HLR-Voxel (Sec. II.E)
def voxel_lift(xhat: np.ndarray, M: int) -> np.ndarray:
    """Per-pixel Toeplitz matrices of eq. ``eq: MORASA-objective`` / ``eq:Toeplitz_g``:
    T(rho(r)) in C^{(T-M+1) x M}, row n = M-1..T-1, column m holding rho_{n-m}(r),
    rho = F^-1 xhat the images.  Returned as [P][Q][T-M+1][M].  Tiny inputs only."""
    rho = idft2(xhat)
    T, P, Q = rho.shape
    out = np.zeros((P, Q, T - M + 1, M), dtype=np.complex128)
    for r1 in range(P):
        for r2 in range(Q):
            for n in range(M - 1, T):
                for m in range(M):
                    out[r1, r2, n - M + 1, m] = rho[n - m, r1, r2]
    return out


def voxel_gram(xhat: np.ndarray, M: int) -> np.ndarray:
    """Per-pixel Gram matrices G_r = T(rho(r))^H T(rho(r)) (M x M, the filter side):
    G_r[m, m'] = sum_{n=M-1}^{T-1} conj(rho_{n-m}(r)) rho_{n-m'}(r).  [P][Q][M][M]."""
    rho = idft2(xhat)
    T = rho.shape[0]
    G = np.zeros(rho.shape[1:] + (M, M), dtype=np.complex128)
    for m in range(M):
        for mp in range(M):
            G[..., m, mp] = sum(np.conj(rho[n - m]) * rho[n - mp] for n in range(M - 1, T))
    return G


def voxel_weights(G: np.ndarray, eps: float, p: float):
    """IRLS weights of the pixel-wise Hankel low-rank prior (HLR-Voxel, Sec. II.E; solved
    by IRLS as in Sec. IV): per pixel, H_r = (G_r + eps I)^(p/2-1) from the eigen-
    decomposition of G_r, eigenvalues clamped at 0.  The penalty
    sum_r ||T_r H_r^(1/2)||_F^2 = sum_r sum_n z^H E_r z (z_m = rho_{n-m}(r)) has
    E_r = conj(H_r), the per-pixel masks the CG operator takes.  G: [P][Q][M][M].
    Returns (E [M][M][P][Q], eigenvalues [P][Q][M] ascending)."""
    lam, U = np.linalg.eigh(G)                   # per pixel, eigenvector i in U[..., :, i]
    alpha = (np.maximum(lam, 0.0) + eps) ** (p / 2.0 - 1.0)
    E = np.einsum("...i,...mi,...ni->...mn", alpha, np.conj(U), U)   # sum_i alpha_i conj(U_mi) U_ni
    return np.moveaxis(E, (-2, -1), (0, 1)).copy(), lam


def voxel_masks(xhat: np.ndarray, M: int, eps: float, p: float):
    """E [M][M][P][Q] of voxel_weights for the per-pixel Gram matrices of xhat, and the
    largest eigenvalue over all pixels."""
    E, lam = voxel_weights(voxel_gram(xhat, M), eps, p)
    return E, float(lam[..., -1].max())


def irls_voxel(b: np.ndarray, S: np.ndarray, M: int, lam: float, n_irls: int, n_cg: int,
               p: float = 0.6, gamma: float = 1.4, eps0_frac: float = 0.01,
               trace: dict | None = None, return_kspace: bool = False,
               coils: np.ndarray | None = None) -> np.ndarray:
    """HLR-Voxel (the comparison system of Sec. II.E / Sec. IV) by the IRLS loop of
    Algorithm 1 with per-pixel weights: each outer iteration forms every pixel's Gram
    matrix, eps^(0) = eps0_frac times the largest eigenvalue over all pixels (first
    iteration), the masks E_r of voxel_weights, n_cg CG iterations on
    (S + lam F G F^*) xhat = S o b with those masks, then eps <- eps / gamma.
    With ``coils`` the least-squares step is the multichannel one of Sec. II.A, as
    in ``irls`` (the paper compares HLR-Voxel on multichannel data too, Sec. IV)."""
    S = S.astype(np.float64)
    if coils is None:
        b = S * b.astype(np.complex128)
        normal = lambda v, E: normal_apply(v, S, E, lam)
    else:
        C = coils.astype(np.complex128)
        b = coil_adjoint(S[None] * b.astype(np.complex128), S, C)
        normal = lambda v, E: coil_normal(v, S, C, E, lam)
    x = b.copy()
    eps = None
    for _ in range(n_irls):
        G = voxel_gram(x, M)
        lmax = float(np.linalg.eigvalsh(G)[..., -1].max())
        if eps is None:
            eps = eps0_frac * lmax
        E, _ = voxel_weights(G, eps, p)
        cg_trace = [] if trace is not None else None
        x = cg(lambda v: normal(v, E), b, x, n_cg, cg_trace)
        if trace is not None:
            trace.setdefault("eps", []).append(eps)
            trace.setdefault("lambda_max", []).append(lmax)
            trace.setdefault("cg_rr", []).append(cg_trace)
        eps = eps / gamma
    return x if return_kspace else idft2(x)


# ---------------------------------------------------------------- T2 maps
def t2_fit(img: np.ndarray, te_ms: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Mono-exponential fit per pixel (Sec. IV: T2 maps from the reconstructed series).

    Reading: least-squares line through y_t = log|rho_t| (|rho| floored at 1e-30)
    against TE_t; T2 = -1/slope where the slope is negative, +inf otherwise, and
    the amplitude exp(intercept at TE = 0).  Returns (T2 [ms], amplitude), each
    shaped like one frame.
    """
    te = np.asarray(te_ms, dtype=np.float64)
    y = np.log(np.maximum(np.abs(img.astype(np.complex128)), 1e-30))
    tc = te - te.mean()
    ybar = y.mean(axis=0)
    slope = np.tensordot(tc, y - ybar[None], axes=(0, 0)) / (tc * tc).sum()
    amp = np.exp(ybar - slope * te.mean())
    with np.errstate(divide="ignore"):
        t2 = np.where(slope < 0.0, -1.0 / np.where(slope < 0.0, slope, -1.0), np.inf)
    return t2, amp
