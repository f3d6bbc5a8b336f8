"""Seeded synthetic inputs for the multi-echo recovery problem.

This module only *draws data*: smooth parameter maps, the damped-exponential
image series of the signal model (Sec. II.B, eq. ``eq:signal model``), its
k-space via the unitary 2-D DFT, variable-density sampling masks and noise.
It holds none of the reconstruction method's arithmetic; both the FP64 oracle
and the HIP path receive the arrays it returns.

Layout conventions shared by every consumer:
  * k-space ``b`` and images are complex arrays ``[T][P][Q]`` (frame-major,
    row-major frames), DC at index ``[0, 0]`` (no fftshift);
  * masks ``S`` are ``uint8`` ``[T][P][Q]`` with values 0/1, drawn
    independently per frame (echo);
  * echo times are ``TE_t = 10 (t + 1)`` ms, i.e. a 10 ms echo spacing as in
    the paper's experiments (Sec. IV).

The paper's dataset (a 12-coil turbo spin echo acquisition, Sec. IV) is not
available; these recipes stand in for it with the same matrix sizes and echo
spacing.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Problem",
    "bumps",
    "make_images",
    "make_mask",
    "make_coils",
    "make_problem",
    "make_mc_problem",
    "CONFIGS",
    "MC_CONFIGS",
    "config_problem",
    "batch_specs",
]


@dataclasses.dataclass
class Problem:
    """One synthetic reconstruction problem (all arrays host-side)."""

    b: np.ndarray          # complex64 [T][P][Q], S∘(x + noise)
    S: np.ndarray          # uint8 [T][P][Q]
    truth: np.ndarray      # complex128 [T][P][Q] ground-truth images
    N1: int
    N2: int
    M: int
    lam: float
    n_irls: int
    n_cg: int
    p: float = 0.6
    gamma: float = 1.4
    eps0_frac: float = 0.01
    name: str = ""
    t2_maps: tuple = ()    # ground-truth T2 maps (ms), one per component
    frac: np.ndarray | None = None
    coils: np.ndarray | None = None  # complex64 [Nc][P][Q] sensitivities; b is then [Nc][T][P][Q]

    @property
    def shape(self):
        return self.b.shape


def bumps(rng: np.random.Generator, P: int, Q: int, lo: float, hi: float,
          n: int = 6) -> np.ndarray:
    """Smooth field: sum of ``n`` Gaussian bumps, min-max normalised to [lo, hi].

    Centres are uniform on the grid, widths uniform in [0.08, 0.25]*P and
    amplitudes uniform in [0.3, 1].
    """
    r1 = np.arange(P)[:, None].astype(np.float64)
    r2 = np.arange(Q)[None, :].astype(np.float64)
    f = np.zeros((P, Q))
    for _ in range(n):
        c1 = rng.uniform(0, P)
        c2 = rng.uniform(0, Q)
        sig = rng.uniform(0.08, 0.25) * P
        amp = rng.uniform(0.3, 1.0)
        f += amp * np.exp(-((r1 - c1) ** 2 + (r2 - c2) ** 2) / (2.0 * sig * sig))
    f -= f.min()
    mx = f.max()
    if mx > 0:
        f /= mx
    return lo + (hi - lo) * f


def make_images(rng: np.random.Generator, P: int, Q: int, T: int, K: int,
                phase: bool) -> tuple[np.ndarray, tuple, np.ndarray | None]:
    """Damped-exponential image series rho_t(r) = rho0 e^{i phi} sum_k f_k exp(-TE_t/T2_k).

    K = 1: T2 in [20, 150] ms.  K = 2: T2a in [15, 40], T2b in [60, 200] ms with
    fractions f and 1 - f from a smooth field.  ``phase`` adds a smooth phase
    map in [-pi, pi].
    """
    rho0 = bumps(rng, P, Q, 0.0, 1.0)
    te = 10.0 * (np.arange(T) + 1.0)
    if K == 1:
        t2 = bumps(rng, P, Q, 20.0, 150.0)
        sig = np.exp(-te[:, None, None] / t2[None])
        t2s = (t2,)
        frac = None
    elif K == 2:
        t2a = bumps(rng, P, Q, 15.0, 40.0)
        t2b = bumps(rng, P, Q, 60.0, 200.0)
        frac = bumps(rng, P, Q, 0.0, 1.0)
        sig = (frac[None] * np.exp(-te[:, None, None] / t2a[None])
               + (1.0 - frac[None]) * np.exp(-te[:, None, None] / t2b[None]))
        t2s = (t2a, t2b)
    else:
        raise ValueError("K must be 1 or 2")
    img = rho0[None] * sig
    if phase:
        phi = bumps(rng, P, Q, -math.pi, math.pi)
        img = img * np.exp(1j * phi)[None]
    return img.astype(np.complex128), t2s, frac


def make_mask(rng: np.random.Generator, P: int, Q: int, R: float) -> np.ndarray:
    """Variable-density random mask with exactly round(P*Q/R) samples (DC at [0,0]).

    Sampling weight (1 - |k|/|k|max)^2 with |k| from ``fftfreq``; a disc
    |k| < 4/P is always sampled; the remainder is drawn without replacement
    with probability proportional to the weight.
    """
    k1 = np.fft.fftfreq(P)[:, None]
    k2 = np.fft.fftfreq(Q)[None, :]
    kr = np.sqrt(k1 * k1 + k2 * k2)
    w = (1.0 - kr / kr.max()) ** 2
    n_tot = int(round(P * Q / R))
    S = np.zeros((P, Q), dtype=np.uint8)
    core = kr < 4.0 / P
    S[core] = 1
    n_core = int(core.sum())
    rest = np.flatnonzero(~core.ravel())
    n_more = max(0, n_tot - n_core)
    if n_more > 0:
        pw = w.ravel()[rest]
        pw = pw / pw.sum()
        pick = rng.choice(rest, size=n_more, replace=False, p=pw)
        S.ravel()[pick] = 1
    return S


def _unitary_fft2(img: np.ndarray) -> np.ndarray:
    return np.fft.fft2(img, norm="ortho")


def make_problem(seed: int, P: int, Q: int, T: int, K: int, R: float,
                 N1: int, N2: int, M: int, lam: float = 1e-3,
                 n_irls: int = 15, n_cg: int = 10, phase: bool = False,
                 snr_db: float = 40.0, name: str = "") -> Problem:
    """Draw one problem: images, per-echo masks, noisy sampled k-space."""
    rng = np.random.default_rng(seed)
    img, t2s, frac = make_images(rng, P, Q, T, K, phase)
    x = _unitary_fft2(img)
    S = np.stack([make_mask(rng, P, Q, R) for _ in range(T)])
    sel = S.astype(bool)
    nsel = int(sel.sum())
    sig = np.linalg.norm(x[sel]) / math.sqrt(max(nsel, 1)) * 10.0 ** (-snr_db / 20.0)
    noise = (rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape)) * (sig / math.sqrt(2.0))
    b = (S * (x + noise)).astype(np.complex64)
    return Problem(b=b, S=S, truth=img, N1=N1, N2=N2, M=M, lam=lam,
                   n_irls=n_irls, n_cg=n_cg, name=name, t2_maps=t2s, frac=frac)


def make_coils(rng: np.random.Generator, P: int, Q: int, ncoils: int) -> np.ndarray:
    """Smooth receive sensitivities, complex64 [Nc][P][Q], normalised to sum_j |C_j|^2 = 1.

    Coil j sits on a circle of radius 0.7 P around the frame centre at angle
    2 pi j / Nc (plus a uniform jitter of 0.2 rad); its magnitude is a Gaussian
    of width uniform in [0.35, 0.55] P around that point and its phase a plane
    wave with a uniform random gradient of at most pi across the frame plus a
    uniform offset.
    """
    r1 = np.arange(P)[:, None].astype(np.float64) - P / 2.0
    r2 = np.arange(Q)[None, :].astype(np.float64) - Q / 2.0
    C = np.zeros((ncoils, P, Q), dtype=np.complex128)
    for j in range(ncoils):
        ang = 2.0 * math.pi * j / ncoils + rng.uniform(-0.2, 0.2)
        c1, c2 = 0.7 * P * math.cos(ang), 0.7 * Q * math.sin(ang)
        sig = rng.uniform(0.35, 0.55) * P
        mag = np.exp(-((r1 - c1) ** 2 + (r2 - c2) ** 2) / (2.0 * sig * sig))
        g1, g2 = rng.uniform(-1.0, 1.0, size=2) * math.pi
        ph = g1 * r1 / P + g2 * r2 / Q + rng.uniform(-math.pi, math.pi)
        C[j] = mag * np.exp(1j * ph)
    C /= np.sqrt((np.abs(C) ** 2).sum(axis=0, keepdims=True))
    return C.astype(np.complex64)


def make_mc_problem(seed: int, P: int, Q: int, T: int, K: int, R: float, ncoils: int,
                    N1: int, N2: int, M: int, lam: float = 1e-3, n_irls: int = 15,
                    n_cg: int = 10, phase: bool = False, snr_db: float = 40.0,
                    name: str = "") -> Problem:
    """Multichannel problem (the measurement model of Sec. II.A): coil j of frame t
    is sampled as S_t o (F(C_j rho_t) + noise), with one mask per frame shared by
    the coils and complex Gaussian noise at ``snr_db`` per coil."""
    rng = np.random.default_rng(seed)
    img, t2s, frac = make_images(rng, P, Q, T, K, phase)
    C = make_coils(rng, P, Q, ncoils)
    S = np.stack([make_mask(rng, P, Q, R) for _ in range(T)])
    sel = S.astype(bool)
    nsel = int(sel.sum())
    b = np.zeros((ncoils, T, P, Q), dtype=np.complex64)
    for j in range(ncoils):
        x = _unitary_fft2(C[j].astype(np.complex128)[None] * img)
        sig = np.linalg.norm(x[sel]) / math.sqrt(max(nsel, 1)) * 10.0 ** (-snr_db / 20.0)
        noise = (rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape)) * (sig / math.sqrt(2.0))
        b[j] = (S * (x + noise)).astype(np.complex64)
    return Problem(b=b, S=S, truth=img, N1=N1, N2=N2, M=M, lam=lam, n_irls=n_irls,
                   n_cg=n_cg, name=name, t2_maps=t2s, frac=frac, coils=C)


# Named workloads: sizes, filter supports and iteration counts of the
# single-problem configurations (64^2 x 8 echoes, 128^2 x 16, 256^2 x 20).
CONFIGS = {
    "c1": dict(seed=1, P=64, Q=64, T=8, K=1, R=4, N1=5, N2=5, M=3, lam=1e-3,
               n_irls=15, n_cg=10, phase=False),
    "c2": dict(seed=2, P=128, Q=128, T=16, K=2, R=6, N1=9, N2=9, M=5, lam=1e-3,
               n_irls=15, n_cg=10, phase=False),
    "c3": dict(seed=3, P=256, Q=256, T=20, K=2, R=8, N1=15, N2=15, M=5, lam=1e-3,
               n_irls=20, n_cg=15, phase=True),
    # the c3 data under the pixel-wise prior (HLR-Voxel): a 1 x 1 x 5 filter per pixel
    "hlr": dict(seed=3, P=256, Q=256, T=20, K=2, R=8, N1=1, N2=1, M=5, lam=1e-3,
                n_irls=20, n_cg=15, phase=True),
}


# Multichannel workload shaped like the paper's multichannel experiment
# (128 x 128, 12 echoes 10 ms apart, 12 coils; Sec. IV).
MC_CONFIGS = {
    "mc": dict(seed=4, P=128, Q=128, T=12, K=2, R=8, ncoils=12, N1=9, N2=9, M=5, lam=1e-3,
               n_irls=15, n_cg=10, phase=False),
}


def config_problem(name: str, **over) -> Problem:
    if name in MC_CONFIGS:
        kw = dict(MC_CONFIGS[name])
        kw.update(over)
        return make_mc_problem(name=name, **kw)
    kw = dict(CONFIGS[name])
    kw.update(over)
    return make_problem(name=name, **kw)


def batch_specs(n: int = 32, seed: int = 11) -> list[dict]:
    """Uneven batch of slices: sizes {96..256}^2, T in {8,12,16,20}, K in {1,2},
    R in {4,6,8}, filter 9x9x5, 15 IRLS x 10 CG; slice j uses seed 1000 + j."""
    rng = np.random.default_rng(seed)
    out = []
    for j in range(n):
        P = int(rng.choice([96, 128, 160, 192, 256]))
        T = int(rng.choice([8, 12, 16, 20]))
        K = int(rng.choice([1, 2]))
        R = int(rng.choice([4, 6, 8]))
        out.append(dict(seed=1000 + j, P=P, Q=P, T=T, K=K, R=R, N1=9, N2=9, M=5,
                        lam=1e-3, n_irls=15, n_cg=10, phase=False))
    return out
