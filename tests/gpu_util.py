"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import sys

import numpy as np


def say(msg: str):
    """Name the case on stdout before a GPU step (flushed, so it survives a crash)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def nrmse(a, ref):
    ref = np.asarray(ref)
    return float(np.linalg.norm(np.asarray(a) - ref) / np.linalg.norm(ref))


def crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def pairs(M):
    return [(m, mp) for m in range(M) for mp in range(m, M)]


def masks_to_pairs(E_full):
    """[M][M][P][Q] masks -> the [W][P][Q] upper-triangle layout of the C ABI."""
    M = E_full.shape[0]
    return np.stack([E_full[m, mp] for m, mp in pairs(M)]).astype(np.complex64)


def pairs_to_masks(E_w, M):
    P, Q = E_w.shape[1:]
    E = np.zeros((M, M, P, Q), np.complex128)
    for w, (m, mp) in enumerate(pairs(M)):
        E[m, mp] = E_w[w]
        E[mp, m] = np.conj(E_w[w])
    return E
