"""Mutation check of the oracle's pins: a plausible mistake planted in a copy of
the oracle (a conjugate on the wrong factor, a sign, an index, an exponent, a
dropped term, a wrong schedule) must make the pin suite fail.  Runs on the CPU
only; the repository's own oracle is never modified."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (original text, planted mistake) in oracle/slr.py
MUTATIONS = {
    "gram_conj_swap": ("c += np.conj(rho[(n - m) % T]) * rho[(n - mp) % T]",
                       "c += rho[(n - m) % T] * np.conj(rho[(n - mp) % T])"),
    "gram_lag_sign": ("d1 = (a1[:, None] - a1[None, :]) % P", "d1 = (a1[None, :] - a1[:, None]) % P"),
    "gram_range": ("for n in range(0 if circ_t else M - 1, T):\n                c +=",
                   "for n in range(0 if circ_t else M, T):\n                c +="),
    "spectra_sign": ("return scipy.fft.ifft2(frames, workers=-1) * (P * Q)", "return scipy.fft.fft2(frames, workers=-1)"),
    "alpha_exponent": ("alpha = (np.maximum(lam, 0.0) + eps) ** (p / 2.0 - 1.0)",
                       "alpha = (np.maximum(lam, 0.0) + eps) ** (p / 2.0 - 0.5)"),
    "mask_conj": ('E[m, mp] += np.einsum("ir,ir->r", cmu[:, m], mu[:, mp])',
                  'E[m, mp] += np.einsum("ir,ir->r", mu[:, m], cmu[:, mp])'),
    "penalty_swap": ("out[(n - m) % T] += E[m, mp] * rho[(n - mp) % T]",
                     "out[(n - mp) % T] += E[m, mp] * rho[(n - m) % T]"),
    "normal_transform_order": ("return S * xhat + lam * dft2(penalty_apply(idft2(xhat), E, circ_t))",
                               "return S * xhat + lam * idft2(penalty_apply(dft2(xhat), E, circ_t))"),
    "cg_beta": ("p = r + (rr_new / rr) * p", "p = r + (rr / rr_new) * p"),
    "eps_schedule": ("eps = eps / gamma", "eps = eps * gamma"),
    "eps_start": ("eps = eps0_frac * float(lamR.max())", "eps = eps0_frac * float(lamR.min() + lamR.max()/2)"),
    "lift_shift": ("vals = xhat[(n - m) % T][(w1 - a1[ia]) % P, (w2 - a2[ia]) % Q]",
                   "vals = xhat[(n - m) % T][(w1 + a1[ia]) % P, (w2 - a2[ia]) % Q]"),
}
# mistakes in the multichannel data term, checked against its own pins
COIL_MUTATIONS = {
    "coil_adjoint_conj": ("acc += np.conj(C[j])[None] * idft2(S * b[j])", "acc += C[j][None] * idft2(S * b[j])"),
    "coil_normal_conj": ("acc = acc + np.conj(C[j])[None] * idft2(S * dft2(C[j][None] * rho))",
                         "acc = acc + C[j][None] * idft2(S * dft2(C[j][None] * rho))"),
    "coil_normal_mask": ("acc = acc + np.conj(C[j])[None] * idft2(S * dft2(C[j][None] * rho))",
                         "acc = acc + np.conj(C[j])[None] * idft2(dft2(C[j][None] * rho))"),
    "coil_forward_transform": ("return np.stack([S * dft2(C[j][None] * rho) for j in range(C.shape[0])])",
                               "return np.stack([S * idft2(C[j][None] * rho) for j in range(C.shape[0])])"),
}
# mistakes in the mono-exponential fit, checked against its own pins
T2_MUTATIONS = {
    "t2_sign": ("t2 = np.where(slope < 0.0, -1.0 / np.where(slope < 0.0, slope, -1.0), np.inf)",
                "t2 = np.where(slope < 0.0, 1.0 / np.where(slope < 0.0, slope, -1.0), np.inf)"),
    "t2_uncentred": ("tc = te - te.mean()", "tc = te"),
    "t2_amplitude": ("amp = np.exp(ybar - slope * te.mean())", "amp = np.exp(ybar)"),
}
# mistakes in the circular (GIRAF) variant, checked against its own pins
GIRAF_MUTATIONS = {
    "giraf_gram_range": ("for n in range(0 if circ_t else M - 1, T):\n                c +=",
                         "for n in range(1 if circ_t else M - 1, T):\n                c +="),
    "giraf_penalty_wrap": ("out[(n - m) % T] += E[m, mp] * rho[(n - mp) % T]",
                           "out[(n - m) % T] += E[m, mp] * rho[max(n - mp, 0)]"),
}
# mistakes in the pixel-wise (HLR-Voxel) prior, checked against its own pins
VOXEL_MUTATIONS = {
    "voxel_mask_conj": ('E = np.einsum("...i,...mi,...ni->...mn", alpha, np.conj(U), U)',
                        'E = np.einsum("...i,...mi,...ni->...mn", alpha, U, np.conj(U))'),
    "voxel_gram_range": ("for n in range(M - 1, T))", "for n in range(M, T))"),
    "voxel_gram_conj": ("sum(np.conj(rho[n - m]) * rho[n - mp]", "sum(rho[n - m] * np.conj(rho[n - mp])"),
    "voxel_lambda_max": ("lmax = float(np.linalg.eigvalsh(G)[..., -1].max())",
                         "lmax = float(np.linalg.eigvalsh(G)[..., -1].mean())"),
}
# mistakes in the IRLS-direct functions (linear lifting), checked against their own pins
DIRECT_MUTATIONS = {
    "direct_lift_sign": ("out[rows, m * NN + ia] = xc[n - m][w1 - a1[ia], w2 - a2[ia]]",
                         "out[rows, m * NN + ia] = xc[n - m][w1 - a1[ia], w2 + a2[ia] - 1]"),
    "direct_adjoint_frame": ("np.add.at(xc[n - m], (w1 - a1[ia], w2 - a2[ia])",
                             "np.add.at(xc[n - m - 1], (w1 - a1[ia], w2 - a2[ia])"),
    "direct_weight_transpose": ("lift_linear(v, N1, N2, M) @ H, T, P, Q, N1, N2, M)",
                                "lift_linear(v, N1, N2, M) @ H.T, T, P, Q, N1, N2, M)"),
    "direct_rows_range": ("w1 = np.arange(a1.max(), P + a1.min())", "w1 = np.arange(a1.max(), P + a1.min() - 1)"),
}
PIN_FILE = {name: "tests/test_oracle_pins.py" for name in MUTATIONS}
PIN_FILE.update({name: "tests/test_oracle_giraf.py" for name in GIRAF_MUTATIONS})
PIN_FILE.update({name: "tests/test_oracle_coils.py" for name in COIL_MUTATIONS})
PIN_FILE.update({name: "tests/test_oracle_t2.py" for name in T2_MUTATIONS})
PIN_FILE.update({name: "tests/test_oracle_voxel.py" for name in VOXEL_MUTATIONS})
PIN_FILE.update({name: "tests/test_oracle_direct.py" for name in DIRECT_MUTATIONS})
ALL = dict(MUTATIONS, **COIL_MUTATIONS, **T2_MUTATIONS, **GIRAF_MUTATIONS, **VOXEL_MUTATIONS, **DIRECT_MUTATIONS)


@pytest.mark.parametrize("name", sorted(ALL))
def test_planted_mistake_is_caught(name, tmp_path):
    src = open(os.path.join(ROOT, "oracle", "slr.py")).read()
    orig, planted = ALL[name]
    assert orig in src, f"mutation site of {name} not found in the oracle"
    for d in ("oracle", "workload", "tests"):
        shutil.copytree(os.path.join(ROOT, d), tmp_path / d, ignore=shutil.ignore_patterns("__pycache__"))
    shutil.copy(os.path.join(ROOT, "pytest.ini"), tmp_path)
    (tmp_path / "oracle" / "slr.py").write_text(src.replace(orig, planted))
    env = dict(os.environ, PYTHONDONTWRITEBYTECODE="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        PIN_FILE[name]], cwd=tmp_path, capture_output=True, text=True, env=env,
                       timeout=600)
    assert r.returncode != 0, f"pins did not catch {name}:\n{r.stdout[-2000:]}"
