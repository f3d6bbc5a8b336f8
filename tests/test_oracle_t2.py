"""Pins of the oracle's per-pixel mono-exponential fit (Sec. IV: T2 maps from the
reconstructed series): exact recovery of noiseless decays, agreement with a
library least-squares line fit, and the no-decay case."""
import numpy as np

import oracle


def test_t2_fit_recovers_noiseless_decays_exactly():
    rng = np.random.default_rng(10)
    te = 10.0 * (np.arange(12) + 1)
    t2 = rng.uniform(15.0, 200.0, size=(8, 9))
    amp = rng.uniform(0.1, 2.0, size=(8, 9))
    ph = np.exp(1j * rng.uniform(-np.pi, np.pi, size=(8, 9)))
    img = amp[None] * ph[None] * np.exp(-te[:, None, None] / t2[None])
    t2f, ampf = oracle.t2_fit(img, te)
    np.testing.assert_allclose(t2f, t2, rtol=1e-12)
    np.testing.assert_allclose(ampf, amp, rtol=1e-12)


def test_t2_fit_equals_a_library_line_fit():
    rng = np.random.default_rng(11)
    te = np.array([8.0, 17.0, 31.0, 44.0, 60.0, 71.0])
    img = rng.uniform(0.05, 1.0, size=(6, 5, 4)) * np.exp(1j * rng.standard_normal((6, 5, 4)))
    t2f, ampf = oracle.t2_fit(img, te)
    y = np.log(np.abs(img)).reshape(6, -1)
    coef = np.polyfit(te, y, 1)  # rows: slope, intercept
    slope, icpt = coef[0].reshape(5, 4), coef[1].reshape(5, 4)
    np.testing.assert_allclose(np.exp(icpt), ampf, rtol=1e-10)
    neg = slope < 0
    np.testing.assert_allclose(t2f[neg], -1.0 / slope[neg], rtol=1e-10)
    assert np.all(np.isinf(t2f[~neg]))


def test_t2_fit_of_a_constant_series_is_infinite():
    img = np.full((5, 2, 3), 0.7 + 0.2j)
    t2f, ampf = oracle.t2_fit(img, 10.0 * (np.arange(5) + 1))
    assert np.all(np.isinf(t2f)) and np.allclose(ampf, abs(0.7 + 0.2j), rtol=1e-13)
