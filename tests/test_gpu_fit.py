"""GPU parity of the per-pixel mono-exponential fit (Sec. IV: T2 maps of the
reconstructed series) against the FP64 oracle on the same complex64 series.

Both sides fit in FP64 from the same FP32 values, so they differ only by
summation order and the last bit of log and exp: decay rates 1/T2 (0 for no
decay) agree to 1e-12 of the largest rate and amplitudes to 1e-12 relative.
Comparing rates rather than T2 keeps pixels whose slope is zero up to
rounding (T2 near infinity on either side) meaningful.
"""
import ctypes

import numpy as np
import pytest

import oracle
import workload
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

slrx = pytest.importorskip("paper_1704_04511_amd")


def _rates(t2):
    return np.where(np.isinf(t2), 0.0, 1.0 / t2)


@pytest.mark.parametrize("T,P,Q,K", [(16, 64, 64, 2), (2, 8, 8, 1), (32, 16, 96, 1), (20, 256, 256, 2)])
def test_fit_matches_oracle(T, P, Q, K):
    say(f"t2 fit T={T} P={P} Q={Q}")
    rng = np.random.default_rng(71)
    img, _, _ = workload.make_images(rng, P, Q, T, K, True)
    img = img + 0.01 * (rng.standard_normal(img.shape) + 1j * rng.standard_normal(img.shape))
    img = img.astype(np.complex64)
    img[:, 0, 0] = 0.0  # a pixel with no signal: floored magnitudes, slope 0
    te = 10.0 * (np.arange(T) + 1)
    with slrx.Plan(P, Q, T, 1, 1, 1) as pl:
        t2, amp = pl.fit_t2(te, img)
    t2_ref, amp_ref = oracle.t2_fit(img, te)
    r, r_ref = _rates(t2), _rates(t2_ref)
    assert np.abs(r - r_ref).max() <= 1e-12 * np.abs(r_ref).max()
    np.testing.assert_allclose(amp, amp_ref, rtol=1e-12)
    assert np.isinf(t2[0, 0]) and np.isinf(t2_ref[0, 0])


def test_fit_recovers_noiseless_decays():
    say("t2 fit noiseless")
    rng = np.random.default_rng(72)
    T, P, Q = 12, 32, 32
    te = 10.0 * (np.arange(T) + 1)
    t2 = rng.uniform(20.0, 150.0, size=(P, Q))
    amp = rng.uniform(0.2, 1.0, size=(P, Q))
    img = (amp[None] * np.exp(-te[:, None, None] / t2[None])).astype(np.complex64)
    with slrx.Plan(P, Q, T, 1, 1, 1) as pl:
        t2f, ampf = pl.fit_t2(te, img)
    np.testing.assert_allclose(t2f, t2, rtol=1e-5)  # float32 images: log|rho| to ~6e-8
    np.testing.assert_allclose(ampf, amp, rtol=1e-5)


def test_fit_of_the_reconstruction_equals_fit_of_its_images():
    say("t2 fit of a run")
    pb = workload.make_problem(seed=73, P=32, Q=32, T=8, K=1, R=3, N1=3, N2=3, M=2, n_irls=2, n_cg=4)
    te = 10.0 * (np.arange(8) + 1)
    with slrx.Plan(32, 32, 8, 3, 3, 2, slrx.make_params(lam=pb.lam, n_irls=2, n_cg=4)) as pl:
        pl.set_kspace(pb.b)
        pl.set_mask(pb.S)
        with pytest.raises(slrx.SlrxError):
            pl.fit_t2(te)  # no completed run yet
        pl.run()
        pl.sync()
        a = pl.fit_t2(te)
        img = pl.images()
        b = pl.fit_t2(te, img)
        c = pl.fit_t2(te)  # the reconstruction is kept
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    for u, v in zip(a, c):
        assert np.array_equal(u, v)


def test_fit_rejects_bad_arguments():
    say("t2 fit argument checks")
    lib = slrx.lib()
    out = np.zeros((8, 8))
    img = np.zeros((4, 8, 8), np.complex64)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    with slrx.Plan(8, 8, 4, 1, 1, 1) as pl:
        same = np.full(4, 5.0)
        assert lib.slrx_fit_t2(pl.handle, ptr(img), ptr(same), ptr(out), None, slrx.SLRX_MEM_HOST) == -1
        nan = np.array([1.0, np.nan, 3.0, 4.0])
        assert lib.slrx_fit_t2(pl.handle, ptr(img), ptr(nan), ptr(out), None, slrx.SLRX_MEM_HOST) == -1
        te = np.arange(4.0)
        assert lib.slrx_fit_t2(pl.handle, ptr(img), None, ptr(out), None, slrx.SLRX_MEM_HOST) == -1
        assert lib.slrx_fit_t2(pl.handle, ptr(img), ptr(te), None, None, slrx.SLRX_MEM_HOST) == -1
        assert lib.slrx_fit_t2(pl.handle, ptr(img), ptr(te), ptr(out), None, 9) == -1
        assert lib.slrx_fit_t2(pl.handle, ptr(img), ptr(te), ptr(out), None, slrx.SLRX_MEM_HOST) == 0
    with slrx.Plan(8, 8, 1, 1, 1, 1) as pl:
        one = np.zeros((1, 8, 8), np.complex64)
        assert lib.slrx_fit_t2(pl.handle, ptr(one), ptr(np.ones(1)), ptr(out), None, slrx.SLRX_MEM_HOST) == -1
