"""slrx_apply_noalloc, the allocation-free variant of slrx_step_apply: through the
C ABI on device tensors, two calls in a row (the second on a smaller problem,
so stale scratch contents of the first are in the way), each checked against
slrx_step_apply on the same inputs and against the FP64 oracle; sizes beyond
the scratch limit are refused before any device work; device memory in use
does not change across calls."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import crandn, masks_to_pairs, nrmse, pairs_to_masks, say

pytestmark = pytest.mark.gpu

slrx = pytest.importorskip("paper_1704_04511_amd")
torch = pytest.importorskip("torch")


def case(seed, T, P, Q, N1, N2, M, giraf=False):
    rng = np.random.default_rng(seed)
    x = crandn(rng, T, P, Q).astype(np.complex64)
    S = (rng.random((T, P, Q)) < 0.4).astype(np.uint8)
    R = oracle.gram(x.astype(np.complex128), N1, N2, M, circ_t=giraf)
    lam_R, U, alpha = oracle.eig_weights(R, 0.05 * np.linalg.eigvalsh(R).max(), 0.6)
    Ew = masks_to_pairs(oracle.penalty_masks(U, alpha, N1, N2, M, P, Q))
    v = crandn(rng, T, P, Q).astype(np.complex64)
    lam = 0.7 / np.abs(Ew).max()
    return x, S, Ew, v, lam


def via_plan(shape, x, S, Ew, v, lam, giraf):
    T, P, Q, N1, N2, M = shape
    prm = slrx.make_params(lam=lam, n_irls=1, n_cg=1, giraf=giraf)
    with slrx.Plan(P, Q, T, N1, N2, M, prm) as pl:
        pl.set_kspace(x)
        pl.set_mask(S)
        return pl.step_apply(Ew, v)


def test_noalloc_apply_matches_step_apply_twice_then_smaller():
    shapes = [((20, 256, 256, 15, 15, 5), False), ((8, 64, 64, 5, 5, 3), False), ((6, 32, 96, 4, 5, 3), True)]
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    for i, (shape, giraf) in enumerate(shapes):
        T, P, Q, N1, N2, M = shape
        say(f"apply_noalloc call {i}: {shape} giraf={giraf}")
        x, S, Ew, v, lam = case(40 + i, *shape, giraf=giraf)
        dS, dE, dv = (torch.from_numpy(a).cuda() for a in (S, Ew, v))
        out = torch.empty((T, P, Q), dtype=torch.complex64, device="cuda")
        torch.cuda.synchronize()
        slrx.apply_noalloc(slrx.Dims(P, Q, T, N1, N2, M), lam, dS, dE, dv, out, stream=stream.cuda_stream,
                           giraf=giraf)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        ref = via_plan(shape, x, S, Ew, v, lam, giraf)
        e_plan = nrmse(got, ref)
        e_ora = nrmse(got, oracle.normal_apply(v.astype(np.complex128), S, pairs_to_masks(Ew, M), lam,
                                               circ_t=giraf))
        print(f"  vs slrx_step_apply {e_plan:.2e}, vs oracle {e_ora:.2e}", flush=True)
        # same kernels; only the twiddle tables are formed on the device instead of the host
        assert e_plan < 1e-6
        assert e_ora < 2e-6
        del dS, dE, dv, out
    torch.cuda.synchronize()


def test_noalloc_apply_makes_no_device_allocation():
    torch.cuda.set_device(0)
    T, P, Q, N1, N2, M = 8, 64, 64, 5, 5, 3
    x, S, Ew, v, lam = case(60, T, P, Q, N1, N2, M)
    dS, dE, dv = (torch.from_numpy(a).cuda() for a in (S, Ew, v))
    out = torch.empty((T, P, Q), dtype=torch.complex64, device="cuda")
    dims = slrx.Dims(P, Q, T, N1, N2, M)
    slrx.apply_noalloc(dims, lam, dS, dE, dv, out)  # first call on this device looks up the scratch
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(5):
        slrx.apply_noalloc(dims, lam, dS, dE, dv, out)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0


def test_noalloc_apply_refuses_sizes_beyond_its_scratch():
    torch.cuda.set_device(0)
    limit = int(slrx.lib().slrx_apply_noalloc_limit())
    assert limit == 24 << 20
    T, P, Q, M = 32, 256, 256, 8  # 8 (2 097 152 + 36 x 65 536) bytes > 24 MiB
    assert 8 * (T * P * Q + M * (M + 1) // 2 * P * Q) > limit
    dims = slrx.Dims(P, Q, T, 3, 3, M)
    S = torch.zeros((T, P, Q), dtype=torch.uint8, device="cuda")
    E = torch.zeros((M * (M + 1) // 2, P, Q), dtype=torch.complex64, device="cuda")
    v = torch.zeros((T, P, Q), dtype=torch.complex64, device="cuda")
    out = torch.zeros_like(v)
    with pytest.raises(slrx.SlrxError) as ei:
        slrx.apply_noalloc(dims, 1e-3, S, E, v, out)
    assert ei.value.name == "SLRX_EINVAL"
    assert "limit" in str(ei.value)
    assert not out.any()
