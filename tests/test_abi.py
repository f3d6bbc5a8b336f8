"""C ABI checks that need no GPU: the library loads, exports every symbol the
header declares, validates arguments before touching the device and reports
errors through status codes and messages."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "slrx.h")

slrx = pytest.importorskip("paper_1704_04511_amd")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(slrx_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    path = slrx.library_path()
    assert os.path.exists(path), "build the library first"
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (slrx_[a-z_0-9]+)", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    L = slrx.lib()
    for f in declared_functions():
        assert hasattr(L, f)


def test_binding_covers_declared_functions():
    assert set(declared_functions()) <= set(slrx.exported_symbols())


def test_default_params():
    p = slrx.default_params()
    assert (p.p, p.gamma, p.eps0_frac, p.n_irls, p.n_cg) == (0.6, 1.4, 0.01, 15, 10)


@pytest.mark.parametrize("dims,msg", [
    ((60, 64, 8, 5, 5, 3), "unsupported frame size"),
    ((64, 64, 0, 5, 5, 3), "T=0"),
    ((64, 64, 40, 5, 5, 3), "T=40"),
    ((64, 64, 8, 5, 5, 9), "M=9"),
    ((64, 64, 4, 5, 5, 5), "M=5"),
    ((64, 64, 8, 65, 5, 3), "does not fit"),
    ((64, 64, 8, 5, 0, 3), "does not fit"),
    ((256, 256, 32, 40, 40, 8), "exceeds"),
    ((256, 256, 32, 25, 25, 5), "exceeds"),  # s = 3125: beyond the eigensolver chain (3000)
])
def test_invalid_dims_rejected(dims, msg):
    with pytest.raises(slrx.SlrxError) as ei:
        slrx.validate(slrx.Dims(*dims))
    assert ei.value.name == "SLRX_EINVAL"
    assert msg in str(ei.value)


@pytest.mark.parametrize("kw,msg", [
    (dict(lam=-1.0), "lambda"),
    (dict(lam=float("nan")), "lambda"),
    (dict(p=1.5), "p must"),
    (dict(gamma=1.0), "gamma"),
    (dict(eps0_frac=0.0), "eps0_frac"),
    (dict(n_irls=0), "n_irls"),
    (dict(n_irls=1000), "n_irls"),
    (dict(n_cg=-1), "n_cg"),
])
def test_invalid_params_rejected(kw, msg):
    with pytest.raises(slrx.SlrxError) as ei:
        slrx.validate(slrx.Dims(64, 64, 8, 5, 5, 3), slrx.make_params(**kw))
    assert ei.value.name == "SLRX_EINVAL"
    assert msg in str(ei.value)


@pytest.mark.parametrize("dims,kw,msg", [
    ((64, 64, 8, 3, 1, 3), dict(voxel=True), "N1 = N2 = 1"),
    ((64, 64, 8, 1, 1, 3), dict(voxel=True, giraf=True), "does not combine"),
    ((64, 64, 8, 1, 1, 3), dict(voxel=True, lib_eigh=True), "does not combine"),
    ((64, 64, 8, 3, 3, 3), dict(direct=True, giraf=True), "does not combine"),
    ((64, 64, 8, 1, 1, 3), dict(direct=True, voxel=True), "does not combine"),
    ((64, 64, 8, 3, 3, 3), dict(direct=True, lib_eigh=True), "does not combine"),
])
def test_voxel_flag_constraints(dims, kw, msg):
    with pytest.raises(slrx.SlrxError) as ei:
        slrx.validate(slrx.Dims(*dims), slrx.make_params(**kw))
    assert ei.value.name == "SLRX_EINVAL"
    assert msg in str(ei.value)
    slrx.validate(slrx.Dims(64, 64, 8, 1, 1, 3), slrx.make_params(voxel=True))


def test_footprint_grows_with_problem():
    f1 = slrx.footprint(slrx.Dims(64, 64, 8, 5, 5, 3))
    f2 = slrx.footprint(slrx.Dims(128, 128, 16, 9, 9, 5))
    f3 = slrx.footprint(slrx.Dims(256, 256, 20, 15, 15, 5))
    assert 0 < f1 < f2 < f3
    # nine complex64 volumes plus the s x s FP64 matrices at least
    V, s = 256 * 256 * 20, 15 * 15 * 5
    assert f3 >= 9 * V * 8 + 4 * s * s * 8
    assert slrx.footprint(slrx.Dims(60, 64, 8, 5, 5, 3)) == 0


def test_status_strings():
    L = slrx.lib()
    assert L.slrx_status_str(0) == b"ok"
    assert L.slrx_status_str(-1) == b"invalid argument"
    assert L.slrx_status_str(-7) == b"not ready"
    assert L.slrx_status_str(-8) == b"canceled"
    assert L.slrx_status_str(-9) == b"timed out"


def test_thread_last_error_without_a_plan():
    L = slrx.lib()
    assert L.slrx_validate(None, None) == -1
    msg = L.slrx_last_error(None)
    assert b"dims is NULL" in msg
    # a failure on another thread leaves this thread's message alone
    import threading
    t = threading.Thread(target=lambda: L.slrx_footprint(None))
    t.start()
    t.join()
    assert L.slrx_last_error(None) == msg


def test_null_arguments_rejected():
    L = slrx.lib()
    assert L.slrx_validate(None, None) == -1
    assert b"NULL" in L.slrx_last_error(None)
    assert L.slrx_plan_create(None, None, None, None) == -1
    assert L.slrx_run(None) == -1
    assert L.slrx_sync(None) == -1
    assert L.slrx_get_images(None, None, 0) == -1
    assert L.slrx_run_batch(None, 1, None) == -1


def test_plan_create_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(slrx.SlrxError) as ei:
        slrx.Plan(64, 64, 8, 5, 5, 3)
    assert ei.value.name == "SLRX_EDEVICE"


def test_kernel_classes_match_header():
    import re
    src = open(HEADER).read()
    enum = {m.group(1).lower(): int(m.group(2)) for m in re.finditer(r"SLRX_K_([A-Z]+)\s*=\s*(\d+)", src)}
    n = enum.pop("nclass")
    assert [k for k, _ in sorted(enum.items(), key=lambda kv: kv[1])] == list(slrx.KERNEL_CLASSES)
    assert n == len(slrx.KERNEL_CLASSES) <= 16
    # int32 + pad, three FP64 histories, five timings, 16 class times, 16 class counts
    assert ctypes.sizeof(slrx.Stats) == 8 + 3 * 8 * slrx.MAX_IRLS + 5 * 8 + 16 * 8 + 16 * 4
