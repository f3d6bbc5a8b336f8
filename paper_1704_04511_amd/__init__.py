"""Python binding of libslrx: IRLS structured low-rank recovery on MI355X.

Argument marshalling only.  Every step of the reconstruction runs in the HIP
library ``libslrx.so`` (built in-tree by ``paper_1704_04511_amd.build``); this
module converts NumPy arrays / torch tensors to pointers and C structs.  There
is no fallback: if the library is missing, importing :func:`lib` raises.

Arrays: complex64 ``[T, P, Q]`` k-space or images (DC at [0, 0]); uint8 masks.
Host NumPy arrays are copied by the library before a setter returns; torch
CUDA tensors are passed as device pointers on the plan's stream.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

# PyTorch's HIP runtime must be the one in the process before libslrx loads.
import torch  # noqa: F401

__all__ = [
    "Dims", "Params", "Stats", "RequestInfo", "Plan", "Server", "SlrxError", "lib", "library_path",
    "footprint", "validate", "default_params", "run_batch", "exported_symbols", "apply_noalloc",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
# SLRX_LIBRARY: another build of the library (e.g. the host-sanitizer build the tests make)
_LIB_PATH = os.environ.get("SLRX_LIBRARY") or os.path.join(_HERE, "libslrx.so")
_lib = None
_lock = threading.Lock()

SLRX_MEM_HOST = 0
SLRX_MEM_DEVICE = 1
SLRX_FLAG_TIMING = 1
SLRX_FLAG_KTIME = 2
SLRX_FLAG_LIBEIGH = 4
SLRX_FLAG_GIRAF = 8
SLRX_FLAG_NO_GRAPH = 32
SLRX_FLAG_HLR_VOXEL = 64
SLRX_FLAG_DIRECT = 128
MAX_IRLS = 256
KERNEL_CLASSES = ("rows", "cols", "fin", "update", "gram", "tri", "tdeig", "backtr", "filter", "masks", "coil",
                  "voxel", "direct")

STATUS = {0: "SLRX_OK", -1: "SLRX_EINVAL", -2: "SLRX_ENOMEM", -3: "SLRX_EDEVICE", -4: "SLRX_ESTATE",
          -5: "SLRX_ENUMERIC", -6: "SLRX_EBUSY", -7: "SLRX_ENOTREADY", -8: "SLRX_ECANCELED",
          -9: "SLRX_ETIMEDOUT"}


class SlrxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class Dims(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int32), ("Q", ctypes.c_int32), ("T", ctypes.c_int32),
                ("N1", ctypes.c_int32), ("N2", ctypes.c_int32), ("M", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("lam", ctypes.c_double), ("p", ctypes.c_double), ("gamma", ctypes.c_double),
                ("eps0_frac", ctypes.c_double), ("n_irls", ctypes.c_int32), ("n_cg", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class Stats(ctypes.Structure):
    _fields_ = [("n_irls_done", ctypes.c_int32),
                ("eps", ctypes.c_double * MAX_IRLS),
                ("lambda_max", ctypes.c_double * MAX_IRLS),
                ("cg_rr_final", ctypes.c_double * MAX_IRLS),
                ("ms_total", ctypes.c_double), ("ms_gram", ctypes.c_double), ("ms_eigh", ctypes.c_double),
                ("ms_weights", ctypes.c_double), ("ms_cg", ctypes.c_double),
                ("kt_ms", ctypes.c_double * 16), ("kt_count", ctypes.c_int32 * 16)]

    def as_dict(self) -> dict:
        n = self.n_irls_done
        return {"n_irls": n, "eps": list(self.eps[:n]), "lambda_max": list(self.lambda_max[:n]),
                "cg_rr_final": list(self.cg_rr_final[:n]), "ms_total": self.ms_total,
                "ms_gram": self.ms_gram, "ms_eigh": self.ms_eigh, "ms_weights": self.ms_weights,
                "ms_cg": self.ms_cg,
                "kernel_ms": {k: self.kt_ms[i] for i, k in enumerate(KERNEL_CLASSES)},
                "kernel_count": {k: self.kt_count[i] for i, k in enumerate(KERNEL_CLASSES)}}


class RequestInfo(ctypes.Structure):
    _fields_ = [("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("state", ctypes.c_int32), ("status", ctypes.c_int32), ("bytes", ctypes.c_size_t)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_SIGS = {
    "slrx_default_params": (None, [ctypes.POINTER(Params)]),
    "slrx_fault_alloc": (None, [ctypes.c_int32]),
    "slrx_set_cg_grouping": (None, [ctypes.c_int32]),
    "slrx_validate": (_I, [ctypes.POINTER(Dims), ctypes.POINTER(Params)]),
    "slrx_footprint": (ctypes.c_size_t, [ctypes.POINTER(Dims)]),
    "slrx_plan_create": (_I, [ctypes.POINTER(Dims), ctypes.POINTER(Params), _P, ctypes.POINTER(_P)]),
    "slrx_plan_destroy": (None, [_P]),
    "slrx_set_kspace": (_I, [_P, _P, _I]),
    "slrx_set_mask": (_I, [_P, _P, _I]),
    "slrx_set_coils": (_I, [_P, ctypes.c_int32, _P, _P, _I]),
    "slrx_fit_t2": (_I, [_P, _P, _P, _P, _P, _I]),
    "slrx_set_init": (_I, [_P, _P, _I]),
    "slrx_clear_init": (_I, [_P]),
    "slrx_set_filter": (_I, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "slrx_set_params": (_I, [_P, ctypes.POINTER(Params)]),
    "slrx_run": (_I, [_P]),
    "slrx_sync": (_I, [_P]),
    "slrx_get_images": (_I, [_P, _P, _I]),
    "slrx_get_kspace": (_I, [_P, _P, _I]),
    "slrx_get_stats": (_I, [_P, ctypes.POINTER(Stats)]),
    "slrx_run_batch": (_I, [ctypes.POINTER(_P), ctypes.c_int32, _P]),
    "slrx_step_gram": (_I, [_P, _P, _I]),
    "slrx_step_weights": (_I, [_P, ctypes.c_double, _P, _P, _P, _I]),
    "slrx_step_tdeig": (_I, [_P, _P, _P, _P, _P, _I]),
    "slrx_step_apply": (_I, [_P, _P, _P, _P, _I]),
    "slrx_step_cg": (_I, [_P, _P, ctypes.c_int32]),
    "slrx_server_create": (_I, [ctypes.c_size_t, ctypes.c_int32, _P, ctypes.POINTER(_P)]),
    "slrx_server_destroy": (None, [_P]),
    "slrx_submit": (_I, [_P, _P, ctypes.POINTER(ctypes.c_uint64)]),
    "slrx_poll": (_I, [_P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32)]),
    "slrx_wait": (_I, [_P, ctypes.c_uint64]),
    "slrx_submit_data": (_I, [_P, ctypes.POINTER(Dims), ctypes.POINTER(Params), _P, _P,
                              ctypes.POINTER(ctypes.c_uint64)]),
    "slrx_get_request_info": (_I, [_P, ctypes.c_uint64, ctypes.POINTER(RequestInfo)]),
    "slrx_server_usage": (_I, [_P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_int32)]),
    "slrx_fetch_images": (_I, [_P, ctypes.c_uint64, _P]),
    "slrx_release": (_I, [_P, ctypes.c_uint64]),
    "slrx_wait_for": (_I, [_P, ctypes.c_uint64, ctypes.c_double]),
    "slrx_cancel": (_I, [_P, ctypes.c_uint64]),
    "slrx_server_set_queue_timeout": (_I, [_P, ctypes.c_double]),
    "slrx_tri_workgroup_budget": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32]),
    "slrx_apply_noalloc_limit": (ctypes.c_size_t, []),
    "slrx_apply_noalloc": (_I, [ctypes.POINTER(Dims), ctypes.c_double, ctypes.c_uint32, _P, _P, _P, _P, _P]),
    "slrx_status_str": (ctypes.c_char_p, [_I]),
    "slrx_last_error": (ctypes.c_char_p, [_P]),
}


def exported_symbols() -> list[str]:
    return list(_SIGS)


def library_path() -> str:
    return _LIB_PATH


def lib():
    """Load libslrx.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                raise RuntimeError(f"libslrx.so not built at {_LIB_PATH}; run python -m paper_1704_04511_amd.build")
            L = ctypes.CDLL(_LIB_PATH)
            for name, (res, args) in _SIGS.items():
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            _lib = L
    return _lib


def _check(status: int, plan=None):
    """Raise SlrxError for a failed call; the message is the plan's last error
    (or the calling thread's, for calls without a plan)."""
    if status != 0:
        raise SlrxError(status, lib().slrx_last_error(plan).decode(errors="replace"))


def default_params() -> Params:
    p = Params()
    lib().slrx_default_params(ctypes.byref(p))
    return p


def make_params(lam=1e-3, n_irls=15, n_cg=10, p=0.6, gamma=1.4, eps0_frac=0.01, timing=False,
                ktime=False, lib_eigh=False, ktime_classes=None, giraf=False, no_graph=False,
                voxel=False, direct=False) -> Params:
    """ktime_classes: names from KERNEL_CLASSES to time (default: all, when ktime is set);
    giraf: the lifting circular along the parameter axis too (SLRX_FLAG_GIRAF);
    no_graph: CG kernels launched one by one instead of a replayed graph (SLRX_FLAG_NO_GRAPH);
    voxel: the pixel-wise prior HLR-Voxel (SLRX_FLAG_HLR_VOXEL; needs an N1 = N2 = 1 filter);
    direct: IRLS-direct on the explicit linear lifting (SLRX_FLAG_DIRECT)."""
    flags = ((SLRX_FLAG_TIMING if timing else 0) | (SLRX_FLAG_KTIME if ktime else 0)
             | (SLRX_FLAG_LIBEIGH if lib_eigh else 0) | (SLRX_FLAG_GIRAF if giraf else 0)
             | (SLRX_FLAG_NO_GRAPH if no_graph else 0) | (SLRX_FLAG_HLR_VOXEL if voxel else 0)
             | (SLRX_FLAG_DIRECT if direct else 0))
    for c in ktime_classes or ():
        flags |= 1 << (16 + KERNEL_CLASSES.index(c))
    return Params(float(lam), float(p), float(gamma), float(eps0_frac), int(n_irls), int(n_cg), flags)


def set_cg_grouping(mode: int) -> None:
    """CG strategy of batches and servers: -1 tuned online (default), 0 per problem, 1 grouped."""
    lib().slrx_set_cg_grouping(int(mode))


def validate(dims: Dims, params: Params | None = None) -> None:
    _check(lib().slrx_validate(ctypes.byref(dims), ctypes.byref(params) if params is not None else None))


def footprint(dims: Dims) -> int:
    return int(lib().slrx_footprint(ctypes.byref(dims)))


def _ptr(a, dtype, shape=None):
    """(pointer, mem kind, keep-alive) for a NumPy array or a torch device tensor."""
    if isinstance(a, torch.Tensor):
        if not a.is_cuda:
            a = a.contiguous().numpy()
        else:
            if not a.is_contiguous():
                raise ValueError("device tensors must be contiguous")
            tdt = {np.complex64: torch.complex64, np.uint8: torch.uint8, np.float64: torch.float64,
                   np.complex128: torch.complex128}[dtype]
            if a.dtype != tdt:
                raise TypeError(f"expected {tdt}, got {a.dtype}")
            if shape is not None and tuple(a.shape) != tuple(shape):
                raise ValueError(f"expected shape {shape}, got {tuple(a.shape)}")
            return ctypes.c_void_p(a.data_ptr()), SLRX_MEM_DEVICE, a
    arr = np.ascontiguousarray(a, dtype=dtype)
    if shape is not None and arr.shape != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {arr.shape}")
    return arr.ctypes.data_as(ctypes.c_void_p), SLRX_MEM_HOST, arr


class Plan:
    """One reconstruction problem resident on the GPU."""

    def __init__(self, P, Q, T, N1, N2, M, params: Params | None = None, stream=None):
        self.dims = Dims(P, Q, T, N1, N2, M)
        self.params = params if params is not None else default_params()
        h = ctypes.c_void_p()
        st = None if stream is None else ctypes.c_void_p(int(stream))
        _check(lib().slrx_plan_create(ctypes.byref(self.dims), ctypes.byref(self.params), st, ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def _c(self, status: int):
        _check(status, self._h)

    @property
    def shape(self):
        d = self.dims
        return (d.T, d.P, d.Q)

    @property
    def W(self):
        return self.dims.M * (self.dims.M + 1) // 2

    @property
    def s(self):
        d = self.dims
        return d.N1 * d.N2 * d.M

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().slrx_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_kspace(self, b):
        ptr, mem, keep = _ptr(b, np.complex64, self.shape)
        self._c(lib().slrx_set_kspace(self._h, ptr, mem))
        self._keep_b = keep

    def set_mask(self, S):
        ptr, mem, keep = _ptr(S, np.uint8, self.shape)
        self._c(lib().slrx_set_mask(self._h, ptr, mem))
        self._keep_S = keep

    def set_coils(self, C, b):
        """Multichannel data (``slrx_set_coils``): sensitivities C [Nc][P][Q] and
        coil k-space b [Nc][T][P][Q], both complex64, both host arrays or both
        device tensors; ``C=None`` returns to the single-channel model."""
        if C is None:
            self._c(lib().slrx_set_coils(self._h, 0, None, None, SLRX_MEM_HOST))
            self._keep_coils = None
            return
        d = self.dims
        nc = int(C.shape[0])
        cp, cm, ck = _ptr(C, np.complex64, (nc, d.P, d.Q))
        bp, bm, bk = _ptr(b, np.complex64, (nc, d.T, d.P, d.Q))
        if cm != bm:
            raise ValueError("coil maps and coil data must both be host arrays or both device tensors")
        self._c(lib().slrx_set_coils(self._h, nc, cp, bp, cm))
        self._keep_coils = (ck, bk)

    def fit_t2(self, te_ms, img=None):
        """Mono-exponential fit per pixel (``slrx_fit_t2``) of ``img`` (complex64
        [T][P][Q], host array) or, with ``img=None``, of the plan's reconstruction.
        Returns (T2, amplitude), float64 [P][Q] each."""
        d = self.dims
        te = np.ascontiguousarray(te_ms, dtype=np.float64)
        if te.shape != (d.T,):
            raise ValueError(f"expected {d.T} echo times, got {te.shape}")
        t2 = np.empty((d.P, d.Q), np.float64)
        amp = np.empty((d.P, d.Q), np.float64)
        ip, keep = (None, None)
        if img is not None:
            ip, _, keep = _ptr(np.ascontiguousarray(img, dtype=np.complex64), np.complex64, self.shape)
        self._c(lib().slrx_fit_t2(self._h, ip, te.ctypes.data_as(ctypes.c_void_p),
                                 t2.ctypes.data_as(ctypes.c_void_p), amp.ctypes.data_as(ctypes.c_void_p),
                                 SLRX_MEM_HOST))
        return t2, amp

    def set_init(self, x0):
        ptr, mem, keep = _ptr(x0, np.complex64, self.shape)
        self._c(lib().slrx_set_init(self._h, ptr, mem))
        self._keep_x0 = keep

    def clear_init(self):
        self._c(lib().slrx_clear_init(self._h))

    def set_filter(self, N1, N2, M):
        self._c(lib().slrx_set_filter(self._h, N1, N2, M))
        self.dims.N1, self.dims.N2, self.dims.M = N1, N2, M

    def set_params(self, params: Params):
        self._c(lib().slrx_set_params(self._h, ctypes.byref(params)))
        self.params = params

    def run(self):
        self._c(lib().slrx_run(self._h))

    def sync(self):
        self._c(lib().slrx_sync(self._h))

    def images(self, out=None):
        if out is None:
            out = np.empty(self.shape, np.complex64)
        ptr, mem, _ = _ptr(out, np.complex64, self.shape)
        self._c(lib().slrx_get_images(self._h, ptr, mem))
        return out

    def kspace(self, out=None):
        if out is None:
            out = np.empty(self.shape, np.complex64)
        ptr, mem, _ = _ptr(out, np.complex64, self.shape)
        self._c(lib().slrx_get_kspace(self._h, ptr, mem))
        return out

    def stats(self) -> dict:
        s = Stats()
        self._c(lib().slrx_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    # ---- single steps
    def step_gram(self):
        s = self.s
        R = np.empty((s, s), np.complex128, order="F")
        self._c(lib().slrx_step_gram(self._h, R.ctypes.data_as(ctypes.c_void_p), SLRX_MEM_HOST))
        return R

    def step_weights(self, eps: float):
        s, d = self.s, self.dims
        lam = np.empty(s, np.float64)
        H = np.empty((s, s), np.complex128)
        E = np.empty((self.W, d.P, d.Q), np.complex64)
        self._c(lib().slrx_step_weights(self._h, float(eps), lam.ctypes.data_as(ctypes.c_void_p),
                                       H.ctypes.data_as(ctypes.c_void_p), E.ctypes.data_as(ctypes.c_void_p),
                                       SLRX_MEM_HOST))
        return lam, H, E

    def step_voxel_masks(self, eps: float):
        """HLR-Voxel plans: the per-pixel masks E [W][P][Q] for the given eps (no lam or H)."""
        d = self.dims
        E = np.empty((self.W, d.P, d.Q), np.complex64)
        self._c(lib().slrx_step_weights(self._h, float(eps), None, None, E.ctypes.data_as(ctypes.c_void_p),
                                       SLRX_MEM_HOST))
        return E

    def step_tdeig(self, D, E):
        """Eigenpairs of the real symmetric tridiagonal (D, E) of size s (divide and conquer)."""
        s = self.s
        D = np.ascontiguousarray(D, np.float64)
        E = np.ascontiguousarray(E, np.float64)
        if D.shape != (s,) or E.shape != (max(s - 1, 0),):
            raise ValueError(f"expected D of {s} and E of {max(s - 1, 0)} entries")
        lam = np.empty(s, np.float64)
        Z = np.empty((s, s), np.complex128)  # column-major: Z[c] is eigenvector c
        Ep = E.ctypes.data_as(ctypes.c_void_p) if s > 1 else None
        self._c(lib().slrx_step_tdeig(self._h, D.ctypes.data_as(ctypes.c_void_p), Ep,
                                     lam.ctypes.data_as(ctypes.c_void_p), Z.ctypes.data_as(ctypes.c_void_p),
                                     SLRX_MEM_HOST))
        return lam, Z.T

    def step_apply(self, E, v):
        d = self.dims
        Ep, _, Ek = _ptr(E, np.complex64, (self.W, d.P, d.Q))
        vp, _, vk = _ptr(v, np.complex64, self.shape)
        out = np.empty(self.shape, np.complex64)
        self._c(lib().slrx_step_apply(self._h, Ep, vp, out.ctypes.data_as(ctypes.c_void_p), SLRX_MEM_HOST))
        return out

    def step_cg(self, E, n_cg: int):
        d = self.dims
        Ep, _, Ek = _ptr(E, np.complex64, (self.W, d.P, d.Q))
        self._c(lib().slrx_step_cg(self._h, Ep, int(n_cg)))


def apply_noalloc(dims: Dims, lam: float, S, E, v, out, stream=None, giraf: bool = False):
    """``slrx_apply_noalloc``: out = S o v + lam F G F^-1 v on device tensors (S uint8,
    E complex64 [W][P][Q], v and out complex64 [T][P][Q]), without a plan or any
    device allocation; enqueued on ``stream`` (a hipStream_t handle, None: default)."""
    shape = (dims.T, dims.P, dims.Q)
    W = dims.M * (dims.M + 1) // 2
    ptrs = []
    for a, dt, shp in ((S, np.uint8, shape), (E, np.complex64, (W, dims.P, dims.Q)), (v, np.complex64, shape),
                       (out, np.complex64, shape)):
        if not (isinstance(a, torch.Tensor) and a.is_cuda):
            raise TypeError("slrx_apply_noalloc takes device tensors")
        p, _, _ = _ptr(a, dt, shp)
        ptrs.append(p)
    st = None if stream is None else ctypes.c_void_p(int(stream))
    _check(lib().slrx_apply_noalloc(ctypes.byref(dims), float(lam), SLRX_FLAG_GIRAF if giraf else 0, *ptrs, st))


def run_batch(plans, stream=None, sync=True):
    """Run independent plans: in lock step on the engine when stream is None
    (one eigen-decomposition launch sequence per Gram size, other kernels on
    each plan's own stream), else one after another on the given stream."""
    arr = (ctypes.c_void_p * len(plans))(*[p.handle.value for p in plans])
    st = None if stream is None else ctypes.c_void_p(int(stream))
    _check(lib().slrx_run_batch(arr, len(plans), st))
    if sync:
        for p in plans:
            p.sync()


class Server:
    """Continuous-batching request server (see slrx.h)."""

    def __init__(self, budget_bytes: int, max_slots: int = 8, stream=None):
        h = ctypes.c_void_p()
        st = None if stream is None else ctypes.c_void_p(int(stream))
        _check(lib().slrx_server_create(int(budget_bytes), int(max_slots), st, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().slrx_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def wait_for(self, ticket: int, timeout_s: float) -> bool:
        """True when the request finished (ok) within timeout_s; False if not yet done."""
        st = lib().slrx_wait_for(self._h, ticket, float(timeout_s))
        if st == -7:
            return False
        _check(st)
        return True

    def cancel(self, ticket: int):
        _check(lib().slrx_cancel(self._h, ticket))

    def set_queue_timeout(self, seconds: float):
        _check(lib().slrx_server_set_queue_timeout(self._h, float(seconds)))

    def submit(self, plan: Plan) -> int:
        t = ctypes.c_uint64()
        _check(lib().slrx_submit(self._h, plan.handle, ctypes.byref(t)))
        return t.value

    def submit_data(self, b, S, N1, N2, M, params: Params | None = None) -> int:
        """Queue a reconstruction of host arrays; the server allocates its plan at admission."""
        b = np.ascontiguousarray(b, np.complex64)
        S = np.ascontiguousarray(S, np.uint8)
        if b.shape != S.shape or b.ndim != 3:
            raise ValueError("b and S must both be [T, P, Q]")
        T, P, Q = b.shape
        dims = Dims(P, Q, T, N1, N2, M)
        prm = params if params is not None else default_params()
        t = ctypes.c_uint64()
        _check(lib().slrx_submit_data(self._h, ctypes.byref(dims), ctypes.byref(prm),
                                      b.ctypes.data_as(ctypes.c_void_p), S.ctypes.data_as(ctypes.c_void_p),
                                      ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int) -> bool:
        d = ctypes.c_int32()
        _check(lib().slrx_poll(self._h, ticket, ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket: int):
        _check(lib().slrx_wait(self._h, ticket))

    def info(self, ticket: int) -> dict:
        ri = RequestInfo()
        _check(lib().slrx_get_request_info(self._h, ticket, ctypes.byref(ri)))
        return {"t_submit": ri.t_submit, "t_admit": ri.t_admit, "t_done": ri.t_done, "state": ri.state,
                "status": ri.status, "bytes": ri.bytes}

    def usage(self) -> tuple[int, int]:
        used = ctypes.c_size_t()
        q = ctypes.c_int32()
        _check(lib().slrx_server_usage(self._h, ctypes.byref(used), ctypes.byref(q)))
        return used.value, q.value

    def fetch(self, ticket: int, shape) -> np.ndarray:
        out = np.empty(shape, np.complex64)
        _check(lib().slrx_fetch_images(self._h, ticket, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def release(self, ticket: int):
        _check(lib().slrx_release(self._h, ticket))
