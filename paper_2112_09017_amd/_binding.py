"""ctypes binding of ``libla.so`` (the C ABI in ``include/la.h``).

Argument marshalling only: torch tensors provide device memory and streams,
every computation runs in the library's HIP kernels.  There is no fallback:
if ``libla.so`` is missing or the device is not gfx950, calls raise.
"""
from __future__ import annotations

import ctypes
import enum
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libla.so")

_lib = None
_lock = threading.Lock()
_contexts: dict[int, ctypes.c_void_p] = {}


class Precision(enum.IntEnum):
    AUTO = 0
    FP32 = 1
    BF16X3 = 2
    BF16X6 = 3


class Status(enum.IntEnum):
    OK = 0
    INVALID_ARG = 1
    SHAPE = 2
    NONFINITE = 3
    NOT_CONVERGED = 4
    OUT_OF_MEMORY = 5
    DEVICE = 6
    QUEUE_FULL = 7
    TOO_LARGE = 8
    NOT_READY = 9
    UNKNOWN_REQUEST = 10
    BREAKDOWN = 11


class LAError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = Status(status) if status in Status._value2member_map_ else status
        super().__init__(f"{getattr(self.status, 'name', status)}: {message}")


class PolarOpts(ctypes.Structure):
    _fields_ = [
        ("s_minus", ctypes.c_double),
        ("s0", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("max_iter", ctypes.c_int),
        ("prec_precond", ctypes.c_int),
        ("prec_ns", ctypes.c_int),
        ("prec_h", ctypes.c_int),
        ("polish", ctypes.c_int),
        ("no_stagnation", ctypes.c_int),
        ("max_acc_k", ctypes.c_int),
        ("reserved", ctypes.c_int * 2),
    ]


class PolarInfo(ctypes.Structure):
    _fields_ = [
        ("iters_precond", ctypes.c_int),
        ("iters_ns", ctypes.c_int),
        ("fro_norm_a", ctypes.c_double),
        ("last_delta", ctypes.c_double),
        ("stop_reason", ctypes.c_int),
        ("prec_precond", ctypes.c_int),
        ("prec_ns", ctypes.c_int),
        ("prec_h", ctypes.c_int),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class InverseOpts(ctypes.Structure):
    _fields_ = [
        ("eps", ctypes.c_double),
        ("max_iter", ctypes.c_int),
        ("prec", ctypes.c_int),
        ("polish", ctypes.c_int),
        ("literal_delta", ctypes.c_int),
        ("reserved", ctypes.c_int * 4),
    ]


class InverseInfo(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int),
        ("product_side", ctypes.c_int),
        ("gram_norm", ctypes.c_double),
        ("last_delta", ctypes.c_double),
        ("last_tol", ctypes.c_double),
        ("stop_reason", ctypes.c_int),
        ("prec", ctypes.c_int),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServeConfig(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int), ("max_queue", ctypes.c_int),
                ("bands", ctypes.c_int), ("reserved", ctypes.c_int * 5)]


class ServeStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64),
        ("completed", ctypes.c_uint64),
        ("failed", ctypes.c_uint64),
        ("ticks", ctypes.c_uint64),
        ("active", ctypes.c_int),
        ("queued", ctypes.c_int),
        ("busy_seconds", ctypes.c_double),
        ("arena_high_water", ctypes.c_size_t),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


# Every symbol include/la.h declares, with its ctypes signature.
_VP = ctypes.c_void_p
_I64 = ctypes.c_int64
SIGNATURES = {
    "la_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_VP)]),
    "la_destroy": (ctypes.c_int, [_VP]),
    "la_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "la_last_error": (ctypes.c_char_p, []),
    "la_gemm": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, _I64, _I64, _I64, ctypes.c_float,
                               _VP, _I64, _VP, _I64, ctypes.c_float, _VP, _I64, ctypes.c_int,
                               _VP]),
    "la_gemm_workspace_size": (ctypes.c_size_t, [_I64, _I64, _I64]),
    "la_gemm_ws": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, _I64, _I64, _I64,
                                  ctypes.c_float, _VP, _I64, _VP, _I64, ctypes.c_float, _VP, _I64,
                                  ctypes.c_int, _VP, ctypes.c_size_t, _VP]),
    "la_pack_size": (ctypes.c_size_t, [_I64, _I64]),
    "la_pack_bf16x3": (ctypes.c_int, [_VP, ctypes.c_int, _I64, _I64, _VP, _I64, _VP,
                                      ctypes.c_size_t, _VP]),
    "la_gemm_packed": (ctypes.c_int, [_VP, _I64, _I64, _I64, ctypes.c_float, _VP, _VP,
                                      ctypes.c_float, _VP, _I64, _VP]),
    "la_polar_workspace_size": (ctypes.c_size_t, [_I64, _I64, ctypes.POINTER(PolarOpts)]),
    "la_polar": (ctypes.c_int, [_VP, _I64, _I64, _VP, _I64, _VP, _I64, _VP, _I64, _VP,
                                ctypes.c_size_t, ctypes.POINTER(PolarOpts),
                                ctypes.POINTER(PolarInfo), _VP]),
    "la_polar_noalloc": (ctypes.c_int, [_VP, _I64, _I64, _VP, _I64, _VP, _I64, _VP, _I64,
                                        ctypes.POINTER(PolarOpts), ctypes.POINTER(PolarInfo),
                                        _VP]),
    "la_inverse_workspace_size": (ctypes.c_size_t, [_I64, _I64, ctypes.POINTER(InverseOpts)]),
    "la_inverse": (ctypes.c_int, [_VP, _I64, _I64, _VP, _I64, _VP, _I64, _VP, ctypes.c_size_t,
                                  ctypes.POINTER(InverseOpts), ctypes.POINTER(InverseInfo), _VP]),
    "la_matfunc_workspace_size": (ctypes.c_size_t, [_I64, _I64]),
    "la_matfunc_odd": (ctypes.c_int, [_VP, _I64, _I64, _VP, _I64, _VP, ctypes.c_int, _VP, _I64,
                                      _VP, ctypes.c_size_t, ctypes.c_int, _VP]),
    "la_matfunc_cheb": (ctypes.c_int, [_VP, _I64, _VP, _I64, ctypes.c_double, ctypes.c_double,
                                       _VP, ctypes.c_int, _VP, _I64, _VP, ctypes.c_size_t,
                                       ctypes.c_int, _VP]),
    "la_tsqr_workspace_size": (ctypes.c_size_t, [_I64, _I64]),
    "la_tsqr": (ctypes.c_int, [_VP, _I64, _I64, _VP, _I64, _VP, _I64, _VP, _I64, _VP,
                               ctypes.c_size_t, _VP]),
    "la_wy_workspace_size": (ctypes.c_size_t, [_I64]),
    "la_wy": (ctypes.c_int, [_VP, _I64, _I64, _VP, _I64, _VP, _I64, _VP, _I64, _VP,
                             ctypes.c_size_t, _VP]),
    "la_caqr_workspace_size": (ctypes.c_size_t, [_I64, _I64, ctypes.c_int, ctypes.c_int]),
    "la_caqr": (ctypes.c_int, [_VP, _I64, _I64, _VP, _I64, _VP, _I64, ctypes.c_int, _VP,
                               ctypes.c_size_t, ctypes.c_int, _VP]),
    "la_serve_create": (ctypes.c_int, [_VP, ctypes.POINTER(ServeConfig), _VP, ctypes.c_size_t,
                                       ctypes.POINTER(_VP)]),
    "la_serve_submit": (ctypes.c_int, [_VP, _I64, _I64, _VP, _I64, ctypes.POINTER(PolarOpts),
                                       ctypes.POINTER(ctypes.c_uint64)]),
    "la_serve_poll": (ctypes.c_int, [_VP, ctypes.c_uint64, _VP, _VP, ctypes.POINTER(PolarInfo),
                                     ctypes.POINTER(ctypes.c_int)]),
    "la_serve_stats_get": (ctypes.c_int, [_VP, ctypes.POINTER(ServeStats)]),
    "la_serve_destroy": (ctypes.c_int, [_VP]),
}


def lib():
    """The loaded ``libla.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(
                    f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                    "(hipcc, gfx950); there is no fallback implementation")
            L = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            _lib = L
    return _lib


def check(status: int):
    if status != 0:
        L = lib()
        raise LAError(status, (L.la_last_error() or b"").decode(errors="replace"))


def context(device: int) -> ctypes.c_void_p:
    with _lock:
        ctx = _contexts.get(device)
    if ctx is not None:
        return ctx
    L = lib()
    out = _VP()
    check(L.la_create(device, ctypes.byref(out)))
    with _lock:
        _contexts.setdefault(device, out)
        return _contexts[device]


def make_opts(s_minus=0.0, s0=0.0, eps=0.0, max_iter=0, prec_precond=Precision.AUTO,
              prec_ns=Precision.AUTO, prec_h=Precision.AUTO, polish=False,
              stagnation=True, max_acc_k=0) -> PolarOpts:
    o = PolarOpts()
    o.s_minus = s_minus
    o.s0 = s0
    o.eps = eps
    o.max_iter = max_iter
    o.prec_precond = int(prec_precond)
    o.prec_ns = int(prec_ns)
    o.prec_h = int(prec_h)
    o.polish = 1 if polish else 0
    o.no_stagnation = 0 if stagnation else 1
    o.max_acc_k = int(max_acc_k)
    return o


def make_inverse_opts(eps=0.0, max_iter=0, prec=Precision.AUTO, polish=False,
                      literal_delta=False) -> InverseOpts:
    o = InverseOpts()
    o.eps = eps
    o.max_iter = max_iter
    o.prec = int(prec)
    o.polish = 1 if polish else 0
    o.literal_delta = 1 if literal_delta else 0
    return o
