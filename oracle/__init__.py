"""FP64 CPU oracle (test infrastructure only).

Plain, slow and obviously correct double-precision implementations of what the
GPU library computes, written from the paper (arXiv 2112.09017):

* ``gemm``      -- eq. (Matmul), section III.A: C_ij = sum_k A_ik B_kj;
* ``polar``     -- Algorithm NS_Polar with eqs. (a_def), (RogueScalar),
                   (RogueMatrix) and (NewtonSchulz), section III.D;
* ``polar_2x2`` -- the closed-form polar factor of a 2 x 2 matrix
                   (eqs. PolarDecomp, SVDdef);
* ``inverse``   -- Algorithm NS_Inverse (Newton-Schulz inversion), with its
                   scalar step ``inv_map``;
* ``matfunc_odd``  -- odd polynomial of the singular values (eq. OddPoly);
* ``matfunc_cheb`` -- Chebyshev polynomial of the eigenvalues
                   (eq. EigenvaluePolynomial);
* ``householder_qr`` -- reduced QR by Householder reflections (the local
                   factorisation of section III.B);
* ``tsqr``      -- Algorithm tsqr (row blocks, pairwise reduction of R);
* ``yamamoto``  -- the W, Y factors of eq. (Yamamoto);
* ``caqr``      -- Algorithm caqr (right-looking panel QR);
* scalar maps   -- eqs. (NS_scalar), (a_def), (RogueScalar) and the
                   preconditioning step count of Algorithm NS_Polar.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU library
and never imports it.  The arithmetic lives in ``la_oracle.c`` (built with gcc
by ``oracle/build.py``); this module only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_default = None


class _Info(ctypes.Structure):
    _fields_ = [
        ("iters_precond", ctypes.c_int),
        ("iters_ns", ctypes.c_int),
        ("fro_norm_a", ctypes.c_double),
        ("last_delta", ctypes.c_double),
        ("stop_reason", ctypes.c_int),
    ]


@dataclass
class PolarInfo:
    iters_precond: int
    iters_ns: int
    fro_norm_a: float
    last_delta: float
    stop_reason: str


_REASONS = {0: "tol", 1: "stagnation", 2: "cap"}


class _InvInfo(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int),
        ("stop_reason", ctypes.c_int),
        ("gram_norm", ctypes.c_double),
        ("last_delta", ctypes.c_double),
        ("last_tol", ctypes.c_double),
    ]


@dataclass
class InverseInfo:
    iters: int
    stop_reason: str
    gram_norm: float
    last_delta: float
    last_tol: float


def _bind(path: str):
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    lib.orc_gemm.argtypes = [ctypes.c_int, ctypes.c_int, i64, i64, i64, ctypes.c_double,
                             dp, i64, dp, i64, ctypes.c_double, dp, i64]
    lib.orc_gemm.restype = ctypes.c_int
    lib.orc_fro.argtypes = [i64, i64, dp, i64]
    lib.orc_fro.restype = ctypes.c_double
    lib.orc_precond_a.argtypes = [ctypes.c_double]
    lib.orc_precond_a.restype = ctypes.c_double
    lib.orc_precond_map.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.orc_precond_map.restype = ctypes.c_double
    lib.orc_ns_map.argtypes = [ctypes.c_double]
    lib.orc_ns_map.restype = ctypes.c_double
    lib.orc_precond_steps.argtypes = [ctypes.c_double, ctypes.c_double, dp]
    lib.orc_precond_steps.restype = ctypes.c_int
    lib.orc_polar.argtypes = [i64, i64, dp, i64, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                              dp, i64, dp, i64, ctypes.POINTER(_Info)]
    lib.orc_polar.restype = ctypes.c_int
    lib.orc_polar_2x2.argtypes = [dp, dp, dp]
    lib.orc_polar_2x2.restype = ctypes.c_int
    lib.orc_inv_map.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.orc_inv_map.restype = ctypes.c_double
    lib.orc_inverse.argtypes = [i64, i64, dp, i64, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                dp, i64, ctypes.c_void_p]
    lib.orc_inverse.restype = ctypes.c_int
    lib.orc_matfunc_odd.argtypes = [i64, i64, dp, i64, dp, ctypes.c_int, dp, i64]
    lib.orc_matfunc_odd.restype = ctypes.c_int
    lib.orc_matfunc_cheb.argtypes = [i64, dp, i64, ctypes.c_double, ctypes.c_double, dp,
                                     ctypes.c_int, dp, i64]
    lib.orc_matfunc_cheb.restype = ctypes.c_int
    lib.orc_householder_qr.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64]
    lib.orc_householder_qr.restype = ctypes.c_int
    lib.orc_tsqr.argtypes = [i64, i64, dp, i64, i64, dp, i64, dp, i64]
    lib.orc_tsqr.restype = ctypes.c_int
    lib.orc_yamamoto.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64]
    lib.orc_yamamoto.restype = ctypes.c_int
    lib.orc_caqr.argtypes = [i64, i64, dp, i64, i64, i64, dp, i64, dp, i64]
    lib.orc_caqr.restype = ctypes.c_int
    lib.orc_num_threads.argtypes = []
    lib.orc_num_threads.restype = ctypes.c_int
    return lib


def _load():
    global _default
    if _default is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b

            _b.build()
        _default = Oracle(_LIB_PATH)
    return _default


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Oracle:
    """One loaded build of ``la_oracle.c`` (the default one, or a variant)."""

    def __init__(self, path: str):
        self.path = path
        self._lib = _bind(path)

    def gemm(self, A, B, trans_a: bool = False, trans_b: bool = False, alpha: float = 1.0,
             beta: float = 0.0, C=None) -> np.ndarray:
        """alpha * op(A) @ op(B) + beta * C in FP64 (eq. Matmul). Inputs widen exactly."""
        lib = self._lib
        A = _f64(A)
        B = _f64(B)
        m, k = (A.shape[1], A.shape[0]) if trans_a else A.shape
        k2, n = (B.shape[1], B.shape[0]) if trans_b else B.shape
        if k != k2:
            raise ValueError(f"inner dimensions differ: {k} vs {k2}")
        out = _f64(C).copy() if (C is not None and beta != 0.0) else np.zeros((m, n), np.float64)
        rc = lib.orc_gemm(int(trans_a), int(trans_b), m, n, k, alpha, _ptr(A), A.shape[1],
                          _ptr(B), B.shape[1], beta, _ptr(out), n)
        if rc != 0:
            raise MemoryError("orc_gemm allocation failed")
        return out

    def fro(self, A) -> float:
        """||A||_F = sqrt(tr(A A^T)) in FP64."""
        A = _f64(A)
        if A.ndim == 1:
            A = A.reshape(1, -1)
        return float(self._lib.orc_fro(A.shape[0], A.shape[1], _ptr(A), A.shape[1]))

    def precond_a(self, s_minus: float) -> float:
        """eq. (a_def)."""
        return float(self._lib.orc_precond_a(s_minus))

    def precond_map(self, a: float, x: float) -> float:
        """eq. (RogueScalar)."""
        return float(self._lib.orc_precond_map(a, x))

    def ns_map(self, x: float) -> float:
        """eq. (NS_scalar)."""
        return float(self._lib.orc_ns_map(x))

    def precond_steps(self, s0: float, s_minus: float = 0.1) -> tuple[int, float]:
        """Preconditioning step count of Algorithm NS_Polar and the final s."""
        end = ctypes.c_double(0.0)
        k = self._lib.orc_precond_steps(s0, s_minus, ctypes.byref(end))
        return int(k), float(end.value)

    def polar(self, A, s_minus: float = 0.1, s0: float = 2.0 ** -52, eps: float = 2.0 ** -52,
              max_iter: int = 200, stagnation: bool = True, want_h: bool = True,
              max_precond: int = -1):
        """Algorithm NS_Polar in FP64.  Returns (U, H or None, PolarInfo).

        ``max_precond >= 0`` caps the preconditioning loop and ``max_iter`` the
        Newton-Schulz loop, so intermediate iterates can be inspected.
        """
        lib = self._lib
        A = _f64(A)
        m, n = A.shape
        U = np.zeros((m, n), np.float64)
        H = np.zeros((n, n), np.float64) if want_h else None
        info = _Info()
        rc = lib.orc_polar(m, n, _ptr(A), n, s_minus, s0, eps, max_precond, max_iter,
                           int(stagnation),
                           _ptr(U), n, _ptr(H) if H is not None else None, n,
                           ctypes.byref(info))
        if rc == -2:
            raise FloatingPointError("||A||_F is zero or not finite")
        if rc != 0:
            raise ValueError("orc_polar: bad arguments or allocation failure")
        pi = PolarInfo(info.iters_precond, info.iters_ns, info.fro_norm_a, info.last_delta,
                       _REASONS.get(info.stop_reason, "?"))
        return U, H, pi

    def num_threads(self) -> int:
        """OpenMP threads the oracle's GEMM uses."""
        return int(self._lib.orc_num_threads())

    def inv_map(self, d: float, x: float) -> float:
        """One Newton-Schulz inversion step on a scalar: x (2 - d x)."""
        return float(self._lib.orc_inv_map(d, x))

    def inverse(self, A, u: float = 2.0 ** -53, normalize: bool = True, max_iter: int = 200):
        """Algorithm NS_Inverse in FP64.  A is n x m; returns (X (m x n), InverseInfo).
        X A = I for n >= m, A X = I for n <= m.  ``u`` is the starting tolerance
        (the unit roundoff of the precision being emulated); ``normalize``
        measures the step on A / sqrt(||A A^T||_F) (see la_oracle.c)."""
        A = _f64(A)
        n, m = A.shape
        X = np.zeros((m, n), np.float64)
        info = _InvInfo()
        rc = self._lib.orc_inverse(n, m, _ptr(A), m, u, int(normalize), max_iter, _ptr(X), n,
                                   ctypes.byref(info))
        if rc == -2:
            raise FloatingPointError("||A A^T||_F is zero or not finite")
        if rc != 0:
            raise ValueError("orc_inverse: bad arguments or allocation failure")
        return X, InverseInfo(info.iters, _REASONS.get(info.stop_reason, "?"), info.gram_norm,
                              info.last_delta, info.last_tol)

    def matfunc_odd(self, A, coef):
        """F = sum_j coef[j] A (A^T A)^j in FP64 (eq. OddPoly)."""
        A = _f64(A)
        c = _f64(coef).ravel()
        m, n = A.shape
        F = np.zeros((m, n), np.float64)
        if self._lib.orc_matfunc_odd(m, n, _ptr(A), n, _ptr(c), len(c), _ptr(F), n) != 0:
            raise ValueError("orc_matfunc_odd: bad arguments or allocation failure")
        return F

    def matfunc_cheb(self, A, lo, hi, coef):
        """F = sum_k coef[k] T_k((2A - (lo+hi) I) / (hi - lo)) in FP64
        (eq. EigenvaluePolynomial); coef[0] carries full weight."""
        A = _f64(A)
        c = _f64(coef).ravel()
        n = A.shape[0]
        if A.shape != (n, n):
            raise ValueError("A must be square")
        F = np.zeros((n, n), np.float64)
        if self._lib.orc_matfunc_cheb(n, _ptr(A), n, lo, hi, _ptr(c), len(c), _ptr(F), n) != 0:
            raise ValueError("orc_matfunc_cheb: bad arguments or allocation failure")
        return F

    def householder_qr(self, A):
        """Reduced QR (Q m x n, R n x n upper triangular) of an m x n A, m >= n,
        by Householder reflections with R_jj of the sign opposite to A_jj."""
        A = _f64(A)
        m, n = A.shape
        Q = np.zeros((m, n))
        R = np.zeros((n, n))
        if self._lib.orc_householder_qr(m, n, _ptr(A), n, _ptr(Q), n, _ptr(R), n) != 0:
            raise ValueError("orc_householder_qr: bad arguments or allocation failure")
        return Q, R

    def tsqr(self, A, block_rows: int):
        """Algorithm tsqr with row blocks of ``block_rows`` (>= n) rows; the last
        block takes the remainder.  Returns (Q, R)."""
        A = _f64(A)
        m, n = A.shape
        Q = np.zeros((m, n))
        R = np.zeros((n, n))
        if self._lib.orc_tsqr(m, n, _ptr(A), n, block_rows, _ptr(Q), n, _ptr(R), n) != 0:
            raise ValueError("orc_tsqr: bad arguments or allocation failure")
        return Q, R

    def yamamoto(self, Q):
        """W = Q - [I; 0] and Y = W (I - Q_1)^-1 (eq. Yamamoto with T^-1 read as
        (I - Q_1)^T), so that I - W Y^T is the full orthogonal factor whose
        first n columns are Q."""
        Q = _f64(Q)
        m, n = Q.shape
        W = np.zeros((m, n))
        Y = np.zeros((m, n))
        rc = self._lib.orc_yamamoto(m, n, _ptr(Q), n, _ptr(W), n, _ptr(Y), n)
        if rc == -3:
            raise np.linalg.LinAlgError("I - Q_1 is singular")
        if rc != 0:
            raise ValueError("orc_yamamoto: bad arguments or allocation failure")
        return W, Y

    def caqr(self, A, panel: int, block_rows: int, want_q: bool = True):
        """Algorithm caqr: panels of ``panel`` columns (dividing n), each by tsqr
        with row blocks of ``block_rows``.  Returns (Q or None, R)."""
        A = _f64(A)
        m, n = A.shape
        Q = np.zeros((m, n)) if want_q else None
        R = np.zeros((n, n))
        rc = self._lib.orc_caqr(m, n, _ptr(A), n, panel, block_rows,
                                _ptr(Q) if want_q else None, n, _ptr(R), n)
        if rc == -3:
            raise np.linalg.LinAlgError("I - Q_1 is singular in a panel")
        if rc != 0:
            raise ValueError("orc_caqr: bad arguments or allocation failure")
        return Q, R

    def polar_2x2(self, A):
        """Closed-form polar factors (U, H) of a full-rank 2 x 2 matrix."""
        A = _f64(A).reshape(2, 2)
        U = np.zeros((2, 2))
        H = np.zeros((2, 2))
        if self._lib.orc_polar_2x2(_ptr(A), _ptr(U), _ptr(H)) != 0:
            raise ValueError("singular 2x2 input")
        return U, H


def gemm(*a, **k):
    return _load().gemm(*a, **k)


def fro(*a, **k):
    return _load().fro(*a, **k)


def precond_a(*a, **k):
    return _load().precond_a(*a, **k)


def precond_map(*a, **k):
    return _load().precond_map(*a, **k)


def ns_map(*a, **k):
    return _load().ns_map(*a, **k)


def precond_steps(*a, **k):
    return _load().precond_steps(*a, **k)


def polar(*a, **k):
    return _load().polar(*a, **k)


def polar_2x2(*a, **k):
    return _load().polar_2x2(*a, **k)


def inv_map(*a, **k):
    return _load().inv_map(*a, **k)


def inverse(*a, **k):
    return _load().inverse(*a, **k)


def matfunc_odd(*a, **k):
    return _load().matfunc_odd(*a, **k)


def matfunc_cheb(*a, **k):
    return _load().matfunc_cheb(*a, **k)


def householder_qr(*a, **k):
    return _load().householder_qr(*a, **k)


def tsqr(*a, **k):
    return _load().tsqr(*a, **k)


def yamamoto(*a, **k):
    return _load().yamamoto(*a, **k)


def caqr(*a, **k):
    return _load().caqr(*a, **k)


def num_threads():
    return _load().num_threads()


gemm.__doc__ = Oracle.gemm.__doc__
polar.__doc__ = Oracle.polar.__doc__
polar_2x2.__doc__ = Oracle.polar_2x2.__doc__
