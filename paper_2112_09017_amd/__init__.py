"""MI355X (gfx950) FP32-accurate GEMM, Newton-Schulz polar factorisation and
Newton-Schulz inversion.

Python face of the C ABI in ``include/la.h`` (arXiv 2112.09017, sections III.A
and III.D).  Tensors are torch float32 CUDA (HIP) tensors; a 2-D tensor whose
last stride is 1 is passed as a row-major matrix, one whose first stride is 1
as the transpose of one (so ``A.T`` costs nothing).  All arithmetic runs in the
library's HIP kernels; nothing here computes.
"""
from __future__ import annotations

import ctypes

import torch

from ._binding import (InverseInfo, LAError, PolarInfo, PolarOpts, Precision, ServeConfig,
                       ServeStats, Status, check, context, lib, make_inverse_opts, make_opts,
                       LIB_PATH, SIGNATURES)

__all__ = ["gemm", "gemm_ws", "gemm_workspace_size", "pack_bf16x3", "gemm_packed", "polar", "polar_noalloc", "polar_workspace_size", "inverse", "inverse_workspace_size",
           "matfunc_odd", "matfunc_cheb", "tsqr", "wy", "caqr", "caqr_workspace_size",
           "Precision", "LAError", "Status", "lib", "LIB_PATH",
           "Server"]


def _stream_ptr(stream) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _as_matrix(t: torch.Tensor, name: str):
    """(pointer, rows, cols, ld, transposed) of a 2-D float32 device tensor."""
    if t.dtype != torch.float32 or t.dim() != 2 or not t.is_cuda:
        raise TypeError(f"{name} must be a 2-D float32 GPU tensor")
    r, c = t.shape
    s0, s1 = t.stride()
    if s1 == 1 and (s0 >= max(c, 1) or r <= 1):
        return t.data_ptr(), r, c, max(s0, c, 1), False
    if s0 == 1 and (s1 >= max(r, 1) or c <= 1):
        return t.data_ptr(), r, c, max(s1, r, 1), True
    raise ValueError(f"{name} must be row-major or a transpose of row-major (strides {t.stride()})")


def gemm(A: torch.Tensor, B: torch.Tensor, C: torch.Tensor | None = None, *, alpha: float = 1.0,
         beta: float = 0.0, prec: Precision = Precision.BF16X3, stream=None) -> torch.Tensor:
    """C <- alpha A @ B + beta C through ``la_gemm`` (eq. Matmul)."""
    pa, m, k, lda, ta = _as_matrix(A, "A")
    pb, k2, n, ldb, tb = _as_matrix(B, "B")
    if k != k2:
        raise ValueError(f"inner dimensions differ: {k} vs {k2}")
    if C is None:
        C = torch.empty((m, n), dtype=torch.float32, device=A.device)
        beta = 0.0
    pc, mc, nc, ldc, tc = _as_matrix(C, "C")
    if (mc, nc) != (m, n) or tc:
        raise ValueError("C must be a row-major m x n tensor")
    ctx = context(A.device.index if A.device.index is not None else torch.cuda.current_device())
    check(lib().la_gemm(ctx, int(ta), int(tb), m, n, k, float(alpha), pa, lda, pb, ldb,
                        float(beta), pc, ldc, int(prec), _stream_ptr(stream)))
    return C


def gemm_workspace_size(m: int, n: int, k: int) -> int:
    return int(lib().la_gemm_workspace_size(m, n, k))


def gemm_ws(A: torch.Tensor, B: torch.Tensor, C: torch.Tensor | None = None, *,
            alpha: float = 1.0, beta: float = 0.0, prec: Precision = Precision.BF16X3,
            workspace: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """C <- alpha A @ B + beta C through ``la_gemm_ws`` (packed 3xBF16 operands
    for large products; the same result as ``gemm``)."""
    pa, m, k, lda, ta = _as_matrix(A, "A")
    pb, k2, n, ldb, tb = _as_matrix(B, "B")
    if k != k2:
        raise ValueError(f"inner dimensions differ: {k} vs {k2}")
    if C is None:
        C = torch.empty((m, n), dtype=torch.float32, device=A.device)
        beta = 0.0
    pc, mc, nc, ldc, tc = _as_matrix(C, "C")
    if (mc, nc) != (m, n) or tc:
        raise ValueError("C must be a row-major m x n tensor")
    if workspace is None:
        workspace = torch.empty(gemm_workspace_size(m, n, k) + 256, dtype=torch.uint8,
                                device=A.device)
    wp = workspace.data_ptr()
    wp_al = (wp + 255) & ~255
    avail = max(workspace.numel() - (wp_al - wp), 0)
    ctx = context(A.device.index if A.device.index is not None else torch.cuda.current_device())
    check(lib().la_gemm_ws(ctx, int(ta), int(tb), m, n, k, float(alpha), pa, lda, pb, ldb,
                           float(beta), pc, ldc, int(prec), wp_al, avail, _stream_ptr(stream)))
    return C


def pack_bf16x3(X: torch.Tensor, *, out: torch.Tensor | None = None, stream=None):
    """Pack op(X) (rows x k, with X or X.T passed) through ``la_pack_bf16x3``:
    returns a uint8 device tensor usable by ``gemm_packed``."""
    px, r, c, ld, tx = _as_matrix(X, "X")
    # a row-major tensor is op(X) with k contiguous; a transposed view has rows contiguous
    need = int(lib().la_pack_size(r, c))
    if out is None:
        out = torch.empty(max(need, 1), dtype=torch.uint8, device=X.device)
    ctx = context(X.device.index if X.device.index is not None else torch.cuda.current_device())
    check(lib().la_pack_bf16x3(ctx, 0 if tx else 1, r, c, px, ld, out.data_ptr(), out.numel(),
                               _stream_ptr(stream)))
    return out


def gemm_packed(Ap: torch.Tensor, Bp: torch.Tensor, m: int, n: int, k: int,
                C: torch.Tensor | None = None, *, alpha: float = 1.0, beta: float = 0.0,
                stream=None) -> torch.Tensor:
    """C <- alpha op(A) op(B) + beta C from packed op(A) (m x k) and packed op(B)^T
    (n x k) through ``la_gemm_packed``."""
    if C is None:
        C = torch.empty((m, n), dtype=torch.float32, device=Ap.device)
        beta = 0.0
    pc, mc, nc, ldc, tc = _as_matrix(C, "C")
    if (mc, nc) != (m, n) or tc:
        raise ValueError("C must be a row-major m x n tensor")
    ctx = context(Ap.device.index if Ap.device.index is not None else torch.cuda.current_device())
    check(lib().la_gemm_packed(ctx, m, n, k, float(alpha), Ap.data_ptr(), Bp.data_ptr(),
                               float(beta), pc, ldc, _stream_ptr(stream)))
    return C


def polar_workspace_size(m: int, n: int, **opts) -> int:
    o = make_opts(**opts)
    return int(lib().la_polar_workspace_size(m, n, ctypes.byref(o)))


def polar(A: torch.Tensor, *, want_h: bool = True, U: torch.Tensor | None = None,
          H: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
          stream=None, raise_not_converged: bool = True, **opts):
    """Polar factorisation A = U H through ``la_polar`` (Algorithm NS_Polar).

    Returns (U, H or None, info dict).  ``opts`` are the fields of
    ``la_polar_opts`` (s_minus, s0, eps, max_iter, prec_precond, prec_ns,
    prec_h, polish, stagnation)."""
    pa, m, n, lda, ta = _as_matrix(A, "A")
    if ta:
        A = A.contiguous()
        pa, m, n, lda, ta = _as_matrix(A, "A")
    dev = A.device
    if U is None:
        U = torch.empty((m, n), dtype=torch.float32, device=dev)
    if want_h and H is None:
        H = torch.empty((n, n), dtype=torch.float32, device=dev)
    o = make_opts(**opts)
    need = int(lib().la_polar_workspace_size(m, n, ctypes.byref(o)))
    if need == 0:
        raise LAError(Status.SHAPE, f"bad polar shape {m} x {n}")
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    wp = workspace.data_ptr()
    wp_al = (wp + 255) & ~255
    avail = workspace.numel() - (wp_al - wp)
    pu, _, _, ldu, _ = _as_matrix(U, "U")
    ph, ldh = (0, n)
    if H is not None:
        ph, _, _, ldh, _ = _as_matrix(H, "H")
    info = PolarInfo()
    ctx = context(dev.index if dev.index is not None else torch.cuda.current_device())
    st = lib().la_polar(ctx, m, n, pa, lda, pu, ldu, ph or None, ldh, wp_al, avail,
                        ctypes.byref(o), ctypes.byref(info), _stream_ptr(stream))
    if st == Status.NOT_CONVERGED and not raise_not_converged:
        return U, H, info.as_dict()
    check(st)
    return U, (H if want_h else None), info.as_dict()


def polar_noalloc(A: torch.Tensor, *, want_h: bool = True, U: torch.Tensor | None = None,
                  H: torch.Tensor | None = None, stream=None, raise_not_converged: bool = True,
                  **opts):
    """``la_polar_noalloc``: la_polar with the library's static workspace
    (LA_POLAR_NOALLOC_BYTES per GPU); the library allocates nothing.  Returns
    (U, H or None, info dict) like ``polar``."""
    pa, m, n, lda, ta = _as_matrix(A, "A")
    if ta:
        raise ValueError("A must be row-major (contiguous rows)")
    dev = A.device
    if U is None:
        U = torch.empty((m, n), dtype=torch.float32, device=dev)
    if want_h and H is None:
        H = torch.empty((n, n), dtype=torch.float32, device=dev)
    o = make_opts(**opts)
    pu, _, _, ldu, _ = _as_matrix(U, "U")
    ph, ldh = (0, n)
    if H is not None:
        ph, _, _, ldh, _ = _as_matrix(H, "H")
    info = PolarInfo()
    ctx = context(dev.index if dev.index is not None else torch.cuda.current_device())
    st = lib().la_polar_noalloc(ctx, m, n, pa, lda, pu, ldu, ph or None, ldh, ctypes.byref(o),
                                ctypes.byref(info), _stream_ptr(stream))
    if st == Status.NOT_CONVERGED and not raise_not_converged:
        return U, H, info.as_dict()
    check(st)
    return U, (H if want_h else None), info.as_dict()


def inverse_workspace_size(n: int, m: int, **opts) -> int:
    o = make_inverse_opts(**opts)
    return int(lib().la_inverse_workspace_size(n, m, ctypes.byref(o)))


def inverse(A: torch.Tensor, *, X: torch.Tensor | None = None,
            workspace: torch.Tensor | None = None, stream=None,
            raise_not_converged: bool = True, **opts):
    """X with X A = I (A tall or square) or A X = I (A wide) through
    ``la_inverse`` (Algorithm NS_Inverse).  Returns (X, info dict).  ``opts``
    are the fields of ``la_inverse_opts`` (eps, max_iter, prec, polish,
    literal_delta)."""
    pa, n, m, lda, ta = _as_matrix(A, "A")
    if ta:
        A = A.contiguous()
        pa, n, m, lda, ta = _as_matrix(A, "A")
    dev = A.device
    if X is None:
        X = torch.empty((m, n), dtype=torch.float32, device=dev)
    o = make_inverse_opts(**opts)
    need = int(lib().la_inverse_workspace_size(n, m, ctypes.byref(o)))
    if need == 0:
        raise LAError(Status.SHAPE, f"bad inverse shape {n} x {m}")
    if workspace is None:
        workspace = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    wp = workspace.data_ptr()
    wp_al = (wp + 255) & ~255
    avail = max(workspace.numel() - (wp_al - wp), 0)   # a short one is reported by the library
    px, mx, nx, ldx, tx = _as_matrix(X, "X")
    if (mx, nx) != (m, n) or tx:
        raise ValueError("X must be a row-major m x n tensor")
    info = InverseInfo()
    ctx = context(dev.index if dev.index is not None else torch.cuda.current_device())
    st = lib().la_inverse(ctx, n, m, pa, lda, px, ldx, wp_al, avail, ctypes.byref(o),
                          ctypes.byref(info), _stream_ptr(stream))
    if st == Status.NOT_CONVERGED and not raise_not_converged:
        return X, info.as_dict()
    check(st)
    return X, info.as_dict()


def _coef_array(coef):
    import numpy as np
    c = np.ascontiguousarray(np.asarray(coef, dtype=np.float64).ravel())
    return c, c.ctypes.data


def _matfunc_workspace(workspace, m, n, dev):
    need = int(lib().la_matfunc_workspace_size(m, n))
    if workspace is None:
        workspace = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    wp = workspace.data_ptr()
    wp_al = (wp + 255) & ~255
    return workspace, wp_al, max(workspace.numel() - (wp_al - wp), 0)


def matfunc_odd(A: torch.Tensor, coef, *, F: torch.Tensor | None = None,
                prec: Precision = Precision.AUTO, workspace: torch.Tensor | None = None,
                stream=None) -> torch.Tensor:
    """F = sum_j coef[j] A (A^T A)^j through ``la_matfunc_odd`` (eq. OddPoly)."""
    pa, m, n, lda, ta = _as_matrix(A, "A")
    if ta:
        A = A.contiguous()
        pa, m, n, lda, ta = _as_matrix(A, "A")
    if F is None:
        F = torch.empty((m, n), dtype=torch.float32, device=A.device)
    pf, mf, nf, ldf, tf = _as_matrix(F, "F")
    if (mf, nf) != (m, n) or tf:
        raise ValueError("F must be a row-major m x n tensor")
    c, cp = _coef_array(coef)
    workspace, wp, avail = _matfunc_workspace(workspace, m, n, A.device)
    ctx = context(A.device.index if A.device.index is not None else torch.cuda.current_device())
    check(lib().la_matfunc_odd(ctx, m, n, pa, lda, cp, len(c), pf, ldf, wp, avail, int(prec),
                               _stream_ptr(stream)))
    return F


def matfunc_cheb(A: torch.Tensor, lo: float, hi: float, coef, *, F: torch.Tensor | None = None,
                 prec: Precision = Precision.AUTO, workspace: torch.Tensor | None = None,
                 stream=None) -> torch.Tensor:
    """F = sum_k coef[k] T_k((2A - (lo + hi) I) / (hi - lo)) through ``la_matfunc_cheb``
    (eq. EigenvaluePolynomial, Clenshaw's recurrence)."""
    pa, n, n2, lda, ta = _as_matrix(A, "A")
    if ta:
        A = A.contiguous()
        pa, n, n2, lda, ta = _as_matrix(A, "A")
    if n != n2:
        raise ValueError("A must be square")
    if F is None:
        F = torch.empty((n, n), dtype=torch.float32, device=A.device)
    pf, mf, nf, ldf, tf = _as_matrix(F, "F")
    if (mf, nf) != (n, n) or tf:
        raise ValueError("F must be a row-major n x n tensor")
    c, cp = _coef_array(coef)
    workspace, wp, avail = _matfunc_workspace(workspace, n, n, A.device)
    ctx = context(A.device.index if A.device.index is not None else torch.cuda.current_device())
    check(lib().la_matfunc_cheb(ctx, n, pa, lda, float(lo), float(hi), cp, len(c), pf, ldf, wp,
                                avail, int(prec), _stream_ptr(stream)))
    return F


def _workspace(workspace, need, dev):
    if workspace is None:
        workspace = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    wp = workspace.data_ptr()
    wp_al = (wp + 255) & ~255
    return workspace, wp_al, max(workspace.numel() - (wp_al - wp), 0)


def _ctx(t: torch.Tensor):
    return context(t.device.index if t.device.index is not None else torch.cuda.current_device())


def _row_major(A: torch.Tensor, name: str):
    pa, m, n, lda, ta = _as_matrix(A, name)
    if ta:
        A = A.contiguous()
        pa, m, n, lda, ta = _as_matrix(A, name)
    return A, pa, m, n, lda


def tsqr(A: torch.Tensor, *, workspace: torch.Tensor | None = None, stream=None):
    """Reduced QR (Q m x n, R n x n) of an m x n A (n <= 128) through ``la_tsqr``
    (Algorithm tsqr)."""
    A, pa, m, n, lda = _row_major(A, "A")
    Q = torch.empty((m, n), dtype=torch.float32, device=A.device)
    R = torch.empty((n, n), dtype=torch.float32, device=A.device)
    workspace, wp, avail = _workspace(workspace, int(lib().la_tsqr_workspace_size(m, n)), A.device)
    check(lib().la_tsqr(_ctx(A), m, n, pa, lda, Q.data_ptr(), n, R.data_ptr(), n, wp, avail,
                        _stream_ptr(stream)))
    return Q, R


def wy(Q: torch.Tensor, *, workspace: torch.Tensor | None = None, stream=None):
    """W = Q - [I; 0] and Y = W (I - Q_1)^-1 of a reduced Q (m x n, n <= 128)
    through ``la_wy`` (eq. Yamamoto): I - W Y^T is orthogonal with first n columns Q."""
    Q, pq, m, n, ldq = _row_major(Q, "Q")
    W = torch.empty((m, n), dtype=torch.float32, device=Q.device)
    Y = torch.empty((m, n), dtype=torch.float32, device=Q.device)
    workspace, wp, avail = _workspace(workspace, int(lib().la_wy_workspace_size(n)), Q.device)
    check(lib().la_wy(_ctx(Q), m, n, pq, ldq, W.data_ptr(), n, Y.data_ptr(), n, wp, avail,
                      _stream_ptr(stream)))
    return W, Y


def caqr_workspace_size(m: int, n: int, panel: int = 64, want_q: bool = True) -> int:
    return int(lib().la_caqr_workspace_size(m, n, panel, int(want_q)))


def caqr(A: torch.Tensor, *, panel: int = 64, want_q: bool = True, inplace: bool = False,
         prec: Precision = Precision.AUTO, workspace: torch.Tensor | None = None, stream=None):
    """QR of an m x n A (m >= n) through ``la_caqr`` (Algorithm caqr).  Returns
    (Q or None, R) with R the n x n upper triangle; the factorisation runs in
    place on A when ``inplace`` (A must then be row-major), else on a copy."""
    if inplace:
        pa, m, n, lda, ta = _as_matrix(A, "A")
        if ta:
            raise ValueError("inplace needs a row-major A")
        X = A
    else:
        X = A.contiguous().clone()
        pa, m, n, lda, _ = _as_matrix(X, "A")
    Q = torch.empty((m, n), dtype=torch.float32, device=A.device) if want_q else None
    workspace, wp, avail = _workspace(workspace, caqr_workspace_size(m, n, panel, want_q),
                                      A.device)
    check(lib().la_caqr(_ctx(A), m, n, pa, lda, Q.data_ptr() if want_q else None, n, panel, wp,
                        avail, int(prec), _stream_ptr(stream)))
    return Q, X[:n]


from .serve import Server  # noqa: E402
