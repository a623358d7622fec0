"""The C-ABI library loads, exports every symbol include/la.h declares, and
rejects bad arguments before touching a device (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "la.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(la_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2112_09017_amd import _binding
    return _binding.lib()


def test_header_declares_expected_api():
    names = declared_functions()
    for n in ("la_create", "la_destroy", "la_gemm", "la_polar", "la_polar_workspace_size",
              "la_inverse", "la_inverse_workspace_size", "la_matfunc_odd", "la_matfunc_cheb",
              "la_matfunc_workspace_size", "la_tsqr", "la_tsqr_workspace_size", "la_wy",
              "la_wy_workspace_size", "la_caqr", "la_caqr_workspace_size", "la_serve_create", "la_serve_submit", "la_serve_poll", "la_serve_destroy",
              "la_status_string", "la_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(L):
    from paper_2112_09017_amd import _binding
    for name in declared_functions():
        assert hasattr(L, name), name
        assert name in _binding.SIGNATURES, f"binding lacks {name}"


def test_library_is_built_for_gfx950():
    from paper_2112_09017_amd import _binding
    blob = open(_binding.LIB_PATH, "rb").read()
    assert b"gfx950" in blob


def test_status_strings(L):
    # every status the header declares is named by la_status_string
    header = open(HEADER).read()
    enum = header[header.index("typedef enum {"):header.index("} la_status;")]
    declared = re.findall(r"\b(LA_(?:OK|ERR_\w+))\s*=\s*(\d+)", enum)
    assert len(declared) >= 12
    for name, value in declared:
        assert L.la_status_string(int(value)) == name.encode(), name
    assert L.la_status_string(999) == b"LA_ERR_UNKNOWN_STATUS"


def test_gemm_argument_validation_without_device(L):
    # bad precision, negative size, short leading dimension, then NULL context
    assert L.la_gemm(None, 0, 0, 4, 4, 4, 1.0, None, 4, None, 4, 0.0, None, 4, 7, None) == 1
    assert L.la_last_error().startswith(b"la_gemm: invalid precision")
    assert L.la_gemm(None, 0, 0, -1, 4, 4, 1.0, None, 4, None, 4, 0.0, None, 4, 0, None) == 2
    assert L.la_gemm(None, 0, 0, 4, 4, 8, 1.0, None, 4, None, 4, 0.0, None, 4, 0, None) == 2
    assert L.la_gemm(None, 1, 0, 8, 4, 4, 1.0, None, 4, None, 4, 0.0, None, 4, 0, None) == 2
    assert L.la_gemm(None, 0, 0, 4, 4, 4, 1.0, None, 4, None, 4, 0.0, None, 4, 0, None) == 1
    assert b"ctx is NULL" in L.la_last_error()


def test_polar_argument_validation_without_device(L):
    from paper_2112_09017_amd import _binding
    assert L.la_polar_workspace_size(3, 5, None) == 0          # M < N
    assert L.la_polar_workspace_size(0, 0, None) == 0
    ws = L.la_polar_workspace_size(300, 200, None)
    assert ws >= 4 * (300 * 200 + 200 * 200)
    o = _binding.make_opts(prec_ns=9)
    assert L.la_polar_workspace_size(8, 8, ctypes.byref(o)) == 0
    assert L.la_polar(None, 3, 5, None, 5, None, 5, None, 5, None, 0, None, None, None) == 2
    assert L.la_polar(None, 8, 8, None, 4, None, 8, None, 8, None, 0, None, None, None) == 2
    assert L.la_polar(None, 8, 8, None, 8, None, 8, None, 8, None, 0, None, None, None) == 1


def test_inverse_argument_validation_without_device(L):
    from paper_2112_09017_amd import _binding
    assert L.la_inverse_workspace_size(0, 4, None) == 0
    assert L.la_inverse_workspace_size(4, -1, None) == 0
    tall = L.la_inverse_workspace_size(300, 200, None)      # X is 200 x 300, product 200 x 200
    assert tall >= 4 * (300 * 200 + 200 * 200)
    wide = L.la_inverse_workspace_size(200, 300, None)      # product 200 x 200 as well
    assert wide >= 4 * (300 * 200 + 200 * 200)
    o = _binding.make_inverse_opts(prec=9)
    assert L.la_inverse_workspace_size(8, 8, ctypes.byref(o)) == 0
    o = _binding.make_inverse_opts(eps=-1.0)
    assert L.la_inverse_workspace_size(8, 8, ctypes.byref(o)) == 0
    # sizes, leading dimensions, then NULL arguments
    assert L.la_inverse(None, 0, 4, None, 4, None, 0, None, 0, None, None, None) == 2
    assert L.la_inverse(None, 8, 6, None, 5, None, 8, None, 0, None, None, None) == 2
    assert L.la_inverse(None, 8, 6, None, 6, None, 7, None, 0, None, None, None) == 2
    assert L.la_inverse(None, 8, 6, None, 6, None, 8, None, 0, None, None, None) == 1
    assert L.la_last_error() == b"la_inverse: NULL argument"


def test_matfunc_argument_validation_without_device(L):
    import numpy as np
    assert L.la_matfunc_workspace_size(0, 4) == 0
    assert L.la_matfunc_workspace_size(300, 200) >= 3 * 4 * 200 * 200
    c = np.array([1.0, 2.0])
    cp = c.ctypes.data
    # shape, coefficients, precision, then NULL arguments
    assert L.la_matfunc_odd(None, 0, 4, None, 4, cp, 2, None, 4, None, 0, 0, None) == 2
    assert L.la_matfunc_odd(None, 4, 4, None, 3, cp, 2, None, 4, None, 0, 0, None) == 2
    assert L.la_matfunc_odd(None, 4, 4, None, 4, cp, 0, None, 4, None, 0, 0, None) == 1
    assert L.la_matfunc_odd(None, 4, 4, None, 4, None, 2, None, 4, None, 0, 0, None) == 1
    bad = np.array([1.0, np.nan])
    assert L.la_matfunc_odd(None, 4, 4, None, 4, bad.ctypes.data, 2, None, 4, None, 0, 0,
                            None) == 1
    assert L.la_matfunc_odd(None, 4, 4, None, 4, cp, 2, None, 4, None, 0, 7, None) == 1
    assert L.la_matfunc_odd(None, 4, 4, None, 4, cp, 2, None, 4, None, 0, 0, None) == 1
    assert L.la_last_error() == b"la_matfunc_odd: NULL argument"
    assert L.la_matfunc_cheb(None, 4, None, 4, 1.0, 1.0, cp, 2, None, 4, None, 0, 0, None) == 1
    assert L.la_matfunc_cheb(None, 4, None, 4, 0.0, np.inf, cp, 2, None, 4, None, 0, 0,
                             None) == 1
    assert L.la_matfunc_cheb(None, 4, None, 2, 0.0, 1.0, cp, 2, None, 4, None, 0, 0, None) == 2
    assert L.la_matfunc_cheb(None, 4, None, 4, 0.0, 1.0, cp, 2, None, 4, None, 0, 0, None) == 1


def test_qr_argument_validation_without_device(L):
    # workspace sizes: 0 for rejected shapes
    assert L.la_tsqr_workspace_size(100, 0) == 0
    assert L.la_tsqr_workspace_size(100, 129) == 0
    assert L.la_tsqr_workspace_size(10, 20) == 0
    assert L.la_tsqr_workspace_size(256, 64) > 0          # one block: no tree buffers
    # 70000 x 32: 274 blocks, then 8768, 1120 and 160 stacked rows
    assert L.la_tsqr_workspace_size(70000, 32) >= 4 * 32 * (8768 + 1120 + 160)
    assert L.la_wy_workspace_size(0) == 0 and L.la_wy_workspace_size(64) >= 64 * 64 * 4
    assert L.la_caqr_workspace_size(100, 200, 64, 1) == 0
    assert L.la_caqr_workspace_size(100, 100, 0, 1) == 0
    assert L.la_caqr_workspace_size(100, 100, 129, 1) == 0
    with_q = L.la_caqr_workspace_size(1000, 512, 64, 1)
    assert with_q >= 2 * 4 * 1000 * 512 > L.la_caqr_workspace_size(1000, 512, 64, 0)
    # shape errors come before any device work
    assert L.la_tsqr(None, 10, 20, None, 20, None, 20, None, 20, None, 0, None) == 2
    assert L.la_tsqr(None, 300, 129, None, 129, None, 129, None, 129, None, 0, None) == 2
    assert L.la_tsqr(None, 300, 64, None, 63, None, 64, None, 64, None, 0, None) == 2
    assert L.la_tsqr(None, 300, 64, None, 64, None, 64, None, 64, None, 0, None) == 1
    assert L.la_wy(None, 300, 0, None, 64, None, 64, None, 64, None, 0, None) == 2
    assert L.la_wy(None, 300, 64, None, 64, None, 64, None, 64, None, 0, None) == 1
    assert L.la_caqr(None, 100, 200, None, 200, None, 200, 64, None, 0, 0, None) == 2
    assert L.la_caqr(None, 300, 200, None, 200, None, 200, 129, None, 0, 0, None) == 2
    assert L.la_caqr(None, 300, 200, None, 200, None, 200, 64, None, 0, 9, None) == 1
    assert L.la_caqr(None, 300, 200, None, 200, None, 200, 64, None, 0, 0, None) == 1
    assert L.la_last_error() == b"la_caqr: NULL argument"


def test_qr_rejects_workspace_over_inputs(L):
    # The checks compare address ranges only and come before the context is
    # read, so host addresses stand in for device ones (nothing is accessed).
    buf = ctypes.create_string_buffer(1 << 22)
    base = (ctypes.addressof(buf) + 255) & ~255
    ctx = base
    m, n = 300, 64
    need = L.la_tsqr_workspace_size(m, n)
    A, Q, R = base + (1 << 20), base + (2 << 20), base + (3 << 20)
    assert L.la_tsqr(ctx, m, n, A, n, Q, n, R, n, A, need, None) == 1
    assert b"must not overlap" in L.la_last_error()
    wneed = L.la_wy_workspace_size(n)
    assert L.la_wy(ctx, m, n, Q, n, A, n, R, n, Q, wneed, None) == 1
    assert b"must not overlap" in L.la_last_error()


def test_create_reports_missing_device(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    out = ctypes.c_void_p()
    st = L.la_create(0, ctypes.byref(out))
    assert st == 6 and not out.value
    assert L.la_last_error()


def test_destroy_accepts_null(L):
    assert L.la_destroy(None) == 0
    assert L.la_serve_destroy(None) == 0


def test_workspace_sizes_follow_the_slice_and_pack_policies(L):
    # host logic only: the sizes say how many split-K parts la_polar keeps
    # (Gram, update and H slices of at most max_acc_k = 4096 rows of K each,
    # or more slices to fill the CUs) and whether it holds packed 3xBF16 copies
    # for the update
    from paper_2112_09017_amd._binding import InverseOpts, PolarOpts
    MiB = 1 << 20
    m, n = 131072, 4096
    o = PolarOpts()
    o.prec_ns = 1                       # FP32 NS steps: no step at 3xBF16
    fp32_ns = L.la_polar_workspace_size(m, n, ctypes.byref(o))
    auto = L.la_polar_workspace_size(m, n, None)
    # the Gram takes 32 slices of 4096 rows (more than the 15 that fill the
    # CUs); H takes 32 slices of U^T A and 32 of A^T U: 64 n x n parts
    base = 4 * (m * n + n * n + 64 * n * n)
    assert base <= fp32_ns < base + MiB
    # packed copies: X and P for the update, or X^T for the Gram (136 upper
    # tiles), whichever is larger
    packed = max(L.la_pack_size(m, n) + L.la_pack_size(n, n), L.la_pack_size(n, m))
    assert base + packed <= auto < base + packed + MiB
    # a deeper accumulation: 16 Gram slices (still at least the 15 that fill
    # the CUs) and 2 x 16 for H
    o.max_acc_k = 8192
    base = 4 * (m * n + n * n + 32 * n * n)
    assert base <= L.la_polar_workspace_size(m, n, ctypes.byref(o)) < base + MiB
    o.max_acc_k = -1
    assert L.la_polar_workspace_size(m, n, ctypes.byref(o)) == 0
    # square 16384: Gram and update in 4 slices each, H in 2 x 4; packed
    # copies of U and P for the 3xBF16 update
    m = n = 16384
    base = 4 * (m * n + n * n + 8 * n * n)
    packed = L.la_pack_size(m, n) + L.la_pack_size(n, n)
    assert base + packed <= L.la_polar_workspace_size(m, n, None) < base + packed + MiB
    # accumulation over the whole K: only H's two parts
    o = PolarOpts()
    o.max_acc_k = 16384
    base2 = 4 * (m * n + n * n + 2 * n * n)
    assert base2 + packed <= L.la_polar_workspace_size(m, n, ctypes.byref(o)) < base2 + packed + MiB
    # the inverse keeps the packed operands of the larger of its two products,
    # and A packed once
    base = 4 * (m * n + n * n)
    packed += L.la_pack_size(n, n)
    assert base + packed <= L.la_inverse_workspace_size(n, n, None) < base + packed + MiB
    io = InverseOpts()
    io.prec = 1
    assert base <= L.la_inverse_workspace_size(n, n, ctypes.byref(io)) < base + MiB


def test_small_s_minus_is_rejected(L):
    """s_- below 1e-3 is rejected: the preconditioning polynomial's positive
    root 1/sqrt(c) sits only 0.385 s_- above 1, and the oracle's scalar map
    shows an FP32-size excess of the largest singular value over 1 flipping its
    sign there, while at s_- = 1e-3 the margin is far above such errors."""
    import oracle
    from paper_2112_09017_amd._binding import PolarOpts
    o = PolarOpts()
    o.s_minus = 1e-4
    assert L.la_polar_workspace_size(256, 256, ctypes.byref(o)) == 0
    o.s_minus = 1e-3
    assert L.la_polar_workspace_size(256, 256, ctypes.byref(o)) > 0
    a7 = oracle.precond_a(1e-7)
    assert oracle.precond_map(a7, 1.0 + 1e-7) < 0.0
    a3 = oracle.precond_map(oracle.precond_a(1e-3), 1.0 + 1e-5)
    assert a3 > 0.0
