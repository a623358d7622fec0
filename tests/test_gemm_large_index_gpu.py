"""GEMMs with an operand of 2^31 elements (A 65536 x 32768 FP32, 8 GiB): element
offsets past 2^31 must be formed in 64-bit arithmetic on every path.

* C = A B (A k-contiguous) and C' = A^T B' (the same storage read as the
  transposed operand, k-major) through la_gemm_ws (packed operands) and la_gemm
  (unpacked), which take every product in the same order: bitwise equal;
* sampled 64-row blocks of each result, including the last rows, whose operand
  offsets lie beyond 2^31, against the FP64 oracle (eq. Matmul): normwise error
  per block within the GEMM tolerance of 1e-6;
* an operand whose leading dimension (2^23 + 64) is past the interior loader's
  32-bit offset range, on the guarded loader, against the oracle.
"""
import numpy as np
import pytest
import torch

import la_inputs
import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

M, K, N = 65536, 32768, 256
T = 64
TOL = 1e-6


@pytest.fixture(scope="module")
def la():
    import paper_2112_09017_amd as la
    la.lib()
    return la


def check_blocks(C, rows, ref_fn, name):
    for r in rows:
        ref = ref_fn(r)
        a_norm, b_norm = ref[1], ref[2]
        d = np.linalg.norm(C[r:r + T].astype(np.float64) - ref[0])
        err = d / (a_norm * b_norm)
        assert err <= TOL, f"{name}: rows {r}..{r + T}: normwise error {err:.3g}"


def test_operand_of_2_31_elements(la):
    A = la_inputs.gaussian((M, K), 221)
    B = la_inputs.gaussian((K, N), 222)
    B2 = la_inputs.gaussian((M, N), 223)
    Ad = torch.from_numpy(A).to("cuda")
    prec = la.Precision.BF16X3
    g = np.random.default_rng(224)
    B64 = B.astype(np.float64)
    B264 = B2.astype(np.float64)
    nB, nB2 = float(np.linalg.norm(B64)), float(np.linalg.norm(B264))

    # A B: rows of A are k-contiguous
    Bd = torch.from_numpy(B).to("cuda")
    C_ws = la.gemm_ws(Ad, Bd, prec=prec)
    C_un = la.gemm(Ad, Bd, prec=prec)
    torch.cuda.synchronize()
    assert torch.equal(C_ws, C_un), "packed and unpacked results differ (A B)"
    C = C_ws.cpu().numpy()
    del C_ws, C_un, Bd
    rows = [0, M - T] + [int(g.integers(0, M // T)) * T for _ in range(2)]

    def ref_ab(r):
        a = A[r:r + T]
        return (oracle.gemm(a, B), float(np.linalg.norm(a.astype(np.float64))), nB)

    check_blocks(C, rows, ref_ab, "A B")

    # A^T B2: the same storage as a k-major operand (element (i, k) at k * K + i)
    B2d = torch.from_numpy(B2).to("cuda")
    C_ws = la.gemm_ws(Ad.T, B2d, prec=prec)
    C_un = la.gemm(Ad.T, B2d, prec=prec)
    torch.cuda.synchronize()
    assert torch.equal(C_ws, C_un), "packed and unpacked results differ (A^T B)"
    Ct = C_ws.cpu().numpy()
    assert Ct.shape == (K, N)
    rows = [0, K - T] + [int(g.integers(0, K // T)) * T for _ in range(2)]

    def ref_atb(r):
        a = np.ascontiguousarray(A[:, r:r + T])   # M x T: columns r.. of A
        return (oracle.gemm(a, B2, trans_a=True), float(np.linalg.norm(a.astype(np.float64))),
                nB2)

    check_blocks(Ct, rows, ref_atb, "A^T B")


def test_leading_dimension_beyond_2_23(la):
    # A 128 x (2^23 + 64), k-contiguous: its leading dimension is past 2^23,
    # beyond which the interior loader's 32-bit offsets are not used, so the
    # tile runs on the guarded loader (64-bit indexing) and must still agree
    # with the oracle
    k = (1 << 23) + 64
    A = la_inputs.gaussian((128, k), 225)
    B = la_inputs.gaussian((k, 128), 226)
    Ad = torch.from_numpy(A).to("cuda")
    Bd = torch.from_numpy(B).to("cuda")
    C = la.gemm(Ad, Bd, prec=la.Precision.BF16X3)
    torch.cuda.synchronize()
    C = C.cpu().numpy()
    assert np.isfinite(C).all()
    a = A[:16]
    bt = np.ascontiguousarray(B[:, 112:].T)
    ref = oracle.gemm(a, bt, trans_b=True)
    err = np.linalg.norm(C[:16, 112:].astype(np.float64) - ref) / (
        np.linalg.norm(a.astype(np.float64)) * np.linalg.norm(bt.astype(np.float64)))
    assert err <= TOL, f"normwise error {err:.3g}"
