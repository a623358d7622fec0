"""The block GEMM at its full size, A 16384 x 32768 times B 32768 x 16384
(FP32, N(0, 1), seeds 201/202: the per-core block of the paper's
distributed product, Section I), through the same calls the benchmark times.

* la_gemm_ws (pack both operands, then the packed-operand kernel),
  la_gemm_packed on operands packed once, and the unpacked la_gemm take every
  product in the same order, so the three results are compared bit for bit over
  all 16384 x 16384 outputs;
* sampled 64 x 64 output tiles (the four corners and random tiles, full K) are
  compared with the FP64 oracle (eq. Matmul): the normwise error over the
  sample, and over each tile against the norms of its own rows of A and
  columns of B, stays within the GEMM tolerance of 1e-6 (for K = 32768 the
  3xBF16 estimate 2^-16 / sqrt(K) is 8e-8).
"""
import numpy as np
import pytest
import torch

import la_inputs
import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

M, N, K = 16384, 16384, 32768
T = 64
TOL = 1e-6


@pytest.fixture(scope="module")
def la():
    import paper_2112_09017_amd as la
    la.lib()
    return la


def test_block_gemm_full_size(la):
    A = la_inputs.gaussian((M, K), 201)
    B = la_inputs.gaussian((K, N), 202)
    Ad = torch.from_numpy(A).to("cuda")
    Bd = torch.from_numpy(B).to("cuda")
    prec = la.Precision.BF16X3

    C_ws = la.gemm_ws(Ad, Bd, prec=prec)
    Ap = la.pack_bf16x3(Ad)
    Bp = la.pack_bf16x3(Bd.T)
    C_pk = la.gemm_packed(Ap, Bp, M, N, K)
    torch.cuda.synchronize()
    assert torch.equal(C_ws, C_pk), "la_gemm_ws and la_gemm_packed differ"
    del C_pk, Ap, Bp
    C_un = la.gemm(Ad, Bd, prec=prec)
    torch.cuda.synchronize()
    assert torch.equal(C_ws, C_un), "packed and unpacked 3xBF16 products differ"
    del C_un, Ad, Bd
    torch.cuda.empty_cache()
    C = C_ws.cpu().numpy()
    assert np.isfinite(C).all()

    g = np.random.default_rng(211)
    tiles = [(0, 0), (0, N - T), (M - T, 0), (M - T, N - T)]
    tiles += [(int(g.integers(0, M // T)) * T, int(g.integers(0, N // T)) * T) for _ in range(4)]
    err2 = ref2 = 0.0
    for r, c in tiles:
        a = A[r:r + T]
        bt = np.ascontiguousarray(B[:, c:c + T].T)
        ref = oracle.gemm(a, bt, trans_b=True)
        d2 = float(np.sum((C[r:r + T, c:c + T].astype(np.float64) - ref) ** 2))
        na = float(np.linalg.norm(a.astype(np.float64)))
        nb = float(np.linalg.norm(bt.astype(np.float64)))
        tile_err = np.sqrt(d2) / (na * nb)
        assert tile_err <= TOL, f"tile ({r}, {c}): normwise error {tile_err:.3g}"
        err2 += d2
        ref2 += (na * nb) ** 2
    est = np.sqrt(err2 / ref2)
    print(f"\nfull-size block GEMM: sampled normwise error {est:.3g} over {len(tiles)} tiles")
    assert est <= TOL
