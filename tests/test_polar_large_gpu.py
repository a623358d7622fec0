"""la_polar at the full benchmark sizes, checked by properties that hold at any
size (the N^3 FP64 oracle is out of reach on the host):

* ||U^T U - I||_F / sqrt(N) and ||A - U H||_F / ||A||_F computed exactly, by
  FP64 products on the GPU (torch, test tooling only: the product path never
  calls them);
* H against the exact V diag(s) V^T of the construction, also in FP64;
* H exactly symmetric;
* the preconditioning count equals the host recurrence, and the
  Newton-Schulz count matches the exact-arithmetic model run on the known
  spectrum (matrix steps act on the singular values) to within 2.
Sizes: polar of N = 16384 with cond 1e6, and a 131072 x 4096 tall matrix with
cond 1e4.  Both the split-BF16 default (AUTO) and plain FP32 MFMA must meet
the 1e-5 bounds.
"""
import math
import time

import numpy as np
import pytest
import torch

import la_inputs
import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

TOL = 1e-5


@pytest.fixture(scope="module")
def la():
    import paper_2112_09017_amd as la
    la.lib()
    return la


def exact_metrics(Ad, U, H, V, sd):
    """FP64 ||U^T U - I||_F / sqrt(n), ||A - U H||_F / ||A||_F and
    ||H - V diag(s) V^T||_F / ||A||_F on the GPU."""
    n = U.shape[1]
    U64 = U.double()
    G = U64.t().contiguous() @ U64
    G.diagonal().sub_(1.0)
    orth = torch.linalg.norm(G).item() / math.sqrt(n)
    del G
    A64 = Ad.double()
    nA = torch.linalg.norm(A64).item()
    R = A64 - U64 @ H.double()
    resid = torch.linalg.norm(R).item() / nA
    del R, A64, U64
    Hex = (V * sd[None, :]) @ V.t().contiguous()
    dh = torch.linalg.norm(H.double() - Hex).item() / nA
    del Hex
    torch.cuda.empty_cache()
    return orth, resid, dh


def model_steps(s_scaled, m, n, eps=2.0 ** -23):
    a = oracle.precond_a(0.1)
    k, _ = oracle.precond_steps(2.0 ** -23, 0.1)
    x = np.array(s_scaled, np.float64)
    c = (4.0 / 27.0) * a * a
    for _ in range(k):
        x = a * x * (1.0 - c * x * x)
    steps = 0
    while True:
        xn = 0.5 * x * (3.0 - x * x)
        d = math.sqrt(np.sum((xn - x) ** 2))
        x = xn
        steps += 1
        if d <= max(m, n) * eps or steps > 200:
            return k, steps


@pytest.mark.parametrize("shape", [(16384, 16384, 1e-6, (301, 302, 303)),
                                   (131072, 4096, 1e-4, (501, 502, 503))],
                         ids=["square16384_cond1e6", "tall131072x4096_cond1e4"])
def test_full_size_polar(la, shape):
    m, n, lo, seeds = shape
    t0 = time.time()
    A, Q, s, V = la_inputs.polar_case_torch(m, n, lo, seeds)
    del Q
    torch.cuda.empty_cache()
    sd = torch.from_numpy(s).to("cuda")
    print(f"inputs {m}x{n} in {time.time() - t0:.1f} s", flush=True)
    Ad = torch.from_numpy(A).to("cuda")
    nA = math.sqrt(float(np.sum(s * s)))
    kp, kn = model_steps(s / nA, m, n)
    for name, opts in (("auto", {}), ("fp32", dict(prec_precond=1, prec_ns=1, prec_h=1))):
        torch.cuda.synchronize()
        t1 = time.time()
        U, H, info = la.polar(Ad, **opts)
        torch.cuda.synchronize()
        dt = time.time() - t1
        orth, resid, dh = exact_metrics(Ad, U, H, V, sd)
        print(f"{name} {m}x{n}: {dt:.2f} s, info {info}; orth={orth:.3e} resid={resid:.3e} "
              f"dH={dh:.3e}; model k_pre={kp} k_ns={kn}", flush=True)
        assert torch.equal(H, H.t())
        assert orth <= TOL and resid <= TOL and dh <= TOL, (name, orth, resid, dh)
        assert info["iters_precond"] == kp
        assert abs(info["iters_ns"] - kn) <= 2
        del U, H
        torch.cuda.empty_cache()
