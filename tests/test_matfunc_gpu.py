"""la_matfunc_odd / la_matfunc_cheb on the GPU against the FP64 oracle
(eqs. OddPoly and EigenvaluePolynomial).

Tolerances, from the GEMM target g = 1e-6 (normwise, relative to the
operands):
  * odd series: Horner's rule performs d + 1 products (Gram, d - 1 Horner
    steps, final), each adding at most about g times the magnitude of the
    terms it carries, so ||F - F64||_F <= 2 (d + 1) g sum_j |c_j| ||A||_F
    ||A||_2^(2j) (each term A (A^T A)^j has Frobenius norm at most
    ||A||_F ||A||_2^(2j));
  * Chebyshev series with the spectrum in [lo, hi]: ||T_k(B)||_2 <= 1, and
    Clenshaw's recurrence grows rounding errors by at most (d + 1)^2, so
    ||F - F64||_F <= 2 (d + 1)^2 g sum_k |c_k| sqrt(n).
"""
import math

import numpy as np
import pytest
import torch

import la_inputs
import oracle

pytestmark = pytest.mark.gpu

G = 1e-6


@pytest.fixture(scope="module")
def la():
    import paper_2112_09017_amd as la
    la.lib()
    return la


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


PRECS = {"auto": 0, "fp32": 1, "x3": 2, "x6": 3}
ODD_COEFS = {"ns_step": [1.5, -0.5], "one": [0.75], "random5": [0.9, -0.6, 0.35, -0.2, 0.05]}


@pytest.mark.parametrize("prec", sorted(PRECS))
@pytest.mark.parametrize("coefs", sorted(ODD_COEFS))
@pytest.mark.parametrize("shape", [(256, 256), (300, 200), (130, 64)])
def test_odd_vs_oracle(la, prec, coefs, shape):
    m, n = shape
    case = la_inputs.polar_case(m, n, 1e-2, seeds=(190 + m, 191 + n, 192))
    A = case.A32.astype(np.float64)
    c = np.array(ODD_COEFS[coefs])
    F = host(la.matfunc_odd(dev(case.A32), c, prec=PRECS[prec]))
    Fo = oracle.matfunc_odd(A, c)
    d = len(c) - 1
    s2 = float(np.linalg.norm(A, 2))
    bound = 2 * (d + 1) * G * sum(abs(cj) * np.linalg.norm(A) * s2 ** (2 * j)
                                  for j, cj in enumerate(c))
    err = float(np.linalg.norm(F - Fo))
    print(f"\nodd {prec} {coefs} {shape}: err {err:.3g} bound {bound:.3g} "
          f"rel {err / np.linalg.norm(Fo):.3g}")
    assert err <= bound
    # the exact construction: f acts on the singular values (eq. MatFunc)
    f = sum(cj * case.s ** (2 * j + 1) for j, cj in enumerate(c))
    exact = (case.Q * f[None, :]) @ case.V.T
    assert np.linalg.norm(F - exact) <= bound + 1e-6 * np.linalg.norm(exact)


def _symmetric_case(n, lo, hi, seed):
    V = la_inputs.haar(n, seed)
    lam = la_inputs.rng(seed + 1).uniform(lo, hi, size=n)
    lam[0], lam[-1] = lo, hi
    A32 = ((V * lam[None, :]) @ V.T).astype(np.float32)
    return A32, V, lam


@pytest.mark.parametrize("prec", sorted(PRECS))
@pytest.mark.parametrize("degree", [0, 1, 2, 3, 8, 16])
def test_cheb_vs_oracle(la, prec, degree):
    n, lo, hi = 256, -0.5, 2.0
    A32, V, lam = _symmetric_case(n, lo, hi, 200 + degree)
    A = A32.astype(np.float64)
    c = la_inputs.rng(210 + degree).standard_normal(degree + 1)
    F = host(la.matfunc_cheb(dev(A32), lo, hi, c, prec=PRECS[prec]))
    Fo = oracle.matfunc_cheb(A, lo, hi, c)
    bound = 2 * (degree + 1) ** 2 * G * float(np.sum(np.abs(c))) * math.sqrt(n)
    err = float(np.linalg.norm(F - Fo))
    print(f"\ncheb {prec} degree {degree}: err {err:.3g} bound {bound:.3g} "
          f"rel {err / max(np.linalg.norm(Fo), 1e-30):.3g}")
    assert err <= bound


def test_cheb_nonsymmetric_and_ragged(la):
    """A diagonalisable non-symmetric A (spectrum in [lo, hi]) at a ragged size."""
    n, lo, hi = 300, 0.0, 1.0
    P = np.eye(n) + 0.05 * la_inputs.gaussian((n, n), 220).astype(np.float64) / math.sqrt(n)
    lam = la_inputs.rng(221).uniform(0.05, 0.95, size=n)
    A32 = (P @ np.diag(lam) @ np.linalg.inv(P)).astype(np.float32)
    c = la_inputs.rng(222).standard_normal(10)
    F = host(la.matfunc_cheb(dev(A32), lo, hi, c))
    Fo = oracle.matfunc_cheb(A32.astype(np.float64), lo, hi, c)
    kP = float(np.linalg.cond(P))
    bound = 2 * 10 ** 2 * G * float(np.sum(np.abs(c))) * math.sqrt(n) * kP
    err = float(np.linalg.norm(F - Fo))
    print(f"\ncheb nonsymmetric: err {err:.3g} bound {bound:.3g}")
    assert err <= bound


def test_cheb_exponential(la):
    """exp(A) through a degree-16 Chebyshev interpolant (numpy) against the
    exact V diag(exp(lam)) V^T: FP32-level agreement."""
    n, lo, hi = 300, -1.0, 1.5
    A32, V, lam = _symmetric_case(n, lo, hi, 230)
    c = np.polynomial.chebyshev.chebinterpolate(
        lambda t: np.exp(0.5 * (t * (hi - lo) + lo + hi)), 16)
    F = host(la.matfunc_cheb(dev(A32), lo, hi, c))
    exact = (V * np.exp(lam)[None, :]) @ V.T
    rel = np.linalg.norm(F - exact) / np.linalg.norm(exact)
    print(f"\nexp(A) rel err {rel:.3g}")
    assert rel < 1e-5


def test_determinism_and_workspace_reuse(la):
    A32, _, _ = _symmetric_case(200, -1.0, 1.0, 240)
    c = la_inputs.rng(241).standard_normal(7)
    ws = torch.empty(la.lib().la_matfunc_workspace_size(200, 200) + 256, dtype=torch.uint8,
                     device="cuda")
    F1 = host(la.matfunc_cheb(dev(A32), -1.0, 1.0, c, workspace=ws))
    F2 = host(la.matfunc_cheb(dev(A32), -1.0, 1.0, c, workspace=ws))
    assert np.array_equal(F1, F2)
    G1 = host(la.matfunc_odd(dev(A32), c[:4], workspace=ws))
    G2 = host(la.matfunc_odd(dev(A32), c[:4], workspace=ws))
    assert np.array_equal(G1, G2)


def test_error_paths(la):
    from paper_2112_09017_amd import LAError, Status
    A = dev(la_inputs.gaussian((64, 64), 250))
    with pytest.raises(LAError) as e:
        la.matfunc_cheb(A, 1.0, -1.0, [1.0, 2.0])
    assert e.value.status == Status.INVALID_ARG
    with pytest.raises(LAError) as e:
        la.matfunc_odd(A, [])
    assert e.value.status == Status.INVALID_ARG
    with pytest.raises(LAError) as e:
        la.matfunc_odd(A, [1.0, 2.0], F=A)                 # F aliases A
    assert e.value.status == Status.INVALID_ARG
    with pytest.raises(LAError) as e:
        la.matfunc_cheb(A, -1.0, 1.0, [1.0, 2.0, 3.0],
                        workspace=torch.empty(4096, dtype=torch.uint8, device="cuda"))
    assert e.value.status == Status.OUT_OF_MEMORY


def test_auto_no_worse_than_fp32(la):
    """AUTO (6xBF16 products) is at least as accurate as plain FP32 MFMA
    (within 1.25x) on a degree-16 Chebyshev series and a 5-term odd series."""
    n, lo, hi = 384, -1.0, 1.0
    A32, _, _ = _symmetric_case(n, lo, hi, 260)
    A = A32.astype(np.float64)
    c = la_inputs.rng(261).standard_normal(17)
    Fo = oracle.matfunc_cheb(A, lo, hi, c)
    errs = {p: float(np.linalg.norm(host(la.matfunc_cheb(dev(A32), lo, hi, c, prec=PRECS[p])) - Fo))
            for p in ("auto", "fp32")}
    assert errs["auto"] <= 1.25 * errs["fp32"], errs
    c5 = np.array(ODD_COEFS["random5"])
    Go = oracle.matfunc_odd(A, c5)
    errs = {p: float(np.linalg.norm(host(la.matfunc_odd(dev(A32), c5, prec=PRECS[p])) - Go))
            for p in ("auto", "fp32")}
    assert errs["auto"] <= 1.25 * errs["fp32"], errs
