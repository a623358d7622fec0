"""QR on the GPU (section III.B): la_tsqr, la_wy and la_caqr against the
FP64 oracle (Algorithm tsqr, eq. Yamamoto, Algorithm caqr).

Tolerances.  The factors are FP32-accurate in the sense used for the polar
factorisation: ||A - Q R||_F / ||A||_F <= 1e-5 and ||Q^T Q - I||_F / sqrt(n)
<= 1e-5.  A Householder reflection applied in FP32 commits a relative error
of a few u = 2^-24 per element; an element of the result passes through n
reflections per tree level plus, in CAQR, one GEMM update per panel (with
the GEMM target g <= 1e-6), and these errors add like a random walk:
sqrt(n (levels + 1)) u + sqrt(panels) g stays below 1e-5 for every shape
here (n <= 4096, at most 64 panels).  QR is unique up to the signs of R's
rows (the GPU's tree and the oracle's pairwise tree may choose them
differently), so R and Q are compared after scaling both to a positive
diagonal; by the perturbation theory of the QR factorisation a backward
error e changes R and Q by at most about cond(A) e, so those comparisons
use 4 cond(A) 1e-5.
"""
import math

import numpy as np
import pytest
import torch

import la_inputs
import oracle

pytestmark = pytest.mark.gpu

TOL = 1e-5


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


def pos(Q, R):
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d[None, :], R * d[:, None]


def cond2(A):
    s = np.linalg.svd(A, compute_uv=False)
    return float(s[0] / s[-1])


def check_factors(A, Q, R, Qo, Ro, label, tol=TOL):
    m, n = A.shape
    assert np.array_equal(np.tril(R, -1), np.zeros((n, n))), "R not upper triangular"
    back = np.linalg.norm(A - Q @ R) / np.linalg.norm(A)
    orth = np.linalg.norm(Q.T @ Q - np.eye(n)) / math.sqrt(n)
    kappa = cond2(A)
    Qp, Rp = pos(Q, R)
    Qop, Rop = pos(Qo, Ro)
    dR = np.linalg.norm(Rp - Rop) / np.linalg.norm(Rop)
    dQ = np.linalg.norm(Qp - Qop) / math.sqrt(n)
    print(f"\n{label}: backward {back:.3g} orth {orth:.3g} dR {dR:.3g} dQ {dQ:.3g} "
          f"cond {kappa:.3g}")
    assert back <= tol and orth <= tol
    assert dR <= 4 * kappa * tol and dQ <= 4 * kappa * tol
    return back, orth


TSQR_SHAPES = [(256, 64), (1000, 64), (300, 37), (600, 100), (131, 100), (64, 64), (1, 1),
               (5000, 128), (70000, 32), (257, 1), (45, 45), (520, 61)]


@pytest.mark.parametrize("shape", TSQR_SHAPES)
def test_tsqr_vs_oracle(la, shape):
    """Blocks of 256 rows, ragged remainders (600 x 100 splits its last 344
    rows in two), one-block panels and a four-level tree (70000 x 32)."""
    m, n = shape
    A32 = la_inputs.gaussian(shape, 800 + m + n)
    A = A32.astype(np.float64)
    Q, R = la.tsqr(dev(A32))
    Qo, Ro = oracle.tsqr(A, 256)
    check_factors(A, host(Q), host(R), Qo, Ro, f"tsqr {shape}")


def test_tsqr_conditioned_input(la):
    """A = Q0 diag(s) V^T with cond 1e4: backward error and orthogonality
    stay at the FP32 level regardless of the conditioning."""
    case = la_inputs.polar_case(2000, 96, 1e-4, seeds=(810, 811, 812))
    A = case.A32.astype(np.float64)
    Q, R = la.tsqr(dev(case.A32))
    Qo, Ro = oracle.tsqr(A, 256)
    check_factors(A, host(Q), host(R), Qo, Ro, "tsqr cond 1e4")


def test_tsqr_special_inputs(la):
    """An upper-triangular input is its own R up to signs (Q = diag(+-1)); a
    zero column of A is a zero column of R (no reflection is applied for it,
    and the earlier ones leave it zero)."""
    R0 = np.triu(la_inputs.gaussian((48, 48), 820).astype(np.float64)) + 3 * np.eye(48)
    Q, R = la.tsqr(dev(R0))
    Qp, Rp = pos(host(Q), host(R))
    assert np.max(np.abs(Rp - R0)) < 1e-5 * np.max(np.abs(R0))
    assert np.max(np.abs(Qp - np.eye(48))) < 1e-5
    A = la_inputs.gaussian((700, 16), 821)
    A[:, 5] = 0.0
    Q, R = la.tsqr(dev(A))
    Rh = host(R)
    assert np.all(Rh[:, 5] == 0.0)
    assert np.linalg.norm(A - host(Q) @ Rh) <= TOL * np.linalg.norm(A)


def test_tsqr_rank_deficient(la):
    """Repeated and scaled columns: their parts below the diagonal vanish (up
    to rounding) once the column they repeat is reflected, so the later
    reflections come from rounding-level vectors or none at all.  Q stays
    orthonormal and A = Q R holds to the tolerance; the diagonal of R is
    negligible in the dependent columns."""
    A = la_inputs.gaussian((700, 48), 823).astype(np.float64)
    A[:, 7] = A[:, 3]
    A[:, 20] = 2.0 * A[:, 5]
    A[:, 33] = 0.0
    A32 = A.astype(np.float32)
    Q, R = la.tsqr(dev(A32))
    Qh, Rh = host(Q), host(R)
    A = A32.astype(np.float64)
    assert np.linalg.norm(A - Qh @ Rh) <= TOL * np.linalg.norm(A)
    assert np.linalg.norm(Qh.T @ Qh - np.eye(48)) / math.sqrt(48) <= TOL
    scale = np.max(np.abs(np.diag(Rh)))
    for j in (7, 20, 33):
        assert abs(Rh[j, j]) <= 1e-5 * scale


@pytest.mark.parametrize("shape", [(300, 64), (5000, 128), (90, 12), (20, 1)])
def test_wy_vs_oracle(la, shape):
    """eq. (Yamamoto) on a reduced Q from the oracle: W and Y against the
    oracle's, and I - W Y^T orthogonal with first n columns Q."""
    m, n = shape
    A = la_inputs.gaussian(shape, 830 + m).astype(np.float64)
    Qo, _ = oracle.tsqr(A, 256)
    Q32 = Qo.astype(np.float32)
    W, Y = la.wy(dev(Q32))
    W, Y = host(W), host(Y)
    Wo, Yo = oracle.yamamoto(Q32.astype(np.float64))
    kM = cond2(np.eye(n) - Q32[:n].astype(np.float64))
    assert np.max(np.abs(W - Wo)) <= 2.0 ** -24
    dY = np.linalg.norm(Y - Yo) / np.linalg.norm(Yo)
    print(f"\nwy {shape}: dY {dY:.3g} cond(I - Q_1) {kM:.3g}")
    assert dY <= 4 * kM * TOL
    if m <= 5000:
        F = np.eye(m) - W @ Y.T
        assert np.linalg.norm(F[:, :n] - Q32) <= TOL * math.sqrt(n)
        assert np.linalg.norm(F.T @ F - np.eye(m)) / math.sqrt(m) <= 4 * kM * TOL


def test_wy_breakdown(la):
    """Q = [I; 0] makes I - Q_1 = 0: the WY form does not exist and the
    call says so."""
    from paper_2112_09017_amd import LAError, Status
    Q = np.zeros((100, 8), np.float32)
    Q[:8, :8] = np.eye(8)
    with pytest.raises(LAError) as e:
        la.wy(dev(Q))
    assert e.value.status == Status.BREAKDOWN


CAQR_CASES = [
    # (m, n, panel)
    (256, 256, 64),
    (300, 200, 64),     # ragged rows
    (520, 300, 64),     # ragged last panel (44 columns)
    (1024, 512, 128),
    (2000, 96, 32),
    (64, 64, 64),       # one panel
    (700, 130, 100),    # panel width not a power of two
    (1, 1, 1),
]


@pytest.mark.parametrize("case", CAQR_CASES, ids=lambda c: "x".join(map(str, c)))
def test_caqr_vs_oracle(la, case):
    m, n, b = case
    A32 = la_inputs.gaussian((m, n), 840 + m + n + b)
    A = A32.astype(np.float64)
    Q, R = la.caqr(dev(A32), panel=b)
    Qo, Ro = oracle.caqr(A, b, 256)
    check_factors(A, host(Q), host(R), Qo, Ro, f"caqr {case}")


# A 3xBF16 product drops the lo*lo term and the operands' residuals below
# 2^-16 of each term, about 2^-16 relative per term; in the update
# A_r - Y Z the sum runs over only the panel width, so the error is not
# averaged down to FP32 level: each panel adds about 2^-16 / sqrt(b) relative
# to ||Y|| ||Z||, and a factorisation of p panels about sqrt(p) times that
# (12 panels of 64 here: 3.4e-6), with Y up to cond(I - Q_1) times larger
# than W.  The bar for BF16X3 is therefore 4x the FP32 one.
X3_TOL = 4 * TOL


@pytest.mark.parametrize("prec", ["auto", "fp32", "x3", "x6"])
def test_caqr_precisions(la, prec):
    """Every product precision meets its bar on a cond-1e3 input, and AUTO
    (6xBF16 products) is no less accurate than plain FP32 MFMA beyond 1.5x."""
    P = {"auto": 0, "fp32": 1, "x3": 2, "x6": 3}
    case = la_inputs.polar_case(768, 768, 1e-3, seeds=(850, 851, 852))
    A = case.A32.astype(np.float64)
    Qo, Ro = oracle.caqr(A, 64, 256)
    res = {}
    for p in sorted({prec, "fp32"}):
        Q, R = la.caqr(dev(case.A32), panel=64, prec=P[p])
        res[p] = check_factors(A, host(Q), host(R), Qo, Ro, f"caqr 768 {p}",
                               tol=X3_TOL if p == "x3" else TOL)
    if prec in ("auto", "x6"):
        assert res[prec][0] <= 1.5 * res["fp32"][0] + 1e-7


def test_caqr_r_without_q_and_in_place(la):
    """R alone equals R from the run that also forms Q (the Q pass runs after
    the panels); inplace overwrites A with [R; 0]; two runs agree bitwise."""
    A32 = la_inputs.gaussian((900, 320), 860)
    Q1, R1 = la.caqr(dev(A32), panel=64)
    _, R2 = la.caqr(dev(A32), panel=64, want_q=False)
    assert torch.equal(R1, R2)
    Q3, R3 = la.caqr(dev(A32), panel=64)
    assert torch.equal(Q1, Q3) and torch.equal(R1, R3)
    X = dev(A32)
    la.caqr(X, panel=64, want_q=False, inplace=True)
    Xh = host(X)
    assert np.array_equal(Xh[:320], host(R1)) and np.all(Xh[320:] == 0.0)


def test_caqr_huge_leading_dimension(la):
    """A leading dimension above 2^21 floats takes the short-K update's
    pointer path (its buffer path keeps a 128-row tile's offsets below 2^31
    bytes); both paths compute every element identically, so the factors
    equal those of a contiguous A bit for bit."""
    m, n = 640, 320
    A32 = la_inputs.gaussian((m, n), 862)
    Q1, R1 = la.caqr(dev(A32), panel=64)
    base = torch.zeros((m, (1 << 21) + 64), dtype=torch.float32, device="cuda")
    X = base[:, :n]
    X.copy_(dev(A32))
    Q2, _ = la.caqr(X, panel=64, inplace=True)
    assert torch.equal(Q1, Q2)
    assert torch.equal(torch.triu(X[:n]), R1)
    assert torch.count_nonzero(base[:, n:]) == 0    # nothing written beyond A


def test_caqr_error_paths(la):
    from paper_2112_09017_amd import LAError, Status
    A = dev(la_inputs.gaussian((128, 64), 870))
    for panel in (0, 129):
        with pytest.raises(LAError) as e:
            la.caqr(A, panel=panel)
        assert e.value.status == Status.SHAPE
    with pytest.raises(LAError) as e:
        la.caqr(dev(la_inputs.gaussian((64, 128), 871)))
    assert e.value.status == Status.SHAPE
    with pytest.raises(LAError) as e:
        la.caqr(A, workspace=torch.empty(4096, dtype=torch.uint8, device="cuda"))
    assert e.value.status == Status.OUT_OF_MEMORY
    with pytest.raises(LAError) as e:
        la.tsqr(dev(la_inputs.gaussian((300, 129), 872)))
    assert e.value.status == Status.SHAPE


def _probe(A, Q, R, k=16, seed=880):
    """||A - Q R||_F / ||A||_F and ||Q^T Q - I||_F / sqrt(n) estimated in FP64
    on the host with k Gaussian probes."""
    n = A.shape[1]
    g = la_inputs.rng(seed).standard_normal(size=(n, k))
    r1 = A @ g - Q @ (R @ g)
    back = math.sqrt(float(np.sum(r1 * r1)) / k) / np.linalg.norm(A)
    q = Q @ g
    r2 = Q.T @ q - g
    orth = math.sqrt(float(np.sum(r2 * r2)) / k) / math.sqrt(n)
    return back, orth


def test_caqr_full_size_4096(la):
    """4096 x 4096, cond 1e3, panel 64: backward error and orthogonality by
    probes, no worse than the FP32-MFMA run beyond 1.5x."""
    n = 4096
    A32, _, _, _ = la_inputs.polar_case_torch(n, n, 1e-3, (890, 891, 892))
    A = A32.astype(np.float64)
    out = {}
    for name, p in (("auto", 0), ("fp32", 1)):
        Q, R = la.caqr(dev(A32), panel=64, prec=p)
        out[name] = _probe(A, host(Q), host(R))
        print(f"\n4096 {name}: backward ~{out[name][0]:.3g} orth ~{out[name][1]:.3g}")
        assert out[name][0] <= TOL and out[name][1] <= TOL
        del Q, R
    assert out["auto"][0] <= 1.5 * out["fp32"][0] + 1e-7


def test_caqr_bench_size_16384(la):
    """The bench configuration (16384², panel 64, AUTO, R and Q): backward
    error and orthogonality by 16 FP64 probes on the GPU (the factors stay
    on the device)."""
    n = 16384
    A = torch.randn((n, n), device="cuda", generator=torch.Generator(device="cuda").manual_seed(801))
    Q, R = la.caqr(A, panel=64)
    g = torch.randn((n, 16), dtype=torch.float64, device="cuda",
                    generator=torch.Generator(device="cuda").manual_seed(802))
    Qd = Q.double()
    r1 = A.double() @ g - Qd @ (R.double() @ g)
    back = float(torch.sqrt((r1 * r1).sum() / 16)) / float(torch.linalg.norm(A.double()))
    del r1
    r2 = Qd.T @ (Qd @ g) - g
    orth = float(torch.sqrt((r2 * r2).sum() / 16)) / math.sqrt(n)
    print(f"\n16384 caqr: backward ~{back:.3g} orth ~{orth:.3g}")
    assert back <= TOL and orth <= TOL
    assert torch.equal(torch.tril(R, -1), torch.zeros_like(R))
