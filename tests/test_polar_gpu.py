"""la_polar on the GPU against the FP64 oracle (Algorithm NS_Polar).

Tolerances of the polar factors: ||U^T U - I||_F / sqrt(N) <= 1e-5 and
||A - U H||_F / ||A||_F <= 1e-5.  Derived here:
  * H is well conditioned (perturbation of H is bounded by about sqrt(2)
    times that of A), so ||H - H_oracle||_F / ||A||_F <= 1e-5;
  * U is not: ||dU||_F <= 2 ||dA||_F / (s_n + s_{n-1}), so U is compared with
    the oracle's U at that bound with ||dA||_F = 1e-5 ||A||_F.
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


def run(la, A32, **opts):
    U, H, info = la.polar(torch.from_numpy(np.ascontiguousarray(A32)).to("cuda"), **opts)
    torch.cuda.synchronize()
    return U.cpu().numpy().astype(np.float64), H.cpu().numpy().astype(np.float64), info


def metrics(A32, U, H):
    A = A32.astype(np.float64)
    n = U.shape[1]
    orth = np.linalg.norm(U.T @ U - np.eye(n)) / math.sqrt(n)
    resid = np.linalg.norm(A - U @ H) / np.linalg.norm(A)
    return orth, resid


def predicted_ns_steps(s_scaled, m, n, eps=2.0 ** -23, s_minus=0.1, s0=2.0 ** -23):
    """Exact-arithmetic model: the matrix steps act on the singular values
    (eq. odd_power), so run the scalar maps on the spectrum of A / ||A||_F and
    stop as Algorithm NS_Polar does."""
    a = oracle.precond_a(s_minus)
    k, _ = oracle.precond_steps(s0, s_minus)
    x = np.array(s_scaled, dtype=np.float64)
    for _ in range(k):
        x = np.array([oracle.precond_map(a, v) for v in x])
    steps = 0
    while True:
        xn = np.array([oracle.ns_map(v) for v in x])
        d = np.sqrt(np.sum((xn - x) ** 2))
        x = xn
        steps += 1
        if d <= max(m, n) * eps or steps > 200:
            return k, steps


AUTO = {}
POLICIES = {
    "auto": {},
    "fp32": dict(prec_precond=1, prec_ns=1, prec_h=1),
    "x6": dict(prec_precond=3, prec_ns=3, prec_h=3),
    "auto_polish": dict(polish=True),
}


@pytest.mark.parametrize("policy", sorted(POLICIES))
def test_small_config_vs_oracle(la, policy):
    """256 x 256, Q diag(s) V^T with Haar Q, V and s log-uniform in [1e-3, 1]."""
    case = la_inputs.polar_case(256, 256, 1e-3, seeds=(103, 104, 105))
    U, H, info = run(la, case.A32, **POLICIES[policy])
    orth, resid = metrics(case.A32, U, H)
    Uo, Ho, _ = oracle.polar(case.A32.astype(np.float64))
    nA = np.linalg.norm(case.A32.astype(np.float64))
    s = np.sort(case.s)
    u_bound = 2 * TOL * nA / (s[0] + s[1])
    du = np.linalg.norm(U - Uo)
    dh = np.linalg.norm(H - Ho) / nA
    print(policy, info, f"orth={orth:.2e} resid={resid:.2e} dU={du:.2e} (bound {u_bound:.2e}) "
          f"dH={dh:.2e}")
    assert orth <= TOL and resid <= TOL
    assert dh <= TOL
    assert du <= u_bound
    assert info["iters_precond"] == oracle.precond_steps(2.0 ** -23, 0.1)[0] == 15
    assert info["stop_reason"] in (0, 1)


def test_iteration_count_matches_scalar_model(la):
    case = la_inputs.polar_case(256, 256, 1e-3, seeds=(103, 104, 105))
    U, H, info = run(la, case.A32)
    nA = np.linalg.norm(case.A64)
    k_pre, k_ns = predicted_ns_steps(case.s / nA, 256, 256)
    print(info, "predicted", k_pre, k_ns)
    assert info["iters_precond"] == k_pre
    assert abs(info["iters_ns"] - k_ns) <= 2


@pytest.mark.parametrize("shape", [(512, 128), (300, 200), (1000, 37), (129, 129)])
def test_tall_and_ragged(la, shape):
    m, n = shape
    case = la_inputs.polar_case(m, n, 1e-2, seeds=(110 + m, 111 + n, 112))
    U, H, info = run(la, case.A32)
    orth, resid = metrics(case.A32, U, H)
    Uo, Ho, _ = oracle.polar(case.A32.astype(np.float64))
    nA = np.linalg.norm(case.A32.astype(np.float64))
    print(shape, info, orth, resid)
    assert orth <= TOL and resid <= TOL
    assert np.linalg.norm(H - Ho) / nA <= TOL


@pytest.mark.parametrize("policy", ["auto", "fp32", "x6"])
@pytest.mark.parametrize("shape", [(300, 200), (1000, 37), (640, 256)])
def test_split_k_paths_vs_oracle(la, policy, shape):
    """A short FP32 accumulation depth (max_acc_k = 96) splits every Gram,
    update and H product along K into slices with a ragged last one, added in
    FP64: same tolerances against the oracle as the unsplit products."""
    m, n = shape
    case = la_inputs.polar_case(m, n, 1e-3, seeds=(130 + m, 131 + n, 132))
    U, H, info = run(la, case.A32, max_acc_k=96, **POLICIES[policy])
    orth, resid = metrics(case.A32, U, H)
    Uo, Ho, _ = oracle.polar(case.A32.astype(np.float64))
    nA = np.linalg.norm(case.A32.astype(np.float64))
    s = np.sort(case.s)
    u_bound = 2 * TOL * nA / (s[0] + s[1])
    print(shape, policy, info, f"orth={orth:.2e} resid={resid:.2e}")
    assert orth <= TOL and resid <= TOL
    assert np.linalg.norm(H - Ho) / nA <= TOL
    assert np.array_equal(H, H.T)
    assert np.linalg.norm(U - Uo) <= u_bound


def test_split_k_packed_update_by_fp64_properties(la):
    """4096 x 2048 takes the packed 3xBF16 update (128 tiles of 256 x 256);
    with max_acc_k = 512 its K = 2048 runs as four packed slices.  Checked by
    FP64 products on the GPU (test tooling): orthogonality, residual and H
    against V diag(s) V^T of the construction."""
    m, n = 4096, 2048
    A, Q, s, V = la_inputs.polar_case_torch(m, n, 1e-3, (141, 142, 143))
    del Q
    Ad = torch.from_numpy(A).to("cuda")
    U, H, info = la.polar(Ad, max_acc_k=512)
    torch.cuda.synchronize()
    A64, U64, H64 = Ad.double(), U.double(), H.double()
    orth = torch.linalg.norm(U64.t().contiguous() @ U64 - torch.eye(n, dtype=torch.float64,
                                                                     device="cuda")).item()
    orth /= math.sqrt(n)
    nA = torch.linalg.norm(A64).item()
    resid = torch.linalg.norm(A64 - U64 @ H64).item() / nA
    sd = torch.from_numpy(s).to("cuda")
    dh = torch.linalg.norm(H64 - (V * sd[None, :]) @ V.t().contiguous()).item() / nA
    print(info, f"orth={orth:.2e} resid={resid:.2e} dH={dh:.2e}")
    assert orth <= TOL and resid <= TOL and dh <= TOL
    assert torch.equal(H, H.t())


def test_h_against_exact_construction(la):
    """H = V diag(s) V^T is well conditioned even at cond 1e6."""
    case = la_inputs.polar_case(384, 384, 1e-6, seeds=(120, 121, 122))
    U, H, info = run(la, case.A32)
    orth, resid = metrics(case.A32, U, H)
    dh = np.linalg.norm(H - case.H_exact) / np.linalg.norm(case.A64)
    print(info, orth, resid, dh)
    assert orth <= TOL and resid <= TOL and dh <= TOL


def test_special_cases(la):
    Qh = la_inputs.haar(160, 130).astype(np.float32)
    U, H, _ = run(la, Qh)                         # orthogonal -> (A, I)
    assert np.abs(U - Qh).max() < 1e-5 and np.abs(H - np.eye(160)).max() < 1e-5
    d = np.exp(la_inputs.rng(131).uniform(-2, 0, size=96)).astype(np.float32)
    U, H, _ = run(la, np.diag(d))                 # positive diagonal -> (I, A)
    assert np.abs(U - np.eye(96)).max() < 1e-5 and np.abs(H - np.diag(d)).max() < 1e-5
    U, H, _ = run(la, np.array([[-2.5]], np.float32))   # 1 x 1 -> (sign a, |a|)
    assert abs(U[0, 0] + 1.0) < 1e-6 and abs(H[0, 0] - 2.5) < 1e-5


def test_two_by_two_closed_form(la):
    for A in ([[3.0, 0.0], [4.0, 5.0]], [[1.0, 2.0], [3.0, 4.0]], [[0.3, -1.2], [0.7, 0.9]]):
        A = np.array(A, np.float32)
        U, H, _ = run(la, A)
        Uc, Hc = oracle.polar_2x2(A.astype(np.float64))
        assert np.abs(U - Uc).max() < 1e-5 and np.abs(H - Hc).max() < 1e-5 * np.abs(A).max()


def test_scale_invariance_is_bitwise(la):
    case = la_inputs.polar_case(200, 160, 1e-3, seeds=(140, 141, 142))
    U, H, _ = run(la, case.A32)
    for k in (-6, 9):
        Uk, Hk, _ = run(la, case.A32 * np.float32(2.0 ** k))
        assert np.array_equal(Uk, U)
        assert np.array_equal(Hk, H * 2.0 ** k)


def test_deterministic(la):
    case = la_inputs.polar_case(300, 300, 1e-4, seeds=(150, 151, 152))
    U1, H1, i1 = run(la, case.A32)
    U2, H2, i2 = run(la, case.A32)
    assert np.array_equal(U1, U2) and np.array_equal(H1, H2) and i1 == i2


def test_error_paths(la):
    with pytest.raises(la.LAError) as e:
        run(la, np.full((8, 8), np.nan, np.float32))
    assert e.value.status == la.Status.NONFINITE
    with pytest.raises(la.LAError) as e:
        run(la, np.zeros((8, 8), np.float32))
    assert e.value.status == la.Status.NONFINITE
    with pytest.raises(la.LAError) as e:
        run(la, np.ones((3, 5), np.float32))
    assert e.value.status == la.Status.SHAPE
    case = la_inputs.polar_case(64, 64, 1e-3, seeds=(160, 161, 162))
    with pytest.raises(la.LAError) as e:
        run(la, case.A32, max_iter=1)
    assert e.value.status == la.Status.NOT_CONVERGED
    with pytest.raises(la.LAError) as e:
        Ad = torch.from_numpy(case.A32).to("cuda")
        la.polar(Ad, U=Ad)
    assert e.value.status == la.Status.INVALID_ARG
