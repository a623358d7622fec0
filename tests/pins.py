"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each ``pin_*`` takes an ``oracle.Oracle`` instance and raises AssertionError
if the oracle disagrees with something established independently of it: a
number the paper states (``tests/golden/paper_claims.json``), a hand-derived
closed form (``tests/golden/polar_2x2.json``), a textbook routine (numpy's
SVD / float64 matmul / exact integer arithmetic), an exact construction
A = Q diag(s) V^T, or an invariant of the polar factorisation.  The same pins
run against builds of the oracle with planted mistakes
(``test_oracle_mutants.py``) to show that they would catch them.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

import la_inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _polar_svd(A):
    """Polar factors from numpy's SVD (eq. SVDdef): U = U_s V_s^T, H = V_s S V_s^T."""
    Us, S, Vt = np.linalg.svd(np.asarray(A, np.float64), full_matrices=False)
    return Us @ Vt, (Vt.T * S[None, :]) @ Vt


# --------------------------------------------------------------------------- scalar maps

def pin_paper_iteration_counts(orc):
    g = _golden("paper_claims.json")
    c = g["precond_steps_single"]
    k, s_end = orc.precond_steps(c["s0"], c["s_minus"])
    assert c["min"] <= k <= c["max"], f"k_pre={k} outside the paper's {c['min']}-{c['max']}"
    assert s_end >= c["s_minus"]

    def ns_count(x, tol, cap=1000):
        n = 0
        while abs(1.0 - x) > tol and n < cap:
            x = orc.ns_map(x)
            n += 1
        return n

    c2 = g["ns_steps_from_0p1"]
    k2 = ns_count(c2["x0"], c2["tol"])
    assert abs(k2 - c2["approx"]) <= c2["slack"], f"NS from 0.1 took {k2}"
    c3 = g["ns_steps_plain_small_s0"]
    k3 = ns_count(c3["x0"], c3["tol"])
    assert c3["min"] <= k3 <= c3["max"], f"plain NS from 1e-7 took {k3}"
    c4 = g["total_iterations"]
    total = k + ns_count(s_end, c2["tol"])
    assert abs(total - c4["approx"]) <= c4["slack"], f"total {total}"


def pin_scalar_map_properties(orc):
    g = _golden("paper_claims.json")
    # eq. (NS_scalar): 0 and 1 fixed, sqrt(3) -> 0, (0, sqrt 3) -> 1 under iteration
    r3 = g["ns_stability_bound"]["value"]
    assert orc.ns_map(0.0) == 0.0
    assert orc.ns_map(1.0) == 1.0
    assert abs(orc.ns_map(r3)) < 1e-15
    for x0 in (1e-3, 0.3, 1.0, 1.5, 1.7):
        x = x0
        for _ in range(200):
            x = orc.ns_map(x)
        assert abs(x - 1.0) < 1e-14, (x0, x)
    # eq. (RogueScalar): maximum over [0, 1] is exactly 1, at x = 3 / (2a)
    # (calculus: p'(x) = a - (4/9) a^3 x^2 = 0); [s-, 1] maps into [s-, 1];
    # values beneath s- are pushed up faster than by eq. (NS_scalar).
    for sm in g["precond_keeps_above_s_minus"]["s_minus_values"]:
        a = orc.precond_a(sm)
        assert abs(a - (1.5 * math.sqrt(3.0) - sm)) < 1e-15
        xs = 1.5 / a
        assert abs(orc.precond_map(a, xs) - 1.0) < 1e-14
        grid = np.linspace(sm, 1.0, 2001)
        vals = np.array([orc.precond_map(a, x) for x in grid])
        assert vals.min() >= sm - 1e-12, (sm, vals.min())
        assert vals.max() <= 1.0 + 1e-12
        for x in (1e-6, 1e-3, 0.5 * sm):
            assert orc.precond_map(a, x) > orc.ns_map(x) > x


# --------------------------------------------------------------------------- GEMM

def pin_gemm_exact_integers(orc):
    A = la_inputs.integer_matrix((37, 53), 11)
    B = la_inputs.integer_matrix((53, 29), 12)
    ref = A.astype(np.int64) @ B.astype(np.int64)
    assert np.array_equal(orc.gemm(A, B), ref.astype(np.float64))
    assert np.array_equal(orc.gemm(A.T.copy(), B, trans_a=True), ref)
    assert np.array_equal(orc.gemm(A, B.T.copy(), trans_b=True), ref)
    assert np.array_equal(orc.gemm(A.T.copy(), B.T.copy(), trans_a=True, trans_b=True), ref)
    C0 = la_inputs.integer_matrix((37, 29), 13)
    got = orc.gemm(A, B, alpha=2.0, beta=-3.0, C=C0)
    assert np.array_equal(got, 2 * ref - 3 * C0.astype(np.int64))


def pin_gemm_vs_numpy(orc):
    A = la_inputs.gaussian((64, 96), 21)
    B = la_inputs.gaussian((96, 80), 22)
    ref = A.astype(np.float64) @ B.astype(np.float64)
    got = orc.gemm(A, B)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    # identity and permutation
    eye = np.eye(96)
    assert np.array_equal(orc.gemm(A, eye), A.astype(np.float64))
    perm = np.random.default_rng(3).permutation(80)
    Pm = np.eye(80)[:, perm]
    assert np.array_equal(orc.gemm(B, Pm), B.astype(np.float64)[:, perm])


# --------------------------------------------------------------------------- polar

def pin_polar_2x2_golden(orc):
    for case in _golden("polar_2x2.json")["cases"]:
        A = np.array(case["A"], np.float64)
        if "U_times_sqrt5" in case:
            Ue = np.array(case["U_times_sqrt5"]) / math.sqrt(5.0)
            He = np.array(case["H_over_sqrt5"]) * math.sqrt(5.0)
        elif "U_times_sqrt34" in case:
            Ue = np.array(case["U_times_sqrt34"]) / math.sqrt(34.0)
            He = np.array(case["H_times_sqrt34"]) / math.sqrt(34.0)
        else:
            Ue = np.array(case["U"], np.float64)
            He = np.array(case["H"], np.float64)
        Uc, Hc = orc.polar_2x2(A)
        assert np.max(np.abs(Uc - Ue)) < 1e-14 and np.max(np.abs(Hc - He)) < 1e-13
        U, H, info = orc.polar(A)
        assert info.stop_reason == "tol", info
        assert np.max(np.abs(U - Ue)) < 1e-13, (A, U, Ue)
        assert np.max(np.abs(H - He)) < 1e-12, (A, H, He)


def pin_polar_2x2_random_vs_svd(orc):
    g = la_inputs.rng(31)
    for _ in range(50):
        A = g.standard_normal((2, 2))
        Us, Hs = _polar_svd(A)
        Uc, Hc = orc.polar_2x2(A)
        assert np.max(np.abs(Uc - Us)) < 1e-9, (A, Uc, Us)
        assert np.max(np.abs(Hc - Hs)) < 1e-9


def pin_polar_block_embedding(orc):
    """diag(B_1..B_k) conjugated by permutations has factors (P1 U P2, P2^T H P2)."""
    g = la_inputs.rng(41)
    k = 8
    n = 2 * k
    A = np.zeros((n, n))
    Ue = np.zeros((n, n))
    He = np.zeros((n, n))
    for b in range(k):
        blk = g.standard_normal((2, 2)) + (2.0 if b % 2 else -2.0) * np.eye(2)
        ub, hb = orc.polar_2x2(blk)
        sl = slice(2 * b, 2 * b + 2)
        A[sl, sl] = blk
        Ue[sl, sl] = ub
        He[sl, sl] = hb
    P1 = np.eye(n)[g.permutation(n)]
    P2 = np.eye(n)[g.permutation(n)]
    Ad = P1 @ A @ P2
    U, H, info = orc.polar(Ad)
    assert info.stop_reason in ("tol", "stagnation")
    assert np.max(np.abs(U - P1 @ Ue @ P2)) < 1e-11
    assert np.max(np.abs(H - P2.T @ He @ P2)) < 1e-11


def pin_polar_exact_construction(orc):
    """A = Q diag(s) V^T (float64) has U = Q V^T and H = V diag(s) V^T."""
    for (m, n, lo) in ((48, 48, 1e-3), (80, 32, 1e-2)):
        case = la_inputs.polar_case(m, n, lo, seeds=(51 + m, 52 + n, 53))
        A = case.A64
        U, H, info = orc.polar(A)
        assert info.stop_reason in ("tol", "stagnation")
        assert np.max(np.abs(U - case.U_exact)) < 1e-10
        assert np.max(np.abs(H - case.H_exact)) < 1e-12


def pin_polar_vs_numpy_svd(orc):
    for (m, n, lo) in ((64, 64, 1e-4), (96, 40, 1e-3)):
        case = la_inputs.polar_case(m, n, lo, seeds=(61 + m, 62, 63 + n))
        A = case.A32.astype(np.float64)
        Us, Hs = _polar_svd(A)
        U, H, info = orc.polar(A)
        assert np.linalg.norm(U - Us) < 1e-9
        assert np.linalg.norm(H - Hs) < 1e-12 * np.linalg.norm(A) * 10


def pin_polar_invariants(orc):
    case = la_inputs.polar_case(72, 56, 1e-5, seeds=(71, 72, 73))
    A = case.A32.astype(np.float64)
    U, H, info = orc.polar(A)
    n = A.shape[1]
    assert np.linalg.norm(U.T @ U - np.eye(n)) / math.sqrt(n) < 1e-13
    assert np.array_equal(H, H.T)
    assert np.linalg.eigvalsh(H).min() > -1e-12
    assert np.linalg.norm(A - U @ H) / np.linalg.norm(A) < 1e-13
    assert info.iters_precond == orc.precond_steps(2.0 ** -52, 0.1)[0]


def pin_polar_matrix_steps_act_on_singular_values(orc):
    """eqs. (odd_power), (RogueMatrix), (NewtonSchulz): each matrix step maps the
    singular values of the iterate by its scalar polynomial and keeps the
    singular vectors."""
    case = la_inputs.polar_case(40, 24, 1e-3, seeds=(81, 82, 83))
    A = case.A64
    sig = np.sort(case.s)[::-1] / np.linalg.norm(A)
    a = 1.5 * math.sqrt(3.0) - 0.1
    for kpre in (0, 1, 3, 6):
        X, _, info = orc.polar(A, max_precond=kpre, max_iter=0, want_h=False)
        assert info.iters_precond == kpre
        s_exp = sig.copy()
        for _ in range(kpre):
            s_exp = a * s_exp * (1.0 - (4.0 / 27.0) * a * a * s_exp ** 2)
        sv = np.linalg.svd(X, compute_uv=False)
        assert np.max(np.abs(np.sort(sv) - np.sort(s_exp))) < 1e-13, kpre
        # singular vectors unchanged: X V = Q diag(s_exp) up to sorting
        XV = X @ case.V
        col = np.linalg.norm(XV, axis=0)
        ratio = XV / col[None, :]
        assert np.max(np.abs(np.abs(np.sum(ratio * case.Q, axis=0)) - 1.0)) < 1e-10
    for kns in (1, 2, 4):
        kpre = 3
        X, _, info = orc.polar(A, max_precond=kpre, max_iter=kns, want_h=False,
                               stagnation=False)
        assert info.iters_ns == kns
        s_exp = sig.copy()
        for _ in range(kpre):
            s_exp = a * s_exp * (1.0 - (4.0 / 27.0) * a * a * s_exp ** 2)
        for _ in range(kns):
            s_exp = 0.5 * s_exp * (3.0 - s_exp ** 2)
        sv = np.linalg.svd(X, compute_uv=False)
        assert np.max(np.abs(np.sort(sv) - np.sort(s_exp))) < 1e-13, kns


def pin_polar_special_cases(orc):
    g = la_inputs.rng(91)
    Qh = la_inputs.haar(20, 92)
    U, H, _ = orc.polar(Qh)                      # orthogonal -> (A, I)
    assert np.max(np.abs(U - Qh)) < 1e-13 and np.max(np.abs(H - np.eye(20))) < 1e-13
    d = np.exp(g.uniform(-3, 0, size=20))
    U, H, _ = orc.polar(np.diag(d))              # positive diagonal -> (I, A)
    assert np.max(np.abs(U - np.eye(20))) < 1e-13 and np.max(np.abs(H - np.diag(d))) < 1e-13
    U, H, _ = orc.polar(3.5 * np.eye(7))         # c I -> (I, c I)
    assert np.max(np.abs(U - np.eye(7))) < 1e-14 and np.max(np.abs(H - 3.5 * np.eye(7))) < 1e-13
    U, H, _ = orc.polar(np.array([[-2.5]]))      # 1 x 1 -> (sign a, |a|)
    assert abs(U[0, 0] + 1.0) < 1e-15 and abs(H[0, 0] - 2.5) < 1e-14
    # transposition: polar(A^T) = (U^T, U H U^T) for square A
    A = la_inputs.polar_case(24, 24, 1e-2, seeds=(93, 94, 95)).A64
    U, H, _ = orc.polar(A)
    Ut, Ht, _ = orc.polar(A.T.copy())
    assert np.max(np.abs(Ut - U.T)) < 1e-12
    assert np.max(np.abs(Ht - U @ H @ U.T)) < 1e-12


def pin_polar_scale_invariance(orc):
    A = la_inputs.polar_case(32, 24, 1e-2, seeds=(96, 97, 98)).A32.astype(np.float64)
    U, H, _ = orc.polar(A)
    for k in (-7, 5):
        Uk, Hk, _ = orc.polar(A * 2.0 ** k)
        assert np.array_equal(Uk, U)
        assert np.array_equal(Hk, H * 2.0 ** k)


def pin_polar_rank_deficient(orc):
    """NS sends singular value 0 to 0 (eq. NS_scalar): U is a partial isometry.
    Run without preconditioning (s0 = s-), which would amplify rounding noise
    in the null space."""
    g = la_inputs.rng(99)
    n, r = 16, 11
    Q = la_inputs.haar(n, 100)
    V = la_inputs.haar(n, 101)
    s = np.zeros(n)
    s[:r] = g.uniform(0.5, 1.0, size=r)
    A = (Q * s[None, :]) @ V.T
    U, H, info = orc.polar(A, s0=0.1)
    assert info.iters_precond == 0
    assert np.max(np.abs(U @ U.T @ U - U)) < 1e-11
    assert np.max(np.abs(A - U @ H)) < 1e-12
    assert np.max(np.abs(U - Q[:, :r] @ V[:, :r].T)) < 1e-11


# --------------------------------------------------------------------------- inversion

def _inv_closed_form_iterate(d, a, k):
    """Algorithm NS_Inverse on a diagonal A = diag(d): with r = d x the residual
    e = 1 - r squares at every step (1 - r(2 - r) = (1 - r)^2), and X_0 = A^T / a
    gives e_0 = 1 - d^2 / a, so after k steps x = (1 - e_0^(2^k)) / d."""
    e0 = 1.0 - d * d / a
    return (1.0 - e0 ** (2 ** k)) / d


def pin_inverse_2x2_golden(orc):
    g = _golden("inverse_2x2.json")
    for case in g["cases"]:
        A = np.array(case["A"], np.float64)
        X, info = orc.inverse(A)
        want = np.array(case["inv_times_det"], np.float64) / case["det"]
        assert info.stop_reason == "tol"
        assert np.max(np.abs(X - want)) < 1e-13, (case, X)


def pin_inverse_vs_numpy(orc):
    """Square: numpy.linalg.inv; tall / wide: numpy.linalg.pinv, and the
    one-sided identity the algorithm promises (X A = I or A X = I)."""
    c = la_inputs.polar_case(48, 48, 1e-2, seeds=(120, 121, 122))
    A = c.A32.astype(np.float64)
    X, _ = orc.inverse(A)
    ref = np.linalg.inv(A)
    assert np.linalg.norm(X - ref) / np.linalg.norm(ref) < 1e-12
    T = la_inputs.gaussian((72, 40), 123).astype(np.float64)
    Xt, _ = orc.inverse(T)
    assert Xt.shape == (40, 72)
    assert np.max(np.abs(Xt @ T - np.eye(40))) < 1e-12
    assert np.linalg.norm(Xt - np.linalg.pinv(T)) / np.linalg.norm(Xt) < 1e-12
    W = la_inputs.gaussian((40, 72), 124).astype(np.float64)
    Xw, _ = orc.inverse(W)
    assert Xw.shape == (72, 40)
    assert np.max(np.abs(W @ Xw - np.eye(40))) < 1e-12
    assert np.linalg.norm(Xw - np.linalg.pinv(W)) / np.linalg.norm(Xw) < 1e-12


def pin_inverse_diagonal_closed_form(orc):
    """Every iterate of a diagonal input, from the closed form of the residual."""
    d = np.array([1.0, 0.5, 0.25, 3.0, 0.01, 1.5])
    A = np.diag(d)
    a = math.sqrt(float(np.sum(d ** 4)))          # ||A A^T||_F
    for k in range(0, 7):
        X, info = orc.inverse(A, max_iter=k)
        assert info.iters == k
        assert abs(info.gram_norm - a) <= 1e-15 * a
        want = np.diag(_inv_closed_form_iterate(d, a, k))
        assert np.max(np.abs(X - want) / np.abs(1.0 / d)[None, :].max()) < 1e-14, k
    X, info = orc.inverse(A)
    assert np.max(np.abs(X * d[:, None] - np.eye(len(d)))) < 1e-13
    # the scalar step squares the residual and has 1/d as its fixed point
    for dd, x in ((0.5, 0.3), (2.0, 0.1), (1e-3, 7.0), (3.0, 1.0 / 3.0)):
        y = orc.inv_map(dd, x)
        assert abs((1.0 - dd * y) - (1.0 - dd * x) ** 2) < 1e-15
    assert orc.inv_map(4.0, 0.25) == 0.25


def pin_inverse_orthogonal_stop_rule(orc):
    """A = Q orthogonal: A A^T = I, a = sqrt(n), X_k = Q^T (1 - e0^(2^k)) with
    e0 = 1 - 1/sqrt(n).  The step norm is then known in closed form, so the
    stopping step of the growing tolerance (eps_k = u 2^k, compared after the
    k-th step) is fixed; both readings of delta are checked."""
    n = 16
    Q = la_inputs.haar(n, 125)
    a = math.sqrt(n)
    e0 = 1.0 - 1.0 / a
    for u in (2.0 ** -24, 2.0 ** -40):
        for normalize in (True, False):
            scale = math.sqrt(a) if normalize else 1.0
            k, eps = 0, u
            while True:
                k += 1
                delta = scale * math.sqrt(n) * (e0 ** (2 ** (k - 1)) - e0 ** (2 ** k))
                eps *= 2.0
                if not delta > eps:
                    break
            X, info = orc.inverse(Q, u=u, normalize=normalize)
            assert info.iters == k, (u, normalize, info.iters, k)
            assert abs(info.last_tol - u * 2.0 ** k) == 0.0
            assert np.max(np.abs(X - Q.T * (1.0 - e0 ** (2 ** k)))) < 1e-14


def pin_inverse_scale_invariance(orc):
    """With the step measured on the normalised problem, A -> 2^k A gives
    X -> 2^-k X bitwise and the same step count; at ||A A^T||_F = 1 the two
    readings of the stop test coincide."""
    A = la_inputs.polar_case(24, 24, 1e-2, seeds=(126, 127, 128)).A32.astype(np.float64)
    X, info = orc.inverse(A, u=2.0 ** -24)
    for k in (-6, 4):
        Xk, ik = orc.inverse(A * 2.0 ** k, u=2.0 ** -24)
        assert ik.iters == info.iters
        assert np.array_equal(Xk, X * 2.0 ** -k)
    Q = la_inputs.haar(16, 129) * 0.5          # ||Q Q^T / 4||_F = 4 / 4 = 1 exactly
    X1, i1 = orc.inverse(Q, u=2.0 ** -24, normalize=True)
    X2, i2 = orc.inverse(Q, u=2.0 ** -24, normalize=False)
    assert i1.gram_norm == 1.0 or abs(i1.gram_norm - 1.0) < 1e-15
    assert i1.iters == i2.iters
    assert np.max(np.abs(X1 - X2)) < 1e-15


# --------------------------------------------------------------------------- matrix functions

def pin_matfunc_odd_exact_construction(orc):
    """eq. MatFunc: for A = Q diag(s) V^T the odd series acts on s alone."""
    c = la_inputs.polar_case(40, 24, 1e-2, seeds=(180, 181, 182))
    coef = np.array([1.25, -0.75, 0.5, -0.125])
    F = orc.matfunc_odd(c.A64, coef)
    f = sum(ck * c.s ** (2 * k + 1) for k, ck in enumerate(coef))
    want = (c.Q * f[None, :]) @ c.V.T
    assert np.max(np.abs(F - want)) < 1e-13


def pin_matfunc_odd_vs_numpy_svd(orc):
    A = la_inputs.gaussian((20, 20), 183).astype(np.float64)
    Us, S, Vt = np.linalg.svd(A)
    A = A / S[0]
    S = S / S[0]
    coef = np.array([0.3, 0.9, -0.4])
    F = orc.matfunc_odd(A, coef)
    f = coef[0] * S + coef[1] * S ** 3 + coef[2] * S ** 5
    assert np.max(np.abs(F - (Us * f[None, :]) @ Vt)) < 1e-13
    # one coefficient: c0 A exactly; [0, 1]: A (A^T A)
    assert np.array_equal(orc.matfunc_odd(A, [2.0]), 2.0 * A)
    assert np.max(np.abs(orc.matfunc_odd(A, [0.0, 1.0]) - A @ (A.T @ A))) < 1e-14


def _cheb_values(lam, lo, hi, coef):
    """sum_k c_k T_k(t) with T_k(cos th) = cos(k th), t = (2 lam - lo - hi) / (hi - lo)."""
    t = np.clip((2.0 * lam - (lo + hi)) / (hi - lo), -1.0, 1.0)
    th = np.arccos(t)
    return sum(ck * np.cos(k * th) for k, ck in enumerate(coef))


def pin_matfunc_cheb_symmetric_closed_form(orc):
    """eq. MatFuncEig for A = V diag(lam) V^T: the series acts on lam alone."""
    n = 30
    V = la_inputs.haar(n, 184)
    lam = np.linspace(-0.3, 2.0, n)
    A = (V * lam[None, :]) @ V.T
    lo, hi = -0.5, 2.5
    coef = la_inputs.rng(185).standard_normal(11)
    F = orc.matfunc_cheb(A, lo, hi, coef)
    want = (V * _cheb_values(lam, lo, hi, coef)[None, :]) @ V.T
    assert np.max(np.abs(F - want)) < 1e-12


def pin_matfunc_cheb_nonsymmetric(orc):
    """A = P diag(lam) P^-1 (diagonalisable, not symmetric): F = P g(lam) P^-1,
    g evaluated with numpy's Chebyshev series routine."""
    n = 16
    P = np.eye(n) + 0.1 * la_inputs.gaussian((n, n), 186).astype(np.float64)
    lam = np.linspace(0.1, 0.9, n)
    A = P @ np.diag(lam) @ np.linalg.inv(P)
    lo, hi = 0.0, 1.0
    coef = np.array([0.5, -0.25, 0.125, 0.3, -0.2, 0.05])
    g = np.polynomial.chebyshev.chebval((2 * lam - (lo + hi)) / (hi - lo), coef)
    want = P @ np.diag(g) @ np.linalg.inv(P)
    F = orc.matfunc_cheb(A, lo, hi, coef)
    assert np.max(np.abs(F - want)) < 1e-12


def pin_matfunc_cheb_low_degree(orc):
    A = la_inputs.gaussian((12, 12), 187).astype(np.float64) * 0.1
    lo, hi = -2.0, 3.0
    B = (2 * A - (lo + hi) * np.eye(12)) / (hi - lo)
    assert np.array_equal(orc.matfunc_cheb(A, lo, hi, [1.0]), np.eye(12))
    assert np.max(np.abs(orc.matfunc_cheb(A, lo, hi, [0.0, 1.0]) - B)) < 1e-15
    assert np.max(np.abs(orc.matfunc_cheb(A, lo, hi, [0.0, 0.0, 1.0]) -
                         (2 * B @ B - np.eye(12)))) < 1e-14
    assert np.max(np.abs(orc.matfunc_cheb(A, -1.0, 1.0, [0.0, 1.0]) - A)) < 1e-16


def pin_matfunc_cheb_exponential(orc):
    """A smooth function through its Chebyshev interpolant (numpy) against
    scipy's matrix exponential, for a symmetric A with spectrum in [lo, hi]."""
    import scipy.linalg
    n = 24
    V = la_inputs.haar(n, 188)
    lam = la_inputs.rng(189).uniform(-1.0, 1.5, size=n)
    A = (V * lam[None, :]) @ V.T
    lo, hi = -1.0, 1.5
    coef = np.polynomial.chebyshev.chebinterpolate(
        lambda t: np.exp(0.5 * (t * (hi - lo) + lo + hi)), 20)
    F = orc.matfunc_cheb(A, lo, hi, coef)
    assert np.max(np.abs(F - scipy.linalg.expm(A))) < 1e-12


# --------------------------------------------------------------------------- QR (section III.B)

def _pos_diag(Q, R):
    """Normalise a QR pair to a positive diagonal of R (QR is unique up to
    the signs of R's rows for a full-rank A)."""
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d[None, :], R * d[:, None]


def _check_qr(A, Q, R, tol=1e-12):
    m, n = A.shape
    assert Q.shape == (m, n) and R.shape == (n, n)
    assert np.max(np.abs(np.tril(R, -1))) == 0.0
    assert np.linalg.norm(Q @ R - A) <= tol * np.linalg.norm(A)
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= tol * math.sqrt(n)
    Qn, Rn = _pos_diag(*np.linalg.qr(A))     # LAPACK's Householder QR
    Qp, Rp = _pos_diag(Q, R)
    assert np.max(np.abs(Rp - Rn)) <= tol * 100 * np.max(np.abs(Rn))
    assert np.max(np.abs(Qp - Qn)) <= tol * 100


def pin_qr_2x2_golden(orc):
    g = _golden("qr_2x2.json")
    Q, R = orc.householder_qr(np.array(g["A"]))
    assert np.max(np.abs(Q - np.array(g["Q"]))) < 1e-15
    assert np.max(np.abs(R - np.array(g["R"]))) < 1e-14
    q, r = orc.householder_qr(np.array([[3.0], [4.0]]))
    assert abs(r[0, 0] + 5.0) < 1e-15 and np.max(np.abs(q[:, 0] + np.array([0.6, 0.8]))) < 1e-15


def pin_qr_householder_vs_numpy(orc):
    for shape, seed in (((60, 20), 700), ((33, 33), 701), ((257, 64), 702)):
        A = la_inputs.gaussian(shape, seed).astype(np.float64)
        _check_qr(A, *orc.householder_qr(A))
    # an upper-triangular input with a positive diagonal is its own R up to signs
    R0 = np.triu(la_inputs.gaussian((16, 16), 703).astype(np.float64)) + 4 * np.eye(16)
    Q, R = _pos_diag(*orc.householder_qr(R0))
    assert np.max(np.abs(R - R0)) < 1e-13 and np.max(np.abs(Q - np.eye(16))) < 1e-14


def pin_qr_tsqr(orc):
    """Algorithm tsqr gives the same factorisation as one Householder QR (up to
    the row signs of R) for every block height, including a ragged remainder
    and trees of 2, 3 and 5 levels; one block is the local QR itself."""
    A = la_inputs.gaussian((300, 24), 704).astype(np.float64)
    Q1, R1 = orc.householder_qr(A)
    for mr in (24, 37, 50, 64, 100, 150, 300):
        Q, R = orc.tsqr(A, mr)
        _check_qr(A, Q, R)
    Q, R = orc.tsqr(A, 300)
    assert np.array_equal(Q, Q1) and np.array_equal(R, R1)


def pin_qr_yamamoto(orc):
    """eq. (Yamamoto): I - W Y^T is orthogonal and its first n columns are Q;
    for one column it is the reflection taking e_1 to q."""
    A = la_inputs.gaussian((90, 12), 705).astype(np.float64)
    Q, _ = orc.tsqr(A, 30)
    W, Y = orc.yamamoto(Q)
    E = np.zeros_like(Q)
    E[:12, :12] = np.eye(12)
    assert np.array_equal(W, Q - E)
    F = np.eye(90) - W @ Y.T
    assert np.linalg.norm(F.T @ F - np.eye(90)) < 1e-13
    assert np.max(np.abs(F[:, :12] - Q)) < 1e-14
    q = la_inputs.gaussian((20, 1), 706).astype(np.float64)
    q /= np.linalg.norm(q)
    W, Y = orc.yamamoto(q)
    v = q[:, 0] - np.eye(20)[:, 0]
    assert np.max(np.abs(np.eye(20) - W @ Y.T - (np.eye(20) - 2 * np.outer(v, v) / (v @ v)))) < 1e-14


def pin_qr_caqr(orc):
    """Algorithm caqr: A = Q R with orthonormal Q and the same R (up to row
    signs) as LAPACK, for several panel widths (some not dividing n, so the
    last panel is narrower) and block heights; one panel gives exactly the R
    of tsqr."""
    A = la_inputs.gaussian((200, 48), 707).astype(np.float64)
    for b, mr in ((8, 64), (16, 50), (12, 48), (48, 100), (20, 64), (7, 30)):
        Q, R = orc.caqr(A, b, mr)
        _check_qr(A, Q, R)
        _, R2 = orc.caqr(A, b, mr, want_q=False)
        assert np.array_equal(R, R2)
    _, Rt = orc.tsqr(A, 64)
    _, Rc = orc.caqr(A, 48, 64)
    assert np.array_equal(Rt, Rc)
    S = la_inputs.gaussian((40, 40), 708).astype(np.float64)
    _check_qr(S, *orc.caqr(S, 8, 16))


ALL_PINS = [
    pin_paper_iteration_counts,
    pin_scalar_map_properties,
    pin_gemm_exact_integers,
    pin_gemm_vs_numpy,
    pin_polar_2x2_golden,
    pin_polar_2x2_random_vs_svd,
    pin_polar_block_embedding,
    pin_polar_exact_construction,
    pin_polar_vs_numpy_svd,
    pin_polar_invariants,
    pin_polar_matrix_steps_act_on_singular_values,
    pin_polar_special_cases,
    pin_polar_scale_invariance,
    pin_polar_rank_deficient,
    pin_inverse_2x2_golden,
    pin_inverse_vs_numpy,
    pin_inverse_diagonal_closed_form,
    pin_inverse_orthogonal_stop_rule,
    pin_inverse_scale_invariance,
    pin_matfunc_odd_exact_construction,
    pin_matfunc_odd_vs_numpy_svd,
    pin_matfunc_cheb_symmetric_closed_form,
    pin_matfunc_cheb_nonsymmetric,
    pin_matfunc_cheb_low_degree,
    pin_matfunc_cheb_exponential,
    pin_qr_2x2_golden,
    pin_qr_householder_vs_numpy,
    pin_qr_tsqr,
    pin_qr_yamamoto,
    pin_qr_caqr,
]
