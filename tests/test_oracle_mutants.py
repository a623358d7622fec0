"""Planted mistakes in the oracle must each fail at least one pin (no GPU).

Each mutant is a copy of ``oracle/la_oracle.c`` with one plausible slip (a
dropped term, a wrong sign, constant or index, a transposed operand), built
with gcc into a temporary directory and run through every pin in ``pins``.
"""
import os
import subprocess

import pytest

import oracle
import pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "la_oracle.c")

MUTANTS = {
    "precond_constant": ("double c = (4.0 / 27.0) * a * a;", "double c = (4.0 / 9.0) * a * a;"),
    "precond_sign": ("(i == j ? 1.0 : 0.0) - c * G[i * n + j]", "(i == j ? 1.0 : 0.0) + c * G[i * n + j]"),
    "precond_drop_a": ("orc_gemm(0, 0, m, n, n, a, X, n, T, n, 0.0, Xn, n);",
                       "orc_gemm(0, 0, m, n, n, 1.0, X, n, T, n, 0.0, Xn, n);"),
    "a_def_sign": ("return 1.5 * sqrt(3.0) - s_minus;", "return 1.5 * sqrt(3.0) + s_minus;"),
    "ns_three": ("(i == j ? 3.0 : 0.0) - G[i * n + j]", "(i == j ? 2.0 : 0.0) - G[i * n + j]"),
    "ns_half": ("orc_gemm(0, 0, m, n, n, 0.5, X, n, T, n, 0.0, Xn, n);",
                "orc_gemm(0, 0, m, n, n, 1.0, X, n, T, n, 0.0, Xn, n);"),
    "gram_transposed": ("orc_gemm(1, 0, n, n, m, 1.0, X, n, X, n, 0.0, G, n);\n        /* T = I",
                        "orc_gemm(0, 1, n, n, n, 1.0, X, n, X, n, 0.0, G, n);\n        /* T = I"),
    "no_fro_scaling": ("X[i * n + j] = A[i * lda + j] / fro;", "X[i * n + j] = A[i * lda + j];"),
    "delta_sign": ("d2 += (Xn[i] - X[i]) * (Xn[i] - X[i]);", "d2 += (Xn[i] + X[i]) * (Xn[i] + X[i]);"),
    "h_not_symmetrised": ("0.5 * (G[i * n + j] + G[j * n + i])", "G[i * n + j]"),
    "gemm_trans_a_index": ("trans_a ? A[p * lda + i] : A[i * lda + p]", "trans_a ? A[i * lda + p] : A[i * lda + p]"),
    "gemm_drop_beta": ("c += beta * C[i * ldc + j];", "c += 0.0;"),
    "fro_missing_sqrt": ("    return sqrt(s);\n}", "    return s;\n}"),
    "closed_form_sign": ("u10 = (c - b) / r; u11 = (a + d) / r;", "u10 = (b - c) / r; u11 = (a + d) / r;"),
    "scalar_map_const": ("return 0.5 * x * (3.0 - x * x);", "return 0.5 * x * (3.0 - 0.9 * x * x);"),
    "precond_steps_off_by_one": ("    while (s < s_minus && count < 10000) {", "    while (s <= 2 * s_minus && count < 10000) {"),
    "inv_step_constant": ("T[i * n + j] = (i == j ? 2.0 : 0.0) - G[i * n + j];",
                          "T[i * n + j] = (i == j ? 1.9 : 0.0) - G[i * n + j];"),
    "inv_x0_scale": ("Xc[i * n + j] = A[j * lda + i] / a;", "Xc[i * n + j] = A[j * lda + i] / sqrt(a);"),
    "inv_fro_of_a": ("double a = orc_fro(n, n, G, n);", "double a = orc_fro(n, m, A, lda);"),
    "inv_eps_fixed": ("eps = 2.0 * eps;\n        double *t = Xc;", "eps = 1.0 * eps;\n        double *t = Xc;"),
    "inv_delta_literal": ("const double scale = normalize ? sqrt(a) : 1.0;", "const double scale = 1.0;"),
    "inv_delta_sign": ("d2 += (Xn[i] - Xc[i]) * (Xn[i] - Xc[i]);", "d2 += (Xn[i] + Xc[i]) * (Xn[i] + Xc[i]);"),
    "inv_map_sign": ("return x * (2.0 - d * x);", "return x * (2.0 + d * x);"),
    "odd_gram_transposed": ("orc_gemm(1, 0, n, n, m, 1.0, A, lda, A, lda, 0.0, G, n);",
                            "orc_gemm(0, 1, n, n, n, 1.0, A, lda, A, lda, 0.0, G, n);"),
    "odd_coef_index": ("F[i * ldf + j] += c[p] * T[i * n + j];",
                       "F[i * ldf + j] += c[p - 1] * T[i * n + j];"),
    "cheb_recurrence_sign": ("Tn[e] -= Tp[e];", "Tn[e] += Tp[e];"),
    "cheb_factor_two": ("orc_gemm(0, 0, n, n, n, 2.0, B, n, Tc, n, 0.0, Tn, n);",
                        "orc_gemm(0, 0, n, n, n, 1.0, B, n, Tc, n, 0.0, Tn, n);"),
    "cheb_affine_map": ("(2.0 * A[i * lda + j] - (i == j ? lo + hi : 0.0)) / w;",
                        "(A[i * lda + j] - (i == j ? lo : 0.0)) / w;"),
    "cheb_first_term": ("F[i * ldf + j] += c[1] * Tc[i * n + j];",
                        "F[i * ldf + j] += c[1] * Tp[i * n + j];"),
    "hh_beta_sign": ("const double beta = x0 >= 0.0 ? -nrm : nrm;",
                     "const double beta = x0 >= 0.0 ? nrm : -nrm;"),
    "hh_tau": ("tau[j] = (beta - x0) / beta;", "tau[j] = (x0 - beta) / beta;"),
    "hh_drop_unit_term": ("            double d = W[j * n + c];", "            double d = 0.0;"),
    "hh_q_forward_order": ("        for (int64_t j = n - 1; j >= 0; --j) {\n            if (tau[j] == 0.0)",
                           "        for (int64_t j = 0; j < n; ++j) {\n            if (tau[j] == 0.0)"),
    "tsqr_halves_swapped": ("const double *H = Qp + (half ? n * n : 0);",
                            "const double *H = Qp + (half ? 0 : n * n);"),
    "tsqr_stack_same_r": ("S[(n + i) * n + j] = Rs[b * n * n + i * n + j];",
                          "S[(n + i) * n + j] = Rs[a * n * n + i * n + j];"),
    "tsqr_group_end": ("const int64_t end = (b + g < p) ? b + g : p;",
                       "const int64_t end = (b + 1 < p) ? b + 1 : p;"),
    "yamamoto_printed_t": ("M[i * n + j] = ((i == j) ? 1.0 : 0.0) - Q[j * ldq + i];",
                           "M[i * n + j] = ((i == j) ? 1.0 : 0.0) - Q[i * ldq + j];"),
    "yamamoto_w_sign": ("W[i * ldw + j] = Q[i * ldq + j] - ((i == j) ? 1.0 : 0.0);",
                        "W[i * ldw + j] = Q[i * ldq + j] + ((i == j) ? 1.0 : 0.0);"),
    "caqr_update_sign": ("orc_gemm(0, 0, ml, nr, nc, -1.0, Y, n, Z, nr, 1.0, X + c * n + c + nc, n);",
                         "orc_gemm(0, 0, ml, nr, nc, 1.0, Y, n, Z, nr, 1.0, X + c * n + c + nc, n);"),
    "caqr_applies_q_not_qt": ("orc_gemm(1, 0, nc, nr, ml, 1.0, W, n, X + c * n + c + nc, n, 0.0, Z, nr);",
                              "orc_gemm(1, 0, nc, nr, ml, 1.0, Y, n, X + c * n + c + nc, n, 0.0, Z, nr);"),
    "caqr_drops_last_panel": ("const int64_t np = (n + b - 1) / b;\n    double *X",
                              "const int64_t np = n / b;\n    double *X"),
    "caqr_q_forward_order": ("for (int64_t jp = np - 1; jp >= 0; --jp) {",
                             "for (int64_t jp = 0; jp < np; ++jp) {"),
}


@pytest.fixture(scope="module")
def src_text():
    with open(SRC) as f:
        return f.read()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, src_text, tmp_path):
    old, new = MUTANTS[name]
    assert src_text.count(old) == 1, f"mutation anchor for {name} not unique/present"
    mutated = src_text.replace(old, new)
    c_path = tmp_path / "mut.c"
    c_path.write_text(mutated)
    so = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                    "-ffp-contract=off", str(c_path), "-o", str(so), "-lm"], check=True)
    orc = oracle.Oracle(str(so))
    failed = []
    for pin in pins.ALL_PINS:
        try:
            pin(orc)
        except Exception as e:  # noqa: BLE001 - any failure of a pin counts
            failed.append((pin.__name__, type(e).__name__))
    assert failed, f"mutant {name} passed every pin"
