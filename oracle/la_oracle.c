/*
 * FP64 CPU oracle for the FP32-accurate GEMM and the preconditioned
 * Newton-Schulz polar factorisation of "Large Scale Distributed Linear
 * Algebra With Tensor Processing Units" (arXiv 2112.09017).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It is deliberately plain and slow: every routine is
 * the paper's definition or algorithm written out in double precision, with
 * no blocking, fusion or reordering of the arithmetic.  It shares no code,
 * header or constant with the GPU library.
 *
 * Conventions: real matrices, row-major with explicit leading dimension
 * (element (i, j) of an R x C matrix X is X[i * ldx + j]).  The paper writes
 * conjugate transposes; for real data they are plain transposes.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* GEMM: eq. (Matmul), section III.A: C_ij = sum_k A_ik B_kj.               */
/* ------------------------------------------------------------------------ */

/*
 * C <- alpha * op(A) op(B) + beta * C, op(X) = X or X^T.
 * op(A) is m x k, op(B) is k x n, C is m x n.  Each output element is the
 * dot product of row i of op(A) with column j of op(B), summed in k order.
 * The operands are first copied to contiguous row/column buffers (a layout
 * copy only; it changes no arithmetic) so that the dot products stream.
 * beta == 0 means C is not read.
 * Returns 0, or -1 if a buffer could not be allocated.
 */
int orc_gemm(int trans_a, int trans_b, int64_t m, int64_t n, int64_t k,
             double alpha, const double *A, int64_t lda, const double *B,
             int64_t ldb, double beta, double *C, int64_t ldc)
{
    double *ar = (double *)malloc(sizeof(double) * (size_t)(m * k + 1));
    double *bc = (double *)malloc(sizeof(double) * (size_t)(n * k + 1));
    if (!ar || !bc) {
        free(ar);
        free(bc);
        return -1;
    }
    /* ar[i*k + p] = op(A)(i, p);  bc[j*k + p] = op(B)(p, j) */
    for (int64_t i = 0; i < m; ++i)
        for (int64_t p = 0; p < k; ++p)
            ar[i * k + p] = trans_a ? A[p * lda + i] : A[i * lda + p];
    for (int64_t j = 0; j < n; ++j)
        for (int64_t p = 0; p < k; ++p)
            bc[j * k + p] = trans_b ? B[j * ldb + p] : B[p * ldb + j];

#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            double s = 0.0;
            const double *x = ar + i * k;
            const double *y = bc + j * k;
            for (int64_t p = 0; p < k; ++p)
                s += x[p] * y[p];
            double c = alpha * s;
            if (beta != 0.0)
                c += beta * C[i * ldc + j];
            C[i * ldc + j] = c;
        }
    }
    free(ar);
    free(bc);
    return 0;
}

/* Threads the OpenMP loops use (for reporting CPU-baseline core counts). */
int orc_num_threads(void) { return omp_get_max_threads(); }

/* Frobenius norm, ||A||_F = sqrt(tr(A A^T)) (section III.D). */
double orc_fro(int64_t m, int64_t n, const double *A, int64_t lda)
{
    double s = 0.0;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j)
            s += A[i * lda + j] * A[i * lda + j];
    return sqrt(s);
}

/* ------------------------------------------------------------------------ */
/* Scalar maps of section III.D.                                            */
/* ------------------------------------------------------------------------ */

/* eq. (a_def): a = (3/2) sqrt(3) - s_minus */
double orc_precond_a(double s_minus) { return 1.5 * sqrt(3.0) - s_minus; }

/* eq. (RogueScalar): x -> a x (1 - (4/27) (a x)^2) */
double orc_precond_map(double a, double x)
{
    return a * x * (1.0 - (4.0 / 27.0) * (a * x) * (a * x));
}

/* eq. (NS_scalar): x -> (1/2) x (3 - x^2) */
double orc_ns_map(double x) { return 0.5 * x * (3.0 - x * x); }

/*
 * Number of preconditioning steps of Algorithm NS_Polar: feed the estimate
 * s0 through eq. (RogueScalar) until it is no longer below s_minus.  The
 * final value of s is written to *s_end (nullable).  Capped at 10000.
 */
int orc_precond_steps(double s0, double s_minus, double *s_end)
{
    double a = orc_precond_a(s_minus);
    double s = s0;
    int count = 0;
    while (s < s_minus && count < 10000) {
        s = orc_precond_map(a, s);
        ++count;
    }
    if (s_end)
        *s_end = s;
    return count;
}

/* ------------------------------------------------------------------------ */
/* Polar factorisation: Algorithm NS_Polar with eqs. (a_def)-(RogueMatrix)  */
/* and (NewtonSchulz), section III.D.                                       */
/* ------------------------------------------------------------------------ */

typedef struct {
    int iters_precond;  /* preconditioning steps taken                     */
    int iters_ns;       /* Newton-Schulz steps taken                       */
    double fro_norm_a;  /* ||A||_F                                          */
    double last_delta;  /* ||U' - U||_F of the last Newton-Schulz step      */
    int stop_reason;    /* 0 tolerance, 1 stagnation, 2 iteration cap       */
} orc_polar_info;

/*
 * A is m x n (m >= n).  On return U (m x n, ldu) holds the polar factor and,
 * if H is not NULL, H (n x n, ldh) holds (U^T A + A^T U) / 2.
 *
 * Steps, in the algorithm's order:
 *   U <- A / ||A||_F
 *   s <- s0;  a <- (3/2) sqrt(3) - s_minus
 *   while s < s_minus:  s <- a s (1 - (4/27) a^2 s^2)
 *                       U <- a U (I - (4/27) a^2 U^T U)
 *   while delta > max(m, n) eps:  U' <- (1/2) U (3 I - U^T U)
 *                                 delta <- ||U' - U||_F;  U <- U'
 * Readings where the algorithm is silent: delta starts at +infinity (so at
 * least one Newton-Schulz step runs); the loop also stops after max_iter
 * steps, and, if stagnation != 0, when delta has fallen below 1e-2 sqrt(n)
 * and then fails to halve from one step to the next (rounding noise floor).
 * max_precond >= 0 caps the preconditioning loop (to inspect intermediate
 * iterates); a negative value leaves it to the s-recurrence alone.
 *
 * Returns 0 on success, -1 on bad arguments or allocation failure, -2 if
 * ||A||_F is zero or not finite.
 */
int orc_polar(int64_t m, int64_t n, const double *A, int64_t lda,
              double s_minus, double s0, double eps, int max_precond,
              int max_iter, int stagnation, double *U, int64_t ldu, double *H,
              int64_t ldh, orc_polar_info *info)
{
    if (m < n || n < 1 || lda < n || ldu < n || (H && ldh < n))
        return -1;
    orc_polar_info loc;
    memset(&loc, 0, sizeof loc);

    double *X = (double *)malloc(sizeof(double) * (size_t)(m * n));
    double *Xn = (double *)malloc(sizeof(double) * (size_t)(m * n));
    double *G = (double *)malloc(sizeof(double) * (size_t)(n * n));
    double *T = (double *)malloc(sizeof(double) * (size_t)(n * n));
    if (!X || !Xn || !G || !T) {
        free(X); free(Xn); free(G); free(T);
        return -1;
    }

    /* U <- A / ||A||_F */
    double fro = orc_fro(m, n, A, lda);
    loc.fro_norm_a = fro;
    if (!(fro > 0.0) || !isfinite(fro)) {
        free(X); free(Xn); free(G); free(T);
        if (info) *info = loc;
        return -2;
    }
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j)
            X[i * n + j] = A[i * lda + j] / fro;

    /* preconditioning loop */
    double a = orc_precond_a(s_minus);
    double c = (4.0 / 27.0) * a * a;
    double s = s0;
    int pre_cap = max_precond >= 0 ? max_precond : 10000;
    while (s < s_minus && loc.iters_precond < pre_cap) {
        s = a * s * (1.0 - c * s * s);
        /* G = U^T U */
        orc_gemm(1, 0, n, n, m, 1.0, X, n, X, n, 0.0, G, n);
        /* T = I - (4/27) a^2 G */
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j)
                T[i * n + j] = (i == j ? 1.0 : 0.0) - c * G[i * n + j];
        /* U <- a U T */
        orc_gemm(0, 0, m, n, n, a, X, n, T, n, 0.0, Xn, n);
        double *t = X; X = Xn; Xn = t;
        loc.iters_precond++;
    }

    /* Newton-Schulz loop */
    double tol = (double)(m > n ? m : n) * eps;
    double delta = INFINITY, prev = INFINITY;
    loc.stop_reason = 2;
    while (delta > tol) {
        if (loc.iters_ns >= max_iter) {
            loc.stop_reason = 2;
            break;
        }
        /* G = U^T U;  T = 3 I - G;  U' = (1/2) U T */
        orc_gemm(1, 0, n, n, m, 1.0, X, n, X, n, 0.0, G, n);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j)
                T[i * n + j] = (i == j ? 3.0 : 0.0) - G[i * n + j];
        orc_gemm(0, 0, m, n, n, 0.5, X, n, T, n, 0.0, Xn, n);
        /* delta = ||U' - U||_F */
        double d2 = 0.0;
        for (int64_t i = 0; i < m * n; ++i)
            d2 += (Xn[i] - X[i]) * (Xn[i] - X[i]);
        prev = delta;
        delta = sqrt(d2);
        double *t = X; X = Xn; Xn = t;
        loc.iters_ns++;
        if (delta <= tol) {
            loc.stop_reason = 0;
            break;
        }
        if (stagnation && delta < 1e-2 * sqrt((double)n) && delta > 0.5 * prev) {
            loc.stop_reason = 1;
            break;
        }
    }
    loc.last_delta = delta;

    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j)
            U[i * ldu + j] = X[i * n + j];

    if (H) {
        /* H = (U^T A + A^T U) / 2 */
        orc_gemm(1, 0, n, n, m, 1.0, X, n, A, lda, 0.0, G, n);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j)
                H[i * ldh + j] = 0.5 * (G[i * n + j] + G[j * n + i]);
    }
    free(X); free(Xn); free(G); free(T);
    if (info) *info = loc;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 2 x 2 closed form of the polar factor (eqs. PolarDecomp, SVDdef).        */
/* ------------------------------------------------------------------------ */

/*
 * For a real 2 x 2 A = [[a, b], [c, d]] of full rank, the orthogonal polar
 * factor is the rotation (det A > 0) or reflection (det A < 0) nearest to A:
 *   det > 0:  U = [[a + d, b - c], [c - b, a + d]] / sqrt((a + d)^2 + (b - c)^2)
 *   det < 0:  U = [[a - d, b + c], [b + c, d - a]] / sqrt((a - d)^2 + (b + c)^2)
 * (from Cayley-Hamilton: H^2 = A^T A and H = (A^T A + |det A| I) / tr H, so
 * U = A H^-1 is A + sign(det A) adj(A)^T up to a positive factor), and
 * H = U^T A.  Row-major in and out.  Returns -1 if det A == 0.
 */
int orc_polar_2x2(const double *A, double *U, double *H)
{
    double a = A[0], b = A[1], c = A[2], d = A[3];
    double det = a * d - b * c;
    double u00, u01, u10, u11, r;
    if (det > 0.0) {
        r = sqrt((a + d) * (a + d) + (b - c) * (b - c));
        u00 = (a + d) / r; u01 = (b - c) / r;
        u10 = (c - b) / r; u11 = (a + d) / r;
    } else if (det < 0.0) {
        r = sqrt((a - d) * (a - d) + (b + c) * (b + c));
        u00 = (a - d) / r; u01 = (b + c) / r;
        u10 = (b + c) / r; u11 = (d - a) / r;
    } else {
        return -1;
    }
    U[0] = u00; U[1] = u01; U[2] = u10; U[3] = u11;
    if (H) {
        H[0] = u00 * a + u10 * c;
        H[1] = u00 * b + u10 * d;
        H[2] = u01 * a + u11 * c;
        H[3] = u01 * b + u11 * d;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Newton-Schulz matrix inversion (Algorithm NS_Inverse, section III.D).    */
/* ------------------------------------------------------------------------ */

/* The scalar form of one step on a singular value d: x <- x (2 - d x).  For
 * a diagonal A every diagonal entry of X follows it independently. */
double orc_inv_map(double d, double x) { return x * (2.0 - d * x); }

typedef struct {
    int iters;
    int stop_reason;      /* 0 tolerance, 2 iteration cap */
    double gram_norm;     /* a = ||A A^T||_F */
    double last_delta;    /* delta of the last step (as compared) */
    double last_tol;      /* the tolerance it was compared with */
} orc_inverse_info;

/*
 * A is n x m (row-major, lda >= m) of full rank; X (m x n, ldx >= n)
 * receives X with X A = I (n >= m) or A X = I (n <= m):
 *   a <- ||A A^T||_F;  X <- A^T / a;  eps <- u;  delta <- 2 eps
 *   while delta > eps:  X' <- X (2 I - A X);  delta <- ||X' - X||_F
 *                       eps <- 2 eps;  X <- X'
 * X (2 I - A X) is the step for both shapes (it equals (2 I - X A) X); the
 * second form printed for A X = I only has matching dimensions when A is
 * square.
 * Reading where the algorithm is silent: the tolerance is absolute, so it
 * presumes X at unit scale.  With normalize != 0, delta is measured on the
 * normalised problem A / sqrt(a) (whose inverse is sqrt(a) X):
 * delta = sqrt(a) ||X' - X||_F, which makes the stop independent of the
 * scale of A and equal to the printed test whenever ||A A^T||_F = 1.
 * normalize == 0 compares ||X' - X||_F as printed.  The loop also stops
 * after max_iter steps.
 *
 * Returns 0, -1 on bad arguments or allocation failure, -2 if a is zero or
 * not finite.
 */
int orc_inverse(int64_t n, int64_t m, const double *A, int64_t lda, double u,
                int normalize, int max_iter, double *X, int64_t ldx,
                orc_inverse_info *info)
{
    if (n < 1 || m < 1 || lda < m || ldx < n || !(u > 0.0))
        return -1;
    orc_inverse_info loc;
    memset(&loc, 0, sizeof loc);

    double *G = (double *)malloc(sizeof(double) * (size_t)(n * n));
    double *T = (double *)malloc(sizeof(double) * (size_t)(n * n));
    double *Xc = (double *)malloc(sizeof(double) * (size_t)(m * n));
    double *Xn = (double *)malloc(sizeof(double) * (size_t)(m * n));
    if (!G || !T || !Xc || !Xn) {
        free(G); free(T); free(Xc); free(Xn);
        return -1;
    }

    /* a <- ||A A^T||_F */
    orc_gemm(0, 1, n, n, m, 1.0, A, lda, A, lda, 0.0, G, n);
    double a = orc_fro(n, n, G, n);
    loc.gram_norm = a;
    if (!(a > 0.0) || !isfinite(a)) {
        free(G); free(T); free(Xc); free(Xn);
        if (info) *info = loc;
        return -2;
    }
    /* X <- A^T / a */
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j)
            Xc[i * n + j] = A[j * lda + i] / a;

    const double scale = normalize ? sqrt(a) : 1.0;
    double eps = u;
    double delta = 2.0 * eps;
    loc.stop_reason = 0;
    while (delta > eps) {
        if (loc.iters >= max_iter) {
            loc.stop_reason = 2;
            break;
        }
        /* T = 2 I - A X  (n x n) */
        orc_gemm(0, 0, n, n, m, 1.0, A, lda, Xc, n, 0.0, G, n);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j)
                T[i * n + j] = (i == j ? 2.0 : 0.0) - G[i * n + j];
        /* X' = X T */
        orc_gemm(0, 0, m, n, n, 1.0, Xc, n, T, n, 0.0, Xn, n);
        double d2 = 0.0;
        for (int64_t i = 0; i < m * n; ++i)
            d2 += (Xn[i] - Xc[i]) * (Xn[i] - Xc[i]);
        delta = scale * sqrt(d2);
        eps = 2.0 * eps;
        double *t = Xc; Xc = Xn; Xn = t;
        loc.iters++;
    }
    loc.last_delta = delta;
    loc.last_tol = eps;

    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j)
            X[i * ldx + j] = Xc[i * n + j];
    free(G); free(T); free(Xc); free(Xn);
    if (info) *info = loc;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Polynomial matrix functions (section III.D, eqs. OddPoly and             */
/* EigenvaluePolynomial).                                                   */
/* ------------------------------------------------------------------------ */

/*
 * Odd polynomial acting on the singular values (eqs. MatFunc, odd_power,
 * OddPoly): for an m x n A,
 *   F = sum_{j=0}^{ncoef-1} c[j] A (A^T A)^j
 * i.e. f(x) = c[0] x + c[1] x^3 + c[2] x^5 + ...  Evaluated by its
 * definition: the terms A (A^T A)^j are formed one after another
 * (term <- term G, G = A^T A) and accumulated.  F is m x n (ldf >= n).
 * Returns 0 or -1.
 */
int orc_matfunc_odd(int64_t m, int64_t n, const double *A, int64_t lda,
                    const double *c, int ncoef, double *F, int64_t ldf)
{
    if (m < 1 || n < 1 || lda < n || ldf < n || ncoef < 1 || !c)
        return -1;
    double *G = (double *)malloc(sizeof(double) * (size_t)(n * n));
    double *T = (double *)malloc(sizeof(double) * (size_t)(m * n));
    double *Tn = (double *)malloc(sizeof(double) * (size_t)(m * n));
    if (!G || !T || !Tn) {
        free(G); free(T); free(Tn);
        return -1;
    }
    orc_gemm(1, 0, n, n, m, 1.0, A, lda, A, lda, 0.0, G, n);
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) {
            T[i * n + j] = A[i * lda + j];
            F[i * ldf + j] = c[0] * A[i * lda + j];
        }
    for (int p = 1; p < ncoef; ++p) {
        orc_gemm(0, 0, m, n, n, 1.0, T, n, G, n, 0.0, Tn, n);
        double *t = T; T = Tn; Tn = t;
        for (int64_t i = 0; i < m; ++i)
            for (int64_t j = 0; j < n; ++j)
                F[i * ldf + j] += c[p] * T[i * n + j];
    }
    free(G); free(T); free(Tn);
    return 0;
}

/*
 * Chebyshev polynomial acting on the eigenvalues (eqs. MatFuncEig,
 * any_power, EigenvaluePolynomial): for an n x n A whose eigenvalues lie in
 * [lo, hi],
 *   F = sum_{k=0}^{ncoef-1} c[k] T_k(B),  B = (2 A - (lo + hi) I) / (hi - lo)
 * (c[0] carries full weight).  Evaluated by its definition: T_0 = I,
 * T_1 = B, T_{k+1} = 2 B T_k - T_{k-1}, each T_k formed and accumulated.
 * Returns 0 or -1.
 */
int orc_matfunc_cheb(int64_t n, const double *A, int64_t lda, double lo,
                     double hi, const double *c, int ncoef, double *F,
                     int64_t ldf)
{
    if (n < 1 || lda < n || ldf < n || ncoef < 1 || !c || !(hi > lo))
        return -1;
    const size_t nn = (size_t)(n * n);
    double *B = (double *)malloc(sizeof(double) * nn);
    double *Tp = (double *)malloc(sizeof(double) * nn);   /* T_{k-1} */
    double *Tc = (double *)malloc(sizeof(double) * nn);   /* T_k */
    double *Tn = (double *)malloc(sizeof(double) * nn);   /* T_{k+1} */
    if (!B || !Tp || !Tc || !Tn) {
        free(B); free(Tp); free(Tc); free(Tn);
        return -1;
    }
    const double w = hi - lo;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            B[i * n + j] = (2.0 * A[i * lda + j] - (i == j ? lo + hi : 0.0)) / w;
            Tp[i * n + j] = (i == j ? 1.0 : 0.0);
            Tc[i * n + j] = B[i * n + j];
            F[i * ldf + j] = c[0] * Tp[i * n + j];
        }
    if (ncoef > 1)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j)
                F[i * ldf + j] += c[1] * Tc[i * n + j];
    for (int k = 2; k < ncoef; ++k) {
        orc_gemm(0, 0, n, n, n, 2.0, B, n, Tc, n, 0.0, Tn, n);
        for (size_t e = 0; e < nn; ++e)
            Tn[e] -= Tp[e];
        double *t = Tp; Tp = Tc; Tc = Tn; Tn = t;
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j)
                F[i * ldf + j] += c[k] * Tc[i * n + j];
    }
    free(B); free(Tp); free(Tc); free(Tn);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* QR factorisation (section III.B): Householder QR as the local step,      */
/* Algorithm tsqr, the Yamamoto WY form (eq. Yamamoto) and Algorithm caqr.  */
/* ------------------------------------------------------------------------ */

/*
 * Reduced QR of an m x n A (m >= n) by Householder reflections: for column
 * j, x = A[j:, j], beta = -sign(x_0) ||x||, v = x - beta e_1 scaled so that
 * v_0 = 1, tau = (beta - x_0) / beta, and A[j:, j:] <- (I - tau v v^T)
 * A[j:, j:].  R (n x n, ldr) = the upper triangle; Q (m x n, ldq) =
 * H_0 ... H_{n-1} [I_n; 0], formed by applying the reflections to [I; 0]
 * in reverse order.  Either output may be NULL.  Returns 0 or -1.
 */
int orc_householder_qr(int64_t m, int64_t n, const double *A, int64_t lda,
                       double *Q, int64_t ldq, double *R, int64_t ldr)
{
    if (m < n || n < 1 || lda < n)
        return -1;
    double *W = (double *)malloc(sizeof(double) * (size_t)(m * n));
    double *tau = (double *)malloc(sizeof(double) * (size_t)n);
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    if (!W || !tau || !w) {
        free(W); free(tau); free(w);
        return -1;
    }
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j)
            W[i * n + j] = A[i * lda + j];
    for (int64_t j = 0; j < n; ++j) {
        double s = 0.0;
        for (int64_t i = j; i < m; ++i)
            s += W[i * n + j] * W[i * n + j];
        const double nrm = sqrt(s);
        const double x0 = W[j * n + j];
        if (nrm == 0.0) {           /* zero column: no reflection */
            tau[j] = 0.0;
            continue;
        }
        const double beta = x0 >= 0.0 ? -nrm : nrm;
        tau[j] = (beta - x0) / beta;
        const double scale = 1.0 / (x0 - beta);
        for (int64_t i = j + 1; i < m; ++i)
            W[i * n + j] *= scale;          /* v below the diagonal, v_0 = 1 */
        W[j * n + j] = beta;
        /* A[j:, j+1:] <- (I - tau v v^T) A[j:, j+1:] */
        for (int64_t c = j + 1; c < n; ++c) {
            double d = W[j * n + c];
            for (int64_t i = j + 1; i < m; ++i)
                d += W[i * n + j] * W[i * n + c];
            w[c] = tau[j] * d;
        }
        for (int64_t c = j + 1; c < n; ++c) {
            W[j * n + c] -= w[c];
            for (int64_t i = j + 1; i < m; ++i)
                W[i * n + c] -= W[i * n + j] * w[c];
        }
    }
    if (R)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j)
                R[i * ldr + j] = j >= i ? W[i * n + j] : 0.0;
    if (Q) {
        for (int64_t i = 0; i < m; ++i)
            for (int64_t j = 0; j < n; ++j)
                Q[i * ldq + j] = (i == j) ? 1.0 : 0.0;
        for (int64_t j = n - 1; j >= 0; --j) {
            if (tau[j] == 0.0)
                continue;
            /* Q[j:, :] <- (I - tau v v^T) Q[j:, :] */
            for (int64_t c = 0; c < n; ++c) {
                double d = Q[j * ldq + c];
                for (int64_t i = j + 1; i < m; ++i)
                    d += W[i * n + j] * Q[i * ldq + c];
                w[c] = tau[j] * d;
            }
            for (int64_t c = 0; c < n; ++c) {
                Q[j * ldq + c] -= w[c];
                for (int64_t i = j + 1; i < m; ++i)
                    Q[i * ldq + c] -= W[i * n + j] * w[c];
            }
        }
    }
    free(W); free(tau); free(w);
    return 0;
}

/*
 * Algorithm tsqr: A (m x n) is split into row blocks of mr rows (mr >= n;
 * the last block takes the remainder and is merged into the one before it
 * if it has fewer than n rows).  Each block is factored (Householder QR);
 * then, while more than one R remains, neighbouring groups are paired, their
 * R factors stacked and factored again, and each group's Q rows are
 * multiplied by its half of the pair's Q factor (the optional step, here
 * always taken).  Q (m x n, ldq) and R (n x n, ldr).  Returns 0 or -1.
 */
int orc_tsqr(int64_t m, int64_t n, const double *A, int64_t lda, int64_t mr,
             double *Q, int64_t ldq, double *R, int64_t ldr)
{
    if (m < n || n < 1 || lda < n || mr < n || ldq < n || ldr < n)
        return -1;
    int64_t p = m / mr;   /* blocks of mr rows; the last one takes the remainder */
    if (p < 1)
        p = 1;
    int64_t *r0 = (int64_t *)malloc(sizeof(int64_t) * (size_t)(p + 1));
    double *Rs = (double *)malloc(sizeof(double) * (size_t)(p * n * n));
    double *S = (double *)malloc(sizeof(double) * (size_t)(2 * n * n));
    double *Qp = (double *)malloc(sizeof(double) * (size_t)(2 * n * n));
    double *T = (double *)malloc(sizeof(double) * (size_t)(m * n));
    if (!r0 || !Rs || !S || !Qp || !T) {
        free(r0); free(Rs); free(S); free(Qp); free(T);
        return -1;
    }
    for (int64_t i = 0; i < p; ++i)
        r0[i] = i * mr;
    r0[p] = m;
    /* local factorisations */
    for (int64_t i = 0; i < p; ++i) {
        const int64_t rows = r0[i + 1] - r0[i];
        if (orc_householder_qr(rows, n, A + r0[i] * lda, lda, Q + r0[i] * ldq, ldq,
                               Rs + i * n * n, n) != 0) {
            free(r0); free(Rs); free(S); free(Qp); free(T);
            return -1;
        }
    }
    /* binary reduction: groups of size g (in blocks), leader = first block */
    for (int64_t g = 1; g < p; g *= 2) {
        for (int64_t a = 0; a + g < p; a += 2 * g) {
            const int64_t b = a + g;             /* leader of the right group */
            const int64_t end = (b + g < p) ? b + g : p;
            /* stack R_a over R_b and factor */
            for (int64_t i = 0; i < n; ++i)
                for (int64_t j = 0; j < n; ++j) {
                    S[i * n + j] = Rs[a * n * n + i * n + j];
                    S[(n + i) * n + j] = Rs[b * n * n + i * n + j];
                }
            if (orc_householder_qr(2 * n, n, S, n, Qp, n, Rs + a * n * n, n) != 0) {
                free(r0); free(Rs); free(S); free(Qp); free(T);
                return -1;
            }
            /* Q rows of the left group times the top half, right group times the bottom */
            for (int half = 0; half < 2; ++half) {
                const int64_t lo = r0[half ? b : a], hi = r0[half ? end : b];
                const double *H = Qp + (half ? n * n : 0);
                orc_gemm(0, 0, hi - lo, n, n, 1.0, Q + lo * ldq, ldq, H, n, 0.0, T, n);
                for (int64_t i = lo; i < hi; ++i)
                    for (int64_t j = 0; j < n; ++j)
                        Q[i * ldq + j] = T[(i - lo) * n + j];
            }
        }
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            R[i * ldr + j] = Rs[i * n + j];
    free(r0); free(Rs); free(S); free(Qp); free(T);
    return 0;
}

/*
 * eq. (Yamamoto): from the reduced Q (m x n) of a panel, W = Q - [I_n; 0],
 * Q_1 = the first n rows of Q, and Y with Y^T = T W^T.  The full factor
 * Q_f = I - W Y^T must reproduce Q in its first n columns (A_l = Q_f R_f),
 * i.e. [I; 0] + W = [I; 0] - W T (Q_1 - I)^T, which fixes T^{-1} =
 * (I - Q_1)^T: the equation read with T^{-1} as the transpose of I - Q_1.
 * Then Y = W (I - Q_1)^{-1}: each row y of Y solves (I - Q_1)^T y^T = w^T,
 * by Gaussian elimination with partial pivoting.  W, Y: m x n (ldw, ldy).
 * Returns 0, -1 on bad arguments, -3 if I - Q_1 is singular.
 */
int orc_yamamoto(int64_t m, int64_t n, const double *Q, int64_t ldq, double *W,
                 int64_t ldw, double *Y, int64_t ldy)
{
    if (m < n || n < 1 || ldq < n || ldw < n || ldy < n)
        return -1;
    double *M = (double *)malloc(sizeof(double) * (size_t)(n * n));
    int64_t *piv = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    double *x = (double *)malloc(sizeof(double) * (size_t)n);
    if (!M || !piv || !x) {
        free(M); free(piv); free(x);
        return -1;
    }
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j)
            W[i * ldw + j] = Q[i * ldq + j] - ((i == j) ? 1.0 : 0.0);
    /* M = (I - Q_1)^T, LU with partial pivoting: P M = L U (in place) */
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            M[i * n + j] = ((i == j) ? 1.0 : 0.0) - Q[j * ldq + i];
    for (int64_t k = 0; k < n; ++k) {
        int64_t pr = k;
        for (int64_t i = k + 1; i < n; ++i)
            if (fabs(M[i * n + k]) > fabs(M[pr * n + k]))
                pr = i;
        piv[k] = pr;
        if (M[pr * n + k] == 0.0) {
            free(M); free(piv); free(x);
            return -3;
        }
        if (pr != k)
            for (int64_t j = 0; j < n; ++j) {
                double t = M[k * n + j]; M[k * n + j] = M[pr * n + j]; M[pr * n + j] = t;
            }
        for (int64_t i = k + 1; i < n; ++i) {
            M[i * n + k] /= M[k * n + k];
            for (int64_t j = k + 1; j < n; ++j)
                M[i * n + j] -= M[i * n + k] * M[k * n + j];
        }
    }
    /* each row: (I - Q_1)^T y^T = w^T */
    for (int64_t r = 0; r < m; ++r) {
        for (int64_t j = 0; j < n; ++j)
            x[j] = W[r * ldw + j];
        for (int64_t k = 0; k < n; ++k)
            if (piv[k] != k) {
                double t = x[k]; x[k] = x[piv[k]]; x[piv[k]] = t;
            }
        for (int64_t i = 1; i < n; ++i)
            for (int64_t j = 0; j < i; ++j)
                x[i] -= M[i * n + j] * x[j];
        for (int64_t i = n - 1; i >= 0; --i) {
            for (int64_t j = i + 1; j < n; ++j)
                x[i] -= M[i * n + j] * x[j];
            x[i] /= M[i * n + i];
        }
        for (int64_t j = 0; j < n; ++j)
            Y[r * ldy + j] = x[j];
    }
    free(M); free(piv); free(x);
    return 0;
}

/*
 * Algorithm caqr (right-looking): for each panel of b columns starting at
 * column c = j b, A_l = A[c:, c:c+b] is factored by tsqr (row blocks of mr),
 * A_l is replaced by [R_r; 0], W and Y are formed (eq. Yamamoto) and the
 * columns to the right are replaced by Q_f^T A_r = A_r - Y (W^T A_r).  R
 * (n x n, ldr) is the upper triangle of the result; Q (m x n, ldq, may be
 * NULL) is the reduced Q factor, Q_f(0) Q_f(1) ... [I_n; 0] with each Q_f
 * acting on rows c:.  When b does not divide n the last panel has the
 * remaining n mod b columns.  Returns 0, -1, or -3 (a singular I - Q_1).
 */
int orc_caqr(int64_t m, int64_t n, const double *A, int64_t lda, int64_t b, int64_t mr,
             double *Q, int64_t ldq, double *R, int64_t ldr)
{
    if (m < n || n < 1 || b < 1 || mr < b || lda < n || ldr < n || (Q && ldq < n))
        return -1;
    if (b > n)
        b = n;
    const int64_t np = (n + b - 1) / b;
    double *X = (double *)malloc(sizeof(double) * (size_t)(m * n));
    double *Qr = (double *)malloc(sizeof(double) * (size_t)(m * b));
    double *Rr = (double *)malloc(sizeof(double) * (size_t)(b * b));
    double *Ws = (double *)malloc(sizeof(double) * (size_t)(m * n));   /* W of every panel */
    double *Ys = (double *)malloc(sizeof(double) * (size_t)(m * n));
    double *Z = (double *)malloc(sizeof(double) * (size_t)(b * n));
    double *Ac = (double *)malloc(sizeof(double) * (size_t)(m * b));
    if (!X || !Qr || !Rr || !Ws || !Ys || !Z || !Ac) {
        free(X); free(Qr); free(Rr); free(Ws); free(Ys); free(Z); free(Ac);
        return -1;
    }
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j)
            X[i * n + j] = A[i * lda + j];
    int rc = 0;
    for (int64_t jp = 0; jp < np && rc == 0; ++jp) {
        const int64_t c = jp * b, ml = m - c;
        const int64_t nc = (n - c < b) ? n - c : b;   /* the last panel may be narrower */
        const int64_t nr = n - c - nc;
        double *W = Ws + c * n + c;   /* W of panel jp: rows c.., columns c..c+nc (ld n) */
        double *Y = Ys + c * n + c;
        for (int64_t i = 0; i < ml; ++i)
            for (int64_t j = 0; j < nc; ++j)
                Ac[i * nc + j] = X[(c + i) * n + c + j];
        rc = orc_tsqr(ml, nc, Ac, nc, mr < ml ? mr : ml, Qr, nc, Rr, nc);
        if (rc == 0)
            rc = orc_yamamoto(ml, nc, Qr, nc, W, n, Y, n);
        if (rc != 0)
            break;
        for (int64_t i = 0; i < ml; ++i)
            for (int64_t j = 0; j < nc; ++j)
                X[(c + i) * n + c + j] = i < nc ? Rr[i * nc + j] : 0.0;
        if (nr > 0) {
            /* Z = W^T A_r (nc x nr);  A_r <- A_r - Y Z */
            orc_gemm(1, 0, nc, nr, ml, 1.0, W, n, X + c * n + c + nc, n, 0.0, Z, nr);
            orc_gemm(0, 0, ml, nr, nc, -1.0, Y, n, Z, nr, 1.0, X + c * n + c + nc, n);
        }
    }
    if (rc == 0) {
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j)
                R[i * ldr + j] = j >= i ? X[i * n + j] : 0.0;
        if (Q) {
            /* Q = Q_f(0) ... Q_f(np-1) [I_n; 0], applied from the last panel back */
            for (int64_t i = 0; i < m; ++i)
                for (int64_t j = 0; j < n; ++j)
                    Q[i * ldq + j] = (i == j) ? 1.0 : 0.0;
            for (int64_t jp = np - 1; jp >= 0; --jp) {
                const int64_t c = jp * b, ml = m - c;
                const int64_t nc = (n - c < b) ? n - c : b;
                const double *W = Ws + c * n + c, *Y = Ys + c * n + c;
                /* Q[c:, :] <- Q[c:, :] - W (Y^T Q[c:, :]) */
                orc_gemm(1, 0, nc, n, ml, 1.0, Y, n, Q + c * ldq, ldq, 0.0, Z, n);
                orc_gemm(0, 0, ml, n, nc, -1.0, W, n, Z, n, 1.0, Q + c * ldq, ldq);
            }
        }
    }
    free(X); free(Qr); free(Rr); free(Ws); free(Ys); free(Z); free(Ac);
    return rc;
}
