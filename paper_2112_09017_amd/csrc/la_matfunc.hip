// Polynomial matrix functions (section III.D of arXiv 2112.09017).
//
// la_matfunc_odd: an odd polynomial acting on the singular values
// (eqs. MatFunc, odd_power, OddPoly):
//   F = sum_j c_j A (A^T A)^j = A p(G),  G = A^T A,  p(x) = sum_j c_j x^j,
// evaluated as one symmetric Gram launch, Horner's rule in G (one GEMM per
// coefficient beyond the second, c_j I added in the epilogue), and F = A P.
//
// la_matfunc_cheb: a Chebyshev series acting on the eigenvalues
// (eqs. MatFuncEig, any_power, EigenvaluePolynomial):
//   F = sum_k c_k T_k(B),  B = (2A - (lo + hi) I) / (hi - lo),
// evaluated by Clenshaw's recurrence b_k = 2 B b_{k+1} - b_{k+2} + c_k I,
// F = B b_1 - b_2 + c_0 I: d - 1 GEMM launches for degree d >= 2, each with
// the -b_{k+2} + c_k I update in its epilogue (written in place over b_{k+2}).
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include "la_internal.h"

namespace la {
namespace {

size_t matfunc_bytes(int64_t n) { return 3 * align_up256((size_t)n * n * sizeof(float)); }

la_status check_coef(const double *coef, int ncoef, const char *who)
{
    if (!coef || ncoef < 1) {
        set_error("%s: need at least one coefficient", who);
        return LA_ERR_INVALID_ARG;
    }
    for (int i = 0; i < ncoef; ++i)
        if (!isfinite(coef[i])) {
            set_error("%s: coefficient %d is not finite", who, i);
            return LA_ERR_INVALID_ARG;
        }
    return LA_OK;
}

// out = alpha X Y + beta E + gamma I, X (M x K) and Y (K x N) row-major.
hipError_t product(int prec, const float *X, int64_t ldx, const float *Y, int64_t ldy, float *out,
                   int64_t ldo, int64_t M, int64_t N, int64_t K, float alpha, float beta,
                   const float *E, int64_t lde, float gamma, hipStream_t s)
{
    GemmDesc d;
    memset(&d, 0, sizeof d);
    d.A = X;
    d.lda = ldx;
    d.a_kcontig = 1;
    d.B = Y;
    d.ldb = ldy;
    d.b_kcontig = 0;
    d.C = out;
    d.ldc = ldo;
    d.M = M;
    d.N = N;
    d.K = K;
    d.alpha = alpha;
    d.gamma = gamma;
    if (E) {
        d.E = E;
        d.lde = lde;
        d.beta = beta;
    }
    gemm_finalize(d, prec);
    return launch_gemm(prec, d, s);
}

}  // namespace
}  // namespace la

using namespace la;

extern "C" {

size_t la_matfunc_workspace_size(int64_t m, int64_t n)
{
    if (m < 1 || n < 1)
        return 0;
    return matfunc_bytes(n);
}

la_status la_matfunc_odd(la_context *ctx, int64_t m, int64_t n, const float *A, int64_t lda,
                         const double *coef, int ncoef, float *F, int64_t ldf, void *workspace,
                         size_t ws_bytes, la_precision prec, void *hip_stream)
{
    static const char *who = "la_matfunc_odd";
    set_error("%s", "");
    if (m < 1 || n < 1 || lda < n || ldf < n) {
        set_error("%s: bad shape (m %lld, n %lld, lda %lld, ldf %lld)", who, (long long)m,
                  (long long)n, (long long)lda, (long long)ldf);
        return LA_ERR_SHAPE;
    }
    la_status st = check_coef(coef, ncoef, who);
    if (st != LA_OK)
        return st;
    if (!valid_prec(prec)) {
        set_error("%s: unknown precision %d", who, (int)prec);
        return LA_ERR_INVALID_ARG;
    }
    if (!ctx || !A || !F || !workspace) {
        set_error("%s: NULL argument", who);
        return LA_ERR_INVALID_ARG;
    }
    if (((uintptr_t)workspace & 255u) != 0) {
        set_error("%s: workspace must be 256-byte aligned", who);
        return LA_ERR_INVALID_ARG;
    }
    const size_t need = matfunc_bytes(n);
    if (ws_bytes < need) {
        set_error("%s: workspace %zu bytes, need %zu", who, ws_bytes, need);
        return LA_ERR_OUT_OF_MEMORY;
    }
    const size_t fb = extent_bytes(m, n, ldf);
    if (overlaps(F, fb, A, extent_bytes(m, n, lda)) || overlaps(F, fb, workspace, need)) {
        set_error("%s: F overlaps A or the workspace", who);
        return LA_ERR_INVALID_ARG;
    }
    const int pr = resolve_prec(prec, PREC_BF16X6);
    LA_HIP(hipSetDevice(ctx->device), "la_matfunc_odd: hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    const int d = ncoef - 1;
    if (d == 0) {
        // F = c_0 A (FP64 per element: A / (1 / c_0), and 0 for c_0 = 0)
        LA_HIP(launch_scale(A, lda, F, ldf, m, n, 1.0 / coef[0], s), "la_matfunc_odd: scale");
        LA_HIP(hipStreamSynchronize(s), "la_matfunc_odd: sync");
        return LA_OK;
    }
    const size_t nb = align_up256((size_t)n * n * sizeof(float));
    float *G = (float *)workspace;
    float *P[2] = {(float *)((char *)workspace + nb), (float *)((char *)workspace + 2 * nb)};

    // G = A^T A (symmetric tiles only, mirror-written)
    {
        GemmDesc g;
        memset(&g, 0, sizeof g);
        g.A = A;
        g.B = A;
        g.lda = lda;
        g.ldb = lda;
        g.a_kcontig = 0;
        g.b_kcontig = 0;
        g.C = G;
        g.ldc = n;
        g.M = n;
        g.N = n;
        g.K = m;
        g.alpha = 1.0f;
        g.gram = 1;
        gemm_finalize(g, pr);
        LA_HIP(launch_gemm(pr, g, s), "la_matfunc_odd: gram");
    }
    // Horner in G: P = c_d G + c_{d-1} I, then P <- G P + c_j I for j = d-2 .. 0
    int cur = 0;
    LA_HIP(launch_affine(G, n, P[cur], n, n, coef[d], coef[d - 1], s), "la_matfunc_odd: affine");
    for (int j = d - 2; j >= 0; --j) {
        LA_HIP(product(pr, G, n, P[cur], n, P[cur ^ 1], n, n, n, n, 1.0f, 0.0f, nullptr, 0,
                       (float)coef[j], s),
               "la_matfunc_odd: horner");
        cur ^= 1;
    }
    // F = A P
    LA_HIP(product(pr, A, lda, P[cur], n, F, ldf, m, n, n, 1.0f, 0.0f, nullptr, 0, 0.0f, s),
           "la_matfunc_odd: final product");
    LA_HIP(hipStreamSynchronize(s), "la_matfunc_odd: sync");
    return LA_OK;
}

la_status la_matfunc_cheb(la_context *ctx, int64_t n, const float *A, int64_t lda, double lo,
                          double hi, const double *coef, int ncoef, float *F, int64_t ldf,
                          void *workspace, size_t ws_bytes, la_precision prec, void *hip_stream)
{
    static const char *who = "la_matfunc_cheb";
    set_error("%s", "");
    if (n < 1 || lda < n || ldf < n) {
        set_error("%s: bad shape (n %lld, lda %lld, ldf %lld)", who, (long long)n,
                  (long long)lda, (long long)ldf);
        return LA_ERR_SHAPE;
    }
    la_status st = check_coef(coef, ncoef, who);
    if (st != LA_OK)
        return st;
    if (!isfinite(lo) || !isfinite(hi) || !(hi > lo)) {
        set_error("%s: need finite lo < hi", who);
        return LA_ERR_INVALID_ARG;
    }
    if (!valid_prec(prec)) {
        set_error("%s: unknown precision %d", who, (int)prec);
        return LA_ERR_INVALID_ARG;
    }
    if (!ctx || !A || !F || !workspace) {
        set_error("%s: NULL argument", who);
        return LA_ERR_INVALID_ARG;
    }
    if (((uintptr_t)workspace & 255u) != 0) {
        set_error("%s: workspace must be 256-byte aligned", who);
        return LA_ERR_INVALID_ARG;
    }
    const size_t need = matfunc_bytes(n);
    if (ws_bytes < need) {
        set_error("%s: workspace %zu bytes, need %zu", who, ws_bytes, need);
        return LA_ERR_OUT_OF_MEMORY;
    }
    const size_t fb = extent_bytes(n, n, ldf);
    if (overlaps(F, fb, A, extent_bytes(n, n, lda)) || overlaps(F, fb, workspace, need)) {
        set_error("%s: F overlaps A or the workspace", who);
        return LA_ERR_INVALID_ARG;
    }
    const int pr = resolve_prec(prec, PREC_BF16X6);
    LA_HIP(hipSetDevice(ctx->device), "la_matfunc_cheb: hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    // B = sc A + t I maps [lo, hi] onto [-1, 1]
    const double sc = 2.0 / (hi - lo), t = -(hi + lo) / (hi - lo);
    const int d = ncoef - 1;
    const double *c = coef;
    if (d <= 1) {
        // c_0 I  or  c_0 I + c_1 B
        const double c1 = d == 1 ? c[1] : 0.0;
        LA_HIP(launch_affine(A, lda, F, ldf, n, c1 * sc, c1 * t + c[0], s),
               "la_matfunc_cheb: affine");
        LA_HIP(hipStreamSynchronize(s), "la_matfunc_cheb: sync");
        return LA_OK;
    }
    const size_t nb = align_up256((size_t)n * n * sizeof(float));
    float *B = (float *)workspace;
    float *P[2] = {(float *)((char *)workspace + nb), (float *)((char *)workspace + 2 * nb)};
    LA_HIP(launch_affine(A, lda, B, n, n, sc, t, s), "la_matfunc_cheb: B");
    // b_{d-1} = 2 c_d B + c_{d-1} I (b_d = c_d I, b_{d+1} = 0)
    LA_HIP(launch_affine(A, lda, P[0], n, n, 2.0 * c[d] * sc, 2.0 * c[d] * t + c[d - 1], s),
           "la_matfunc_cheb: b_{d-1}");
    if (d == 2) {
        // F = B b_1 - b_2 + c_0 I with b_2 = c_2 I
        LA_HIP(product(pr, B, n, P[0], n, F, ldf, n, n, n, 1.0f, 0.0f, nullptr, 0,
                       (float)(c[0] - c[2]), s),
               "la_matfunc_cheb: final product");
        LA_HIP(hipStreamSynchronize(s), "la_matfunc_cheb: sync");
        return LA_OK;
    }
    // b_{d-2} = 2 B b_{d-1} - c_d I + c_{d-2} I
    LA_HIP(product(pr, B, n, P[0], n, P[1], n, n, n, n, 2.0f, 0.0f, nullptr, 0,
                   (float)(c[d - 2] - c[d]), s),
           "la_matfunc_cheb: clenshaw");
    int cur = 1;   // P[cur] = b_{k+1}, P[cur ^ 1] = b_{k+2}
    for (int k = d - 3; k >= 1; --k) {
        // b_k = 2 B b_{k+1} - b_{k+2} + c_k I, written over b_{k+2}
        float *prev = P[cur ^ 1];
        LA_HIP(product(pr, B, n, P[cur], n, prev, n, n, n, n, 2.0f, -1.0f, prev, n, (float)c[k],
                       s),
               "la_matfunc_cheb: clenshaw");
        cur ^= 1;
    }
    // F = B b_1 - b_2 + c_0 I
    LA_HIP(product(pr, B, n, P[cur], n, F, ldf, n, n, n, 1.0f, -1.0f, P[cur ^ 1], n, (float)c[0],
                   s),
           "la_matfunc_cheb: final product");
    LA_HIP(hipStreamSynchronize(s), "la_matfunc_cheb: sync");
    return LA_OK;
}

}  // extern "C"
