// polar_host.h -- host-side plan and stop test of Algorithm NS_Polar
// (section III.D), shared by la_polar, the server and the server's CPU tests.
// Plain C++ (no HIP).
#pragma once

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>

#include "../../include/la.h"

namespace la {

// Resolved product arithmetic (la_precision without AUTO).
enum Prec : int { PREC_FP32 = 1, PREC_BF16X3 = 2, PREC_BF16X6 = 3 };

// Thread-local error text (defined by the library, or by a test harness).
void set_error(const char *fmt, ...);

// FP32 accumulation depth.  Every product accumulates in FP32 on the matrix
// cores, one rounding per MFMA, so the rounding error of an output grows with
// the number of accumulation steps along K; inside the preconditioning steps
// it is amplified (the polynomial's relative condition near sigma = 1 is about
// 23 at s_- = 0.1).  The iteration's products with K above kMaxAccK are
// therefore split along K into slices of at most kMaxAccK, each accumulated in
// FP32, and the slices are added in FP64 in slice order and rounded once.
// (la_polar_opts.max_acc_k overrides the depth.)
constexpr int64_t kMaxAccK = 4096;

// Smallest accepted s_- (see polar_plan).
constexpr double kMinSminus = 1e-3;

struct PolarPlan {
    int64_t m, n;
    double s_minus, s0, eps, a, c;
    int k_pre, max_iter, polish, stagnation;
    int prec_pre, prec_ns, prec_h;
    int64_t max_acc;   // FP32 accumulation depth of the split-K products
};

inline bool plan_valid_prec(int p)
{
    return p == LA_PREC_AUTO || p == LA_PREC_FP32 || p == LA_PREC_BF16X3 || p == LA_PREC_BF16X6;
}

// Validates the options and fixes everything the iteration needs before any
// matrix work: the coefficients of eq. (a_def), and the preconditioning count
// from the scalar recurrence of eq. (RogueScalar) run from s0 until s >= s_-.
inline la_status polar_plan(int64_t m, int64_t n, const la_polar_opts *opts, PolarPlan *out)
{
    la_polar_opts o;
    memset(&o, 0, sizeof o);
    if (opts)
        o = *opts;
    if (m < 1 || n < 1 || m < n) {
        set_error("polar needs m >= n >= 1 (got m=%lld n=%lld)", (long long)m, (long long)n);
        return LA_ERR_SHAPE;
    }
    if (!plan_valid_prec(o.prec_precond) || !plan_valid_prec(o.prec_ns) ||
        !plan_valid_prec(o.prec_h)) {
        set_error("invalid la_precision in la_polar_opts");
        return LA_ERR_INVALID_ARG;
    }
    PolarPlan p;
    p.m = m;
    p.n = n;
    p.s_minus = o.s_minus > 0 ? o.s_minus : 0.1;
    p.s0 = o.s0 > 0 ? o.s0 : ldexp(1.0, -23);
    p.eps = o.eps > 0 ? o.eps : ldexp(1.0, -23);
    p.max_iter = o.max_iter > 0 ? o.max_iter : 100;
    p.polish = o.polish != 0;
    p.stagnation = o.no_stagnation == 0;
    if (o.max_acc_k < 0) {
        set_error("la_polar_opts: max_acc_k must be >= 0");
        return LA_ERR_INVALID_ARG;
    }
    p.max_acc = o.max_acc_k > 0 ? ((int64_t)o.max_acc_k + 31) / 32 * 32 : kMaxAccK;
    // The preconditioning polynomial a x (1 - c x^2) is positive up to its root
    // 1/sqrt(c) = 1 + 0.385 s_- (to first order), and the iterate starts with
    // its largest singular value at or just below 1.  Rounding and product
    // errors of FP32 size must not push it past the root (the polynomial's sign
    // would flip and U^T A would lose definiteness), so s_- below
    // kMinSminus, whose margin 3.8e-4 is far above them, is rejected.
    if (!(p.s_minus < 1.0) || p.s_minus < kMinSminus || !isfinite(p.s0) || !isfinite(p.eps)) {
        set_error("la_polar_opts: need %g <= s_minus < 1 and finite s0, eps", kMinSminus);
        return LA_ERR_INVALID_ARG;
    }
    p.prec_pre = o.prec_precond == LA_PREC_AUTO ? (int)PREC_BF16X6 : o.prec_precond;
    p.prec_ns = o.prec_ns == LA_PREC_AUTO ? (int)PREC_BF16X3 : o.prec_ns;
    // H = sym(U^T A) is one product (about 2 of the ~85 N^3 of a polar) but its
    // error enters the residual directly: at 3xBF16 it alone is about
    // 2^-16 ||A||_F, so AUTO computes it at 6xBF16.
    p.prec_h = o.prec_h == LA_PREC_AUTO ? (int)PREC_BF16X6 : o.prec_h;
    p.a = 1.5 * sqrt(3.0) - p.s_minus;
    p.c = (4.0 / 27.0) * p.a * p.a;
    double s = p.s0;
    int k = 0;
    while (s < p.s_minus && k < 1000) {
        s = p.a * s * (1.0 - p.c * s * s);
        ++k;
    }
    p.k_pre = k;
    *out = p;
    return LA_OK;
}

// Stop test of the Newton-Schulz loop: the algorithm's ||U' - U||_F <=
// max(M, N) eps, a stagnation stop (the step norm no longer halves once it is
// below 1e-2 sqrt(N): rounding noise has been reached) and the step cap.  With
// polish, one more step (at 6xBF16) follows the stop.
struct StopState {
    double prev = INFINITY;
    bool stopped = false;   // tolerance or stagnation met; a polish step may follow
    int reason = 2;         // 0 tolerance, 1 stagnation, 2 cap
};

enum StopDecision { STOP_CONTINUE, STOP_DONE, STOP_CAP };

// After Newton-Schulz step number `steps` (1-based) with step norm delta.
inline StopDecision stop_test(const PolarPlan &p, int64_t m, int64_t n, double delta,
                              StopState &s, int steps)
{
    if (s.stopped)          // that was the polish step
        return STOP_DONE;
    const double tol = (double)std::max(m, n) * p.eps;
    if (delta <= tol) {
        s.reason = 0;
        s.stopped = true;
    } else if (p.stagnation && delta < 1e-2 * sqrt((double)n) && delta > 0.5 * s.prev) {
        s.reason = 1;
        s.stopped = true;
    }
    s.prev = delta;
    if (s.stopped)
        return p.polish ? STOP_CONTINUE : STOP_DONE;
    if (steps >= p.max_iter) {
        s.reason = 2;
        return STOP_CAP;
    }
    return STOP_CONTINUE;
}

}  // namespace la
