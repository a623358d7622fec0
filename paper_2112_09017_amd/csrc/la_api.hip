// C ABI: context, error reporting, la_gemm, the la_polar driver and the
// la_inverse driver (Algorithm NS_Inverse, at the end of this file).
//
// la_polar follows Algorithm NS_Polar (section III.D of arXiv 2112.09017):
//   U <- A / ||A||_F                                   (FP64 norm on the GPU)
//   k_pre steps  U <- a U (I - (4/27) a^2 U^T U)       (eqs. a_def, RogueMatrix)
//     with k_pre from the scalar recurrence of eq. (RogueScalar) on the host
//   Newton-Schulz U' <- U (3I - U^T U) / 2 until ||U' - U||_F <= max(M,N) eps
//     (eq. NewtonSchulz), evaluated as U' = U + U (I - U^T U) / 2, which is the
//     same polynomial written so the small correction is formed separately
//   H <- (U^T A + A^T U) / 2
// Each step is two launches: the symmetric Gram (only upper tiles, the
// polynomial coefficients applied in its epilogue) and the product with the
// update applied in the epilogue.  The only host synchronisation per step is
// the 8-byte readback of ||U' - U||_F^2 for the data-dependent stop test.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "la_internal.h"

namespace la {

static thread_local char g_err[512];

// The one statically allocated device buffer of the library: the workspace of
// la_polar_noalloc, for callers that cannot allocate device memory.  Each GPU
// the library runs on holds its own copy until the process ends; its address
// on a device comes from hipGetSymbolAddress, taken once per device when the
// first context on that device is created.
constexpr size_t kScratchBytes = LA_POLAR_NOALLOC_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on `device` (the caller has made it current).
static hipError_t scratch_address(int device, void **out)
{
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

la_status dev_fail(hipError_t e, const char *where)
{
    set_error("%s: %s", where, hipGetErrorString(e));
    return LA_ERR_DEVICE;
}

bool overlaps(const void *a, size_t abytes, const void *b, size_t bbytes)
{
    if (!a || !b || abytes == 0 || bbytes == 0)
        return false;
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + bbytes && b0 < a0 + abytes;
}

size_t extent_bytes(int64_t rows, int64_t cols, int64_t ld)
{
    if (rows <= 0 || cols <= 0)
        return 0;
    return (size_t)((rows - 1) * ld + cols) * sizeof(float);
}

int resolve_prec(int p, int dflt)
{
    return p == LA_PREC_AUTO ? dflt : p;
}

bool valid_prec(int p)
{
    return p == LA_PREC_AUTO || p == LA_PREC_FP32 || p == LA_PREC_BF16X3 ||
           p == LA_PREC_BF16X6;
}

// ------------------------------------------------------------------ polar plan

// (polar_plan, the FP32 accumulation depth kMaxAccK and the stop test are in
// polar_host.h)

int acc_splits(int64_t K, int64_t max_acc)
{
    const int64_t a = max_acc > 0 ? max_acc : kMaxAccK;
    return K > a ? (int)std::min<int64_t>(65535, (K + a - 1) / a) : 1;
}

// Slices of K for a requested count: the slice length is a multiple of 32 (whole
// K stages of every kernel), so the count that results may be smaller.
static int slice_plan(int64_t K, int want, int64_t *slice_k)
{
    int64_t sk = (K + want - 1) / want;
    sk = (sk + 31) / 32 * 32;
    *slice_k = sk;
    return (int)((K + sk - 1) / sk);
}

// Split-K slices of a Gram: enough to keep each slice's FP32 accumulation
// within kMaxAccK, and, when the tiles cannot fill the 256 CUs, enough to
// fill them (the slices run in one launch; each keeps at least 2048 of the
// K = m rows).
int gram_splits(int64_t m, int64_t n, int prec, int64_t max_acc)
{
    const int64_t nb = (n + tile_n(prec) - 1) / tile_n(prec);
    const int64_t tiles = nb * (nb + 1) / 2;
    int fill = 1;
    const int64_t cap = std::max<int64_t>(1, std::min<int64_t>(16, m / 2048));
    if (tiles >= 256) {
        fill = 1;
    } else if (tiles >= 128) {
        // large tiles, one per CU: take the count whose rounds of 256 tiles
        // cost least per unit of K (N = 4096: 136 tiles x 15 slices = 2040,
        // 8 rounds of K / 15, against 3 rounds of K / 4 with 4 slices)
        int64_t best = 1, best_rounds = 1;
        for (int64_t sp = 2; sp <= cap; ++sp) {
            const int64_t rounds = (tiles * sp + 255) / 256;
            if (rounds * best < best_rounds * sp) {
                best = sp;
                best_rounds = rounds;
            }
        }
        fill = (int)best;
    } else {
        // small tiles: about two tiles per CU
        const int64_t sp = (512 + tiles - 1) / tiles;
        fill = (int)std::max<int64_t>(1, std::min<int64_t>(sp, cap));
    }
    int64_t sk = 0;
    return slice_plan(m, std::max(fill, acc_splits(m, max_acc)), &sk);
}

size_t align_up256(size_t x) { return (x + 255) & ~(size_t)255; }
static size_t align256(size_t x) { return align_up256(x); }

struct PolarWs {
    float *X;        // m x n, ld n: the iterate's second buffer
    float *P;        // n x n: I - c U^T U or I - U^T U
    float *parts;    // split-K slices of a Gram, an update or H (may be null)
    double *tiles;   // per-tile (or per-block) step-norm partials
    double *sumsq;   // norm partials
    double *scal;    // [0] ||A||_F^2, [1] ||U' - U||_F^2
    char *pk;        // packed 3xBF16 copies of U and P for the update (may be null)
    size_t parts_floats;
};

// Whether an M x N x K product takes the packed-operand kernel inside an
// iteration: 3xBF16 on 256 x 256 tiles (at least 128 of them) with K >= 256,
// as in la_gemm_ws.  The packed kernel computes every product exactly as the
// unpacked one, so the choice never changes a result.
static bool packs(int prec, int64_t M, int64_t N, int64_t K)
{
    return prec == PREC_BF16X3 && K >= 256 && ((M + 255) / 256) * ((N + 255) / 256) >= 128;
}

// Bytes of the packed op(A) and op(B)^T of such a product (0 if it does not pack).
static size_t pack_bytes(int prec, int64_t M, int64_t N, int64_t K)
{
    if (!packs(prec, M, N, K))
        return 0;
    return align_up256(packed_x3_bytes(M, K)) + align_up256(packed_x3_bytes(N, K));
}

// Launch d, through the packed-operand kernel when it qualifies and pk (of at
// least pack_bytes) is given: op(A) and op(B)^T are packed into pk first,
// unless an operand packed earlier is passed (pre_a / pre_b).  K-slices of d
// (d.slices > 1) run on whichever kernel is chosen.
static hipError_t gemm_packed_or_plain(int prec, GemmDesc d, char *pk, hipStream_t s,
                                       const char *pre_a = nullptr, const char *pre_b = nullptr)
{
    if (pk && !d.gram && !d.small && packs(prec, d.M, d.N, d.K)) {
        char *pa = pk, *pb = pk + align_up256(packed_x3_bytes(d.M, d.K));
        hipError_t e = hipSuccess;
        if (!pre_a)
            e = launch_pack_x3(d.A, d.lda, d.a_kcontig, d.M, d.K, pa, s);
        if (e == hipSuccess && !pre_b)
            e = launch_pack_x3(d.B, d.ldb, d.b_kcontig, d.N, d.K, pb, s);
        if (e != hipSuccess)
            return e;
        d.A = (const float *)(pre_a ? pre_a : pa);
        d.B = (const float *)(pre_b ? pre_b : pb);
        return launch_gemm_packed_x3(d, s);
    }
    return launch_gemm(prec, d, s);
}

// Whether a Gram X^T X (n x n, K = m) at prec runs on the packed-operand
// kernel: 3xBF16 with at least 128 upper 256 x 256 tiles and K >= 256.  X^T is
// packed once and serves as both operands.
static bool gram_packs(int prec, int64_t m, int64_t n)
{
    const int64_t nb = (n + 255) / 256;
    return prec == PREC_BF16X3 && m >= 256 && nb * (nb + 1) / 2 >= 128;
}

// Packed copies the iteration keeps: X and P for a packed update, or X^T for
// a packed Gram (the Gram's pack is consumed before the update packs).
static size_t packed_update_bytes(const PolarPlan &p)
{
    size_t b = std::max(pack_bytes(p.prec_pre, p.m, p.n, p.n), pack_bytes(p.prec_ns, p.m, p.n, p.n));
    for (int pr : {p.prec_pre, p.prec_ns})
        if (gram_packs(pr, p.m, p.n))
            b = std::max(b, align_up256(packed_x3_bytes(p.n, p.m)));
    return b;
}

// Slices of the update X P (K = n) and of each half of H (K = m).
static int update_splits(const PolarPlan &p)
{
    int64_t sk = 0;
    return slice_plan(p.n, acc_splits(p.n, p.max_acc), &sk);
}

static int h_splits(const PolarPlan &p)
{
    int64_t sk = 0;
    return slice_plan(p.m, acc_splits(p.m, p.max_acc), &sk);
}

// Floats of split-K slices the iteration and H need at most: a Gram's
// slices (n x n each), an update's (m x n each, when its K = n is split),
// and H's two sets of n x n slices (U^T A and A^T U).
static size_t parts_floats(const PolarPlan &p)
{
    size_t f = 0;
    for (int pr : {p.prec_pre, p.prec_ns, (int)PREC_BF16X6}) {
        const int g = gram_splits(p.m, p.n, pr, p.max_acc);
        if (g > 1)
            f = std::max(f, (size_t)g * p.n * p.n);
    }
    const int u = update_splits(p);
    if (u > 1)
        f = std::max(f, (size_t)u * p.m * p.n);
    f = std::max(f, (size_t)2 * h_splits(p) * p.n * p.n);
    return f;
}

static size_t max_update_tiles(const PolarPlan &p)
{
    size_t t = (size_t)splitk_update_num_partials();
    for (int pr : {PREC_FP32, PREC_BF16X3, PREC_BF16X6}) {
        const size_t tm = (size_t)((p.m + tile_m(pr, 1) - 1) / tile_m(pr, 1));
        const size_t tn = (size_t)((p.n + tile_n(pr, 1) - 1) / tile_n(pr, 1));
        t = std::max(t, tm * tn);
    }
    return t;
}

size_t polar_workspace_bytes(const PolarPlan &p)
{
    size_t b = 0;
    b += align256((size_t)p.m * p.n * sizeof(float));
    b += align256((size_t)p.n * p.n * sizeof(float));
    b += align256(parts_floats(p) * sizeof(float));
    b += align256(max_update_tiles(p) * sizeof(double));
    b += align256((size_t)sumsq_num_partials() * sizeof(double));
    b += align256(8 * sizeof(double));
    b += packed_update_bytes(p);
    return b;
}

static PolarWs carve(const PolarPlan &p, void *ws)
{
    PolarWs w;
    char *b = (char *)ws;
    w.X = (float *)b;
    b += align256((size_t)p.m * p.n * sizeof(float));
    w.P = (float *)b;
    b += align256((size_t)p.n * p.n * sizeof(float));
    w.parts_floats = parts_floats(p);
    w.parts = (float *)b;
    b += align256(w.parts_floats * sizeof(float));
    w.tiles = (double *)b;
    b += align256(max_update_tiles(p) * sizeof(double));
    w.sumsq = (double *)b;
    b += align256((size_t)sumsq_num_partials() * sizeof(double));
    w.scal = (double *)b;
    b += align256(8 * sizeof(double));
    w.pk = packed_update_bytes(p) ? b : nullptr;
    return w;
}

// X1^T X2 for K x n operands X1, X2 (row-major, leading dimensions ld1, ld2)
// as about `want` K-slices in one Gram-mode launch: slice y writes the upper
// triangle (i <= j) of its n x n part, the sum over its k range, at
// parts + y n^2.  *count receives the number of slices.
static hipError_t gram_slices(int prec, const float *X1, int64_t ld1, const float *X2,
                              int64_t ld2, int64_t K, int64_t n, int want, float *parts,
                              int *count, hipStream_t s, char *pk = nullptr)
{
    GemmDesc d;
    memset(&d, 0, sizeof d);
    d.A = X1;
    d.B = X2;
    d.a_kcontig = 0;
    d.b_kcontig = 0;
    d.lda = ld1;
    d.ldb = ld2;
    d.M = n;
    d.N = n;
    d.K = K;
    d.gram = 1;
    d.gram_upper = 1;
    d.C = parts;
    d.ldc = n;
    d.alpha = 1.0f;
    gemm_finalize(d, prec);
    d.slices = slice_plan(K, want, &d.slice_k);
    d.slice_stride = n * n;
    *count = d.slices;
    if (pk && X1 == X2 && ld1 == ld2 && gram_packs(prec, K, n) && !d.small) {
        // X^T (n rows, K) packed once and read as both operands; the packed
        // kernel computes every product exactly as the unpacked one
        hipError_t e = launch_pack_x3(X1, ld1, 0, n, K, pk, s);
        if (e != hipSuccess)
            return e;
        d.A = (const float *)pk;
        d.B = (const float *)pk;
        return launch_gemm_packed_x3(d, s);
    }
    return launch_gemm(prec, d, s);
}

// P <- alpha X^T X + gamma I (exactly symmetric), X m x n with leading dim ldx.
static hipError_t gram_step(const PolarPlan &p, int prec, const float *X, int64_t ldx,
                            double alpha, double gamma, float *P, const PolarWs &w,
                            hipStream_t s)
{
    const int64_t m = p.m, n = p.n;
    const int splits = gram_splits(m, n, prec, p.max_acc);
    if (splits <= 1 || (size_t)splits * n * n > w.parts_floats) {
        GemmDesc d;
        memset(&d, 0, sizeof d);
        d.a_kcontig = 0;
        d.b_kcontig = 0;
        d.lda = ldx;
        d.ldb = ldx;
        d.M = n;
        d.N = n;
        d.gram = 1;
        d.A = X;
        d.B = X;
        d.C = P;
        d.ldc = n;
        d.K = m;
        d.alpha = (float)alpha;
        d.gamma = (float)gamma;
        gemm_finalize(d, prec);
        return launch_gemm(prec, d, s);
    }
    // the slices run in one launch; slice y sums k in [y ks, (y + 1) ks) into
    // the upper triangle of its own n x n part, and the parts are added in
    // slice order in FP64
    int count = 0;
    hipError_t e = gram_slices(prec, X, ldx, X, ldx, m, n, splits, w.parts, &count, s, w.pk);
    if (e != hipSuccess)
        return e;
    return launch_splitk_sym_reduce(w.parts, n * n, count, n, alpha, gamma, P, n, s);
}

// Xn <- alpha X P + beta X (partials of (Xn - X)^2 in tiles if tiles != null;
// *ntiles receives their count).
static hipError_t update_step(const PolarPlan &p, int prec, const float *X, int64_t ldx,
                              const float *P, double alpha, double beta, float *Xn, int64_t ldxn,
                              double *tiles, int *ntiles, const PolarWs &w, hipStream_t s)
{
    const int64_t m = p.m, n = p.n;
    GemmDesc d;
    memset(&d, 0, sizeof d);
    d.A = X;
    d.lda = ldx;
    d.a_kcontig = 1;
    d.B = P;
    d.ldb = n;
    d.b_kcontig = 0;
    d.M = m;
    d.N = n;
    d.K = n;
    const int splits = update_splits(p);
    if (splits > 1 && (size_t)splits * m * n <= w.parts_floats) {
        // K-slices into m x n parts, added in FP64 with the update applied
        d.C = w.parts;
        d.ldc = n;
        d.alpha = 1.0f;
        gemm_finalize(d, prec);
        d.slices = slice_plan(n, splits, &d.slice_k);
        d.slice_stride = m * n;
        hipError_t e = gemm_packed_or_plain(prec, d, w.pk, s);
        if (e != hipSuccess)
            return e;
        if (ntiles)
            *ntiles = splitk_update_num_partials();
        return launch_splitk_update_reduce(w.parts, d.slices, m, n, alpha, beta,
                                           beta != 0.0 ? X : nullptr, ldx, Xn, ldxn, tiles, s);
    }
    d.C = Xn;
    d.ldc = ldxn;
    d.alpha = (float)alpha;
    if (beta != 0.0) {
        d.E = X;
        d.lde = ldx;
        d.beta = (float)beta;
    }
    d.partials = tiles;
    gemm_finalize(d, prec);
    if (ntiles)
        *ntiles = d.tiles_m * d.tiles_n;
    return gemm_packed_or_plain(prec, d, w.pk, s);
}

// H = (U^T A + A^T U) / 2 in one symmetric pass: the upper triangle of U^T A
// and of A^T U = (U^T A)^T are accumulated as Gram-mode slices (each of at most
// kMaxAccK rows of the K = m sum), and the 2 s slices are added in FP64 with
// the factor 1/2 and written to both triangles, so H is exactly symmetric.
static hipError_t h_step(const PolarPlan &p, const float *U, int64_t ldu, const float *A,
                         int64_t lda, float *H, int64_t ldh, const PolarWs &w, hipStream_t s)
{
    const int64_t n = p.n;
    const int want = h_splits(p);
    int c1 = 0, c2 = 0;
    hipError_t e = gram_slices(p.prec_h, U, ldu, A, lda, p.m, n, want, w.parts, &c1, s);
    if (e != hipSuccess)
        return e;
    e = gram_slices(p.prec_h, A, lda, U, ldu, p.m, n, want, w.parts + (size_t)c1 * n * n, &c2, s);
    if (e != hipSuccess)
        return e;
    return launch_splitk_sym_reduce(w.parts, n * n, c1 + c2, n, 0.5, 0.0, H, ldh, s);
}

// ------------------------------------------------------------------ inverse

// Algorithm NS_Inverse (section III.D) for an n x m A: X0 = A^T / ||A A^T||_F,
// X' = X (2I - A X) = (2I - X A) X.  The step forms the smaller product:
// A X (n x n) when n <= m, X A (m x m) when n > m.
struct InvPlan {
    int64_t n, m;
    int64_t r;       // side of the formed product
    int wide;        // 1: n <= m (forms A X); 0: n > m (forms X A)
    double eps;
    int max_iter, polish, literal;
    int prec;
};

static la_status inverse_plan(int64_t n, int64_t m, const la_inverse_opts *opts, InvPlan *out)
{
    if (n < 1 || m < 1) {
        set_error("la_inverse: sizes must be positive (n %lld, m %lld)", (long long)n,
                  (long long)m);
        return LA_ERR_SHAPE;
    }
    la_inverse_opts o;
    memset(&o, 0, sizeof o);
    if (opts)
        o = *opts;
    if (!valid_prec(o.prec)) {
        set_error("la_inverse: unknown precision %d", o.prec);
        return LA_ERR_INVALID_ARG;
    }
    if (!(o.eps >= 0.0) || !isfinite(o.eps) || o.max_iter < 0) {
        set_error("la_inverse: bad eps or max_iter");
        return LA_ERR_INVALID_ARG;
    }
    InvPlan p;
    p.n = n;
    p.m = m;
    p.wide = n <= m;
    p.r = p.wide ? n : m;
    p.eps = o.eps > 0.0 ? o.eps : ldexp(1.0, -24);
    p.max_iter = o.max_iter > 0 ? o.max_iter : 100;
    // AUTO: 3xBF16 steps, then one 6xBF16 step.  Forming I - A X near the
    // fixed point cancels to O(1) from terms of size ~cond(A), so the dropped
    // lo*lo products of 3xBF16 (2^-18 relative) limit its accuracy; the
    // iteration converges quadratically, so one 6xBF16 step restores FP32-level
    // accuracy.
    p.polish = o.polish != 0 || o.prec == LA_PREC_AUTO;
    p.literal = o.literal_delta != 0;
    p.prec = resolve_prec(o.prec, PREC_BF16X3);
    *out = p;
    return LA_OK;
}

static size_t inverse_max_tiles(const InvPlan &p)
{
    size_t t = 0;
    for (int pr : {PREC_FP32, PREC_BF16X3, PREC_BF16X6}) {
        const size_t tm = (size_t)((p.m + tile_m(pr, 1) - 1) / tile_m(pr, 1));
        const size_t tn = (size_t)((p.n + tile_n(pr, 1) - 1) / tile_n(pr, 1));
        t = std::max(t, tm * tn);
    }
    return t;
}

struct InvWs {
    float *X;        // m x n, ld n: the iterate's second buffer
    float *R;        // r x r: the Gram A A^T (or A^T A), then I - A X (or I - X A)
    double *tiles;   // per-tile step-norm partials
    double *sumsq;   // norm partials
    double *scal;    // [0] ||A A^T||_F^2, [1] ||X' - X||_F^2
    char *pk;        // packed 3xBF16 operands of the step's products (may be null)
    char *pka;       // A packed once for the first product (may be null)
};

// Packed operands of the larger of the two products of a step: R = A X
// (r x r, K = m) or X A (K = n), then X R (m x n, K = n) or R X (K = m);
// and A itself, packed once, as op(A) of A X or op(B)^T of X A (r rows, K = m
// or n).
static size_t inverse_step_pack_bytes(const InvPlan &p)
{
    const int64_t k1 = p.wide ? p.m : p.n, k2 = p.wide ? p.n : p.m;
    return std::max(pack_bytes(p.prec, p.r, p.r, k1), pack_bytes(p.prec, p.m, p.n, k2));
}

static size_t inverse_a_pack_bytes(const InvPlan &p)
{
    const int64_t k1 = p.wide ? p.m : p.n;
    return packs(p.prec, p.r, p.r, k1) ? align_up256(packed_x3_bytes(p.r, k1)) : 0;
}

static size_t inverse_pack_bytes(const InvPlan &p)
{
    return inverse_step_pack_bytes(p) + inverse_a_pack_bytes(p);
}

static size_t inverse_workspace_bytes(const InvPlan &p)
{
    size_t b = 0;
    b += align256((size_t)p.m * p.n * sizeof(float));
    b += align256((size_t)p.r * p.r * sizeof(float));
    b += align256(inverse_max_tiles(p) * sizeof(double));
    b += align256((size_t)sumsq_num_partials() * sizeof(double));
    b += align256(8 * sizeof(double));
    b += inverse_pack_bytes(p);
    return b;
}

static InvWs inverse_carve(const InvPlan &p, void *ws)
{
    InvWs w;
    char *b = (char *)ws;
    w.X = (float *)b;
    b += align256((size_t)p.m * p.n * sizeof(float));
    w.R = (float *)b;
    b += align256((size_t)p.r * p.r * sizeof(float));
    w.tiles = (double *)b;
    b += align256(inverse_max_tiles(p) * sizeof(double));
    w.sumsq = (double *)b;
    b += align256((size_t)sumsq_num_partials() * sizeof(double));
    w.scal = (double *)b;
    b += align256(8 * sizeof(double));
    w.pk = inverse_step_pack_bytes(p) ? b : nullptr;
    b += inverse_step_pack_bytes(p);
    w.pka = inverse_a_pack_bytes(p) ? b : nullptr;
    return w;
}

// One step X' = X + X (I - A X)  (wide / square)  or  X + (I - X A) X  (tall),
// with FP64 per-tile partials of (X' - X)^2 in w.tiles.
static hipError_t inverse_step(const InvPlan &p, int prec, const float *A, int64_t lda,
                               const float *X, int64_t ldx, float *Xn, int64_t ldxn,
                               const InvWs &w, int *ntiles, hipStream_t s)
{
    GemmDesc d;
    memset(&d, 0, sizeof d);
    d.C = w.R;
    d.ldc = p.r;
    d.M = p.r;
    d.N = p.r;
    d.alpha = -1.0f;
    d.gamma = 1.0f;
    if (p.wide) {               // R = I - A X: A (n x m) . X (m x n)
        d.A = A;
        d.lda = lda;
        d.a_kcontig = 1;
        d.B = X;
        d.ldb = ldx;
        d.b_kcontig = 0;
        d.K = p.m;
    } else {                    // R = I - X A: X (m x n) . A (n x m)
        d.A = X;
        d.lda = ldx;
        d.a_kcontig = 1;
        d.B = A;
        d.ldb = lda;
        d.b_kcontig = 0;
        d.K = p.n;
    }
    gemm_finalize(d, prec);
    // A was packed once for the step precision (the polish step does not pack)
    const char *pre = prec == p.prec ? w.pka : nullptr;
    hipError_t e = gemm_packed_or_plain(prec, d, w.pk, s, p.wide ? pre : nullptr,
                                        p.wide ? nullptr : pre);
    if (e != hipSuccess)
        return e;

    GemmDesc u;
    memset(&u, 0, sizeof u);
    u.C = Xn;
    u.ldc = ldxn;
    u.M = p.m;
    u.N = p.n;
    u.alpha = 1.0f;
    u.beta = 1.0f;
    u.E = X;
    u.lde = ldx;
    u.partials = w.tiles;
    if (p.wide) {               // X' = X + X R: X (m x n) . R (n x n)
        u.A = X;
        u.lda = ldx;
        u.a_kcontig = 1;
        u.B = w.R;
        u.ldb = p.r;
        u.b_kcontig = 0;
        u.K = p.n;
    } else {                    // X' = X + R X: R (m x m) . X (m x n)
        u.A = w.R;
        u.lda = p.r;
        u.a_kcontig = 1;
        u.B = X;
        u.ldb = ldx;
        u.b_kcontig = 0;
        u.K = p.m;
    }
    gemm_finalize(u, prec);
    *ntiles = u.tiles_m * u.tiles_n;
    return gemm_packed_or_plain(prec, u, w.pk, s);
}

// Validation and descriptor of a la_gemm-style call.  *empty: nothing to do
// (m or n is 0) after successful validation.
static la_status gemm_prepare(const char *who, la_context *ctx, int trans_a, int trans_b,
                              int64_t m, int64_t n, int64_t k, float alpha, const float *A,
                              int64_t lda, const float *B, int64_t ldb, float beta, float *C,
                              int64_t ldc, int prec, GemmDesc *out, int *prec_out, bool *empty)
{
    *empty = false;
    if (!valid_prec(prec)) {
        set_error("%s: invalid precision %d", who, prec);
        return LA_ERR_INVALID_ARG;
    }
    if (m < 0 || n < 0 || k < 0) {
        set_error("%s: negative size", who);
        return LA_ERR_SHAPE;
    }
    const int64_t a_cols = trans_a ? m : k, a_rows = trans_a ? k : m;
    const int64_t b_cols = trans_b ? k : n, b_rows = trans_b ? n : k;
    if (lda < std::max<int64_t>(a_cols, 1) || ldb < std::max<int64_t>(b_cols, 1) ||
        ldc < std::max<int64_t>(n, 1)) {
        set_error("%s: leading dimension smaller than the row length", who);
        return LA_ERR_SHAPE;
    }
    if (!ctx) {
        set_error("%s: ctx is NULL", who);
        return LA_ERR_INVALID_ARG;
    }
    if (m == 0 || n == 0) {
        *empty = true;
        return LA_OK;
    }
    if (!C || (k > 0 && (!A || !B))) {
        set_error("%s: NULL matrix pointer", who);
        return LA_ERR_INVALID_ARG;
    }
    const size_t cb = extent_bytes(m, n, ldc);
    if (k > 0 && (overlaps(C, cb, A, extent_bytes(a_rows, a_cols, lda)) ||
                  overlaps(C, cb, B, extent_bytes(b_rows, b_cols, ldb)))) {
        set_error("%s: C overlaps A or B", who);
        return LA_ERR_INVALID_ARG;
    }
    LA_HIP(hipSetDevice(ctx->device), "la_gemm: hipSetDevice");
    const int p = resolve_prec(prec, PREC_BF16X3);
    GemmDesc d;
    memset(&d, 0, sizeof d);
    d.A = A;
    d.lda = lda;
    d.a_kcontig = trans_a ? 0 : 1;
    d.B = B;
    d.ldb = ldb;
    d.b_kcontig = trans_b ? 1 : 0;
    d.C = C;
    d.ldc = ldc;
    d.M = m;
    d.N = n;
    d.K = k;
    d.alpha = alpha;
    if (beta != 0.0f) {
        d.E = C;
        d.lde = ldc;
        d.beta = beta;
    }
    gemm_finalize(d, p);
    *out = d;
    *prec_out = p;
    return LA_OK;
}

}  // namespace la

using namespace la;

extern "C" {

const char *la_status_string(la_status s)
{
    switch (s) {
    case LA_OK: return "LA_OK";
    case LA_ERR_INVALID_ARG: return "LA_ERR_INVALID_ARG";
    case LA_ERR_SHAPE: return "LA_ERR_SHAPE";
    case LA_ERR_NONFINITE: return "LA_ERR_NONFINITE";
    case LA_ERR_NOT_CONVERGED: return "LA_ERR_NOT_CONVERGED";
    case LA_ERR_OUT_OF_MEMORY: return "LA_ERR_OUT_OF_MEMORY";
    case LA_ERR_DEVICE: return "LA_ERR_DEVICE";
    case LA_ERR_QUEUE_FULL: return "LA_ERR_QUEUE_FULL";
    case LA_ERR_TOO_LARGE: return "LA_ERR_TOO_LARGE";
    case LA_ERR_NOT_READY: return "LA_ERR_NOT_READY";
    case LA_ERR_UNKNOWN_REQUEST: return "LA_ERR_UNKNOWN_REQUEST";
    case LA_ERR_BREAKDOWN: return "LA_ERR_BREAKDOWN";
    }
    return "LA_ERR_UNKNOWN_STATUS";
}

const char *la_last_error(void) { return g_err; }

la_status la_create(int device, la_context **out)
{
    g_err[0] = 0;
    if (!out) {
        set_error("la_create: out is NULL");
        return LA_ERR_INVALID_ARG;
    }
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0) {
        set_error("la_create: no HIP device (%s)", hipGetErrorString(e));
        return LA_ERR_DEVICE;
    }
    if (device < 0 || device >= count) {
        set_error("la_create: device %d out of range [0, %d)", device, count);
        return LA_ERR_INVALID_ARG;
    }
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess)
        return dev_fail(e, "la_create: hipGetDeviceProperties");
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        set_error("la_create: device %d is %s; this library is built for gfx950 only", device,
                  prop.gcnArchName);
        return LA_ERR_DEVICE;
    }
    if (device >= kMaxDevices) {
        set_error("la_create: device %d beyond the %d this library tracks", device, kMaxDevices);
        return LA_ERR_INVALID_ARG;
    }
    // the static workspace's address on this device, with the device current
    // (the caller's current device is restored)
    int prev = -1;
    e = hipGetDevice(&prev);
    if (e != hipSuccess)
        return dev_fail(e, "la_create: hipGetDevice");
    e = hipSetDevice(device);
    if (e != hipSuccess)
        return dev_fail(e, "la_create: hipSetDevice");
    void *sp = nullptr;
    e = scratch_address(device, &sp);
    const hipError_t e2 = hipSetDevice(prev);
    if (e != hipSuccess)
        return dev_fail(e, "la_create: hipGetSymbolAddress(scratch)");
    if (e2 != hipSuccess)
        return dev_fail(e2, "la_create: restoring the current device");
    la_context *c = new (std::nothrow) la_context;
    if (!c) {
        set_error("la_create: out of host memory");
        return LA_ERR_OUT_OF_MEMORY;
    }
    c->device = device;
    c->num_cus = prop.multiProcessorCount;
    c->scratch = sp;
    *out = c;
    return LA_OK;
}

la_status la_destroy(la_context *ctx)
{
    delete ctx;
    return LA_OK;
}

la_status la_gemm(la_context *ctx, int trans_a, int trans_b, int64_t m, int64_t n, int64_t k,
                  float alpha, const float *A, int64_t lda, const float *B, int64_t ldb,
                  float beta, float *C, int64_t ldc, la_precision prec, void *hip_stream)
{
    g_err[0] = 0;
    GemmDesc d;
    int p = 0;
    bool empty = false;
    la_status st = gemm_prepare("la_gemm", ctx, trans_a, trans_b, m, n, k, alpha, A, lda, B, ldb,
                                beta, C, ldc, prec, &d, &p, &empty);
    if (st != LA_OK || empty)
        return st;
    LA_HIP(launch_gemm(p, d, (hipStream_t)hip_stream), "la_gemm: launch");
    return LA_OK;
}

size_t la_pack_size(int64_t rows, int64_t k)
{
    if (rows < 0 || k < 0)
        return 0;
    return packed_x3_bytes(rows, k);
}

la_status la_pack_bf16x3(la_context *ctx, int kc, int64_t rows, int64_t k, const float *X,
                         int64_t ld, void *packed, size_t packed_bytes, void *hip_stream)
{
    g_err[0] = 0;
    if (rows < 0 || k < 0 || ld < std::max<int64_t>(kc ? k : rows, 1)) {
        set_error("la_pack_bf16x3: bad shape (rows %lld, k %lld, ld %lld)", (long long)rows,
                  (long long)k, (long long)ld);
        return LA_ERR_SHAPE;
    }
    if (!ctx || (rows > 0 && k > 0 && (!X || !packed))) {
        set_error("la_pack_bf16x3: NULL argument");
        return LA_ERR_INVALID_ARG;
    }
    const size_t need = packed_x3_bytes(rows, k);
    if (packed_bytes < need) {
        set_error("la_pack_bf16x3: buffer %zu bytes, need %zu", packed_bytes, need);
        return LA_ERR_OUT_OF_MEMORY;
    }
    if (need == 0)
        return LA_OK;
    if (overlaps(packed, need, X, extent_bytes(kc ? rows : k, kc ? k : rows, ld))) {
        set_error("la_pack_bf16x3: output overlaps X");
        return LA_ERR_INVALID_ARG;
    }
    LA_HIP(hipSetDevice(ctx->device), "la_pack_bf16x3: hipSetDevice");
    LA_HIP(launch_pack_x3(X, ld, kc ? 1 : 0, rows, k, packed, (hipStream_t)hip_stream),
           "la_pack_bf16x3: launch");
    return LA_OK;
}

la_status la_gemm_packed(la_context *ctx, int64_t m, int64_t n, int64_t k, float alpha,
                         const void *Ap, const void *Bp, float beta, float *C, int64_t ldc,
                         void *hip_stream)
{
    g_err[0] = 0;
    if (m < 0 || n < 0 || k < 0 || ldc < std::max<int64_t>(n, 1)) {
        set_error("la_gemm_packed: bad shape");
        return LA_ERR_SHAPE;
    }
    if (!ctx) {
        set_error("la_gemm_packed: ctx is NULL");
        return LA_ERR_INVALID_ARG;
    }
    if (m == 0 || n == 0)
        return LA_OK;
    if (!C || (k > 0 && (!Ap || !Bp))) {
        set_error("la_gemm_packed: NULL argument");
        return LA_ERR_INVALID_ARG;
    }
    const size_t cb = extent_bytes(m, n, ldc);
    if (k > 0 && (overlaps(C, cb, Ap, packed_x3_bytes(m, k)) ||
                  overlaps(C, cb, Bp, packed_x3_bytes(n, k)))) {
        set_error("la_gemm_packed: C overlaps a packed operand");
        return LA_ERR_INVALID_ARG;
    }
    LA_HIP(hipSetDevice(ctx->device), "la_gemm_packed: hipSetDevice");
    GemmDesc d;
    memset(&d, 0, sizeof d);
    d.A = (const float *)Ap;
    d.B = (const float *)Bp;
    d.C = C;
    d.ldc = ldc;
    d.M = m;
    d.N = n;
    d.K = k;
    d.alpha = alpha;
    if (beta != 0.0f) {
        d.E = C;
        d.lde = ldc;
        d.beta = beta;
    }
    d.tiles_m = (int)((m + 255) / 256);
    d.tiles_n = (int)((n + 255) / 256);
    d.num_tiles = d.tiles_m * d.tiles_n;
    LA_HIP(launch_gemm_packed_x3(d, (hipStream_t)hip_stream), "la_gemm_packed: launch");
    return LA_OK;
}

size_t la_gemm_workspace_size(int64_t m, int64_t n, int64_t k)
{
    if (m < 0 || n < 0 || k < 0)
        return 0;
    return align256(packed_x3_bytes(m, k)) + align256(packed_x3_bytes(n, k));
}

la_status la_gemm_ws(la_context *ctx, int trans_a, int trans_b, int64_t m, int64_t n, int64_t k,
                     float alpha, const float *A, int64_t lda, const float *B, int64_t ldb,
                     float beta, float *C, int64_t ldc, la_precision prec, void *workspace,
                     size_t ws_bytes, void *hip_stream)
{
    g_err[0] = 0;
    GemmDesc d;
    int p = 0;
    bool empty = false;
    la_status st = gemm_prepare("la_gemm_ws", ctx, trans_a, trans_b, m, n, k, alpha, A, lda, B,
                                ldb, beta, C, ldc, prec, &d, &p, &empty);
    if (st != LA_OK || empty)
        return st;
    hipStream_t s = (hipStream_t)hip_stream;
    // packed path: 3xBF16 on 256 x 256 tiles with enough K to repay the pack pass
    if (p != PREC_BF16X3 || d.small || k < 256) {
        LA_HIP(launch_gemm(p, d, s), "la_gemm_ws: launch");
        return LA_OK;
    }
    const size_t pa = align256(packed_x3_bytes(m, k)), need = pa + align256(packed_x3_bytes(n, k));
    if (!workspace || ((uintptr_t)workspace & 255u) != 0) {
        set_error("la_gemm_ws: workspace must be non-NULL and 256-byte aligned");
        return LA_ERR_INVALID_ARG;
    }
    if (ws_bytes < need) {
        set_error("la_gemm_ws: workspace %zu bytes, need %zu", ws_bytes, need);
        return LA_ERR_OUT_OF_MEMORY;
    }
    const int64_t a_cols = trans_a ? m : k, a_rows = trans_a ? k : m;
    const int64_t b_cols = trans_b ? k : n, b_rows = trans_b ? n : k;
    if (overlaps(workspace, need, A, extent_bytes(a_rows, a_cols, lda)) ||
        overlaps(workspace, need, B, extent_bytes(b_rows, b_cols, ldb)) ||
        overlaps(workspace, need, C, extent_bytes(m, n, ldc))) {
        set_error("la_gemm_ws: workspace overlaps A, B or C");
        return LA_ERR_INVALID_ARG;
    }
    char *wa = (char *)workspace, *wb = wa + pa;
    // op(A) rows are the output rows; op(B)^T rows are the output columns
    LA_HIP(launch_pack_x3(A, lda, trans_a ? 0 : 1, m, k, wa, s), "la_gemm_ws: pack A");
    LA_HIP(launch_pack_x3(B, ldb, trans_b ? 1 : 0, n, k, wb, s), "la_gemm_ws: pack B");
    d.A = (const float *)wa;
    d.B = (const float *)wb;
    d.tiles_m = (int)((m + 255) / 256);
    d.tiles_n = (int)((n + 255) / 256);
    d.num_tiles = d.tiles_m * d.tiles_n;
    LA_HIP(launch_gemm_packed_x3(d, s), "la_gemm_ws: launch");
    return LA_OK;
}

size_t la_polar_workspace_size(int64_t m, int64_t n, const la_polar_opts *opts)
{
    PolarPlan p;
    if (polar_plan(m, n, opts, &p) != LA_OK)
        return 0;
    return polar_workspace_bytes(p);
}

}  // extern "C"

namespace la {

static la_status polar_impl(la_context *ctx, const PolarPlan &p, const float *A, int64_t lda,
                            float *U, int64_t ldu, float *H, int64_t ldh, void *workspace,
                            size_t ws_bytes, la_polar_info *info, void *hip_stream);

}  // namespace la

extern "C" {

la_status la_polar(la_context *ctx, int64_t m, int64_t n, const float *A, int64_t lda, float *U,
                   int64_t ldu, float *H, int64_t ldh, void *workspace, size_t ws_bytes,
                   const la_polar_opts *opts, la_polar_info *info, void *hip_stream)
{
    g_err[0] = 0;
    PolarPlan p;
    la_status st = polar_plan(m, n, opts, &p);
    if (st != LA_OK)
        return st;
    return polar_impl(ctx, p, A, lda, U, ldu, H, ldh, workspace, ws_bytes, info, hip_stream);
}

la_status la_polar_noalloc(la_context *ctx, int64_t m, int64_t n, const float *A, int64_t lda,
                           float *U, int64_t ldu, float *H, int64_t ldh,
                           const la_polar_opts *opts, la_polar_info *info, void *hip_stream)
{
    g_err[0] = 0;
    PolarPlan p;
    la_status st = polar_plan(m, n, opts, &p);
    if (st != LA_OK)
        return st;
    if (!ctx) {
        set_error("la_polar_noalloc: ctx is NULL");
        return LA_ERR_INVALID_ARG;
    }
    const size_t need = polar_workspace_bytes(p);
    if (need > kScratchBytes) {
        set_error("la_polar_noalloc: a %lld x %lld polar needs %zu bytes of workspace; the "
                  "static buffer holds %zu (use la_polar with a workspace)",
                  (long long)m, (long long)n, need, kScratchBytes);
        return LA_ERR_TOO_LARGE;
    }
    return polar_impl(ctx, p, A, lda, U, ldu, H, ldh, ctx->scratch, kScratchBytes, info,
                      hip_stream);
}

}  // extern "C"

namespace la {

static la_status polar_impl(la_context *ctx, const PolarPlan &p, const float *A, int64_t lda,
                            float *U, int64_t ldu, float *H, int64_t ldh, void *workspace,
                            size_t ws_bytes, la_polar_info *info, void *hip_stream)
{
    const int64_t m = p.m, n = p.n;
    if (lda < n || ldu < n || (H && ldh < n)) {
        set_error("la_polar: leading dimension smaller than n");
        return LA_ERR_SHAPE;
    }
    if (!ctx || !A || !U || !workspace) {
        set_error("la_polar: NULL argument");
        return LA_ERR_INVALID_ARG;
    }
    if (((uintptr_t)workspace & 255u) != 0) {
        set_error("la_polar: workspace must be 256-byte aligned");
        return LA_ERR_INVALID_ARG;
    }
    const size_t need = polar_workspace_bytes(p);
    if (ws_bytes < need) {
        set_error("la_polar: workspace %zu bytes, need %zu", ws_bytes, need);
        return LA_ERR_OUT_OF_MEMORY;
    }
    const size_t ab = extent_bytes(m, n, lda), ub = extent_bytes(m, n, ldu);
    const size_t hb = H ? extent_bytes(n, n, ldh) : 0;
    if (overlaps(U, ub, A, ab) || overlaps(U, ub, workspace, need) ||
        (H && (overlaps(H, hb, A, ab) || overlaps(H, hb, U, ub) ||
               overlaps(H, hb, workspace, need)))) {
        set_error("la_polar: U / H overlap A, each other or the workspace");
        return LA_ERR_INVALID_ARG;
    }
    LA_HIP(hipSetDevice(ctx->device), "la_polar: hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    PolarWs w = carve(p, workspace);

    la_polar_info inf;
    memset(&inf, 0, sizeof inf);
    inf.prec_precond = p.prec_pre;
    inf.prec_ns = p.prec_ns;
    inf.prec_h = p.prec_h;
    inf.last_delta = INFINITY;
    inf.stop_reason = 2;

    // ||A||_F in FP64
    double h2[2];
    LA_HIP(launch_sumsq(A, m, n, lda, w.sumsq, s), "la_polar: norm");
    LA_HIP(launch_reduce_fixed(w.sumsq, sumsq_num_partials(), w.scal, s), "la_polar: norm");
    LA_HIP(hipMemcpyAsync(h2, w.scal, sizeof(double), hipMemcpyDeviceToHost, s),
           "la_polar: readback");
    LA_HIP(hipStreamSynchronize(s), "la_polar: sync");
    const double fro = sqrt(h2[0]);
    inf.fro_norm_a = fro;
    if (!(fro > 0.0) || !isfinite(fro)) {
        if (info)
            *info = inf;
        set_error("la_polar: ||A||_F = %g (zero or not finite)", fro);
        return LA_ERR_NONFINITE;
    }

    // ping-pong between U (ld ldu) and the workspace copy (ld n)
    float *buf[2] = {U, w.X};
    int64_t ld[2] = {ldu, n};
    int cur = 0;
    LA_HIP(launch_scale(A, lda, buf[cur], ld[cur], m, n, fro, s), "la_polar: scale");

    // preconditioning: U <- a U (I - c U^T U), c = (4/27) a^2
    for (int i = 0; i < p.k_pre; ++i) {
        LA_HIP(gram_step(p, p.prec_pre, buf[cur], ld[cur], -p.c, 1.0, w.P, w, s),
               "la_polar: precondition gram");
        LA_HIP(update_step(p, p.prec_pre, buf[cur], ld[cur], w.P, p.a, 0.0, buf[cur ^ 1],
                           ld[cur ^ 1], nullptr, nullptr, w, s),
               "la_polar: precondition update");
        cur ^= 1;
        inf.iters_precond++;
    }

    // Newton-Schulz: U' = U + U (I - U^T U) / 2, delta = ||U' - U||_F, until the
    // stop test (polar_host.h); a polish step runs at BF16X6
    StopState stop;
    bool converged = false;
    for (;;) {
        const int prec = stop.stopped ? PREC_BF16X6 : p.prec_ns;
        int ntiles = 0;
        LA_HIP(gram_step(p, prec, buf[cur], ld[cur], -1.0, 1.0, w.P, w, s),
               "la_polar: NS gram");
        LA_HIP(update_step(p, prec, buf[cur], ld[cur], w.P, 0.5, 1.0, buf[cur ^ 1], ld[cur ^ 1],
                           w.tiles, &ntiles, w, s),
               "la_polar: NS update");
        LA_HIP(launch_reduce_fixed(w.tiles, ntiles, w.scal + 1, s), "la_polar: delta");
        LA_HIP(hipMemcpyAsync(h2 + 1, w.scal + 1, sizeof(double), hipMemcpyDeviceToHost, s),
               "la_polar: readback");
        LA_HIP(hipStreamSynchronize(s), "la_polar: sync");
        cur ^= 1;
        inf.iters_ns++;
        const double delta = sqrt(h2[1]);
        inf.last_delta = delta;
        if (!isfinite(delta)) {
            if (info)
                *info = inf;
            set_error("la_polar: step norm is not finite");
            return LA_ERR_NONFINITE;
        }
        const StopDecision d = stop_test(p, m, n, delta, stop, inf.iters_ns);
        inf.stop_reason = stop.reason;
        if (d == STOP_DONE) {
            converged = true;
            break;
        }
        if (d == STOP_CAP)
            break;
    }
    if (cur != 0)
        LA_HIP(launch_copy(buf[cur], ld[cur], U, ldu, m, n, s), "la_polar: copy");

    if (H)
        LA_HIP(h_step(p, U, ldu, A, lda, H, ldh, w, s), "la_polar: H");
    LA_HIP(hipStreamSynchronize(s), "la_polar: final sync");
    if (info)
        *info = inf;
    if (!converged) {
        set_error("la_polar: no convergence after %d Newton-Schulz steps (delta %g)",
                  inf.iters_ns, inf.last_delta);
        return LA_ERR_NOT_CONVERGED;
    }
    return LA_OK;
}

}  // namespace la

extern "C" {

size_t la_inverse_workspace_size(int64_t n, int64_t m, const la_inverse_opts *opts)
{
    InvPlan p;
    if (inverse_plan(n, m, opts, &p) != LA_OK)
        return 0;
    return inverse_workspace_bytes(p);
}

la_status la_inverse(la_context *ctx, int64_t n, int64_t m, const float *A, int64_t lda,
                     float *X, int64_t ldx, void *workspace, size_t ws_bytes,
                     const la_inverse_opts *opts, la_inverse_info *info, void *hip_stream)
{
    g_err[0] = 0;
    InvPlan p;
    la_status st = inverse_plan(n, m, opts, &p);
    if (st != LA_OK)
        return st;
    if (lda < m || ldx < n) {
        set_error("la_inverse: leading dimension too small (lda %lld < m or ldx %lld < n)",
                  (long long)lda, (long long)ldx);
        return LA_ERR_SHAPE;
    }
    if (!ctx || !A || !X || !workspace) {
        set_error("la_inverse: NULL argument");
        return LA_ERR_INVALID_ARG;
    }
    if (((uintptr_t)workspace & 255u) != 0) {
        set_error("la_inverse: workspace must be 256-byte aligned");
        return LA_ERR_INVALID_ARG;
    }
    const size_t need = inverse_workspace_bytes(p);
    if (ws_bytes < need) {
        set_error("la_inverse: workspace %zu bytes, need %zu", ws_bytes, need);
        return LA_ERR_OUT_OF_MEMORY;
    }
    const size_t ab = extent_bytes(n, m, lda), xb = extent_bytes(m, n, ldx);
    if (overlaps(X, xb, A, ab) || overlaps(X, xb, workspace, need)) {
        set_error("la_inverse: X overlaps A or the workspace");
        return LA_ERR_INVALID_ARG;
    }
    LA_HIP(hipSetDevice(ctx->device), "la_inverse: hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    InvWs w = inverse_carve(p, workspace);

    la_inverse_info inf;
    memset(&inf, 0, sizeof inf);
    inf.product_side = p.wide;
    inf.prec = p.prec;
    inf.last_delta = INFINITY;
    inf.stop_reason = 2;

    // a = ||A A^T||_F = ||A^T A||_F, from the smaller symmetric Gram (FP64 norm)
    {
        GemmDesc g;
        memset(&g, 0, sizeof g);
        g.A = A;
        g.B = A;
        g.lda = lda;
        g.ldb = lda;
        g.C = w.R;
        g.ldc = p.r;
        g.M = p.r;
        g.N = p.r;
        g.alpha = 1.0f;
        g.gram = 1;
        if (p.wide) {           // A A^T: op(A)(i, k) = A[i][k], op(B)(k, j) = A[j][k]
            g.a_kcontig = 1;
            g.b_kcontig = 1;
            g.K = p.m;
        } else {                // A^T A: op(A)(i, k) = A[k][i], op(B)(k, j) = A[k][j]
            g.a_kcontig = 0;
            g.b_kcontig = 0;
            g.K = p.n;
        }
        gemm_finalize(g, p.prec);
        LA_HIP(launch_gemm(p.prec, g, s), "la_inverse: gram");
    }
    double h2[2];
    LA_HIP(launch_sumsq(w.R, p.r, p.r, p.r, w.sumsq, s), "la_inverse: norm");
    LA_HIP(launch_reduce_fixed(w.sumsq, sumsq_num_partials(), w.scal, s), "la_inverse: norm");
    LA_HIP(hipMemcpyAsync(h2, w.scal, sizeof(double), hipMemcpyDeviceToHost, s),
           "la_inverse: readback");
    LA_HIP(hipStreamSynchronize(s), "la_inverse: sync");
    const double a = sqrt(h2[0]);
    inf.gram_norm = a;
    if (!(a > 0.0) || !isfinite(a)) {
        if (info)
            *info = inf;
        set_error("la_inverse: ||A A^T||_F = %g (zero or not finite)", a);
        return LA_ERR_NONFINITE;
    }

    // X0 = A^T / a; ping-pong between X (ld ldx) and the workspace copy (ld n)
    float *buf[2] = {X, w.X};
    int64_t ld[2] = {ldx, n};
    int cur = 0;
    LA_HIP(launch_transpose_scale(A, lda, buf[cur], ld[cur], n, m, a, s), "la_inverse: X0");
    if (w.pka)   // A as op(A) of A X (k contiguous) or as op(B)^T of X A (k-major)
        LA_HIP(launch_pack_x3(A, lda, p.wide ? 1 : 0, p.r, p.wide ? p.m : p.n, w.pka, s),
               "la_inverse: pack A");

    const double scale = p.literal ? 1.0 : sqrt(a);
    double eps = p.eps;
    const int total = p.max_iter + (p.polish ? 1 : 0);
    bool stopped = false;
    for (int it = 0; it < total; ++it) {
        const bool polishing = stopped;
        const int prec = polishing ? PREC_BF16X6 : p.prec;
        int ntiles = 0;
        LA_HIP(inverse_step(p, prec, A, lda, buf[cur], ld[cur], buf[cur ^ 1], ld[cur ^ 1], w,
                            &ntiles, s),
               "la_inverse: step");
        LA_HIP(launch_reduce_fixed(w.tiles, ntiles, w.scal + 1, s), "la_inverse: delta");
        LA_HIP(hipMemcpyAsync(h2 + 1, w.scal + 1, sizeof(double), hipMemcpyDeviceToHost, s),
               "la_inverse: readback");
        LA_HIP(hipStreamSynchronize(s), "la_inverse: sync");
        cur ^= 1;
        inf.iters++;
        const double delta = scale * sqrt(h2[1]);
        if (!isfinite(delta)) {
            if (info)
                *info = inf;
            set_error("la_inverse: step norm is not finite");
            return LA_ERR_NONFINITE;
        }
        if (polishing)
            break;
        eps *= 2.0;                 // the tolerance grows after every step
        inf.last_delta = delta;
        inf.last_tol = eps;
        if (!(delta > eps)) {
            inf.stop_reason = 0;
            stopped = true;
        }
        if (stopped && !p.polish)
            break;
        if (!stopped && it + 1 >= p.max_iter)
            break;
    }
    if (cur != 0)
        LA_HIP(launch_copy(buf[cur], ld[cur], X, ldx, m, n, s), "la_inverse: copy");
    LA_HIP(hipStreamSynchronize(s), "la_inverse: final sync");
    if (info)
        *info = inf;
    if (!stopped) {
        set_error("la_inverse: tolerance not met after %d steps (delta %g, tol %g)", inf.iters,
                  inf.last_delta, inf.last_tol);
        return LA_ERR_NOT_CONVERGED;
    }
    return LA_OK;
}

}  // extern "C"
