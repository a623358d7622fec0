/*
 * la.h -- C ABI of the MI355X (gfx950) FP32-accurate GEMM and Newton-Schulz
 * polar factorisation library.
 *
 * The operations follow "Large Scale Distributed Linear Algebra With Tensor
 * Processing Units" (arXiv 2112.09017):
 *   la_gemm   -- C = A B (section III, task list; eq. (Matmul) of III.A), with
 *                transposed operands (III.A: SUMMA handles transposes);
 *   la_polar  -- A = U H for an (M, N) A with M >= N, U with orthonormal
 *                columns and H positive semi-definite (eq. (PolarDecomp),
 *                III.D), computed by the preconditioned Newton-Schulz
 *                iteration of Algorithm NS_Polar (eqs. (a_def)-(RogueMatrix),
 *                (NewtonSchulz));
 *   la_inverse -- X with X A = I or A X = I for a full-rank (N, M) A, by the
 *                Newton-Schulz inversion of Algorithm NS_Inverse (III.D);
 *   la_matfunc_odd / la_matfunc_cheb -- polynomial matrix functions of the
 *                singular values (eq. OddPoly) and of the eigenvalues by a
 *                Chebyshev series (eq. EigenvaluePolynomial, III.D);
 *   la_tsqr / la_wy / la_caqr -- QR factorisation (III.B): Algorithm tsqr
 *                for tall panels, the WY form of eq. (Yamamoto), and the
 *                right-looking Algorithm caqr;
 *   la_serve_* -- a continuous-batching server of la_polar requests.
 *
 * Conventions (the paper is silent on all of them):
 *   - real FP32 data, ROW-MAJOR with explicit leading dimensions: element
 *     (i, j) of X with leading dimension ldx is X[i * ldx + j];
 *   - every matrix pointer passed to la_gemm / la_polar / la_inverse /
 *     la_matfunc_* / la_tsqr / la_wy / la_caqr is DEVICE memory owned by the
 *     caller; the library never frees or retains it;
 *   - hip_stream is a hipStream_t (NULL = the legacy default stream); la_gemm
 *     only enqueues work, la_polar and la_inverse block on a per-iteration
 *     8-byte readback, the other calls return after their last kernel
 *     (la_caqr also uses a second stream of its own, joined before it
 *     returns);
 *   - no exceptions cross the ABI and nothing aborts: every call returns a
 *     la_status; la_last_error() gives a message for the calling thread.
 */
#ifndef LA_H
#define LA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LA_OK = 0,
    LA_ERR_INVALID_ARG = 1,    /* null pointer, bad enum, aliasing, ...          */
    LA_ERR_SHAPE = 2,          /* negative size, ld < row length, M < N (polar)  */
    LA_ERR_NONFINITE = 3,      /* ||A||_F or a step norm is Inf/NaN, or A == 0   */
    LA_ERR_NOT_CONVERGED = 4,  /* max_iter reached without meeting the tolerance */
    LA_ERR_OUT_OF_MEMORY = 5,  /* workspace / arena smaller than required        */
    LA_ERR_DEVICE = 6,         /* HIP runtime error or unsupported device        */
    LA_ERR_QUEUE_FULL = 7,     /* serving queue at capacity                      */
    LA_ERR_TOO_LARGE = 8,      /* request footprint exceeds the serving arena    */
    LA_ERR_NOT_READY = 9,      /* serving request still pending                  */
    LA_ERR_UNKNOWN_REQUEST = 10,
    LA_ERR_BREAKDOWN = 11      /* I - Q_1 singular or nearly so (eq. Yamamoto)   */
} la_status;

/* Arithmetic of the GEMM products.  All paths read and write FP32 and
 * accumulate in FP32 on the matrix cores.
 *   FP32   : v_mfma_f32_32x32x2_f32 on the FP32 operands.
 *   BF16X3 : each operand x = hi + lo with hi = bf16(x), lo = bf16(x - hi)
 *            (round to nearest even); products hi*hi + hi*lo + lo*hi on the
 *            BF16 matrix cores (each product exact in FP32).
 *   BF16X6 : x = hi + mid + lo (three bf16 terms, 24 significant bits);
 *            products hh + hm + mh + mm + hl + lh.
 *   AUTO   : la_gemm -> BF16X3; la_polar -> per phase (see la_polar_opts):
 *            preconditioning and H at BF16X6, Newton-Schulz at BF16X3;
 *            la_inverse -> BF16X3 steps and one BF16X6 step; la_matfunc_* ->
 *            BF16X6.
 * The paper's TPU "fp32" matmul is itself a bf16-based emulation at about
 * six times the bf16 cost (section II); BF16X6 is the analogue here. */
typedef enum {
    LA_PREC_AUTO = 0,
    LA_PREC_FP32 = 1,
    LA_PREC_BF16X3 = 2,
    LA_PREC_BF16X6 = 3
} la_precision;

typedef struct la_context la_context;

/* Create a context on HIP device `device` (must be gfx950).  Allocates no
 * device memory.  *out is set only on LA_OK. */
la_status la_create(int device, la_context **out);
/* Destroy a context (NULL is accepted).  Does not synchronise any stream. */
la_status la_destroy(la_context *ctx);

/* Static text for a status code (never NULL). */
const char *la_status_string(la_status s);
/* Message describing the last failed call made by this thread ("" if none).
 * Valid until the next library call on this thread. */
const char *la_last_error(void);

/* ------------------------------------------------------------------------
 * GEMM (section III.A, eq. (Matmul)):  C <- alpha op(A) op(B) + beta C
 *   op(A) is m x k: A is m x k (lda >= k) if trans_a == 0, else k x m
 *                   (lda >= m);
 *   op(B) is k x n: B is k x n (ldb >= n) if trans_b == 0, else n x k
 *                   (ldb >= k);
 *   C is m x n (ldc >= n) and must not overlap A or B.
 * beta == 0 means C is not read (it may hold NaN).  m, n, k may be 0
 * (k == 0 gives C <- beta C).  Enqueued on hip_stream; returns without
 * waiting.  Arguments are validated before any device call.
 * ---------------------------------------------------------------------- */
la_status la_gemm(la_context *ctx, int trans_a, int trans_b, int64_t m,
                  int64_t n, int64_t k, float alpha, const float *A,
                  int64_t lda, const float *B, int64_t ldb, float beta,
                  float *C, int64_t ldc, la_precision prec, void *hip_stream);

/* Workspace variant of la_gemm (same arguments, same result bit for bit).
 * When the product runs at BF16X3 (prec BF16X3 or AUTO) on 256 x 256 tiles
 * with k >= 256, op(A) and op(B) are first split into their bf16 terms and
 * written to `workspace` in the order the GEMM's LDS tiles use (one HBM pass
 * over each operand), and the product then streams them straight from HBM to
 * LDS, with no split in its inner loop.  Otherwise it runs exactly as
 * la_gemm and does not touch the workspace.  workspace: device memory of at
 * least la_gemm_workspace_size(m, n, k) bytes, 256-byte aligned, overlapping
 * none of A, B, C.  Enqueued on hip_stream; returns without waiting. */
size_t la_gemm_workspace_size(int64_t m, int64_t n, int64_t k);
la_status la_gemm_ws(la_context *ctx, int trans_a, int trans_b, int64_t m,
                     int64_t n, int64_t k, float alpha, const float *A,
                     int64_t lda, const float *B, int64_t ldb, float beta,
                     float *C, int64_t ldc, la_precision prec, void *workspace,
                     size_t ws_bytes, void *hip_stream);

/* The two halves of la_gemm_ws, for callers that reuse an operand (pack it
 * once, multiply many times).  la_pack_bf16x3 splits op(X) (rows x k; kc = 1:
 * element (r, p) is X[r * ld + p], kc = 0: X[p * ld + r]) into its bf16
 * hi/lo terms in the GEMM's LDS tile order, zero-padded; `packed` is device
 * memory of at least la_pack_size(rows, k) bytes.  la_gemm_packed computes
 * C <- alpha op(A) op(B) + beta C from Ap = pack of op(A) (m x k) and Bp =
 * pack of op(B)^T (n x k), bitwise as la_gemm at BF16X3 would.  Both are
 * enqueued on hip_stream and return without waiting. */
size_t la_pack_size(int64_t rows, int64_t k);
la_status la_pack_bf16x3(la_context *ctx, int kc, int64_t rows, int64_t k, const float *X,
                         int64_t ld, void *packed, size_t packed_bytes, void *hip_stream);
la_status la_gemm_packed(la_context *ctx, int64_t m, int64_t n, int64_t k, float alpha,
                         const void *Ap, const void *Bp, float beta, float *C, int64_t ldc,
                         void *hip_stream);

/* ------------------------------------------------------------------------
 * Polar factorisation (section III.D, Algorithm NS_Polar).
 * ---------------------------------------------------------------------- */

/* Options; a zero-initialised struct means the defaults in brackets. */
typedef struct {
    double s_minus;   /* threshold s_- of eq. (a_def), in [1e-3, 1)      [0.1]   */
    double s0;        /* estimate of the smallest singular value of
                         A / ||A||_F; fixes the preconditioning count     [2^-23] */
    double eps;       /* tolerance: stop once ||U' - U||_F <= max(M,N) eps [2^-23] */
    int max_iter;     /* cap on Newton-Schulz steps                     [100]   */
    int prec_precond; /* la_precision of the preconditioning GEMMs [AUTO=BF16X6] */
    int prec_ns;      /* la_precision of the Newton-Schulz GEMMs   [AUTO=BF16X3] */
    int prec_h;       /* la_precision of H = sym(U^T A)            [AUTO=BF16X6] */
    int polish;       /* 1: one extra Newton-Schulz step at BF16X6 after the
                         stop test                                          [0] */
    int no_stagnation;/* 1: disable the stagnation stop                     [0] */
    int max_acc_k;    /* FP32 accumulation depth: a product of the iteration
                         or of H whose inner dimension exceeds it is split
                         along K into slices of at most this length (rounded
                         up to a multiple of 32), each accumulated in FP32,
                         and the slices are added in FP64           [4096] */
    int reserved[2];
} la_polar_opts;

typedef struct {
    int iters_precond;   /* preconditioning steps (from the s recurrence)     */
    int iters_ns;        /* Newton-Schulz steps, polish included              */
    double fro_norm_a;   /* ||A||_F, accumulated in FP64 on the GPU            */
    double last_delta;   /* ||U' - U||_F of the last step (FP64)               */
    int stop_reason;     /* 0 tolerance, 1 stagnation, 2 iteration cap        */
    int prec_precond;    /* resolved precisions actually used                 */
    int prec_ns;
    int prec_h;
} la_polar_info;

/* Bytes of device workspace la_polar needs for an m x n input (0 on bad
 * arguments).  opts may be NULL.  It holds the second iterate (m n floats),
 * P (n^2), split-K Gram parts for tall inputs (up to 16 n^2), FP64 partials,
 * and, when a step runs at 3xBF16 on 256 x 256 tiles, packed copies of the
 * iterate and of P for the update (about m n + n^2 floats). */
size_t la_polar_workspace_size(int64_t m, int64_t n, const la_polar_opts *opts);

/* A (m x n, lda >= n, m >= n >= 1) is read only.  U (m x n, ldu >= n)
 * receives the polar factor; H (n x n, ldh >= n) receives
 * (U^T A + A^T U) / 2 (the paper's H = U^T A, symmetrised) unless H is NULL.
 * U and H must not overlap A, each other or the workspace.
 * workspace: device memory of at least la_polar_workspace_size() bytes,
 * 256-byte aligned.  Runs on hip_stream and returns after the last kernel
 * has completed (it reads one FP64 norm back per iteration).
 * LA_ERR_NONFINITE if ||A||_F is 0, Inf or NaN, or a step norm is not
 * finite; LA_ERR_NOT_CONVERGED if the cap was hit (U then holds the last
 * iterate).  info may be NULL. */
la_status la_polar(la_context *ctx, int64_t m, int64_t n, const float *A,
                   int64_t lda, float *U, int64_t ldu, float *H, int64_t ldh,
                   void *workspace, size_t ws_bytes, const la_polar_opts *opts,
                   la_polar_info *info, void *hip_stream);

/* la_polar without a caller workspace, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid allocation): the same computation as la_polar, bit for bit,
 * with the workspace taken from a buffer of LA_POLAR_NOALLOC_BYTES that the
 * library holds statically on every GPU it runs on (from the first la_create
 * on that device until the process ends).  Allocates nothing: no device or
 * host allocation is made by the call.  LA_ERR_TOO_LARGE if
 * la_polar_workspace_size(m, n, opts) exceeds LA_POLAR_NOALLOC_BYTES (square
 * inputs up to about n = 2000 fit at the default options).  The buffer keeps
 * the last call's contents (nothing in it needs to start at zero), and all
 * calls on one GPU share it: calls that overlap in time on one GPU (from
 * several threads, or on several streams) race and must be serialised by the
 * caller.  Other arguments, results and errors as for la_polar. */
#define LA_POLAR_NOALLOC_BYTES ((size_t)64 << 20)
la_status la_polar_noalloc(la_context *ctx, int64_t m, int64_t n, const float *A,
                           int64_t lda, float *U, int64_t ldu, float *H, int64_t ldh,
                           const la_polar_opts *opts, la_polar_info *info,
                           void *hip_stream);

/* ------------------------------------------------------------------------
 * Newton-Schulz matrix inversion (section III.D, Algorithm NS_Inverse).
 * For an n x m A of full rank it returns the m x n X with X A = I_m
 * (n >= m) or A X = I_n (n <= m): the inverse when A is square, else the
 * Moore-Penrose pseudo-inverse.  a = ||A A^T||_F, X0 = A^T / a, then
 *   X' = X (2I - A X) = (2I - X A) X,   evaluated as X + X (I - A X) when
 *   n <= m and as X + (I - X A) X when n > m (the smaller product; the two
 *   are the same polynomial in exact arithmetic),
 * until the step norm delta = sqrt(a) ||X' - X||_F is at most the
 * tolerance, which starts at eps and doubles after every step.  (delta is
 * measured on the normalised problem A / sqrt(a), so the stop does not
 * depend on the scale of A; literal_delta = 1 compares ||X' - X||_F as the
 * algorithm prints it.)
 * ---------------------------------------------------------------------- */
typedef struct {
    double eps;        /* starting tolerance (unit roundoff)      [2^-24]      */
    int max_iter;      /* cap on steps                             [100]        */
    int prec;          /* la_precision of the products; AUTO = BF16X3 steps
                          followed by one BF16X6 step                 [AUTO] */
    int polish;        /* 1: one extra step at BF16X6 after the stop (always
                          on for AUTO)                                    [0] */
    int literal_delta; /* 1: compare ||X' - X||_F without the sqrt(a) factor [0] */
    int reserved[4];
} la_inverse_opts;

typedef struct {
    int iters;          /* steps taken, polish included                       */
    int product_side;   /* 1: the step formed A X (n x n, n <= m);
                           0: it formed X A (m x m, n > m)                    */
    double gram_norm;   /* a = ||A A^T||_F, accumulated in FP64 on the GPU     */
    double last_delta;  /* the step norm last compared (FP64)                 */
    double last_tol;    /* the tolerance it was compared with                 */
    int stop_reason;    /* 0 tolerance, 2 iteration cap                       */
    int prec;           /* resolved precision                                 */
} la_inverse_info;

/* Bytes of device workspace la_inverse needs for an n x m A (0 on bad
 * arguments).  opts may be NULL. */
size_t la_inverse_workspace_size(int64_t n, int64_t m, const la_inverse_opts *opts);

/* A (n x m, lda >= m, n, m >= 1) is read only; X (m x n, ldx >= n) receives
 * the result and must not overlap A or the workspace.  workspace: device
 * memory of at least la_inverse_workspace_size() bytes, 256-byte aligned.
 * Runs on hip_stream and returns after the last kernel has completed (one
 * 8-byte readback per step).  LA_ERR_NONFINITE if a is 0, Inf or NaN or a
 * step norm is not finite; LA_ERR_NOT_CONVERGED if max_iter steps ran
 * without meeting the tolerance (X then holds the last iterate).  info may
 * be NULL. */
la_status la_inverse(la_context *ctx, int64_t n, int64_t m, const float *A, int64_t lda,
                     float *X, int64_t ldx, void *workspace, size_t ws_bytes,
                     const la_inverse_opts *opts, la_inverse_info *info, void *hip_stream);

/* ------------------------------------------------------------------------
 * Polynomial matrix functions (section III.D, eqs. MatFunc-OddPoly and
 * MatFuncEig-EigenvaluePolynomial).  coef is a HOST array of ncoef >= 1
 * finite doubles (rounded to FP32 where they enter a product's epilogue).
 * workspace: device memory of at least la_matfunc_workspace_size() bytes,
 * 256-byte aligned (three n x n FP32 buffers).  prec: AUTO = BF16X6 (the
 * recurrences accumulate the products' errors, so every product is kept at
 * FP32-level accuracy).  Both run on hip_stream and return after the last
 * kernel has completed.  F must not overlap A or the workspace.
 * ---------------------------------------------------------------------- */
size_t la_matfunc_workspace_size(int64_t m, int64_t n);

/* Odd polynomial of the singular values of an m x n A (lda >= n):
 *   F = sum_{j=0}^{ncoef-1} coef[j] A (A^T A)^j      (F m x n, ldf >= n),
 * i.e. f(A) = U_s f(S) V_s^T for f(x) = coef[0] x + coef[1] x^3 + ...
 * Evaluated as A p(A^T A) with Horner's rule in the Gram matrix: one
 * symmetric Gram launch, ncoef - 2 products of n x n matrices and a final
 * m x n product. */
la_status la_matfunc_odd(la_context *ctx, int64_t m, int64_t n, const float *A, int64_t lda,
                         const double *coef, int ncoef, float *F, int64_t ldf, void *workspace,
                         size_t ws_bytes, la_precision prec, void *hip_stream);

/* Chebyshev series of the eigenvalues of an n x n A (lda >= n) on
 * [lo, hi] (finite, lo < hi):
 *   F = sum_{k=0}^{ncoef-1} coef[k] T_k(B),  B = (2A - (lo + hi) I) / (hi - lo)
 * (coef[0] carries full weight; F n x n, ldf >= n).  Evaluated by
 * Clenshaw's recurrence: ncoef - 2 GEMM launches for ncoef >= 3.  The
 * series approximates g(A) when the eigenvalues of A lie in [lo, hi]; it is
 * computed for any A. */
la_status la_matfunc_cheb(la_context *ctx, int64_t n, const float *A, int64_t lda, double lo,
                          double hi, const double *coef, int ncoef, float *F, int64_t ldf,
                          void *workspace, size_t ws_bytes, la_precision prec,
                          void *hip_stream);

/* ------------------------------------------------------------------------
 * QR factorisation (section III.B): Algorithm tsqr, the WY form of
 * eq. (Yamamoto) and Algorithm caqr.  Matrices are FP32 row-major in device
 * memory; workspaces are device memory, 256-byte aligned, of at least the
 * size the matching *_workspace_size() returns (0 for a shape the call
 * rejects).  Each call runs on hip_stream and returns after its last kernel
 * has completed.  The local factorisations are Householder reflections in
 * FP32 with FP64 column norms; R_jj takes the sign opposite to the pivot
 * entry it replaces, so R's diagonal signs depend on the tree and may differ
 * from another QR of the same matrix (QR is unique up to those signs).
 * ---------------------------------------------------------------------- */

/* Algorithm tsqr: reduced QR of an m x n A (1 <= n <= 128, m >= n; lda,
 * ldq, ldr >= n): Q (m x n, orthonormal columns) and R (n x n, upper
 * triangular, zeros below the diagonal) with A = Q R.  The rows are split
 * into blocks of at most 256 rows, each factored in one workgroup; the
 * blocks' R factors are stacked and factored again until one remains, and
 * the Q factors are multiplied down the tree.  A, Q, R and the workspace
 * must not overlap. */
size_t la_tsqr_workspace_size(int64_t m, int64_t n);
la_status la_tsqr(la_context *ctx, int64_t m, int64_t n, const float *A, int64_t lda, float *Q,
                  int64_t ldq, float *R, int64_t ldr, void *workspace, size_t ws_bytes,
                  void *hip_stream);

/* eq. (Yamamoto): for a reduced Q (m x n, 1 <= n <= 128, m >= n), W = Q -
 * [I_n; 0] and Y = W (I - Q_1)^-1 with Q_1 the first n rows of Q, both
 * m x n, so that Q_f = I - W Y^T is orthogonal with Q_f [I_n; 0] = Q.  (The
 * equation's T^-1 = I - Q_1 is read as its transpose: only that makes the
 * first n columns of Q_f equal Q.)  The inverse is formed by Gauss-Jordan
 * elimination with partial pivoting in FP64.  LA_ERR_BREAKDOWN if a pivot
 * falls below 2^-16 in magnitude or is not finite (W and Y are then
 * unreliable): the breakdown the method has when Q_1 is close to a matrix
 * with eigenvalue 1.  Q, W, Y and the workspace must not overlap. */
size_t la_wy_workspace_size(int64_t n);
la_status la_wy(la_context *ctx, int64_t m, int64_t n, const float *Q, int64_t ldq, float *W,
                int64_t ldw, float *Y, int64_t ldy, void *workspace, size_t ws_bytes,
                void *hip_stream);

/* Algorithm caqr (right-looking): QR of an m x n A (m >= n, lda >= n) in
 * place, in panels of `panel` columns (1..128; the last panel takes the
 * remainder).  Each panel A_l: la_tsqr, la_wy, A_l <- [R; 0], and the
 * columns to its right A_r <- Q_f^T A_r = A_r - Y (W^T A_r) by two GEMM
 * launches of precision prec (AUTO = BF16X6: the second product's K is the
 * panel width, too short for BF16X3's per-term error of about 2^-16 to
 * average out to FP32 level).  On return the first n rows
 * of A hold R (upper triangle; zeros below) and the rows below are zero.  If
 * Q is not NULL (ldq >= n) it receives the reduced Q factor
 * Q_f(0) Q_f(1) ... [I_n; 0] (m x n), formed after the last panel by the
 * same two-launch update per panel in reverse order; the workspace then
 * also keeps every panel's W and Y (2 m n floats).  LA_ERR_BREAKDOWN as for
 * la_wy (A then holds a partial result).  A, Q and the workspace must not
 * overlap. */
size_t la_caqr_workspace_size(int64_t m, int64_t n, int panel, int want_q);
la_status la_caqr(la_context *ctx, int64_t m, int64_t n, float *A, int64_t lda, float *Q,
                  int64_t ldq, int panel, void *workspace, size_t ws_bytes, la_precision prec,
                  void *hip_stream);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of polar requests.
 * Requests are admitted while their device footprint fits the arena and a
 * slot is free; every tick advances all active requests of a size band by
 * one iteration with grouped launches (one Gram launch and one update launch
 * for all of them), so requests of different sizes and phases share the GPU.
 * The bands (small and large requests) tick independently on streams of
 * their own and share the arena and the slots.
 * ---------------------------------------------------------------------- */
typedef struct {
    int max_slots;     /* requests in flight at once                    [32]   */
    int max_queue;     /* requests waiting for admission                [4096] */
    int bands;         /* size bands ticking independently               [2]   */
                       /*   2: m n^2 <= 2048^3 and larger; 1: one band        */
    int reserved[5];
} la_serve_config;

typedef struct {
    uint64_t submitted, completed, failed, ticks;
    int active, queued;
    double busy_seconds;   /* host wall time with a band inside a tick     */
    size_t arena_high_water;
} la_serve_stats;

typedef struct la_server la_server;

/* arena: caller-owned device memory (256-byte aligned) the server carves
 * request state from (the first 8 MiB hold the bands' launch staging); it is
 * not freed by the library.  cfg may be NULL.  Starts one scheduler thread
 * per band, bound to ctx's device.  LA_ERR_INVALID_ARG for bands outside
 * 0..2. */
la_status la_serve_create(la_context *ctx, const la_serve_config *cfg,
                          void *arena, size_t arena_bytes, la_server **out);

/* Queue a polar of the m x n HOST matrix A_host (row-major, lda >= n).  A
 * is copied before the call returns.  LA_ERR_TOO_LARGE if the request could
 * never fit the arena; LA_ERR_QUEUE_FULL if the queue is at capacity.
 * opts may be NULL. *req_id receives a handle (unique per server). */
la_status la_serve_submit(la_server *srv, int64_t m, int64_t n,
                          const float *A_host, int64_t lda,
                          const la_polar_opts *opts, uint64_t *req_id);

/* Non-blocking.  LA_ERR_NOT_READY while the request is pending.  Once it is
 * done, copies U (m x n, row-major, contiguous) and, if H_host is not NULL,
 * H (n x n) to host memory, fills *info (nullable), stores the request's
 * own status in *req_status and forgets the request (a second poll returns
 * LA_ERR_UNKNOWN_REQUEST). */
la_status la_serve_poll(la_server *srv, uint64_t req_id, float *U_host,
                        float *H_host, la_polar_info *info,
                        la_status *req_status);

la_status la_serve_stats_get(la_server *srv, la_serve_stats *out);

/* Stops the scheduler (pending requests are cancelled) and frees host
 * state.  NULL is accepted. */
la_status la_serve_destroy(la_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* LA_H */
