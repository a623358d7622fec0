// Internal declarations shared by the host-side translation units of the
// library (launchers, polar driver, server).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/la.h"
#include "polar_host.h"

struct la_context {
    int device;
    int num_cus;
    void *scratch;   // this device's static polar workspace (la_polar_noalloc)
};

namespace la {

// One GEMM-shaped launch: out = alpha * op(A) op(B) + beta * E + gamma * I.
//   op(A) (M x K): a_kcontig ? A[i * lda + k] : A[k * lda + i]
//   op(B) (K x N): b_kcontig ? B[j * ldb + k] : B[k * ldb + j]
//   out  (M x N): C[i * ldc + j]
//   E: optional addend (may equal C for beta * C), E[i * lde + j]
//   gram: output is symmetric (M == N): only tiles on or above the diagonal
//         are computed; element (i, j), i <= j, is written to (i, j) and
//         (j, i), so the result is exactly symmetric.
//   partials: optional, one FP64 per output tile: sum over the tile of
//         (out - E)^2, for the step norm ||X' - X||_F; requires E.
struct GemmDesc {
    const float *A;
    const float *B;
    float *C;
    const float *E;
    double *partials;
    int64_t lda, ldb, ldc, lde;
    int64_t M, N, K;
    float alpha, beta, gamma;
    int a_kcontig, b_kcontig;
    int gram;
    int gram_upper;    // gram: write only the upper triangle (no mirror)
    int vec_a, vec_b;  // operand addresses allow 16-byte vector loads
    int tiles_m, tiles_n;
    int num_tiles;     // tiles launched (upper triangle only for gram)
    int small;         // 128 x 128 tiles (chosen from the problem's own shape)
    int quarters;      // small tiles covering large Gram tiles tail_first.. (4 per tile)
    int tail_first;
    // split-K slices in one launch: slice y takes k in [y slice_k, min(K,
    // (y + 1) slice_k)) and writes C + y slice_stride (slice_k a multiple of
    // 32, so every slice but the last is whole K stages)
    int slices;
    int64_t slice_k, slice_stride;
};

// Tile geometry of each precision and tile class.  Both tile classes use the
// same K stages and product order, so the choice (made from the problem's own
// shape only) never changes a result.
int tile_m(int prec, int small = 0);
int tile_n(int prec, int small = 0);

// Fills the derived fields (tile class, vec flags, tile counts) of d.
void gemm_finalize(GemmDesc &d, int prec);
// Sets d's tile class (small: 128 x 128, else the precision's large tiles)
// and the tile counts that follow from it; the products are the same either way.
void gemm_set_class(GemmDesc &d, int prec, int small);

hipError_t launch_gemm(int prec, const GemmDesc &d, hipStream_t s);

// MI355X dispatches consecutive workgroups round-robin over its 8 XCDs.
constexpr int kXcds = 8;

// Grouped launch: every item is one output tile of one problem; all problems
// share precision and operand layouts.  probs / items live in device memory.
// grid_size > 0: that many persistent workgroups per CU-occupancy slot at
// most (the items loop over them, leaving CUs to other streams); 0: one
// workgroup per item, item b on workgroup b, hence on XCD b % kXcds.  The
// results are the same bits either way.  An item with prob < 0 is empty
// (padding of a list laid out for the XCDs).
struct GroupItem {
    int prob;
    int tile;   // linear tile index within the problem
};
hipError_t launch_gemm_grouped(int prec, int a_kcontig, int b_kcontig, int small,
                               const GemmDesc *probs_dev,
                               const GroupItem *items_dev, int num_items,
                               int grid_size, hipStream_t s);

// Packed 3xBF16 operands (gemm_x3.hip): op(X) (rows x k; kc: k contiguous,
// X[r * ld + k], else X[k * ld + r]) split into bf16 hi/lo terms and laid out
// in the GEMM's LDS fragment order, zero-padded to 256 rows and 16 k.
size_t packed_x3_bytes(int64_t rows, int64_t k);
hipError_t launch_pack_x3(const float *X, int64_t ld, int kc, int64_t rows, int64_t k, void *out,
                          hipStream_t s);
// GEMM on packed operands: d.A and d.B point at packed op(A) (M x K) and
// packed op(B)^T (N x K); 256 x 256 tiles (d.small must be 0).  Computes the
// same products in the same order as the 3xBF16 kernel of launch_gemm.
hipError_t launch_gemm_packed_x3(const GemmDesc &d, hipStream_t s);

// C (rows x cols, ldc) <- C - Y Z with Y (rows x K, k contiguous, ldy) and
// Z (K x cols, ldz), K <= 128 (qr_update.hip): the short-K update of
// Algorithm caqr, every element as launch_gemm computes alpha Y Z + beta C
// with alpha = -1, beta = 1 on the 128 x 128 tile class.
hipError_t launch_short_update(int prec, const float *Y, int64_t ldy, const float *Z, int64_t ldz,
                               float *C, int64_t ldc, int64_t rows, int64_t cols, int K,
                               hipStream_t s);

// Auxiliary kernels (aux_kernels.hip).
// Sum of squares of an m x n strided matrix into nparts FP64 partials.
int sumsq_num_partials();
hipError_t launch_sumsq(const float *X, int64_t m, int64_t n, int64_t ld,
                        double *partials, hipStream_t s);
// out[0] = sum of parts[0..count) in a fixed order (deterministic).
hipError_t launch_reduce_fixed(const double *parts, int64_t count, double *out,
                               hipStream_t s);
// Y = X / nrm, element-wise in FP64 then rounded to FP32 (so scaling A by a
// power of two leaves Y bitwise unchanged).
hipError_t launch_scale(const float *X, int64_t ldx, float *Y, int64_t ldy,
                        int64_t m, int64_t n, double nrm, hipStream_t s);
// The same with nrm = sqrt(*nrm2) read on the device (no host round trip).
hipError_t launch_scale_by_norm(const float *X, int64_t ldx, float *Y, int64_t ldy,
                                int64_t m, int64_t n, const double *nrm2, hipStream_t s);
// X = A^T / a (FP64 division, rounded once); A is n x m, X is m x n.
hipError_t launch_transpose_scale(const float *A, int64_t lda, float *X, int64_t ldx,
                                  int64_t n, int64_t m, double a, hipStream_t s);
// Y = s A + t I for an n x n A (FP64 per element, rounded once).
hipError_t launch_affine(const float *A, int64_t lda, float *Y, int64_t ldy, int64_t n,
                         double sc, double t, hipStream_t s);
// Y = X (strided copy).
hipError_t launch_copy(const float *X, int64_t ldx, float *Y, int64_t ldy,
                       int64_t m, int64_t n, hipStream_t s);
// In place H <- (H + H^T) / 2 for an n x n matrix.
hipError_t launch_symmetrize(float *H, int64_t ldh, int64_t n, hipStream_t s);
// Split-K reduction for a symmetric (gram) output: out(i, j) =
// alpha * sum_s part_s(i, j) + gamma * [i == j], summed over s in order in
// FP64 and rounded once; parts are `splits` exactly symmetric n x n slices
// (row-major, ld n).
// Slice s is at parts + s * stride (elements; any distance within one
// allocation).
hipError_t launch_splitk_sym_reduce(const float *parts, int64_t stride, int splits, int64_t n,
                                    double alpha, double gamma, float *out,
                                    int64_t ldo, hipStream_t s);
// Split-K reduction of an m x n product: out = alpha * sum_s part_s + beta * E
// (FP64, rounded once; E may be null), parts m x n row-major (ld n).  If step
// is not null, FP64 partial sums of (out - E)^2 go to
// step[0 .. splitk_update_num_partials()).
int splitk_update_num_partials();
hipError_t launch_splitk_update_reduce(const float *parts, int splits, int64_t m, int64_t n,
                                       double alpha, double beta, const float *E, int64_t lde,
                                       float *out, int64_t ldo, double *step, hipStream_t s);

// Grouped fixed-order FP64 reduction: one workgroup per item,
// out[0] = sum of parts[0..count) (same order as launch_reduce_fixed).
struct ReduceItem {
    const double *parts;
    int64_t count;
    double *out;
};
hipError_t launch_reduce_grouped(const ReduceItem *items_dev, int n, hipStream_t s);

// Polar building blocks shared by la_polar and the server (PolarPlan,
// polar_plan and the stop test are in polar_host.h).
// Number of split-K slices the Gram of an m x n iterate uses, and the number
// needed to keep an inner dimension K within the FP32 accumulation depth.
int gram_splits(int64_t m, int64_t n, int prec, int64_t max_acc);
int acc_splits(int64_t K, int64_t max_acc);
size_t polar_workspace_bytes(const PolarPlan &p);


// Argument helpers shared by the ABI entry points (la_api.hip).
la_status dev_fail(hipError_t e, const char *where);   // sets the error, LA_ERR_DEVICE
bool overlaps(const void *a, size_t abytes, const void *b, size_t bbytes);
size_t extent_bytes(int64_t rows, int64_t cols, int64_t ld);   // bytes spanned by a matrix
int resolve_prec(int p, int dflt);                      // AUTO -> dflt
bool valid_prec(int p);
size_t align_up256(size_t x);

#define LA_HIP(call, where)                        \
    do {                                           \
        hipError_t e_ = (call);                    \
        if (e_ != hipSuccess)                      \
            return ::la::dev_fail(e_, where);      \
    } while (0)

}  // namespace la
