// Auxiliary kernels of the polar, inversion and matrix-function drivers: FP64
// norm reductions (the scaling ||A||_F and the step norm ||U' - U||_F of
// Algorithm NS_Polar, section III.D), scaling, transpose-scaling, the affine
// map s A + t I, copies, symmetrisation of H, split-K reduction, and the
// precision dispatch of the GEMM launchers.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "la_internal.h"

namespace la {

hipError_t launch_gemm_fp32(const GemmDesc &d, hipStream_t s);
hipError_t launch_gemm_x3(const GemmDesc &d, hipStream_t s);
hipError_t launch_gemm_x6(const GemmDesc &d, hipStream_t s);
hipError_t launch_grouped_fp32(int, int, int, const GemmDesc *, const GroupItem *, int, int,
                               hipStream_t);
hipError_t launch_grouped_x3(int, int, int, const GemmDesc *, const GroupItem *, int, int,
                             hipStream_t);
hipError_t launch_grouped_x6(int, int, int, const GemmDesc *, const GroupItem *, int, int,
                             hipStream_t);
int tile_m_fp32(int);
int tile_n_fp32(int);
int tile_m_x3(int);
int tile_n_x3(int);
int tile_m_x6(int);
int tile_n_x6(int);

int tile_m(int prec, int small)
{
    return prec == PREC_FP32 ? tile_m_fp32(small)
                             : prec == PREC_BF16X3 ? tile_m_x3(small) : tile_m_x6(small);
}
int tile_n(int prec, int small)
{
    return prec == PREC_FP32 ? tile_n_fp32(small)
                             : prec == PREC_BF16X3 ? tile_n_x3(small) : tile_n_x6(small);
}

static bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

void gemm_finalize(GemmDesc &d, int prec)
{
    // The interior loader keeps 32-bit element offsets of up to 255 rows (or 24
    // k rows) from a 64-bit stage base; an operand with a longer leading
    // dimension takes the guarded loader, which indexes in 64 bits.
    constexpr int64_t kMaxFastLd = (int64_t)1 << 23;
    d.vec_a = aligned16(d.A) && (d.lda % 4 == 0) && d.lda < kMaxFastLd;
    d.vec_b = aligned16(d.B) && (d.ldb % 4 == 0) && d.ldb < kMaxFastLd;
    // small tiles when large ones would leave most CUs idle
    {
        const int64_t lm = (d.M + tile_m(prec) - 1) / tile_m(prec);
        const int64_t ln = (d.N + tile_n(prec) - 1) / tile_n(prec);
        const int64_t large = d.gram ? ln * (ln + 1) / 2 : lm * ln;
        d.small = large < 128 ? 1 : 0;
    }
    gemm_set_class(d, prec, d.small);
}

void gemm_set_class(GemmDesc &d, int prec, int small)
{
    d.small = small;
    const int bm = tile_m(prec, d.small), bn = tile_n(prec, d.small);
    d.tiles_m = (int)((d.M + bm - 1) / bm);
    d.tiles_n = (int)((d.N + bn - 1) / bn);
    if (d.gram)
        d.num_tiles = d.tiles_n * (d.tiles_n + 1) / 2;
    else
        d.num_tiles = d.tiles_m * d.tiles_n;
    if (d.M == 0 || d.N == 0)
        d.num_tiles = 0;
}

hipError_t launch_gemm(int prec, const GemmDesc &d, hipStream_t s)
{
    switch (prec) {
    case PREC_FP32: return launch_gemm_fp32(d, s);
    case PREC_BF16X3: return launch_gemm_x3(d, s);
    case PREC_BF16X6: return launch_gemm_x6(d, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gemm_grouped(int prec, int akc, int bkc, int small, const GemmDesc *probs,
                               const GroupItem *items, int num_items, int grid_size,
                               hipStream_t s)
{
    switch (prec) {
    case PREC_FP32:
        return launch_grouped_fp32(akc, bkc, small, probs, items, num_items, grid_size, s);
    case PREC_BF16X3:
        return launch_grouped_x3(akc, bkc, small, probs, items, num_items, grid_size, s);
    case PREC_BF16X6:
        return launch_grouped_x6(akc, bkc, small, probs, items, num_items, grid_size, s);
    default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------ norms

namespace {

constexpr int kSumsqBlocks = 1024;
constexpr int kThreads = 256;

// Block-wide FP64 sum in a fixed order: wave64 butterfly, then wave 0.
__device__ double block_sum(double v, double *sh)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0)
        sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k)
            s += sh[k];
    return s;
}

// Block b sums the squares of rows b, b + grid, ... ; thread t takes columns
// t, t + 256, ...  Each square is formed and accumulated in FP64.
__global__ void __launch_bounds__(kThreads) sumsq_kernel(const float *__restrict__ X, int64_t m,
                                                         int64_t n, int64_t ld,
                                                         double *__restrict__ parts)
{
    __shared__ double sh[kThreads / 64];
    double acc = 0.0;
    for (int64_t r = blockIdx.x; r < m; r += gridDim.x) {
        const float *row = X + r * ld;
        for (int64_t c = threadIdx.x; c < n; c += kThreads) {
            const double x = (double)row[c];
            acc += x * x;
        }
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0)
        parts[blockIdx.x] = s;
}

// One block: thread t sums parts t, t + 256, ... in order; then block_sum.
__global__ void __launch_bounds__(kThreads) reduce_fixed_kernel(const double *__restrict__ parts,
                                                                int64_t count,
                                                                double *__restrict__ out)
{
    __shared__ double sh[kThreads / 64];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += kThreads)
        acc += parts[i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0)
        out[0] = s;
}

__global__ void __launch_bounds__(kThreads) reduce_grouped_kernel(const ReduceItem *__restrict__ items)
{
    __shared__ double sh[kThreads / 64];
    const ReduceItem it = items[blockIdx.x];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < it.count; i += kThreads)
        acc += it.parts[i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0)
        it.out[0] = s;
}

__global__ void scale_kernel(const float *__restrict__ X, int64_t ldx, float *__restrict__ Y,
                             int64_t ldy, int64_t m, int64_t n, double nrm)
{
    for (int64_t r = blockIdx.y; r < m; r += gridDim.y)
        for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n;
             c += (int64_t)gridDim.x * blockDim.x)
            Y[r * ldy + c] = (float)((double)X[r * ldx + c] / nrm);
}

// scale_kernel with nrm = sqrt(*nrm2) taken on the device (FP64, correctly
// rounded as on the host).
__global__ void scale_by_norm_kernel(const float *__restrict__ X, int64_t ldx,
                                     float *__restrict__ Y, int64_t ldy, int64_t m, int64_t n,
                                     const double *__restrict__ nrm2)
{
    const double nrm = sqrt(*nrm2);
    for (int64_t r = blockIdx.y; r < m; r += gridDim.y)
        for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n;
             c += (int64_t)gridDim.x * blockDim.x)
            Y[r * ldy + c] = (float)((double)X[r * ldx + c] / nrm);
}

// X = A^T / a for an n x m A (X is m x n): 32 x 32 tiles staged through LDS
// (padded rows) so that both the read of A and the write of X are coalesced.
// The division is done in FP64 and rounded once, as in scale_kernel.
__global__ void transpose_scale_kernel(const float *__restrict__ A, int64_t lda,
                                       float *__restrict__ X, int64_t ldx, int64_t n,
                                       int64_t m, double a)
{
    __shared__ float t[32][33];
    const int64_t tiles_m = (m + 31) / 32;
    for (int64_t bm = blockIdx.y; bm < tiles_m; bm += gridDim.y) {
        const int64_t i0 = (int64_t)blockIdx.x * 32;   // rows of A = columns of X
        const int64_t j0 = bm * 32;                     // columns of A = rows of X
        for (int r = threadIdx.y; r < 32; r += 8) {
            const int64_t i = i0 + r, j = j0 + threadIdx.x;
            t[r][threadIdx.x] = (i < n && j < m) ? A[i * lda + j] : 0.0f;
        }
        __syncthreads();
        for (int r = threadIdx.y; r < 32; r += 8) {
            const int64_t row = j0 + r, col = i0 + threadIdx.x;
            if (row < m && col < n)
                X[row * ldx + col] = (float)((double)t[threadIdx.x][r] / a);
        }
        __syncthreads();
    }
}

// Y = s A + t I for an n x n A, in FP64 per element, rounded once (A is not
// read when s == 0).
__global__ void affine_kernel(const float *__restrict__ A, int64_t lda, float *__restrict__ Y,
                              int64_t ldy, int64_t n, double sc, double t)
{
    for (int64_t r = blockIdx.y; r < n; r += gridDim.y)
        for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n;
             c += (int64_t)gridDim.x * blockDim.x)
            Y[r * ldy + c] =
                (float)((sc != 0.0 ? sc * (double)A[r * lda + c] : 0.0) + (r == c ? t : 0.0));
}

__global__ void copy_kernel(const float *__restrict__ X, int64_t ldx, float *__restrict__ Y,
                            int64_t ldy, int64_t m, int64_t n)
{
    for (int64_t r = blockIdx.y; r < m; r += gridDim.y)
        for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n;
             c += (int64_t)gridDim.x * blockDim.x)
            Y[r * ldy + c] = X[r * ldx + c];
}

// 32 x 32 blocks on or above the diagonal; each (i < j) pair is owned by one
// thread, so the in-place update is race free.
__global__ void symmetrize_kernel(float *H, int64_t ldh, int64_t n)
{
    const int64_t bi = blockIdx.y, bj = blockIdx.x;
    if (bj < bi)
        return;
    const int64_t i = bi * 32 + threadIdx.y, j = bj * 32 + threadIdx.x;
    if (i >= n || j >= n || j <= i)
        return;
    const float a = H[i * ldh + j], b = H[j * ldh + i];
    const float h = 0.5f * (a + b);
    H[i * ldh + j] = h;
    H[j * ldh + i] = h;
}

// Split-K sums of a symmetric product: the slices hold only their upper
// triangles (i <= j; what lies below is not read).  Block (bj, bi), bj >= bi,
// adds the 64 x 64 tile (bi, bj) of the slices in FP64 in slice order,
// applies the epilogue in FP64, rounds once, writes the tile and, through
// LDS, its transpose at (bj, bi), so out is exactly symmetric and both
// writes are coalesced.  VEC (n, ldo and the slice stride multiples of 4,
// 16-byte aligned bases): each thread moves 4 x 4 elements as float4 rows.
constexpr int kSymTile = 64;

template <bool VEC>
__global__ void __launch_bounds__(256) splitk_sym_reduce_kernel(
    const float *__restrict__ parts, int64_t stride, int splits, int64_t n, double alpha,
    double gamma, float *__restrict__ out, int64_t ldo)
{
    const int64_t bi = blockIdx.y, bj = blockIdx.x;
    if (bj < bi)
        return;
    __shared__ float t[kSymTile][kSymTile + 1];
    const bool diag = bi == bj;
    if constexpr (VEC) {
        const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;   // float4 column, row phase
        const int64_t j0 = bj * kSymTile + 4 * tx;
        for (int r = ty; r < kSymTile; r += 16) {
            const int64_t i = bi * kSymTile + r;
            if (i >= n || j0 >= n)
                continue;
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            for (int sl = 0; sl < splits; ++sl) {
                const float4 v =
                    *reinterpret_cast<const float4 *>(parts + sl * stride + i * n + j0);
                acc[0] += (double)v.x;
                acc[1] += (double)v.y;
                acc[2] += (double)v.z;
                acc[3] += (double)v.w;
            }
            float f[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                double v = alpha * acc[q];
                if (i == j0 + q)
                    v += gamma;
                f[q] = (float)v;
                t[r][4 * tx + q] = f[q];
            }
            if (!diag) {
                *reinterpret_cast<float4 *>(out + i * ldo + j0) = make_float4(f[0], f[1], f[2], f[3]);
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (i <= j0 + q)
                        out[i * ldo + j0 + q] = f[q];
            }
        }
        __syncthreads();
        // out(j, i) for i < j: row j of the (bj, bi) tile, columns i0 .. i0 + 3
        const int64_t i0 = bi * kSymTile + 4 * tx;
        for (int r = ty; r < kSymTile; r += 16) {
            const int64_t j = bj * kSymTile + r;
            if (j >= n || i0 >= n)
                continue;
            float f[4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                f[q] = t[4 * tx + q][r];
            if (!diag) {
                *reinterpret_cast<float4 *>(out + j * ldo + i0) = make_float4(f[0], f[1], f[2], f[3]);
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (i0 + q < j)
                        out[j * ldo + i0 + q] = f[q];
            }
        }
    } else {
        const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
        for (int r = ty; r < kSymTile; r += 4) {
            const int64_t i = bi * kSymTile + r, j = bj * kSymTile + tx;
            if (i < n && j < n && i <= j) {
                double acc = 0.0;
                for (int sl = 0; sl < splits; ++sl)
                    acc += (double)parts[sl * stride + i * n + j];
                double v = alpha * acc;
                if (i == j)
                    v += gamma;
                const float f = (float)v;
                out[i * ldo + j] = f;
                t[r][tx] = f;
            }
        }
        __syncthreads();
        for (int r = ty; r < kSymTile; r += 4) {
            const int64_t j = bj * kSymTile + r, i = bi * kSymTile + tx;   // out(j, i), i < j
            if (i < n && j < n && i < j)
                out[j * ldo + i] = t[tx][r];
        }
    }
}

// out = alpha sum_s part_s + beta E for an m x n product whose slices are
// m x n row-major (ld n), with the FP64 partial sum of (out - E)^2 of block b
// in step[b] (step may be null).  Every thread visits its elements in a fixed
// order and the block sum is a fixed tree, so the partials are reproducible.
// VEC (n, lde, ldo multiples of 4, 16-byte aligned bases): four consecutive
// columns per thread and step, as float4 loads and stores.
template <bool VEC>
__global__ void __launch_bounds__(kThreads) splitk_update_reduce_kernel(
    const float *__restrict__ parts, int splits, int64_t m, int64_t n, double alpha, double beta,
    const float *__restrict__ E, int64_t lde, float *__restrict__ out, int64_t ldo,
    double *__restrict__ step)
{
    __shared__ double sh[kThreads / 64];
    const int64_t mn = m * n;
    double ss = 0.0;
    if constexpr (VEC) {
        for (int64_t r = blockIdx.x; r < m; r += gridDim.x)
            for (int64_t c = 4 * (int64_t)threadIdx.x; c < n; c += 4 * kThreads) {
                double acc[4] = {0.0, 0.0, 0.0, 0.0};
                for (int sl = 0; sl < splits; ++sl) {
                    const float4 v = *reinterpret_cast<const float4 *>(parts + sl * mn + r * n + c);
                    acc[0] += (double)v.x;
                    acc[1] += (double)v.y;
                    acc[2] += (double)v.z;
                    acc[3] += (double)v.w;
                }
                float4 e = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (E)
                    e = *reinterpret_cast<const float4 *>(E + r * lde + c);
                const double ev[4] = {(double)e.x, (double)e.y, (double)e.z, (double)e.w};
                float o[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    o[q] = (float)(alpha * acc[q] + beta * ev[q]);
                    const double df = (double)o[q] - ev[q];
                    ss += df * df;
                }
                *reinterpret_cast<float4 *>(out + r * ldo + c) = make_float4(o[0], o[1], o[2], o[3]);
            }
    } else {
        for (int64_t r = blockIdx.x; r < m; r += gridDim.x)
            for (int64_t c = threadIdx.x; c < n; c += kThreads) {
                double acc = 0.0;
                for (int sl = 0; sl < splits; ++sl)
                    acc += (double)parts[sl * mn + r * n + c];
                const double e = E ? (double)E[r * lde + c] : 0.0;
                const float v = (float)(alpha * acc + beta * e);
                out[r * ldo + c] = v;
                const double df = (double)v - e;
                ss += df * df;
            }
    }
    if (step) {
        const double t = block_sum(ss, sh);
        if (threadIdx.x == 0)
            step[blockIdx.x] = t;
    }
}

dim3 grid2d(int64_t m, int64_t n)
{
    int64_t gx = (n + kThreads - 1) / kThreads;
    if (gx > 64)
        gx = 64;
    int64_t gy = m < 4096 ? m : 4096;
    if (gx < 1) gx = 1;
    if (gy < 1) gy = 1;
    return dim3((unsigned)gx, (unsigned)gy);
}

}  // namespace

int sumsq_num_partials() { return kSumsqBlocks; }

hipError_t launch_sumsq(const float *X, int64_t m, int64_t n, int64_t ld, double *partials,
                        hipStream_t s)
{
    hipLaunchKernelGGL(sumsq_kernel, dim3(kSumsqBlocks), dim3(kThreads), 0, s, X, m, n, ld,
                       partials);
    return hipGetLastError();
}

hipError_t launch_reduce_fixed(const double *parts, int64_t count, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_fixed_kernel, dim3(1), dim3(kThreads), 0, s, parts, count, out);
    return hipGetLastError();
}

hipError_t launch_reduce_grouped(const ReduceItem *items, int n, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(reduce_grouped_kernel, dim3(n), dim3(kThreads), 0, s, items);
    return hipGetLastError();
}

hipError_t launch_scale(const float *X, int64_t ldx, float *Y, int64_t ldy, int64_t m, int64_t n,
                        double nrm, hipStream_t s)
{
    if (m == 0 || n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(scale_kernel, grid2d(m, n), dim3(kThreads), 0, s, X, ldx, Y, ldy, m, n,
                       nrm);
    return hipGetLastError();
}

hipError_t launch_scale_by_norm(const float *X, int64_t ldx, float *Y, int64_t ldy, int64_t m,
                                int64_t n, const double *nrm2, hipStream_t s)
{
    if (m == 0 || n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(scale_by_norm_kernel, grid2d(m, n), dim3(kThreads), 0, s, X, ldx, Y, ldy,
                       m, n, nrm2);
    return hipGetLastError();
}

hipError_t launch_transpose_scale(const float *A, int64_t lda, float *X, int64_t ldx, int64_t n,
                                  int64_t m, double a, hipStream_t s)
{
    if (m == 0 || n == 0)
        return hipSuccess;
    const int64_t tn = (n + 31) / 32, tm = (m + 31) / 32;
    if (tn > 0x7fffffff)
        return hipErrorInvalidValue;
    const unsigned gy = (unsigned)std::min<int64_t>(tm, 65535);
    hipLaunchKernelGGL(transpose_scale_kernel, dim3((unsigned)tn, gy), dim3(32, 8), 0, s, A, lda,
                       X, ldx, n, m, a);
    return hipGetLastError();
}

hipError_t launch_affine(const float *A, int64_t lda, float *Y, int64_t ldy, int64_t n,
                         double sc, double t, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(affine_kernel, grid2d(n, n), dim3(kThreads), 0, s, A, lda, Y, ldy, n, sc,
                       t);
    return hipGetLastError();
}

hipError_t launch_copy(const float *X, int64_t ldx, float *Y, int64_t ldy, int64_t m, int64_t n,
                       hipStream_t s)
{
    if (m == 0 || n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(copy_kernel, grid2d(m, n), dim3(kThreads), 0, s, X, ldx, Y, ldy, m, n);
    return hipGetLastError();
}

hipError_t launch_symmetrize(float *H, int64_t ldh, int64_t n, hipStream_t s)
{
    if (n <= 1)
        return hipSuccess;
    const int64_t nb = (n + 31) / 32;
    hipLaunchKernelGGL(symmetrize_kernel, dim3((unsigned)nb, (unsigned)nb), dim3(32, 32), 0, s,
                       H, ldh, n);
    return hipGetLastError();
}

int splitk_update_num_partials() { return kSumsqBlocks; }

hipError_t launch_splitk_update_reduce(const float *parts, int splits, int64_t m, int64_t n,
                                       double alpha, double beta, const float *E, int64_t lde,
                                       float *out, int64_t ldo, double *step, hipStream_t s)
{
    if (m == 0 || n == 0)
        return hipSuccess;
    const bool vec = n % 4 == 0 && aligned16(parts) && aligned16(out) && ldo % 4 == 0 &&
                     (!E || (aligned16(E) && lde % 4 == 0));
    if (vec)
        hipLaunchKernelGGL(splitk_update_reduce_kernel<true>, dim3(kSumsqBlocks), dim3(kThreads),
                           0, s, parts, splits, m, n, alpha, beta, E, lde, out, ldo, step);
    else
        hipLaunchKernelGGL(splitk_update_reduce_kernel<false>, dim3(kSumsqBlocks), dim3(kThreads),
                           0, s, parts, splits, m, n, alpha, beta, E, lde, out, ldo, step);
    return hipGetLastError();
}

hipError_t launch_splitk_sym_reduce(const float *parts, int64_t stride, int splits, int64_t n,
                                    double alpha, double gamma, float *out, int64_t ldo,
                                    hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    const int64_t nb = (n + kSymTile - 1) / kSymTile;
    if (nb > 65535)
        return hipErrorInvalidValue;
    const bool vec = n % 4 == 0 && stride % 4 == 0 && ldo % 4 == 0 && aligned16(parts) &&
                     aligned16(out);
    if (vec)
        hipLaunchKernelGGL(splitk_sym_reduce_kernel<true>, dim3((unsigned)nb, (unsigned)nb),
                           dim3(256), 0, s, parts, stride, splits, n, alpha, gamma, out, ldo);
    else
        hipLaunchKernelGGL(splitk_sym_reduce_kernel<false>, dim3((unsigned)nb, (unsigned)nb),
                           dim3(256), 0, s, parts, stride, splits, n, alpha, gamma, out, ldo);
    return hipGetLastError();
}

}  // namespace la
