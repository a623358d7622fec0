// gemm_tile.h -- LDS-tiled MFMA GEMM tile for gfx950 (CDNA4), included by
// the per-precision translation units gemm_fp32.hip / gemm_x3.hip /
// gemm_x6.hip.
//
// Computes one BM x BN output tile of out = alpha op(A) op(B) + beta E +
// gamma I, the matrix product of eq. (Matmul) (section III.A) with a fused
// epilogue for the polynomial updates of Algorithm NS_Polar (section III.D).
//
// Structure (one workgroup = 4 wave64s in a 2 x 2 grid, 128 x 128 per wave):
//   * global -> registers: each thread loads 8(k) x 4(row) blocks of FP32 as
//     float4s, for the next K stage, while the current stage computes;
//   * registers -> LDS: the FP32 values are split into bf16 terms
//     (hi/lo or hi/mid/lo, round to nearest even) and written in MFMA
//     fragment order: for every 32-row x 16-k block, 64 lane entries of
//     8 consecutive k, so each fragment read is one conflict-free 16-byte
//     ds_read per lane.  Transposed and non-transposed operands differ only
//     in the global load pattern; the LDS image is the same;
//   * LDS -> MFMA: v_mfma_f32_32x32x16_bf16 (3 or 6 products per operand
//     pair, smallest terms first) or v_mfma_f32_32x32x2_f32, FP32
//     accumulators;
//   * epilogue straight from the accumulators, with optional FP64 per-tile
//     sum of (out - E)^2 for the step norm.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "la_internal.h"

namespace la {
namespace dev {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// MI355X dispatches consecutive workgroups round-robin over its 8 XCDs.
constexpr int kXcds = 8;

// ---------------------------------------------------------------- configs

template <int PREC> struct Cfg;
template <> struct Cfg<PREC_FP32> {
    static constexpr int BM = 256, BN = 256, BK = 16, WM = 2, WN = 2;
    static constexpr int terms = 1, entry_bytes = 32;
};
template <> struct Cfg<PREC_BF16X3> {
    static constexpr int BM = 256, BN = 256, BK = 32, WM = 2, WN = 2;
    static constexpr int terms = 2, entry_bytes = 16;
};
template <> struct Cfg<PREC_BF16X6> {
    static constexpr int BM = 256, BN = 256, BK = 16, WM = 2, WN = 2;
    static constexpr int terms = 3, entry_bytes = 16;
};

template <int PREC> struct Geo {
    using C = Cfg<PREC>;
    static constexpr int NT = C::WM * C::WN * 64;
    static constexpr int TM = C::BM / C::WM, TN = C::BN / C::WN;
    static constexpr int FM = TM / 32, FN = TN / 32;
    static constexpr int KF = C::BK / 16;  // 16-k fragment blocks per stage
    static constexpr int a_bytes = C::terms * (C::BM / 32) * KF * 64 * C::entry_bytes;
    static constexpr int b_bytes = C::terms * (C::BN / 32) * KF * 64 * C::entry_bytes;
    static constexpr int stage_bytes = a_bytes + b_bytes;
};

// ---------------------------------------------------------------- splitting

__device__ __forceinline__ uint32_t pk_bf16(float a, float b)
{
    f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}
__device__ __forceinline__ float bf_lo(uint32_t p) { return __uint_as_float(p << 16); }
__device__ __forceinline__ float bf_hi(uint32_t p) { return __uint_as_float(p & 0xffff0000u); }
// Remainder x - t after taking the leading bf16 term t (exact in FP32).  A
// non-finite leading term keeps Inf/NaN in that term alone.
__device__ __forceinline__ float rest(float x, float t)
{
    return fabsf(t) <= 3.40282347e38f ? x - t : 0.0f;
}

// Split 8 FP32 values into the LDS terms of the precision.
template <int PREC> struct Split;
template <> struct Split<PREC_FP32> {
    __device__ __forceinline__ static void run(const float *v, u32x4 *o)
    {
        o[0] = u32x4{__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]),
                     __float_as_uint(v[3])};
        o[1] = u32x4{__float_as_uint(v[4]), __float_as_uint(v[5]), __float_as_uint(v[6]),
                     __float_as_uint(v[7])};
    }
};
template <> struct Split<PREC_BF16X3> {
    __device__ __forceinline__ static void run(const float *v, u32x4 *o)
    {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            uint32_t h = pk_bf16(v[2 * p], v[2 * p + 1]);
            float r0 = rest(v[2 * p], bf_lo(h));
            float r1 = rest(v[2 * p + 1], bf_hi(h));
            o[0][p] = h;
            o[1][p] = pk_bf16(r0, r1);
        }
    }
};
template <> struct Split<PREC_BF16X6> {
    __device__ __forceinline__ static void run(const float *v, u32x4 *o)
    {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            uint32_t h = pk_bf16(v[2 * p], v[2 * p + 1]);
            float r0 = rest(v[2 * p], bf_lo(h));
            float r1 = rest(v[2 * p + 1], bf_hi(h));
            uint32_t m = pk_bf16(r0, r1);
            float q0 = r0 - bf_lo(m);
            float q1 = r1 - bf_hi(m);
            o[0][p] = h;
            o[1][p] = m;
            o[2][p] = pk_bf16(q0, q1);
        }
    }
};

// ---------------------------------------------------------------- LDS layout

// Slot of lane entry `lane` inside a 64-entry fragment block; rotates each
// group of 8 slots so that both the fragment reads (8 consecutive lanes) and
// the split writes (rows 4 apart or k8 pairs) hit distinct 16-byte banks.
__device__ __forceinline__ int swz(int lane, int fk)
{
    return (lane & 56) | ((lane + (lane >> 3) + 2 * fk) & 7);
}

// Byte offset of the entry holding op(X)(row, 8*k8 .. 8*k8+7) of term `t`.
template <int ROWS, int KF, int EB>
__device__ __forceinline__ int entry_off(int t, int row, int k8)
{
    const int lane = (row & 31) | ((k8 & 1) << 5);
    const int fk = k8 >> 1;
    return (((t * (ROWS / 32) + (row >> 5)) * KF + fk) * 64 + swz(lane, fk)) * EB;
}

template <int ROWS, int KF, int EB>
__device__ __forceinline__ int frag_off(int t, int frow, int fk, int lane)
{
    return (((t * (ROWS / 32) + frow) * KF + fk) * 64 + swz(lane, fk)) * EB;
}

// ---------------------------------------------------------------- loader

// Loads one K stage of op(X) rows [r0, r0+ROWS) x k [k0, k0+BK) into
// registers.  KC: k is contiguous in memory (X[r * ld + k]); otherwise the
// row index is (X[k * ld + r]).  Work unit = 8 k x 4 rows (8 float4 loads).
template <int ROWS, int BK, int NT, bool KC>
struct Loader {
    static constexpr int UNITS = ROWS * BK / 32;
    static constexpr int UPT = (UNITS + NT - 1) / NT;
    float v[UPT][4][8];

    __device__ __forceinline__ static bool active(int uid) { return (UNITS % NT) == 0 || uid < UNITS; }

    // (row, k8) of entry q of unit uid
    __device__ __forceinline__ static int row_of(int uid, int q)
    {
        if constexpr (KC)
            return uid / (BK / 8) + q * (ROWS / 4);
        else
            return 4 * (uid % (ROWS / 4)) + q;
    }
    __device__ __forceinline__ static int k8_of(int uid)
    {
        if constexpr (KC)
            return uid % (BK / 8);
        else
            return uid / (ROWS / 4);
    }

    __device__ __forceinline__ void load(const float *__restrict__ X, int64_t ld, int64_t R,
                                         int64_t K, int64_t r0, int64_t k0, bool fast)
    {
        const int t = threadIdx.x;
#pragma unroll
        for (int u = 0; u < UPT; ++u) {
            const int uid = t + u * NT;
            if (!active(uid))
                continue;
            const int k8 = k8_of(uid);
            if constexpr (KC) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t gr = r0 + row_of(uid, q);
                    const int64_t gk = k0 + 8 * k8;
                    if (fast) {
                        const f32x4 *p = reinterpret_cast<const f32x4 *>(X + gr * ld + gk);
                        const f32x4 a = p[0], b = p[1];
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            v[u][q][j] = a[j];
                            v[u][q][4 + j] = b[j];
                        }
                    } else {
#pragma unroll
                        for (int j = 0; j < 8; ++j) {
                            float x = 0.0f;
                            if (gr < R && gk + j < K)
                                x = X[gr * ld + gk + j];
                            v[u][q][j] = x;
                        }
                    }
                }
            } else {
                const int64_t gr = r0 + row_of(uid, 0);
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int64_t gk = k0 + 8 * k8 + j;
                    if (fast) {
                        const f32x4 a = *reinterpret_cast<const f32x4 *>(X + gk * ld + gr);
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            v[u][q][j] = a[q];
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            float x = 0.0f;
                            if (gk < K && gr + q < R)
                                x = X[gk * ld + gr + q];
                            v[u][q][j] = x;
                        }
                    }
                }
            }
        }
    }

    template <int PREC>
    __device__ __forceinline__ void store(char *base) const
    {
        using C = Cfg<PREC>;
        constexpr int KF = BK / 16;
        const int t = threadIdx.x;
#pragma unroll
        for (int u = 0; u < UPT; ++u) {
            const int uid = t + u * NT;
            if (!active(uid))
                continue;
            const int k8 = k8_of(uid);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = row_of(uid, q);
                u32x4 parts[C::terms * (C::entry_bytes / 16)];
                Split<PREC>::run(v[u][q], parts);
                if constexpr (PREC == PREC_FP32) {
                    u32x4 *dst = reinterpret_cast<u32x4 *>(
                        base + entry_off<ROWS, KF, C::entry_bytes>(0, row, k8));
                    dst[0] = parts[0];
                    dst[1] = parts[1];
                } else {
#pragma unroll
                    for (int tt = 0; tt < C::terms; ++tt)
                        *reinterpret_cast<u32x4 *>(
                            base + entry_off<ROWS, KF, C::entry_bytes>(tt, row, k8)) = parts[tt];
                }
            }
        }
    }
};

// ---------------------------------------------------------------- MFMA stage

template <int PREC>
__device__ __forceinline__ void compute_stage(const char *sA, const char *sB,
                                              f32x16 (&acc)[Geo<PREC>::FM][Geo<PREC>::FN],
                                              int wm, int wn, int lane)
{
    using C = Cfg<PREC>;
    using G = Geo<PREC>;
    constexpr int FM = G::FM, FN = G::FN, KF = G::KF, EB = C::entry_bytes;
#pragma unroll
    for (int kk = 0; kk < KF; ++kk) {
        if constexpr (PREC == PREC_FP32) {
            f32x4 a[FM][2], b[FN][2];
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                const f32x4 *p = reinterpret_cast<const f32x4 *>(
                    sA + frag_off<C::BM, KF, EB>(0, wm * FM + i, kk, lane));
                a[i][0] = p[0];
                a[i][1] = p[1];
            }
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const f32x4 *p = reinterpret_cast<const f32x4 *>(
                    sB + frag_off<C::BN, KF, EB>(0, wn * FN + j, kk, lane));
                b[j][0] = p[0];
                b[j][1] = p[1];
            }
#pragma unroll
            for (int e = 0; e < 8; ++e)
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                            a[i][e >> 2][e & 3], b[j][e >> 2][e & 3], acc[i][j], 0, 0, 0);
        } else {
            constexpr int T = C::terms;
            bf16x8 a[FM][T], b[FN][T];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int t = 0; t < T; ++t)
                    a[i][t] = *reinterpret_cast<const bf16x8 *>(
                        sA + frag_off<C::BM, KF, EB>(t, wm * FM + i, kk, lane));
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int t = 0; t < T; ++t)
                    b[j][t] = *reinterpret_cast<const bf16x8 *>(
                        sB + frag_off<C::BN, KF, EB>(t, wn * FN + j, kk, lane));
            // products of split terms, smallest first
            constexpr int NP = (PREC == PREC_BF16X3) ? 3 : 6;
            constexpr int pa[6] = {(PREC == PREC_BF16X3) ? 1 : 2, 0, 1, 1, 0, 0};
            constexpr int pb[6] = {0, (PREC == PREC_BF16X3) ? 1 : 2, 1, 0, 1, 0};
            constexpr int pa3[3] = {1, 0, 0};
            constexpr int pb3[3] = {0, 1, 0};
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int ta = (PREC == PREC_BF16X3) ? pa3[p] : pa[p];
                const int tb = (PREC == PREC_BF16X3) ? pb3[p] : pb[p];
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            a[i][ta], b[j][tb], acc[i][j], 0, 0, 0);
            }
        }
    }
}

// ---------------------------------------------------------------- tiles

// XCD-aware remap of the hardware workgroup index to a logical tile index:
// each XCD receives one contiguous range of logical tiles, so neighbouring
// tiles (which share operand panels) share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int bid, int nb)
{
    const int x = bid % kXcds, i = bid / kXcds;
    const int q = nb / kXcds, r = nb % kXcds;
    return x * q + min(x, r) + i;
}

// Logical tile index -> (tile row, tile column).  General: groups of 8 tile
// rows, column-major inside a group.  Gram: upper-triangle tiles row by row.
__device__ __forceinline__ void tile_coords(const GemmDesc &d, int lin, int &tm, int &tn)
{
    if (d.gram) {
        int r = 0, rem = lin;
        while (rem >= d.tiles_n - r) {
            rem -= d.tiles_n - r;
            ++r;
        }
        tm = r;
        tn = r + rem;
    } else {
        constexpr int G = 8;
        const int per_group = G * d.tiles_n;
        const int g = lin / per_group;
        const int first = g * G;
        const int gs = min(G, d.tiles_m - first);
        const int in = lin - g * per_group;
        tm = first + in % gs;
        tn = in / gs;
    }
}

template <int PREC>
__device__ __forceinline__ void epilogue(const GemmDesc &d,
                                         f32x16 (&acc)[Geo<PREC>::FM][Geo<PREC>::FN],
                                         int tm, int tn, int wm, int wn, int lane,
                                         double *red)
{
    using G = Geo<PREC>;
    const int64_t rb = (int64_t)tm * Cfg<PREC>::BM + wm * G::TM + (lane >> 5) * 4;
    const int64_t cb = (int64_t)tn * Cfg<PREC>::BN + wn * G::TN + (lane & 31);
    double ss = 0.0;
    const bool want_ss = d.partials != nullptr;
#pragma clang loop unroll(full)
    for (int i = 0; i < G::FM; ++i)
#pragma clang loop unroll(full)
        for (int j = 0; j < G::FN; ++j)
#pragma clang loop unroll(full)
            for (int e = 0; e < 16; ++e) {
                const int64_t row = rb + i * 32 + (e >> 2) * 8 + (e & 3);
                const int64_t col = cb + j * 32;
                if (row >= d.M || col >= d.N || (d.gram && row > col))
                    continue;
                float val = d.alpha * acc[i][j][e];
                float ev = 0.0f;
                if (d.E) {
                    ev = d.E[row * d.lde + col];
                    val = val + d.beta * ev;
                }
                if (row == col)
                    val = val + d.gamma;
                d.C[row * d.ldc + col] = val;
                if (d.gram && row != col)
                    d.C[col * d.ldc + row] = val;
                if (want_ss) {
                    const double df = (double)val - (double)ev;
                    ss += df * df;
                }
            }
    if (want_ss) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
            ss += __shfl_xor(ss, off, 64);
        const int w = threadIdx.x >> 6;
        if (lane == 0)
            red[w] = ss;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int k = 0; k < Cfg<PREC>::WM * Cfg<PREC>::WN; ++k)
                s += red[k];
            d.partials[(int64_t)tm * d.tiles_n + tn] = s;
        }
    }
}

template <int PREC, bool AKC, bool BKC>
__device__ __forceinline__ void gemm_tile(const GemmDesc &d, int tm, int tn, char *smem,
                                          double *red)
{
    using C = Cfg<PREC>;
    using G = Geo<PREC>;
    constexpr int BK = C::BK;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w / C::WN, wn = w % C::WN;
    const int64_t row0 = (int64_t)tm * C::BM, col0 = (int64_t)tn * C::BN;

    f32x16 acc[G::FM][G::FN];
#pragma clang loop unroll(full)
    for (int i = 0; i < G::FM; ++i)
#pragma clang loop unroll(full)
        for (int j = 0; j < G::FN; ++j)
            acc[i][j] = f32x16{};

    Loader<C::BM, BK, G::NT, AKC> la;
    Loader<C::BN, BK, G::NT, BKC> lb;
    const int64_t nst = (d.K + BK - 1) / BK;
    const bool in_m = row0 + C::BM <= d.M, in_n = col0 + C::BN <= d.N;
    const bool va = d.vec_a && in_m, vb = d.vec_b && in_n;

    if (nst > 0) {
        const bool full0 = BK <= d.K;
        la.load(d.A, d.lda, d.M, d.K, row0, 0, va && full0);
        lb.load(d.B, d.ldb, d.N, d.K, col0, 0, vb && full0);
        la.template store<PREC>(smem);
        lb.template store<PREC>(smem + G::a_bytes);
        __syncthreads();
        for (int64_t s = 0; s < nst; ++s) {
            const int cur = (int)(s & 1);
            const bool more = s + 1 < nst;
            if (more) {
                const int64_t k0 = (s + 1) * BK;
                const bool full = k0 + BK <= d.K;
                la.load(d.A, d.lda, d.M, d.K, row0, k0, va && full);
                lb.load(d.B, d.ldb, d.N, d.K, col0, k0, vb && full);
            }
            char *sc = smem + cur * G::stage_bytes;        // stage being computed
            char *sn = smem + (cur ^ 1) * G::stage_bytes;  // stage being filled
            compute_stage<PREC>(sc, sc + G::a_bytes, acc, wm, wn, lane);
            if (more) {
                la.template store<PREC>(sn);
                lb.template store<PREC>(sn + G::a_bytes);
            }
            __syncthreads();
        }
    }
    epilogue<PREC>(d, acc, tm, tn, wm, wn, lane, red);
}

// ---------------------------------------------------------------- kernels

template <int PREC, bool AKC, bool BKC>
__global__ void __launch_bounds__(Geo<PREC>::NT, 1) gemm_kernel(GemmDesc d)
{
    __shared__ __attribute__((aligned(16))) char smem[2 * Geo<PREC>::stage_bytes];
    __shared__ double red[Cfg<PREC>::WM * Cfg<PREC>::WN];
    const int lin = xcd_remap(blockIdx.x, d.num_tiles);
    int tm, tn;
    tile_coords(d, lin, tm, tn);
    gemm_tile<PREC, AKC, BKC>(d, tm, tn, smem, red);
}

// Persistent grouped kernel: workgroup b runs items b, b + grid, ...; each
// item is one tile of one problem, computed exactly as gemm_kernel would.
template <int PREC, bool AKC, bool BKC>
__global__ void __launch_bounds__(Geo<PREC>::NT, 1)
    gemm_grouped_kernel(const GemmDesc *__restrict__ probs, const GroupItem *__restrict__ items,
                        int num_items)
{
    __shared__ __attribute__((aligned(16))) char smem[2 * Geo<PREC>::stage_bytes];
    __shared__ double red[Cfg<PREC>::WM * Cfg<PREC>::WN];
    for (int it = blockIdx.x; it < num_items; it += gridDim.x) {
        const GroupItem gi = items[it];
        const GemmDesc d = probs[gi.prob];
        int tm, tn;
        tile_coords(d, gi.tile, tm, tn);
        gemm_tile<PREC, AKC, BKC>(d, tm, tn, smem, red);
        __syncthreads();
    }
}

// ---------------------------------------------------------------- launchers

template <int PREC>
hipError_t launch_t(const GemmDesc &d, hipStream_t s)
{
    if (d.num_tiles <= 0)
        return hipSuccess;
    dim3 grid(d.num_tiles), block(Geo<PREC>::NT);
    if (d.a_kcontig && d.b_kcontig)
        hipLaunchKernelGGL((gemm_kernel<PREC, true, true>), grid, block, 0, s, d);
    else if (d.a_kcontig)
        hipLaunchKernelGGL((gemm_kernel<PREC, true, false>), grid, block, 0, s, d);
    else if (d.b_kcontig)
        hipLaunchKernelGGL((gemm_kernel<PREC, false, true>), grid, block, 0, s, d);
    else
        hipLaunchKernelGGL((gemm_kernel<PREC, false, false>), grid, block, 0, s, d);
    return hipGetLastError();
}

template <int PREC>
hipError_t launch_grouped_t(int akc, int bkc, const GemmDesc *probs, const GroupItem *items,
                            int num_items, int grid_size, hipStream_t s)
{
    if (num_items <= 0)
        return hipSuccess;
    dim3 grid(grid_size < num_items ? grid_size : num_items), block(Geo<PREC>::NT);
    if (akc && bkc)
        hipLaunchKernelGGL((gemm_grouped_kernel<PREC, true, true>), grid, block, 0, s, probs,
                           items, num_items);
    else if (akc)
        hipLaunchKernelGGL((gemm_grouped_kernel<PREC, true, false>), grid, block, 0, s, probs,
                           items, num_items);
    else if (bkc)
        hipLaunchKernelGGL((gemm_grouped_kernel<PREC, false, true>), grid, block, 0, s, probs,
                           items, num_items);
    else
        hipLaunchKernelGGL((gemm_grouped_kernel<PREC, false, false>), grid, block, 0, s, probs,
                           items, num_items);
    return hipGetLastError();
}

}  // namespace dev
}  // namespace la
