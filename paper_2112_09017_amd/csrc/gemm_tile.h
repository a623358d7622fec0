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

#include <atomic>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "la_internal.h"

namespace la {
namespace dev {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// s_waitcnt immediate (gfx9 encoding) that waits for vmcnt == 0 only:
// vmcnt bits [3:0] and [15:14] zero, expcnt [6:4] and lgkmcnt [11:8] at their
// maxima (no wait).
constexpr int kWaitVmcnt0 = (7 << 4) | (15 << 8);

// ---------------------------------------------------------------- configs

// A kernel's PREC template argument is the arithmetic (PREC_FP32 / _BF16X3 /
// _BF16X6) plus kSmall for the 128 x 128 tile variant.
constexpr int kSmall = 16;
constexpr int base_prec(int P) { return P & 15; }

template <int PREC> struct Cfg;
// PIPE 1: one register stage, BK = 32, the next stage's split/stores run in
// the second 16-k half of the current stage.  PIPE 2: two register stages,
// BK = 16, the split of stage s+1 runs under the MFMAs of stage s.
template <> struct Cfg<PREC_FP32> {
    static constexpr int BM = 256, BN = 256, BK = 32, WM = 2, WN = 2, OCC = 1, PIPE = 1, GOCC = 1;
    static constexpr int terms = 1, entry_bytes = 32;
};
template <> struct Cfg<PREC_BF16X3> {
    static constexpr int BM = 256, BN = 256, BK = 32, WM = 2, WN = 2, OCC = 1, PIPE = 1, GOCC = 1;
    static constexpr int terms = 2, entry_bytes = 16;
};
template <> struct Cfg<PREC_BF16X6> {
    static constexpr int BM = 256, BN = 256, BK = 16, WM = 2, WN = 2, OCC = 1, PIPE = 2, GOCC = 1;
    static constexpr int terms = 3, entry_bytes = 16;
};
// 128 x 128 tiles (64 x 64 per wave), two workgroups per CU: problems too
// small to give every CU a 256 x 256 tile.  Same BK and product order as the
// large tiles, so every output element is computed identically.
template <> struct Cfg<PREC_FP32 | kSmall> {
    static constexpr int BM = 128, BN = 128, BK = 32, WM = 2, WN = 2, OCC = 2, PIPE = 1, GOCC = 2;
    static constexpr int terms = 1, entry_bytes = 32;
};
template <> struct Cfg<PREC_BF16X3 | kSmall> {
    static constexpr int BM = 128, BN = 128, BK = 32, WM = 2, WN = 2, OCC = 2, PIPE = 1, GOCC = 2;
    static constexpr int terms = 2, entry_bytes = 16;
};
template <> struct Cfg<PREC_BF16X6 | kSmall> {
    // two register stages of three terms fit within the 256 registers of two
    // workgroups per CU (at most 212 used), so one workgroup's loads and split
    // overlap the other's MFMAs; the grouped kernel (one register stage) runs two
    // per CU too
    static constexpr int BM = 128, BN = 128, BK = 16, WM = 2, WN = 2, OCC = 2, PIPE = 2, GOCC = 2;
    static constexpr int terms = 3, entry_bytes = 16;
};

// Packed 3xBF16 operands (kPacked): the operands were split into bf16 terms
// and laid out in the LDS fragment order by a pack pass, so the K loop moves
// them with direct global -> LDS loads; one 16-k block per stage, four LDS
// stages in flight.
constexpr int kPacked = 32;
constexpr int kPackStages = 4;
template <> struct Cfg<PREC_BF16X3 | kPacked> {
    static constexpr int BM = 256, BN = 256, BK = 16, WM = 2, WN = 2, OCC = 1, PIPE = 0, GOCC = 1;
    static constexpr int terms = 2, entry_bytes = 16;
};

// Workgroups per CU a kernel is compiled for: the tile class's OCC, except
// that the small 6xBF16 tile with both operands k-major (its loader keeps a
// 64-bit address per row it loads) would spill at two and keeps one.
template <int PREC, bool AKC, bool BKC>
constexpr int kernel_occ()
{
    return (PREC == (PREC_BF16X6 | kSmall) && !AKC && !BKC) ? 1 : Cfg<PREC>::OCC;
}

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
// Remainder x - t after taking the leading bf16 term t; exact in FP32 for
// finite x.  (A non-finite x leaves a NaN remainder, so non-finite inputs
// give non-finite, possibly NaN, outputs.)
__device__ __forceinline__ float rest(float x, float t) { return x - t; }

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

// Slot of lane entry `lane` inside a 64-entry fragment block.  Measured on
// gfx950: 16-byte-per-lane LDS accesses are conflict free when the 16 lanes
// of each group of consecutive lanes touch 16 distinct slots modulo 16 and the
// lane-to-slot map is the same shift for every group; the identity map gives
// conflict-free fragment reads, and the loaders below assign rows so that
// their writes also hit 16 consecutive slots.
__device__ __forceinline__ int swz(int lane, int fk) { return lane; }

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

// p as a pointer to global (device) memory.  Operands and outputs are read and
// written through such pointers, so the accesses are global instructions even
// where the compiler cannot see that a pointer is global (a descriptor the
// grouped kernels read from memory): flat accesses would also count against
// the LDS counter, and every wait for a stage's LDS reads would then wait for
// the next stage's operand loads in flight as well.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gmem(T *p)
{
    return (__attribute__((address_space(1))) T *)p;
}
typedef const __attribute__((address_space(1))) f32x4 gf32x4;
typedef const __attribute__((address_space(1))) f32x2 gf32x2;

// Loads one K stage of op(X) rows [r0, r0+ROWS) x k [k0, k0+BK) into
// registers.  KC: k is contiguous in memory (X[r * ld + k]); otherwise the
// row index is (X[k * ld + r]).  Work unit = 8 k x R rows: R float4 pairs
// (KC) or 8 float-R vectors (row-contiguous), R = 4 or 2 so that every
// thread has work.  Interior stages use load_fast (no bounds checks, loop-
// invariant 32-bit offsets from a uniform stage base); edge tiles and the K
// tail use load_guarded.
template <int ROWS, int BK, int NT, bool KC>
struct Loader {
    // up to 4 rows per unit, fewer when the stage is too small to give every
    // thread 4; the row map below keeps 16 consecutive lanes writing 16
    // consecutive fragment slots
    static constexpr int R = (ROWS * BK / (8 * NT) >= 4) ? 4 : (ROWS * BK / (8 * NT) >= 2) ? 2 : 1;
    static constexpr int NK8 = BK / 8;
    static constexpr int UNITS = ROWS * BK / (8 * R);
    static constexpr int UPT = (UNITS + NT - 1) / NT;
    static_assert(UNITS % NT == 0, "every thread must own whole units");
    float v[UPT][R][8];
    int off[UPT];  // element offset of the unit's first element from the stage base

    // (row, k8) of entry q of unit uid.  KC: within each 16 consecutive units
    // the row advances and k8 is fixed; k8 changes every 16 units, so a load
    // instruction still covers whole 128-byte row segments.
    __device__ __forceinline__ static int row_of(int uid, int q)
    {
        if constexpr (KC)
            return (uid % 16) + 16 * (uid / (16 * NK8)) + q * (ROWS / R);
        else
            return R * (uid % (ROWS / R)) + q;
    }
    __device__ __forceinline__ static int k8_of(int uid)
    {
        if constexpr (KC)
            return (uid / 16) % NK8;
        else
            return uid / (ROWS / R);
    }

    __device__ __forceinline__ void init(int64_t ld)
    {
#pragma unroll
        for (int u = 0; u < UPT; ++u) {
            const int uid = threadIdx.x + u * NT;
            const int row = row_of(uid, 0), k8 = k8_of(uid);
            off[u] = KC ? (int)(row * ld + 8 * k8) : (int)(8 * k8 * ld + row);
        }
    }

    // base = &op(X)(r0, k0) (uniform), stage fully in bounds, 16-byte aligned.
    __device__ __forceinline__ void load_fast(const float *__restrict__ base, int64_t ld)
    {
#pragma unroll
        for (int u = 0; u < UPT; ++u) {
            if constexpr (KC) {
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    gf32x4 *p = reinterpret_cast<gf32x4 *>(
                        gmem(base) + off[u] + (int64_t)q * (ROWS / R) * ld);
                    const f32x4 a = p[0], b = p[1];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        v[u][q][j] = a[j];
                        v[u][q][4 + j] = b[j];
                    }
                }
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const auto p = gmem(base) + off[u] + (int64_t)j * ld;
                    if constexpr (R == 4) {
                        const f32x4 a = *reinterpret_cast<gf32x4 *>(p);
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            v[u][q][j] = a[q];
                    } else if constexpr (R == 2) {
                        const f32x2 a = *reinterpret_cast<gf32x2 *>(p);
                        v[u][0][j] = a[0];
                        v[u][1][j] = a[1];
                    } else {
                        v[u][0][j] = *p;
                    }
                }
            }
        }
    }

    __device__ __forceinline__ void load_guarded(const float *__restrict__ X, int64_t ld,
                                                 int64_t Rn, int64_t K, int64_t r0, int64_t k0)
    {
        const int t = threadIdx.x;
        const auto gX = gmem(X);
#pragma unroll
        for (int u = 0; u < UPT; ++u) {
            const int uid = t + u * NT;
            const int k8 = k8_of(uid);
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int64_t gr = r0 + row_of(uid, q);
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int64_t gk = k0 + 8 * k8 + j;
                    float x = 0.0f;
                    if (gr < Rn && gk < K)
                        x = KC ? gX[gr * ld + gk] : gX[gk * ld + gr];
                    v[u][q][j] = x;
                }
            }
        }
    }

    // Split and write one entry (unit u, row q) of the stage.
    template <int PREC>
    __device__ __forceinline__ void store_entry(char *base, int u, int q) const
    {
        using C = Cfg<PREC>;
        constexpr int KF = BK / 16;
        const int uid = threadIdx.x + u * NT;
        const int k8 = k8_of(uid);
        const int row = row_of(uid, q);
        u32x4 parts[C::terms * (C::entry_bytes / 16)];
        Split<base_prec(PREC)>::run(v[u][q], parts);
        if constexpr (base_prec(PREC) == PREC_FP32) {
            u32x4 *dst =
                reinterpret_cast<u32x4 *>(base + entry_off<ROWS, KF, C::entry_bytes>(0, row, k8));
            dst[0] = parts[0];
            dst[1] = parts[1];
        } else {
#pragma unroll
            for (int tt = 0; tt < C::terms; ++tt)
                *reinterpret_cast<u32x4 *>(base + entry_off<ROWS, KF, C::entry_bytes>(tt, row, k8)) =
                    parts[tt];
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
            const int k8 = k8_of(uid);
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int row = row_of(uid, q);
                u32x4 parts[C::terms * (C::entry_bytes / 16)];
                Split<base_prec(PREC)>::run(v[u][q], parts);
                if constexpr (base_prec(PREC) == PREC_FP32) {
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

// Products of split terms (a term, b term), smallest magnitude first.
template <int PREC> struct Products;
template <> struct Products<PREC_BF16X3> {
    static constexpr int n = 3;
    static constexpr int a[3] = {1, 0, 0};
    static constexpr int b[3] = {0, 1, 0};
};
template <> struct Products<PREC_BF16X6> {
    static constexpr int n = 6;
    static constexpr int a[6] = {2, 0, 1, 1, 0, 0};
    static constexpr int b[6] = {0, 2, 1, 0, 1, 0};
};

// One K stage of MFMAs from LDS.  Fragment reads are issued in the order the
// MFMAs first need them (the first MFMA waits for two reads, later ones for
// at most one more), so the matrix core starts early in each stage.
template <int PREC, int KK0 = 0, int KK1 = Geo<PREC>::KF>
__device__ __forceinline__ void compute_stage(const char *sA, const char *sB,
                                              f32x16 (&acc)[Geo<PREC>::FM][Geo<PREC>::FN],
                                              int wm, int wn, int lane)
{
    using C = Cfg<PREC>;
    using G = Geo<PREC>;
    constexpr int FM = G::FM, FN = G::FN, KF = G::KF, EB = C::entry_bytes;
#pragma unroll
    for (int kk = KK0; kk < KK1; ++kk) {
        if constexpr (base_prec(PREC) == PREC_FP32) {
            f32x4 a[FM][2], b[FN][2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
#pragma unroll
                for (int i = 0; i < FM; ++i) {
                    a[i][h] = reinterpret_cast<const f32x4 *>(
                        sA + frag_off<C::BM, KF, EB>(0, wm * FM + i, kk, lane))[h];
                    if (i == 0)
#pragma unroll
                        for (int j = 0; j < FN; ++j)
                            b[j][h] = reinterpret_cast<const f32x4 *>(
                                sB + frag_off<C::BN, KF, EB>(0, wn * FN + j, kk, lane))[h];
                }
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
            using P = Products<base_prec(PREC)>;
            constexpr int T = C::terms;
            bf16x8 a[FM][T], b[FN][T];
            // reads in first-use order: for each product, a[0], b[*], a[1..]
            bool have_a[T] = {}, have_b[T] = {};
#pragma unroll
            for (int p = 0; p < P::n; ++p) {
                const int ta = P::a[p], tb = P::b[p];
                const bool need_a = !have_a[ta], need_b = !have_b[tb];
#pragma unroll
                for (int i = 0; i < FM; ++i) {
                    if (need_a)
                        a[i][ta] = *reinterpret_cast<const bf16x8 *>(
                            sA + frag_off<C::BM, KF, EB>(ta, wm * FM + i, kk, lane));
                    if (i == 0 && need_b)
#pragma unroll
                        for (int j = 0; j < FN; ++j)
                            b[j][tb] = *reinterpret_cast<const bf16x8 *>(
                                sB + frag_off<C::BN, KF, EB>(tb, wn * FN + j, kk, lane));
                }
                have_a[ta] = true;
                have_b[tb] = true;
            }
#pragma unroll
            for (int p = 0; p < P::n; ++p)
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            a[i][P::a[p]], b[j][P::b[p]], acc[i][j], 0, 0, 0);
        }
    }
}

// One 16-k half of a stage whose MFMAs are issued in NG equal groups; after
// group g, between(g) runs (one LDS entry of the next stage), and a fence
// keeps each group's MFMAs and split work in one small scheduling region so
// they interleave.
template <int PREC, int KK, int NG, typename F>
__device__ __forceinline__ void compute_half_interleaved(const char *sA, const char *sB,
                                                         f32x16 (&acc)[Geo<PREC>::FM][Geo<PREC>::FN],
                                                         int wm, int wn, int lane, F &&between)
{
    using C = Cfg<PREC>;
    using G = Geo<PREC>;
    constexpr int FM = G::FM, FN = G::FN, KF = G::KF, EB = C::entry_bytes;
    if constexpr (base_prec(PREC) == PREC_FP32) {
        constexpr int NM = 8 * FM * FN, GS = NM / NG;
        f32x4 a[FM][2], b[FN][2];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                a[i][h] = reinterpret_cast<const f32x4 *>(
                    sA + frag_off<C::BM, KF, EB>(0, wm * FM + i, KK, lane))[h];
                if (i == 0)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        b[j][h] = reinterpret_cast<const f32x4 *>(
                            sB + frag_off<C::BN, KF, EB>(0, wn * FN + j, KK, lane))[h];
            }
        __builtin_amdgcn_sched_barrier(0);
#pragma clang loop unroll(full)
        for (int m = 0; m < NM; ++m) {
            const int e = m / (FM * FN), i = (m / FN) % FM, j = m % FN;
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i][e >> 2][e & 3],
                                                            b[j][e >> 2][e & 3], acc[i][j], 0,
                                                            0, 0);
            if (m % GS == GS - 1) {
                between(m / GS);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    } else {
        using P = Products<base_prec(PREC)>;
        constexpr int T = C::terms;
        constexpr int NM = P::n * FM * FN, GS = NM / NG;
        bf16x8 a[FM][T], b[FN][T];
        bool have_a[T] = {}, have_b[T] = {};
#pragma unroll
        for (int p = 0; p < P::n; ++p) {
            const int ta = P::a[p], tb = P::b[p];
            const bool need_a = !have_a[ta], need_b = !have_b[tb];
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                if (need_a)
                    a[i][ta] = *reinterpret_cast<const bf16x8 *>(
                        sA + frag_off<C::BM, KF, EB>(ta, wm * FM + i, KK, lane));
                if (i == 0 && need_b)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        b[j][tb] = *reinterpret_cast<const bf16x8 *>(
                            sB + frag_off<C::BN, KF, EB>(tb, wn * FN + j, KK, lane));
            }
            have_a[ta] = true;
            have_b[tb] = true;
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma clang loop unroll(full)
        for (int m = 0; m < NM; ++m) {
            const int p = m / (FM * FN), i = (m / FN) % FM, j = m % FN;
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][P::a[p]], b[j][P::b[p]],
                                                               acc[i][j], 0, 0, 0);
            if (m % GS == GS - 1) {
                between(m / GS);
                // split work of one entry: ~6 VALU per 2 values per term
                constexpr int VPER = (12 * T + GS - 1) / GS;
#pragma unroll
                for (int q = 0; q < GS; ++q) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                    __builtin_amdgcn_sched_group_barrier(0x002, VPER, 0);
                }
                __builtin_amdgcn_sched_group_barrier(0x200, T, 0);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
}

// Fragment read helpers (bf16 terms).
template <int PREC>
__device__ __forceinline__ void read_a(bf16x8 (&a)[Geo<PREC>::FM][Cfg<PREC>::terms], const char *sA,
                                       int t, int kk, int wm, int lane)
{
    using C = Cfg<PREC>;
    using G = Geo<PREC>;
#pragma unroll
    for (int i = 0; i < G::FM; ++i)
        a[i][t] = *reinterpret_cast<const bf16x8 *>(
            sA + frag_off<C::BM, G::KF, C::entry_bytes>(t, wm * G::FM + i, kk, lane));
}
template <int PREC>
__device__ __forceinline__ void read_b(bf16x8 (&b)[Geo<PREC>::FN][Cfg<PREC>::terms], const char *sB,
                                       int t, int kk, int wn, int lane)
{
    using C = Cfg<PREC>;
    using G = Geo<PREC>;
#pragma unroll
    for (int j = 0; j < G::FN; ++j)
        b[j][t] = *reinterpret_cast<const bf16x8 *>(
            sB + frag_off<C::BN, G::KF, C::entry_bytes>(t, wn * G::FN + j, kk, lane));
}

// Steady-state stage of the 3xBF16 PIPE 1 loop (BK = 32, two 16-k halves).
// The second half's first fragments (lo of A, hi of B) are read into the
// registers the first half frees after its second product, and the rest as
// soon as the first half ends, so the matrix core does not drain between the
// halves.  The split/writes of the next stage interleave with the second
// half's MFMAs in NG groups (between(g) after each group).
template <int PR, int NG, typename F>
__device__ __forceinline__ void stage_x3_pipe1(const char *sA, const char *sB,
                                               f32x16 (&acc)[Geo<PR>::FM][Geo<PR>::FN],
                                               int wm, int wn, int lane, F &&between)
{
    constexpr int FM = Geo<PR>::FM, FN = Geo<PR>::FN;
    bf16x8 a0[FM][2], b0[FN][2], a1[FM][2], b1[FN][2];
    read_a<PR>(a0, sA, 1, 0, wm, lane);   // lo A
    read_b<PR>(b0, sB, 0, 0, wn, lane);   // hi B
    read_a<PR>(a0, sA, 0, 0, wm, lane);   // hi A
    read_b<PR>(b0, sB, 1, 0, wn, lane);   // lo B
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0[i][1], b0[j][0], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0[i][0], b0[j][1], acc[i][j], 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
    read_a<PR>(a1, sA, 1, 1, wm, lane);   // second half: lo A, hi B first
    read_b<PR>(b1, sB, 0, 1, wn, lane);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0[i][0], b0[j][0], acc[i][j], 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
    read_a<PR>(a1, sA, 0, 1, wm, lane);
    read_b<PR>(b1, sB, 1, 1, wn, lane);
    __builtin_amdgcn_sched_barrier(0);
    constexpr int NM = 3 * FM * FN, GS = NM / NG;
#pragma clang loop unroll(full)
    for (int m = 0; m < NM; ++m) {
        const int p = m / (FM * FN), i = (m / FN) % FM, j = m % FN;
        const int ta = p == 0 ? 1 : 0, tb = p == 1 ? 1 : 0;
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1[i][ta], b1[j][tb], acc[i][j], 0, 0, 0);
        if (m % GS == GS - 1) {
            between(m / GS);
#pragma unroll
            for (int q = 0; q < GS; ++q) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);
            }
            __builtin_amdgcn_sched_group_barrier(0x200, 2, 0);
            __builtin_amdgcn_sched_barrier(0);
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
__device__ __forceinline__ void gram_tile(int lin, int nt, int &tm, int &tn)
{
    int r = 0, rem = lin;
    while (rem >= nt - r) {
        rem -= nt - r;
        ++r;
    }
    tm = r;
    tn = r + rem;
}

__device__ __forceinline__ void tile_coords(const GemmDesc &d, int lin, int &tm, int &tn)
{
    if (d.gram) {
        gram_tile(lin, d.tiles_n, tm, tn);
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

// Tile of a workgroup of a 256 x 256-tile launch (one workgroup per CU).
// Workgroups reach the XCDs round-robin and each XCD runs 32 at a time, so the
// 256 tiles in flight form one 16 x 16 block of tiles, each XCD a 4 x 8 part
// of it: such a round reads 16 A and 16 B operand panels, and each XCD's 32
// tiles share 4 A and 8 B panels in its L2; consecutive rounds move down the
// tile rows, keeping their B panels.  (With every XCD sweeping its own band of
// tile rows across all columns instead, the packed kernel fetched 1.6 times as
// much from HBM.)  A Gram launch over a whole upper triangle of 16k x 16k
// tiles takes its off-diagonal 16 x 16 blocks the same way, column by column
// (consecutive rounds keep their B panels), then the 136-tile triangles of the
// diagonal blocks, each XCD a contiguous half of one (row by row in it); in
// plain row order an XCD's 32 tiles would share one A panel and need 32 B
// panels.  Other tile counts, and Gram launches over part of the triangle,
// use the general order.
__device__ __forceinline__ void round_tile_coords(const GemmDesc &d, int &tm, int &tn)
{
    if (kXcds == 8 && d.tiles_m % 16 == 0 && d.tiles_n % 16 == 0 && !d.gram) {
        const int x = blockIdx.x % kXcds, i = blockIdx.x / kXcds;
        const int r = i / 32, sl = i % 32;
        const int sm = d.tiles_m / 16;
        tm = 16 * (r % sm) + 4 * (x % 4) + sl % 4;
        tn = 16 * (r / sm) + 8 * (x / 4) + sl / 4;
    } else if (kXcds == 8 && d.gram && d.tiles_n % 16 == 0 &&
               d.num_tiles == d.tiles_n * (d.tiles_n + 1) / 2) {
        const int x = blockIdx.x % kXcds, i = blockIdx.x / kXcds;
        const int nb = d.tiles_n / 16, noff = nb * (nb - 1) / 2;
        if (i < 32 * noff) {
            // off-diagonal block r: column C, row R < C
            const int r = i / 32, sl = i % 32;
            int C = 1;
            while (C * (C + 1) / 2 <= r)
                ++C;
            const int R = r - C * (C - 1) / 2;
            tm = 16 * R + 4 * (x % 4) + sl % 4;
            tn = 16 * C + 8 * (x / 4) + sl / 4;
        } else {
            // diagonal blocks: 136 upper tiles each, 17 nb per XCD
            const int g = x * (17 * nb) + (i - 32 * noff);
            int lr, lc;
            gram_tile(g % 136, 16, lr, lc);
            tm = 16 * (g / 136) + lr;
            tn = 16 * (g / 136) + lc;
        }
    } else {
        tile_coords(d, xcd_remap(blockIdx.x, d.num_tiles), tm, tn);
    }
}

// Epilogue of one tile: out = alpha acc + beta E + gamma I, written to C (and
// mirrored for a full Gram), with the FP64 sum of (out - E)^2 for the step
// norm.  Each 32 x 32 block's 16 addend values per lane are loaded together,
// before any of the block's stores (C may alias E, so a load placed after a
// store would have to wait for it), and one explicit wait for them follows:
// without it the per-element bounds branches make the compiler wait for every
// outstanding memory operation, stores included, before each element.
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
        for (int j = 0; j < G::FN; ++j) {
            const int64_t col = cb + j * 32;
            float ev[16];
            if (d.E) {
                // past the edge a clamped in-range element is read and not used
                const int64_t cc = col < d.N ? col : d.N - 1;
#pragma clang loop unroll(full)
                for (int e = 0; e < 16; ++e) {
                    int64_t row = rb + i * 32 + (e >> 2) * 8 + (e & 3);
                    row = row < d.M ? row : d.M - 1;
                    ev[e] = gmem(d.E)[row * d.lde + cc];
                }
                __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
            }
#pragma clang loop unroll(full)
            for (int e = 0; e < 16; ++e) {
                const int64_t row = rb + i * 32 + (e >> 2) * 8 + (e & 3);
                if (row >= d.M || col >= d.N || (d.gram && row > col))
                    continue;
                float val = d.alpha * acc[i][j][e];
                float evv = 0.0f;
                if (d.E) {
                    evv = ev[e];
                    val = val + d.beta * evv;
                }
                if (row == col)
                    val = val + d.gamma;
                gmem(d.C)[row * d.ldc + col] = val;
                if (d.gram && !d.gram_upper && row != col)
                    gmem(d.C)[col * d.ldc + row] = val;
                if (want_ss) {
                    const double df = (double)val - (double)evv;
                    ss += df * df;
                }
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
            gmem(d.partials)[(int64_t)tm * d.tiles_n + tn] = s;
        }
    }
}

// Address of op(X)(r, k) for the two storage orders.
template <bool KC>
__device__ __forceinline__ const float *op_ptr(const float *X, int64_t ld, int64_t r, int64_t k)
{
    return KC ? X + r * ld + k : X + k * ld + r;
}

// Instruction interleave of one stage: all fragment reads first, then each
// MFMA followed by a share of the split VALU work and, every few MFMAs, one
// LDS write of the next stage.  (Hints to the scheduler; data dependences
// still decide.)
template <int PREC, int NKF = Geo<PREC>::KF>
__device__ __forceinline__ void interleave_hint()
{
    using G = Geo<PREC>;
    using C = Cfg<PREC>;
    constexpr int BP = base_prec(PREC);
    constexpr int NPROD = BP == PREC_FP32 ? 8 : BP == PREC_BF16X3 ? 3 : 6;
    constexpr int NMFMA = G::FM * G::FN * NPROD * NKF;
    constexpr int NREAD = (G::FM + G::FN) * C::terms * (C::entry_bytes / 16) * NKF;
    // LDS writes of one stage: (rows of A + rows of B) x BK / 8 entries per
    // term, spread over the workgroup
    constexpr int NWRITE = (C::BM + C::BN) * (C::BK / 8) * C::terms * (C::entry_bytes / 16) / G::NT;
    constexpr int VALU_PER = BP == PREC_FP32 ? 0 : BP == PREC_BF16X3 ? 4 : 2;
    constexpr int W_EVERY = NMFMA / NWRITE > 0 ? NMFMA / NWRITE : 1;
    __builtin_amdgcn_sched_group_barrier(0x100, NREAD, 0);
#pragma unroll
    for (int i = 0; i < NMFMA; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        if (VALU_PER > 0)
            __builtin_amdgcn_sched_group_barrier(0x002, VALU_PER, 0);
        if (i % W_EVERY == W_EVERY - 1)
            __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
    }
}

// K loop of one tile, software pipelined two stages deep: while the MFMAs of
// stage s run from LDS buffer s%2, the registers holding stage s+1 (loaded
// one stage earlier) are split into LDS buffer (s+1)%2, and stage s+2 is
// being loaded into the other register set.  GUARD: every load is bounds
// checked (edge tiles, unaligned operands); otherwise stages [0, K / BK) use
// unguarded vector loads and only a partial last stage is guarded.
template <int PREC, bool AKC, bool BKC, bool GUARD>
__device__ __forceinline__ void k_loop2(const GemmDesc &d, int64_t row0, int64_t col0,
                                        f32x16 (&acc)[Geo<PREC>::FM][Geo<PREC>::FN],
                                        char *smem, int wm, int wn, int lane)
{
    using C = Cfg<PREC>;
    using G = Geo<PREC>;
    constexpr int BK = C::BK;
    using LA = Loader<C::BM, BK, G::NT, AKC>;
    using LB = Loader<C::BN, BK, G::NT, BKC>;
    LA la[2];
    LB lb[2];
    const int64_t nst = (d.K + BK - 1) / BK;
    const int64_t nfull = GUARD ? 0 : d.K / BK;
    if (nst == 0)
        return;
    if (!GUARD) {
        la[0].init(d.lda);
        lb[0].init(d.ldb);
        la[1].init(d.lda);
        lb[1].init(d.ldb);
    }
    auto fetch = [&](LA &a, LB &b, int64_t st) {
        const int64_t k0 = st * BK;
        if (st < nfull) {
            a.load_fast(op_ptr<AKC>(d.A, d.lda, row0, k0), d.lda);
            b.load_fast(op_ptr<BKC>(d.B, d.ldb, col0, k0), d.ldb);
        } else {
            a.load_guarded(d.A, d.lda, d.M, d.K, row0, k0);
            b.load_guarded(d.B, d.ldb, d.N, d.K, col0, k0);
        }
    };
    // one pipelined stage; register set P receives stage s+2, set Q (= 1-P)
    // holds stage s+1
    auto step = [&](auto pset, int64_t st, auto steady) {
        constexpr int P = decltype(pset)::value, Q = 1 - P;
        constexpr bool fast_next = decltype(steady)::value;
        if constexpr (fast_next) {
            const int64_t k2 = (st + 2) * BK;
            la[P].load_fast(op_ptr<AKC>(d.A, d.lda, row0, k2), d.lda);
            lb[P].load_fast(op_ptr<BKC>(d.B, d.ldb, col0, k2), d.ldb);
        } else if (st + 2 < nst) {
            fetch(la[P], lb[P], st + 2);
        }
        __builtin_amdgcn_sched_barrier(0);
        char *sc = smem + (int)(st & 1) * G::stage_bytes;        // stage being computed
        char *sn = smem + (int)((st + 1) & 1) * G::stage_bytes;  // stage being filled
        if constexpr (fast_next && G::KF == 1) {
            constexpr int EA = LA::UPT * LA::R, EB_ = LB::UPT * LB::R;
            compute_half_interleaved<PREC, 0, EA + EB_>(
                sc, sc + G::a_bytes, acc, wm, wn, lane, [&](int g) {
                    if (g < EA)
                        la[Q].template store_entry<PREC>(sn, g / LA::R, g % LA::R);
                    else
                        lb[Q].template store_entry<PREC>(sn + G::a_bytes, (g - EA) / LB::R,
                                                         (g - EA) % LB::R);
                });
        } else {
            compute_stage<PREC>(sc, sc + G::a_bytes, acc, wm, wn, lane);
            if (fast_next || st + 1 < nst) {
                la[Q].template store<PREC>(sn);
                lb[Q].template store<PREC>(sn + G::a_bytes);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        __syncthreads();
    };
    fetch(la[0], lb[0], 0);
    la[0].template store<PREC>(smem);
    lb[0].template store<PREC>(smem + G::a_bytes);
    if (nst > 1)
        fetch(la[1], lb[1], 1);
    __syncthreads();
    int64_t s = 0;
    // steady state: the stages fetched (s+2, s+3) are full ones
    for (; s + 3 < nfull; s += 2) {
        step(std::integral_constant<int, 0>{}, s, std::true_type{});
        step(std::integral_constant<int, 1>{}, s + 1, std::true_type{});
    }
    for (; s < nst; s += 2) {
        step(std::integral_constant<int, 0>{}, s, std::false_type{});
        if (s + 1 < nst)
            step(std::integral_constant<int, 1>{}, s + 1, std::false_type{});
    }
}

// K loop, one register stage (PIPE 1, BK = 32): the loads of stage s+1 are
// issued at the top of stage s, the first 16-k half of stage s computes while
// they are in flight, and the split/LDS writes of stage s+1 are interleaved
// with the MFMAs of the second half.
template <int PREC, bool AKC, bool BKC, bool GUARD>
__device__ __forceinline__ void k_loop1(const GemmDesc &d, int64_t row0, int64_t col0,
                                        f32x16 (&acc)[Geo<PREC>::FM][Geo<PREC>::FN],
                                        char *smem, int wm, int wn, int lane)
{
    using C = Cfg<PREC>;
    using G = Geo<PREC>;
    constexpr int BK = C::BK;
    Loader<C::BM, BK, G::NT, AKC> la;
    Loader<C::BN, BK, G::NT, BKC> lb;
    const int64_t nst = (d.K + BK - 1) / BK;
    const int64_t nfull = GUARD ? 0 : d.K / BK;
    if (nst == 0)
        return;
    if (!GUARD) {
        la.init(d.lda);
        lb.init(d.ldb);
    }
    if (nfull > 0) {
        la.load_fast(op_ptr<AKC>(d.A, d.lda, row0, 0), d.lda);
        lb.load_fast(op_ptr<BKC>(d.B, d.ldb, col0, 0), d.ldb);
    } else {
        la.load_guarded(d.A, d.lda, d.M, d.K, row0, 0);
        lb.load_guarded(d.B, d.ldb, d.N, d.K, col0, 0);
    }
    la.template store<PREC>(smem);
    lb.template store<PREC>(smem + G::a_bytes);
    __syncthreads();
    int64_t s = 0;
    for (; s + 1 < nfull; ++s) {
        const int64_t k1 = (s + 1) * BK;
        la.load_fast(op_ptr<AKC>(d.A, d.lda, row0, k1), d.lda);
        lb.load_fast(op_ptr<BKC>(d.B, d.ldb, col0, k1), d.ldb);
        __builtin_amdgcn_sched_barrier(0);
        char *sc = smem + (int)(s & 1) * G::stage_bytes;
        char *sn = smem + (int)((s + 1) & 1) * G::stage_bytes;
        // entries of the next stage: A rows then B rows, one per MFMA group
        constexpr int EA = decltype(la)::UPT * decltype(la)::R;
        constexpr int EB_ = decltype(lb)::UPT * decltype(lb)::R;
        auto between = [&](int g) {
            if (g < EA)
                la.template store_entry<PREC>(sn, g / decltype(la)::R, g % decltype(la)::R);
            else
                lb.template store_entry<PREC>(sn + G::a_bytes, (g - EA) / decltype(lb)::R,
                                              (g - EA) % decltype(lb)::R);
        };
        if constexpr (G::KF == 1) {
            // one 16-k block per stage: compute, then split the next stage
            compute_stage<PREC>(sc, sc + G::a_bytes, acc, wm, wn, lane);
            __builtin_amdgcn_sched_barrier(0);
            la.template store<PREC>(sn);
            lb.template store<PREC>(sn + G::a_bytes);
        } else if constexpr (base_prec(PREC) == PREC_BF16X3) {
            stage_x3_pipe1<PREC, EA + EB_>(sc, sc + G::a_bytes, acc, wm, wn, lane, between);
        } else {
            compute_stage<PREC, 0, 1>(sc, sc + G::a_bytes, acc, wm, wn, lane);
            __builtin_amdgcn_sched_barrier(0);
            compute_half_interleaved<PREC, 1, EA + EB_>(sc, sc + G::a_bytes, acc, wm, wn, lane,
                                                        between);
        }
        __builtin_amdgcn_sched_barrier(0);
        __syncthreads();
    }
    for (; s < nst; ++s) {
        const bool more = s + 1 < nst;
        if (more) {
            const int64_t k1 = (s + 1) * BK;
            if (s + 1 < nfull) {
                la.load_fast(op_ptr<AKC>(d.A, d.lda, row0, k1), d.lda);
                lb.load_fast(op_ptr<BKC>(d.B, d.ldb, col0, k1), d.ldb);
            } else {
                la.load_guarded(d.A, d.lda, d.M, d.K, row0, k1);
                lb.load_guarded(d.B, d.ldb, d.N, d.K, col0, k1);
            }
        }
        char *sc = smem + (int)(s & 1) * G::stage_bytes;
        char *sn = smem + (int)((s + 1) & 1) * G::stage_bytes;
        compute_stage<PREC>(sc, sc + G::a_bytes, acc, wm, wn, lane);
        if (more) {
            la.template store<PREC>(sn);
            lb.template store<PREC>(sn + G::a_bytes);
        }
        __syncthreads();
    }
}

// GROUPED: the persistent kernel keeps extra state live across tiles; where
// two register stages would spill there, one stage is used (same arithmetic,
// same k order, so identical results).
template <int PREC, bool AKC, bool BKC, bool GUARD, bool GROUPED = false>
__device__ __forceinline__ void k_loop(const GemmDesc &d, int64_t row0, int64_t col0,
                                       f32x16 (&acc)[Geo<PREC>::FM][Geo<PREC>::FN],
                                       char *smem, int wm, int wn, int lane)
{
    if constexpr (Cfg<PREC>::PIPE == 1 || GROUPED)
        k_loop1<PREC, AKC, BKC, GUARD>(d, row0, col0, acc, smem, wm, wn, lane);
    else
        k_loop2<PREC, AKC, BKC, GUARD>(d, row0, col0, acc, smem, wm, wn, lane);
}

template <int PREC, bool AKC, bool BKC, bool GROUPED = false>
__device__ __forceinline__ void gemm_tile(const GemmDesc &d, int tm, int tn, char *smem,
                                          double *red)
{
    using C = Cfg<PREC>;
    using G = Geo<PREC>;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w / C::WN, wn = w % C::WN;
    const int64_t row0 = (int64_t)tm * C::BM, col0 = (int64_t)tn * C::BN;

    f32x16 acc[G::FM][G::FN];
#pragma clang loop unroll(full)
    for (int i = 0; i < G::FM; ++i)
#pragma clang loop unroll(full)
        for (int j = 0; j < G::FN; ++j)
            acc[i][j] = f32x16{};

    const bool interior = row0 + C::BM <= d.M && col0 + C::BN <= d.N && d.vec_a && d.vec_b;
    if (interior)
        k_loop<PREC, AKC, BKC, false, GROUPED>(d, row0, col0, acc, smem, wm, wn, lane);
    else
        k_loop<PREC, AKC, BKC, true, GROUPED>(d, row0, col0, acc, smem, wm, wn, lane);
    epilogue<PREC>(d, acc, tm, tn, wm, wn, lane, red);
}

// ---------------------------------------------------------------- kernels

template <int PREC, bool AKC, bool BKC>
__global__ void __launch_bounds__(Geo<PREC>::NT, (kernel_occ<PREC, AKC, BKC>())) gemm_kernel(GemmDesc d)
{
    __shared__ __attribute__((aligned(16))) char smem[2 * Geo<PREC>::stage_bytes];
    __shared__ double red[Cfg<PREC>::WM * Cfg<PREC>::WN];
    int tm, tn;
    if (Cfg<PREC>::BM == 256) {
        round_tile_coords(d, tm, tn);
    } else if (d.quarters) {
        // quarter (blockIdx.x & 3) of large Gram tile tail_first + blockIdx.x / 4
        int TM, TN;
        gram_tile(d.tail_first + (int)(blockIdx.x >> 2), (d.tiles_n + 1) / 2, TM, TN);
        tm = 2 * TM + (int)((blockIdx.x >> 1) & 1);
        tn = 2 * TN + (int)(blockIdx.x & 1);
        if (tm > tn || tm >= d.tiles_m || tn >= d.tiles_n)
            return;   // below the diagonal or past the edge: nothing of it is written
    } else {
        tile_coords(d, xcd_remap(blockIdx.x, d.num_tiles), tm, tn);
    }
    gemm_tile<PREC, AKC, BKC>(d, tm, tn, smem, red);
}

// Split-K slices of one product in a single launch, so that they run side by
// side: slice blockIdx.y takes k in [y slice_k, min(K, (y + 1) slice_k)) and
// writes its own output at C + y slice_stride, computing exactly what a launch
// of that slice alone would.  slice_k is a multiple of the K stage, so every
// slice but the last is made of whole stages and keeps the operands' 16-byte
// alignment.
template <int PREC, bool AKC, bool BKC>
__global__ void __launch_bounds__(Geo<PREC>::NT, (kernel_occ<PREC, AKC, BKC>()))
    gemm_sliced_kernel(GemmDesc d)
{
    __shared__ __attribute__((aligned(16))) char smem[2 * Geo<PREC>::stage_bytes];
    __shared__ double red[Cfg<PREC>::WM * Cfg<PREC>::WN];
    const int64_t k0 = (int64_t)blockIdx.y * d.slice_k;
    const int64_t kl = d.K - k0 < d.slice_k ? d.K - k0 : d.slice_k;
    d.A += AKC ? k0 : k0 * d.lda;
    d.B += BKC ? k0 : k0 * d.ldb;
    d.K = kl > 0 ? kl : 0;
    d.C += (int64_t)blockIdx.y * d.slice_stride;
    int tm, tn;
    if (Cfg<PREC>::BM == 256)
        round_tile_coords(d, tm, tn);
    else
        tile_coords(d, xcd_remap(blockIdx.x, d.num_tiles), tm, tn);
    gemm_tile<PREC, AKC, BKC>(d, tm, tn, smem, red);
}

// Persistent grouped kernel: workgroup b runs items b, b + grid, ...; each
// item is one tile of one problem, computed exactly as gemm_kernel would.  A
// capped grid leaves CUs to work on other streams (the panel chain of CAQR).
template <int PREC, bool AKC, bool BKC>
__global__ void __launch_bounds__(Geo<PREC>::NT, Cfg<PREC>::GOCC)
    gemm_grouped_kernel(const GemmDesc *__restrict__ probs, const GroupItem *__restrict__ items,
                        int num_items)
{
    __shared__ __attribute__((aligned(16))) char smem[2 * Geo<PREC>::stage_bytes];
    __shared__ double red[Cfg<PREC>::WM * Cfg<PREC>::WN];
    for (int it = blockIdx.x; it < num_items; it += gridDim.x) {
        const GroupItem gi = items[it];
        if (gi.prob < 0)
            continue;   // empty item (uniform over the workgroup)
        const GemmDesc d = probs[gi.prob];
        int tm, tn;
        tile_coords(d, gi.tile, tm, tn);
        gemm_tile<PREC, AKC, BKC, true>(d, tm, tn, smem, red);
        __syncthreads();
    }
}

// Grouped kernel, one workgroup per item: workgroup b computes item b exactly
// as gemm_kernel would (the same loop, so the same bits as the persistent
// kernel too); workgroup b runs on XCD b % kXcds, so the caller places the
// items on the XCDs by their position in the list.
template <int PREC, bool AKC, bool BKC>
__global__ void __launch_bounds__(Geo<PREC>::NT, (kernel_occ<PREC, AKC, BKC>()))
    gemm_items_kernel(const GemmDesc *__restrict__ probs, const GroupItem *__restrict__ items,
                      int num_items)
{
    __shared__ __attribute__((aligned(16))) char smem[2 * Geo<PREC>::stage_bytes];
    __shared__ double red[Cfg<PREC>::WM * Cfg<PREC>::WN];
    const int it = blockIdx.x;
    if (it >= num_items)
        return;
    const GroupItem gi = items[it];
    if (gi.prob < 0)
        return;   // empty item
    const GemmDesc d = probs[gi.prob];
    int tm, tn;
    tile_coords(d, gi.tile, tm, tn);
    gemm_tile<PREC, AKC, BKC>(d, tm, tn, smem, red);
}

// ---------------------------------------------------------------- packed operands

// Packed layout of an R x K operand op(X) (R = output rows for A, output
// columns for B), written by pack_x3_kernel and read by gemm_packed_kernel:
// 1 KiB chunks, chunk (rb, kb, t) at byte kb * packed_kstride(RB) +
// (rb * 2 + t) * 1024, rb = block of 32 rows (RB of them), kb = block of 16
// k, t = term (0 hi, 1 lo).  k-block-major: one stage of one tile is 16
// contiguous KiB, and all tiles at the same k step read one contiguous
// region (a row-block-major order put the chunks in flight a power of two
// apart, which defeated the L2).  Inside
// a chunk, the 16 bytes of lane l hold the 8 bf16 of row 32 rb + (l & 31),
// k = 16 kb + 8 (l >> 5) .. + 7: exactly one fragment block of the LDS image
// (entry_off with KF = 1).  Rows are padded with zeros to a multiple of 256,
// k to a multiple of 16, so the GEMM needs no bounds checks.
constexpr int kPackRows = 256;
constexpr int kPackSlabK = 128;   // k covered by one workgroup of the pack kernel
// Bytes from one k block to the next in a packed operand with rbt row
// blocks: the 2 rbt KiB of chunks plus 17 KiB of padding.  Without it the
// stride is a power of two for power-of-two sizes, consecutive k blocks land
// in the same L2 sets, and the L2 misses doubled (measured at
// 16384 x 32768 x 16384: 151 GiB fetched per launch unpadded, 72 GiB with
// 17 KiB, which fetched the least among the paddings tried).
constexpr int kPackPadKiB = 17;
__host__ __device__ inline int64_t packed_kstride(int64_t rbt)
{
    return (2 * rbt + kPackPadKiB) << 10;
}

template <bool KC>
__global__ void __launch_bounds__(256) pack_x3_kernel(const float *__restrict__ X, int64_t ld,
                                                      int64_t R, int64_t K, int64_t kbt,
                                                      int64_t rbt, int vec,
                                                      char *__restrict__ out)
{
    __shared__ float tile[32][kPackSlabK + 1];
    const int t = threadIdx.x;
    for (int64_t rb = blockIdx.y; rb < rbt; rb += gridDim.y) {
        const int64_t r0 = rb * 32, k0 = (int64_t)blockIdx.x * kPackSlabK;
        // stage 32 rows x 128 k through LDS, 4 consecutive elements of the
        // contiguous direction per thread and load (consecutive threads read
        // consecutive 16 bytes); zero outside R x K.  vec: the operand allows
        // 16-byte loads (aligned base, ld a multiple of 4)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = t + 256 * u;            // 1024 groups of 4 elements
            int r, k;                             // first element of the group
            if (KC) {
                r = i / (kPackSlabK / 4);
                k = (i % (kPackSlabK / 4)) * 4;
            } else {
                k = i / 8;
                r = (i % 8) * 4;
            }
            const int64_t gr = r0 + r, gk = k0 + k;
            float v[4];
            const bool full = KC ? (gr < R && gk + 3 < K) : (gk < K && gr + 3 < R);
            if (vec && full) {
                const f32x4 q = *reinterpret_cast<const f32x4 *>(KC ? X + gr * ld + gk
                                                                    : X + gk * ld + gr);
                v[0] = q[0];
                v[1] = q[1];
                v[2] = q[2];
                v[3] = q[3];
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int64_t er = KC ? gr : gr + e, ek = KC ? gk + e : gk;
                    v[e] = (er < R && ek < K) ? (KC ? X[er * ld + ek] : X[ek * ld + er]) : 0.0f;
                }
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (KC)
                    tile[r][k + e] = v[e];
                else
                    tile[r + e][k] = v[e];
            }
        }
        __syncthreads();
        // 8 k blocks x 64 lane entries per term; two entries per thread
        for (int e = t; e < (kPackSlabK / 16) * 64; e += 256) {
            const int kbl = e >> 6, lane = e & 63;
            const int64_t kb = (int64_t)blockIdx.x * (kPackSlabK / 16) + kbl;
            if (kb >= kbt)
                continue;
            const int r = lane & 31, kk = kbl * 16 + (lane >> 5) * 8;
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                v[j] = tile[r][kk + j];
            u32x4 parts[2];
            Split<PREC_BF16X3>::run(v, parts);
            char *chunk = out + kb * packed_kstride(rbt) + ((rb * 2) << 10);
            *reinterpret_cast<u32x4 *>(chunk + lane * 16) = parts[0];
            *reinterpret_cast<u32x4 *>(chunk + 1024 + lane * 16) = parts[1];
        }
        __syncthreads();
    }
}

template <int N>
__device__ __forceinline__ void wait_vmcnt()
{
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// One 16-byte-per-lane global -> LDS load: lane l's 16 bytes at base + voff
// go to LDS byte lds + 16 l.  Written as an asm statement so that the
// compiler does not treat the pending LDS writes as aliasing every later LDS
// read (it would drain all loads in flight before each stage); the K loop
// waits for exactly the stages it needs with wait_vmcnt.  The compiler
// writes M0 (the LDS base, wave-uniform); s_nop 0 is the one wait state an
// M0 write needs before an LDS-DMA load.  The load has no register result.
__device__ __forceinline__ void dma16(const void *base, uint32_t voff, uint32_t lds)
{
    // base: wave-uniform 64-bit address (SGPR pair); voff: per-lane byte offset
    asm volatile("s_nop 0\n\tglobal_load_lds_dwordx4 %0, %1" ::"v"(voff), "s"(base), "{m0}"(lds)
                 : "memory");
}

__device__ __forceinline__ uint32_t lds_offset(const void *p)
{
    return (uint32_t)(uintptr_t)(__attribute__((address_space(3))) const void *)p;
}

// Direct global -> LDS loads of one packed stage (k block kb): 16 chunks of
// A (2 terms x 8 row blocks) and 16 of B.  Wave w moves operand (w >= 2 ? B
// : A), term (w & 1), row blocks 0..7: eight 1 KiB chunks, each one
// global_load_lds_dwordx4.  stage_lds: LDS byte offset of the stage buffer.
// rbta / rbtb: row blocks of the packed A / B (the RB of the layout).
template <int P>
__device__ __forceinline__ void packed_issue(const char *pa, const char *pb, int64_t rbta,
                                             int64_t rbtb, int64_t rba, int64_t rbb, int64_t kb,
                                             uint32_t stage_lds, int w, int lane)
{
    using G = Geo<P>;
    const bool isb = w >= 2;
    const char *base = isb ? pb : pa;
    const int64_t rb0 = isb ? rbb : rba, rbt = isb ? rbtb : rbta;
    const uint32_t dst0 = stage_lds + (isb ? G::a_bytes : 0);
    const int tt = w & 1;
    const uint64_t wb = (uint64_t)(base + kb * packed_kstride(rbt) + ((rb0 * 2 + tt) << 10));
    const char *wbase = (const char *)(
        ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(wb >> 32)) << 32) |
        (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)wb));
#pragma unroll
    for (int frow = 0; frow < 8; ++frow)   // consecutive row blocks are 2 KiB apart
        dma16(wbase + (frow << 11), lane * 16, dst0 + ((tt * 8 + frow) << 10));
}

// Fragments of one packed stage for this wave, in two halves: the operands
// of the first product lo*hi (A lo, B hi) and the rest (A hi, B lo).
template <int P>
__device__ __forceinline__ void packed_read_first(const char *st, bf16x8 (&alo)[Geo<P>::FM],
                                                  bf16x8 (&bhi)[Geo<P>::FN], int wm, int wn,
                                                  int lane)
{
    using C = Cfg<P>;
    using G = Geo<P>;
#pragma unroll
    for (int i = 0; i < G::FM; ++i)
        alo[i] = *reinterpret_cast<const bf16x8 *>(st + frag_off<C::BM, 1, 16>(1, wm * G::FM + i, 0, lane));
#pragma unroll
    for (int j = 0; j < G::FN; ++j)
        bhi[j] = *reinterpret_cast<const bf16x8 *>(st + G::a_bytes +
                                                   frag_off<C::BN, 1, 16>(0, wn * G::FN + j, 0, lane));
}

template <int P>
__device__ __forceinline__ void packed_read_rest(const char *st, bf16x8 (&ahi)[Geo<P>::FM],
                                                 bf16x8 (&blo)[Geo<P>::FN], int wm, int wn,
                                                 int lane)
{
    using C = Cfg<P>;
    using G = Geo<P>;
#pragma unroll
    for (int i = 0; i < G::FM; ++i)
        ahi[i] = *reinterpret_cast<const bf16x8 *>(st + frag_off<C::BM, 1, 16>(0, wm * G::FM + i, 0, lane));
#pragma unroll
    for (int j = 0; j < G::FN; ++j)
        blo[j] = *reinterpret_cast<const bf16x8 *>(st + G::a_bytes +
                                                   frag_off<C::BN, 1, 16>(1, wn * G::FN + j, 0, lane));
}

// Wait until this wave's chunks of the next stage have landed, given how
// many later stages (0..3, eight chunks each) may stay in flight.
__device__ __forceinline__ void packed_wait(int later)
{
    if (later >= 3)
        wait_vmcnt<24>();
    else if (later == 2)
        wait_vmcnt<16>();
    else if (later == 1)
        wait_vmcnt<8>();
    else
        wait_vmcnt<0>();
}

// One 16-k stage.  alo / bhi hold this stage's first-product fragments on
// entry and the next stage's on exit.  The rest of this stage's fragments
// are read while the lo*hi MFMAs run; after the hi*lo MFMAs (alo is dead
// from here), wait for stage s+1, barrier, start the loads of stage s+4 into
// this stage's buffer (every wave has consumed it) and read stage s+1's A lo
// fragments; the hi*hi MFMAs run column by column, each B hi fragment
// replaced by stage s+1's once its column is done.  Every accumulator sees
// the products in the same order as in the unpacked 3xBF16 kernel.
template <int P>
__device__ __forceinline__ void packed_stage(int ss, int nst, f32x16 (&acc)[Geo<P>::FM][Geo<P>::FN],
                                             bf16x8 (&alo)[Geo<P>::FM], bf16x8 (&bhi)[Geo<P>::FN],
                                             const char *smem, uint32_t smem_lds, const char *pa,
                                             const char *pb, int64_t rbta, int64_t rbtb,
                                             int64_t rba, int64_t rbb, int w, int wm, int wn,
                                             int lane)
{
    using C = Cfg<P>;
    using G = Geo<P>;
    constexpr int FM = G::FM, FN = G::FN, NS = kPackStages;
    bf16x8 ahi[FM], blo[FN];
    packed_read_rest<P>(smem + (ss & (NS - 1)) * G::stage_bytes, ahi, blo, wm, wn, lane);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo[i], bhi[j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[i], blo[j], acc[i][j], 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
    const bool more = ss + 1 < nst;
    const char *nst_ = smem + ((ss + 1) & (NS - 1)) * G::stage_bytes;
    if (more) {
        packed_wait(min(nst - 2 - ss, NS - 2));
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        if (ss + NS < nst)
            packed_issue<P>(pa, pb, rbta, rbtb, rba, rbb, ss + NS,
                            smem_lds + (ss & (NS - 1)) * G::stage_bytes, w, lane);
#pragma unroll
        for (int i = 0; i < FM; ++i)
            alo[i] = *reinterpret_cast<const bf16x8 *>(nst_ + frag_off<C::BM, 1, 16>(1, wm * FM + i, 0, lane));
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < FN; ++j) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[i], bhi[j], acc[i][j], 0, 0, 0);
        if (more)
            bhi[j] = *reinterpret_cast<const bf16x8 *>(nst_ + G::a_bytes +
                                                       frag_off<C::BN, 1, 16>(0, wn * FN + j, 0, lane));
    }
    __builtin_amdgcn_sched_barrier(0);
}

// GEMM on packed operands: d.A / d.B point at the packed buffers, d.K is
// the (unpadded) inner dimension; the epilogue is the common one.
// With d.slices > 1, slice blockIdx.y takes the k blocks of [y slice_k,
// min(K, (y + 1) slice_k)) (slice_k a multiple of 16) and writes C + y
// slice_stride, as the split-K launch of the unpacked kernels does.
template <int P>
__global__ void __launch_bounds__(256, 1) gemm_packed_kernel(GemmDesc d)
{
    using G = Geo<P>;
    static_assert(G::KF == 1 && G::NT == 256, "one 16-k block per stage, four waves");
    constexpr int FM = G::FM, FN = G::FN, NS = kPackStages;
    __shared__ __attribute__((aligned(1024))) char smem[NS * G::stage_bytes];
    __shared__ double red[4];
    int tm, tn;
    round_tile_coords(d, tm, tn);
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w / 2, wn = w % 2;
    f32x16 acc[FM][FN];
#pragma clang loop unroll(full)
    for (int i = 0; i < FM; ++i)
#pragma clang loop unroll(full)
        for (int j = 0; j < FN; ++j)
            acc[i][j] = f32x16{};
    const char *pa = reinterpret_cast<const char *>(d.A);
    const char *pb = reinterpret_cast<const char *>(d.B);
    const int64_t rba = (int64_t)tm * 8, rbb = (int64_t)tn * 8;
    const int64_t rbta = (int64_t)d.tiles_m * 8, rbtb = (int64_t)d.tiles_n * 8;
    if (d.slices > 1) {
        const int64_t k0 = (int64_t)blockIdx.y * d.slice_k;
        const int64_t kl = d.K - k0 < d.slice_k ? d.K - k0 : d.slice_k;
        pa += (k0 / 16) * packed_kstride(rbta);
        pb += (k0 / 16) * packed_kstride(rbtb);
        d.K = kl > 0 ? kl : 0;
        d.C += (int64_t)blockIdx.y * d.slice_stride;
    }
    const int64_t kbt = (d.K + 15) / 16;
    const int nst = (int)kbt;
    const uint32_t smem_lds = __builtin_amdgcn_readfirstlane(lds_offset(smem));
    // first-product fragments of the current stage
    bf16x8 alo[FM], bhi[FN];
    if (nst > 0) {
#pragma unroll
        for (int s = 0; s < NS; ++s)
            if (s < nst)
                packed_issue<P>(pa, pb, rbta, rbtb, rba, rbb, s, smem_lds + s * G::stage_bytes, w,
                                lane);
        packed_wait(min(nst - 1, NS - 1));
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        packed_read_first<P>(smem, alo, bhi, wm, wn, lane);
    }
    for (int s = 0; s < nst; ++s)
        packed_stage<P>(s, nst, acc, alo, bhi, smem, smem_lds, pa, pb, rbta, rbtb, rba, rbb, w, wm,
                        wn, lane);
    epilogue<P>(d, acc, tm, tn, wm, wn, lane, red);
}

// ---------------------------------------------------------------- launchers

template <int PREC>
hipError_t launch_one(const GemmDesc &d, hipStream_t s)
{
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

// Compute units of the current device (cached per device).
inline int device_cu_count()
{
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 0;
    int v = cache[dev].load(std::memory_order_relaxed);
    if (v == 0) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        cache[dev].store(v, std::memory_order_relaxed);
    }
    return v;
}

// A large-tile Gram launch runs one tile per CU at a time.  When its tile
// count leaves a last round of at most a quarter of the CUs busy (N = 16384:
// 2080 tiles = 8 rounds + 32), the whole rounds keep the large tiles and the
// rest run in a second launch as 128 x 128 quarters, one small-tile round.
// The small tile class takes the same K steps in the same order, so every
// element is computed exactly as before.
template <int PREC>
bool split_gram_tail(const GemmDesc &d, GemmDesc &big, GemmDesc &tail)
{
    if (!d.gram || d.small || d.quarters)
        return false;
    const int cus = device_cu_count();
    if (cus <= 0 || d.num_tiles <= cus)
        return false;
    const int rest = d.num_tiles % cus;
    if (rest == 0 || 4 * rest > cus)
        return false;
    big = d;
    big.num_tiles = d.num_tiles - rest;
    tail = d;
    tail.small = 1;
    tail.tiles_m = (int)((d.M + Cfg<PREC | kSmall>::BM - 1) / Cfg<PREC | kSmall>::BM);
    tail.tiles_n = (int)((d.N + Cfg<PREC | kSmall>::BN - 1) / Cfg<PREC | kSmall>::BN);
    tail.quarters = 1;
    tail.tail_first = big.num_tiles;
    tail.num_tiles = 4 * rest;
    return true;
}

template <int PREC>
hipError_t launch_sliced(const GemmDesc &d, hipStream_t s)
{
    if (d.slice_k <= 0 || d.slice_k % Cfg<PREC>::BK != 0 || d.slices > 65535)
        return hipErrorInvalidValue;
    dim3 grid(d.num_tiles, d.slices), block(Geo<PREC>::NT);
    if (d.a_kcontig && d.b_kcontig)
        hipLaunchKernelGGL((gemm_sliced_kernel<PREC, true, true>), grid, block, 0, s, d);
    else if (d.a_kcontig)
        hipLaunchKernelGGL((gemm_sliced_kernel<PREC, true, false>), grid, block, 0, s, d);
    else if (d.b_kcontig)
        hipLaunchKernelGGL((gemm_sliced_kernel<PREC, false, true>), grid, block, 0, s, d);
    else
        hipLaunchKernelGGL((gemm_sliced_kernel<PREC, false, false>), grid, block, 0, s, d);
    return hipGetLastError();
}

template <int PREC>
hipError_t launch_t(const GemmDesc &d, hipStream_t s)
{
    if (d.num_tiles <= 0)
        return hipSuccess;
    if (d.slices > 1)
        return d.small ? launch_sliced<PREC | kSmall>(d, s) : launch_sliced<PREC>(d, s);
    GemmDesc big, tail;
    if (split_gram_tail<PREC>(d, big, tail)) {
        const hipError_t e = launch_one<PREC>(big, s);
        if (e != hipSuccess)
            return e;
        return launch_one<PREC | kSmall>(tail, s);
    }
    return d.small ? launch_one<PREC | kSmall>(d, s) : launch_one<PREC>(d, s);
}

// grid_size is the number of CUs; small tiles run two workgroups per CU.
template <int PREC, bool AKC, bool BKC>
void launch_grouped_kern(bool persist, dim3 grid, dim3 block, hipStream_t s,
                         const GemmDesc *probs, const GroupItem *items, int num_items)
{
    if (persist)
        hipLaunchKernelGGL((gemm_grouped_kernel<PREC, AKC, BKC>), grid, block, 0, s, probs,
                           items, num_items);
    else
        hipLaunchKernelGGL((gemm_items_kernel<PREC, AKC, BKC>), grid, block, 0, s, probs, items,
                           num_items);
}

template <int PREC>
hipError_t launch_grouped_one(int akc, int bkc, const GemmDesc *probs, const GroupItem *items,
                              int num_items, int grid_size, hipStream_t s)
{
    // grid_size > 0: persistent workgroups, at most grid_size per GOCC; else
    // one workgroup per item
    const bool persist = grid_size > 0;
    grid_size *= Cfg<PREC>::GOCC;
    dim3 grid(persist && grid_size < num_items ? grid_size : num_items), block(Geo<PREC>::NT);
    if (akc && bkc)
        launch_grouped_kern<PREC, true, true>(persist, grid, block, s, probs, items, num_items);
    else if (akc)
        launch_grouped_kern<PREC, true, false>(persist, grid, block, s, probs, items, num_items);
    else if (bkc)
        launch_grouped_kern<PREC, false, true>(persist, grid, block, s, probs, items, num_items);
    else
        launch_grouped_kern<PREC, false, false>(persist, grid, block, s, probs, items, num_items);
    return hipGetLastError();
}

template <int PREC>
hipError_t launch_grouped_t(int akc, int bkc, int small, const GemmDesc *probs,
                            const GroupItem *items, int num_items, int grid_size, hipStream_t s)
{
    if (num_items <= 0)
        return hipSuccess;
    return small ? launch_grouped_one<PREC | kSmall>(akc, bkc, probs, items, num_items,
                                                     grid_size, s)
                 : launch_grouped_one<PREC>(akc, bkc, probs, items, num_items, grid_size, s);
}

// Packed operand bytes for R rows and inner dimension K.
inline size_t packed_bytes(int64_t R, int64_t K)
{
    const int64_t rbt = (R + kPackRows - 1) / kPackRows * (kPackRows / 32);
    const int64_t kbt = (K + 15) / 16;
    return rbt == 0 ? 0 : (size_t)kbt * (size_t)packed_kstride(rbt);
}

inline hipError_t launch_pack_x3(const float *X, int64_t ld, int kc, int64_t R, int64_t K,
                                 char *out, hipStream_t s)
{
    const int64_t rbt = (R + kPackRows - 1) / kPackRows * (kPackRows / 32);
    const int64_t kbt = (K + 15) / 16;
    if (rbt == 0 || kbt == 0)
        return hipSuccess;
    const int64_t gx = (kbt * 16 + kPackSlabK - 1) / kPackSlabK;
    if (gx > 0x7fffffff)
        return hipErrorInvalidValue;
    const unsigned gy = (unsigned)(rbt < 65535 ? rbt : 65535);
    const int vec = ((uintptr_t)X % 16 == 0 && ld % 4 == 0) ? 1 : 0;
    if (kc)
        hipLaunchKernelGGL((pack_x3_kernel<true>), dim3((unsigned)gx, gy), dim3(256), 0, s, X, ld,
                           R, K, kbt, rbt, vec, out);
    else
        hipLaunchKernelGGL((pack_x3_kernel<false>), dim3((unsigned)gx, gy), dim3(256), 0, s, X, ld,
                           R, K, kbt, rbt, vec, out);
    return hipGetLastError();
}

inline hipError_t launch_packed_x3(const GemmDesc &d, hipStream_t s)
{
    if (d.num_tiles <= 0)
        return hipSuccess;
    const int sl = d.slices > 1 ? d.slices : 1;
    if (sl > 1 && (d.slice_k <= 0 || d.slice_k % 16 != 0 || sl > 65535))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((gemm_packed_kernel<PREC_BF16X3 | kPacked>), dim3(d.num_tiles, sl),
                       dim3(256), 0, s, d);
    return hipGetLastError();
}

}  // namespace dev
}  // namespace la
