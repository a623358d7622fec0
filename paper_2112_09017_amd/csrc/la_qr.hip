// QR factorisation (section III.B of arXiv 2112.09017) on one GPU.
//
// la_tsqr -- Algorithm tsqr for an m x n panel, n <= 128.  The rows are cut
//            into blocks of at most 256 rows (each with at least n rows).
//            One workgroup factors one block by Householder reflections with
//            the block resident in registers (each wave owns whole columns),
//            writes its R and forms its Q in place.
//            The R factors are stacked and factored again the same way (a
//            256-row block holds 256 / n of them, so the tree reduces by that
//            factor per level rather than pairwise) until one R remains.  The
//            Q factors are then multiplied down the tree: every row of a
//            level's Q times the n x n slice of the level above that belongs
//            to its block.
// la_wy   -- eq. (Yamamoto): W = Q - [I; 0] and Y = W (I - Q_1)^-1, the
//            inverse by Gauss-Jordan elimination with partial pivoting in FP64
//            in one workgroup, then one row-parallel product.
// la_caqr -- Algorithm caqr (right-looking): per panel of b columns, la_tsqr,
//            la_wy, A_l <- [R; 0] and A_r <- A_r - Y (W^T A_r) as two GEMM
//            launches (the first split along its long K = rows dimension),
//            with one panel of look-ahead: the next panel's columns are
//            updated on the caller's stream and the rest on a second stream
//            (the update is the short-K kernel of qr_update.hip); optionally
//            Q = Q_f(0) ... Q_f(last) [I; 0] afterwards.  AUTO runs
//            the products as 6xBF16: the update's K is only the panel width,
//            too short for the 3xBF16 products' per-term error (about 2^-16
//            relative) to average out.
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "la_internal.h"

namespace la {
namespace {

constexpr int kRows = 256;        // rows of one local factorisation
constexpr int kMaxPanel = 128;
constexpr int kMaxLevels = 40;
constexpr int kMaxSplits = 16;
// The next panel's product W^T A_next (b x b output, K = the panel's rows) is
// on the critical path of every panel: it takes up to 64 slices of at least
// 256 rows, so its launch is short, where the other split products (wide
// outputs) keep slices of at least 1024 rows.
constexpr int kMaxSplitsNext = 64;
constexpr int64_t kMinSliceNext = 256;
constexpr int64_t kMinSlice = 1024;
// A Gauss-Jordan pivot of I - Q_1 below this magnitude is reported as the
// breakdown of eq. (Yamamoto): Y would carry errors of order u / pivot.
constexpr double kPivotFloor = 1.0 / 65536.0;

// Row partition of a tall matrix into blocks of 256 rows.  When the last
// block would hold fewer than nc rows, the last two blocks share their rows
// evenly (at least 128 >= nc each), so every block has at least nc rows.
struct Part {
    int64_t rows;
    int64_t last_start;
    int nb;
};

__host__ __device__ inline Part make_part(int64_t rows, int nc)
{
    Part p;
    p.rows = rows;
    const int64_t nb = (rows + kRows - 1) / kRows;
    p.nb = (int)nb;
    const int64_t rem = rows - kRows * (nb - 1);
    p.last_start = (nb > 1 && rem < nc) ? kRows * (nb - 2) + (kRows + rem) / 2 : kRows * (nb - 1);
    return p;
}

__host__ __device__ inline int64_t part_start(const Part &p, int64_t i)
{
    if (i >= p.nb)
        return p.rows;
    return i == p.nb - 1 ? p.last_start : kRows * i;
}

// ---------------------------------------------------------------- kernels

// Sum over the L consecutive lanes of an aligned lane group (L = 4 or 8),
// returned in every lane of the group, by DPP moves within the group
// (lane ^ 1, lane ^ 2, then the mirror of each half-row of 8).
template <int CTRL>
__device__ inline float dpp_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <int L, typename T>
__device__ inline T group_sum(T v)
{
    static_assert(L == 4 || L == 8, "lane groups of 4 or 8");
    if constexpr (sizeof(T) == 4) {
        v += dpp_f32<0xB1>(v);        // quad_perm [1, 0, 3, 2]
        v += dpp_f32<0x4E>(v);        // quad_perm [2, 3, 0, 1]
        if constexpr (L == 8)
            v += dpp_f32<0x141>(v);   // row_half_mirror
    } else {
        v += dpp_f64<0xB1>(v);
        v += dpp_f64<0x4E>(v);
        if constexpr (L == 8)
            v += dpp_f64<0x141>(v);
    }
    return v;
}

// Sum over the 64 lanes of a wave, returned as a wave-uniform value: DPP
// within rows of 16 lanes (lane ^ 1, lane ^ 2, half-row and row mirrors),
// then row 0 into row 1 and row 2 into row 3 (row_bcast:15), rows 0 + 1 into
// rows 2 and 3 (row_bcast:31); lane 63 ends with the total.
template <int CTRL, int ROWS>
__device__ inline float bcast_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, false));
}
template <int CTRL, int ROWS>
__device__ inline double bcast_f64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ inline float wave_sum(float v)
{
    v += dpp_f32<0xB1>(v);
    v += dpp_f32<0x4E>(v);
    v += dpp_f32<0x141>(v);          // row_half_mirror
    v += dpp_f32<0x140>(v);          // row_mirror: each row of 16 holds its sum
    v += bcast_f32<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
    v += bcast_f32<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
// Maximum over the 64 lanes of a wave of an unsigned key, wave-uniform: the
// DPP steps of wave_sum with max in place of the sum (keys are >= 0, so the
// zeros that the masked broadcast rows read change nothing).
__device__ inline unsigned wave_max(unsigned v)
{
    auto mx = [](unsigned a, unsigned b) { return a > b ? a : b; };
    v = mx(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, true));
    v = mx(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, true));
    v = mx(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, true));
    v = mx(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, true));
    v = mx(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, true));
    v = mx(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, true));
    return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// wave_sum of v[first .. N - 1], the N - first sums step by step side by side
// (each step a DPP add: the moves read zero outside their rows)
template <int CTRL, int ROWS = 0xF>
__device__ inline float dppz_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, true));
}
template <int N>
__device__ inline void wave_sums(float (&v)[N], int first)
{
#pragma unroll
    for (int k = 0; k < N; ++k)
        if (k >= first)
            v[k] += dppz_f32<0xB1>(v[k]);
#pragma unroll
    for (int k = 0; k < N; ++k)
        if (k >= first)
            v[k] += dppz_f32<0x4E>(v[k]);
#pragma unroll
    for (int k = 0; k < N; ++k)
        if (k >= first)
            v[k] += dppz_f32<0x141>(v[k]);
#pragma unroll
    for (int k = 0; k < N; ++k)
        if (k >= first)
            v[k] += dppz_f32<0x140>(v[k]);
#pragma unroll
    for (int k = 0; k < N; ++k)
        if (k >= first)
            v[k] += dppz_f32<0x142, 0xA>(v[k]);
#pragma unroll
    for (int k = 0; k < N; ++k)
        if (k >= first)
            v[k] += dppz_f32<0x143, 0xC>(v[k]);
#pragma unroll
    for (int k = 0; k < N; ++k)
        if (k >= first)
            v[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[k]), 63));
}
__device__ inline double wave_sum(double v)
{
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0x141>(v);
    v += dpp_f64<0x140>(v);
    v += bcast_f64<0x142, 0xA>(v);
    v += bcast_f64<0x143, 0xC>(v);
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// Q = H_0 ... H_{nc-1} [I; 0] of a block's 64-column reflector set, in
// compact WY form: H_0 ... H_{nc-1} = I - U T U^T with U = [u_0 ... u_{nc-1}]
// (u_j zero above row j) and T upper triangular, T^-1 = diag(1/kappa) +
// N, N the strict upper part of S = U^T U; T = (I + diag(kappa) N)^-1
// diag(kappa) needs no division (a column without a reflection, kappa = 0,
// gives a zero row and column of T).  So Q = [I; 0] - U Z with Z = T U_top^T
// (U_top: the first 64 rows of U).  With T in 32 x 32 blocks, T_LH =
// -T_LL N_LH T_HH (two reflector sets joined).
//   1. each lane writes its 32 entries of U (zero above the diagonal, u_j on
//      it, the stored x below) to LDS, row r at r * 64, column j at slot
//      j ^ (r & 31), so both a row and a column of 32 are conflict-free;
//   2. three waves form the blocks (0,0), (0,1), (1,1) of S on the matrix
//      cores (v_mfma_f32_32x32x2f32, K = the block's rows) and write S
//      transposed (S[i][k] at k * 64 + i);
//   3. wave 0 forms T_LL and T_HH (lane = column), 32 steps each, side by
//      side in the two halves of the wave;
//   4. wave 1 forms T_LH on the matrix cores;
//   5. four waves form Z = T U_top^T on the matrix cores;
//   6. all eight waves form [I; 0] - U Z, 16 blocks of 32 x 32, on the matrix
//      cores and write it to Q (rows of this block; ldq).
// write_u(Us): stores this thread's entries of U (step 1), given the values it
// read from LDS before the call (the space is reused); s_kap: kappa_j in LDS
// (read before the reuse); lds: the kernel's 80 KiB buffer.
template <class WriteU>
__device__ __forceinline__ void form_q64(WriteU write_u, int nc, int lane, int w, int rows,
                                         const float *s_kap, float *lds, float *Qb, int64_t ldq)
{
    typedef float f32x16_t __attribute__((ext_vector_type(16)));
    const float kapl = lane < nc ? s_kap[lane] : 0.0f;
    __syncthreads();   // every wave is past the reflections and has its u_j / kappa
    float *Us = lds;
    float *SZ = lds + kRows * 64;
    write_u(Us);
    __syncthreads();
    const int li = lane & 31, hk = lane >> 5;
    if (w < 3) {
        const int bi = w == 2 ? 1 : 0, bj = w == 0 ? 0 : 1;
        f32x16_t acc = {};
        // 16 rows per step, the loads ahead of the products (U is zero below
        // the block's rows, so the padding adds exact zeros)
        const int kend = (rows + 15) & ~15;
        for (int k0 = 0; k0 < kend; k0 += 16) {
            float a[8], b[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int r = k0 + 2 * q + hk;
                a[q] = Us[r * 64 + ((bi * 32 + li) ^ (r & 31))];
                b[q] = Us[r * 64 + ((bj * 32 + li) ^ (r & 31))];
            }
#pragma unroll
            for (int q = 0; q < 8; ++q)
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[q], b[q], acc, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int i = bi * 32 + 8 * (e >> 2) + 4 * hk + (e & 3), j = bj * 32 + li;
            SZ[j * 64 + i] = acc[e];
        }
    }
    __syncthreads();
    // 3. T_LL and T_HH, the diagonal 32 x 32 blocks of T, in one wave: lane
    // c of half h solves (I + diag(kappa_h) N_hh) t = kappa_c e_c from the
    // last row up without a division (t_k *= kappa_k once final, then
    // t_i -= N[i][k] t_k for i < k), then stores row-major, column slot
    // c ^ r, over the S block it has read
    if (w == 0) {
        const int hf = lane >> 5, c = lane & 31;
        float *sb = SZ + hf * (32 * 64 + 32);   // S[32 hf + i][32 hf + k] at sb[k * 64 + i]
        float z[32];
#pragma unroll
        for (int i = 0; i < 32; ++i)
            z[i] = i == c ? 1.0f : 0.0f;
#pragma unroll
        for (int k = 31; k >= 0; --k) {
            const float klo = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(kapl), k));
            const float khi =
                __int_as_float(__builtin_amdgcn_readlane(__float_as_int(kapl), 32 + k));
            z[k] *= hf ? khi : klo;
            const float *sk = sb + k * 64;
#pragma unroll
            for (int i = 0; i < (k & ~3); i += 4) {
                const float4 sv = *reinterpret_cast<const float4 *>(sk + i);
                z[i] = fmaf(-sv.x, z[k], z[i]);
                z[i + 1] = fmaf(-sv.y, z[k], z[i + 1]);
                z[i + 2] = fmaf(-sv.z, z[k], z[i + 2]);
                z[i + 3] = fmaf(-sv.w, z[k], z[i + 3]);
            }
#pragma unroll
            for (int i = k & ~3; i < k; ++i)
                z[i] = fmaf(-sk[i], z[k], z[i]);
        }
        // every lane's reads of the block before any lane's stores over it
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
        for (int r = 0; r < 32; ++r)
            sb[r * 64 + (c ^ r)] = z[r];           // T_hh[r][c]
    }
    __syncthreads();
    // 4. T_LH = -T_LL (N_LH T_HH) in one wave on the matrix cores: P =
    // N_LH T_HH into the unused lower-left block (P[i][j] at i * 64 + 32 + j),
    // then -T_LL P over N_LH (T_LH[i][j] at (32 + j) * 64 + i)
    if (w == 1) {
        f32x16_t acc = {};
#pragma unroll
        for (int k0 = 0; k0 < 32; k0 += 16) {
            float a[8], b[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int kk = k0 + 2 * q + hk;
                a[q] = SZ[(32 + kk) * 64 + li];                 // N_LH[li][kk]
                b[q] = SZ[(32 + kk) * 64 + 32 + (li ^ kk)];     // T_HH[kk][li]
            }
#pragma unroll
            for (int q = 0; q < 8; ++q)
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[q], b[q], acc, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 16; ++e)
            SZ[(8 * (e >> 2) + 4 * hk + (e & 3)) * 64 + 32 + li] = acc[e];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        f32x16_t acc2 = {};
#pragma unroll
        for (int k0 = 0; k0 < 32; k0 += 16) {
            float a[8], b[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int kk = k0 + 2 * q + hk;
                a[q] = SZ[li * 64 + (kk ^ li)];                 // T_LL[li][kk]
                b[q] = SZ[kk * 64 + 32 + li];                   // P[kk][li]
            }
#pragma unroll
            for (int q = 0; q < 8; ++q)
                acc2 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[q], b[q], acc2, 0, 0, 0);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
        for (int e = 0; e < 16; ++e)
            SZ[(32 + li) * 64 + 8 * (e >> 2) + 4 * hk + (e & 3)] = -acc2[e];
    }
    __syncthreads();
    // 5. Z = T U_top^T, four 32 x 32 blocks on four waves (T_HL = 0), then Z
    // row-major over T
    f32x16_t zacc = {};
    if (w < 4) {
        const int bi = w >> 1, col = (w & 1) * 32 + li;
#pragma unroll
        for (int k0 = 0; k0 < 64; k0 += 16) {
            if (k0 < 32 * bi)
                continue;
            float a[8], b[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int kk = k0 + 2 * q + hk;
                if (bi == 1)
                    a[q] = SZ[(32 + li) * 64 + 32 + ((kk - 32) ^ li)];   // T_HH[li][kk - 32]
                else if (k0 < 32)
                    a[q] = SZ[li * 64 + (kk ^ li)];                       // T_LL[li][kk]
                else
                    a[q] = SZ[kk * 64 + li];                              // T_LH[li][kk - 32]
                b[q] = Us[col * 64 + (kk ^ (col & 31))];                  // U[col][kk]
            }
#pragma unroll
            for (int q = 0; q < 8; ++q)
                zacc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[q], b[q], zacc, 0, 0, 0);
        }
    }
    __syncthreads();
    if (w < 4) {
        const int bi = w >> 1, col = (w & 1) * 32 + li;
#pragma unroll
        for (int e = 0; e < 16; ++e)
            SZ[(32 * bi + 8 * (e >> 2) + 4 * hk + (e & 3)) * 64 + col] = zacc[e];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int bid = 2 * w + q, br = bid >> 1, bc = bid & 1;
        if (br * 32 >= rows)
            continue;
        f32x16_t acc = {};
        // 16 columns of U per step, the loads ahead of the products (U's
        // columns and Z's rows from nc on are zero)
        const int kend = (nc + 15) & ~15;
        for (int k0 = 0; k0 < kend; k0 += 16) {
            float a[8], b[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int kk = k0 + 2 * q + hk, r = br * 32 + li;
                a[q] = Us[r * 64 + (kk ^ (r & 31))];
                b[q] = SZ[kk * 64 + bc * 32 + li];
            }
#pragma unroll
            for (int q = 0; q < 8; ++q)
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[q], b[q], acc, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int rr = br * 32 + 8 * (e >> 2) + 4 * hk + (e & 3), cc = bc * 32 + li;
            if (rr < rows && cc < nc)
                Qb[(int64_t)rr * ldq + cc] = (rr == cc ? 1.0f : 0.0f) - acc[e];
        }
    }
}

// Householder QR of one row block (rows x nc, rows <= 256, 64 < nc <= 128)
// per workgroup of 1024 threads, the block in registers.  Wave w owns columns
// 8 w .. 8 w + 7; within the wave a column is held by L = 8 consecutive
// lanes, each with RPL = 32 consecutive rows, so the column dot products
// reduce inside the wave (group_sum) without a barrier.  (Blocks of at most
// 64 columns: qr_block64_kernel.)
//
// Reflection j uses u = x - beta e_j (x = column j from row j down,
// beta = -sign(x_j) ||x||) unscaled, H_j = I - kappa u u^T,
// kappa = 1 / (beta (beta - x_j)).  ||x||^2 is summed in FP32, four
// independent partial sums per lane and then across the lane group, and
// beta and kappa are formed in FP32: these sit on the one-wave chain between
// two barriers that every step waits for.  A column whose squares could
// leave the FP32 range (sum outside [2^-96, 2^96], zero or non-finite) takes
// FP64 squares, which are exact for FP32 entries, and FP64 beta and kappa.
// The owners of column j form u (zero above row j, u_j = x_j - beta on it,
// x below it) and publish it to one of two LDS buffers with kappa; after one
// barrier every column c > j forms u^T x_c and x_c -= kappa (u^T x_c) u, and
// the owners of column j + 1 (already updated) prepare the next reflection
// into the other buffer.  One barrier per step.  Column j keeps x below the
// diagonal and the pivot x_j on it; u_j, kappa and beta go to LDS arrays.
// R (row block blk of R, ld ldr) is then written from the registers, and
// Q = H_0 ... H_{nc-1} [I; 0] is formed in place and written to Q (ldq; X
// may equal Q): last reflection first (column j becomes H_j e_j once the
// columns to its right hold H_{j+1} ... e_c), one barrier per reflection.
template <int B>
__global__ __launch_bounds__(8 * B) void qr_block_kernel(const float *X, int64_t ldx, Part part,
                                                         int nc, float *Q, int64_t ldq, float *R,
                                                         int64_t ldr)
{
    static_assert(B == 128, "blocks of at most 64 columns: qr_block64_kernel");
    constexpr int CPW = 8;              // columns per wave
    constexpr int L = 64 / CPW;         // lanes per column
    constexpr int RPL = kRows / L;      // rows per lane
    // LDS: the two u buffers (alternating reflections) and u_j, kappa, beta
    constexpr int kLdsF = 2 * kRows + 3 * B;
    __shared__ __attribute__((aligned(16))) float lds[kLdsF];
    float(*ubuf)[kRows] = reinterpret_cast<float(*)[kRows]>(lds);
    float *s_u0 = lds + 2 * kRows, *s_kap = s_u0 + B, *s_beta = s_kap + B;

    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int c = w * CPW + lane / L;
    const int rlo = (lane % L) * RPL;
    const int64_t blk = blockIdx.x;
    const int64_t r0 = part_start(part, blk);
    const int rows = (int)(part_start(part, blk + 1) - r0);
    nc = __builtin_amdgcn_readfirstlane(nc);
    const bool col = c < nc;

    float f[RPL], u[RPL];
#pragma unroll
    for (int i = 0; i < RPL; ++i)
        f[i] = (col && rlo + i < rows) ? X[(r0 + rlo + i) * ldx + c] : 0.0f;

    // owners of column jn (all L lanes): reflection jn from their column.
    // The column from row jn down (zero above) goes to ubuf[jn & 1] while its
    // squares accumulate; the pivot x_jn is read back from LDS (one wave's LDS
    // accesses complete in order), and its lane overwrites it with u_jn once
    // beta is known.
    auto prepare = [&](int jn, float *ub) {
        float s4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int i = 0; i < RPL; i += 4) {
            float o[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                o[e] = rlo + i + e < jn ? 0.0f : f[i + e];
                s4[e] = fmaf(o[e], o[e], s4[e]);
            }
            *(float4 *)&ub[rlo + i] = make_float4(o[0], o[1], o[2], o[3]);
        }
        // the pivot x_jn, read back below, was stored by one of the owner lanes
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const float ss = group_sum<L>((s4[0] + s4[1]) + (s4[2] + s4[3]));
        float u0 = 0.0f, kap = 0.0f, beta = 0.0f;   // a zero column needs no reflection
        if (ss >= 0x1p-96f && ss <= 0x1p96f) {
            const float nrm = sqrtf(ss), x0 = ub[jn];
            beta = x0 >= 0.0f ? -nrm : nrm;
            u0 = x0 - beta;
            kap = 1.0f / (beta * (beta - x0));
        } else {
            double sd = 0.0;
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                const double v = rlo + i < jn ? 0.0 : (double)f[i];
                sd = fma(v, v, sd);
            }
            const double nrm = sqrt(group_sum<L>(sd));
            const double x0 = ub[jn];
            if (nrm > 0.0) {
                const double bt = x0 >= 0.0 ? -nrm : nrm;
                u0 = (float)(x0 - bt);
                kap = (float)(1.0 / (bt * (bt - x0)));
                beta = (float)bt;
            }
        }
        if (rlo == 0) {
            s_u0[jn] = u0;
            s_kap[jn] = kap;
            s_beta[jn] = beta;
        }
        if (rlo <= jn && jn < rlo + RPL)
            ub[jn] = u0;
    };
    // owners of column jn: its stored reflector (x below the diagonal) to ubuf[jn & 1]
    auto republish = [&](int jn) {
        const float u0 = s_u0[jn];
        float *ub = ubuf[jn & 1];
#pragma unroll
        for (int i = 0; i < RPL; i += 4) {
            float o[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = rlo + i + e;
                o[e] = r < jn ? 0.0f : (r == jn ? u0 : f[i + e]);
            }
            *(float4 *)&ub[rlo + i] = make_float4(o[0], o[1], o[2], o[3]);
        }
    };

    // f -= sc u with the u of the current step
    auto axpy_u = [&](float sc) {
#pragma unroll
        for (int i = 0; i < RPL; ++i)
            f[i] = fmaf(-sc, u[i], f[i]);
    };

    // f -= kappa_j (u_j^T f) u_j for this lane's column, u_j read from ub
    auto reflect = [&](const float *ub, float kap, bool apply) {
        float d4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int i = 0; i < RPL; i += 4) {
            const float4 uv = *(const float4 *)&ub[rlo + i];
            const float ua[4] = {uv.x, uv.y, uv.z, uv.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                u[i + e] = ua[e];
                d4[e] = fmaf(ua[e], f[i + e], d4[e]);
            }
        }
        const float d = group_sum<L>((d4[0] + d4[1]) + (d4[2] + d4[3]));
        axpy_u(apply ? kap * d : 0.0f);
    };

    if (c == 0)
        prepare(0, ubuf[0]);
    __syncthreads();
    for (int jv = 0; jv < nc; ++jv) {
        const int j = __builtin_amdgcn_readfirstlane(jv);
        reflect(ubuf[j & 1], s_kap[j], col && c > j);
        if (c == j + 1 && col)
            prepare(j + 1, ubuf[(j + 1) & 1]);
        __syncthreads();
    }

    float *Rb = R + blk * nc * ldr;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
        const int rr = rlo + i;
        if (col && rr < nc)
            Rb[(int64_t)rr * ldr + c] = c > rr ? f[i] : (c == rr ? s_beta[rr] : 0.0f);
    }

    if (c == nc - 1)
        republish(nc - 1);
    __syncthreads();
    for (int jv = nc - 1; jv >= 0; --jv) {
        const int j = __builtin_amdgcn_readfirstlane(jv);
        const float *ub = ubuf[j & 1];
        const float kap = s_kap[j], u0 = s_u0[j];
        float d4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int i = 0; i < RPL; i += 4) {
            const float4 uv = *(const float4 *)&ub[rlo + i];
            const float ua[4] = {uv.x, uv.y, uv.z, uv.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                u[i + e] = ua[e];
                d4[e] = fmaf(ua[e], f[i + e], d4[e]);
            }
        }
        const float d = group_sum<L>((d4[0] + d4[1]) + (d4[2] + d4[3]));
        if (col && c > j) {
            axpy_u(kap * d);
        } else if (c == j) {
            // column j = H_j e_j = e_j - kappa u_j u (u is zero above row j)
            const float s2 = kap * u0;
#pragma unroll
            for (int i = 0; i < RPL; ++i)
                f[i] = rlo + i == j ? 1.0f : 0.0f;
            axpy_u(s2);
        }
        if (c == j - 1)
            republish(j - 1);
        __syncthreads();
    }

#pragma unroll
    for (int i = 0; i < RPL; ++i)
        if (col && rlo + i < rows)
            Q[(r0 + rlo + i) * ldq + c] = f[i];
}

// Householder QR of one row block (rows x nc, rows <= 256, nc <= 64) per
// workgroup of 8 waves, the block in registers with the rows across the
// lanes: lane l holds rows 4 l .. 4 l + 3 of its wave's 8 columns (wave w:
// columns 8 w .. 8 w + 7).  A column vector such as u_j is then spread over
// the lanes of every wave alike, so the wave that forms a reflection keeps
// u_j in registers and a column dot product is a sum over the wave
// (wave_sum: DPP and one readlane).
//
// Reflection j uses u = x - beta e_j (x = column j from row j down,
// beta = -sign(x_j) ||x||) unscaled, H_j = I - kappa u u^T,
// kappa = 1 / (beta (beta - x_j)); ||x||^2, beta and kappa in FP32, or in
// FP64 (squares exact for FP32 entries) when the FP32 sum of squares leaves
// [2^-96, 2^96] (zero or non-finite included).  Each wave applies the
// reflections in order: those of the waves to its left as they are
// published (u_j from LDS, then u_j^T x_c and x_c -= kappa (u^T x_c) u for its
// 8 columns), then its own, each formed from its column, published and
// applied at once to the wave's later columns.  A reflection is published
// by a workgroup-scope release store of the count of published reflections
// after u_j, kappa_j and beta_j are in LDS; a wave waits for reflection j
// with acquire loads of that count.  No barrier until all reflections are
// done: a wave starts its own columns once it has applied the last
// reflection of the wave to its left.  Every wait is for a reflection that a
// wave to its left publishes without waiting on this one; it is bounded all
// the same, and a wait that runs out marks the block's R with NaN instead of
// hanging.  Column j keeps x below the diagonal and the pivot x_j on it.
// R (row block blk of R, ld ldr) is then written from the registers, and
// Q = H_0 ... H_{nc-1} [I; 0] is formed in compact WY form (form_q64) and
// written to Q (ldq); X may equal Q.
__global__ __launch_bounds__(512) void qr_block64_kernel(const float *X, int64_t ldx, Part part,
                                                         int nc, float *Q, int64_t ldq, float *R,
                                                         int64_t ldr)
{
    constexpr int CPW = 8;              // columns per wave
    constexpr int RPL = kRows / 64;     // rows per lane
    // LDS: u_j of every reflection (each stays until every wave has applied
    // it), u_j's pivot entry, kappa, beta and the count of published
    // reflections; the same space then holds U and S / Z of the compact WY
    // form (80 KiB in all, so two workgroups share a CU)
    constexpr int kLdsF = kRows * 64 + 64 * 64;
    static_assert(64 * kRows + 3 * 64 + 1 <= kLdsF, "reflection buffers fit the WY space");
    __shared__ __attribute__((aligned(16))) float lds[kLdsF];
    float(*ubuf)[kRows] = reinterpret_cast<float(*)[kRows]>(lds);
    float *s_u0 = lds + 64 * kRows, *s_kap = s_u0 + 64, *s_beta = s_kap + 64;
    int *s_pub = reinterpret_cast<int *>(s_beta + 64);

    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int rlo = lane * RPL;
    const int64_t blk = blockIdx.x;
    const int64_t r0 = part_start(part, blk);
    const int rows = (int)(part_start(part, blk + 1) - r0);
    nc = __builtin_amdgcn_readfirstlane(nc);
    const int own = __builtin_amdgcn_readfirstlane(w * CPW);   // the wave's first column

    float f[CPW][RPL];
    const bool vec = own + CPW <= nc && (ldx & 3) == 0 && ((uintptr_t)X & 15) == 0;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
        const int r = rlo + i;
        if (vec) {
            float4 a = make_float4(0.0f, 0.0f, 0.0f, 0.0f), b = a;
            if (r < rows) {
                const float *xr = X + (r0 + r) * ldx + own;
                a = *(const float4 *)xr;
                b = *(const float4 *)(xr + 4);
            }
            f[0][i] = a.x, f[1][i] = a.y, f[2][i] = a.z, f[3][i] = a.w;
            f[4][i] = b.x, f[5][i] = b.y, f[6][i] = b.z, f[7][i] = b.w;
        } else {
#pragma unroll
            for (int cc = 0; cc < CPW; ++cc)
                f[cc][i] = (own + cc < nc && r < rows) ? X[(r0 + r) * ldx + own + cc] : 0.0f;
        }
    }

    // x_c -= kappa (u^T x_c) u for columns cc >= first (compile time) of the
    // wave; the column sums go through wave_sum's steps side by side
    auto apply = [&](const float (&u)[RPL], float kap, int first) {
        float d[CPW];
#pragma unroll
        for (int cc = 0; cc < CPW; ++cc) {
            d[cc] = 0.0f;
            if (cc < first)
                continue;
#pragma unroll
            for (int i = 0; i < RPL; ++i)
                d[cc] = fmaf(u[i], f[cc][i], d[cc]);
        }
        wave_sums<CPW>(d, first);
#pragma unroll
        for (int cc = 0; cc < CPW; ++cc) {
            if (cc < first)
                continue;
            const float sc = kap * d[cc];
#pragma unroll
            for (int i = 0; i < RPL; ++i)
                f[cc][i] = fmaf(-sc, u[i], f[cc][i]);
        }
    };

    if (t == 0)
        *s_pub = 0;
    __syncthreads();
    bool timed_out = false;
    if (own < nc) {
        // the reflections of the waves to the left, as they are published
        for (int jv = 0; jv < own; ++jv) {
            const int j = __builtin_amdgcn_readfirstlane(jv);
            int spins = 0;
            while (__hip_atomic_load(s_pub, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) <= j) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > (1 << 22)) {
                    timed_out = true;
                    break;
                }
            }
            const float4 uv = *(const float4 *)&ubuf[j][rlo];
            const float u[RPL] = {uv.x, uv.y, uv.z, uv.w};
            apply(u, s_kap[j], 0);
        }
        // this wave's reflections
#pragma unroll
        for (int cj = 0; cj < CPW; ++cj) {
            const int j = own + cj;
            if (j >= nc)
                break;
            float o[RPL], s4 = 0.0f;
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                o[i] = rlo + i < j ? 0.0f : f[cj][i];
                s4 = fmaf(o[i], o[i], s4);
            }
            const float ss = wave_sum(s4);
            // x_j: row j is entry j % 4 (= cj % 4) of lane j / 4
            const float x0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(f[cj][cj & 3]),
                                                                      j >> 2));
            float u0 = 0.0f, kap = 0.0f, beta = 0.0f;   // a zero column needs no reflection
            if (ss >= 0x1p-96f && ss <= 0x1p96f) {
                const float nrm = sqrtf(ss);
                beta = x0 >= 0.0f ? -nrm : nrm;
                u0 = x0 - beta;
                kap = 1.0f / (beta * (beta - x0));
            } else {
                double sd = 0.0;
#pragma unroll
                for (int i = 0; i < RPL; ++i)
                    sd = fma((double)o[i], (double)o[i], sd);
                const double nrm = sqrt(wave_sum(sd));
                if (nrm > 0.0) {
                    const double bt = x0 >= 0.0f ? -nrm : nrm;
                    u0 = (float)((double)x0 - bt);
                    kap = (float)(1.0 / (bt * (bt - (double)x0)));
                    beta = (float)bt;
                }
            }
            if (rlo + (cj & 3) == j)
                o[cj & 3] = u0;
            *(float4 *)&ubuf[j][rlo] = make_float4(o[0], o[1], o[2], o[3]);
            if (lane == 0) {
                s_u0[j] = u0;
                s_kap[j] = kap;
                s_beta[j] = beta;
            }
            __hip_atomic_store(s_pub, j + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            apply(o, kap, cj + 1);
        }
    }
    __syncthreads();
    if (timed_out)
        f[0][0] = NAN;

    float *Rb = R + blk * nc * ldr;
#pragma unroll
    for (int cc = 0; cc < CPW; ++cc) {
        const int c = own + cc;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int rr = rlo + i;
            if (c < nc && rr < nc)
                Rb[(int64_t)rr * ldr + c] = c > rr ? f[cc][i] : (c == rr ? s_beta[rr] : 0.0f);
        }
    }

    float u0c[CPW];
#pragma unroll
    for (int cc = 0; cc < CPW; ++cc)
        u0c[cc] = own + cc < nc ? s_u0[own + cc] : 0.0f;
    form_q64(
        [&](float *Us) {
#pragma unroll
            for (int cc = 0; cc < CPW; ++cc) {
                const int c = own + cc;
#pragma unroll
                for (int i = 0; i < RPL; ++i) {
                    const int r = rlo + i;
                    const float v = (c >= nc || r < c) ? 0.0f : (r == c ? u0c[cc] : f[cc][i]);
                    Us[r * 64 + (c ^ (r & 31))] = v;
                }
            }
        },
        nc, lane, w, rows, s_kap, lds, Q + r0 * ldq, ldq);
}

// out[r, :] = (in[r, :] - sub [r < nc] e_r^T) M_b for every row r < part.rows,
// with M_b = Mb + b * nc * nc (nc x nc, ld nc) for the partition block b
// holding row r, or M_0 for every row when single; wout (optional) receives
// in[r, :] - sub e_r^T.  Workgroup (b, y) takes rows 32 y .. 32 y + 31 of
// block b, staged in LDS with M_b; 8 threads per row, each forming B / 8 of
// its outputs.  out may equal in: every row is read whole before any
// thread of the workgroup writes.
template <int B>
__global__ __launch_bounds__(256) void rowmul_kernel(const float *in, int64_t ldi, Part part,
                                                     int single, int nc,
                                                     const float *__restrict__ Mb, float *out,
                                                     int64_t ldo, float *wout, int64_t ldw,
                                                     int sub)
{
    constexpr int CG = 8, CPT = B / CG, RPB = 256 / CG;
    __shared__ float xs[RPB * (B + 1)];
    __shared__ __attribute__((aligned(16))) float ms[B * B];
    const int t = threadIdx.x, rr = t / CG, cg = t % CG;
    const int64_t b = blockIdx.x;
    const int64_t rbase = part_start(part, b) + (int64_t)blockIdx.y * RPB;
    const int64_t rend = part_start(part, b + 1);
    if (rbase >= rend)
        return;
    const float *M = Mb + (single ? 0 : b * nc * nc);
    for (int idx = t; idx < nc * nc; idx += 256)
        ms[(idx / nc) * B + idx % nc] = M[idx];
    for (int idx = t; idx < RPB * B; idx += 256) {
        const int i = idx / B, k = idx % B;
        const int64_t r = rbase + i;
        float v = 0.0f;
        if (r < rend && k < nc) {
            v = in[r * ldi + k];
            if (sub && r == k)
                v -= 1.0f;
            if (wout)
                wout[r * ldw + k] = v;
        }
        xs[i * (B + 1) + k] = v;
    }
    __syncthreads();
    const int64_t r = rbase + rr;
    if (r >= rend)
        return;
    float acc[CPT];
#pragma unroll
    for (int e = 0; e < CPT; ++e)
        acc[e] = 0.0f;
    for (int k = 0; k < nc; ++k) {
        const float xv = xs[rr * (B + 1) + k];
#pragma unroll
        for (int e = 0; e < CPT; e += 4) {
            const float4 mv = *(const float4 *)&ms[k * B + cg * CPT + e];
            acc[e] = fmaf(xv, mv.x, acc[e]);
            acc[e + 1] = fmaf(xv, mv.y, acc[e + 1]);
            acc[e + 2] = fmaf(xv, mv.z, acc[e + 2]);
            acc[e + 3] = fmaf(xv, mv.w, acc[e + 3]);
        }
    }
#pragma unroll
    for (int e = 0; e < CPT; ++e)
        if (cg * CPT + e < nc)
            out[r * ldo + cg * CPT + e] = acc[e];
}

// Minv = (I - Q_1)^-1 for the top nc x nc block Q_1 of Q (ld ldq), by
// Gauss-Jordan elimination with partial pivoting in FP64 in LDS (512
// threads; thread (i0, c) owns column c of rows i0, i0 + 512 / B, ...).
// Rows are not moved: step k pivots on the unused row p_k with the largest
// |M[p_k][k]| (compared in FP32, ties to the lower row; every wave finds it
// itself), scales row p_k and eliminates column k from the other rows, with
// one barrier between reading the operands and writing the results and one
// after.  The array then holds (P M)^-1 in pivot order, and
// Minv[k][p_c] = B[p_k][c].  Rounded to FP32 (nc x nc, ld nc).  flag[0] = 1
// if a pivot is below kPivotFloor in magnitude or not finite.
template <int B>
__global__ __launch_bounds__(512) void wy_inverse_kernel(const float *__restrict__ Q, int64_t ldq,
                                                         int nc, float *__restrict__ Minv,
                                                         int *flag)
{
    constexpr int LD = B + 1;
    constexpr int RP = 512 / B;   // row phases: thread (i0, c) takes rows i0 + RP q
    constexpr int RO = B / RP;    // rows owned per thread
    constexpr int RL = B / 64;    // rows per lane in the pivot search
    __shared__ double M[B * LD];
    __shared__ int piv[B];
    const int t = threadIdx.x, lane = t & 63;
    const int cc = t % B, i0 = t / B;
    nc = __builtin_amdgcn_readfirstlane(nc);
    const bool ccol = cc < nc;
    for (int i = i0; i < nc; i += RP)
        if (ccol)
            M[i * LD + cc] = (i == cc ? 1.0 : 0.0) - (double)Q[(int64_t)i * ldq + cc];
    bool used[RL];
#pragma unroll
    for (int q = 0; q < RL; ++q)
        used[q] = false;
    __syncthreads();
    for (int kv = 0; kv < nc; ++kv) {
        const int k = __builtin_amdgcn_readfirstlane(kv);
        // pivot (every wave): key = FP32 magnitude bits (low 7 mantissa bits dropped) | (127 - row)
        unsigned key = 0;
#pragma unroll
        for (int q = 0; q < RL; ++q) {
            const int r = lane + 64 * q;
            if (r < nc && !used[q]) {
                const unsigned kk = ((unsigned)__float_as_int((float)fabs(M[r * LD + k])) & ~0x7Fu) |
                                    (unsigned)(127 - r);
                key = kk > key ? kk : key;
            }
        }
        key = wave_max(key);
        const int p = __builtin_amdgcn_readfirstlane(127 - (int)(key & 0x7Fu));
#pragma unroll
        for (int q = 0; q < RL; ++q)
            if (lane + 64 * q == p)
                used[q] = true;
        const double pv = M[p * LD + k];
        const double inv = 1.0 / pv;
        const double prc = ccol ? M[p * LD + cc] : 0.0;
        double mic[RO], fic[RO];
#pragma unroll
        for (int q = 0; q < RO; ++q) {
            const int i = i0 + RP * q;
            mic[q] = (i < nc && ccol) ? M[i * LD + cc] : 0.0;
            fic[q] = i < nc ? M[i * LD + k] : 0.0;
        }
        if (t == 0) {
            piv[k] = p;
            if (!(fabs(pv) >= kPivotFloor && isfinite(pv)))
                flag[0] = 1;
        }
        __syncthreads();
        if (ccol) {
#pragma unroll
            for (int q = 0; q < RO; ++q) {
                const int i = i0 + RP * q;
                if (i >= nc)
                    continue;
                double v;
                if (i == p)
                    v = cc == k ? inv : prc * inv;
                else
                    v = cc == k ? -fic[q] * inv : fma(-fic[q] * inv, prc, mic[q]);
                M[i * LD + cc] = v;
            }
        }
        __syncthreads();
    }
    for (int k = i0; k < nc; k += RP)
        if (ccol)
            Minv[(int64_t)k * nc + piv[cc]] = (float)M[piv[k] * LD + cc];
}

// A (ml x nc, lda) <- [R; 0] with R upper triangular (nc x nc, ldr).
__global__ void place_r_kernel(float *A, int64_t lda, int64_t ml, int nc, const float *R,
                               int64_t ldr)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= ml * nc)
        return;
    const int64_t i = idx / nc;
    const int j = (int)(idx % nc);
    A[i * lda + j] = (i < nc && j >= i) ? R[i * ldr + j] : 0.0f;
}

// Q (m x n, ldq) <- [I_n; 0].
__global__ void eye_kernel(float *Q, int64_t ldq, int64_t m, int64_t n)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= m * n)
        return;
    const int64_t i = idx / n, j = idx % n;
    Q[i * ldq + j] = i == j ? 1.0f : 0.0f;
}

__global__ void clear_flag_kernel(int *flag) { flag[threadIdx.x] = 0; }

// out (rows x cols, ldo) = sum over s of parts[s] (rows x cols, ld cols), in order.
__global__ void sum_slices_kernel(const float *__restrict__ parts, int splits, int64_t rows,
                                  int64_t cols, float *__restrict__ out, int64_t ldo)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= rows * cols)
        return;
    float acc = 0.0f;
    for (int s = 0; s < splits; ++s)
        acc += parts[(int64_t)s * rows * cols + idx];
    out[(idx / cols) * ldo + idx % cols] = acc;
}

unsigned grid1d(int64_t count) { return (unsigned)((count + 255) / 256); }

// ----------------------------------------------------------------- planning

size_t al(size_t b) { return align_up256(b); }

// Levels of the TSQR tree for an m x nc panel: level 0 factors the rows of
// A, level l >= 1 factors the stacked R factors of level l - 1
// (rows[l] = nb[l - 1] * nc rows, held in buffer l of the workspace, which
// then receives that level's Q in place).  The top level has one block.
struct TsqrPlan {
    int levels;                 // index of the top level
    int64_t rows[kMaxLevels];
    int nb[kMaxLevels];
    size_t off[kMaxLevels];     // byte offset of buffer l (l >= 1)
    size_t bytes;
};

TsqrPlan tsqr_plan(int64_t m, int nc)
{
    TsqrPlan p;
    memset(&p, 0, sizeof p);
    p.rows[0] = m;
    p.nb[0] = make_part(m, nc).nb;
    int l = 0;
    size_t b = 0;
    while (p.nb[l] > 1 && l + 1 < kMaxLevels) {
        ++l;
        p.rows[l] = (int64_t)p.nb[l - 1] * nc;
        p.nb[l] = make_part(p.rows[l], nc).nb;
        p.off[l] = b;
        b += al((size_t)p.rows[l] * nc * sizeof(float));
    }
    p.levels = l;
    p.bytes = b;
    return p;
}

template <int B>
hipError_t tsqr_run_b(const float *A, int64_t lda, int nc, float *Q, int64_t ldq, float *R,
                      int64_t ldr, char *ws, const TsqrPlan &tp, hipStream_t s)
{
    const int L = tp.levels;
    auto buf = [&](int l) { return (float *)(ws + tp.off[l]); };
    for (int l = 0; l <= L; ++l) {
        const Part pl = make_part(tp.rows[l], nc);
        const float *in = l == 0 ? A : buf(l);
        const int64_t ldi = l == 0 ? lda : nc;
        float *qo = l == 0 ? Q : buf(l);
        const int64_t ldo = l == 0 ? ldq : nc;
        float *ro = l == L ? R : buf(l + 1);
        const int64_t ldro = l == L ? ldr : nc;
        if constexpr (B == 64)
            hipLaunchKernelGGL(qr_block64_kernel, dim3(pl.nb), dim3(512), 0, s, in, ldi, pl, nc,
                               qo, ldo, ro, ldro);
        else
            hipLaunchKernelGGL(qr_block_kernel<B>, dim3(pl.nb), dim3(8 * B), 0, s, in, ldi, pl,
                               nc, qo, ldo, ro, ldro);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    for (int l = L - 1; l >= 0; --l) {
        const Part pl = make_part(tp.rows[l], nc);
        float *io = l == 0 ? Q : buf(l);
        const int64_t ld = l == 0 ? ldq : nc;
        hipLaunchKernelGGL(rowmul_kernel<B>, dim3(pl.nb, kRows / 32), dim3(256), 0, s,
                           (const float *)io, ld, pl, 0, nc, (const float *)buf(l + 1), io, ld,
                           (float *)nullptr, (int64_t)0, 0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t tsqr_run(const float *A, int64_t lda, int nc, float *Q, int64_t ldq, float *R,
                    int64_t ldr, char *ws, const TsqrPlan &tp, hipStream_t s)
{
    if (nc <= 64)
        return tsqr_run_b<64>(A, lda, nc, Q, ldq, R, ldr, ws, tp, s);
    return tsqr_run_b<128>(A, lda, nc, Q, ldq, R, ldr, ws, tp, s);
}

// W = Q - [I; 0], Y = W (I - Q_1)^-1 for an m x nc Q; Minv: nc x nc scratch.
template <int B>
hipError_t wy_run_b(int64_t m, int nc, const float *Q, int64_t ldq, float *W, int64_t ldw,
                    float *Y, int64_t ldy, float *Minv, int *flag, hipStream_t s)
{
    hipLaunchKernelGGL(wy_inverse_kernel<B>, dim3(1), dim3(512), 0, s, Q, ldq, nc, Minv, flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const Part p = make_part(m, nc);
    hipLaunchKernelGGL(rowmul_kernel<B>, dim3(p.nb, kRows / 32), dim3(256), 0, s, Q, ldq, p, 1,
                       nc, (const float *)Minv, Y, ldy, W, ldw, 1);
    return hipGetLastError();
}

hipError_t wy_run(int64_t m, int nc, const float *Q, int64_t ldq, float *W, int64_t ldw, float *Y,
                  int64_t ldy, float *Minv, int *flag, hipStream_t s)
{
    if (nc <= 64)
        return wy_run_b<64>(m, nc, Q, ldq, W, ldw, Y, ldy, Minv, flag, s);
    return wy_run_b<128>(m, nc, Q, ldq, W, ldw, Y, ldy, Minv, flag, s);
}

size_t wy_bytes(int nc) { return al((size_t)nc * nc * sizeof(float)) + 256; }

// Split count for a GEMM whose output (rows x cols) is small beside its K:
// enough slices to give every compute unit about two tiles, each slice at
// least min_slice deep, at most max_splits.
int splits_for(int prec, int64_t rows, int64_t cols, int64_t K, int num_cus, int max_splits,
               int64_t min_slice)
{
    GemmDesc d;
    memset(&d, 0, sizeof d);
    d.M = rows;
    d.N = cols;
    d.K = K;
    d.lda = K;
    d.ldb = cols;
    d.ldc = cols;
    d.a_kcontig = 0;
    d.b_kcontig = 0;
    gemm_finalize(d, prec);
    const int64_t tiles = std::max<int64_t>(1, (int64_t)d.tiles_m * d.tiles_n);
    int64_t sp = (2 * num_cus + tiles - 1) / tiles;
    sp = std::min<int64_t>(sp, std::max<int64_t>(1, K / min_slice));
    return (int)std::max<int64_t>(1, std::min<int64_t>(sp, max_splits));
}

// Split-K GEMMs Z (rows x cols, ld cols) = X^T V with X (K x rows, ldx) and
// V (K x cols, ldv): the slices are independent problems of one grouped
// persistent launch (so they run side by side), each writing its own slice
// of parts (max_splits x rows x cols scratch), summed in slice order.  The
// descriptors of every such product of a factorisation are built on the host
// first and uploaded once.
struct SplitGemm {
    int first_prob, first_item, num_items, splits, small;
    float *Z, *parts;
    int64_t rows, cols;
};

struct SplitBatch {
    std::vector<GemmDesc> probs;
    std::vector<GroupItem> items;
    std::vector<SplitGemm> gemms;
};

void add_split(SplitBatch &sb, int prec, const float *X, int64_t ldx, const float *V, int64_t ldv,
               int64_t rows, int64_t cols, int64_t K, float *Z, float *parts, int num_cus,
               int max_splits, int64_t min_slice)
{
    const int splits = splits_for(prec, rows, cols, K, num_cus, max_splits, min_slice);
    const int64_t ks = (K + splits - 1) / splits;
    SplitGemm g;
    g.first_prob = (int)sb.probs.size();
    g.first_item = (int)sb.items.size();
    g.splits = splits;
    g.Z = Z;
    g.parts = parts;
    g.rows = rows;
    g.cols = cols;
    g.small = 0;
    for (int sp = 0; sp < splits; ++sp) {
        const int64_t k0 = sp * ks;
        const int64_t kl = std::min<int64_t>(ks, K - k0);
        GemmDesc d;
        memset(&d, 0, sizeof d);
        d.A = X + k0 * ldx;
        d.lda = ldx;
        d.a_kcontig = 0;
        d.B = V + k0 * ldv;
        d.ldb = ldv;
        d.b_kcontig = 0;
        d.C = splits == 1 ? Z : parts + (size_t)sp * rows * cols;
        d.ldc = cols;
        d.M = rows;
        d.N = cols;
        d.K = kl > 0 ? kl : 0;
        d.alpha = 1.0f;
        gemm_finalize(d, prec);
        g.small = d.small;   // the same for every slice (it depends on M and N only)
        const int pid = (int)sb.probs.size() - g.first_prob;
        sb.probs.push_back(d);
        for (int tt = 0; tt < d.num_tiles; ++tt)
            sb.items.push_back(GroupItem{pid, tt});
    }
    g.num_items = (int)sb.items.size() - g.first_item;
    sb.gemms.push_back(g);
}

// Upper bound of the items one split product of `cols` output columns adds
// (rows <= 128, so one tile row): splits * tiles <= 2 num_cus + tiles, and
// at most kMaxSplits * tiles; num_cus is taken as at most 1024.
size_t split_items_bound(int64_t cols)
{
    const size_t tiles = (size_t)((cols + 127) / 128);
    return std::min<size_t>(kMaxSplits * tiles, 2048 + tiles);
}

hipError_t run_split(int prec, const SplitBatch &sb, int which, const GemmDesc *probs_dev,
                     const GroupItem *items_dev, int num_cus, hipStream_t s)
{
    const SplitGemm &g = sb.gemms[which];
    hipError_t e = launch_gemm_grouped(prec, 0, 0, g.small, probs_dev + g.first_prob,
                                       items_dev + g.first_item, g.num_items, num_cus, s);
    if (e != hipSuccess || g.splits == 1)
        return e;
    hipLaunchKernelGGL(sum_slices_kernel, dim3(grid1d(g.rows * g.cols)), dim3(256), 0, s,
                       (const float *)g.parts, g.splits, g.rows, g.cols, g.Z, g.cols);
    return hipGetLastError();
}

// C (rows x cols, ldc) -= X Z with X (rows x K, ldx) and Z (K x cols, ld cols):
// K is the panel width, so the short-K kernel streams C once with its reads
// issued ahead of the products.
hipError_t gemm_sub(int prec, const float *X, int64_t ldx, const float *Z, int64_t rows,
                    int64_t cols, int64_t K, float *C, int64_t ldc, hipStream_t s)
{
    return launch_short_update(prec, X, ldx, Z, cols, C, ldc, rows, cols, (int)K, s);
}

// Workspace of la_caqr, in order: Qr (m x b), Rr (b x b), the TSQR tree of an
// m x b panel, Minv + flag, W and Y (m x n each with Q; without Q two m x b
// buffers each, alternating between panels), then for the critical stream Z0
// (b x b) and its split-K parts, for the trailing stream Z1 (b x n) and its
// parts, and the split-K descriptors.
struct CaqrWs {
    size_t qr, rr, tree, wy, w, y, z0, parts0, z1, parts1, probs, items, bytes;
};

CaqrWs caqr_ws(int64_t m, int64_t n, int b, int want_q)
{
    CaqrWs w;
    size_t o = 0;
    w.qr = o;
    o += al((size_t)m * b * sizeof(float));
    w.rr = o;
    o += al((size_t)b * b * sizeof(float));
    w.tree = o;
    o += tsqr_plan(m, b).bytes;
    w.wy = o;
    o += wy_bytes(b);
    const size_t wyb = al((size_t)m * (want_q ? n : 2 * b) * sizeof(float));
    w.w = o;
    o += wyb;
    w.y = o;
    o += wyb;
    w.z0 = o;
    o += al((size_t)b * b * sizeof(float));
    // a split product's K is at most m, so it takes at most m / min_slice slices
    const size_t sp_next = (size_t)std::min<int64_t>(kMaxSplitsNext,
                                                     std::max<int64_t>(1, m / kMinSliceNext));
    const size_t sp_wide = (size_t)std::min<int64_t>(kMaxSplits,
                                                     std::max<int64_t>(1, m / kMinSlice));
    w.parts0 = o;
    o += al(sp_next * b * b * sizeof(float));
    w.z1 = o;
    o += al((size_t)b * n * sizeof(float));
    w.parts1 = o;
    o += al(sp_wide * b * n * sizeof(float));
    // split-K descriptors: next-panel and trailing products of every panel,
    // and the Q pass
    const int64_t np = (n + b - 1) / b;
    // (a next-panel product has one tile row and one tile column, b <= 128)
    const size_t nwide = (size_t)np * (want_q ? 2 : 1);
    w.probs = o;
    o += al(((size_t)np * sp_next + nwide * sp_wide) * sizeof(GemmDesc));
    w.items = o;
    o += al(((size_t)np * sp_next + nwide * split_items_bound(n)) * sizeof(GroupItem));
    w.bytes = o;
    return w;
}

// The second stream and the two events of one la_caqr call.
struct LookAhead {
    hipStream_t s1 = nullptr;
    hipEvent_t wy_ready = nullptr, trail_done = nullptr;
    ~LookAhead()
    {
        if (wy_ready)
            (void)hipEventDestroy(wy_ready);
        if (trail_done)
            (void)hipEventDestroy(trail_done);
        if (s1)
            (void)hipStreamDestroy(s1);
    }
};

la_status read_flag(const int *flag, hipStream_t s, const char *who)
{
    int h = 0;
    LA_HIP(hipMemcpyAsync(&h, flag, sizeof h, hipMemcpyDeviceToHost, s), who);
    LA_HIP(hipStreamSynchronize(s), who);
    if (h) {
        set_error("%s: I - Q_1 is singular or nearly so (a pivot below 2^-16): the WY form of "
                  "eq. (Yamamoto) breaks down", who);
        return LA_ERR_BREAKDOWN;
    }
    return LA_OK;
}

la_status check_ws(void *ws, size_t ws_bytes, size_t need, const char *who)
{
    if (need > 0 && !ws) {
        set_error("%s: NULL workspace", who);
        return LA_ERR_INVALID_ARG;
    }
    if (((uintptr_t)ws & 255u) != 0) {
        set_error("%s: workspace must be 256-byte aligned", who);
        return LA_ERR_INVALID_ARG;
    }
    if (ws_bytes < need) {
        set_error("%s: workspace %zu bytes, need %zu", who, ws_bytes, need);
        return LA_ERR_OUT_OF_MEMORY;
    }
    return LA_OK;
}

}  // namespace
}  // namespace la

using namespace la;

extern "C" {

size_t la_tsqr_workspace_size(int64_t m, int64_t n)
{
    if (n < 1 || n > kMaxPanel || m < n)
        return 0;
    return std::max<size_t>(256, tsqr_plan(m, (int)n).bytes);
}

la_status la_tsqr(la_context *ctx, int64_t m, int64_t n, const float *A, int64_t lda, float *Q,
                  int64_t ldq, float *R, int64_t ldr, void *workspace, size_t ws_bytes,
                  void *hip_stream)
{
    static const char *who = "la_tsqr";
    set_error("%s", "");
    if (n < 1 || n > kMaxPanel || m < n || lda < n || ldq < n || ldr < n) {
        set_error("%s: bad shape (m %lld, n %lld (1..128, <= m), lda %lld, ldq %lld, ldr %lld)",
                  who, (long long)m, (long long)n, (long long)lda, (long long)ldq,
                  (long long)ldr);
        return LA_ERR_SHAPE;
    }
    if (!ctx || !A || !Q || !R) {
        set_error("%s: NULL argument", who);
        return LA_ERR_INVALID_ARG;
    }
    const TsqrPlan tp = tsqr_plan(m, (int)n);
    la_status st = check_ws(workspace, ws_bytes, tp.bytes, who);
    if (st != LA_OK)
        return st;
    const size_t ab = extent_bytes(m, n, lda), qb = extent_bytes(m, n, ldq),
                 rb = extent_bytes(n, n, ldr);
    if (overlaps(Q, qb, A, ab) || overlaps(R, rb, A, ab) || overlaps(Q, qb, R, rb) ||
        overlaps(A, ab, workspace, tp.bytes) || overlaps(Q, qb, workspace, tp.bytes) ||
        overlaps(R, rb, workspace, tp.bytes)) {
        set_error("%s: A, Q, R and the workspace must not overlap", who);
        return LA_ERR_INVALID_ARG;
    }
    LA_HIP(hipSetDevice(ctx->device), "la_tsqr: hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    LA_HIP(tsqr_run(A, lda, (int)n, Q, ldq, R, ldr, (char *)workspace, tp, s), "la_tsqr: launch");
    LA_HIP(hipStreamSynchronize(s), "la_tsqr: sync");
    return LA_OK;
}

size_t la_wy_workspace_size(int64_t n)
{
    if (n < 1 || n > kMaxPanel)
        return 0;
    return wy_bytes((int)n);
}

la_status la_wy(la_context *ctx, int64_t m, int64_t n, const float *Q, int64_t ldq, float *W,
                int64_t ldw, float *Y, int64_t ldy, void *workspace, size_t ws_bytes,
                void *hip_stream)
{
    static const char *who = "la_wy";
    set_error("%s", "");
    if (n < 1 || n > kMaxPanel || m < n || ldq < n || ldw < n || ldy < n) {
        set_error("%s: bad shape (m %lld, n %lld (1..128, <= m), ldq %lld, ldw %lld, ldy %lld)",
                  who, (long long)m, (long long)n, (long long)ldq, (long long)ldw,
                  (long long)ldy);
        return LA_ERR_SHAPE;
    }
    if (!ctx || !Q || !W || !Y) {
        set_error("%s: NULL argument", who);
        return LA_ERR_INVALID_ARG;
    }
    const size_t need = wy_bytes((int)n);
    la_status st = check_ws(workspace, ws_bytes, need, who);
    if (st != LA_OK)
        return st;
    const size_t qb = extent_bytes(m, n, ldq), wb = extent_bytes(m, n, ldw),
                 yb = extent_bytes(m, n, ldy);
    if (overlaps(W, wb, Q, qb) || overlaps(Y, yb, Q, qb) || overlaps(W, wb, Y, yb) ||
        overlaps(Q, qb, workspace, need) || overlaps(W, wb, workspace, need) ||
        overlaps(Y, yb, workspace, need)) {
        set_error("%s: Q, W, Y and the workspace must not overlap", who);
        return LA_ERR_INVALID_ARG;
    }
    LA_HIP(hipSetDevice(ctx->device), "la_wy: hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    float *Minv = (float *)workspace;
    int *flag = (int *)((char *)workspace + al((size_t)n * n * sizeof(float)));
    hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(1), 0, s, flag);
    LA_HIP(hipGetLastError(), "la_wy: clear");
    LA_HIP(wy_run(m, (int)n, Q, ldq, W, ldw, Y, ldy, Minv, flag, s), "la_wy: launch");
    return read_flag(flag, s, who);
}

size_t la_caqr_workspace_size(int64_t m, int64_t n, int panel, int want_q)
{
    if (n < 1 || m < n || panel < 1 || panel > kMaxPanel)
        return 0;
    return caqr_ws(m, n, (int)std::min<int64_t>(panel, n), want_q).bytes;
}

la_status la_caqr(la_context *ctx, int64_t m, int64_t n, float *A, int64_t lda, float *Q,
                  int64_t ldq, int panel, void *workspace, size_t ws_bytes, la_precision prec,
                  void *hip_stream)
{
    static const char *who = "la_caqr";
    set_error("%s", "");
    if (n < 1 || m < n || lda < n || (Q && ldq < n) || panel < 1 || panel > kMaxPanel) {
        set_error("%s: bad shape (m %lld, n %lld, lda %lld, ldq %lld, panel %d (1..128))", who,
                  (long long)m, (long long)n, (long long)lda, (long long)ldq, panel);
        return LA_ERR_SHAPE;
    }
    if (!valid_prec(prec)) {
        set_error("%s: unknown precision %d", who, (int)prec);
        return LA_ERR_INVALID_ARG;
    }
    if (!ctx || !A) {
        set_error("%s: NULL argument", who);
        return LA_ERR_INVALID_ARG;
    }
    const int b = (int)std::min<int64_t>(panel, n);
    const CaqrWs cw = caqr_ws(m, n, b, Q != nullptr);
    la_status st = check_ws(workspace, ws_bytes, cw.bytes, who);
    if (st != LA_OK)
        return st;
    const size_t ab = extent_bytes(m, n, lda);
    if (overlaps(A, ab, workspace, cw.bytes) ||
        (Q && (overlaps(Q, extent_bytes(m, n, ldq), A, ab) ||
               overlaps(Q, extent_bytes(m, n, ldq), workspace, cw.bytes)))) {
        set_error("%s: A, Q and the workspace must not overlap", who);
        return LA_ERR_INVALID_ARG;
    }
    const int pr = resolve_prec(prec, PREC_BF16X6);
    LA_HIP(hipSetDevice(ctx->device), "la_caqr: hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    char *ws = (char *)workspace;
    float *Qr = (float *)(ws + cw.qr), *Rr = (float *)(ws + cw.rr);
    float *Minv = (float *)(ws + cw.wy);
    int *flag = (int *)(ws + cw.wy + al((size_t)b * b * sizeof(float)));
    float *Wb = (float *)(ws + cw.w), *Yb = (float *)(ws + cw.y);
    float *Z0 = (float *)(ws + cw.z0), *P0 = (float *)(ws + cw.parts0);
    float *Z1 = (float *)(ws + cw.z1), *P1 = (float *)(ws + cw.parts1);
    const int64_t ldwy = Q ? n : b;
    const int64_t np = (n + b - 1) / b;
    auto wpan = [&](int64_t jp) { return Q ? Wb + jp * b * (n + 1) : Wb + (jp & 1) * m * b; };
    auto ypan = [&](int64_t jp) { return Q ? Yb + jp * b * (n + 1) : Yb + (jp & 1) * m * b; };

    // Look-ahead: panel j's reflector is applied first to panel j + 1's
    // columns on the caller's stream (the critical path: the next panel is
    // factored right after), and to the columns beyond on a second stream,
    // where it overlaps the next panels' factorisations.  The next-panel
    // update of panel j waits for the trailing update of panel j - 1 (which
    // covers those columns); a trailing update waits for its panel's W and Y.
    SplitBatch sb;
    std::vector<int> zn(np, -1), zt(np, -1), zq(np, -1);
    for (int64_t jp = 0; jp < np; ++jp) {
        const int64_t c = jp * b, ml = m - c;
        const int nc = (int)std::min<int64_t>(b, n - c);
        const int64_t nx = c + nc, nc2 = std::min<int64_t>(b, n - nx), rest = nx + nc2;
        if (nc2 > 0) {
            zn[jp] = (int)sb.gemms.size();
            add_split(sb, pr, wpan(jp), ldwy, A + c * lda + nx, lda, nc, nc2, ml, Z0, P0,
                      ctx->num_cus, kMaxSplitsNext, kMinSliceNext);
        }
        if (rest < n) {
            zt[jp] = (int)sb.gemms.size();
            add_split(sb, pr, wpan(jp), ldwy, A + c * lda + rest, lda, nc, n - rest, ml, Z1, P1,
                      ctx->num_cus, kMaxSplits, kMinSlice);
        }
    }
    if (Q)
        for (int64_t jp = np - 1; jp >= 0; --jp) {
            const int64_t c = jp * b, ml = m - c;
            const int nc = (int)std::min<int64_t>(b, n - c);
            zq[jp] = (int)sb.gemms.size();
            add_split(sb, pr, ypan(jp), n, Q + c * ldq + c, ldq, nc, n - c, ml, Z1, P1,
                      ctx->num_cus, kMaxSplits, kMinSlice);
        }
    if (sb.probs.size() * sizeof(GemmDesc) > cw.items - cw.probs ||
        sb.items.size() * sizeof(GroupItem) > cw.bytes - cw.items) {
        set_error("%s: split-K descriptors exceed their workspace region", who);
        return LA_ERR_OUT_OF_MEMORY;
    }
    GemmDesc *probs_dev = (GemmDesc *)(ws + cw.probs);
    GroupItem *items_dev = (GroupItem *)(ws + cw.items);
    if (!sb.probs.empty()) {
        LA_HIP(hipMemcpyAsync(probs_dev, sb.probs.data(), sb.probs.size() * sizeof(GemmDesc),
                              hipMemcpyHostToDevice, s),
               "la_caqr: descriptors");
        LA_HIP(hipMemcpyAsync(items_dev, sb.items.data(), sb.items.size() * sizeof(GroupItem),
                              hipMemcpyHostToDevice, s),
               "la_caqr: items");
    }
    LookAhead la;
    LA_HIP(hipStreamCreateWithFlags(&la.s1, hipStreamNonBlocking), "la_caqr: stream");
    LA_HIP(hipEventCreateWithFlags(&la.wy_ready, hipEventDisableTiming), "la_caqr: event");
    LA_HIP(hipEventCreateWithFlags(&la.trail_done, hipEventDisableTiming), "la_caqr: event");
    // the second stream starts after everything already queued on the caller's
    LA_HIP(hipEventRecord(la.wy_ready, s), "la_caqr: record");
    LA_HIP(hipStreamWaitEvent(la.s1, la.wy_ready, 0), "la_caqr: wait");

    hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(1), 0, s, flag);
    LA_HIP(hipGetLastError(), "la_caqr: clear");
    bool trail_pending = false;   // a trailing update was queued since the last wait on it
    for (int64_t jp = 0; jp < np; ++jp) {
        const int64_t c = jp * b, ml = m - c;
        const int nc = (int)std::min<int64_t>(b, n - c);
        const int64_t nx = c + nc, nc2 = std::min<int64_t>(b, n - nx), rest = nx + nc2;
        float *Ap = A + c * lda + c;
        float *W = wpan(jp), *Y = ypan(jp);
        const TsqrPlan tp = tsqr_plan(ml, nc);
        LA_HIP(tsqr_run(Ap, lda, nc, Qr, b, Rr, b, ws + cw.tree, tp, s), "la_caqr: tsqr");
        LA_HIP(wy_run(ml, nc, Qr, b, W, ldwy, Y, ldwy, Minv, flag, s), "la_caqr: wy");
        hipLaunchKernelGGL(place_r_kernel, dim3(grid1d(ml * nc)), dim3(256), 0, s, Ap, lda, ml,
                           nc, (const float *)Rr, (int64_t)b);
        LA_HIP(hipGetLastError(), "la_caqr: place R");
        if (rest < n)
            LA_HIP(hipEventRecord(la.wy_ready, s), "la_caqr: record");
        if (nc2 > 0) {
            if (trail_pending) {
                LA_HIP(hipStreamWaitEvent(s, la.trail_done, 0), "la_caqr: wait");
                trail_pending = false;
            }
            // next panel's columns <- Q_f^T (...) = (...) - Y (W^T (...))
            LA_HIP(run_split(pr, sb, zn[jp], probs_dev, items_dev, ctx->num_cus, s),
                   "la_caqr: W^T A_next");
            LA_HIP(gemm_sub(pr, Y, ldwy, Z0, ml, nc2, nc, A + c * lda + nx, lda, s),
                   "la_caqr: next-panel update");
        }
        if (rest < n) {
            LA_HIP(hipStreamWaitEvent(la.s1, la.wy_ready, 0), "la_caqr: wait");
            LA_HIP(run_split(pr, sb, zt[jp], probs_dev, items_dev, ctx->num_cus, la.s1),
                   "la_caqr: W^T A_rest");
            LA_HIP(gemm_sub(pr, Y, ldwy, Z1, ml, n - rest, nc, A + c * lda + rest, lda, la.s1),
                   "la_caqr: trailing update");
            LA_HIP(hipEventRecord(la.trail_done, la.s1), "la_caqr: record");
            trail_pending = true;
        }
    }
    // join: the caller's stream continues after the last trailing update
    LA_HIP(hipEventRecord(la.trail_done, la.s1), "la_caqr: record");
    LA_HIP(hipStreamWaitEvent(s, la.trail_done, 0), "la_caqr: wait");
    if (Q) {
        hipLaunchKernelGGL(eye_kernel, dim3(grid1d(m * n)), dim3(256), 0, s, Q, ldq, m, n);
        LA_HIP(hipGetLastError(), "la_caqr: eye");
        for (int64_t jp = np - 1; jp >= 0; --jp) {
            const int64_t c = jp * b, ml = m - c;
            const int nc = (int)std::min<int64_t>(b, n - c);
            float *Qc = Q + c * ldq + c;
            // Q[c:, c:] <- Q_f Q[c:, c:] = Q[c:, c:] - W (Y^T Q[c:, c:])
            LA_HIP(run_split(pr, sb, zq[jp], probs_dev, items_dev, ctx->num_cus, s),
                   "la_caqr: Y^T Q");
            LA_HIP(gemm_sub(pr, wpan(jp), n, Z1, ml, n - c, nc, Qc, ldq, s), "la_caqr: Q");
        }
    }
    return read_flag(flag, s, who);
}

}  // extern "C"
