// Short-K update C <- C - Y Z of Algorithm caqr (section III.B): the panel's
// block reflector applied to the columns on its right, A_r - Y (W^T A_r),
// and to Q in the Q pass.  K is the panel width (at most 128), so each
// output element takes K multiply-adds against 8 bytes of C moved: the
// update streams C through HBM and its products are short.
//
// One workgroup (four wave64s, 2 x 2) per 128 x 128 tile of C.  The tile's
// slices of Y (128 x K) and Z (K x 128) are loaded first and the 64 values
// of C each lane updates right after them, so the C reads are in flight
// while Y and Z are split into bf16 terms in LDS and multiplied; the
// accumulators start at zero and the tile is written as C - acc.  The MFMAs
// see the same k blocks, fragments and product order as the generic tile
// GEMM (gemm_tile.h), and C - acc is the generic epilogue's alpha acc + beta
// E with alpha = -1, beta = 1, so every element is the same as with la_gemm
// on the 128 x 128 tile class.
#include "gemm_tile.h"

namespace la {
namespace dev {
namespace {

constexpr int kUT = 128;        // tile rows and columns
constexpr int kUK = 64;         // k per LDS stage
constexpr int kULs = kUK + 4;   // LDS row stride (floats): conflict-free fragment reads

struct UpdateArgs {
    const float *Y;
    int64_t ldy;
    const float *Z;
    int64_t ldz;
    float *C;
    int64_t ldc;
    int64_t rows, cols;
    int K, tiles_m, tiles_n, yvec, zvec;
    int full_m, full_n;   // whole 128 x 128 tiles along each side (interior launch)
    int all_edge;         // the edge launch covers every tile
};

// Word 3 of a raw (untyped) buffer resource on gfx9-family GPUs: data format
// 32 bits, no swizzle, no index stride.
constexpr int kBufWord3 = 0x00020000;

// Y (rows x K, k contiguous) and Z (K x cols, k the row index) of one 64-k
// stage into LDS: Y rows as they are, Z transposed (column-major), both with
// stride kULs, so an MFMA fragment (8 consecutive k of one row or column) is
// two 16-byte reads.  Zero past the edges and past K.
__device__ __forceinline__ void update_stage(const UpdateArgs &p, int64_t r0, int64_t c0, int k0,
                                             float *ys, float *zs, int t)
{
    float4 yv[8], zv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int idx = t + 256 * u;
        const int row = idx >> 4, k4 = (idx & 15) * 4;
        const int64_t gr = r0 + row;
        const int gk = k0 + k4;
        if (p.yvec && gr < p.rows && gk + 3 < p.K) {
            yv[u] = *reinterpret_cast<const float4 *>(p.Y + gr * p.ldy + gk);
        } else {
            float v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e)
                v[e] = (gr < p.rows && gk + e < p.K) ? p.Y[gr * p.ldy + gk + e] : 0.0f;
            yv[u] = make_float4(v[0], v[1], v[2], v[3]);
        }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int idx = t + 256 * u;
        const int kk = idx >> 5, c4 = (idx & 31) * 4;
        const int gk = k0 + kk;
        const int64_t gc = c0 + c4;
        if (p.zvec && gk < p.K && gc + 3 < p.cols) {
            zv[u] = *reinterpret_cast<const float4 *>(p.Z + (int64_t)gk * p.ldz + gc);
        } else {
            float v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e)
                v[e] = (gk < p.K && gc + e < p.cols) ? p.Z[(int64_t)gk * p.ldz + gc + e] : 0.0f;
            zv[u] = make_float4(v[0], v[1], v[2], v[3]);
        }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int idx = t + 256 * u;
        *reinterpret_cast<float4 *>(ys + (idx >> 4) * kULs + (idx & 15) * 4) = yv[u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int idx = t + 256 * u;
        const int kk = idx >> 5, c4 = (idx & 31) * 4;
        zs[(c4 + 0) * kULs + kk] = zv[u].x;
        zs[(c4 + 1) * kULs + kk] = zv[u].y;
        zs[(c4 + 2) * kULs + kk] = zv[u].z;
        zs[(c4 + 3) * kULs + kk] = zv[u].w;
    }
}

// The products of one 16-k block for this wave's 2 x 2 blocks of 32 x 32.
// Lane l holds op(Y)(row l & 31, 8 (l >> 5) .. + 7) of each A block and the
// same k of column l & 31 of each B block: the fragment of
// v_mfma_f32_32x32x16_bf16, and for v_mfma_f32_32x32x2f32 (which takes one
// k per lane half) MFMA e pairs k = e and k = 8 + e, as the generic tile does.
template <int PREC>
__device__ __forceinline__ void update_block(const float *ys, const float *zs, int kb, int wm,
                                             int wn, int lane, f32x16 (&acc)[2][2])
{
    const int k = kb * 16 + (lane >> 5) * 8;
    float a[2][8], b[2][8];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const float *src = ys + (wm * 64 + i * 32 + (lane & 31)) * kULs + k;
        const float4 lo = reinterpret_cast<const float4 *>(src)[0];
        const float4 hi = reinterpret_cast<const float4 *>(src)[1];
        a[i][0] = lo.x; a[i][1] = lo.y; a[i][2] = lo.z; a[i][3] = lo.w;
        a[i][4] = hi.x; a[i][5] = hi.y; a[i][6] = hi.z; a[i][7] = hi.w;
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const float *src = zs + (wn * 64 + j * 32 + (lane & 31)) * kULs + k;
        const float4 lo = reinterpret_cast<const float4 *>(src)[0];
        const float4 hi = reinterpret_cast<const float4 *>(src)[1];
        b[j][0] = lo.x; b[j][1] = lo.y; b[j][2] = lo.z; b[j][3] = lo.w;
        b[j][4] = hi.x; b[j][5] = hi.y; b[j][6] = hi.z; b[j][7] = hi.w;
    }
    if constexpr (PREC == PREC_FP32) {
#pragma unroll
        for (int e = 0; e < 8; ++e)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i][e], b[j][e], acc[i][j],
                                                                     0, 0, 0);
    } else {
        using P = Products<PREC>;
        constexpr int T = PREC == PREC_BF16X6 ? 3 : 2;
        u32x4 at[2][T], bt[2][T];
#pragma unroll
        for (int i = 0; i < 2; ++i)
            Split<PREC>::run(a[i], at[i]);
#pragma unroll
        for (int j = 0; j < 2; ++j)
            Split<PREC>::run(b[j], bt[j]);
#pragma unroll
        for (int q = 0; q < P::n; ++q)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                        __builtin_bit_cast(bf16x8, at[i][P::a[q]]),
                        __builtin_bit_cast(bf16x8, bt[j][P::b[q]]), acc[i][j], 0, 0, 0);
    }
}

// Tile of a workgroup.  Interior launch: the full_m x full_n whole tiles.
// Edge launch: the partial last tile column (rows of whole tiles), then the
// partial last tile row (every column), or every tile with all_edge.
template <bool EDGE>
__device__ __forceinline__ void update_tile(const UpdateArgs &p, int &tm, int &tn)
{
    const int bid = blockIdx.x;
    if (!EDGE) {
        tm = bid / p.full_n;
        tn = bid % p.full_n;
    } else if (p.all_edge) {
        tm = bid / p.tiles_n;
        tn = bid % p.tiles_n;
    } else {
        const bool pn = p.full_n < p.tiles_n;
        if (pn && bid < p.full_m) {
            tm = bid;
            tn = p.full_n;
        } else {
            tm = p.full_m;
            tn = bid - (pn ? p.full_m : 0);
        }
    }
}

// EDGE = false: whole tiles only, C addressed through a buffer resource at
// the tile's first element: one per-lane byte offset (the lane's row and
// column) plus a wave-uniform offset per element, so the 64 addresses cost
// no registers between the loads and the stores.  EDGE = true: tiles that
// cross an edge, with clamped loads and guarded stores.
template <int PREC, bool EDGE>
__global__ void __launch_bounds__(256, (EDGE ? 1 : 2)) short_update_kernel(UpdateArgs p)
{
    __shared__ __attribute__((aligned(16))) float ys[kUT * kULs];
    __shared__ __attribute__((aligned(16))) float zs[kUT * kULs];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w >> 1, wn = w & 1;
    int tm, tn;
    update_tile<EDGE>(p, tm, tn);
    const int64_t r0 = (int64_t)tm * kUT, c0 = (int64_t)tn * kUT;
    // this lane's elements: rows rb + 32 i + 8 (e >> 2) + (e & 3), columns cb + 32 j
    const int64_t rb = r0 + wm * 64 + (lane >> 5) * 4;
    const int64_t cb = c0 + wn * 64 + (lane & 31);

    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
            acc[i][j] = f32x16{};
    float cv[2][2][16];
    constexpr bool interior = !EDGE;
    const int voff = (int)(((rb - r0) * p.ldc + (cb - c0)) * 4);
    const __amdgpu_buffer_rsrc_t crs =
        __builtin_amdgcn_make_buffer_rsrc(p.C + r0 * p.ldc + c0, 0, 0x7fffffff, kBufWord3);
    for (int k0 = 0; k0 < p.K; k0 += kUK) {
        update_stage(p, r0, c0, k0, ys, zs, t);
        if (k0 == 0) {
            // C after the first stage's loads: in flight under the products.
            // Past the edge a clamped in-range element is read and not used.
            if constexpr (interior) {
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
#pragma unroll
                        for (int e = 0; e < 16; ++e) {
                            const int so = (int)(((i * 32 + (e >> 2) * 8 + (e & 3)) * p.ldc + j * 32) * 4);
                            cv[i][j][e] = __builtin_bit_cast(
                                float, __builtin_amdgcn_raw_buffer_load_b32(crs, voff, so, 0));
                        }
            } else {
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        const int64_t col = cb + j * 32;
                        const int64_t cc = col < p.cols ? col : p.cols - 1;
#pragma unroll
                        for (int e = 0; e < 16; ++e) {
                            int64_t row = rb + i * 32 + (e >> 2) * 8 + (e & 3);
                            row = row < p.rows ? row : p.rows - 1;
                            cv[i][j][e] = p.C[row * p.ldc + cc];
                        }
                    }
            }
        }
        __syncthreads();
        const int kbs = min(kUK, p.K - k0 + 15) / 16;
        for (int kb = 0; kb < kbs; ++kb)
            update_block<PREC>(ys, zs, kb, wm, wn, lane, acc);
        __syncthreads();
    }
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    if constexpr (interior) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int so = (int)(((i * 32 + (e >> 2) * 8 + (e & 3)) * p.ldc + j * 32) * 4);
                    const float v = -acc[i][j][e] + cv[i][j][e];
                    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), crs,
                                                          voff, so, 0);
                }
    } else {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int64_t col = cb + j * 32;
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int64_t row = rb + i * 32 + (e >> 2) * 8 + (e & 3);
                    if (row < p.rows && col < p.cols)
                        p.C[row * p.ldc + col] = -acc[i][j][e] + cv[i][j][e];
                }
            }
    }
}

}  // namespace
}  // namespace dev

hipError_t launch_short_update(int prec, const float *Y, int64_t ldy, const float *Z, int64_t ldz,
                               float *C, int64_t ldc, int64_t rows, int64_t cols, int K,
                               hipStream_t s)
{
    if (rows <= 0 || cols <= 0 || K <= 0)
        return hipSuccess;
    if (K > 128)
        return hipErrorInvalidValue;
    dev::UpdateArgs p;
    p.Y = Y;
    p.ldy = ldy;
    p.Z = Z;
    p.ldz = ldz;
    p.C = C;
    p.ldc = ldc;
    p.rows = rows;
    p.cols = cols;
    p.K = K;
    const int64_t tiles_m = (rows + dev::kUT - 1) / dev::kUT;
    const int64_t tiles_n = (cols + dev::kUT - 1) / dev::kUT;
    if (tiles_m * tiles_n > 0x7fffffff)
        return hipErrorInvalidValue;
    p.tiles_m = (int)tiles_m;
    p.tiles_n = (int)tiles_n;
    p.yvec = ((uintptr_t)Y % 16 == 0) && (ldy % 4 == 0);
    p.zvec = ((uintptr_t)Z % 16 == 0) && (ldz % 4 == 0);
    // buffer offsets within one 128-row tile must stay below 2^31 bytes
    const bool cbuf = ldc <= (int64_t)1 << 21;
    p.full_m = cbuf ? (int)(rows / dev::kUT) : 0;
    p.full_n = cbuf ? (int)(cols / dev::kUT) : 0;
    p.all_edge = cbuf ? 0 : 1;
    const int64_t inner = (int64_t)p.full_m * p.full_n;
    const int64_t edge = tiles_m * tiles_n - inner;
    const dim3 block(256);
    if (inner > 0) {
        const dim3 grid((unsigned)inner);
        if (prec == PREC_FP32)
            hipLaunchKernelGGL((dev::short_update_kernel<PREC_FP32, false>), grid, block, 0, s, p);
        else if (prec == PREC_BF16X3)
            hipLaunchKernelGGL((dev::short_update_kernel<PREC_BF16X3, false>), grid, block, 0, s, p);
        else
            hipLaunchKernelGGL((dev::short_update_kernel<PREC_BF16X6, false>), grid, block, 0, s, p);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    if (edge > 0) {
        const dim3 grid((unsigned)edge);
        if (prec == PREC_FP32)
            hipLaunchKernelGGL((dev::short_update_kernel<PREC_FP32, true>), grid, block, 0, s, p);
        else if (prec == PREC_BF16X3)
            hipLaunchKernelGGL((dev::short_update_kernel<PREC_BF16X3, true>), grid, block, 0, s, p);
        else
            hipLaunchKernelGGL((dev::short_update_kernel<PREC_BF16X6, true>), grid, block, 0, s, p);
    }
    return hipGetLastError();
}

}  // namespace la
