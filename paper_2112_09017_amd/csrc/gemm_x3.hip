// Instantiates the tile GEMM (gemm_tile.h) for one precision, both tile
// classes; kept in its own translation unit so the precisions compile in
// parallel.
#include "gemm_tile.h"

namespace la {

hipError_t launch_gemm_x3(const GemmDesc &d, hipStream_t s)
{
    return dev::launch_t<PREC_BF16X3>(d, s);
}

hipError_t launch_grouped_x3(int akc, int bkc, int small, const GemmDesc *probs,
                             const GroupItem *items, int num_items, int grid_size, hipStream_t s)
{
    return dev::launch_grouped_t<PREC_BF16X3>(akc, bkc, small, probs, items, num_items, grid_size, s);
}

size_t packed_x3_bytes(int64_t rows, int64_t k) { return dev::packed_bytes(rows, k); }

hipError_t launch_pack_x3(const float *X, int64_t ld, int kc, int64_t rows, int64_t k, void *out,
                          hipStream_t s)
{
    return dev::launch_pack_x3(X, ld, kc, rows, k, static_cast<char *>(out), s);
}

hipError_t launch_gemm_packed_x3(const GemmDesc &d, hipStream_t s)
{
    return dev::launch_packed_x3(d, s);
}

int tile_m_x3(int small) { return small ? dev::Cfg<PREC_BF16X3 | dev::kSmall>::BM : dev::Cfg<PREC_BF16X3>::BM; }
int tile_n_x3(int small) { return small ? dev::Cfg<PREC_BF16X3 | dev::kSmall>::BN : dev::Cfg<PREC_BF16X3>::BN; }

}  // namespace la
