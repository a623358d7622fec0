// Instantiates the tile GEMM (gemm_tile.h) for one precision, both tile
// classes; kept in its own translation unit so the precisions compile in
// parallel.
#include "gemm_tile.h"

namespace la {

hipError_t launch_gemm_fp32(const GemmDesc &d, hipStream_t s)
{
    return dev::launch_t<PREC_FP32>(d, s);
}

hipError_t launch_grouped_fp32(int akc, int bkc, int small, const GemmDesc *probs,
                             const GroupItem *items, int num_items, int grid_size, hipStream_t s)
{
    return dev::launch_grouped_t<PREC_FP32>(akc, bkc, small, probs, items, num_items, grid_size, s);
}

int tile_m_fp32(int small) { return small ? dev::Cfg<PREC_FP32 | dev::kSmall>::BM : dev::Cfg<PREC_FP32>::BM; }
int tile_n_fp32(int small) { return small ? dev::Cfg<PREC_FP32 | dev::kSmall>::BN : dev::Cfg<PREC_FP32>::BN; }

}  // namespace la
