// Instantiates the tile GEMM (gemm_tile.h) for one precision, both tile
// classes; kept in its own translation unit so the precisions compile in
// parallel.
#include "gemm_tile.h"

namespace la {

hipError_t launch_gemm_x6(const GemmDesc &d, hipStream_t s)
{
    return dev::launch_t<PREC_BF16X6>(d, s);
}

hipError_t launch_grouped_x6(int akc, int bkc, int small, const GemmDesc *probs,
                             const GroupItem *items, int num_items, int grid_size, hipStream_t s)
{
    return dev::launch_grouped_t<PREC_BF16X6>(akc, bkc, small, probs, items, num_items, grid_size, s);
}

int tile_m_x6(int small) { return small ? dev::Cfg<PREC_BF16X6 | dev::kSmall>::BM : dev::Cfg<PREC_BF16X6>::BM; }
int tile_n_x6(int small) { return small ? dev::Cfg<PREC_BF16X6 | dev::kSmall>::BN : dev::Cfg<PREC_BF16X6>::BN; }

}  // namespace la
