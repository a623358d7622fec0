// Instantiates the tile GEMM (gemm_tile.h) for one precision; kept in its own
// translation unit so the three precisions compile in parallel.
#include "gemm_tile.h"

namespace la {

hipError_t launch_gemm_x6(const GemmDesc &d, hipStream_t s)
{
    return dev::launch_t<PREC_BF16X6>(d, s);
}

hipError_t launch_grouped_x6(int akc, int bkc, const GemmDesc *probs, const GroupItem *items,
                             int num_items, int grid_size, hipStream_t s)
{
    return dev::launch_grouped_t<PREC_BF16X6>(akc, bkc, probs, items, num_items, grid_size, s);
}

int tile_m_x6() { return dev::Cfg<PREC_BF16X6>::BM; }
int tile_n_x6() { return dev::Cfg<PREC_BF16X6>::BN; }

}  // namespace la
