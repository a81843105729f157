// Row-pass instantiations, float fields.
#include "pm_kernels.hpp"

namespace pm {
template hipError_t launch_row<float>(int, const RowArgs<float>&, hipStream_t);
template int row_grid<float>(int);
template int tile_width<float>(int);
}  // namespace pm
