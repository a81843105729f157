// Row-pass instantiations, double fields.
#include "pm_kernels.hpp"

namespace pm {
template hipError_t launch_row<double>(int, const RowArgs<double>&, hipStream_t);
template int row_grid<double>(int);
template int tile_width<double>(int);
}  // namespace pm
