// Row-pass instantiations, double fields.
#include "pm_kernels.hpp"

namespace pm {
template hipError_t launch_row<double>(int, int, int, const Slot<double>*, int, const Extra<double>&, hipStream_t);
template int row_blocks<double>(int, int);
template int tile_width<double>(int);
}  // namespace pm
