// Row-pass instantiations, float fields.
#include "pm_kernels.hpp"

namespace pm {
template hipError_t launch_row<float>(int, int, int, const Slot<float>*, int, const Extra<float>&, hipStream_t);
template int row_blocks<float>(int, int);
template int tile_width<float>(int);
}  // namespace pm
