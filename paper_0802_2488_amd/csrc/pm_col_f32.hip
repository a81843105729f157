// Column-pass instantiations, float fields.
#include "pm_kernels.hpp"

namespace pm {
template hipError_t launch_col<float>(int, int, int, const Slot<float>*, int, const Extra<float>&, hipStream_t);
}  // namespace pm
