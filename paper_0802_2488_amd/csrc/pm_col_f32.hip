// Column-pass instantiations, float fields.
#include "pm_kernels.hpp"

namespace pm {
template hipError_t launch_col<float>(int, const ColArgs<float>&, hipStream_t);
}  // namespace pm
