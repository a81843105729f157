// Column-pass instantiations, double fields.
#include "pm_kernels.hpp"

namespace pm {
template hipError_t launch_col<double>(int, int, int, const Slot<double>*, int, const Extra<double>&, hipStream_t);
}  // namespace pm
