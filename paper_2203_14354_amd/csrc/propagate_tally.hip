// propagate_tally.hip -- the transport kernel with its hit-map and gradient
// tallies summed per workgroup in LDS (kForwardTally), compiled in a
// translation unit of its own so that its code does not change the code
// generated for the other variants.
#include "transport.h"

namespace xp {

hipError_t launch_propagate_tally(const LaunchArgs& a, bool grad, bool offsets, int block,
                                  int grid, size_t lds, hipStream_t s) {
  const dim3 g(grid), b(block);
  if (grad && offsets)
    hipLaunchKernelGGL((propagate_kernel<kForwardTally, true, false, false, true>), g, b, lds, s, a);
  else if (grad)
    hipLaunchKernelGGL((propagate_kernel<kForwardTally, true, false, false, false>), g, b, lds, s, a);
  else if (offsets)
    hipLaunchKernelGGL((propagate_kernel<kForwardTally, false, false, false, true>), g, b, lds, s, a);
  else
    hipLaunchKernelGGL((propagate_kernel<kForwardTally, false, false, false, false>), g, b, lds, s, a);
  return hipGetLastError();
}

hipError_t max_blocks_per_cu_tally(int block, size_t lds_bytes, int* out) {
  // the gradient variant: the larger register footprint of the two
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      out, reinterpret_cast<const void*>(propagate_kernel<kForwardTally, true, false, false, false>),
      block, lds_bytes);
}

}  // namespace xp
