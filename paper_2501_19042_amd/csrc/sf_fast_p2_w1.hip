// MFMA kernel instances: fp16 basis operands, with the workspace rows.
#include "sf_fast_kernel.h"

namespace sf {

hipError_t fast_launch_single_p2_w1(const FastPlan& p, const LaunchArgs& a, const float* tab32, const uint4* a16,
                                     int W) {
  return fastk::launch_single_mp<2, 1>(p, a, tab32, a16, W);
}

hipError_t fast_launch_batched_p2_w1(const FastPlan& p, const LaunchArgs& a, const float* tab32, const uint4* a16,
                                      const int* grid, const int* W, int cls_mask) {
  return fastk::launch_batched_mp<2, 1>(p, a, tab32, a16, grid, W, cls_mask);
}

}  // namespace sf
