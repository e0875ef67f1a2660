// MFMA fast path of the safety filter (3D swarms of supported sizes).
#pragma once

#include "swarmsf.h"
#include "sf_internal.h"

#include <string>
#include <vector>

namespace sf {

struct FastPlan {
  bool ok = false;              // the batch is covered by the fast kernels
  int R = 0;                    // robot tiles of 16
  int KS = 0;                   // k-steps of 4 coefficients
  int TQ = 0;                   // time tiles per wave
  size_t lds_bytes = 0;
};

sf_status fast_plan_build(const std::vector<DevCfg>& cfgs, const std::vector<DevProblem>& probs, FastPlan& out);
void fast_plan_free(FastPlan& p);
hipError_t fast_launch(const FastPlan& p, const LaunchArgs& a, const float* tab32, int precision);
std::string fast_last_error();

}  // namespace sf
