// MFMA fast path of the safety filter.
#include "sf_fast.h"

namespace sf {

static thread_local std::string g_fast_err;

std::string fast_last_error() { return g_fast_err; }

sf_status fast_plan_build(const std::vector<DevCfg>& cfgs, const std::vector<DevProblem>& probs, FastPlan& out) {
  (void)cfgs; (void)probs;
  out.ok = false;
  return SF_OK;
}

void fast_plan_free(FastPlan& p) { p.ok = false; }

hipError_t fast_launch(const FastPlan& p, const LaunchArgs& a, const float* tab32, int precision) {
  (void)p; (void)a; (void)tab32; (void)precision;
  return hipErrorNotSupported;
}

}  // namespace sf
