// MFMA fast path of the safety filter (3D swarms of supported sizes).
#pragma once

#include "swarmsf.h"
#include "sf_internal.h"

#include <string>
#include <vector>

namespace sf {

// Work items of one robot-tile class (R tiles of 16 robots) in a persistent launch sequence.
struct FastClass {
  int R = 0;
  int offset = 0;                       // first item in FastPlan::d_items_sorted
  int n_items = 0;
  int grid = 0;                         // default persistent workgroups
  size_t lds_bytes[3][3] = {};          // LDS per workgroup for W = 2, 3, 4 and fp32 / bf16 / fp16
};

struct FastPlan {
  bool ok = false;              // the batch is covered by the fast kernels
  int R = 0;                    // robot tiles of 16 (single-shape batches)
  int KS = 0;                   // k-steps of 4 coefficients (maximum over the batch)
  int Wp[4] = {4, 4, 4, 4};     // default waves per workgroup (2, 3 or 4) per precision; time tiles
                                // are dealt round-robin to the waves
  size_t lds_bytes[3][3] = {};          // LDS per workgroup for W = 2, 3, 4 and fp32 / bf16 / fp16
  // persistent launch over a ragged batch (mixed swarm sizes, or requested)
  bool batched = false;
  WorkItem* d_items_sorted = nullptr;   // work items by class, most expensive first within a class
  int* d_queue = nullptr;               // work-queue heads (one per class), reset by a kernel before each launch
  FastClass cls[2];                     // 17-32 robots, then up to 16 (empty classes left out)
  int n_cls = 0;
  int ncu = 0;
  int tuned_w[4] = {0, 0, 0, 0};        // autotuned waves per workgroup per precision (0 = not tuned)
  int tuned_wc[4][2] = {};              // persistent launches: autotuned waves per workgroup per precision
  int tuned_gc[4][2] = {};              // and class, and workgroups (0 = not tuned / the class default)
  bool ws = false;                      // some config has a workspace: kernels with its rows, and
                                        // 2 or 3 waves per workgroup
};

// Whether the MFMA kernels cover a config: 3D, up to 32 robots, degree <= 15, horizon <= 256, and
// an LDS plan within 160 KB.
bool fast_cfg_covered(const DevCfg& c);
// Plan over the given work items (all of covered configs); `ok` stays false otherwise.
sf_status fast_plan_build(const std::vector<DevCfg>& cfgs, const std::vector<DevProblem>& probs,
                          const std::vector<WorkItem>& items, bool persistent, FastPlan& out);
void fast_plan_free(FastPlan& p);
hipError_t fast_launch(const FastPlan& p, const LaunchArgs& a, const float* tab32, const void* a16, int precision);
// Persistent launch sequence: the classes in cls_mask (bit c = class c), with per-class waves per
// workgroup W[c] and workgroup counts grid[c] (0 = the class's default).
hipError_t fast_launch_batched(const FastPlan& p, const LaunchArgs& a, const float* tab32, const void* a16,
                               int precision, const int* grid, const int* W, int cls_mask);
hipError_t fast_launch_single(const FastPlan& p, const LaunchArgs& a, const float* tab32, const void* a16,
                              int precision, int W);

// Number of 16-byte entries of the 16-bit S1 basis-operand table of one config (per precision).
int64_t a16_entries(const DevCfg& c);
// Fill the table for one config: [tile][basis][instruction][lane] of 8 x 16-bit values.
void a16_fill(const DevCfg& c, const double* P3, int precision, uint16_t* out);
// fp32 basis operands: [tile][basis][S1 A operand, S4 B operand scaled by rho][lane][4] floats
// (16-byte entries).
int64_t a32_entries(const DevCfg& c);
void a32_fill(const DevCfg& c, const double* P3, float* out);
std::string fast_last_error();

}  // namespace sf
