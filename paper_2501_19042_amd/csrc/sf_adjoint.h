// Adjoint (reverse-mode) kernel of the unrolled safety-filter iterations.
#pragma once

#include "sf_internal.h"

namespace sf {

struct AdjointArgs {
  const DevCfg* cfgs;
  const void* tab;
  const DevProblem* probs;
  const WorkItem* items;
  int32_t n_items;
  const void* xi_bar;
  const void* bvals;
  int32_t iters;
  const void* ckpt;
  int32_t ckpt_every;
  int64_t ckpt_stride;
  const void* g_xi_out;
  const void* g_lam_out;
  const void* g_resid;
  const void* w_fpr;            // [S] cotangent of the fixed-point residual sum, or NULL
  void* g_xi0;
  void* g_lam0;
  void* g_xi_bar;
  void* states;                 // scratch: n_items * state_stride elements
  int64_t state_stride;         // 2 (ckpt_every + 1) * largest n * D * m of the batch (xi, then lambda)
  int32_t tile;
  size_t lds_bytes;
  hipStream_t stream;
};

template <typename T>
hipError_t launch_adjoint(const AdjointArgs& a);

size_t adjoint_lds_bytes(const DevCfg& c, int tile, size_t elem);

}  // namespace sf
