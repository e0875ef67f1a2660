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

// MFMA adjoint path (fp32; 3D, up to 16 robots, degree <= 15, horizon <= 256, no workspace rows).
// The forward states of a checkpoint segment are recomputed by the forward MFMA kernel into
// `states` ([len + 1][2][stride], stride = the batch's coefficient count); the cotangents of (xi,
// lambda, xi_bar) are carried between segments in `carry` ([3][stride]).
struct AdjFastArgs {
  const DevCfg* cfgs;
  const float* tab;
  const void* a32;               // basis operand tables of the MFMA kernels
  const DevProblem* probs;
  const WorkItem* items;
  int32_t n_items;
  const float* states;
  int64_t stride;
  int32_t s0, len, iters;        // the segment's first iteration and length, total iterations
  const float* w_fpr;
  const float* g_xi_out;         // first segment without the final-residual term: carries start here
  const float* g_lam_out;
  bool init;                     // initialise the carries from g_xi_out / g_lam_out (else read them)
  float* carry;
  const float* pend;             // cotangent of xi^{K-1} from the final-residual term, or NULL
  float* g_xi0;                  // last segment (s0 = 0): outputs instead of carries (any may be NULL)
  float* g_lam0;
  float* g_xi_bar;
  bool last;
  size_t lds_bytes;
  hipStream_t stream;
};

// Whether a config is covered by the MFMA adjoint path, its LDS bytes, and the reverse sweep over
// one segment.
bool adjoint_fast_supported(const DevCfg& c);
size_t adjoint_fast_lds_bytes(const DevCfg& c);
hipError_t launch_adjoint_fast(const AdjFastArgs& a, int KS);
// The final-residual term for that path (see sf_adjoint.hip): one workgroup per (sample, time tile
// of a.tile steps) with per-tile partials in `part` ([n_tiles][2][stride]) and an in-order
// reduction into the carries (gxi, glam, gxb) and pend.
size_t adjoint_resid_tile_lds_bytes(const DevCfg& c, int tile);
hipError_t launch_adjoint_resid_tiles(const AdjointArgs& a, const float* states, int64_t stride, int slot,
                                      float* part, int n_tiles, float* carry, float* pend);

}  // namespace sf
