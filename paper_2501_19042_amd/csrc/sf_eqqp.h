// Equality-only QP layer (closed form) and its reverse mode: launch interface.
#pragma once

#include "sf_internal.h"

namespace sf {

struct EqArgs {
  const DevCfg* cfgs;
  const void* tab;               // per-precision constant table (Bmap)
  const DevProblem* probs;
  int32_t n_probs;
  const WorkItem* chunks;        // (problem, first sample, count) chunks
  int32_t n_chunks;
  const int32_t* chunk_first;    // [n_probs + 1]: first chunk of each problem (reverse mode)
  bool forward;
  const void* in;                // xi_in (forward) or g_out (reverse)
  const void* bvals;             // forward only
  void* out;                     // xi_out (forward) or g_xi_in (reverse, may be NULL)
  void* part;                    // reverse: per-chunk partial sums [n_chunks][part_stride], or NULL
  int32_t part_stride;            // slots per chunk (largest n D 6 of the batch)
  int32_t max_rows;               // largest n D of the batch (grid of the final sum)
  void* g_bvals;                 // reverse: [total boundary values], or NULL
  size_t lds_bytes;
  hipStream_t stream;
};

size_t qp_equality_lds_bytes(const DevCfg& c, size_t elem);

template <typename T>
hipError_t launch_qp_equality(const EqArgs& a);

}  // namespace sf
