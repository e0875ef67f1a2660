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

// Allocation-free reverse mode: a fixed device array of the library holds the problem and chunk
// tables and the per-chunk partial sums.
constexpr size_t kEqNoAllocBytes = (size_t)16 << 20;   // size of that array per GPU
constexpr int kEqNoAllocMaxProblems = 64;               // problems per call
struct EqNoAllocBatch {                                 // passed by value to the table kernel
  int32_t n_probs;
  int32_t slot[kEqNoAllocMaxProblems];
  int32_t count[kEqNoAllocMaxProblems];
};
// Offsets (bytes) of the tables and the partial sums inside the array for a batch.
struct EqNoAllocLayout {
  size_t probs, chunks, chunk_first, part, total;
};
EqNoAllocLayout eq_noalloc_layout(int32_t n_probs, int32_t n_chunks, int32_t part_stride, size_t elem);
// Device address of the array on `device` (looked up once per device, with that device current,
// at sf_setup); nullptr before that.
hipError_t eq_noalloc_init(int device);
void* eq_noalloc_scratch(int device);
// Fill the problem table, chunk table and first-chunk index of a batch into the array (the same
// tables, in the same order, as the handle's plan for that batch).
hipError_t launch_eq_noalloc_tables(const DevCfg* cfgs, const EqNoAllocBatch& b, void* scratch,
                                    const EqNoAllocLayout& lay, hipStream_t stream);

template <typename T>
hipError_t launch_qp_equality(const EqArgs& a);

}  // namespace sf
