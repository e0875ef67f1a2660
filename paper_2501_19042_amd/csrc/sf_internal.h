// Internal types shared by the host runtime and the kernels of the safety filter.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "swarmsf.h"

namespace sf {

constexpr int kBlock = 256;          // threads per workgroup of the generic kernels
constexpr int kNFix = 6;             // coefficients pinned by the boundary rows per robot-axis

// Per-config constants on the device.  Matrices live in a per-precision table; the
// offsets below are element offsets into it.
//   basis [3][H][m]   position, velocity, acceleration Bernstein rows (eq. poly)
//   X1    [mf][mf]    (I + n rho_c Gff + Rff)^-1    relative-motion block of the QP step
//   X01   [mf][mf]    (I + Rff)^-1 - X1             mean-motion minus relative block
//   Bmap  [6][6]      pinned coefficients (c0, c1, c2, c_{N-2}, c_{N-1}, c_N) from
//                     (p0, v0, a0, pH, vH, aH)
//   Gfx   [mf][6]     G = P^T P, free rows x pinned columns
//   Rfx   [mf][6]     Rm = rho_v Pd^T Pd + rho_a Pdd^T Pdd (+ rho_w P^T P with a workspace),
//                     free rows x pinned columns
struct DevCfg {
  int32_t n, D, m, mf, H, Np;
  int32_t vel_on, acc_on;
  double a, b, inv_a2, inv_b2, vmax, amax;
  double rho_c, rho_v, rho_a, n_rho_c;
  double lip_v, lip_a;    // max_t sum_k |Pd[t][k]|, max_t sum_k |Pdd[t][k]|: drift bounds of v, acc
  int32_t ws_on, pad_;
  double ws_a, ws_ia2, ws_ib2;  // workspace semi-axis a_w, 1/a_w^2, 1/b_w^2 (eq. workspace_polar)
  double ws_c[3];               // workspace centre p_w
  double rho_w, ws_scale;       // rho of the workspace rows, and rho_w / rho_c
  float ws_f[6];                // fp32 copies (centre, 1/a_w^2, 1/b_w^2, rho_w / rho_c) for the
                                // MFMA kernels, read as scalars without a conversion
  float pad2_[2];
  double skin;            // pair-list margin of the MFMA broad phase, as a fraction of the safety
                          // semi-axes (a for x, y; b for z)
  int64_t off_basis, off_X1, off_X01, off_Bmap, off_Gfx, off_Rfx;
  int64_t off_a16[2];     // 16-byte offsets of the bf16 / fp16 S1 operand tables (MFMA path)
  int64_t off_a32;        // 16-byte offset of the fp32 S1 operand table (MFMA path)
};

struct DevProblem {
  int32_t cfg, count;
  int64_t coef_off;      // element offset of the problem's first coefficient
  int64_t bnd_off;       // element offset of its boundary values
  int64_t sample_base;   // global index of its first sample
};

struct WorkItem {
  int32_t problem, first, count, pad;
};

struct LaunchArgs {
  const DevCfg* cfgs;
  const void* tab;               // per-precision constant table
  const DevProblem* probs;
  const WorkItem* items;
  int32_t n_items;
  const void* xi_bar;
  const void* bvals;
  const void* xi0;
  const void* lam0;
  int32_t iters;
  void* xi_out;
  void* lam_out;
  void* resid_out;
  int32_t* status_out;           // per-sample SF_SAMPLE_* bits, or NULL
  int32_t flags;
  void* ckpt;
  int32_t ckpt_every;
  int64_t ckpt_stride;           // total coefficient elements of the batch
  int32_t tile;                  // time-tile length
  size_t lds_bytes;
  hipStream_t stream;
};

// Bit test for NaN and infinity on the IEEE encoding (all exponent bits set).  The integer goes
// through an empty asm statement first: otherwise the compiler recognises the pattern as a
// floating-point class test, which it may fold for NaN under no-NaN semantics (the MFMA kernels
// are built that way).
template <typename U>
__host__ __device__ inline U opaque_bits(U u) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+v"(u));
#else
  asm volatile("" : "+r"(u));
#endif
  return u;
}
__host__ __device__ inline bool nonfinite_bits(float x) {
  return (opaque_bits(__builtin_bit_cast(uint32_t, x)) & 0x7f800000u) == 0x7f800000u;
}
__host__ __device__ inline bool nonfinite_bits(double x) {
  return (opaque_bits(__builtin_bit_cast(uint64_t, x)) & 0x7ff0000000000000ull) == 0x7ff0000000000000ull;
}

// A quiet NaN built from its bit pattern (a NaN literal is undefined under no-NaN semantics).
__host__ __device__ inline float quiet_nan_f32() { return __builtin_bit_cast(float, opaque_bits(0x7fc00000u)); }
__host__ __device__ inline double quiet_nan_f64() {
  return __builtin_bit_cast(double, opaque_bits(0x7ff8000000000000ull));
}

// Per-sample status (SF_SAMPLE_* bits of swarmsf.h) from what the kernel found: a non-finite input,
// a non-finite value in the result, and the largest block norm of the final primal residual
// (convergence is judged only after at least one iteration).
template <typename T>
__host__ __device__ inline int32_t sample_status(bool bad_input, bool bad_output, T resid_max, int iters) {
  if (bad_input) return SF_SAMPLE_NONFINITE_INPUT;
  int32_t s = 0;
  if (bad_output) s |= SF_SAMPLE_NONFINITE;
  if (nonfinite_bits(resid_max)) s |= SF_SAMPLE_NONFINITE | (iters > 0 ? SF_SAMPLE_NOT_CONVERGED : 0);
  else if (iters > 0 && resid_max > T(SF_CONV_TOL)) s |= SF_SAMPLE_NOT_CONVERGED;
  return s;
}

// Status passes of sf_project (with status_out): before the solve, samples with a non-finite input
// get kStatusInputFlag (negative, so the solve kernels recognise it and skip the sample) and the
// others 0; the solve kernels write the convergence bits; after the solve, flagged samples get NaN
// outputs and SF_SAMPLE_NONFINITE_INPUT, the others SF_SAMPLE_NONFINITE if an output is not finite.
constexpr int32_t kStatusInputFlag = (int32_t)0x80000001u;
hipError_t launch_status_input(const LaunchArgs& a, bool dbl);
hipError_t launch_status_output(const LaunchArgs& a, bool dbl);

// Generic fused kernels (any shape that fits the LDS plan), T = double or float.
template <typename T>
hipError_t launch_generic_project(const LaunchArgs& a);

hipError_t launch_feasibility(const DevCfg* cfgs, const double* tab64, const DevProblem* probs,
                              const WorkItem* items, int32_t n_items, const void* xi, int xi_is_double,
                              const void* bvals, double* viol, int32_t tile, size_t lds_bytes,
                              hipStream_t stream);

// LDS bytes needed by the generic kernel for one config at a given time tile.
size_t generic_lds_bytes(const DevCfg& c, int tile, size_t elem);
size_t feasibility_lds_bytes(const DevCfg& c, int tile);

}  // namespace sf
