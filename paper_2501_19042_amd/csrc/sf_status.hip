// Per-sample status passes of sf_project (SF_SAMPLE_* bits of swarmsf.h), run before and after the
// solve kernels when the caller asks for status_out.  Keeping the input and output checks out of the
// solve kernels keeps their register allocation unchanged.
//
// Finiteness is tested on the IEEE bit patterns (nonfinite_bits), so the result does not depend on
// the floating-point assumptions of any kernel.
#include "sf_internal.h"

namespace sf {
namespace {

constexpr int kStBlock = 256;

// Before the solve: kStatusInputFlag for a sample with a NaN or infinite coefficient in xi_bar, xi0
// or lam0, or boundary value of its problem; 0 otherwise.
template <typename T>
__global__ void __launch_bounds__(kStBlock)
status_input_kernel(const DevCfg* __restrict__ cfgs, const DevProblem* __restrict__ probs,
                    const WorkItem* __restrict__ items, int n_items, const T* __restrict__ xi_bar,
                    const T* __restrict__ xi0, const T* __restrict__ lam0, const T* __restrict__ bvals,
                    int32_t* __restrict__ status) {
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const WorkItem w = items[it];
    const DevProblem pr = probs[w.problem];
    const DevCfg c = cfgs[pr.cfg];
    const int nDm = c.n * c.D * c.m, nD6 = c.n * c.D * kNFix;
    int bvbad = 0;
    for (int q = threadIdx.x; q < nD6; q += kStBlock) bvbad |= nonfinite_bits(bvals[pr.bnd_off + q]);
    bvbad = __syncthreads_or(bvbad);
    for (int sl = w.first; sl < w.first + w.count; ++sl) {
      const int64_t coef = pr.coef_off + (int64_t)sl * nDm;
      int bad = 0;
      for (int q = threadIdx.x; q < nDm; q += kStBlock) {
        bad |= nonfinite_bits(xi_bar[coef + q]);
        if (xi0) bad |= nonfinite_bits(xi0[coef + q]);
        if (lam0) bad |= nonfinite_bits(lam0[coef + q]);
      }
      bad = __syncthreads_or(bad) | bvbad;
      if (threadIdx.x == 0) status[pr.sample_base + sl] = bad ? kStatusInputFlag : 0;
    }
  }
}

// After the solve: NaN outputs and SF_SAMPLE_NONFINITE_INPUT for the flagged samples (the solve left
// them at their initial state); for the others, SF_SAMPLE_NONFINITE added when xi_out or lam_out
// holds a NaN or infinity.
template <typename T>
__global__ void __launch_bounds__(kStBlock)
status_output_kernel(const DevCfg* __restrict__ cfgs, const DevProblem* __restrict__ probs,
                     const WorkItem* __restrict__ items, int n_items, int iters, T* __restrict__ xi_out,
                     T* __restrict__ lam_out, T* __restrict__ resid_out, int resid_cols, T* __restrict__ ckpt,
                     int ckpt_every, int64_t ckpt_stride, int32_t* __restrict__ status) {
  const T qnan = sizeof(T) == 8 ? T(quiet_nan_f64()) : T(quiet_nan_f32());
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const WorkItem w = items[it];
    const DevProblem pr = probs[w.problem];
    const DevCfg c = cfgs[pr.cfg];
    const int nDm = c.n * c.D * c.m;
    for (int sl = w.first; sl < w.first + w.count; ++sl) {
      const int64_t coef = pr.coef_off + (int64_t)sl * nDm;
      const int64_t sidx = pr.sample_base + sl;
      const int32_t v = status[sidx];   // uniform over the workgroup
      if (v < 0) {
        for (int q = threadIdx.x; q < nDm; q += kStBlock) {
          xi_out[coef + q] = qnan;
          if (lam_out) lam_out[coef + q] = qnan;
          if (ckpt)
            for (int k = 0; k < iters; k += ckpt_every) {
              const int64_t base = (int64_t)(k / ckpt_every) * 2 * ckpt_stride + coef;
              ckpt[base + q] = qnan;
              ckpt[base + ckpt_stride + q] = qnan;
            }
        }
        if (resid_out)
          for (int q = threadIdx.x; q < resid_cols; q += kStBlock) resid_out[sidx * resid_cols + q] = qnan;
        __syncthreads();
        if (threadIdx.x == 0) status[sidx] = SF_SAMPLE_NONFINITE_INPUT;
      } else {
        int bad = 0;
        for (int q = threadIdx.x; q < nDm; q += kStBlock) {
          bad |= nonfinite_bits(xi_out[coef + q]);
          if (lam_out) bad |= nonfinite_bits(lam_out[coef + q]);
        }
        bad = __syncthreads_or(bad);
        if (threadIdx.x == 0 && bad) status[sidx] = v | SF_SAMPLE_NONFINITE;
      }
    }
  }
}

template <typename T>
hipError_t status_input(const LaunchArgs& a) {
  hipLaunchKernelGGL(status_input_kernel<T>, dim3(a.n_items), dim3(kStBlock), 0, a.stream, a.cfgs, a.probs, a.items,
                     a.n_items, static_cast<const T*>(a.xi_bar), static_cast<const T*>(a.xi0),
                     static_cast<const T*>(a.lam0), static_cast<const T*>(a.bvals), a.status_out);
  return hipGetLastError();
}

template <typename T>
hipError_t status_output(const LaunchArgs& a) {
  const int cols = (a.flags & SF_RESID_HISTORY) ? 2 * a.iters : ((a.flags & SF_FP_RESIDUAL) ? 3 : 2);
  hipLaunchKernelGGL(status_output_kernel<T>, dim3(a.n_items), dim3(kStBlock), 0, a.stream, a.cfgs, a.probs, a.items,
                     a.n_items, a.iters, static_cast<T*>(a.xi_out), static_cast<T*>(a.lam_out),
                     static_cast<T*>(a.resid_out), cols, static_cast<T*>(a.ckpt), a.ckpt_every, a.ckpt_stride,
                     a.status_out);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_status_input(const LaunchArgs& a, bool dbl) {
  return dbl ? status_input<double>(a) : status_input<float>(a);
}

hipError_t launch_status_output(const LaunchArgs& a, bool dbl) {
  return dbl ? status_output<double>(a) : status_output<float>(a);
}

}  // namespace sf
