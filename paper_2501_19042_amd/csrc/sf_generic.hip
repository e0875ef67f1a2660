// Generic fused safety-filter kernels for gfx950.
//
// One workgroup owns one sample for the whole solve: the state (xi, lambda, xi_bar)
// stays in LDS across all iterations and only the inputs and outputs touch HBM.  Each
// iteration walks the horizon in time tiles:
//   1. basis evaluation   Y = F_b xi for the tile (positions, velocities, accelerations;
//                          eq. poly) into LDS,
//   2. projections        alpha/beta/d steps (eqs. alpha_step .. d_step) written in their
//                          equivalent radial form: for a pair (i, j) with s = M_a^{-1} r,
//                          the residual r - e is r * min(0, 1 - 1/||s||); for a bound ball
//                          it is v * max(0, 1 - vmax/||v||),
//   3. back-projection    g += F^T (rho * residual) for the tile,
// then the multiplier step (eq. lambda_step, minus sign) and the QP step of
// eq. (xi_step) restricted to the free coefficients.  The QP inverse has the exact
// structure J (x) X0 + (I - J) (x) X1 with J = 11^T/n (the pair incidence gives
// F_o^T F_o = (nI - 11^T) (x) P^T P), so the step costs O(n m_f^2) per axis.
//
// This path serves FP64 (parity with the oracle) and plain FP32 for any shape whose
// LDS plan fits; the MFMA kernels cover the production shapes.
#include "sf_generic_impl.h"

namespace sf {
namespace {

using namespace gen;

template <typename T>
__global__ void __launch_bounds__(kBlock)
generic_project_kernel(const DevCfg* __restrict__ cfgs, const T* __restrict__ tab,
                       const DevProblem* __restrict__ probs, const WorkItem* __restrict__ items, int n_items,
                       const T* __restrict__ xi_bar, const T* __restrict__ bvals,
                       const T* __restrict__ xi0, const T* __restrict__ lam0, int iters,
                       T* __restrict__ xi_out, T* __restrict__ lam_out, T* __restrict__ resid_out,
                       int32_t* __restrict__ status_out, int flags,
                       T* __restrict__ ckpt, int ckpt_every, int64_t ckpt_stride, int TT) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  const bool history = (flags & 1) != 0;
  const bool fpr = (flags & 32) != 0;   // resid_out [S][3] with the fixed-point residual sum
  const int rw = fpr ? 3 : 2;

  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const WorkItem w = items[it];
    const DevProblem pr = probs[w.problem];
    const Ctx<T> x = make_ctx<T>(cfgs[pr.cfg], tab);
    const Lds<T> L = carve<T>(smem, lds_plan(x.c, TT));
    const int nDm = x.nDm;
    for (int sl = w.first; sl < w.first + w.count; ++sl) {
      const int64_t coef = pr.coef_off + (int64_t)sl * nDm;
      const int64_t sidx = pr.sample_base + sl;
      setup_sample<T>(x, L, xi_bar + coef, bvals + pr.bnd_off, xi0 ? xi0 + coef : nullptr,
                      lam0 ? lam0 + coef : nullptr);
      // a sample the input check flagged (non-finite input) is not iterated; the status pass then
      // writes NaN over its outputs
      const int32_t in_flag = status_out ? status_out[sidx] : 0;
      const int iters_s = in_flag < 0 ? 0 : iters;
      const bool final_resid = (resid_out || status_out) && !(history && resid_out);
      T last_mx = T(0);   // largest block norm of the last residual in history mode
      T fsum = T(0);   // this thread's share of the fixed-point residual sum
      for (int k = 0; k < iters_s; ++k) {
        if (ckpt && (k % ckpt_every) == 0) {
          const int64_t base = (int64_t)(k / ckpt_every) * 2 * ckpt_stride + coef;
          for (int q = threadIdx.x; q < nDm; q += blockDim.x) {
            ckpt[base + q] = L.xi[q];
            ckpt[base + ckpt_stride + q] = L.lam[q];
          }
        }
        if (history || fpr || (final_resid && k == iters_s - 1))
          for (int q = threadIdx.x; q < nDm; q += blockDim.x) L.xprev[q] = L.xi[q];
        iteration<T>(x, L, TT, k);
        if (fpr) {
          // ||xi^{k+1} - xi^k||^2 + ||lambda^{k+1} - lambda^k||^2, with lambda^{k+1} - lambda^k = -g
          for (int q = threadIdx.x; q < nDm; q += blockDim.x) {
            const T d = L.xi[q] - L.xprev[q];
            fsum = fma(d, d, fsum);
            fsum = fma(L.g[q], L.g[q], fsum);
          }
          __syncthreads();
        }
        if (history && resid_out) {
          T ss, mx;
          residual_pass<T>(x.c, x.basis, L, TT, ss, mx);
          if (threadIdx.x == 0) {
            resid_out[(sidx * iters + k) * 2 + 0] = ss;
            resid_out[(sidx * iters + k) * 2 + 1] = mx;
          }
          last_mx = mx;
        }
      }
      if (final_resid) {
        T ss = T(0), mx = T(0);
        if (iters_s > 0) residual_pass<T>(x.c, x.basis, L, TT, ss, mx);
        if (fpr) {
          T unused = T(0);
          block_reduce_sum_max<T>(L.red, fsum, unused);
        }
        if (threadIdx.x == 0 && resid_out) {
          resid_out[sidx * rw + 0] = ss;
          resid_out[sidx * rw + 1] = mx;
          if (fpr) resid_out[sidx * rw + 2] = fsum;
        }
        last_mx = mx;
      }
      for (int q = threadIdx.x; q < nDm; q += blockDim.x) {
        xi_out[coef + q] = L.xi[q];
        if (lam_out) lam_out[coef + q] = L.lam[q];
      }
      // convergence bits (the status pass adds the finiteness of the outputs)
      if (status_out && threadIdx.x == 0)
        status_out[sidx] = in_flag < 0 ? in_flag : sample_status<T>(false, false, last_mx, iters_s);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------------
// FP64 feasibility check at the grid times.
// ---------------------------------------------------------------------------------

__host__ __device__ inline size_t feas_elems(const DevCfg& c, int TT) {
  return (size_t)c.n * c.D * c.m + (size_t)3 * c.n * c.D * TT + 5 * kBlock;
}

template <typename Tin>
__global__ void __launch_bounds__(kBlock)
feasibility_kernel(const DevCfg* __restrict__ cfgs, const double* __restrict__ tab,
                   const DevProblem* __restrict__ probs, const WorkItem* __restrict__ items, int n_items,
                   const Tin* __restrict__ xi, const Tin* __restrict__ bvals, double* __restrict__ viol, int TT) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* smem = reinterpret_cast<double*>(smem_raw);
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const WorkItem w = items[it];
    const DevProblem pr = probs[w.problem];
    const DevCfg c = cfgs[pr.cfg];
    const int n = c.n, D = c.D, m = c.m, nD = n * D, nDm = nD * m;
    double* x = smem;
    double* Y = x + nDm;
    double* red = Y + (size_t)3 * nD * TT;
    const double* basis = tab + c.off_basis;
    const Tin* bv = bvals + pr.bnd_off;
    for (int sl = w.first; sl < w.first + w.count; ++sl) {
      const int64_t coef = pr.coef_off + (int64_t)sl * nDm;
      const int64_t sidx = pr.sample_base + sl;
      for (int q = threadIdx.x; q < nDm; q += blockDim.x) x[q] = (double)xi[coef + q];
      __syncthreads();
      double smin = DBL_MAX, vmx = 0.0, amx = 0.0, bmx = 0.0, wmx = 0.0;
      for (int q = threadIdx.x; q < nD * kNFix; q += blockDim.x) {
        const int row = q / kNFix, r = q - row * kNFix;
        const int bsel = r % 3;
        const int h = r < 3 ? 0 : c.H - 1;
        const double* brow = basis + ((size_t)bsel * c.H + h) * m;
        double acc = 0.0;
#pragma unroll 4
        for (int k = 0; k < m; ++k) acc = fma(brow[k], x[row * m + k], acc);
        bmx = fmax(bmx, fabs(acc - (double)bv[row * kNFix + r]));
      }
      for (int t0 = 0; t0 < c.H; t0 += TT) {
        const int TTc = min(TT, c.H - t0);
        for (int q = threadIdx.x; q < 3 * nD * TTc; q += blockDim.x) {
          const int bsel = q / (nD * TTc), rem = q - bsel * nD * TTc;
          const int row = rem / TTc, tt = rem - row * TTc;
          const double* brow = basis + ((size_t)bsel * c.H + t0 + tt) * m;
          double acc = 0.0;
#pragma unroll 4
          for (int k = 0; k < m; ++k) acc = fma(brow[k], x[row * m + k], acc);
          Y[(bsel * nD + row) * TT + tt] = acc;
        }
        __syncthreads();
        for (int q = threadIdx.x; q < n * TTc; q += blockDim.x) {
          const int i = q / TTc, tt = q - i * TTc;
          for (int j = i + 1; j < n; ++j) {
            double s = 0.0;
            SF_FOR_DIM(d, D) {
              const double r = Y[(i * D + d) * TT + tt] - Y[(j * D + d) * TT + tt];
              s += r * r * (d == 2 ? c.inv_b2 : c.inv_a2);
            }
            smin = fmin(smin, s);
          }
          double v2 = 0.0, a2 = 0.0;
          SF_FOR_DIM(d, D) {
            const double v = Y[((n + i) * D + d) * TT + tt];
            const double ac = Y[((2 * n + i) * D + d) * TT + tt];
            v2 += v * v;
            a2 += ac * ac;
          }
          vmx = fmax(vmx, v2);
          amx = fmax(amx, a2);
          if (c.ws_on) {   // ||M_w^{-1} (p_i - p_w)||^2 of eq. workspace_con
            double w2 = 0.0;
            SF_FOR_DIM(d, D) {
              const double r = Y[(i * D + d) * TT + tt] - c.ws_c[d];
              w2 += r * r * (d == 2 ? c.ws_ib2 : c.ws_ia2);
            }
            wmx = fmax(wmx, w2);
          }
        }
        __syncthreads();
      }
      const int t = threadIdx.x;
      red[t] = smin; red[kBlock + t] = vmx; red[2 * kBlock + t] = amx; red[3 * kBlock + t] = bmx;
      red[4 * kBlock + t] = wmx;
      __syncthreads();
      for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (t < s) {
          red[t] = fmin(red[t], red[t + s]);
          for (int r = 1; r < 5; ++r) red[r * kBlock + t] = fmax(red[r * kBlock + t], red[r * kBlock + t + s]);
        }
        __syncthreads();
      }
      if (t == 0) {
        viol[sidx * 5 + 0] = c.a * (1.0 - sqrt(red[0]));
        viol[sidx * 5 + 1] = c.vel_on ? sqrt(red[kBlock]) - c.vmax : -DBL_MAX;
        viol[sidx * 5 + 2] = c.acc_on ? sqrt(red[2 * kBlock]) - c.amax : -DBL_MAX;
        viol[sidx * 5 + 3] = red[3 * kBlock];
        viol[sidx * 5 + 4] = c.ws_on ? c.ws_a * (sqrt(red[4 * kBlock]) - 1.0) : 0.0;
      }
      __syncthreads();
    }
  }
}

}  // namespace

size_t generic_lds_bytes(const DevCfg& c, int tile, size_t elem) { return lds_plan(c, tile).total * elem; }

size_t feasibility_lds_bytes(const DevCfg& c, int tile) { return feas_elems(c, tile) * sizeof(double); }

template <typename T>
hipError_t launch_generic_project(const LaunchArgs& a) {
  auto kern = generic_project_kernel<T>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)a.lds_bytes);
  if (e != hipSuccess) return e;
  const int grid = a.n_items;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), a.lds_bytes, a.stream, a.cfgs,
                     static_cast<const T*>(a.tab), a.probs, a.items, a.n_items,
                     static_cast<const T*>(a.xi_bar), static_cast<const T*>(a.bvals),
                     static_cast<const T*>(a.xi0), static_cast<const T*>(a.lam0), a.iters,
                     static_cast<T*>(a.xi_out), static_cast<T*>(a.lam_out), static_cast<T*>(a.resid_out),
                     a.status_out, a.flags, static_cast<T*>(a.ckpt), a.ckpt_every, a.ckpt_stride, a.tile);
  return hipGetLastError();
}

template hipError_t launch_generic_project<double>(const LaunchArgs& a);
template hipError_t launch_generic_project<float>(const LaunchArgs& a);

hipError_t launch_feasibility(const DevCfg* cfgs, const double* tab64, const DevProblem* probs,
                              const WorkItem* items, int32_t n_items, const void* xi, int xi_is_double,
                              const void* bvals, double* viol, int32_t tile, size_t lds_bytes,
                              hipStream_t stream) {
  if (xi_is_double) {
    auto kern = feasibility_kernel<double>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(n_items), dim3(kBlock), lds_bytes, stream, cfgs, tab64, probs, items,
                       n_items, static_cast<const double*>(xi), static_cast<const double*>(bvals), viol, tile);
  } else {
    auto kern = feasibility_kernel<float>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(n_items), dim3(kBlock), lds_bytes, stream, cfgs, tab64, probs, items,
                       n_items, static_cast<const float*>(xi), static_cast<const float*>(bvals), viol, tile);
  }
  return hipGetLastError();
}

}  // namespace sf
