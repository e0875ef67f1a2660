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
#include "sf_internal.h"

#include <cfloat>

namespace sf {
namespace {

template <typename T> __device__ __forceinline__ T rsq(T x);
template <> __device__ __forceinline__ double rsq<double>(double x) { return 1.0 / sqrt(x); }
template <> __device__ __forceinline__ float rsq<float>(float x) { return rsqrtf(x); }

template <typename T> __device__ __forceinline__ T tiny_sq();
template <> __device__ __forceinline__ double tiny_sq<double>() { return DBL_MIN; }
template <> __device__ __forceinline__ float tiny_sq<float>() { return FLT_MIN; }

// LDS layout in elements of T; identical on host (for sizing) and device.
struct LdsPlan {
  size_t xi, lam, xb, xprev, g, xp, dlt, dbar, corr, ybuf, ybar, Y, Rb, red, total;
};

__host__ __device__ inline LdsPlan lds_plan(const DevCfg& c, int TT) {
  const size_t nDm = (size_t)c.n * c.D * c.m;
  const size_t nDf = (size_t)c.n * c.D * c.mf;
  const size_t nD6 = (size_t)c.n * c.D * kNFix;
  const size_t tile = (size_t)3 * c.n * c.D * TT;
  LdsPlan p;
  size_t o = 0;
  p.xi = o; o += nDm;
  p.lam = o; o += nDm;
  p.xb = o; o += nDm;
  p.xprev = o; o += nDm;
  p.g = o; o += nDm;
  p.xp = o; o += nD6;
  p.dlt = o; o += nD6;
  p.dbar = o; o += (size_t)c.D * kNFix;
  p.corr = o; o += nDf;
  p.ybuf = o; o += nDf;
  p.ybar = o; o += (size_t)c.D * (c.mf > 0 ? c.mf : 1);
  p.Y = o; o += tile;
  p.Rb = o; o += tile;
  p.red = o; o += 2 * kBlock;
  p.total = o;
  return p;
}

template <typename T>
struct Lds {
  T *xi, *lam, *xb, *xprev, *g, *xp, *dlt, *dbar, *corr, *ybuf, *ybar, *Y, *Rb, *red;
};

template <typename T>
__device__ Lds<T> carve(T* base, const LdsPlan& p) {
  Lds<T> L;
  L.xi = base + p.xi; L.lam = base + p.lam; L.xb = base + p.xb; L.xprev = base + p.xprev;
  L.g = base + p.g; L.xp = base + p.xp; L.dlt = base + p.dlt; L.dbar = base + p.dbar;
  L.corr = base + p.corr; L.ybuf = base + p.ybuf; L.ybar = base + p.ybar;
  L.Y = base + p.Y; L.Rb = base + p.Rb; L.red = base + p.red;
  return L;
}

// Residual of the collision projection for r = X_lo - X_hi seen from one robot.  For
// coincident robots atan2(0, 0) = 0 puts the target at (0, 0, b) (3D) or (a, 0) (2D)
// for the pair (lo, hi); the lower robot receives r - e, the upper one its negation.
template <typename T>
__device__ __forceinline__ void coll_resid(const T* r, int D, T ia2, T ib2, T a, T b, bool lower, T* R) {
  T ss = r[0] * r[0] * ia2 + r[1] * r[1] * ia2;
  if (D == 3) ss += r[2] * r[2] * ib2;
  if (ss >= tiny_sq<T>()) {
    const T f = min(T(0), T(1) - rsq<T>(ss));
    for (int d = 0; d < D; ++d) R[d] = f * r[d];
  } else {
    for (int d = 0; d < D; ++d) R[d] = T(0);
    if (D == 3) R[2] = lower ? -b : b;
    else R[0] = lower ? -a : a;
  }
}

template <typename T>
__device__ __forceinline__ void ball_resid(const T* v, int D, T lim, T* R) {
  T ss = v[0] * v[0] + v[1] * v[1];
  if (D == 3) ss += v[2] * v[2];
  const T f = (ss > lim * lim) ? T(1) - lim * rsq<T>(ss) : T(0);
  for (int d = 0; d < D; ++d) R[d] = f * v[d];
}

// dst[b][i][d][tt] = sum_k basis[b][t0+tt][k] * src[i][d][k] for the enabled bases.
template <typename T>
__device__ void eval_tile(const DevCfg& c, const T* __restrict__ basis, const T* src, T* dst,
                          int t0, int TTc, int TT) {
  const int nD = c.n * c.D;
  const int total = 3 * nD * TTc;
  for (int q = threadIdx.x; q < total; q += blockDim.x) {
    const int bsel = q / (nD * TTc);
    const int rem = q - bsel * nD * TTc;
    if ((bsel == 1 && !c.vel_on) || (bsel == 2 && !c.acc_on)) continue;
    const int row = rem / TTc;
    const int tt = rem - row * TTc;
    const T* brow = basis + ((size_t)bsel * c.H + t0 + tt) * c.m;
    const T* x = src + row * c.m;
    T acc = T(0);
    for (int k = 0; k < c.m; ++k) acc = fma(brow[k], x[k], acc);
    dst[(bsel * nD + row) * TT + tt] = acc;
  }
}

template <typename T>
__device__ void block_reduce_sum_max(T* red, T& s, T& mx) {
  const int t = threadIdx.x;
  red[t] = s;
  red[kBlock + t] = mx;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (t < w) {
      red[t] += red[t + w];
      red[kBlock + t] = max(red[kBlock + t], red[kBlock + t + w]);
    }
    __syncthreads();
  }
  s = red[0];
  mx = red[kBlock];
  __syncthreads();
}

// Primal residual r_p = F xi_new - e(xi_prev) of eq. (primal_residual):
// (||r_p||^2, largest block norm).
template <typename T>
__device__ void residual_pass(const DevCfg& c, const T* __restrict__ basis, const Lds<T>& L, int TT,
                              T& out_ss, T& out_mx) {
  const int n = c.n, D = c.D, nD = n * D;
  const T ia2 = T(c.inv_a2), ib2 = T(c.inv_b2), a = T(c.a), b = T(c.b);
  T ss = T(0), mx = T(0);
  for (int t0 = 0; t0 < c.H; t0 += TT) {
    const int TTc = min(TT, c.H - t0);
    eval_tile<T>(c, basis, L.xprev, L.Y, t0, TTc, TT);
    eval_tile<T>(c, basis, L.xi, L.Rb, t0, TTc, TT);
    __syncthreads();
    for (int q = threadIdx.x; q < n * TTc; q += blockDim.x) {
      const int i = q / TTc, tt = q - (q / TTc) * TTc;
      for (int j = i + 1; j < n; ++j) {
        T rprev[3], R[3], nrm = T(0);
        for (int d = 0; d < D; ++d) rprev[d] = L.Y[(i * D + d) * TT + tt] - L.Y[(j * D + d) * TT + tt];
        coll_resid<T>(rprev, D, ia2, ib2, a, b, true, R);
        for (int d = 0; d < D; ++d) {
          const T rp = (L.Rb[(i * D + d) * TT + tt] - L.Rb[(j * D + d) * TT + tt]) - (rprev[d] - R[d]);
          nrm += rp * rp;
        }
        ss += nrm;
        mx = max(mx, nrm);
      }
      for (int bsel = 1; bsel < 3; ++bsel) {
        if ((bsel == 1 && !c.vel_on) || (bsel == 2 && !c.acc_on)) continue;
        const T lim = T(bsel == 1 ? c.vmax : c.amax);
        T v[3], R[3], nrm = T(0);
        for (int d = 0; d < D; ++d) v[d] = L.Y[((bsel * n + i) * D + d) * TT + tt];
        ball_resid<T>(v, D, lim, R);
        for (int d = 0; d < D; ++d) {
          const T rp = L.Rb[((bsel * n + i) * D + d) * TT + tt] - (v[d] - R[d]);
          nrm += rp * rp;
        }
        ss += nrm;
        mx = max(mx, nrm);
      }
    }
    __syncthreads();
  }
  block_reduce_sum_max<T>(L.red, ss, mx);
  out_ss = ss;
  out_mx = sqrt(mx);
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
generic_project_kernel(const DevCfg* __restrict__ cfgs, const T* __restrict__ tab,
                       const DevProblem* __restrict__ probs, const WorkItem* __restrict__ items, int n_items,
                       const T* __restrict__ xi_bar, const T* __restrict__ bvals,
                       const T* __restrict__ xi0, const T* __restrict__ lam0, int iters,
                       T* __restrict__ xi_out, T* __restrict__ lam_out, T* __restrict__ resid_out, int flags,
                       T* __restrict__ ckpt, int ckpt_every, int64_t ckpt_stride, int TT) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  const bool history = (flags & 1) != 0;

  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const WorkItem w = items[it];
    const DevProblem pr = probs[w.problem];
    const DevCfg c = cfgs[pr.cfg];
    const LdsPlan plan = lds_plan(c, TT);
    const Lds<T> L = carve<T>(smem, plan);
    const int n = c.n, D = c.D, m = c.m, mf = c.mf, nD = n * D;
    const int nDm = nD * m, nDf = nD * mf, nD6 = nD * kNFix;
    const T* basis = tab + c.off_basis;
    const T* X1 = tab + c.off_X1;
    const T* X01 = tab + c.off_X01;
    const T* Bmap = tab + c.off_Bmap;
    const T* Gfx = tab + c.off_Gfx;
    const T* Rfx = tab + c.off_Rfx;
    const T ia2 = T(c.inv_a2), ib2 = T(c.inv_b2), a = T(c.a), b = T(c.b);
    const T vmax = T(c.vmax), amax = T(c.amax);
    const T rho_c = T(c.rho_c), rho_v = T(c.rho_v), rho_a = T(c.rho_a), n_rho_c = T(c.n_rho_c);
    const T inv_n = T(1) / T(n);
    const T* bv = bvals + pr.bnd_off;

    for (int sl = w.first; sl < w.first + w.count; ++sl) {
      const int64_t coef = pr.coef_off + (int64_t)sl * nDm;
      const int64_t sidx = pr.sample_base + sl;

      // ---- load state, pinned coefficients and the first-step correction ----
      for (int q = threadIdx.x; q < nDm; q += blockDim.x) {
        const T x = xi_bar[coef + q];
        L.xb[q] = x;
        L.xi[q] = xi0 ? xi0[coef + q] : x;
        L.lam[q] = lam0 ? lam0[coef + q] : T(0);
      }
      for (int q = threadIdx.x; q < nD6; q += blockDim.x) {
        const int row = q / kNFix, r = q - row * kNFix;
        T acc = T(0);
        for (int s = 0; s < kNFix; ++s) acc = fma(Bmap[r * kNFix + s], bv[row * kNFix + s], acc);
        L.xp[q] = acc;
      }
      __syncthreads();
      for (int q = threadIdx.x; q < nD6; q += blockDim.x) {
        const int row = q / kNFix, r = q - row * kNFix;
        const int k = r < 3 ? r : m - kNFix + r;
        L.dlt[q] = L.xi[row * m + k] - L.xp[q];
      }
      __syncthreads();
      for (int q = threadIdx.x; q < D * kNFix; q += blockDim.x) {
        const int d = q / kNFix, r = q - d * kNFix;
        T s = T(0);
        for (int i = 0; i < n; ++i) s += L.dlt[(i * D + d) * kNFix + r];
        L.dbar[q] = s * inv_n;
      }
      __syncthreads();
      for (int q = threadIdx.x; q < nDf; q += blockDim.x) {
        const int row = q / mf, f = q - row * mf, d = row % D;
        T acc = T(0);
        for (int r = 0; r < kNFix; ++r) {
          const T dl = L.dlt[row * kNFix + r];
          acc = fma(n_rho_c * Gfx[f * kNFix + r], dl - L.dbar[d * kNFix + r], acc);
          acc = fma(Rfx[f * kNFix + r], dl, acc);
        }
        L.corr[q] = acc;
      }
      __syncthreads();

      // ---- fixed-point iterations ----
      for (int k = 0; k < iters; ++k) {
        if (ckpt && (k % ckpt_every) == 0) {
          const int64_t base = (int64_t)(k / ckpt_every) * 2 * ckpt_stride + coef;
          for (int q = threadIdx.x; q < nDm; q += blockDim.x) {
            ckpt[base + q] = L.xi[q];
            ckpt[base + ckpt_stride + q] = L.lam[q];
          }
        }
        const bool keep_prev = history || (resid_out && k == iters - 1);
        for (int q = threadIdx.x; q < nDm; q += blockDim.x) {
          if (keep_prev) L.xprev[q] = L.xi[q];
          L.g[q] = T(0);
        }
        __syncthreads();
        for (int t0 = 0; t0 < c.H; t0 += TT) {
          const int TTc = min(TT, c.H - t0);
          eval_tile<T>(c, basis, L.xi, L.Y, t0, TTc, TT);
          __syncthreads();
          for (int q = threadIdx.x; q < n * TTc; q += blockDim.x) {
            const int i = q / TTc, tt = q - (q / TTc) * TTc;
            T xi_[3] = {T(0), T(0), T(0)}, C[3] = {T(0), T(0), T(0)};
            for (int d = 0; d < D; ++d) xi_[d] = L.Y[(i * D + d) * TT + tt];
            for (int j = 0; j < n; ++j) {
              if (j == i) continue;
              T r[3], R[3];
              for (int d = 0; d < D; ++d) r[d] = xi_[d] - L.Y[(j * D + d) * TT + tt];
              coll_resid<T>(r, D, ia2, ib2, a, b, i < j, R);
              for (int d = 0; d < D; ++d) C[d] += R[d];
            }
            for (int d = 0; d < D; ++d) L.Rb[(i * D + d) * TT + tt] = C[d];
            if (c.vel_on) {
              T v[3], R[3];
              for (int d = 0; d < D; ++d) v[d] = L.Y[((n + i) * D + d) * TT + tt];
              ball_resid<T>(v, D, vmax, R);
              for (int d = 0; d < D; ++d) L.Rb[((n + i) * D + d) * TT + tt] = R[d];
            }
            if (c.acc_on) {
              T v[3], R[3];
              for (int d = 0; d < D; ++d) v[d] = L.Y[((2 * n + i) * D + d) * TT + tt];
              ball_resid<T>(v, D, amax, R);
              for (int d = 0; d < D; ++d) L.Rb[((2 * n + i) * D + d) * TT + tt] = R[d];
            }
          }
          __syncthreads();
          for (int q = threadIdx.x; q < nDm; q += blockDim.x) {
            const int row = q / m, kk = q - row * m;
            T ac = T(0), av = T(0), aa = T(0);
            for (int tt = 0; tt < TTc; ++tt) {
              const size_t brow = (size_t)(t0 + tt) * m + kk;
              ac = fma(basis[brow], L.Rb[row * TT + tt], ac);
              if (c.vel_on) av = fma(basis[(size_t)c.H * m + brow], L.Rb[(nD + row) * TT + tt], av);
              if (c.acc_on) aa = fma(basis[(size_t)2 * c.H * m + brow], L.Rb[(2 * nD + row) * TT + tt], aa);
            }
            L.g[q] += rho_c * ac + rho_v * av + rho_a * aa;
          }
          __syncthreads();
        }
        // multiplier step and QP step (incremental form on the free coefficients)
        for (int q = threadIdx.x; q < nDm; q += blockDim.x) {
          const T gq = L.g[q];
          const T ln = L.lam[q] - gq;
          L.lam[q] = ln;
          const int row = q / m, kk = q - row * m, f = kk - 3;
          if (f >= 0 && f < mf) {
            T y = L.xb[q] - L.xi[q] + ln - gq;
            if (k == 0) y += L.corr[row * mf + f];
            L.ybuf[row * mf + f] = y;
          }
        }
        __syncthreads();
        for (int q = threadIdx.x; q < D * mf; q += blockDim.x) {
          const int d = q / mf, f = q - d * mf;
          T s = T(0);
          for (int i = 0; i < n; ++i) s += L.ybuf[(i * D + d) * mf + f];
          L.ybar[q] = s * inv_n;
        }
        __syncthreads();
        for (int q = threadIdx.x; q < nDf; q += blockDim.x) {
          const int row = q / mf, f = q - row * mf, d = row % D;
          T acc = T(0);
          for (int f2 = 0; f2 < mf; ++f2) {
            acc = fma(X1[f * mf + f2], L.ybuf[row * mf + f2], acc);
            acc = fma(X01[f * mf + f2], L.ybar[d * mf + f2], acc);
          }
          L.xi[row * m + 3 + f] += acc;
        }
        if (k == 0) {
          for (int q = threadIdx.x; q < nD6; q += blockDim.x) {
            const int row = q / kNFix, r = q - row * kNFix;
            const int kk = r < 3 ? r : m - kNFix + r;
            L.xi[row * m + kk] = L.xp[q];
          }
        }
        __syncthreads();
        if (history && resid_out) {
          T ss, mx;
          residual_pass<T>(c, basis, L, TT, ss, mx);
          if (threadIdx.x == 0) {
            resid_out[(sidx * iters + k) * 2 + 0] = ss;
            resid_out[(sidx * iters + k) * 2 + 1] = mx;
          }
        }
      }
      if (resid_out && !history) {
        T ss = T(0), mx = T(0);
        if (iters > 0) residual_pass<T>(c, basis, L, TT, ss, mx);
        if (threadIdx.x == 0) {
          resid_out[sidx * 2 + 0] = ss;
          resid_out[sidx * 2 + 1] = mx;
        }
      }
      for (int q = threadIdx.x; q < nDm; q += blockDim.x) {
        xi_out[coef + q] = L.xi[q];
        if (lam_out) lam_out[coef + q] = L.lam[q];
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------------
// FP64 feasibility check at the grid times.
// ---------------------------------------------------------------------------------

__host__ __device__ inline size_t feas_elems(const DevCfg& c, int TT) {
  return (size_t)c.n * c.D * c.m + (size_t)3 * c.n * c.D * TT + 4 * kBlock;
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
      double smin = DBL_MAX, vmx = 0.0, amx = 0.0, bmx = 0.0;
      for (int q = threadIdx.x; q < nD * kNFix; q += blockDim.x) {
        const int row = q / kNFix, r = q - row * kNFix;
        const int bsel = r % 3;
        const int h = r < 3 ? 0 : c.H - 1;
        const double* brow = basis + ((size_t)bsel * c.H + h) * m;
        double acc = 0.0;
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
          for (int k = 0; k < m; ++k) acc = fma(brow[k], x[row * m + k], acc);
          Y[(bsel * nD + row) * TT + tt] = acc;
        }
        __syncthreads();
        for (int q = threadIdx.x; q < n * TTc; q += blockDim.x) {
          const int i = q / TTc, tt = q - i * TTc;
          for (int j = i + 1; j < n; ++j) {
            double s = 0.0;
            for (int d = 0; d < D; ++d) {
              const double r = Y[(i * D + d) * TT + tt] - Y[(j * D + d) * TT + tt];
              s += r * r * (d == 2 ? c.inv_b2 : c.inv_a2);
            }
            smin = fmin(smin, s);
          }
          double v2 = 0.0, a2 = 0.0;
          for (int d = 0; d < D; ++d) {
            const double v = Y[((n + i) * D + d) * TT + tt];
            const double ac = Y[((2 * n + i) * D + d) * TT + tt];
            v2 += v * v;
            a2 += ac * ac;
          }
          vmx = fmax(vmx, v2);
          amx = fmax(amx, a2);
        }
        __syncthreads();
      }
      const int t = threadIdx.x;
      red[t] = smin; red[kBlock + t] = vmx; red[2 * kBlock + t] = amx; red[3 * kBlock + t] = bmx;
      __syncthreads();
      for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (t < s) {
          red[t] = fmin(red[t], red[t + s]);
          for (int r = 1; r < 4; ++r) red[r * kBlock + t] = fmax(red[r * kBlock + t], red[r * kBlock + t + s]);
        }
        __syncthreads();
      }
      if (t == 0) {
        viol[sidx * 4 + 0] = c.a * (1.0 - sqrt(red[0]));
        viol[sidx * 4 + 1] = c.vel_on ? sqrt(red[kBlock]) - c.vmax : -DBL_MAX;
        viol[sidx * 4 + 2] = c.acc_on ? sqrt(red[2 * kBlock]) - c.amax : -DBL_MAX;
        viol[sidx * 4 + 3] = red[3 * kBlock];
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
                     a.flags, static_cast<T*>(a.ckpt), a.ckpt_every, a.ckpt_stride, a.tile);
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
