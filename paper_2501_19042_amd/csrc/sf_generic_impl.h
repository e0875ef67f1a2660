// Device helpers shared by the generic forward kernel and the adjoint kernel: LDS plan,
// projections (radial form of the alpha/beta/d steps), basis evaluation of a time tile,
// residual pass, and one fixed-point iteration (eqs. alpha_step .. xi_step).
#pragma once

#include "sf_internal.h"

#include <cfloat>

// Loop over the D <= 3 coordinates with a constant trip count: the per-coordinate arrays (r[3],
// R[3], ...) then have constant indices after unrolling and stay in registers; a loop bounded by
// the run-time D would place them in private scratch memory.
#define SF_FOR_DIM(d, D) _Pragma("unroll") for (int d = 0; d < 3; ++d) if (d < (D))

namespace sf {
namespace gen {

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
    SF_FOR_DIM(d, D) R[d] = f * r[d];
  } else {
    SF_FOR_DIM(d, D) R[d] = T(0);
    if (D == 3) R[2] = lower ? -b : b;
    else R[0] = lower ? -a : a;
  }
}

template <typename T>
__device__ __forceinline__ void ball_resid(const T* v, int D, T lim, T* R) {
  T ss = v[0] * v[0] + v[1] * v[1];
  if (D == 3) ss += v[2] * v[2];
  const T f = (ss > lim * lim) ? T(1) - lim * rsq<T>(ss) : T(0);
  SF_FOR_DIM(d, D) R[d] = f * v[d];
}

// Residual of the workspace projection (eq. workspace_polar, d in [0, 1]) of a robot position p:
// with s = M_w^{-1} (p - p_w) the target is p_w + (p - p_w) min(1, 1/||s||), so the residual is
// (p - p_w) max(0, 1 - 1/||s||).
template <typename T>
__device__ __forceinline__ void ws_resid(const T* p, int D, const T* wc, T ia2, T ib2, T* R) {
  T q[3] = {T(0), T(0), T(0)};
  T ss = T(0);
  SF_FOR_DIM(d, D) {
    q[d] = p[d] - wc[d];
    ss += q[d] * q[d] * (d == 2 ? ib2 : ia2);
  }
  const T f = (ss > T(1)) ? T(1) - rsq<T>(ss) : T(0);
  SF_FOR_DIM(d, D) R[d] = f * q[d];
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
#pragma unroll 4
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
        SF_FOR_DIM(d, D) rprev[d] = L.Y[(i * D + d) * TT + tt] - L.Y[(j * D + d) * TT + tt];
        coll_resid<T>(rprev, D, ia2, ib2, a, b, true, R);
        SF_FOR_DIM(d, D) {
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
        SF_FOR_DIM(d, D) v[d] = L.Y[((bsel * n + i) * D + d) * TT + tt];
        ball_resid<T>(v, D, lim, R);
        SF_FOR_DIM(d, D) {
          const T rp = L.Rb[((bsel * n + i) * D + d) * TT + tt] - (v[d] - R[d]);
          nrm += rp * rp;
        }
        ss += nrm;
        mx = max(mx, nrm);
      }
      if (c.ws_on) {   // workspace rows: positions against the previous iterate's targets
        const T wc[3] = {T(c.ws_c[0]), T(c.ws_c[1]), T(c.ws_c[2])};
        T v[3], R[3], nrm = T(0);
        SF_FOR_DIM(d, D) v[d] = L.Y[(i * D + d) * TT + tt];
        ws_resid<T>(v, D, wc, T(c.ws_ia2), T(c.ws_ib2), R);
        SF_FOR_DIM(d, D) {
          const T rp = L.Rb[(i * D + d) * TT + tt] - (v[d] - R[d]);
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


// Per-sample constants of one config for the generic kernels.
template <typename T>
struct Ctx {
  DevCfg c;
  const T *basis, *X1, *X01, *Bmap, *Gfx, *Rfx;
  T ia2, ib2, a, b, vmax, amax, rho_c, rho_v, rho_a, n_rho_c, inv_n;
  T ws_ia2, ws_ib2, ws_scale, wc[3];
  int n, D, m, mf, nD, nDm, nDf, nD6;
};

template <typename T>
__device__ Ctx<T> make_ctx(const DevCfg& c, const T* tab) {
  Ctx<T> x;
  x.c = c;
  x.basis = tab + c.off_basis; x.X1 = tab + c.off_X1; x.X01 = tab + c.off_X01;
  x.Bmap = tab + c.off_Bmap; x.Gfx = tab + c.off_Gfx; x.Rfx = tab + c.off_Rfx;
  x.ia2 = T(c.inv_a2); x.ib2 = T(c.inv_b2); x.a = T(c.a); x.b = T(c.b);
  x.vmax = T(c.vmax); x.amax = T(c.amax);
  x.rho_c = T(c.rho_c); x.rho_v = T(c.rho_v); x.rho_a = T(c.rho_a); x.n_rho_c = T(c.n_rho_c);
  x.inv_n = T(1) / T(c.n);
  x.ws_ia2 = T(c.ws_ia2); x.ws_ib2 = T(c.ws_ib2); x.ws_scale = T(c.ws_scale);
  for (int d = 0; d < 3; ++d) x.wc[d] = T(c.ws_c[d]);
  x.n = c.n; x.D = c.D; x.m = c.m; x.mf = c.mf; x.nD = c.n * c.D;
  x.nDm = x.nD * c.m; x.nDf = x.nD * c.mf; x.nD6 = x.nD * kNFix;
  return x;
}

// Load xi_bar, the initial state (xi0 / lam0, NULL = xi_bar / 0), the pinned coefficients
// from the boundary values, and the first-step correction Z^T G (xi0 - xi_p).
template <typename T>
__device__ void setup_sample(const Ctx<T>& x, const Lds<T>& L, const T* __restrict__ xb_src,
                             const T* __restrict__ bv, const T* xi_src, const T* lam_src) {
  const int n = x.n, D = x.D, m = x.m, mf = x.mf;
  for (int q = threadIdx.x; q < x.nDm; q += blockDim.x) {
    const T v = xb_src[q];
    L.xb[q] = v;
    L.xi[q] = xi_src ? xi_src[q] : v;
    L.lam[q] = lam_src ? lam_src[q] : T(0);
  }
  for (int q = threadIdx.x; q < x.nD6; q += blockDim.x) {
    const int row = q / kNFix, r = q - row * kNFix;
    T acc = T(0);
    for (int s = 0; s < kNFix; ++s) acc = fma(x.Bmap[r * kNFix + s], bv[row * kNFix + s], acc);
    L.xp[q] = acc;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < x.nD6; q += blockDim.x) {
    const int row = q / kNFix, r = q - row * kNFix;
    const int k = r < 3 ? r : m - kNFix + r;
    L.dlt[q] = L.xi[row * m + k] - L.xp[q];
  }
  __syncthreads();
  for (int q = threadIdx.x; q < D * kNFix; q += blockDim.x) {
    const int d = q / kNFix, r = q - d * kNFix;
    T s = T(0);
    for (int i = 0; i < n; ++i) s += L.dlt[(i * D + d) * kNFix + r];
    L.dbar[q] = s * x.inv_n;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < x.nDf; q += blockDim.x) {
    const int row = q / mf, f = q - row * mf, d = row % D;
    T acc = T(0);
    for (int r = 0; r < kNFix; ++r) {
      const T dl = L.dlt[row * kNFix + r];
      acc = fma(x.n_rho_c * x.Gfx[f * kNFix + r], dl - L.dbar[d * kNFix + r], acc);
      acc = fma(x.Rfx[f * kNFix + r], dl, acc);
    }
    L.corr[q] = acc;
  }
  __syncthreads();
}

// One fixed-point iteration on L.xi / L.lam (k is the global iteration index: k = 0 adds the
// first-step correction and pins the boundary coefficients).
template <typename T>
__device__ void iteration(const Ctx<T>& x, const Lds<T>& L, int TT, int k) {
  const DevCfg& c = x.c;
  const int n = x.n, D = x.D, m = x.m, mf = x.mf, nD = x.nD;
  for (int q = threadIdx.x; q < x.nDm; q += blockDim.x) L.g[q] = T(0);
  __syncthreads();
  for (int t0 = 0; t0 < c.H; t0 += TT) {
    const int TTc = min(TT, c.H - t0);
    eval_tile<T>(c, x.basis, L.xi, L.Y, t0, TTc, TT);
    __syncthreads();
    for (int q = threadIdx.x; q < n * TTc; q += blockDim.x) {
      const int i = q / TTc, tt = q - (q / TTc) * TTc;
      T xi_[3] = {T(0), T(0), T(0)}, C[3] = {T(0), T(0), T(0)};
      SF_FOR_DIM(d, D) xi_[d] = L.Y[(i * D + d) * TT + tt];
      for (int j = 0; j < n; ++j) {
        if (j == i) continue;
        T r[3], R[3];
        SF_FOR_DIM(d, D) r[d] = xi_[d] - L.Y[(j * D + d) * TT + tt];
        coll_resid<T>(r, D, x.ia2, x.ib2, x.a, x.b, i < j, R);
        SF_FOR_DIM(d, D) C[d] += R[d];
      }
      if (c.ws_on) {   // workspace rows share the position basis; weight rho_w = rho_c ws_scale
        T R[3];
        ws_resid<T>(xi_, D, x.wc, x.ws_ia2, x.ws_ib2, R);
        SF_FOR_DIM(d, D) C[d] = fma(x.ws_scale, R[d], C[d]);
      }
      SF_FOR_DIM(d, D) L.Rb[(i * D + d) * TT + tt] = C[d];
      if (c.vel_on) {
        T v[3], R[3];
        SF_FOR_DIM(d, D) v[d] = L.Y[((n + i) * D + d) * TT + tt];
        ball_resid<T>(v, D, x.vmax, R);
        SF_FOR_DIM(d, D) L.Rb[((n + i) * D + d) * TT + tt] = R[d];
      }
      if (c.acc_on) {
        T v[3], R[3];
        SF_FOR_DIM(d, D) v[d] = L.Y[((2 * n + i) * D + d) * TT + tt];
        ball_resid<T>(v, D, x.amax, R);
        SF_FOR_DIM(d, D) L.Rb[((2 * n + i) * D + d) * TT + tt] = R[d];
      }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < x.nDm; q += blockDim.x) {
      const int row = q / m, kk = q - row * m;
      T ac = T(0), av = T(0), aa = T(0);
#pragma unroll 4
      for (int tt = 0; tt < TTc; ++tt) {
        const size_t brow = (size_t)(t0 + tt) * m + kk;
        ac = fma(x.basis[brow], L.Rb[row * TT + tt], ac);
        if (c.vel_on) av = fma(x.basis[(size_t)c.H * m + brow], L.Rb[(nD + row) * TT + tt], av);
        if (c.acc_on) aa = fma(x.basis[(size_t)2 * c.H * m + brow], L.Rb[(2 * nD + row) * TT + tt], aa);
      }
      L.g[q] += x.rho_c * ac + x.rho_v * av + x.rho_a * aa;
    }
    __syncthreads();
  }
  // multiplier step and QP step (incremental form on the free coefficients)
  for (int q = threadIdx.x; q < x.nDm; q += blockDim.x) {
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
    L.ybar[q] = s * x.inv_n;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < x.nDf; q += blockDim.x) {
    const int row = q / mf, f = q - row * mf, d = row % D;
    T acc = T(0);
#pragma unroll 4
    for (int f2 = 0; f2 < mf; ++f2) {
      acc = fma(x.X1[f * mf + f2], L.ybuf[row * mf + f2], acc);
      acc = fma(x.X01[f * mf + f2], L.ybar[d * mf + f2], acc);
    }
    L.xi[row * m + 3 + f] += acc;
  }
  if (k == 0) {
    for (int q = threadIdx.x; q < x.nD6; q += blockDim.x) {
      const int row = q / kNFix, r = q - row * kNFix;
      const int kk = r < 3 ? r : m - kNFix + r;
      L.xi[row * m + kk] = L.xp[q];
    }
  }
  __syncthreads();
}

}  // namespace gen
}  // namespace sf
