// Reverse-mode derivative of the unrolled SF iterations (the differentiable chain of the
// Appendix; used for eq. (NN_loss)-style training of the initialisation).
//
// One iteration, written in the direct form of eq. (xi_step):
//   Y = F xi,  R = Y - Pi(Y) per constraint block,  g = F^T (rho R),  lambda' = lambda - g,
//   xi' = xi_p + Z S_f Z^T (xi_bar + lambda' - g + G_rho (xi - xi_p)),
// where Z selects the free coefficients and S_f = J (x) X0 + (I - J) (x) X1.
// Given cotangents (gxi', glam') and u = Z S_f Z^T gxi' (S_f is symmetric):
//   gxi_bar += u,   glam = glam' + u,   g_g = -glam - u,
//   gY = J_R^T (rho F g_g) per block (J_R the 3x3 Jacobian of the block's residual),
//   gxi = G_rho u + F^T gY, whose free part is gxi'_free - u + (F^T gY)_free.
// Pinned coefficients of xi^k are constants for k >= 1, so their cotangent is only formed at
// k = 0 (G_rho u restricted to them, from Gfx and Rfx).  The fixed-point residual term of
// eq. (NN_loss), w sum_k ||z^{k+1} - z^k||^2 with z = (xi, lambda), adds 2 w (z^{k+1} - z^k) to
// the cotangent of z^{k+1} before each reverse step and subtracts it from that of z^k after.  The forward states inside a
// checkpoint segment are recomputed with the generic iteration and kept in a global scratch.
#include "sf_generic_impl.h"
#include "sf_adjoint.h"

#include <algorithm>

namespace sf {
namespace {

using namespace gen;

struct AdjPlan {
  size_t gxi, glam, gxb, u, gg, pend, ubar, W, GY, total;
};

__host__ __device__ inline AdjPlan adj_plan(const DevCfg& c, int TT) {
  const size_t nDm = (size_t)c.n * c.D * c.m;
  const size_t tile = (size_t)3 * c.n * c.D * TT;
  AdjPlan p;
  size_t o = lds_plan(c, TT).total;
  p.gxi = o; o += nDm;
  p.glam = o; o += nDm;
  p.gxb = o; o += nDm;
  p.u = o; o += nDm;
  p.gg = o; o += nDm;
  p.pend = o; o += nDm;
  p.ubar = o; o += (size_t)c.D * (c.mf > 0 ? c.mf : 1);
  p.W = o; o += tile;
  p.GY = o; o += tile;
  p.total = o;
  return p;
}

// J^T v for the collision residual R(r) = r min(0, 1 - 1/||s||), s = M^{-1} r:
// active (||s|| < 1): f v + rs^3 (M^{-2} r)(r . v), else 0 (also 0 for coincident robots).
template <typename T>
__device__ __forceinline__ void coll_jt(const T* r, const T* v, int D, T ia2, T ib2, T* out) {
  T ss = r[0] * r[0] * ia2 + r[1] * r[1] * ia2;
  if (D == 3) ss += r[2] * r[2] * ib2;
  SF_FOR_DIM(d, D) out[d] = T(0);
  if (ss >= tiny_sq<T>() && ss < T(1)) {
    const T rs = rsq<T>(ss);
    const T f = T(1) - rs;
    T rv = T(0);
    SF_FOR_DIM(d, D) rv += r[d] * v[d];
    const T k3 = rs * rs * rs * rv;
    SF_FOR_DIM(d, D) out[d] = f * v[d] + k3 * r[d] * (d == 2 ? ib2 : ia2);
  }
}

// J^T w for a bound ball R(v) = v max(0, 1 - L/||v||): active: h w + L rs^3 v (v . w).
template <typename T>
__device__ __forceinline__ void ball_jt(const T* v, const T* w, int D, T lim, T* out) {
  T ss = v[0] * v[0] + v[1] * v[1];
  if (D == 3) ss += v[2] * v[2];
  SF_FOR_DIM(d, D) out[d] = T(0);
  if (ss > lim * lim) {
    const T rs = rsq<T>(ss);
    const T h = T(1) - lim * rs;
    T vw = T(0);
    SF_FOR_DIM(d, D) vw += v[d] * w[d];
    const T k3 = lim * rs * rs * rs * vw;
    SF_FOR_DIM(d, D) out[d] = h * w[d] + k3 * v[d];
  }
}

// J^T w for the workspace residual R(p) = q max(0, 1 - 1/||s||), q = p - p_w, s = M_w^{-1} q:
// active (||s|| > 1): f w + rs^3 (M_w^{-2} q)(q . w) with f = 1 - rs, else 0.
template <typename T>
__device__ __forceinline__ void ws_jt(const T* p, const T* w, int D, const T* wc, T ia2, T ib2, T* out) {
  T q[3] = {T(0), T(0), T(0)};
  T ss = T(0);
  SF_FOR_DIM(d, D) {
    q[d] = p[d] - wc[d];
    ss += q[d] * q[d] * (d == 2 ? ib2 : ia2);
  }
  SF_FOR_DIM(d, D) out[d] = T(0);
  if (ss > T(1)) {
    const T rs = rsq<T>(ss);
    const T f = T(1) - rs;
    T qw = T(0);
    SF_FOR_DIM(d, D) qw += q[d] * w[d];
    const T k3 = rs * rs * rs * qw;
    SF_FOR_DIM(d, D) out[d] = f * w[d] + k3 * q[d] * (d == 2 ? ib2 : ia2);
  }
}

// dst[q] += sum_tt basis_b[t0+tt][k] * tile_b[row][tt] over the enabled bases (no weights).
template <typename T>
__device__ void backproject_tile(const Ctx<T>& x, const T* tile, T* dst, int t0, int TTc, int TT) {
  const DevCfg& c = x.c;
  const int m = x.m, nD = x.nD;
  for (int q = threadIdx.x; q < x.nDm; q += blockDim.x) {
    const int row = q / m, kk = q - row * m;
    T acc = T(0);
#pragma unroll 4
    for (int tt = 0; tt < TTc; ++tt) {
      const size_t brow = (size_t)(t0 + tt) * m + kk;
      acc = fma(x.basis[brow], tile[row * TT + tt], acc);
      if (c.vel_on) acc = fma(x.basis[(size_t)c.H * m + brow], tile[(nD + row) * TT + tt], acc);
      if (c.acc_on) acc = fma(x.basis[(size_t)2 * c.H * m + brow], tile[(2 * nD + row) * TT + tt], acc);
    }
    dst[q] += acc;
  }
}

// Final-residual term of the loss, g_resid ||r_p^K||^2 with r_p = F xi^K - e(F xi^{K-1}) (eq.
// primal_residual), needs L.xprev = xi^{K-1} and L.g = xi^K: adds its cotangent of xi^K to gxi and
// keeps the one of xi^{K-1} in pend (added after the reverse step of iteration K - 1).
template <typename T>
__device__ void resid_term(const Ctx<T>& x, const Lds<T>& L, T* Wt, T* GY, T* gxi, T* pend, T gres, int TT,
                           int t_begin = 0, int t_end = 1 << 30) {
  const DevCfg& c = x.c;
  const int n = x.n, D = x.D;
  for (int t0 = t_begin; t0 < min(c.H, t_end); t0 += TT) {
    const int TTc = min(TT, c.H - t0);
    eval_tile<T>(c, x.basis, L.xprev, L.Y, t0, TTc, TT);
    eval_tile<T>(c, x.basis, L.g, Wt, t0, TTc, TT);
    __syncthreads();
    for (int q = threadIdx.x; q < n * TTc; q += blockDim.x) {
      const int i = q / TTc, tt = q - (q / TTc) * TTc;
      T Ai[3] = {T(0), T(0), T(0)}, Bi[3] = {T(0), T(0), T(0)};
      for (int j = 0; j < n; ++j) {
        if (j == i) continue;
        T rp[3], rn[3], R[3], gr[3], jt[3];
        SF_FOR_DIM(d, D) {
          rp[d] = L.Y[(i * D + d) * TT + tt] - L.Y[(j * D + d) * TT + tt];
          rn[d] = Wt[(i * D + d) * TT + tt] - Wt[(j * D + d) * TT + tt];
        }
        coll_resid<T>(rp, D, x.ia2, x.ib2, x.a, x.b, i < j, R);
        SF_FOR_DIM(d, D) gr[d] = T(2) * gres * (rn[d] - (rp[d] - R[d]));
        coll_jt<T>(rp, gr, D, x.ia2, x.ib2, jt);
        SF_FOR_DIM(d, D) {
          Ai[d] += gr[d];
          Bi[d] += jt[d] - gr[d];
        }
      }
      if (c.ws_on) {   // workspace rows: r_p = p_new - e(p_prev)
        T v[3], R[3], gr[3], jt[3];
        SF_FOR_DIM(d, D) v[d] = L.Y[(i * D + d) * TT + tt];
        ws_resid<T>(v, D, x.wc, x.ws_ia2, x.ws_ib2, R);
        SF_FOR_DIM(d, D) gr[d] = T(2) * gres * (Wt[(i * D + d) * TT + tt] - (v[d] - R[d]));
        ws_jt<T>(v, gr, D, x.wc, x.ws_ia2, x.ws_ib2, jt);
        SF_FOR_DIM(d, D) {
          Ai[d] += gr[d];
          Bi[d] += jt[d] - gr[d];
        }
      }
      SF_FOR_DIM(d, D) {
        GY[(i * D + d) * TT + tt] = Ai[d];
        L.Rb[(i * D + d) * TT + tt] = Bi[d];
      }
      for (int bsel = 1; bsel < 3; ++bsel) {
        const bool on = bsel == 1 ? c.vel_on : c.acc_on;
        if (!on) continue;
        const T lim = bsel == 1 ? x.vmax : x.amax;
        T v[3], R[3], gr[3], jt[3];
        SF_FOR_DIM(d, D) v[d] = L.Y[((bsel * n + i) * D + d) * TT + tt];
        ball_resid<T>(v, D, lim, R);
        SF_FOR_DIM(d, D)
          gr[d] = T(2) * gres * (Wt[((bsel * n + i) * D + d) * TT + tt] - (v[d] - R[d]));
        ball_jt<T>(v, gr, D, lim, jt);
        SF_FOR_DIM(d, D) {
          GY[((bsel * n + i) * D + d) * TT + tt] = gr[d];
          L.Rb[((bsel * n + i) * D + d) * TT + tt] = jt[d] - gr[d];
        }
      }
    }
    __syncthreads();
    backproject_tile<T>(x, GY, gxi, t0, TTc, TT);
    backproject_tile<T>(x, L.Rb, pend, t0, TTc, TT);
    __syncthreads();
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
adjoint_kernel(const DevCfg* __restrict__ cfgs, const T* __restrict__ tab, const DevProblem* __restrict__ probs,
               const WorkItem* __restrict__ items, int n_items, const T* __restrict__ xi_bar,
               const T* __restrict__ bvals, int iters, const T* __restrict__ ckpt, int ckpt_every,
               int64_t ckpt_stride, const T* __restrict__ g_xi_out, const T* __restrict__ g_lam_out,
               const T* __restrict__ g_resid, const T* __restrict__ w_fpr, T* __restrict__ g_xi0,
               T* __restrict__ g_lam0,
               T* __restrict__ g_xi_bar, T* __restrict__ states, int64_t state_stride, int TT) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const WorkItem w = items[it];
    const DevProblem pr = probs[w.problem];
    const Ctx<T> x = make_ctx<T>(cfgs[pr.cfg], tab);
    const DevCfg& c = x.c;
    const Lds<T> L = carve<T>(smem, lds_plan(c, TT));
    const AdjPlan A = adj_plan(c, TT);
    T* gxi = smem + A.gxi;
    T* glam = smem + A.glam;
    T* gxb = smem + A.gxb;
    T* u = smem + A.u;
    T* gg = smem + A.gg;
    T* pend = smem + A.pend;
    T* ubar = smem + A.ubar;
    T* Wt = smem + A.W;
    T* GY = smem + A.GY;
    const int n = x.n, D = x.D, m = x.m, mf = x.mf, nD = x.nD, nDm = x.nDm;
    const int nseg = (iters + ckpt_every - 1) / ckpt_every;
    for (int sl = w.first; sl < w.first + w.count; ++sl) {
      const int64_t coef = pr.coef_off + (int64_t)sl * nDm;
      const int64_t sidx = pr.sample_base + sl;
      T* st = states + (int64_t)it * state_stride;   // one sample per work item: xi states,
      T* stl = st + (int64_t)(ckpt_every + 1) * nDm;  // then lambda states of a segment
      const T gres = g_resid ? g_resid[sidx] : T(0);
      const T wf = w_fpr ? w_fpr[sidx] : T(0);
      setup_sample<T>(x, L, xi_bar + coef, bvals + pr.bnd_off, ckpt + coef, ckpt + ckpt_stride + coef);
      for (int q = threadIdx.x; q < nDm; q += blockDim.x) {
        gxi[q] = g_xi_out ? g_xi_out[coef + q] : T(0);
        glam[q] = g_lam_out ? g_lam_out[coef + q] : T(0);
        gxb[q] = T(0);
        pend[q] = T(0);
      }
      __syncthreads();
      for (int seg = nseg - 1; seg >= 0; --seg) {
        const int s0 = seg * ckpt_every, s1 = min(s0 + ckpt_every, iters);
        const int64_t cb = (int64_t)seg * 2 * ckpt_stride + coef;
        for (int q = threadIdx.x; q < nDm; q += blockDim.x) {
          L.xi[q] = ckpt[cb + q];
          L.lam[q] = ckpt[cb + ckpt_stride + q];
          st[q] = ckpt[cb + q];
          stl[q] = ckpt[cb + ckpt_stride + q];
        }
        __syncthreads();
        for (int k = s0; k < s1; ++k) {
          iteration<T>(x, L, TT, k);
          for (int q = threadIdx.x; q < nDm; q += blockDim.x) {
            st[(int64_t)(k - s0 + 1) * nDm + q] = L.xi[q];
            stl[(int64_t)(k - s0 + 1) * nDm + q] = L.lam[q];
          }
          __syncthreads();
        }
        // residual term of the loss: r_p = F xi^K - e(F xi^{K-1}) (eq. primal_residual)
        if (seg == nseg - 1 && g_resid && gres != T(0)) {
          const T* xk = st + (int64_t)(s1 - s0) * nDm;
          const T* xk1 = st + (int64_t)(s1 - s0 - 1) * nDm;
          for (int q = threadIdx.x; q < nDm; q += blockDim.x) {
            L.xprev[q] = xk1[q];
            L.g[q] = xk[q];
          }
          __syncthreads();
          resid_term<T>(x, L, Wt, GY, gxi, pend, gres, TT);
        }
        // reverse sweep over the segment
        for (int k = s1 - 1; k >= s0; --k) {
          // fixed-point residual term: d/dz^{k+1} of w ||z^{k+1} - z^k||^2
          auto fpr_term = [&](T sign) {
            if (wf == T(0)) return;
            for (int q = threadIdx.x; q < nDm; q += blockDim.x) {
              const int64_t a1 = (int64_t)(k - s0 + 1) * nDm + q, a0 = (int64_t)(k - s0) * nDm + q;
              gxi[q] += sign * T(2) * wf * (st[a1] - st[a0]);
              glam[q] += sign * T(2) * wf * (stl[a1] - stl[a0]);
            }
            __syncthreads();
          };
          fpr_term(T(1));
          for (int q = threadIdx.x; q < nDm; q += blockDim.x) L.xprev[q] = st[(int64_t)(k - s0) * nDm + q];
          // u = Z S_f Z^T gxi
          for (int q = threadIdx.x; q < D * mf; q += blockDim.x) {
            const int d = q / mf, f = q - d * mf;
            T s = T(0);
            for (int i = 0; i < n; ++i) s += gxi[(i * D + d) * m + 3 + f];
            ubar[q] = s * x.inv_n;
          }
          __syncthreads();
          for (int q = threadIdx.x; q < nDm; q += blockDim.x) {
            const int row = q / m, kk = q - row * m, f = kk - 3, d = row % D;
            T acc = T(0);
            if (f >= 0 && f < mf) {
#pragma unroll 4
              for (int f2 = 0; f2 < mf; ++f2) {
                acc = fma(x.X1[f * mf + f2], gxi[row * m + 3 + f2], acc);
                acc = fma(x.X01[f * mf + f2], ubar[d * mf + f2], acc);
              }
            }
            u[q] = acc;
          }
          __syncthreads();
          for (int q = threadIdx.x; q < nDm; q += blockDim.x) {
            const T uq = u[q];
            gxb[q] += uq;
            const T gl = glam[q] + uq;
            glam[q] = gl;
            gg[q] = -gl - uq;
          }
          // mean of u over robots (for the pinned cotangent at k = 0)
          for (int q = threadIdx.x; q < D * mf; q += blockDim.x) {
            const int d = q / mf, f = q - d * mf;
            T s = T(0);
            for (int i = 0; i < n; ++i) s += u[(i * D + d) * m + 3 + f];
            ubar[q] = s * x.inv_n;
          }
          __syncthreads();
          for (int q = threadIdx.x; q < nDm; q += blockDim.x) {
            const int row = q / m, kk = q - row * m, f = kk - 3, d = row % D;
            T v;
            if (f >= 0 && f < mf) {
              v = gxi[q] - u[q];
            } else if (k == 0) {
              const int r = kk < 3 ? kk : kk - (m - kNFix);
              T acc = T(0);
              for (int f2 = 0; f2 < mf; ++f2) {
                const T uu = u[row * m + 3 + f2];
                acc = fma(x.n_rho_c * x.Gfx[f2 * kNFix + r], uu - ubar[d * mf + f2], acc);
                acc = fma(x.Rfx[f2 * kNFix + r], uu, acc);
              }
              v = acc;
            } else {
              v = T(0);
            }
            gxi[q] = v;
          }
          __syncthreads();
          for (int t0 = 0; t0 < c.H; t0 += TT) {
            const int TTc = min(TT, c.H - t0);
            eval_tile<T>(c, x.basis, L.xprev, L.Y, t0, TTc, TT);
            eval_tile<T>(c, x.basis, gg, Wt, t0, TTc, TT);
            __syncthreads();
            for (int q = threadIdx.x; q < n * TTc; q += blockDim.x) {
              const int i = q / TTc, tt = q - (q / TTc) * TTc;
              T acc[3] = {T(0), T(0), T(0)};
              for (int j = 0; j < n; ++j) {
                if (j == i) continue;
                T r[3], gr[3], jt[3];
                SF_FOR_DIM(d, D) {
                  r[d] = L.Y[(i * D + d) * TT + tt] - L.Y[(j * D + d) * TT + tt];
                  gr[d] = x.rho_c * (Wt[(i * D + d) * TT + tt] - Wt[(j * D + d) * TT + tt]);
                }
                coll_jt<T>(r, gr, D, x.ia2, x.ib2, jt);
                SF_FOR_DIM(d, D) acc[d] += jt[d];
              }
              if (c.ws_on) {   // workspace rows (weight rho_w) share the position basis
                T p[3], gr[3], jt[3];
                SF_FOR_DIM(d, D) {
                  p[d] = L.Y[(i * D + d) * TT + tt];
                  gr[d] = x.rho_c * x.ws_scale * Wt[(i * D + d) * TT + tt];
                }
                ws_jt<T>(p, gr, D, x.wc, x.ws_ia2, x.ws_ib2, jt);
                SF_FOR_DIM(d, D) acc[d] += jt[d];
              }
              SF_FOR_DIM(d, D) GY[(i * D + d) * TT + tt] = acc[d];
              for (int bsel = 1; bsel < 3; ++bsel) {
                const bool on = bsel == 1 ? c.vel_on : c.acc_on;
                if (!on) continue;
                const T lim = bsel == 1 ? x.vmax : x.amax;
                const T rho = bsel == 1 ? x.rho_v : x.rho_a;
                T v[3], gr[3], jt[3];
                SF_FOR_DIM(d, D) {
                  v[d] = L.Y[((bsel * n + i) * D + d) * TT + tt];
                  gr[d] = rho * Wt[((bsel * n + i) * D + d) * TT + tt];
                }
                ball_jt<T>(v, gr, D, lim, jt);
                SF_FOR_DIM(d, D) GY[((bsel * n + i) * D + d) * TT + tt] = jt[d];
              }
            }
            __syncthreads();
            backproject_tile<T>(x, GY, gxi, t0, TTc, TT);
            __syncthreads();
          }
          if (k == iters - 1 && g_resid && gres != T(0)) {
            for (int q = threadIdx.x; q < nDm; q += blockDim.x) gxi[q] += pend[q];
            __syncthreads();
          }
          fpr_term(T(-1));   // ... and d/dz^k
        }
      }
      for (int q = threadIdx.x; q < nDm; q += blockDim.x) {
        if (g_xi0) g_xi0[coef + q] = gxi[q];
        if (g_lam0) g_lam0[coef + q] = glam[q];
        if (g_xi_bar) g_xi_bar[coef + q] = gxb[q];
      }
      __syncthreads();
    }
  }
}

// The final-residual term for the MFMA adjoint path, from the recomputed states xi^{K-1} (slot
// `slot` of `states`) and xi^K (slot `slot` + 1), slots 2 * stride elements apart.  One workgroup
// per (sample, time tile of TT steps): each writes its tile's contributions to the cotangents of
// xi^K and xi^{K-1} into part ([tile][2][stride]); the reduction kernel below adds them to g_xi_out
// in tile order (the order in which the generic kernel's resid_term accumulates them over the
// tiles).  LDS: xi^{K-1}, xi^K, the two tile accumulators and four tile buffers.
template <typename T>
__global__ void __launch_bounds__(kBlock)
adjoint_resid_tile_kernel(const DevCfg* __restrict__ cfgs, const T* __restrict__ tab,
                          const DevProblem* __restrict__ probs, const WorkItem* __restrict__ items, int n_items,
                          const T* __restrict__ states, int64_t stride, int slot, const T* __restrict__ g_resid,
                          T* __restrict__ part, int TT, int n_tiles) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  for (int wi = blockIdx.x; wi < n_items * n_tiles; wi += gridDim.x) {
    const int it = wi / n_tiles, tile = wi - it * n_tiles;
    const WorkItem w = items[it];
    const DevProblem pr = probs[w.problem];
    const Ctx<T> x = make_ctx<T>(cfgs[pr.cfg], tab);
    const int nDm = x.nDm, tsz = 3 * x.n * x.D * TT;
    Lds<T> L{};
    L.xprev = smem;
    L.g = smem + nDm;
    T* gxi = smem + 2 * nDm;
    T* pd = smem + 3 * nDm;
    L.Y = smem + 4 * nDm;
    L.Rb = L.Y + tsz;
    T* Wt = L.Rb + tsz;
    T* GY = Wt + tsz;
    const int t0 = tile * TT;
    for (int sl = w.first; sl < w.first + w.count; ++sl) {
      const int64_t coef = pr.coef_off + (int64_t)sl * nDm;
      const T gres = g_resid[pr.sample_base + sl];
      const bool live = gres != T(0) && t0 < x.c.H;
      if (live) {
        const T* xk1 = states + (int64_t)slot * 2 * stride + coef;
        const T* xk = xk1 + 2 * stride;
        for (int q = threadIdx.x; q < nDm; q += blockDim.x) {
          L.xprev[q] = xk1[q];
          L.g[q] = xk[q];
          gxi[q] = T(0);
          pd[q] = T(0);
        }
        __syncthreads();
        resid_term<T>(x, L, Wt, GY, gxi, pd, gres, TT, t0, t0 + TT);
      }
      T* out = part + (int64_t)tile * 2 * stride + coef;
      for (int q = threadIdx.x; q < nDm; q += blockDim.x) {
        out[q] = live ? gxi[q] : T(0);
        out[stride + q] = live ? pd[q] : T(0);
      }
      __syncthreads();
    }
  }
}

// carry = (g_xi_out + the tiles' xi^K cotangents in tile order, g_lam_out, 0), pend = the tiles' xi^{K-1}
// cotangents in tile order; one thread per coefficient.
template <typename T>
__global__ void adjoint_resid_reduce_kernel(int64_t stride, int n_tiles, const T* __restrict__ part,
                                            const T* __restrict__ g_xi_out, const T* __restrict__ g_lam_out,
                                            T* __restrict__ carry, T* __restrict__ pend) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < stride; q += (int64_t)gridDim.x * blockDim.x) {
    T gx = g_xi_out ? g_xi_out[q] : T(0), pe = T(0);
    for (int t = 0; t < n_tiles; ++t) {
      gx += part[(int64_t)t * 2 * stride + q];
      pe += part[((int64_t)t * 2 + 1) * stride + q];
    }
    carry[q] = gx;
    carry[stride + q] = g_lam_out ? g_lam_out[q] : T(0);
    carry[2 * stride + q] = T(0);
    pend[q] = pe;
  }
}

}  // namespace

size_t adjoint_lds_bytes(const DevCfg& c, int tile, size_t elem) { return adj_plan(c, tile).total * elem; }

size_t adjoint_resid_tile_lds_bytes(const DevCfg& c, int tile) {
  const size_t nDm = (size_t)c.n * c.D * c.m;
  return (4 * nDm + 4 * (size_t)3 * c.n * c.D * tile) * sizeof(float);
}

hipError_t launch_adjoint_resid_tiles(const AdjointArgs& a, const float* states, int64_t stride, int slot,
                                      float* part, int n_tiles, float* carry, float* pend) {
  auto kern = adjoint_resid_tile_kernel<float>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)a.lds_bytes);
  if (e != hipSuccess) return e;
  const int64_t n_wg = (int64_t)a.n_items * n_tiles;
  hipLaunchKernelGGL(kern, dim3((unsigned)std::min<int64_t>(n_wg, 65536)), dim3(kBlock), a.lds_bytes, a.stream,
                     a.cfgs, static_cast<const float*>(a.tab), a.probs, a.items, a.n_items, states, stride, slot,
                     static_cast<const float*>(a.g_resid), part, a.tile, n_tiles);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t blocks = std::min<int64_t>((stride + 255) / 256, 16384);
  hipLaunchKernelGGL(adjoint_resid_reduce_kernel<float>, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0,
                     a.stream, stride, n_tiles, part, static_cast<const float*>(a.g_xi_out),
                     static_cast<const float*>(a.g_lam_out), carry, pend);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint(const AdjointArgs& a) {
  auto kern = adjoint_kernel<T>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)a.lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(a.n_items), dim3(kBlock), a.lds_bytes, a.stream, a.cfgs,
                     static_cast<const T*>(a.tab), a.probs, a.items, a.n_items, static_cast<const T*>(a.xi_bar),
                     static_cast<const T*>(a.bvals), a.iters, static_cast<const T*>(a.ckpt), a.ckpt_every,
                     a.ckpt_stride, static_cast<const T*>(a.g_xi_out), static_cast<const T*>(a.g_lam_out),
                     static_cast<const T*>(a.g_resid), static_cast<const T*>(a.w_fpr), static_cast<T*>(a.g_xi0),
                     static_cast<T*>(a.g_lam0),
                     static_cast<T*>(a.g_xi_bar), static_cast<T*>(a.states), a.state_stride, a.tile);
  return hipGetLastError();
}

template hipError_t launch_adjoint<double>(const AdjointArgs& a);
template hipError_t launch_adjoint<float>(const AdjointArgs& a);

}  // namespace sf
