// Reverse sweep of the unrolled SF iterations on the matrix cores (fp32), one checkpoint segment per
// launch; the segment's forward states are recomputed beforehand by the forward MFMA kernel.
//
// One iteration, in the direct form of eq. (xi_step) (see sf_adjoint.hip for the derivation):
//   Y = F xi,  R = Y - Pi(Y) per constraint block,  g = F^T (rho R),  lambda' = lambda - g,
//   xi' = xi_p + Z S_f Z^T (xi_bar + lambda' - g + G_rho (xi - xi_p)).
// Given the cotangents (gxi', glam') and u = Z S_f Z^T gxi':
//   gxi_bar += u,  glam = glam' + u,  gg = -glam - u,
//   gxi = (gxi' - u on the free coefficients; G_rho u on the pinned ones at k = 0, else 0)
//         + F^T J_R^T (rho F gg),
// with J_R the 3x3 Jacobian of each active block's residual (collision pairs with ||s|| < 1, bound
// balls with ||v|| > vmax); inactive blocks contribute nothing.
//
// One workgroup of four waves per sample; the cotangents stay in LDS for the segment.  The F and
// F^T products run as in the forward kernel: per 16-step time tile, v_mfma_f32_16x16x4f32 gives
// positions (and velocities, accelerations) of xi^k and of gg for 16 robots at 16 times; the pairs
// whose position boxes over the tile come within the safety distance are listed (the box gap bounds
// every pair-time's gap, so no active pair is missed), their Jacobian-transpose products are
// scattered into an LDS accumulator, and the back-projection F^T is an MFMA product over the
// tiles with a nonzero accumulator.  Bound balls are evaluated in the product registers.
#include "sf_fast_kernel.h"
#include "sf_adjoint.h"

namespace sf {
namespace {

using namespace fastk;

constexpr int kAW = 4;   // waves per workgroup

// LDS plan (words).  Per sample: the cotangents gxi, glam, gxb, the QP-step image u, the multiplier
// cotangent gg and the state xi^k, robot means, the pair table.  Per wave: positions of xi^k (Xt) and
// of gg (Wt) and the Jacobian-transpose accumulator (Ct) of one tile as [axis][robot][time] with the
// forward kernel's swizzled rows, boxes, the tile's pair list, and the wave's partial back-projection.
struct AdjLds {
  int gxi, glam, gxb, uu, gg, xk, ubar, pairs, tiles, per_wave, total;
  int xt, wt, ct, bb, plist, part;
};

__host__ __device__ inline AdjLds adj_fast_plan(const DevCfg& c) {
  const int nDm = c.n * 3 * c.m;
  AdjLds p;
  int o = 0;
  p.gxi = o; o += nDm;
  p.glam = o; o += nDm;
  p.gxb = o; o += nDm;
  p.uu = o; o += nDm;
  p.gg = o; o += nDm;
  p.xk = o; o += nDm;
  p.ubar = o; o += 3 * 16;
  p.pairs = o; o += 16 * 15 / 2;
  o = (o + 3) & ~3;
  p.xt = 0;
  p.wt = 3 * 16 * 16;
  p.ct = 6 * 16 * 16;
  p.bb = 9 * 16 * 16;
  p.plist = p.bb + kBoxRow * 16;
  p.part = (p.plist + 16 * 15 / 2 + 1 + 3) & ~3;
  p.per_wave = (p.part + nDm + 3) & ~3;
  p.tiles = o;
  o += kAW * p.per_wave;
  p.total = o;
  return p;
}

template <int KS>
__global__ void __launch_bounds__(64 * kAW) adjoint_fast_kernel(AdjFastArgs A) {
  extern __shared__ __align__(16) float smem[];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tid = threadIdx.x, lane = tid & 63, col = lane & 15, grp = lane >> 4;
  constexpr int nthr = 64 * kAW;
  const float4* a32 = static_cast<const float4*>(A.a32);
  const int64_t stride = A.stride;
  for (int it = blockIdx.x; it < A.n_items; it += gridDim.x) {
    const WorkItem w = A.items[it];
    const DevProblem pr = A.probs[w.problem];
    const DevCfg c = A.cfgs[pr.cfg];
    const AdjLds Lp = adj_fast_plan(c);
    const int n = c.n, m = c.m, mf = c.mf, H = c.H, nDm = n * 3 * m;
    const int Np = n * (n - 1) / 2, NT = (H + 15) / 16;
    const float* X1 = A.tab + c.off_X1;
    const float* X01 = A.tab + c.off_X01;
    const float* Gfx = A.tab + c.off_Gfx;
    const float* Rfx = A.tab + c.off_Rfx;
    const float ia2 = (float)c.inv_a2, ib2 = (float)c.inv_b2;
    const float vmax = (float)c.vmax, amax = (float)c.amax;
    const float n_rho_c = (float)c.n_rho_c, inv_n = 1.0f / (float)n;
    const float4* a32c = a32 + c.off_a32;
    float* sgxi = smem + Lp.gxi;
    float* sglam = smem + Lp.glam;
    float* sgxb = smem + Lp.gxb;
    float* suu = smem + Lp.uu;
    float* sgg = smem + Lp.gg;
    float* sxk = smem + Lp.xk;
    float* subar = smem + Lp.ubar;
    int* spairs = reinterpret_cast<int*>(smem + Lp.pairs);
    float* wbuf = smem + Lp.tiles + wave * Lp.per_wave;
    float* Xt = wbuf + Lp.xt;
    float* Wt = wbuf + Lp.wt;
    float* Ct = wbuf + Lp.ct;
    float* bb = wbuf + Lp.bb;
    int* tl = reinterpret_cast<int*>(wbuf + Lp.plist);
    float* part = wbuf + Lp.part;
    for (int i = tid; i < n; i += nthr) {
      int p = i * n - i * (i + 1) / 2;
      for (int j = i + 1; j < n; ++j) spairs[p++] = i | (j << 8);
    }
    for (int q = lane; q < 3 * 16 * 16; q += 64) Ct[q] = 0.0f;   // kept zero between tiles
    __syncthreads();
    int mypair[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) mypair[r] = (64 * r + lane < Np) ? spairs[64 * r + lane] : -1;

    for (int sl = w.first; sl < w.first + w.count; ++sl) {
      const int64_t coef = pr.coef_off + (int64_t)sl * nDm;
      const int64_t sidx = pr.sample_base + sl;
      const float wf = A.w_fpr ? A.w_fpr[sidx] : 0.0f;
      float* cg = A.carry + coef;
      for (int q = tid; q < nDm; q += nthr) {
        sgxi[q] = A.init ? (A.g_xi_out ? A.g_xi_out[coef + q] : 0.0f) : cg[q];
        sglam[q] = A.init ? (A.g_lam_out ? A.g_lam_out[coef + q] : 0.0f) : cg[stride + q];
        sgxb[q] = A.init ? 0.0f : cg[2 * stride + q];
      }
      __syncthreads();
      for (int r = A.len - 1; r >= 0; --r) {
        const int k = A.s0 + r;
        const float* xkg = A.states + (int64_t)r * 2 * stride + coef;   // xi^k, then lambda^k
        const float* xk1g = xkg + 2 * stride;                            // xi^{k+1}, lambda^{k+1}
        // the fixed-point residual term's share for z^{k+1}, and the state xi^k
        for (int q = tid; q < nDm; q += nthr) {
          const float x0 = xkg[q];
          sxk[q] = x0;
          if (wf != 0.0f) {
            sgxi[q] += 2.0f * wf * (xk1g[q] - x0);
            sglam[q] += 2.0f * wf * (xk1g[stride + q] - xkg[stride + q]);
          }
        }
        __syncthreads();
        // u = Z S_f Z^T gxi: robot means of the free cotangents, then X1 and X01 per row
        for (int q = tid; q < 3 * mf; q += nthr) {
          const int d = q / mf, f = q - d * mf;
          float s = 0.0f;
          for (int i = 0; i < n; ++i) s += sgxi[(i * 3 + d) * m + 3 + f];
          subar[q] = s * inv_n;
        }
        __syncthreads();
        for (int q = tid; q < nDm; q += nthr) {
          const int row = q / m, kk = q - row * m, f = kk - 3, d = row % 3;
          float u = 0.0f;
          if (f >= 0 && f < mf)
            for (int f2 = 0; f2 < mf; ++f2) {
              u = fmaf(X1[f * mf + f2], sgxi[row * m + 3 + f2], u);
              u = fmaf(X01[f * mf + f2], subar[d * mf + f2], u);
            }
          suu[q] = u;
          sgxb[q] += u;
          const float gl = sglam[q] + u;
          sglam[q] = gl;
          sgg[q] = -gl - u;
        }
        __syncthreads();
        if (k == 0) {   // robot means of u for the pinned coefficients' cotangent
          for (int q = tid; q < 3 * mf; q += nthr) {
            const int d = q / mf, f = q - d * mf;
            float s = 0.0f;
            for (int i = 0; i < n; ++i) s += suu[(i * 3 + d) * m + 3 + f];
            subar[q] = s * inv_n;
          }
          __syncthreads();
        }
        for (int q = tid; q < nDm; q += nthr) {
          const int row = q / m, kk = q - row * m, f = kk - 3, d = row % 3;
          float v = 0.0f;
          if (f >= 0 && f < mf) {
            v = sgxi[q] - suu[q];
          } else if (k == 0) {
            const int r6 = kk < 3 ? kk : kk - (m - kNFix);
            for (int f2 = 0; f2 < mf; ++f2) {
              const float uu = suu[row * m + 3 + f2];
              v = fmaf(n_rho_c * Gfx[f2 * kNFix + r6], uu - subar[d * mf + f2], v);
              v = fmaf(Rfx[f2 * kNFix + r6], uu, v);
            }
          }
          sgxi[q] = v;
        }
        __syncthreads();

        // ---- F^T J_R^T (rho F gg) over this wave's time tiles ----
        {
          float bxk[3][KS], bgg[3][KS];
#pragma unroll
          for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int s = 0; s < KS; ++s) {
              const int kk = 4 * s + grp;
              const bool ok = col < n && kk < m;
              bxk[d][s] = ok ? sxk[(col * 3 + d) * m + kk] : 0.0f;
              bgg[d][s] = ok ? sgg[(col * 3 + d) * m + kk] : 0.0f;
            }
          f4 gacc[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) gacc[d] = f4{0.0f, 0.0f, 0.0f, 0.0f};
          auto s1 = [&](const float4 av, const float (&bx)[3][KS], f4 (&Y)[3]) {
            const float a1[4] = {av.x, av.y, av.z, av.w};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
              for (int s = 0; s < KS; ++s) acc = mfma4(a1[s], bx[d][s], acc);
              Y[d] = acc;
            }
          };
#pragma unroll 1
          for (int tau = wave; tau < NT; tau += kAW) {
            const int nt = min(16, H - 16 * tau);
            {
              f4 Y[3], G[3];
              const float4 av = a32c[((tau * 3) * 2) * 64 + lane];
              s1(av, bxk, Y);
              s1(av, bgg, G);
#pragma unroll
              for (int d = 0; d < 3; ++d) {
                *reinterpret_cast<f4*>(Xt + tile_at(d * 16 + col, 4 * grp)) = Y[d];
                *reinterpret_cast<f4*>(Wt + tile_at(d * 16 + col, 4 * grp)) = G[d];
              }
              float lo[3], hi[3];
#pragma unroll
              for (int d = 0; d < 3; ++d) {
                const f4 v = Y[d];
                lo[d] = grp_min(fminf(fminf(v[0], v[1]), fminf(v[2], v[3])));
                hi[d] = grp_max(fmaxf(fmaxf(v[0], v[1]), fmaxf(v[2], v[3])));
              }
              if (grp == 0) {
                float* bq = bb + col * kBoxRow;
                *reinterpret_cast<f4*>(bq) = f4{lo[0], lo[1], lo[2], 0.0f};
                *reinterpret_cast<f4*>(bq + 4) = f4{hi[0], hi[1], hi[2], 0.0f};
              }
            }
            wave_sync();
            // pairs whose boxes come within the safety distance (1e-4 relative slack): every
            // active pair-time of the tile is among them
            int count = 0;
            {
              bool act[2];
#pragma unroll
              for (int r2 = 0; r2 < 2; ++r2) {
                const int pij = mypair[r2] >= 0 ? mypair[r2] : (1 << 8);
                const int i = pij & 255, j = pij >> 8;
                const f4 li = *reinterpret_cast<const f4*>(bb + i * kBoxRow);
                const f4 hi = *reinterpret_cast<const f4*>(bb + i * kBoxRow + 4);
                const f4 lj = *reinterpret_cast<const f4*>(bb + j * kBoxRow);
                const f4 hj = *reinterpret_cast<const f4*>(bb + j * kBoxRow + 4);
                float g2 = 0.0f;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                  const float gap = fmaxf(0.0f, fmaxf(lj[d] - hi[d], li[d] - hj[d]));
                  g2 += gap * gap * (d == 2 ? ib2 : ia2);
                }
                act[r2] = mypair[r2] >= 0 && g2 < 1.0001f;
              }
#pragma unroll
              for (int r2 = 0; r2 < 2; ++r2) {
                const uint64_t mask = ballot(act[r2]);
                if (act[r2]) tl[1 + count + lanes_below(mask)] = mypair[r2];
                count += __popcll(mask);
              }
            }
            wave_sync();
            // Jacobian-transpose products of the active pair-times (lanes cover (pair, time) items)
            const int tsh = nt <= 4 ? 2 : (nt <= 8 ? 3 : 4);
            const int tt = lane & ((1 << tsh) - 1), ps = lane >> tsh, ppr = 64 >> tsh;
            bool nzc = false;
            for (int base = 0; base < count; base += ppr) {
              const int slot = base + ps;
              if (slot < count && tt < nt) {
                const int pij = tl[1 + slot];
                const int i = pij & 255, j = pij >> 8;
                const float rx = Xt[tile_at(i, tt)] - Xt[tile_at(j, tt)];
                const float ry = Xt[tile_at(16 + i, tt)] - Xt[tile_at(16 + j, tt)];
                const float rz = Xt[tile_at(32 + i, tt)] - Xt[tile_at(32 + j, tt)];
                const float ss = (rx * rx + ry * ry) * ia2 + rz * rz * ib2;
                if (ss >= FLT_MIN && ss < 1.0f) {
                  const float vx = Wt[tile_at(i, tt)] - Wt[tile_at(j, tt)];
                  const float vy = Wt[tile_at(16 + i, tt)] - Wt[tile_at(16 + j, tt)];
                  const float vz = Wt[tile_at(32 + i, tt)] - Wt[tile_at(32 + j, tt)];
                  const float rs = rsqrtf(ss);
                  const float f = 1.0f - rs;
                  const float k3 = rs * rs * rs * (rx * vx + ry * vy + rz * vz);
                  const float jx = f * vx + k3 * rx * ia2, jy = f * vy + k3 * ry * ia2, jz = f * vz + k3 * rz * ib2;
                  nzc = true;
                  atomicAdd(Ct + tile_at(i, tt), jx);
                  atomicAdd(Ct + tile_at(16 + i, tt), jy);
                  atomicAdd(Ct + tile_at(32 + i, tt), jz);
                  atomicAdd(Ct + tile_at(j, tt), -jx);
                  atomicAdd(Ct + tile_at(16 + j, tt), -jy);
                  atomicAdd(Ct + tile_at(32 + j, tt), -jz);
                }
              }
            }
            if (ballot(nzc) != 0) {
              wave_sync();
              const float4 bq = a32c[((tau * 3) * 2 + 1) * 64 + lane];   // rho_c P (zero past the horizon)
              const float b4[4] = {bq.x, bq.y, bq.z, bq.w};
#pragma unroll
              for (int d = 0; d < 3; ++d) {
                f4* cp = reinterpret_cast<f4*>(Ct + tile_at(d * 16 + col, 4 * grp));
                const f4 cr = *cp;
                *cp = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int s = 0; s < 4; ++s) gacc[d] = mfma4(cr[s], b4[s], gacc[d]);
              }
            }
            wave_sync();
            // bound balls: J^T (F_b gg) where ||F_b xi^k|| exceeds the bound
#pragma unroll
            for (int b = 1; b < 3; ++b) {
              if (!(b == 1 ? c.vel_on : c.acc_on)) continue;
              const float lim = b == 1 ? vmax : amax;
              const float4 av = a32c[((tau * 3 + b) * 2) * 64 + lane];
              f4 V[3], G[3];
              s1(av, bxk, V);
              s1(av, bgg, G);
              bool nz = false;
#pragma unroll
              for (int r4 = 0; r4 < 4; ++r4) {
                const float vx = V[0][r4], vy = V[1][r4], vz = V[2][r4];
                const float gx = G[0][r4], gy = G[1][r4], gz = G[2][r4];
                const float ss = vx * vx + vy * vy + vz * vz;
                float jx = 0.0f, jy = 0.0f, jz = 0.0f;
                if (ss > lim * lim) {
                  const float rs = rsqrtf(ss);
                  const float h = 1.0f - lim * rs;
                  const float k3 = lim * rs * rs * rs * (vx * gx + vy * gy + vz * gz);
                  jx = h * gx + k3 * vx;
                  jy = h * gy + k3 * vy;
                  jz = h * gz + k3 * vz;
                  nz = true;
                }
                V[0][r4] = jx;
                V[1][r4] = jy;
                V[2][r4] = jz;
              }
              if (ballot(nz) != 0) {
                const float4 bq = a32c[((tau * 3 + b) * 2 + 1) * 64 + lane];   // rho_b P_b
                const float b4[4] = {bq.x, bq.y, bq.z, bq.w};
#pragma unroll
                for (int d = 0; d < 3; ++d)
#pragma unroll
                  for (int s = 0; s < 4; ++s) gacc[d] = mfma4(V[d][s], b4[s], gacc[d]);
              }
            }
          }
          // this wave's partial back-projection (lane (col, grp): robots 4 grp + r, coefficient col)
#pragma unroll
          for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
              const int robot = 4 * grp + r4;
              if (robot < n && col < m) part[(robot * 3 + d) * m + col] = gacc[d][r4];
            }
        }
        __syncthreads();
        for (int q = tid; q < nDm; q += nthr) {
          float g = sgxi[q];
#pragma unroll
          for (int ww = 0; ww < kAW; ++ww) g += smem[Lp.tiles + ww * Lp.per_wave + Lp.part + q];
          if (A.pend && k == A.iters - 1) g += A.pend[coef + q];
          if (wf != 0.0f) {   // ... and its share for z^k
            g -= 2.0f * wf * (xk1g[q] - xkg[q]);
            sglam[q] -= 2.0f * wf * (xk1g[stride + q] - xkg[stride + q]);
          }
          sgxi[q] = g;
        }
        __syncthreads();
      }
      for (int q = tid; q < nDm; q += nthr) {
        if (A.last) {
          if (A.g_xi0) A.g_xi0[coef + q] = sgxi[q];
          if (A.g_lam0) A.g_lam0[coef + q] = sglam[q];
          if (A.g_xi_bar) A.g_xi_bar[coef + q] = sgxb[q];
        } else {
          cg[q] = sgxi[q];
          cg[stride + q] = sglam[q];
          cg[2 * stride + q] = sgxb[q];
        }
      }
      __syncthreads();
    }
  }
}

template <int KS>
hipError_t launch_ks(const AdjFastArgs& a) {
  auto kern = adjoint_fast_kernel<KS>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)a.lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(a.n_items), dim3(64 * kAW), a.lds_bytes, a.stream, a);
  return hipGetLastError();
}

}  // namespace

bool adjoint_fast_supported(const DevCfg& c) {
  return c.D == 3 && c.n <= 16 && c.m <= 16 && c.H <= 256 && !c.ws_on;
}

size_t adjoint_fast_lds_bytes(const DevCfg& c) { return (size_t)adj_fast_plan(c).total * sizeof(float); }

hipError_t launch_adjoint_fast(const AdjFastArgs& a, int KS) {
  switch (KS) {
    case 2: return launch_ks<2>(a);
    case 3: return launch_ks<3>(a);
    case 4: return launch_ks<4>(a);
    default: return hipErrorNotSupported;
  }
}

}  // namespace sf
