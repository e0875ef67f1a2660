// MFMA fast path of the safety filter for 3D swarms (n <= 32 robots, degree <= 15).
//
// One workgroup (W waves) owns one sample for the whole solve; xi, lambda and xi_bar stay in
// LDS.  The horizon is cut into 16-step time tiles and wave w owns tiles w, w + W, ...
// Per iteration and tile:
//   S1  Y_b = P_b xi for the three bases (position, velocity, acceleration; eq. poly) as
//       v_mfma_f32_16x16x4f32 products: rows = 16 times, columns = 16 robots of one axis.
//       Lane (col, grp) ends up holding robot col at times 4 grp .. 4 grp + 3, all axes.
//   S3  velocity/acceleration ball residuals in those registers (radial form of the d-step
//       with d in [0, 1]).
//   S2  collision residuals (alpha/beta/d steps in radial form): positions go to LDS, an exact
//       broad phase drops every pair whose position boxes over the tile are farther apart than
//       the safety distance (their residual is exactly zero), and the surviving pair-times are
//       projected and scattered into an LDS accumulator.
//   S4  g += P_b^T (rho_b R_b) as MFMA products, skipped for tiles whose residuals are all
//       zero.  The S1 output layout is exactly the A-operand layout this product needs.
// Then the multiplier step and the structured QP step of eq. (xi_step) on the free
// coefficients, as in the generic kernel.
#include "sf_fast.h"

#include <cfloat>

namespace sf {

static thread_local std::string g_fast_err;

std::string fast_last_error() { return g_fast_err; }

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Order LDS traffic between lanes of one wave (LDS instructions of a wave execute in order;
// this keeps the compiler from moving them and waits for outstanding LDS operations).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0));
}

// LDS plan (in 4-byte words).  Per-wave tile buffers: positions Xt and collision residual
// accumulator Ct as [axis][robot (16R)][time], rows padded to kRS words so that the 16-byte
// accesses of 8 consecutive lanes fall in distinct banks; boxes bb [robot][8]; active list.
constexpr int kRS = 20;
struct FastLds {
  int xi, lam, xb, xprev, gpart, xp, dlt, dbar, corr, ybuf, ybar, pairs, red, tiles, per_wave, total;
  int xt, ct, bb, plist;   // offsets inside one wave's tile region
};

__host__ __device__ inline FastLds fast_lds_plan(const DevCfg& c, int R, int W) {
  const int nDm = c.n * 3 * c.m, nDf = c.n * 3 * c.mf, nD6 = c.n * 3 * kNFix;
  const int nr = 16 * R, Npmax = nr * (nr - 1) / 2;
  FastLds p;
  int o = 0;
  p.xi = o; o += nDm;
  p.lam = o; o += nDm;
  p.xb = o; o += nDm;
  p.xprev = o; o += nDm;
  p.xp = o; o += nD6;
  p.dlt = o; o += nD6;
  p.dbar = o; o += 3 * kNFix;
  p.corr = o; o += nDf;
  p.ybuf = o; o += nDf;
  p.ybar = o; o += 3 * (c.mf > 0 ? c.mf : 1);
  p.pairs = o; o += Npmax;
  p.red = o; o += 2 * 64 * W;
  o = (o + 3) & ~3;                       // 16-byte alignment of the tile buffers
  p.xt = 0;
  p.ct = 3 * nr * kRS;
  p.bb = 6 * nr * kRS;
  p.plist = p.bb + 8 * nr;
  p.per_wave = (p.plist + Npmax + 3) & ~3;
  p.tiles = o;
  const int tiles_words = W * p.per_wave;
  const int gpart_words = W * nDm;         // per-wave partial g, aliases the tile buffers
  p.gpart = o;
  o += tiles_words > gpart_words ? tiles_words : gpart_words;
  p.total = o;
  return p;
}

__device__ __forceinline__ void coll_resid3(float rx, float ry, float rz, float ia2, float ib2, float b,
                                            float& Rx, float& Ry, float& Rz) {
  const float ss = (rx * rx + ry * ry) * ia2 + rz * rz * ib2;
  if (ss >= FLT_MIN) {
    const float f = fminf(0.0f, 1.0f - rsqrtf(ss));
    Rx = f * rx;
    Ry = f * ry;
    Rz = f * rz;
  } else {   // coincident: atan2(0, 0) = 0 targets (0, 0, b) for the pair (lower, upper)
    Rx = 0.0f;
    Ry = 0.0f;
    Rz = -b;
  }
}

template <int R, int KS, int W, int TQ>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(2, 2)))
fast_project_kernel(const DevCfg* __restrict__ cfgs, const float* __restrict__ tab,
                    const DevProblem* __restrict__ probs, const WorkItem* __restrict__ items, int n_items,
                    const float* __restrict__ xi_bar, const float* __restrict__ bvals,
                    const float* __restrict__ xi0, const float* __restrict__ lam0, int iters,
                    float* __restrict__ xi_out, float* __restrict__ lam_out, float* __restrict__ resid_out,
                    float* __restrict__ ckpt, int ckpt_every, int64_t ckpt_stride) {
  extern __shared__ __align__(16) float smem[];
  constexpr int NR = 16 * R;
  constexpr int PR = (NR * (NR - 1) / 2 + 63) / 64;   // 64-pair rounds of the broad phase
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int nthr = 64 * W;

  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const WorkItem w = items[it];
    const DevProblem pr = probs[w.problem];
    const DevCfg c = cfgs[pr.cfg];
    const FastLds L = fast_lds_plan(c, R, W);
    const int n = c.n, m = c.m, mf = c.mf, H = c.H;
    const int nDm = n * 3 * m, nDf = n * 3 * mf, nD6 = n * 3 * kNFix;
    const int Np = n * (n - 1) / 2;
    const int NT = (H + 15) / 16;
    const float* basis = tab + c.off_basis;
    const float* X1 = tab + c.off_X1;
    const float* X01 = tab + c.off_X01;
    const float* Bmap = tab + c.off_Bmap;
    const float* Gfx = tab + c.off_Gfx;
    const float* Rfx = tab + c.off_Rfx;
    const float ia2 = (float)c.inv_a2, ib2 = (float)c.inv_b2, sb = (float)c.b;
    const float vmax = (float)c.vmax, amax = (float)c.amax;
    const float n_rho_c = (float)c.n_rho_c, inv_n = 1.0f / (float)n;
    const float* bv = bvals + pr.bnd_off;
    float* sxi = smem + L.xi;
    float* slam = smem + L.lam;
    float* sxb = smem + L.xb;
    float* sxprev = smem + L.xprev;
    float* sxp = smem + L.xp;
    float* sdlt = smem + L.dlt;
    float* sdbar = smem + L.dbar;
    float* scorr = smem + L.corr;
    float* sybuf = smem + L.ybuf;
    float* sybar = smem + L.ybar;
    int* spairs = reinterpret_cast<int*>(smem + L.pairs);
    float* sred = smem + L.red;
    float* wbuf = smem + L.tiles + wave * L.per_wave;
    float* Xt = wbuf + L.xt;
    float* Ct = wbuf + L.ct;
    float* bb = wbuf + L.bb;
    int* plist = reinterpret_cast<int*>(wbuf + L.plist);
    float* gpart = smem + L.gpart;

    // pair table, lexicographic (i, j), i < j
    for (int i = tid; i < n; i += nthr) {
      int p = i * n - i * (i + 1) / 2;
      for (int j = i + 1; j < n; ++j) spairs[p++] = i | (j << 8);
    }
    // loop-invariant MFMA A operands of this wave's tiles (basis rows of S1)
    float a1[TQ][3][KS];
    const float rho[3] = {(float)c.rho_c, (float)c.rho_v, (float)c.rho_a};
#pragma unroll
    for (int q = 0; q < TQ; ++q) {
      const int t0 = 16 * (wave + W * q);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const int t = t0 + col, k = 4 * s + grp;
          a1[q][b][s] = (t < H && k < m) ? basis[((size_t)b * H + t) * m + k] : 0.0f;
        }
      }
    }

    __syncthreads();
    int mypair[PR];
#pragma unroll
    for (int r = 0; r < PR; ++r) mypair[r] = (64 * r + lane < Np) ? spairs[64 * r + lane] : -1;

    for (int sl = w.first; sl < w.first + w.count; ++sl) {
      const int64_t coef = pr.coef_off + (int64_t)sl * nDm;
      const int64_t sidx = pr.sample_base + sl;
      for (int q = tid; q < nDm; q += nthr) {
        const float x = xi_bar[coef + q];
        sxb[q] = x;
        sxi[q] = xi0 ? xi0[coef + q] : x;
        slam[q] = lam0 ? lam0[coef + q] : 0.0f;
      }
      for (int q = tid; q < nD6; q += nthr) {
        const int row = q / kNFix, r = q - row * kNFix;
        float acc = 0.0f;
        for (int s = 0; s < kNFix; ++s) acc = fmaf(Bmap[r * kNFix + s], bv[row * kNFix + s], acc);
        sxp[q] = acc;
      }
      __syncthreads();
      for (int q = tid; q < nD6; q += nthr) {
        const int row = q / kNFix, r = q - row * kNFix;
        const int k = r < 3 ? r : m - kNFix + r;
        sdlt[q] = sxi[row * m + k] - sxp[q];
      }
      __syncthreads();
      for (int q = tid; q < 3 * kNFix; q += nthr) {
        const int d = q / kNFix, r = q - d * kNFix;
        float s = 0.0f;
        for (int i = 0; i < n; ++i) s += sdlt[(i * 3 + d) * kNFix + r];
        sdbar[q] = s * inv_n;
      }
      __syncthreads();
      for (int q = tid; q < nDf; q += nthr) {
        const int row = q / mf, f = q - row * mf, d = row % 3;
        float acc = 0.0f;
        for (int r = 0; r < kNFix; ++r) {
          const float dl = sdlt[row * kNFix + r];
          acc = fmaf(n_rho_c * Gfx[f * kNFix + r], dl - sdbar[d * kNFix + r], acc);
          acc = fmaf(Rfx[f * kNFix + r], dl, acc);
        }
        scorr[q] = acc;
      }
      __syncthreads();

      for (int k = 0; k < iters; ++k) {
        if (ckpt && (k % ckpt_every) == 0) {
          const int64_t base = (int64_t)(k / ckpt_every) * 2 * ckpt_stride + coef;
          for (int q = tid; q < nDm; q += nthr) {
            ckpt[base + q] = sxi[q];
            ckpt[base + ckpt_stride + q] = slam[q];
          }
        }
        if (resid_out && k == iters - 1)
          for (int q = tid; q < nDm; q += nthr) sxprev[q] = sxi[q];
        // S1 B operand: xi^T, lane (col, grp) holds robot col, coefficient 4 s + grp
        float bx[R][3][KS];
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
#pragma unroll
          for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int s = 0; s < KS; ++s) {
              const int robot = 16 * rr + col, kk = 4 * s + grp;
              bx[rr][d][s] = (robot < n && kk < m) ? sxi[(robot * 3 + d) * m + kk] : 0.0f;
            }
        f4 gacc[R][3];
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
#pragma unroll
          for (int d = 0; d < 3; ++d) gacc[rr][d] = f4{0.0f, 0.0f, 0.0f, 0.0f};

#pragma unroll
        for (int q = 0; q < TQ; ++q) {
          const int tau = wave + W * q;
          if (tau >= NT) break;
          const int t0 = 16 * tau;
          const int nt = min(16, H - t0);
          // ---- S1 positions -> LDS, per-robot boxes over the tile in registers ----
          {
            f4 Y[R][3];
#pragma unroll
            for (int rr = 0; rr < R; ++rr)
#pragma unroll
              for (int d = 0; d < 3; ++d) {
                f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int s = 0; s < KS; ++s) acc = mfma4(a1[q][0][s], bx[rr][d][s], acc);
                Y[rr][d] = acc;
              }
#pragma unroll
            for (int rr = 0; rr < R; ++rr)
#pragma unroll
              for (int d = 0; d < 3; ++d) {
                const int o = (d * NR + 16 * rr + col) * kRS + 4 * grp;
                *reinterpret_cast<f4*>(Xt + o) = Y[rr][d];
                *reinterpret_cast<f4*>(Ct + o) = f4{0.0f, 0.0f, 0.0f, 0.0f};
              }
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
              float lo[3], hi[3];
#pragma unroll
              for (int d = 0; d < 3; ++d) {
                lo[d] = FLT_MAX;
                hi[d] = -FLT_MAX;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                  if (4 * grp + r < nt) {
                    lo[d] = fminf(lo[d], Y[rr][d][r]);
                    hi[d] = fmaxf(hi[d], Y[rr][d][r]);
                  }
                lo[d] = fminf(lo[d], __shfl_xor(lo[d], 16));
                hi[d] = fmaxf(hi[d], __shfl_xor(hi[d], 16));
                lo[d] = fminf(lo[d], __shfl_xor(lo[d], 32));
                hi[d] = fmaxf(hi[d], __shfl_xor(hi[d], 32));
              }
              if (grp == 0) {
                float* bq = bb + (16 * rr + col) * 8;
                *reinterpret_cast<f4*>(bq) = f4{lo[0], lo[1], lo[2], 0.0f};
                *reinterpret_cast<f4*>(bq + 4) = f4{hi[0], hi[1], hi[2], 0.0f};
              }
            }
          }
          // ---- S1 velocity / acceleration, S3 bound balls in registers, S4 for nonzero tiles ----
#pragma unroll
          for (int b = 1; b < 3; ++b) {
            const bool on = b == 1 ? c.vel_on : c.acc_on;
            if (!on) continue;
            const float lim = b == 1 ? vmax : amax;
            f4 Y[R][3];
#pragma unroll
            for (int rr = 0; rr < R; ++rr)
#pragma unroll
              for (int d = 0; d < 3; ++d) {
                f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int s = 0; s < KS; ++s) acc = mfma4(a1[q][b][s], bx[rr][d][s], acc);
                Y[rr][d] = acc;
              }
            bool nz = false;
#pragma unroll
            for (int rr = 0; rr < R; ++rr)
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const float vx = Y[rr][0][r], vy = Y[rr][1][r], vz = Y[rr][2][r];
                const float ss = vx * vx + vy * vy + vz * vz;
                const float f = ss > lim * lim ? 1.0f - lim * rsqrtf(ss) : 0.0f;
                Y[rr][0][r] = f * vx;
                Y[rr][1][r] = f * vy;
                Y[rr][2][r] = f * vz;
                nz |= f != 0.0f;
              }
            if (ballot(nz) != 0) {
              float b4[4];
#pragma unroll
              for (int s = 0; s < 4; ++s) {
                const int t = t0 + 4 * grp + s;
                b4[s] = (t < H && col < m) ? rho[b] * basis[((size_t)b * H + t) * m + col] : 0.0f;
              }
#pragma unroll
              for (int rr = 0; rr < R; ++rr)
#pragma unroll
                for (int d = 0; d < 3; ++d)
#pragma unroll
                  for (int s = 0; s < 4; ++s) gacc[rr][d] = mfma4(Y[rr][d][s], b4[s], gacc[rr][d]);
            }
          }
          wave_sync();
          // ---- S2: broad phase over the tile, narrow phase on the surviving pairs ----
          int count = 0;
#pragma unroll
          for (int r = 0; r < PR; ++r) {
            const int pij = mypair[r];
            bool act = false;
            if (pij >= 0) {
              const int i = pij & 255, j = pij >> 8;
              float g2 = 0.0f;
#pragma unroll
              for (int d = 0; d < 3; ++d) {
                const float gap = fmaxf(0.0f, fmaxf(bb[j * 8 + d] - bb[i * 8 + 4 + d], bb[i * 8 + d] - bb[j * 8 + 4 + d]));
                g2 += gap * gap * (d == 2 ? ib2 : ia2);
              }
              act = g2 < 1.0001f;
            }
            const uint64_t mask = ballot(act);
            if (act) plist[count + lanes_below(mask)] = pij;
            count += __popcll(mask);
          }
          wave_sync();
          bool nzc = false;
          for (int base = 0; base < count; base += 4) {
            const int slot = base + grp;
            if (slot < count && col < nt) {
              const int pij = plist[slot];
              const int i = pij & 255, j = pij >> 8;
              const float rx = Xt[(0 * NR + i) * kRS + col] - Xt[(0 * NR + j) * kRS + col];
              const float ry = Xt[(1 * NR + i) * kRS + col] - Xt[(1 * NR + j) * kRS + col];
              const float rz = Xt[(2 * NR + i) * kRS + col] - Xt[(2 * NR + j) * kRS + col];
              float Rx, Ry, Rz;
              coll_resid3(rx, ry, rz, ia2, ib2, sb, Rx, Ry, Rz);
              if (Rx != 0.0f || Ry != 0.0f || Rz != 0.0f) {
                nzc = true;
                atomicAdd(Ct + (0 * NR + i) * kRS + col, Rx);
                atomicAdd(Ct + (1 * NR + i) * kRS + col, Ry);
                atomicAdd(Ct + (2 * NR + i) * kRS + col, Rz);
                atomicAdd(Ct + (0 * NR + j) * kRS + col, -Rx);
                atomicAdd(Ct + (1 * NR + j) * kRS + col, -Ry);
                atomicAdd(Ct + (2 * NR + j) * kRS + col, -Rz);
              }
            }
          }
          if (ballot(nzc) != 0) {
            wave_sync();
            float b4[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
              const int t = t0 + 4 * grp + s;
              b4[s] = (t < H && col < m) ? rho[0] * basis[(size_t)t * m + col] : 0.0f;
            }
#pragma unroll
            for (int rr = 0; rr < R; ++rr)
#pragma unroll
              for (int d = 0; d < 3; ++d) {
                const f4 cr = *reinterpret_cast<const f4*>(Ct + (d * NR + 16 * rr + col) * kRS + 4 * grp);
#pragma unroll
                for (int s = 0; s < 4; ++s) gacc[rr][d] = mfma4(cr[s], b4[s], gacc[rr][d]);
              }
          }
          wave_sync();
        }
        // partial back-projection of this wave -> LDS (aliases the tile buffers)
        __syncthreads();
        {
          float* gp = gpart + wave * nDm;
#pragma unroll
          for (int rr = 0; rr < R; ++rr)
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int robot = 16 * rr + 4 * grp + r;
                if (robot < n && col < m) gp[(robot * 3 + d) * m + col] = gacc[rr][d][r];
              }
        }
        __syncthreads();
        // multiplier step and QP step on the free coefficients
        for (int q = tid; q < nDm; q += nthr) {
          float gq = 0.0f;
#pragma unroll
          for (int ww = 0; ww < W; ++ww) gq += gpart[ww * nDm + q];
          const float ln = slam[q] - gq;
          slam[q] = ln;
          const int row = q / m, kk = q - row * m, f = kk - 3;
          if (f >= 0 && f < mf) {
            float y = sxb[q] - sxi[q] + ln - gq;
            if (k == 0) y += scorr[row * mf + f];
            sybuf[row * mf + f] = y;
          }
        }
        __syncthreads();
        for (int q = tid; q < 3 * mf; q += nthr) {
          const int d = q / mf, f = q - d * mf;
          float s = 0.0f;
          for (int i = 0; i < n; ++i) s += sybuf[(i * 3 + d) * mf + f];
          sybar[q] = s * inv_n;
        }
        __syncthreads();
        for (int q = tid; q < nDf; q += nthr) {
          const int row = q / mf, f = q - row * mf, d = row % 3;
          float acc = 0.0f;
          for (int f2 = 0; f2 < mf; ++f2) {
            acc = fmaf(X1[f * mf + f2], sybuf[row * mf + f2], acc);
            acc = fmaf(X01[f * mf + f2], sybar[d * mf + f2], acc);
          }
          sxi[row * m + 3 + f] += acc;
        }
        if (k == 0) {
          for (int q = tid; q < nD6; q += nthr) {
            const int row = q / kNFix, r = q - row * kNFix;
            const int kk = r < 3 ? r : m - kNFix + r;
            sxi[row * m + kk] = sxp[q];
          }
        }
        __syncthreads();
      }

      // ---- primal residual of the last step (dense over pairs) ----
      if (resid_out) {
        float ss = 0.0f, mx = 0.0f;
        if (iters > 0) {
          float bp[R][3][KS], bn[R][3][KS];
#pragma unroll
          for (int rr = 0; rr < R; ++rr)
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
              for (int s = 0; s < KS; ++s) {
                const int robot = 16 * rr + col, kk = 4 * s + grp;
                const bool ok = robot < n && kk < m;
                bp[rr][d][s] = ok ? sxprev[(robot * 3 + d) * m + kk] : 0.0f;
                bn[rr][d][s] = ok ? sxi[(robot * 3 + d) * m + kk] : 0.0f;
              }
#pragma unroll
          for (int q = 0; q < TQ; ++q) {
            const int tau = wave + W * q;
            if (tau >= NT) break;
            const int t0 = 16 * tau;
            const int nt = min(16, H - t0);
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              f4 Yp[R][3], Yn[R][3];
#pragma unroll
              for (int rr = 0; rr < R; ++rr)
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                  f4 ap = {0.0f, 0.0f, 0.0f, 0.0f}, an = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                  for (int s = 0; s < KS; ++s) {
                    ap = mfma4(a1[q][b][s], bp[rr][d][s], ap);
                    an = mfma4(a1[q][b][s], bn[rr][d][s], an);
                  }
                  Yp[rr][d] = ap;
                  Yn[rr][d] = an;
                }
              if (b == 0) {
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
#pragma unroll
                  for (int d = 0; d < 3; ++d) {
                    const int o = (d * NR + 16 * rr + col) * kRS + 4 * grp;
                    *reinterpret_cast<f4*>(Xt + o) = Yp[rr][d];
                    *reinterpret_cast<f4*>(Ct + o) = Yn[rr][d];
                  }
                continue;
              }
              // bound balls: r_p = v_new - e(v_prev), e = v_prev - R(v_prev)
              const bool on = b == 1 ? c.vel_on : c.acc_on;
              if (!on) continue;
              const float lim = b == 1 ? vmax : amax;
#pragma unroll
              for (int rr = 0; rr < R; ++rr)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                  const float vx = Yp[rr][0][r], vy = Yp[rr][1][r], vz = Yp[rr][2][r];
                  const float s2 = vx * vx + vy * vy + vz * vz;
                  const float f = s2 > lim * lim ? 1.0f - lim * rsqrtf(s2) : 0.0f;
                  const float px = Yn[rr][0][r] - (vx - f * vx);
                  const float py = Yn[rr][1][r] - (vy - f * vy);
                  const float pz = Yn[rr][2][r] - (vz - f * vz);
                  const float nrm = px * px + py * py + pz * pz;
                  ss += nrm;
                  mx = fmaxf(mx, nrm);
                }
            }
            wave_sync();
            for (int base = 0; base < Np; base += 4) {
              const int slot = base + grp;
              if (slot < Np && col < nt) {
                const int pij = spairs[slot];
                const int i = pij & 255, j = pij >> 8;
                float rp[3], rn[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                  rp[d] = Xt[(d * NR + i) * kRS + col] - Xt[(d * NR + j) * kRS + col];
                  rn[d] = Ct[(d * NR + i) * kRS + col] - Ct[(d * NR + j) * kRS + col];
                }
                float Rx, Ry, Rz;
                coll_resid3(rp[0], rp[1], rp[2], ia2, ib2, sb, Rx, Ry, Rz);
                const float px = rn[0] - (rp[0] - Rx), py = rn[1] - (rp[1] - Ry), pz = rn[2] - (rp[2] - Rz);
                const float nrm = px * px + py * py + pz * pz;
                ss += nrm;
                mx = fmaxf(mx, nrm);
              }
            }
            wave_sync();
          }
        }
        sred[tid] = ss;
        sred[nthr + tid] = mx;
        __syncthreads();
        if (tid == 0) {
          float s = 0.0f, mm = 0.0f;
          for (int q = 0; q < nthr; ++q) {
            s += sred[q];
            mm = fmaxf(mm, sred[nthr + q]);
          }
          resid_out[sidx * 2 + 0] = s;
          resid_out[sidx * 2 + 1] = sqrtf(mm);
        }
        __syncthreads();
      }
      for (int q = tid; q < nDm; q += nthr) {
        xi_out[coef + q] = sxi[q];
        if (lam_out) lam_out[coef + q] = slam[q];
      }
      __syncthreads();
    }
  }
}

// Kernel instances: R robot tiles of 16, KS k-steps of 4 coefficients, W waves, TQ tiles per wave.
constexpr int kW = 4;

template <int R, int KS, int TQ>
hipError_t launch_instance(const FastPlan& p, const LaunchArgs& a, const float* tab32) {
  auto kern = fast_project_kernel<R, KS, kW, TQ>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(a.n_items), dim3(64 * kW), p.lds_bytes, a.stream, a.cfgs, tab32, a.probs,
                     a.items, a.n_items, static_cast<const float*>(a.xi_bar), static_cast<const float*>(a.bvals),
                     static_cast<const float*>(a.xi0), static_cast<const float*>(a.lam0), a.iters,
                     static_cast<float*>(a.xi_out), static_cast<float*>(a.lam_out),
                     static_cast<float*>(a.resid_out), static_cast<float*>(a.ckpt), a.ckpt_every, a.ckpt_stride);
  return hipGetLastError();
}

}  // namespace

sf_status fast_plan_build(const std::vector<DevCfg>& cfgs, const std::vector<DevProblem>& probs, FastPlan& out) {
  out = FastPlan();
  if (probs.empty()) return SF_OK;
  const int slot = probs[0].cfg;
  for (const DevProblem& p : probs)
    if (p.cfg != slot) return SF_OK;          // mixed shapes: generic path
  const DevCfg& c = cfgs[slot];
  if (c.D != 3 || c.n > 32 || c.m > 16 || c.H > 16 * kW * 2 || c.n > 255) return SF_OK;
  out.R = c.n <= 16 ? 1 : 2;
  out.KS = (c.m + 3) / 4;
  const int NT = (c.H + 15) / 16;
  out.TQ = (NT + kW - 1) / kW;
  if (out.KS < 2) out.KS = 2;
  out.lds_bytes = (size_t)fast_lds_plan(c, out.R, kW).total * 4;
  if (out.lds_bytes > 160 * 1024) return SF_OK;
  out.ok = true;
  return SF_OK;
}

void fast_plan_free(FastPlan& p) { p.ok = false; }

hipError_t fast_launch(const FastPlan& p, const LaunchArgs& a, const float* tab32, int precision) {
  if (precision != SF_FP32) {
    g_fast_err = "precision not implemented in the MFMA kernels";
    return hipErrorNotSupported;
  }
  const int key = p.R * 100 + p.KS * 10 + p.TQ;
  switch (key) {
    case 121: return launch_instance<1, 2, 1>(p, a, tab32);
    case 122: return launch_instance<1, 2, 2>(p, a, tab32);
    case 131: return launch_instance<1, 3, 1>(p, a, tab32);
    case 132: return launch_instance<1, 3, 2>(p, a, tab32);
    case 141: return launch_instance<1, 4, 1>(p, a, tab32);
    case 142: return launch_instance<1, 4, 2>(p, a, tab32);
    case 231: return launch_instance<2, 3, 1>(p, a, tab32);
    case 232: return launch_instance<2, 3, 2>(p, a, tab32);
    case 241: return launch_instance<2, 4, 1>(p, a, tab32);
    case 242: return launch_instance<2, 4, 2>(p, a, tab32);
    default:
      g_fast_err = "no kernel instance for this shape";
      return hipErrorNotSupported;
  }
}

}  // namespace sf
