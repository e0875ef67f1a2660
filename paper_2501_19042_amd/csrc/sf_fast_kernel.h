// MFMA fast path of the safety filter for 3D swarms (n <= 32 robots, degree <= 15, H <= 256).
//
// One workgroup (W = 2, 3 or 4 waves) owns one sample for the whole solve; xi, lambda and xi_bar
// stay in LDS.  The horizon is cut into 16-step time tiles and wave w owns tiles w, w + W, ...
// Per iteration (two workgroup barriers):
//   tiles (each wave, no barrier)
//     S1  Y_b = P_b xi for the bases (position, velocity, acceleration; eq. poly) as MFMA
//         products (fp32, or bf16/fp16 with hi/lo correction terms): rows = 16 times, columns =
//         16 robots of one axis; lane (col, grp) ends up holding robot col at times 4 grp + r.
//     S3  velocity/acceleration ball residuals in those registers (radial form of the d-step
//         with d in [0, 1]), skipped while a drift bound proves every ball inactive.
//     S2  collision residuals (alpha/beta/d steps in radial form): positions go to LDS; per
//         tile, a list of the pairs whose position boxes come within the safety distance plus a
//         margin, rebuilt only when some robot may have moved by more than the margin; the
//         listed pair-times are projected and scattered into an LDS accumulator.
//     S4  g += P_b^T (rho_b R_b) as MFMA products, only for tiles with a nonzero residual; the
//         S1 output layout is exactly the A-operand layout this product needs.
//   barrier; tail (the 3 x 16R robot-axis rows, two lanes per row where they fit)
//     multiplier step and the structured QP step of eq. (xi_step) on the free coefficients.
//   barrier
//
// This header holds the kernels and their launchers; sf_fast_p<MP>_w<WS>.hip instantiate them per
// operand precision and workspace flag (so the instances compile in parallel), sf_fast.hip holds
// the host side (operand tables, plans, dispatch).
#pragma once

#include "sf_fast.h"

#include <cfloat>
#include <algorithm>
#include <cstring>

namespace sf {

void fast_set_error(const char* msg);

namespace fastk {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// 16-bit operand types of v_mfma_f32_16x16x32_{bf16,f16}: MP = 1 bf16, MP = 2 fp16.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
template <int MP> struct Half;
template <> struct Half<1> { typedef __bf16 E; typedef bf16x8 V; };
template <> struct Half<2> { typedef _Float16 E; typedef f16x8 V; };

__device__ __forceinline__ f4 mfma16(bf16x8 a, bf16x8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16(f16x8 a, f16x8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// B operands of the 16-bit S1 product for one robot tile and axis.  Lane (col, grp) covers
// coefficients 8 (grp & 1) .. + 7 of robot col.  First instruction: grp 0, 1 carry xi_hi against
// P_hi and grp 2, 3 carry xi_hi against P_lo; second instruction: grp 0, 1 carry xi_lo against
// P_hi, grp 2, 3 are zero.  The sum is P_hi xi_hi + P_lo xi_hi + P_hi xi_lo in fp32: the
// rounding residuals of both factors are fed back as correction terms.
template <int MP>
__device__ __forceinline__ void split_xi(const float* x, int robot, int n, int m, int d, int grp,
                                         typename Half<MP>::V& b1, typename Half<MP>::V& b2) {
  typedef typename Half<MP>::E E;
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const int k = 8 * (grp & 1) + v;
    const float xv = (robot < n && k < m) ? x[(robot * 3 + d) * m + k] : 0.0f;
    const E hi = static_cast<E>(xv);
    const E lo = static_cast<E>(xv - static_cast<float>(hi));
    b1[v] = hi;
    b2[v] = grp < 2 ? lo : static_cast<E>(0.0f);
  }
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
// accumulator Ct as [axis][robot (16R)][time] with 16-word rows whose four 16-byte chunks are
// XOR-swizzled by the robot index (tile_at), so that the 16-byte accesses of 16 consecutive lanes
// hit distinct banks; boxes bb [robot][box_row(R)]; per tile, the list of pairs that can collide.  Once
// its time tiles are done, a wave reuses its own region for its partial back-projection (nDm
// words) and, after the final residual pass, for its partial sums.
constexpr int kQPCols = 16;              // QP matrix row in LDS: both halves, each padded (m_f <= 10)
// Row strides (words) chosen so that the 16-byte accesses of 16 consecutive robots hit 16
// distinct groups of 4 banks (64 banks): boxes (lo xyz _, hi xyz _, pad) and 16-bit operands.  The
// forward kernel with two robot tiles keeps its boxes unpadded (two-way conflicts in the broad
// phase, which runs in rebuild iterations only) in the pair-list region, where the list of the tile
// being rebuilt and those after it are rewritten anyway, its pair lists in 16-bit entries, its pair
// table in each wave's pair-list region while that is free (set-up, final residual) and its 16-bit
// operand rows unpadded, with the 16-byte chunks permuted per row instead: an LDS plan that fits
// two workgroups of three or four waves per CU up to degree 12.
constexpr int kBoxRow = 12;
constexpr int kHBRow = 20;
__host__ __device__ constexpr int box_row(int R) { return R == 2 ? 8 : kBoxRow; }
__host__ __device__ constexpr int hb_row(int R) { return R == 2 ? 16 : kHBRow; }
// Index (16-bit units) of entry e of the 16-bit operand row `row` (axis * 16R + robot): e = kk for
// the hi part of coefficient kk, 16 + kk for its lo part.  Unpadded rows (two robot tiles) permute
// their four 16-byte chunks by bits 2-3 of the row, so the 16 rows of one lane group still fall in
// 16 distinct groups of 4 banks.
template <int R>
__device__ __forceinline__ int hb_at(int row, int e) {
  if constexpr (R == 2) return row * 32 + (e ^ (((row >> 2) & 3) << 3));
  else return row * (2 * kHBRow) + e;
}
struct FastLds {
  int xi, lam, xb, xprev, dbar, corr, pairs, vmx, amx, wmx, dxi, cmx, qp, hb, tiles, per_wave, total;
  int xt, ct, bb, plist;   // offsets inside one wave's tile region
};
// Pair table and pair lists of a wave's tiles (count, then pair codes i | j << 8) per tile: 32-bit
// entries with one robot tile, 16-bit with two.
__host__ __device__ constexpr int plist_entries(int nr) { return nr * (nr - 1) / 2 + 1; }
template <int R> struct PairList { typedef int T; };
// Word offset, from the start of a wave's pair lists, of the boxes of its tile q with two robot tiles:
// the first 16-byte boundary after the 16-bit lists of tiles 0 .. q - 1.
__host__ __device__ constexpr int box_at(int q, int nr) { return (((q * plist_entries(nr) + 1) >> 1) + 3) & ~3; }
template <> struct PairList<2> { typedef uint16_t T; };

__host__ __device__ inline FastLds fast_lds_plan(const DevCfg& c, int R, int W, int MP) {
  const int nDm = c.n * 3 * c.m, nDf = c.n * 3 * c.mf;
  const int nr = 16 * R, Npmax = nr * (nr - 1) / 2;
  FastLds p;
  int o = 0;
  // (two robot tiles: the previous iterate of the final residual lives in xi_out and the first-step
  // correction is folded into xi_bar for step 0, so neither takes LDS)
  p.xi = o; o += nDm;
  p.lam = o; o += nDm;
  p.xb = o; o += nDm;
  p.xprev = o; o += R == 1 ? nDm : 0;
  p.dbar = o; o += 3 * kNFix;
  p.corr = o; o += R == 1 ? nDf : 0;
  p.pairs = o; o += R == 2 ? 0 : Npmax;  // (two robot tiles: in the pair-list regions)
  p.vmx = o; o += W * nr;                  // per wave and robot: max ||v||^2 over the wave's tiles
  p.amx = o; o += W * nr;                  // same for the acceleration
  p.dxi = o; o += 3 * nr;                  // per (robot, axis): max |change| of a free coefficient
  p.cmx = o; o += 3 * nr;                  // per (robot, axis): max |coefficient| of the iterate
  o = (o + 3) & ~3;
  // X1, X01 transposed: rows of at most kQPCols floats, or of 4 QC <= 12 floats in the layout of
  // one robot tile with three waves (QC = 16-byte chunks of the free coefficients)
  p.qp = o; o += 2 * c.mf * (R == 1 && W == 3 ? 12 : kQPCols);
  o = (o + 3) & ~3;
  p.hb = o; o += MP ? 3 * nr * hb_row(R) : 0; // 16-bit S1 B operands: [axis][robot][hi x16, lo x16 (, pad)]
  o = (o + 3) & ~3;                        // 16-byte alignment of the tile buffers
  p.xt = 0;
  p.ct = 3 * nr * 16;
  // (two robot tiles: the boxes of tile q sit at the first 16-byte boundary after the pair lists of
  // tiles 0 .. q - 1, see box_at; those of the last tile run past the lists by at most 12 words)
  p.bb = R == 2 ? 0 : 6 * nr * 16;
  p.plist = R == 2 ? 6 * nr * 16 : p.bb + box_row(R) * nr;   // per tile of the wave: [count, pairs...] kept across iterations
  const int NT = (c.H + 15) / 16, TQ = (NT + W - 1) / W;
  int pw = p.plist + (R == 2 ? (TQ * plist_entries(nr) + 1) / 2 + 12 : TQ * plist_entries(nr));
  if (pw < nDm) pw = nDm;
  if (pw < 128) pw = 128;
  p.per_wave = (pw + 3) & ~3;
  p.tiles = o;
  o += W * p.per_wave;
  p.wmx = o; o += c.ws_on ? W * nr : 0;    // per wave and robot: max ||M_w^{-1} (p - p_w)||^2 (workspace)
  p.total = o;
  return p;
}

// Word offset of (row, t) in a tile buffer; row = axis * 16R + robot, t = 0..15.
__device__ __forceinline__ int tile_at(int row, int t) {
  return row * 16 + ((((t >> 2) ^ (row >> 2)) & 3) << 2) + (t & 3);
}

// Minimum / maximum over the four lanes col, col + 16, col + 32, col + 48 (every lane gets the
// result), with the row-swap instructions of gfx950 instead of LDS permutes.
__device__ __forceinline__ float grp_min(float x) {
  const auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  x = fminf(__uint_as_float(a[0]), __uint_as_float(a[1]));
  const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return fminf(__uint_as_float(b[0]), __uint_as_float(b[1]));
}
__device__ __forceinline__ float grp_max(float x) {
  const auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  x = fmaxf(__uint_as_float(a[0]), __uint_as_float(a[1]));
  const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return fmaxf(__uint_as_float(b[0]), __uint_as_float(b[1]));
}

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum over aligned groups of NR (16 or 32) lanes; every lane of a group gets the same value
// (each step adds a lane's value and its partner's, and addition is commutative).
template <int NR>
__device__ __forceinline__ float group_sum(float v) {
  v = v + dpp<0xB1>(v);     // quad_perm [1, 0, 3, 2]
  v = v + dpp<0x4E>(v);     // quad_perm [2, 3, 0, 1]
  v = v + dpp<0x141>(v);    // row_half_mirror
  v = v + dpp<0x140>(v);    // row_mirror
  if constexpr (NR == 32) {
    const auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = __uint_as_float(a[0]) + __uint_as_float(a[1]);
  }
  return v;
}

// Sum over the 64 lanes of a wave (all lanes active; every lane gets the same value).
__device__ __forceinline__ float wave_sum(float v) {
  v = group_sum<32>(v);
  const auto a = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(a[0]) + __uint_as_float(a[1]);
}

// Maximum over the 64 lanes of a wave (all lanes active; every lane gets the result).
__device__ __forceinline__ float wave_max(float v) {
  v = fmaxf(v, dpp<0xB1>(v));
  v = fmaxf(v, dpp<0x4E>(v));
  v = fmaxf(v, dpp<0x141>(v));
  v = fmaxf(v, dpp<0x140>(v));
  return grp_max(v);
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

struct FastArgs {
  const DevCfg* cfgs;
  const float* tab;
  const uint4* a16;
  const DevProblem* probs;
  const WorkItem* items;
  int n_items;
  const float* xi_bar;
  const float* bvals;
  const float* xi0;
  const float* lam0;
  int iters;
  float* xi_out;
  float* lam_out;
  float* resid_out;
  int32_t* status_out;
  float* ckpt;
  int ckpt_every;
  int64_t ckpt_stride;
  int fpr;               // accumulate the fixed-point residual sum (resid_out is [S][3])
};

// The whole solve of one work item (its samples) by one workgroup.  WS: the instance carries the
// workspace rows (evaluated for the configs that have them).
template <int R, int KS, int W, int MP, int WS>
__device__ __forceinline__ void fast_item(const FastArgs& A, int it, float* smem) {
  const DevCfg* __restrict__ cfgs = A.cfgs;
  const float* __restrict__ tab = A.tab;
  const uint4* __restrict__ a16 = A.a16;
  const DevProblem* __restrict__ probs = A.probs;
  const WorkItem* __restrict__ items = A.items;
  const float* __restrict__ xi_bar = A.xi_bar;
  const float* __restrict__ bvals = A.bvals;
  const float* __restrict__ xi0 = A.xi0;
  const float* __restrict__ lam0 = A.lam0;
  const int iters = A.iters;
  float* __restrict__ xi_out = A.xi_out;
  float* __restrict__ lam_out = A.lam_out;
  float* __restrict__ resid_out = A.resid_out;
  int32_t* __restrict__ status_out = A.status_out;
  float* __restrict__ ckpt = A.ckpt;
  const int ckpt_every = A.ckpt_every;
  const int64_t ckpt_stride = A.ckpt_stride;
  const bool fpr = A.fpr != 0;
  const int rw = fpr ? 3 : 2;            // resid_out columns
  constexpr int NR = 16 * R;
  constexpr int PR = (NR * (NR - 1) / 2 + 63) / 64;   // 64-pair rounds of the broad phase
  constexpr int MFX = 4 * KS - 6;                     // free coefficients per robot-axis, at most
  constexpr int HALVES = 6 * NR <= 64 * W ? 2 : 1;    // lanes per row in the multiplier/QP step
  constexpr int FH = (MFX + HALVES - 1) / HALVES;     // free coefficients per lane
  constexpr int FHP = (FH + 3) & ~3;                  // ... padded to whole 16-byte chunks
  static_assert(HALVES * FHP <= kQPCols, "QP matrix rows");
  constexpr int TAILW = (3 * NR * HALVES + 63) / 64;  // waves running the multiplier and QP steps
  // One robot tile and three waves: wave a runs axis a of the multiplier/QP step with four lanes per
  // row (robot, a), so every wave shares it.
  constexpr bool QUART = R == 1 && W == 3;
  constexpr int FQ = (MFX + 3) / 4;                   // free coefficients per lane in that layout
  constexpr int QC = (MFX + 3) / 4;                   // 16-byte chunks of a QP matrix row
  static_assert(!QUART || 4 * QC <= 12, "QP matrix rows of the quarter layout");
  // two robot tiles: no LDS copy of the previous iterate or of the first-step correction (see the plan)
  constexpr bool LEAN = R == 2;
  static_assert(TAILW <= W, "the multiplier/QP step needs 3 x 16R lanes");
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nthr = 64 * W;
  {
    // per-lane indices from an opaque copy, so that the compiler keeps per-lane addresses next to
    // their uses instead of hoisting them to the kernel entry and spilling them
    int tid_i = threadIdx.x;
    asm volatile("" : "+v"(tid_i));
    const int tid = tid_i, lane = tid_i & 63;
    const int col = lane & 15, grp = lane >> 4;
    const WorkItem w = items[it];
    const DevProblem pr = probs[w.problem];
    const DevCfg c = cfgs[pr.cfg];
    const FastLds L = fast_lds_plan(c, R, W, MP);
    const int n = c.n, m = c.m, mf = c.mf, H = c.H;
    const int nDm = n * 3 * m, nDf = n * 3 * mf;
    const int Np = n * (n - 1) / 2;
    const int NT = (H + 15) / 16;
    const int TQ = (NT + W - 1) / W;            // time tiles per wave
    const float* X1 = tab + c.off_X1;
    const float* X01 = tab + c.off_X01;
    const float* Bmap = tab + c.off_Bmap;
    const float* Gfx = tab + c.off_Gfx;
    const float* Rfx = tab + c.off_Rfx;
    const float ia2 = (float)c.inv_a2, ib2 = (float)c.inv_b2, sb = (float)c.b;
    // workspace spheroid (eq. workspace_polar): centre, 1/a_w^2, 1/b_w^2, rho_w / rho_c
    const float wcx = c.ws_f[0], wcy = c.ws_f[1], wcz = c.ws_f[2];
    const float wia2 = c.ws_f[3], wib2 = c.ws_f[4], wsc = c.ws_f[5];
    const float vmax = (float)c.vmax, amax = (float)c.amax;
    const float n_rho_c = (float)c.n_rho_c, inv_n = 1.0f / (float)n;
    const float Lv = (float)c.lip_v, La = (float)c.lip_a;
    const float* bv = bvals + pr.bnd_off;
    float* sxi = smem + L.xi;
    float* slam = smem + L.lam;
    float* sxb = smem + L.xb;
    float* sxprev = smem + L.xprev;
    float* sdbar = smem + L.dbar;
    float* scorr = smem + L.corr;
    // pair table, lexicographic (i, j), i < j: shared with one robot tile; with two, each wave's copy
    // in its pair-list region, written where needed (set-up, final residual)
    typedef typename PairList<R>::T PT;
    PT* spairs = reinterpret_cast<PT*>(R == 2 ? smem + L.tiles + wave * L.per_wave + L.plist : smem + L.pairs);
    auto fill_pairs = [&](int t0, int stride) {
      for (int i = t0; i < n; i += stride) {
        int p = i * n - i * (i + 1) / 2;
        for (int j = i + 1; j < n; ++j) spairs[p++] = static_cast<PT>(i | (j << 8));
      }
    };
    float* s_vmx = smem + L.vmx;
    float* s_amx = smem + L.amx;
    float* s_dxi = smem + L.dxi;
    float* s_cmx = smem + L.cmx;
    float* s_wmx = smem + L.wmx;
    // 16-bit hi/lo split of xi in the S1 B-operand layout, kept current by whoever writes xi
    typedef typename Half<MP == 0 ? 1 : MP>::E HE;
    HE* shb = reinterpret_cast<HE*>(smem + L.hb);
    auto put_split = [&](int robot, int d, int kk, float x) {
      const HE hi = static_cast<HE>(x);
      const HE lo = static_cast<HE>(x - static_cast<float>(hi));
      shb[hb_at<R>(d * NR + robot, kk)] = hi;
      shb[hb_at<R>(d * NR + robot, 16 + kk)] = lo;
    };
    float* wbuf = smem + L.tiles + wave * L.per_wave;
    float* Xt = wbuf + L.xt;
    float* Ct = wbuf + L.ct;
    float* bb = wbuf + L.bb;
    // pinned coefficient r of a robot-axis row after the first step: Bmap (p0, v0, a0, pH, vH, aH)
    auto pinned = [&](int row, int r) {
      float acc = 0.0f;
      for (int s = 0; s < kNFix; ++s) acc = fmaf(Bmap[r * kNFix + s], bv[row * kNFix + s], acc);
      return acc;
    };
    auto fixed_k = [&](int r) { return r < 3 ? r : m - kNFix + r; };

    if constexpr (R == 2) fill_pairs(tid & 63, 64);
    else fill_pairs(tid, nthr);
    // QP matrices X1 (relative motion) and X01 (mean motion minus relative), transposed and cut
    // into the halves of the outputs the lanes own: [matrix][half][f2][j] = X[half * FH + j][f2]
    // (zero-padded)
    float* sX1 = smem + L.qp;
    if constexpr (QUART) {
      // [matrix][f][f2], rows of 4 QC floats (zero-padded)
      for (int q = tid; q < 2 * mf * 4 * QC; q += nthr) {
        const int c4 = q % (4 * QC), f = (q / (4 * QC)) % mf, mat = q / (4 * QC * mf);
        sX1[q] = c4 < mf ? (mat == 0 ? X1 : X01)[f * mf + c4] : 0.0f;
      }
    } else {
      for (int q = tid; q < 2 * HALVES * mf * FHP; q += nthr) {
        const int j = q % FHP, f2 = (q / FHP) % mf, mh = q / (FHP * mf);
        const int h = mh % HALVES, mat = mh / HALVES, f = h * FH + j;
        sX1[q] = (j < FH && f < mf) ? (mat == 0 ? X1 : X01)[f * mf + f2] : 0.0f;
      }
    }
    // basis operand tables: fp32 [tile][basis][S1 A operand, S4 B operand (x rho)][lane],
    // 16-bit [tile][basis][instruction][lane]
    const float4* a32c = reinterpret_cast<const float4*>(a16) + c.off_a32;
    const uint4* a16c = a16 + (MP == 1 ? c.off_a16[0] : c.off_a16[1]);
    __syncthreads();
    int mypair[PR];
#pragma unroll
    for (int r = 0; r < PR; ++r) mypair[r] = (64 * r + lane < Np) ? spairs[64 * r + lane] : -1;

    for (int sl = w.first; sl < w.first + w.count; ++sl) {
      // per-lane indices re-derived per sample from an opaque copy (see the iteration loop)
      int tid_s = threadIdx.x;
      asm volatile("" : "+v"(tid_s));
      const int tid = tid_s, lane = tid_s & 63;
      const int col = lane & 15, grp = lane >> 4;
      const int64_t coef = pr.coef_off + (int64_t)sl * nDm;
      const int64_t sidx = pr.sample_base + sl;
      for (int q = tid; q < nDm; q += nthr) {
        const float x = xi_bar[coef + q];
        sxb[q] = x;
        sxi[q] = xi0 ? xi0[coef + q] : x;
        slam[q] = lam0 ? lam0[coef + q] : 0.0f;
      }
      for (int q = tid; q < 3 * NR; q += nthr) s_dxi[q] = 0.0f;
      for (int q = lane; q < 3 * NR * 16; q += 64) Ct[q] = 0.0f;
      // a sample the input check flagged (non-finite input) is not iterated; the status pass then
      // writes NaN over its outputs
      const int32_t in_flag = status_out ? __builtin_amdgcn_readfirstlane(status_out[sidx]) : 0;
      const int iters_s = in_flag < 0 ? 0 : iters;
      __syncthreads();
      // per-row bound on |coefficient| over the iterates: the initial one and the pinned values
      for (int q = tid; q < 3 * NR; q += nthr) {
        float cm = 0.0f;
        if (q < 3 * n) {
          for (int kk = 0; kk < m; ++kk) cm = fmaxf(cm, fabsf(sxi[q * m + kk]));
          for (int r = 0; r < kNFix; ++r) cm = fmaxf(cm, fabsf(pinned(q, r)));
        }
        s_cmx[q] = cm;
      }
      if constexpr (MP != 0) {
        // one thread per (axis, robot, coefficient) of the padded operand rows (zeros outside)
        for (int q = tid; q < 3 * NR * 16; q += nthr) {
          const int row = q >> 4, kk = q & 15, d = row / NR, robot = row - d * NR;
          put_split(robot, d, kk, (robot < n && kk < m) ? sxi[(robot * 3 + d) * m + kk] : 0.0f);
        }
      }
      // the first QP step also moves the pinned coefficients (from xi0 to their boundary values);
      // its effect on the free ones is the correction G_rho (xi0 - xi_p) restricted to them
      for (int q = tid; q < 3 * kNFix; q += nthr) {
        const int d = q / kNFix, r = q - d * kNFix;
        float s = 0.0f;
        for (int i = 0; i < n; ++i) s += sxi[(i * 3 + d) * m + fixed_k(r)] - pinned(i * 3 + d, r);
        sdbar[q] = s * inv_n;
      }
      __syncthreads();
      for (int q = tid; q < nDf; q += nthr) {
        const int row = q / mf, f = q - row * mf, d = row % 3;
        float acc = 0.0f;
        for (int r = 0; r < kNFix; ++r) {
          const float dl = sxi[row * m + fixed_k(r)] - pinned(row, r);
          acc = fmaf(n_rho_c * Gfx[f * kNFix + r], dl - sdbar[d * kNFix + r], acc);
          acc = fmaf(Rfx[f * kNFix + r], dl, acc);
        }
        if constexpr (LEAN) sxb[row * m + 3 + f] += acc;   // step 0 reads xi_bar + correction
        else scorr[q] = acc;
      }
      __syncthreads();
      // bound-ball drift tracking, lane = robot, identical in every wave: margin to the bound at
      // the last evaluation and accumulated bound on the drift since then
      float mv = -1.0f, dv = 0.0f, ma = -1.0f, da = 0.0f;
      int prev_eval = 0;
      // the same for the workspace rows, as one slack: 1 - max ||M_w^{-1} (p - p_w)|| at the last
      // evaluation minus the scaled drift bounds of the positions since then
      float wsl = -1.0f;
      int ws_prev = 0;
      // pair lists: accumulated bound on the position change of robot `lane` per axis since the lists
      // were built (a position is a convex combination of its coefficients, so it moves by at most
      // the largest change of a coefficient)
      float px_ = 0.0f, py_ = 0.0f, pz_ = 0.0f;
      // this lane's share of the fixed-point residual sum_k ||xi^{k+1} - xi^k||^2 +
      // ||lambda^{k+1} - lambda^k||^2 (multiplier/QP-step lanes; lambda changes by -g)
      float fpsum = 0.0f;
      const float skx = (float)(c.skin * c.a) * 0.999f, skz = (float)(c.skin * c.b) * 0.999f;

      for (int k = 0; k < iters_s; ++k) {
        // Lane-dependent indices are re-derived from an opaque copy every iteration: otherwise the
        // compiler hoists every per-lane address of the loop body out of the sample loop and
        // spills them.
        int lane_o = tid;
        asm volatile("" : "+v"(lane_o));
        const int tid = lane_o, lane = lane_o & 63;
        const int col = lane & 15, grp = lane >> 4;
        if (ckpt && (k % ckpt_every) == 0) {
          const int64_t base = (int64_t)(k / ckpt_every) * 2 * ckpt_stride + coef;
          for (int q = tid; q < nDm; q += nthr) {
            ckpt[base + q] = sxi[q];
            ckpt[base + ckpt_stride + q] = slam[q];
          }
        }
        if ((resid_out || status_out) && k == iters_s - 1)
          for (int q = tid; q < nDm; q += nthr) {
            if constexpr (LEAN) xi_out[coef + q] = sxi[q];   // overwritten with the result at the end
            else sxprev[q] = sxi[q];
          }
        // Velocity/acceleration at every grid time move by at most L * ||max_k |d xi_{i,d,k}| ||_2
        // per step (L = max_t sum_k |basis row|).  While the accumulated drift of every robot stays
        // below its margin to the bound at the last evaluation, the ball residuals are exactly zero
        // and S1/S3/S4 for that basis are skipped.  Iterations 0 and 1 always evaluate (the pinned
        // coefficients change in the first step).
        int eval_flags = 3;
        float cm;   // bound on |coefficient| of robot `lane` over the iterates so far
        {
          float dn = 0.0f;
          cm = 0.0f;
          if (lane < n) {
            // margins to the bounds measured by the previous iteration if it evaluated them
            // (every wave computes the same values).  The hardware square root (1 ulp) serves: the
            // test below keeps a 1e-4 relative slack, far above its error.
            if (prev_eval & 1) {
              float mx = 0.0f;
#pragma unroll
              for (int ww = 0; ww < W; ++ww) mx = fmaxf(mx, s_vmx[ww * NR + lane]);
              mv = vmax - __builtin_amdgcn_sqrtf(mx);
              dv = 0.0f;
            }
            if (prev_eval & 2) {
              float mx = 0.0f;
#pragma unroll
              for (int ww = 0; ww < W; ++ww) mx = fmaxf(mx, s_amx[ww * NR + lane]);
              ma = amax - __builtin_amdgcn_sqrtf(mx);
              da = 0.0f;
            }
            const float d0 = s_dxi[lane * 3], d1 = s_dxi[lane * 3 + 1], d2 = s_dxi[lane * 3 + 2];
            cm = fmaxf(fmaxf(s_cmx[lane * 3], s_cmx[lane * 3 + 1]), s_cmx[lane * 3 + 2]);
            dn = __builtin_amdgcn_sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
            px_ += d0;
            py_ += d1;
            pz_ += d2;
            if constexpr (WS) {
              if (ws_prev) {
                float mx = 0.0f;
#pragma unroll
                for (int ww = 0; ww < W; ++ww) mx = fmaxf(mx, s_wmx[ww * NR + lane]);
                wsl = 1.0f - __builtin_amdgcn_sqrtf(mx);
              }
              // ||M_w^{-1} (sum of steps)|| <= sum of ||M_w^{-1} step|| (triangle inequality)
              wsl -= __builtin_amdgcn_sqrtf((d0 * d0 + d1 * d1) * wia2 + d2 * d2 * wib2);
            }
          }
          dv += Lv * dn;
          da += La * dn;
          const bool fv = c.vel_on && lane < n && dv >= mv - 1e-4f * vmax;
          const bool fa = c.acc_on && lane < n && da >= ma - 1e-4f * amax;
          if (k >= 2) eval_flags = (ballot(fv) != 0 ? 1 : 0) | (ballot(fa) != 0 ? 2 : 0);
        }
        prev_eval = eval_flags;
        // Workspace rows: a position moves per step by at most the largest coefficient change
        // per axis, so while max ||M_w^{-1} (p - p_w)|| at the last evaluation plus the summed
        // scaled drift stays below 1 (1e-4 slack) every workspace residual is exactly zero and the
        // rows are skipped.
        bool ws_eval = false;
        if constexpr (WS) {
          if (c.ws_on) {
            ws_eval = k < 2 || ballot(lane < n && wsl <= 1e-4f) != 0;
            ws_prev = ws_eval;
          }
        }
        // Rebuild the pair lists when some robot may have moved by more than the margin they were
        // built with (and in iterations 0 and 1, where the pinned coefficients jump).
        const bool rebuild = k < 2 || ballot(lane < n && (px_ > skx || py_ > skx || pz_ > skz)) != 0;
        if (rebuild) px_ = py_ = pz_ = 0.0f;
        // Margins of the broad phase: twice the drift margin per axis, plus the rounding of the
        // positions.  A computed position is a rounded convex combination of its coefficients, off by
        // at most ~1.2e-5 of the largest |coefficient| (16-bit split products; fp32 far less); 2^-12
        // of a bound on that over the sample (running maximum, plus the most the coefficients can
        // grow before the next rebuild) holds for both robots of a pair in the build and every reuse
        // iteration.
        float mgx = 0.0f, mgz = 0.0f;
        if (rebuild) {
          const float tol = 2.44140625e-4f * (wave_max(cm) + fmaxf(skx, skz));
          mgx = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(2.0f * skx + tol)));
          mgz = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(2.0f * skz + tol)));
        }
        // S1 B operand: xi^T, lane (col, grp) holds robot col, coefficient 4 s + grp
        float bx[MP == 0 ? R : 1][3][KS];
        // (two robot tiles at two waves per SIMD: the 16-bit operands are re-read from LDS per
        // product instead of held across the tiles, 48 registers fewer)
        constexpr bool HBR = R == 2 && W >= 3;
        // (two robot tiles: offsets of this lane's hi and lo chunks from the first row of its robot
        // tile and axis, robot col, entries 8 (grp & 1) and 16 + 8 (grp & 1); see hb_at)
        const int hb_hi = hb_at<R>(col, 8 * (grp & 1)), hb_lo = hb_at<R>(col, 16 + 8 * (grp & 1));
        typename Half<MP == 0 ? 1 : MP>::V hb1[MP == 0 || HBR ? 1 : R][3], hb2[MP == 0 || HBR ? 1 : R][3];
        if constexpr (MP == 0) {
#pragma unroll
          for (int rr = 0; rr < R; ++rr)
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
              for (int s = 0; s < KS; ++s) {
                const int robot = 16 * rr + col, kk = 4 * s + grp;
                bx[rr][d][s] = (robot < n && kk < m) ? sxi[(robot * 3 + d) * m + kk] : 0.0f;
              }
        } else if constexpr (!HBR) {
          // lane (col, grp) takes coefficients 8 (grp & 1) .. + 7 of robot col: hi in the first
          // instruction, lo in the second (see split_xi).  The second instruction's A operand is zero
          // for grp 2, 3, so their lo values (finite: the split of finite coefficients, zero past m)
          // add exact zeros and need no masking.
          typedef typename Half<MP == 0 ? 1 : MP>::V V;
#pragma unroll
          for (int rr = 0; rr < R; ++rr)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              uint4 hi, lo;
              if constexpr (R == 1) {
                const uint4* hrow = reinterpret_cast<const uint4*>(shb + (d * NR + 16 * rr + col) * (2 * kHBRow));
                hi = hrow[grp & 1];
                lo = hrow[2 + (grp & 1)];
              } else {
                const HE* hrow = shb + (d * NR + 16 * rr) * (2 * hb_row(R));
                hi = *reinterpret_cast<const uint4*>(hrow + hb_hi);
                lo = *reinterpret_cast<const uint4*>(hrow + hb_lo);
              }
              hb1[rr][d] = __builtin_bit_cast(V, hi);
              hb2[rr][d] = __builtin_bit_cast(V, lo);   // (grp 2, 3 meet a zero A operand, see below)
            }
        }
        // S1 product for one basis of one tile: Y[rr][d] (lane (col, grp): robot col, times 4 grp + r)
        auto s1_32 = [&](const float4 av, f4 (&Y)[R][3]) {
          const float a1[4] = {av.x, av.y, av.z, av.w};
#pragma unroll
          for (int rr = 0; rr < R; ++rr)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
              for (int s = 0; s < KS; ++s) acc = mfma4(a1[s], bx[rr][d][s], acc);
              Y[rr][d] = acc;
            }
        };
        auto s1_16 = [&](const uint4 u1, const uint4 u2, f4 (&Y)[R][3]) {
          if constexpr (MP != 0) {
            typedef typename Half<MP>::V V;
            const V A1 = __builtin_bit_cast(V, u1);
            const V A2 = __builtin_bit_cast(V, u2);
#pragma unroll
            for (int rr = 0; rr < R; ++rr)
#pragma unroll
              for (int d = 0; d < 3; ++d) {
                f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
                if constexpr (HBR) {
                  const HE* hrow = shb + (d * NR + 16 * rr) * (2 * hb_row(R));
                  const uint4 lo = *reinterpret_cast<const uint4*>(hrow + hb_lo);
                  acc = mfma16(A1, __builtin_bit_cast(V, *reinterpret_cast<const uint4*>(hrow + hb_hi)), acc);
                  acc = mfma16(A2, __builtin_bit_cast(V, lo), acc);
                } else {
                  acc = mfma16(A1, hb1[rr][d], acc);
                  acc = mfma16(A2, hb2[rr][d], acc);
                }
                Y[rr][d] = acc;
              }
          }
        };
        f4 gacc[R][3];
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
#pragma unroll
          for (int d = 0; d < 3; ++d) gacc[rr][d] = f4{0.0f, 0.0f, 0.0f, 0.0f};
        float vm[2][R];           // max ||v||^2, ||a||^2 of robot col over this wave's tiles
        float wsm[WS ? R : 1];    // max ||M_w^{-1} (p - p_w)||^2 of robot col over this wave's tiles
#pragma unroll
        for (int rr = 0; rr < R; ++rr) vm[0][rr] = vm[1][rr] = 0.0f;
#pragma unroll
        for (int rr = 0; rr < (WS ? R : 1); ++rr) wsm[rr] = 0.0f;
        // position operands of the wave's first tile; each tile prefetches those of its next one
        float4 pa = {0.0f, 0.0f, 0.0f, 0.0f}, pb = {0.0f, 0.0f, 0.0f, 0.0f};
        uint4 pu1 = {0u, 0u, 0u, 0u}, pu2 = {0u, 0u, 0u, 0u};
        if (wave < NT) {
          if constexpr (MP == 0) pa = a32c[((wave * 3) * 2) * 64 + lane];
          else {
            pu1 = a16c[((wave * 3) * 2) * 64 + lane];
            pu2 = a16c[((wave * 3) * 2 + 1) * 64 + lane];
          }
          pb = a32c[((wave * 3) * 2 + 1) * 64 + lane];
        }

        // Issue priority (one robot tile): from the end of a wave's tiles through the partial write,
        // the barriers, the multiplier/QP step and the flags up to here, a wave runs at priority 2
        // (that work is serial for the sample: all its waves wait on it); in the tile phase the waves
        // with the most tiles (priority 1) carry the sample's longest path to the next barrier and
        // the others (0) have slack.  The SIMD issues from the waves of other
        // samples in that order, which shortens every sample's iteration.  (The two-tile kernels
        // gain about 1% from it and are left without.)
        if constexpr (R == 1) {
          if ((NT - 1 - wave) / W + 1 == TQ) __builtin_amdgcn_s_setprio(1);
          else __builtin_amdgcn_s_setprio(0);
        }
#pragma unroll 1
        for (int q = 0; q < TQ; ++q) {
          const int tau = wave + W * q;
          if (tau >= NT) break;
          const int t0 = 16 * tau;
          const int nt = min(16, H - t0);
          const float4 ca = pa, cb = pb;
          const uint4 cu1 = pu1, cu2 = pu2;
          // narrow-phase lane mapping: lanes cover (pair, time) items, 64 / T pairs per round with
          // T = the tile's valid times rounded up to 4, 8 or 16.  A list kept from an earlier
          // iteration is read now (count and first round together), ahead of the products.
          typename PairList<R>::T* tl = reinterpret_cast<typename PairList<R>::T*>(wbuf + L.plist) + q * plist_entries(NR);
          // (two robot tiles: over the lists of this tile and the next, which a rebuild rewrites)
          float* const bbq = R == 2 ? wbuf + L.plist + box_at(q, NR) : bb;
          const int tsh = nt <= 4 ? 2 : (nt <= 8 ? 3 : 4);
          const int tt = lane & ((1 << tsh) - 1), ps = lane >> tsh, ppr = 64 >> tsh;
          const int kept_count = tl[0], kept_first = tl[1 + ps];
          if (tau + W < NT) {
            const int nx = tau + W;
            if constexpr (MP == 0) pa = a32c[((nx * 3) * 2) * 64 + lane];
            else {
              pu1 = a16c[((nx * 3) * 2) * 64 + lane];
              pu2 = a16c[((nx * 3) * 2 + 1) * 64 + lane];
            }
            pb = a32c[((nx * 3) * 2 + 1) * 64 + lane];
          }
          bool ws_nz = false;   // some workspace residual of the tile is nonzero (wave-uniform)
          // ---- S1 positions -> LDS, per-robot boxes over the tile in registers ----
          // (not needed when the tile's kept pair list is empty and no list or workspace row is
          // evaluated: then no residual of the tile is nonzero)
          if (rebuild || __builtin_amdgcn_readfirstlane(kept_count) > 0 || (WS && ws_eval)) {
            f4 Y[R][3];
            if constexpr (MP == 0) s1_32(ca, Y);
            else s1_16(cu1, cu2, Y);
#pragma unroll
            for (int rr = 0; rr < R; ++rr)
#pragma unroll
              for (int d = 0; d < 3; ++d) {
                *reinterpret_cast<f4*>(Xt + tile_at(d * NR + 16 * rr + col, 4 * grp)) = Y[rr][d];
              }
            // (rows past the horizon repeat the last grid time, so all 16 rows count)
#pragma unroll
            for (int rr = 0; rr < R && rebuild; ++rr) {
              float lo[3], hi[3];
#pragma unroll
              for (int d = 0; d < 3; ++d) {
                const f4 v = Y[rr][d];
                lo[d] = grp_min(fminf(fminf(v[0], v[1]), fminf(v[2], v[3])));
                hi[d] = grp_max(fmaxf(fmaxf(v[0], v[1]), fmaxf(v[2], v[3])));
              }
              if (grp == 0) {
                float* bq = bbq + (16 * rr + col) * box_row(R);
                *reinterpret_cast<f4*>(bq) = f4{lo[0], lo[1], lo[2], 0.0f};
                *reinterpret_cast<f4*>(bq + 4) = f4{hi[0], hi[1], hi[2], 0.0f};
              }
            }
            // workspace rows (F_w of eq. f_e) on the same positions: residual (p - p_w) max(0,
            // 1 - 1/||M_w^{-1} (p - p_w)||), scaled by rho_w / rho_c so that it joins the collision
            // residuals in the accumulator (zero until now) and their S4 product
            if (WS && ws_eval) {
              bool wnz = false;
#pragma unroll
              for (int rr = 0; rr < R; ++rr) {
                float mx = 0.0f;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                  const float qx = Y[rr][0][r] - wcx, qy = Y[rr][1][r] - wcy, qz = Y[rr][2][r] - wcz;
                  const float s2 = (qx * qx + qy * qy) * wia2 + qz * qz * wib2;
                  mx = fmaxf(mx, s2);
                  // (s2 > 1 is a normal number, so the bare hardware rsqrt serves)
                  const float f = (16 * rr + col < n && s2 > 1.0f) ? wsc * (1.0f - __builtin_amdgcn_rsqf(s2)) : 0.0f;
                  Y[rr][0][r] = f * qx;
                  Y[rr][1][r] = f * qy;
                  Y[rr][2][r] = f * qz;
                  wnz |= f != 0.0f;
                }
                wsm[WS ? rr : 0] = fmaxf(wsm[WS ? rr : 0], grp_max(mx));
              }
              if (ballot(wnz) != 0) {
                ws_nz = true;
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
#pragma unroll
                  for (int d = 0; d < 3; ++d)
                    *reinterpret_cast<f4*>(Ct + tile_at(d * NR + 16 * rr + col, 4 * grp)) = Y[rr][d];
              }
            }
          }
          // ---- S1 velocity / acceleration, S3 bound balls in registers, S4 for nonzero tiles ----
#pragma unroll
          for (int b = 1; b < 3; ++b) {
            const bool on = b == 1 ? c.vel_on : c.acc_on;
            if (!on || !(eval_flags & b)) continue;
            const float lim = b == 1 ? vmax : amax;
            f4 Y[R][3];
            if constexpr (MP == 0) s1_32(a32c[((tau * 3 + b) * 2) * 64 + lane], Y);
            else s1_16(a16c[((tau * 3 + b) * 2) * 64 + lane], a16c[((tau * 3 + b) * 2 + 1) * 64 + lane], Y);
            bool nz = false;
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
              float mx = 0.0f;
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const float vx = Y[rr][0][r], vy = Y[rr][1][r], vz = Y[rr][2][r];
                const float ss = vx * vx + vy * vy + vz * vz;
                mx = fmaxf(mx, ss);
                // (ss > lim^2 is a normal number, so the bare hardware rsqrt serves)
                const float f = ss > lim * lim ? 1.0f - lim * __builtin_amdgcn_rsqf(ss) : 0.0f;
                Y[rr][0][r] = f * vx;
                Y[rr][1][r] = f * vy;
                Y[rr][2][r] = f * vz;
                nz |= f != 0.0f;
              }
              vm[b - 1][rr] = fmaxf(vm[b - 1][rr], grp_max(mx));
            }
            if (ballot(nz) != 0) {
              const float4 bq = a32c[((tau * 3 + b) * 2 + 1) * 64 + lane];
              const float b4[4] = {bq.x, bq.y, bq.z, bq.w};
#pragma unroll
              for (int rr = 0; rr < R; ++rr)
#pragma unroll
                for (int d = 0; d < 3; ++d)
#pragma unroll
                  for (int s = 0; s < 4; ++s) gacc[rr][d] = mfma4(Y[rr][d][s], b4[s], gacc[rr][d]);
            }
          }
          wave_sync();
          // ---- S2: broad phase over the tile (when the lists are rebuilt), narrow phase on the list ----
          // A pair is listed when its boxes, each gap shrunk by the margins above, are closer than the
          // safety distance (scaled, 1e-4 relative slack); until the next rebuild no unlisted pair can
          // come closer than the safety distance, so its residual is exactly zero.
          // (unused lanes test the pair (0, 1) and discard the result, so all box loads issue at once)
          int count = 0;
          int pnext = 0;
          if (rebuild) {
          bool act[PR];
#pragma unroll
          for (int r = 0; r < PR; ++r) {
            const int pij = mypair[r] >= 0 ? mypair[r] : (1 << 8);
            const int i = pij & 255, j = pij >> 8;
            const f4 li = *reinterpret_cast<const f4*>(bbq + i * box_row(R));
            const f4 hi = *reinterpret_cast<const f4*>(bbq + i * box_row(R) + 4);
            const f4 lj = *reinterpret_cast<const f4*>(bbq + j * box_row(R));
            const f4 hj = *reinterpret_cast<const f4*>(bbq + j * box_row(R) + 4);
            float g2 = 0.0f;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              const float gap = fmaxf(0.0f, fmaxf(lj[d] - hi[d], li[d] - hj[d]) - (d == 2 ? mgz : mgx));
              g2 += gap * gap * (d == 2 ? ib2 : ia2);
            }
            act[r] = mypair[r] >= 0 && g2 < 1.0001f;
            if (r % 2 == 1) __builtin_amdgcn_sched_barrier(0);   // box loads of two rounds in flight at most
          }
#pragma unroll
          for (int r = 0; r < PR; ++r) {
            const uint64_t mask = ballot(act[r]);
            if (act[r]) tl[1 + count + lanes_below(mask)] = mypair[r];
            count += __popcll(mask);
          }
          if (lane == 0) tl[0] = count;
          wave_sync();
          pnext = ps < count ? tl[1 + ps] : 0;
          } else {
            count = __builtin_amdgcn_readfirstlane(kept_count);
            pnext = ps < count ? kept_first : 0;
          }
          // narrow phase, one round of pairs per step; the next round's pair codes load meanwhile
          // (most tiles list at most one round)
          bool nzc = false;
          for (int base = 0; base < count; base += ppr) {
            const int slot = base + ps;
            const int pij = pnext;
            pnext = slot + ppr < count ? tl[1 + slot + ppr] : 0;
            if (slot < count && tt < nt) {
              const int i = pij & 255, j = pij >> 8;
              const float rx = Xt[tile_at(0 * NR + i, tt)] - Xt[tile_at(0 * NR + j, tt)];
              const float ry = Xt[tile_at(1 * NR + i, tt)] - Xt[tile_at(1 * NR + j, tt)];
              const float rz = Xt[tile_at(2 * NR + i, tt)] - Xt[tile_at(2 * NR + j, tt)];
              float Rx, Ry, Rz;
              coll_resid3(rx, ry, rz, ia2, ib2, sb, Rx, Ry, Rz);
              if (Rx != 0.0f || Ry != 0.0f || Rz != 0.0f) {
                nzc = true;
                atomicAdd(Ct + tile_at(0 * NR + i, tt), Rx);
                atomicAdd(Ct + tile_at(1 * NR + i, tt), Ry);
                atomicAdd(Ct + tile_at(2 * NR + i, tt), Rz);
                atomicAdd(Ct + tile_at(0 * NR + j, tt), -Rx);
                atomicAdd(Ct + tile_at(1 * NR + j, tt), -Ry);
                atomicAdd(Ct + tile_at(2 * NR + j, tt), -Rz);
              }
            }
          }
          if (ws_nz || ballot(nzc) != 0) {
            wave_sync();
            const float b4[4] = {cb.x, cb.y, cb.z, cb.w};
#pragma unroll
            for (int rr = 0; rr < R; ++rr)
#pragma unroll
              for (int d = 0; d < 3; ++d) {
                f4* cp = reinterpret_cast<f4*>(Ct + tile_at(d * NR + 16 * rr + col, 4 * grp));
                const f4 cr = *cp;
                *cp = f4{0.0f, 0.0f, 0.0f, 0.0f};     // the accumulator is kept zero between tiles
#pragma unroll
                for (int s = 0; s < 4; ++s) gacc[rr][d] = mfma4(cr[s], b4[s], gacc[rr][d]);
              }
          }
          wave_sync();
        }
        if constexpr (R == 1) __builtin_amdgcn_s_setprio(2);   // (see the tile phase)
        // this wave's partial back-projection and bound maxima -> its own LDS region
        {
          // Every lane stores, without branches: the rows of phantom robots (past n) fall in the
          // dead part of the position buffer (it holds 3 x 16R x 16 words), and lanes of the
          // columns past m (zero products) write distinct spare words after the 3 x 16R rows of m.
          float* gp = wbuf;
          const bool cv = col < m;
          const int spare = NR * 3 * m + (col - m) + (16 - m) * grp;
#pragma unroll
          for (int rr = 0; rr < R; ++rr)
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int robot = 16 * rr + 4 * grp + r;
                gp[cv ? (robot * 3 + d) * m + col : spare] = gacc[rr][d][r];
              }
          if (grp == 0) {
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
              if (eval_flags & 1) s_vmx[wave * NR + 16 * rr + col] = vm[0][rr];
              if (eval_flags & 2) s_amx[wave * NR + 16 * rr + col] = vm[1][rr];
              if constexpr (WS)
                if (ws_eval) s_wmx[wave * NR + 16 * rr + col] = wsm[rr];
            }
          }
        }
        __syncthreads();
        // Multiplier step (all coefficients) and QP step (free coefficients) of row (robot, axis):
        // g = F^T rho R summed over the waves, lambda <- lambda - g,
        // y = xi_bar - xi + lambda - g (+ the first-step correction), and
        // xi_free += X1 y + X01 mean_robots(y).
        // With HALVES = 2 a row is owned by two lanes 32 apart in one wave, each taking half of its
        // free and pinned coefficients; they swap their halves of y and mean(y) for the QP product.
        // Rows are axis-major, so the robots of one axis sit in aligned groups of 16R lanes.
        // Every load of the step is issued first, from clamped (always valid) addresses, and a
        // scheduling barrier keeps the arithmetic after them, so the step waits for LDS once; y is
        // zero past the free coefficients, so the QP product needs no guard either.
        if constexpr (QUART) {
          // Multiplier step and QP step of row (robot, ax), ax = this wave: lane robot + 16 q takes
          // the free coefficients f = q, q + 4, ... and the pinned ones r = q, q + 4.  Every lane
          // gathers its row's y and mean(y) from the four quarters with row swaps.
          const float* gp0 = smem + L.tiles;
          const int q4 = lane >> 4, rb = lane & 15, ax = wave;
          const bool on = rb < n;
          const int row = (on ? rb : 0) * 3 + ax;
          int qf[FQ], qpn[2];
          float xv[FQ], lf[FQ], xb[FQ], cr[FQ], gf[FQ][W], lp[2], gn[2][W];
#pragma unroll
          for (int j = 0; j < FQ; ++j) {
            const int f = q4 + 4 * j, fc = f < mf ? f : 0;
            qf[j] = row * m + 3 + fc;
            xv[j] = sxi[qf[j]];
            lf[j] = slam[qf[j]];
            xb[j] = sxb[qf[j]];
            cr[j] = scorr[row * (mf > 0 ? mf : 1) + fc];
#pragma unroll
            for (int ww = 0; ww < W; ++ww) gf[j][ww] = gp0[ww * L.per_wave + qf[j]];
          }
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            const int r = q4 + 4 * j, rc = r < kNFix ? r : 0;
            qpn[j] = row * m + fixed_k(rc);
            lp[j] = slam[qpn[j]];
#pragma unroll
            for (int ww = 0; ww < W; ++ww) gn[j][ww] = gp0[ww * L.per_wave + qpn[j]];
          }
          float cmax = s_cmx[row];   // running bound on |coefficient| of the row (pinned values included)
          __builtin_amdgcn_sched_barrier(0);
          auto sumw = [&](const float (&g)[W]) {
            float s = g[0];
#pragma unroll
            for (int ww = 1; ww < W; ++ww) s += g[ww];
            return s;
          };
          // the value of `v` in the four quarters of this lane's row, in quarter order
          auto quarters = [&](float v, float* out) {
            const auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
            const auto b0 = __builtin_amdgcn_permlane32_swap(a[0], a[0], false, false);
            const auto b1 = __builtin_amdgcn_permlane32_swap(a[1], a[1], false, false);
            out[0] = __uint_as_float(b0[0]);
            out[1] = __uint_as_float(b1[0]);
            out[2] = __uint_as_float(b0[1]);
            out[3] = __uint_as_float(b1[1]);
          };
          float ln[FQ], yo[FQ], gq[FQ];
#pragma unroll
          for (int j = 0; j < FQ; ++j) {
            gq[j] = sumw(gf[j]);
            ln[j] = lf[j] - gq[j];
            float yv = xb[j] - xv[j] + ln[j] - gq[j];
            if (k == 0) yv += cr[j];
            yo[j] = (on && q4 + 4 * j < mf) ? yv : 0.0f;
          }
          // all free coefficients' y and mean(y): index f = q + 4 j (zero past mf)
          float ya[4 * FQ], yba[4 * FQ];
#pragma unroll
          for (int j = 0; j < FQ; ++j) {
            quarters(yo[j], ya + 4 * j);
            quarters(group_sum<16>(yo[j]) * inv_n, yba + 4 * j);
          }
          float acc[FQ];
#pragma unroll
          for (int j = 0; j < FQ; ++j) {
            const int f = q4 + 4 * j, fr = f < mf ? f : 0;
            float a = 0.0f;
#pragma unroll
            for (int cc = 0; cc < QC; ++cc) {
              const f4 x1 = *reinterpret_cast<const f4*>(sX1 + fr * (4 * QC) + 4 * cc);
              const f4 x01 = *reinterpret_cast<const f4*>(sX1 + (mf + fr) * (4 * QC) + 4 * cc);
#pragma unroll
              for (int e = 0; e < 4; ++e)
                if (4 * cc + e < MFX) {
                  a = fmaf(x1[e], ya[4 * cc + e], a);
                  a = fmaf(x01[e], yba[4 * cc + e], a);
                }
            }
            acc[j] = a;
          }
          float dmax = 0.0f;
#pragma unroll
          for (int j = 0; j < FQ; ++j)
            if (q4 + 4 * j < mf) {
              dmax = fmaxf(dmax, fabsf(acc[j]));
              cmax = fmaxf(cmax, fabsf(xv[j] + acc[j]));
            }
          {
            float t[4];
            quarters(dmax, t);
            dmax = fmaxf(fmaxf(t[0], t[1]), fmaxf(t[2], t[3]));
            quarters(cmax, t);
            cmax = fmaxf(fmaxf(t[0], t[1]), fmaxf(t[2], t[3]));
          }
          if (fpr && on) {
#pragma unroll
            for (int j = 0; j < 2; ++j)
              if (q4 + 4 * j < kNFix) {
                const float g = sumw(gn[j]);
                fpsum = fmaf(g, g, fpsum);
                if (k == 0) {   // the pinned coefficients move to their boundary values in step 0
                  const float dx = pinned(row, q4 + 4 * j) - sxi[qpn[j]];
                  fpsum = fmaf(dx, dx, fpsum);
                }
              }
#pragma unroll
            for (int j = 0; j < FQ; ++j)
              if (q4 + 4 * j < mf) {
                fpsum = fmaf(gq[j], gq[j], fpsum);
                fpsum = fmaf(acc[j], acc[j], fpsum);
              }
          }
          if (on) {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
              const int r = q4 + 4 * j;
              if (r < kNFix) {
                slam[qpn[j]] = lp[j] - sumw(gn[j]);
                if (k == 0) {
                  const float xp = pinned(row, r);
                  sxi[qpn[j]] = xp;
                  if constexpr (MP != 0) put_split(rb, ax, fixed_k(r), xp);
                }
              }
            }
#pragma unroll
            for (int j = 0; j < FQ; ++j) {
              const int f = q4 + 4 * j;
              if (f < mf) {
                const float xn = xv[j] + acc[j];
                slam[qf[j]] = ln[j];
                sxi[qf[j]] = xn;
                if constexpr (MP != 0) put_split(rb, ax, 3 + f, xn);
              }
            }
            if (q4 == 0) {
              s_dxi[row] = dmax;
              s_cmx[row] = cmax;   // (the other quarters read it above, in the same wave)
            }
          }
        } else if (wave < TAILW) {
          const float* gp0 = smem + L.tiles;
          const int hl = HALVES == 2 ? (lane >> 5) : 0;
          const int trow = wave * (64 / HALVES) + (HALVES == 2 ? (lane & 31) : lane);
          const int ax = trow / NR, rb = trow - ax * NR;
          const bool on = ax < 3 && rb < n;
          const int row = on ? rb * 3 + ax : 0;
          constexpr int PF = kNFix / HALVES;                  // pinned coefficients per lane
          constexpr int QD = FHP > 4 ? 1 : 2;                 // QP rows loaded ahead of their use
          int qq[PF];
          float lp[PF], gr[PF + FH][W], xv[FH], lf[FH], xb[FH], cr[FH];
          int qx[FH];
          f4 qa[QD][FHP / 4], qb[QD][FHP / 4];
          auto qp_row = [&](int f2, f4 (&a1)[FHP / 4], f4 (&a2)[FHP / 4]) {
            const int rc = max(0, min(f2, mf - 1));
#pragma unroll
            for (int cc = 0; cc < FHP / 4; ++cc) {
              a1[cc] = *reinterpret_cast<const f4*>(sX1 + ((0 * HALVES + hl) * mf + rc) * FHP + 4 * cc);
              a2[cc] = *reinterpret_cast<const f4*>(sX1 + ((1 * HALVES + hl) * mf + rc) * FHP + 4 * cc);
            }
          };
#pragma unroll
          for (int j = 0; j < PF; ++j) {
            qq[j] = row * m + fixed_k(hl * PF + j);
            lp[j] = slam[qq[j]];
#pragma unroll
            for (int ww = 0; ww < W; ++ww) gr[j][ww] = gp0[ww * L.per_wave + qq[j]];
          }
#pragma unroll
          for (int j = 0; j < FH; ++j) {
            const int fc = max(0, min(hl * FH + j, mf - 1));
            const int q = row * m + 3 + fc;
            qx[j] = q;
            xv[j] = sxi[q];
            lf[j] = slam[q];
            xb[j] = sxb[q];
            cr[j] = LEAN ? 0.0f : scorr[row * (mf > 0 ? mf : 1) + fc];
#pragma unroll
            for (int ww = 0; ww < W; ++ww) gr[PF + j][ww] = gp0[ww * L.per_wave + q];
          }
          float cmax = s_cmx[row];   // running bound on |coefficient| of the row (pinned values included)
#pragma unroll
          for (int f2 = 0; f2 < QD; ++f2) qp_row(f2, qa[f2], qb[f2]);
          __builtin_amdgcn_sched_barrier(0);
          auto gsum = [&](int j) {
            float g = gr[j][0];
#pragma unroll
            for (int ww = 1; ww < W; ++ww) g += gr[j][ww];
            return g;
          };
          // pinned coefficients: multiplier step (their boundary values are set in step 0 below)
          float nl[PF];
#pragma unroll
          for (int j = 0; j < PF; ++j) nl[j] = lp[j] - gsum(j);
          // free coefficients f = hl * FH + j
          float yo[FH], ln[FH];
#pragma unroll
          for (int j = 0; j < FH; ++j) {
            const int f = hl * FH + j;
            const float g = gsum(PF + j);
            ln[j] = lf[j] - g;
            float yv = xb[j] - xv[j] + ln[j] - g;
            if (k == 0) {
              if constexpr (LEAN) {
                if (on && f < mf) sxb[qx[j]] = xi_bar[coef + qx[j]];   // drop the correction again
              } else {
                yv += cr[j];
              }
            }
            yo[j] = (on && f < mf) ? yv : 0.0f;
          }
          float ybo[FH];
#pragma unroll
          for (int j = 0; j < FH; ++j) ybo[j] = group_sum<NR>(yo[j]) * inv_n;
          // all free coefficients' y and mean(y), in order (zero past mf)
          float ya[HALVES * FH], yba[HALVES * FH];
#pragma unroll
          for (int j = 0; j < FH; ++j) {
            if constexpr (HALVES == 2) {
              const auto sy = __builtin_amdgcn_permlane32_swap(__float_as_uint(yo[j]), __float_as_uint(yo[j]), false, false);
              const auto sb2 = __builtin_amdgcn_permlane32_swap(__float_as_uint(ybo[j]), __float_as_uint(ybo[j]), false, false);
              ya[j] = __uint_as_float(sy[0]);        // half 0
              ya[FH + j] = __uint_as_float(sy[1]);   // half 1
              yba[j] = __uint_as_float(sb2[0]);
              yba[FH + j] = __uint_as_float(sb2[1]);
            } else {
              ya[j] = yo[j];
              yba[j] = ybo[j];
            }
          }
          // own outputs: acc[j] = sum_f2 X1[f][f2] y[f2] + X01[f][f2] mean(y)[f2], f2 in order
          float acc[FHP];
#pragma unroll
          for (int j = 0; j < FHP; ++j) acc[j] = 0.0f;
          // (rows QD ahead are loaded as each row is used; the barriers keep that order)
#pragma unroll
          for (int f2 = 0; f2 < MFX; ++f2) {
            const int sl = f2 % QD;
#pragma unroll
            for (int j = 0; j < FHP; ++j) {
              acc[j] = fmaf(qa[sl][j / 4][j % 4], ya[f2], acc[j]);
              acc[j] = fmaf(qb[sl][j / 4][j % 4], yba[f2], acc[j]);
            }
            if (f2 + QD < MFX) qp_row(f2 + QD, qa[sl], qb[sl]);
            __builtin_amdgcn_sched_barrier(0);
          }
          float dmax = 0.0f;
#pragma unroll
          for (int j = 0; j < FH; ++j)
            if (hl * FH + j < mf) {
              dmax = fmaxf(dmax, fabsf(acc[j]));
              cmax = fmaxf(cmax, fabsf(xv[j] + acc[j]));
            }
          if constexpr (HALVES == 2) {
            const auto sd = __builtin_amdgcn_permlane32_swap(__float_as_uint(dmax), __float_as_uint(dmax), false, false);
            dmax = fmaxf(__uint_as_float(sd[0]), __uint_as_float(sd[1]));
            const auto sc = __builtin_amdgcn_permlane32_swap(__float_as_uint(cmax), __float_as_uint(cmax), false, false);
            cmax = fmaxf(__uint_as_float(sc[0]), __uint_as_float(sc[1]));
          }
          if (fpr && on) {
#pragma unroll
            for (int j = 0; j < PF; ++j) {
              const float g = gsum(j);
              fpsum = fmaf(g, g, fpsum);
              if (k == 0) {   // the pinned coefficients move to their boundary values in step 0
                const float dx = pinned(row, hl * PF + j) - sxi[qq[j]];
                fpsum = fmaf(dx, dx, fpsum);
              }
            }
#pragma unroll
            for (int j = 0; j < FH; ++j)
              if (hl * FH + j < mf) {
                const float g = gsum(PF + j);
                fpsum = fmaf(g, g, fpsum);
                fpsum = fmaf(acc[j], acc[j], fpsum);
              }
          }
          if (on) {
#pragma unroll
            for (int j = 0; j < PF; ++j) {
              slam[qq[j]] = nl[j];
              if (k == 0) {
                const float xp = pinned(row, hl * PF + j);
                sxi[qq[j]] = xp;
                if constexpr (MP != 0) put_split(rb, ax, fixed_k(hl * PF + j), xp);
              }
            }
#pragma unroll
            for (int j = 0; j < FH; ++j) {
              const int f = hl * FH + j;
              if (f < mf) {
                const float xn = xv[j] + acc[j];
                slam[row * m + 3 + f] = ln[j];
                sxi[row * m + 3 + f] = xn;
                if constexpr (MP != 0) put_split(rb, ax, 3 + f, xn);
              }
            }
            if (hl == 0) {
              s_dxi[row] = dmax;
              s_cmx[row] = cmax;   // (the other half read it above, in the same wave)
            }
          }
        }
        __syncthreads();
      }

      // ---- primal residual of the last step (dense over pairs) ----
      float rmax = 0.0f;   // its largest block norm (thread 0)
      if (resid_out || status_out) {
        float ss = 0.0f, mx = 0.0f;
        if (iters_s > 0) {
          if constexpr (R == 2) {
            // the wave's pair lists are no longer needed (lane index from an opaque copy, so that
            // nothing of the fill is computed ahead of the iterations)
            int ln = threadIdx.x & 63;
            asm volatile("" : "+v"(ln));
            fill_pairs(ln, 64);
            wave_sync();
          }
          // One basis product of a tile for the iterate in `src` (previous or new).  The B operands
          // are formed per product (this runs once per solve), so that only one iterate's
          // products are live at a time.
          auto prod = [&](const float* src, int tau, int b, f4 (&Y)[R][3]) {
            if constexpr (MP == 0) {
              const float4 av = a32c[((tau * 3 + b) * 2) * 64 + lane];
              const float a1[4] = {av.x, av.y, av.z, av.w};
#pragma unroll
              for (int rr = 0; rr < R; ++rr)
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                  f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                  for (int s = 0; s < KS; ++s) {
                    const int robot = 16 * rr + col, kk = 4 * s + grp;
                    const float v = (robot < n && kk < m) ? src[(robot * 3 + d) * m + kk] : 0.0f;
                    acc = mfma4(a1[s], v, acc);
                  }
                  Y[rr][d] = acc;
                }
            } else {
              typedef typename Half<MP>::V V;
              const uint4* at = a16c + ((tau * 3 + b) * 2) * 64 + lane;
              const V A1 = __builtin_bit_cast(V, at[0]);
              const V A2 = __builtin_bit_cast(V, at[64]);
#pragma unroll
              for (int rr = 0; rr < R; ++rr)
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                  V h1, h2;
                  split_xi<MP>(src, 16 * rr + col, n, m, d, grp, h1, h2);
                  f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
                  acc = mfma16(A1, h1, acc);
                  acc = mfma16(A2, h2, acc);
                  Y[rr][d] = acc;
                }
            }
          };
#pragma unroll 1
          for (int q = 0; q < TQ; ++q) {
            const int tau = wave + W * q;
            if (tau >= NT) break;
            const int t0 = 16 * tau;
            const int nt = min(16, H - t0);
#pragma unroll 1
            for (int b = 0; b < 3; ++b) {
              if (b > 0 && !(b == 1 ? c.vel_on : c.acc_on)) continue;
              const float lim = b == 1 ? vmax : amax;
              f4 Y[R][3];
              if constexpr (LEAN) prod(xi_out + coef, tau, b, Y);
              else prod(sxprev, tau, b, Y);
              if (b == 0) {
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
#pragma unroll
                  for (int d = 0; d < 3; ++d)
                    *reinterpret_cast<f4*>(Xt + tile_at(d * NR + 16 * rr + col, 4 * grp)) = Y[rr][d];
              } else {
                // targets of the bound balls at the previous iterate: e = v - R(v)
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
#pragma unroll
                  for (int r = 0; r < 4; ++r) {
                    const float vx = Y[rr][0][r], vy = Y[rr][1][r], vz = Y[rr][2][r];
                    const float s2 = vx * vx + vy * vy + vz * vz;
                    const float f = s2 > lim * lim ? 1.0f - lim * rsqrtf(s2) : 0.0f;
                    Y[rr][0][r] = vx - f * vx;
                    Y[rr][1][r] = vy - f * vy;
                    Y[rr][2][r] = vz - f * vz;
                  }
              }
              f4 Yn[R][3];
              prod(sxi, tau, b, Yn);
              if (b == 0) {
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
#pragma unroll
                  for (int d = 0; d < 3; ++d)
                    *reinterpret_cast<f4*>(Ct + tile_at(d * NR + 16 * rr + col, 4 * grp)) = Yn[rr][d];
                if (WS && c.ws_on) {
                  // workspace rows: r_p = p_new - e(p_prev), e = p - (p - p_w) max(0, 1 - 1/||s||)
#pragma unroll
                  for (int rr = 0; rr < R; ++rr)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                      const float qx = Y[rr][0][r] - wcx, qy = Y[rr][1][r] - wcy, qz = Y[rr][2][r] - wcz;
                      const float s2 = (qx * qx + qy * qy) * wia2 + qz * qz * wib2;
                      const float f = s2 > 1.0f ? 1.0f - rsqrtf(s2) : 0.0f;
                      const float px = Yn[rr][0][r] - (Y[rr][0][r] - f * qx);
                      const float py = Yn[rr][1][r] - (Y[rr][1][r] - f * qy);
                      const float pz = Yn[rr][2][r] - (Y[rr][2][r] - f * qz);
                      const bool real = 4 * grp + r < nt && 16 * rr + col < n;   // grid times, robots
                      const float nrm = real ? px * px + py * py + pz * pz : 0.0f;
                      ss += nrm;
                      mx = fmaxf(mx, nrm);
                    }
                }
                continue;
              }
              // bound balls: r_p = v_new - e(v_prev)
#pragma unroll
              for (int rr = 0; rr < R; ++rr)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                  const float px = Yn[rr][0][r] - Y[rr][0][r];
                  const float py = Yn[rr][1][r] - Y[rr][1][r];
                  const float pz = Yn[rr][2][r] - Y[rr][2][r];
                  const float nrm = 4 * grp + r < nt ? px * px + py * py + pz * pz : 0.0f;   // grid times only
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
                  rp[d] = Xt[tile_at(d * NR + i, col)] - Xt[tile_at(d * NR + j, col)];
                  rn[d] = Ct[tile_at(d * NR + i, col)] - Ct[tile_at(d * NR + j, col)];
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
        // per-wave sums and maxima (cross-lane, in a fixed order) in the wave's own region, then
        // combined in wave order
        {
          const float ws = wave_sum(ss), wm = wave_max(mx), wf = wave_sum(fpsum);
          if (lane == 0) {
            wbuf[0] = ws;
            wbuf[1] = wm;
            wbuf[2] = wf;
          }
        }
        __syncthreads();
        if (tid == 0) {
          float s = 0.0f, mm = 0.0f, fs = 0.0f;
          for (int ww = 0; ww < W; ++ww) {
            const float* pw = smem + L.tiles + ww * L.per_wave;
            s += pw[0];
            mm = fmaxf(mm, pw[1]);
            fs += pw[2];
          }
          rmax = sqrtf(mm);
          if (resid_out) {
            resid_out[sidx * rw + 0] = s;
            resid_out[sidx * rw + 1] = rmax;
            if (fpr) resid_out[sidx * rw + 2] = fs;
          }
        }
        __syncthreads();
      }
      for (int q = tid; q < nDm; q += nthr) {
        xi_out[coef + q] = sxi[q];
        if (lam_out) lam_out[coef + q] = slam[q];
      }
      // convergence bits (the status pass adds the finiteness of the outputs)
      if (status_out && tid == 0) status_out[sidx] = in_flag < 0 ? in_flag : sample_status<float>(false, false, rmax, iters_s);
      __syncthreads();
    }
  }
}

// One workgroup per work item (grid-stride), single shape class.
template <int R, int KS, int W, int MP, int WPE, int WS>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
fast_project_kernel(FastArgs A) {
  extern __shared__ __align__(16) float smem[];
  for (int it = blockIdx.x; it < A.n_items; it += gridDim.x) fast_item<R, KS, W, MP, WS>(A, it, smem);
}

// Persistent kernel over the work items of one robot-tile class (R tiles of 16 robots) of a
// ragged batch: workgroups pull items (sorted by decreasing cost on the host) from an atomic
// queue until it is empty.  Every wave reaches the exit once the queue is drained.
template <int R, int KS, int W, int MP, int WPE, int WS>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
fast_batched_kernel(FastArgs A, int* __restrict__ queue) {
  extern __shared__ __align__(16) float smem[];
  __shared__ int next;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(queue, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(next);
    __syncthreads();
    if (it >= A.n_items) break;
    fast_item<R, KS, W, MP, WS>(A, it, smem);
  }
}

// Resets the queue heads of a launch sequence (a kernel node rather than a memset, so the
// sequence can be captured in a graph).
__global__ void reset_queue_kernel(int* queue, int n) {
  if (threadIdx.x == 0 && blockIdx.x == 0)
    for (int i = 0; i < n; ++i) queue[i] = 0;
}

// Kernel instances: R robot tiles of 16, KS k-steps of 4 coefficients, W waves per workgroup.
// Target waves per SIMD (the register budget): 3 with one robot tile (168 VGPRs; three waves per
// sample then keep four samples per CU resident); with two robot tiles 2 for three or four waves
// per sample (256 VGPRs; two workgroups per CU by LDS, six or eight waves) and 1 for two (the whole
// register file).
constexpr int waves_per_simd(int R, int MP, int W) { return R == 1 ? 3 : (W >= 3 ? 2 : 1); }

FastArgs make_fast_args(const LaunchArgs& a, const float* tab32, const uint4* a16) {
  FastArgs f;
  f.cfgs = a.cfgs; f.tab = tab32; f.a16 = a16; f.probs = a.probs; f.items = a.items; f.n_items = a.n_items;
  f.xi_bar = static_cast<const float*>(a.xi_bar); f.bvals = static_cast<const float*>(a.bvals);
  f.xi0 = static_cast<const float*>(a.xi0); f.lam0 = static_cast<const float*>(a.lam0); f.iters = a.iters;
  f.xi_out = static_cast<float*>(a.xi_out); f.lam_out = static_cast<float*>(a.lam_out);
  f.resid_out = static_cast<float*>(a.resid_out); f.status_out = a.status_out; f.ckpt = static_cast<float*>(a.ckpt);
  f.ckpt_every = a.ckpt_every; f.ckpt_stride = a.ckpt_stride;
  f.fpr = (a.flags & SF_FP_RESIDUAL) != 0;
  return f;
}

template <int R, int KS, int W, int MP, int WS>
hipError_t launch_instance(const FastPlan& p, const LaunchArgs& a, const float* tab32, const uint4* a16) {
  auto kern = fast_project_kernel<R, KS, W, MP, waves_per_simd(R, MP, W), WS>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds_bytes[W - 2][MP]);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(a.n_items), dim3(64 * W), p.lds_bytes[W - 2][MP], a.stream, make_fast_args(a, tab32, a16));
  return hipGetLastError();
}


template <int R, int KS, int W, int MP, int WS>
hipError_t launch_class(const FastClass& C, const FastArgs& f, int grid, int* queue, hipStream_t stream) {
  auto kern = fast_batched_kernel<R, KS, W, MP, waves_per_simd(R, MP, W), WS>;
  const size_t lds = C.lds_bytes[W - 2][MP];
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * W), lds, stream, f, queue);
  return hipGetLastError();
}

// One class of a persistent launch sequence with W waves per workgroup; grid > 0: workgroups (at most
// the class's work items), 0: the class's default.
template <int R, int KS, int MP, int WS>
hipError_t launch_class_w(const FastClass& C, const FastArgs& f, int grid, int W, int* queue, hipStream_t stream) {
  switch (W) {
    case 2: return launch_class<R, KS, 2, MP, WS>(C, f, grid, queue, stream);
    case 3: return launch_class<R, KS, 3, MP, WS>(C, f, grid, queue, stream);
    case 4:
      if constexpr (WS == 0) return launch_class<R, KS, 4, MP, WS>(C, f, grid, queue, stream);
      break;
    default: break;
  }
  fast_set_error("no persistent kernel instance for this shape");
  return hipErrorNotSupported;
}

// Single-shape launch of the instance for (R, KS, W) of this precision and workspace flag.
template <int MP, int WS>
hipError_t launch_single_mp(const FastPlan& p, const LaunchArgs& a, const float* tab32, const uint4* a16, int W) {
  const int key = p.R * 100 + p.KS * 10 + W;
  if constexpr (WS == 0) {
    switch (key) {
      case 122: return launch_instance<1, 2, 2, MP, 0>(p, a, tab32, a16);
      case 123: return launch_instance<1, 2, 3, MP, 0>(p, a, tab32, a16);
      case 124: return launch_instance<1, 2, 4, MP, 0>(p, a, tab32, a16);
      case 132: return launch_instance<1, 3, 2, MP, 0>(p, a, tab32, a16);
      case 133: return launch_instance<1, 3, 3, MP, 0>(p, a, tab32, a16);
      case 134: return launch_instance<1, 3, 4, MP, 0>(p, a, tab32, a16);
      case 142: return launch_instance<1, 4, 2, MP, 0>(p, a, tab32, a16);
      case 143: return launch_instance<1, 4, 3, MP, 0>(p, a, tab32, a16);
      case 144: return launch_instance<1, 4, 4, MP, 0>(p, a, tab32, a16);
      case 232: return launch_instance<2, 3, 2, MP, 0>(p, a, tab32, a16);
      case 233: return launch_instance<2, 3, 3, MP, 0>(p, a, tab32, a16);
      case 234: return launch_instance<2, 3, 4, MP, 0>(p, a, tab32, a16);
      case 242: return launch_instance<2, 4, 2, MP, 0>(p, a, tab32, a16);
      case 243: return launch_instance<2, 4, 3, MP, 0>(p, a, tab32, a16);
      case 244: return launch_instance<2, 4, 4, MP, 0>(p, a, tab32, a16);
      default: break;
    }
  } else {
    // with the workspace rows: 2 or 3 waves per workgroup
    switch (key) {
      case 122: return launch_instance<1, 2, 2, MP, 1>(p, a, tab32, a16);
      case 123: return launch_instance<1, 2, 3, MP, 1>(p, a, tab32, a16);
      case 132: return launch_instance<1, 3, 2, MP, 1>(p, a, tab32, a16);
      case 133: return launch_instance<1, 3, 3, MP, 1>(p, a, tab32, a16);
      case 142: return launch_instance<1, 4, 2, MP, 1>(p, a, tab32, a16);
      case 143: return launch_instance<1, 4, 3, MP, 1>(p, a, tab32, a16);
      case 232: return launch_instance<2, 3, 2, MP, 1>(p, a, tab32, a16);
      case 233: return launch_instance<2, 3, 3, MP, 1>(p, a, tab32, a16);
      case 242: return launch_instance<2, 4, 2, MP, 1>(p, a, tab32, a16);
      case 243: return launch_instance<2, 4, 3, MP, 1>(p, a, tab32, a16);
      default: break;
    }
  }
  fast_set_error("no kernel instance for this shape");
  return hipErrorNotSupported;
}

// Persistent launch sequence (one kernel per robot-tile class) of this precision and workspace flag:
// the queue heads are reset, then each class selected by cls_mask runs with its own waves per
// workgroup W[c] and workgroup count grid[c] (0 = the class's default).
template <int MP, int WS>
hipError_t launch_batched_mp(const FastPlan& p, const LaunchArgs& a, const float* tab32, const uint4* a16,
                             const int* grid, const int* W, int cls_mask) {
  hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(64), 0, a.stream, p.d_queue, p.n_cls);
  for (int ci = 0; ci < p.n_cls; ++ci) {
    if (!(cls_mask & (1 << ci))) continue;
    const FastClass& C = p.cls[ci];
    FastArgs f = make_fast_args(a, tab32, a16);
    f.items = p.d_items_sorted + C.offset;
    f.n_items = C.n_items;
    const int g = std::max(1, std::min(C.n_items, grid[ci] > 0 ? grid[ci] : C.grid));
    int* q = p.d_queue + ci;
    hipError_t e;
    switch (C.R * 10 + p.KS) {
      case 12: e = launch_class_w<1, 2, MP, WS>(C, f, g, W[ci], q, a.stream); break;
      case 13: e = launch_class_w<1, 3, MP, WS>(C, f, g, W[ci], q, a.stream); break;
      case 14: e = launch_class_w<1, 4, MP, WS>(C, f, g, W[ci], q, a.stream); break;
      case 22: e = launch_class_w<2, 2, MP, WS>(C, f, g, W[ci], q, a.stream); break;
      case 23: e = launch_class_w<2, 3, MP, WS>(C, f, g, W[ci], q, a.stream); break;
      case 24: e = launch_class_w<2, 4, MP, WS>(C, f, g, W[ci], q, a.stream); break;
      default:
        fast_set_error("no persistent kernel instance for this shape");
        return hipErrorNotSupported;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace
}  // namespace fastk
}  // namespace sf
