// Host side of the MFMA fast path: 16-bit and fp32 basis-operand tables, batch plans (default
// launch shape, persistent work-queue classes) and dispatch to the kernel instances, which live in
// sf_fast_p<MP>_w<WS>.hip (kernels in sf_fast_kernel.h).
#include "sf_fast_kernel.h"

namespace sf {

static thread_local std::string g_fast_err;

std::string fast_last_error() { return g_fast_err; }
void fast_set_error(const char* msg) { g_fast_err = msg; }

hipError_t fast_launch_single_p0_w0(const FastPlan&, const LaunchArgs&, const float*, const uint4*, int);
hipError_t fast_launch_batched_p0_w0(const FastPlan&, const LaunchArgs&, const float*, const uint4*, const int*, const int*,
                                     int);
hipError_t fast_launch_single_p0_w1(const FastPlan&, const LaunchArgs&, const float*, const uint4*, int);
hipError_t fast_launch_batched_p0_w1(const FastPlan&, const LaunchArgs&, const float*, const uint4*, const int*, const int*,
                                     int);
hipError_t fast_launch_single_p1_w0(const FastPlan&, const LaunchArgs&, const float*, const uint4*, int);
hipError_t fast_launch_batched_p1_w0(const FastPlan&, const LaunchArgs&, const float*, const uint4*, const int*, const int*,
                                     int);
hipError_t fast_launch_single_p1_w1(const FastPlan&, const LaunchArgs&, const float*, const uint4*, int);
hipError_t fast_launch_batched_p1_w1(const FastPlan&, const LaunchArgs&, const float*, const uint4*, const int*, const int*,
                                     int);
hipError_t fast_launch_single_p2_w0(const FastPlan&, const LaunchArgs&, const float*, const uint4*, int);
hipError_t fast_launch_batched_p2_w0(const FastPlan&, const LaunchArgs&, const float*, const uint4*, const int*, const int*,
                                     int);
hipError_t fast_launch_single_p2_w1(const FastPlan&, const LaunchArgs&, const float*, const uint4*, int);
hipError_t fast_launch_batched_p2_w1(const FastPlan&, const LaunchArgs&, const float*, const uint4*, const int*, const int*,
                                     int);

using fastk::fast_lds_plan;
using fastk::waves_per_simd;


int64_t a16_entries(const DevCfg& c) { return (int64_t)((c.H + 15) / 16) * 3 * 2 * 64; }

namespace {

uint16_t bf16_bits(float f) {            // round to nearest even
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

float bf16_value(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

uint16_t f16_bits(float f) {
  const _Float16 h = static_cast<_Float16>(f);
  uint16_t b;
  std::memcpy(&b, &h, 2);
  return b;
}

float f16_value(uint16_t b) {
  _Float16 h;
  std::memcpy(&h, &b, 2);
  return static_cast<float>(h);
}

}  // namespace

int64_t a32_entries(const DevCfg& c) { return (int64_t)((c.H + 15) / 16) * 3 * 2 * 64; }

void a32_fill(const DevCfg& c, const double* P3, float* out) {
  const int NT = (c.H + 15) / 16;
  const double rho[3] = {c.rho_c, c.rho_v, c.rho_a};
  for (int tau = 0; tau < NT; ++tau)
    for (int b = 0; b < 3; ++b)
      for (int lane = 0; lane < 64; ++lane) {
        const int col = lane & 15, grp = lane >> 4;
        // S1: P[t = 16 tau + col][k = 4 s + grp], times past the horizon repeat the last grid time (so
        // every row of the product is a real point of the trajectory); S4: zero past the horizon
        float* a = out + ((((size_t)tau * 3 + b) * 2 + 0) * 64 + lane) * 4;
        float* bq = out + ((((size_t)tau * 3 + b) * 2 + 1) * 64 + lane) * 4;  // S4: rho P[t = 16 tau + 4 grp + s][k = col]
        for (int s = 0; s < 4; ++s) {
          const int t = std::min(16 * tau + col, c.H - 1), k = 4 * s + grp;
          a[s] = k < c.m ? (float)P3[((size_t)b * c.H + t) * c.m + k] : 0.0f;
          const int t4 = 16 * tau + 4 * grp + s;
          bq[s] = (t4 < c.H && col < c.m) ? (float)(rho[b] * P3[((size_t)b * c.H + t4) * c.m + col]) : 0.0f;
        }
      }
}

void a16_fill(const DevCfg& c, const double* P3, int precision, uint16_t* out) {
  const int NT = (c.H + 15) / 16;
  const bool bf = precision == SF_BF16;
  for (int tau = 0; tau < NT; ++tau)
    for (int b = 0; b < 3; ++b)
      for (int inst = 0; inst < 2; ++inst)
        for (int lane = 0; lane < 64; ++lane) {
          const int col = lane & 15, grp = lane >> 4, t = std::min(16 * tau + col, c.H - 1);
          for (int v = 0; v < 8; ++v) {
            const int k = 8 * (grp & 1) + v;
            uint16_t bits = 0;
            if (k < c.m) {
              const double P = P3[((size_t)b * c.H + t) * c.m + k];
              const uint16_t hi = bf ? bf16_bits((float)P) : f16_bits((float)P);
              const double hv = bf ? bf16_value(hi) : f16_value(hi);
              const uint16_t lo = bf ? bf16_bits((float)(P - hv)) : f16_bits((float)(P - hv));
              if (grp < 2) bits = hi;
              else bits = inst == 0 ? lo : 0;
            }
            out[((((size_t)tau * 3 + b) * 2 + inst) * 64 + lane) * 8 + v] = bits;
          }
        }
}

namespace {

bool cfg_supported(const DevCfg& c) { return c.D == 3 && c.n <= 32 && c.m <= 16 && c.H <= 256; }

// Relative cost of one sample-iteration: S1 MFMA work grows with the robot tiles and time tiles,
// the broad phase with the number of pairs.
double item_cost(const DevCfg& c, int count) {
  const int NT = (c.H + 15) / 16;
  const int R = c.n <= 16 ? 1 : 2;
  return (double)count * NT * (24.0 * R * ((c.m + 3) / 4) + c.n * (c.n - 1) / 2.0);
}

}  // namespace

bool fast_cfg_covered(const DevCfg& c) {
  return cfg_supported(c) && (size_t)fast_lds_plan(c, c.n <= 16 ? 1 : 2, 4, 1).total * 4 <= 160 * 1024;
}

sf_status fast_plan_build(const std::vector<DevCfg>& cfgs, const std::vector<DevProblem>& probs,
                          const std::vector<WorkItem>& items, bool persistent, FastPlan& out) {
  fast_plan_free(out);
  out = FastPlan();
  // the problems the work items refer to
  std::vector<char> used(probs.size(), 0);
  for (const WorkItem& w : items) used[w.problem] = 1;
  int first = -1;
  for (size_t q = 0; q < probs.size() && first < 0; ++q)
    if (used[q]) first = (int)q;
  if (first < 0) return SF_OK;
  bool mixed = false;
  int maxKS = 2, maxNT = 1;
  for (size_t q = 0; q < probs.size(); ++q) {
    if (!used[q]) continue;
    const DevProblem& p = probs[q];
    const DevCfg& c = cfgs[p.cfg];
    if (!cfg_supported(c)) return SF_OK;                 // generic path
    if (p.cfg != probs[first].cfg) mixed = true;
    if (c.ws_on) out.ws = true;
    maxKS = std::max(maxKS, (c.m + 3) / 4);
    maxNT = std::max(maxNT, (c.H + 15) / 16);
    for (int wi = 0; wi < 3; ++wi)
      for (int mp = 0; mp < 3; ++mp)
        out.lds_bytes[wi][mp] = std::max(out.lds_bytes[wi][mp],
                                         (size_t)fast_lds_plan(c, c.n <= 16 ? 1 : 2, wi + 2, mp).total * 4);
  }
  if (out.lds_bytes[2][1] > 160 * 1024) return SF_OK;
  const DevCfg& c0 = cfgs[probs[first].cfg];
  out.KS = maxKS;
  out.R = c0.n <= 16 ? 1 : 2;
  out.batched = mixed || persistent;
  {
    // default waves per workgroup (below)
    int dev = 0, ncu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    out.ncu = ncu > 0 ? ncu : 256;
    // resident work items at W waves per workgroup for the register budget of each precision
    auto slots = [&](int W, int mp) {
      const int by_waves = (4 * waves_per_simd(mixed ? 2 : out.R, mp, W)) / W;
      const int by_lds = (int)((160 * 1024) / std::max<size_t>(out.lds_bytes[W - 2][mp], 1));
      return (int64_t)std::max(1, std::min(by_waves, by_lds)) * out.ncu;
    };
    const int64_t ni = (int64_t)items.size();
    for (int prec = SF_FP32; prec <= SF_FP16; ++prec) {
      const int mp = prec - SF_FP32;
      // the most waves per workgroup that still lets every work item be resident at once; with
      // more items than that, the most waves in flight (the fewer waves per workgroup on a tie,
      // which keeps more items in flight)
      int best = ni <= slots(4, mp) ? 4 : (ni <= slots(3, mp) ? 3 : 0);
      if (best == 0) {
        int64_t most = -1;
        for (int W = 2; W <= 4; ++W) {
          const int64_t waves = std::min(ni, slots(W, mp)) * W;
          if (waves > most) {
            most = waves;
            best = W;
          }
        }
      }
      out.Wp[prec & 3] = best;
    }
  }
  if (out.batched) {
    // One persistent launch per robot-tile class (17-32 robots first, then up to 16), each kernel
    // compiled for its own register budget; inside a class, longest-processing-time order.
    std::vector<std::pair<double, int>> order[2];
    for (size_t i = 0; i < items.size(); ++i) {
      const DevCfg& c = cfgs[probs[items[i].problem].cfg];
      order[c.n > 16 ? 0 : 1].push_back({item_cost(c, items[i].count), (int)i});
    }
    std::vector<WorkItem> sorted;
    const int wdef = out.Wp[SF_FP32 & 3];
    for (int k = 0; k < 2; ++k) {
      if (order[k].empty()) continue;
      std::stable_sort(order[k].begin(), order[k].end(),
                       [](const std::pair<double, int>& a, const std::pair<double, int>& b) { return a.first > b.first; });
      FastClass& C = out.cls[out.n_cls++];
      C.R = k == 0 ? 2 : 1;
      C.offset = (int)sorted.size();
      C.n_items = (int)order[k].size();
      for (const auto& o : order[k]) {
        sorted.push_back(items[o.second]);
        const DevCfg& c = cfgs[probs[items[o.second].problem].cfg];
        for (int wi = 0; wi < 3; ++wi)
          for (int mp = 0; mp < 3; ++mp)
            C.lds_bytes[wi][mp] = std::max(C.lds_bytes[wi][mp], (size_t)fast_lds_plan(c, C.R, wi + 2, mp).total * 4);
      }
      const int per_cu = std::max(1, std::min(4, (int)((160 * 1024) / std::max<size_t>(C.lds_bytes[wdef - 2][0], 1))));
      C.grid = std::min(C.n_items, out.ncu * per_cu);
    }
    hipError_t e = hipMalloc(&out.d_items_sorted, sorted.size() * sizeof(WorkItem));
    if (e == hipSuccess)
      e = hipMemcpy(out.d_items_sorted, sorted.data(), sorted.size() * sizeof(WorkItem), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&out.d_queue, 2 * sizeof(int));
    if (e != hipSuccess) {
      fast_plan_free(out);
      g_fast_err = "persistent plan allocation failed";
      return SF_ENOMEM;
    }
  }
  out.ok = true;
  return SF_OK;
}

void fast_plan_free(FastPlan& p) {
  if (p.d_items_sorted) (void)hipFree(p.d_items_sorted);
  if (p.d_queue) (void)hipFree(p.d_queue);
  p.d_items_sorted = nullptr;
  p.d_queue = nullptr;
  p.ok = false;
}

hipError_t fast_launch_batched(const FastPlan& p, const LaunchArgs& a, const float* tab32, const void* a16,
                               int precision, const int* grid, const int* W, int cls_mask) {
  const uint4* t = static_cast<const uint4*>(a16);
  const bool ws = p.ws;
  switch (precision) {
    case SF_FP32:
      return ws ? fast_launch_batched_p0_w1(p, a, tab32, t, grid, W, cls_mask)
                : fast_launch_batched_p0_w0(p, a, tab32, t, grid, W, cls_mask);
    case SF_BF16:
      return ws ? fast_launch_batched_p1_w1(p, a, tab32, t, grid, W, cls_mask)
                : fast_launch_batched_p1_w0(p, a, tab32, t, grid, W, cls_mask);
    case SF_FP16:
      return ws ? fast_launch_batched_p2_w1(p, a, tab32, t, grid, W, cls_mask)
                : fast_launch_batched_p2_w0(p, a, tab32, t, grid, W, cls_mask);
    default:
      g_fast_err = "precision not implemented in the MFMA kernels";
      return hipErrorNotSupported;
  }
}

hipError_t fast_launch(const FastPlan& p, const LaunchArgs& a, const float* tab32, const void* a16, int precision) {
  const int pi = precision & 3;
  auto waves = [&](int tuned) {
    int W = tuned > 0 ? tuned : p.Wp[pi];
    if (p.ws && W > 3) W = 3;   // the workspace instances have 2 or 3 waves per workgroup
    return W;
  };
  if (p.batched) {
    const int W[2] = {waves(p.tuned_wc[pi][0]), waves(p.tuned_wc[pi][1])};
    return fast_launch_batched(p, a, tab32, a16, precision, p.tuned_gc[pi], W, 3);
  }
  return fast_launch_single(p, a, tab32, a16, precision, waves(p.tuned_w[pi]));
}

hipError_t fast_launch_single(const FastPlan& p, const LaunchArgs& a, const float* tab32, const void* a16,
                              int precision, int W) {
  const uint4* t = static_cast<const uint4*>(a16);
  const bool ws = p.ws;
  switch (precision) {
    case SF_FP32: return ws ? fast_launch_single_p0_w1(p, a, tab32, t, W) : fast_launch_single_p0_w0(p, a, tab32, t, W);
    case SF_BF16: return ws ? fast_launch_single_p1_w1(p, a, tab32, t, W) : fast_launch_single_p1_w0(p, a, tab32, t, W);
    case SF_FP16: return ws ? fast_launch_single_p2_w1(p, a, tab32, t, W) : fast_launch_single_p2_w0(p, a, tab32, t, W);
    default:
      g_fast_err = "precision not implemented in the MFMA kernels";
      return hipErrorNotSupported;
  }
}

}  // namespace sf
