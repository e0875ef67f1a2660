// Host runtime of the safety filter: FP64 factorisation of the QP step, device tables,
// batch plans, argument checks and kernel launches behind the C ABI of swarmsf.h.
#include "swarmsf.h"
#include "sf_internal.h"
#include "sf_fast.h"
#include "sf_adjoint.h"
#include "sf_eqqp.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

namespace {

thread_local std::string g_err;

// Margin of the MFMA kernel's reusable pair lists, as a fraction of the safety semi-axes: a
// list built with it stays a superset of the colliding pairs until some robot has moved that
// far along an axis (then it is rebuilt).
constexpr double kPairSkin = 0.1;

sf_status fail(sf_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

sf_status hip_fail(hipError_t e, const char* what) {
  return fail(SF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// ------------------------------------------------------------------------------------
// FP64 host factorisation (eq. poly, eq. boundary_con, eq. xi_step)
// ------------------------------------------------------------------------------------

double binom(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

double bern(int N, int k, double tau) {
  if (N < 0 || k < 0 || k > N) return 0.0;
  return binom(N, k) * std::pow(tau, k) * std::pow(1.0 - tau, N - k);
}

// In-place Gauss-Jordan inverse with partial pivoting; returns false if singular.
bool invert(std::vector<double>& a, int n) {
  std::vector<double> inv(n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[i * n + i] = 1.0;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(a[r * n + col]) > std::fabs(a[piv * n + col])) piv = r;
    if (std::fabs(a[piv * n + col]) < 1e-300) return false;
    if (piv != col)
      for (int c = 0; c < n; ++c) {
        std::swap(a[piv * n + c], a[col * n + c]);
        std::swap(inv[piv * n + c], inv[col * n + c]);
      }
    const double d = a[col * n + col];
    for (int c = 0; c < n; ++c) {
      a[col * n + c] /= d;
      inv[col * n + c] /= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const double f = a[r * n + col];
      if (f == 0.0) continue;
      for (int c = 0; c < n; ++c) {
        a[r * n + c] -= f * a[col * n + c];
        inv[r * n + c] -= f * inv[col * n + c];
      }
    }
  }
  a.swap(inv);
  return true;
}

struct HostCfg {
  sf_config cfg;
  sf::DevCfg dev;            // offsets relative to this config's table
  std::vector<double> tab;
};

sf_status check_config(const sf_config& c) {
  if (c.n_robots < 2) return fail(SF_EINVAL, "n_robots must be >= 2");
  if (c.dims != 2 && c.dims != 3) return fail(SF_EINVAL, "dims must be 2 or 3");
  if (c.degree < 5) return fail(SF_EINVAL, "degree must be >= 5 (six boundary rows per robot-axis)");
  if (c.horizon < c.degree + 1) return fail(SF_EINVAL, "horizon must be >= degree + 1");
  if (!(c.t_final > 0)) return fail(SF_EINVAL, "t_final must be > 0");
  if (!(c.safety_a > 0) || !(c.safety_b > 0)) return fail(SF_EINVAL, "safety semi-axes must be > 0");
  if (!(c.rho_coll > 0)) return fail(SF_EINVAL, "rho_coll must be > 0");
  if (c.vmax > 0 && !(c.rho_vel > 0)) return fail(SF_EINVAL, "rho_vel must be > 0 when vmax > 0");
  if (c.amax > 0 && !(c.rho_acc > 0)) return fail(SF_EINVAL, "rho_acc must be > 0 when amax > 0");
  if (c.ws_a > 0 && c.dims == 3 && !(c.ws_b > 0)) return fail(SF_EINVAL, "ws_b must be > 0 when ws_a > 0");
  if (c.ws_a > 0 && !(c.rho_ws > 0)) return fail(SF_EINVAL, "rho_ws must be > 0 when ws_a > 0");
  if (c.ws_a > 0 && !(std::isfinite(c.ws_x) && std::isfinite(c.ws_y) && std::isfinite(c.ws_z)))
    return fail(SF_EINVAL, "workspace centre must be finite");
  if (c.n_robots > 64) return fail(SF_EUNSUPPORTED, "n_robots > 64 is not supported");
  if (c.degree > 30 || c.horizon > 4096) return fail(SF_EUNSUPPORTED, "degree > 30 or horizon > 4096");
  return SF_OK;
}

sf_status build_cfg(const sf_config& c, HostCfg& out) {
  sf_status st = check_config(c);
  if (st != SF_OK) return st;
  const int N = c.degree, m = N + 1, mf = m - sf::kNFix, H = c.horizon, n = c.n_robots;
  const double T = c.t_final;
  const bool vel = c.vmax > 0, acc = c.amax > 0, ws = c.ws_a > 0;
  std::vector<double> P(H * m), Pd(H * m), Pdd(H * m);
  for (int h = 0; h < H; ++h) {
    const double tau = (double)h / (H - 1);
    for (int k = 0; k < m; ++k) {
      P[h * m + k] = bern(N, k, tau);
      Pd[h * m + k] = (N / T) * (bern(N - 1, k - 1, tau) - bern(N - 1, k, tau));
      Pdd[h * m + k] = (N * (N - 1) / (T * T)) *
                       (bern(N - 2, k - 2, tau) - 2.0 * bern(N - 2, k - 1, tau) + bern(N - 2, k, tau));
    }
  }
  const int fix[sf::kNFix] = {0, 1, 2, m - 3, m - 2, m - 1};
  const double* rows[sf::kNFix] = {&P[0], &Pd[0], &Pdd[0], &P[(H - 1) * m], &Pd[(H - 1) * m], &Pdd[(H - 1) * m]};
  std::vector<double> Bmap(36);
  for (int r = 0; r < 6; ++r) {
    for (int k = 3; k < m - 3; ++k)
      if (rows[r][k] != 0.0) return fail(SF_EINVAL, "boundary rows touch free coefficients");
    for (int s = 0; s < 6; ++s) Bmap[r * 6 + s] = rows[r][fix[s]];
  }
  if (!invert(Bmap, 6)) return fail(SF_EINVAL, "boundary rows are singular");
  // Gram matrices of the constraint blocks
  std::vector<double> G(m * m, 0.0), Rm(m * m, 0.0);
  for (int k = 0; k < m; ++k)
    for (int l = 0; l < m; ++l) {
      double g = 0, rv = 0, ra = 0;
      for (int h = 0; h < H; ++h) {
        g += P[h * m + k] * P[h * m + l];
        rv += Pd[h * m + k] * Pd[h * m + l];
        ra += Pdd[h * m + k] * Pdd[h * m + l];
      }
      G[k * m + l] = g;
      // per-robot rows: velocity and acceleration bounds, and the workspace (F_w of eq. f_e)
      Rm[k * m + l] = (vel ? c.rho_vel * rv : 0.0) + (acc ? c.rho_acc * ra : 0.0) + (ws ? c.rho_ws * g : 0.0);
    }
  // Free-coefficient blocks of the KKT inverse: Z^T Q Z = J (x) (I + Rff) + (I - J) (x) (I + n rho Gff + Rff)
  std::vector<double> X0(mf * mf), X1(mf * mf), X01(mf * mf), Gfx(mf * 6), Rfx(mf * 6);
  for (int f = 0; f < mf; ++f)
    for (int g2 = 0; g2 < mf; ++g2) {
      const int k = 3 + f, l = 3 + g2;
      const double id = (f == g2) ? 1.0 : 0.0;
      X0[f * mf + g2] = id + Rm[k * m + l];
      X1[f * mf + g2] = id + n * c.rho_coll * G[k * m + l] + Rm[k * m + l];
    }
  if (mf > 0 && (!invert(X0, mf) || !invert(X1, mf))) return fail(SF_EINVAL, "QP block is singular");
  for (int q = 0; q < mf * mf; ++q) X01[q] = X0[q] - X1[q];
  for (int f = 0; f < mf; ++f)
    for (int r = 0; r < 6; ++r) {
      Gfx[f * 6 + r] = G[(3 + f) * m + fix[r]];
      Rfx[f * 6 + r] = Rm[(3 + f) * m + fix[r]];
    }
  sf::DevCfg& d = out.dev;
  std::memset(&d, 0, sizeof(d));
  d.n = n; d.D = c.dims; d.m = m; d.mf = mf; d.H = H; d.Np = n * (n - 1) / 2;
  d.vel_on = vel; d.acc_on = acc;
  d.a = c.safety_a; d.b = c.safety_b;
  d.inv_a2 = 1.0 / (c.safety_a * c.safety_a);
  d.inv_b2 = 1.0 / (c.safety_b * c.safety_b);
  d.vmax = vel ? c.vmax : 0.0; d.amax = acc ? c.amax : 0.0;
  d.rho_c = c.rho_coll; d.rho_v = vel ? c.rho_vel : 0.0; d.rho_a = acc ? c.rho_acc : 0.0;
  d.n_rho_c = n * c.rho_coll;
  d.ws_on = ws;
  if (ws) {
    const double wb = c.dims == 3 ? c.ws_b : c.ws_a;
    d.ws_a = c.ws_a;
    d.ws_ia2 = 1.0 / (c.ws_a * c.ws_a);
    d.ws_ib2 = 1.0 / (wb * wb);
    d.ws_c[0] = c.ws_x; d.ws_c[1] = c.ws_y; d.ws_c[2] = c.dims == 3 ? c.ws_z : 0.0;
    d.rho_w = c.rho_ws;
    d.ws_scale = c.rho_ws / c.rho_coll;
    const double wf[6] = {d.ws_c[0], d.ws_c[1], d.ws_c[2], d.ws_ia2, d.ws_ib2, d.ws_scale};
    for (int q = 0; q < 6; ++q) d.ws_f[q] = (float)wf[q];
  }
  d.lip_v = d.lip_a = 0.0;
  for (int h = 0; h < H; ++h) {
    double sv = 0.0, sa = 0.0;
    for (int k = 0; k < m; ++k) {
      sv += std::fabs(Pd[h * m + k]);
      sa += std::fabs(Pdd[h * m + k]);
    }
    d.lip_v = std::max(d.lip_v, sv);
    d.lip_a = std::max(d.lip_a, sa);
  }
  // round the bounds up so that the fp32 copies used on the device stay upper bounds
  d.lip_v *= 1.0 + 1e-6;
  d.lip_a *= 1.0 + 1e-6;
  d.skin = kPairSkin;
  std::vector<double>& t = out.tab;
  t.clear();
  d.off_basis = t.size();
  t.insert(t.end(), P.begin(), P.end());
  t.insert(t.end(), Pd.begin(), Pd.end());
  t.insert(t.end(), Pdd.begin(), Pdd.end());
  d.off_X1 = t.size(); t.insert(t.end(), X1.begin(), X1.end());
  d.off_X01 = t.size(); t.insert(t.end(), X01.begin(), X01.end());
  d.off_Bmap = t.size(); t.insert(t.end(), Bmap.begin(), Bmap.end());
  d.off_Gfx = t.size(); t.insert(t.end(), Gfx.begin(), Gfx.end());
  d.off_Rfx = t.size(); t.insert(t.end(), Rfx.begin(), Rfx.end());
  while (t.size() % 64) t.push_back(0.0);   // keep each config's table 512-byte aligned
  out.cfg = c;
  return SF_OK;
}

// ------------------------------------------------------------------------------------
// Batch plans: problem table and work items on the device, cached per batch.
// ------------------------------------------------------------------------------------

struct Plan {
  std::vector<int32_t> key;
  sf::DevProblem* d_probs = nullptr;
  sf::WorkItem* d_items = nullptr;
  int32_t n_items = 0;
  int64_t total_samples = 0, total_coef = 0, total_bnd = 0;
  std::vector<sf::DevProblem> probs;
  std::vector<int32_t> slots_used;
  std::vector<sf::WorkItem> items;      // host copy of the work items
  // work items of the problems the MFMA kernels cover (d_items_fast is d_items when that is all of
  // them) and of the others, which run on the generic kernel (none: d_items_gen is NULL)
  std::vector<sf::WorkItem> items_fast;
  sf::WorkItem* d_items_fast = nullptr;
  int32_t n_items_fast = 0;
  sf::WorkItem* d_items_gen = nullptr;
  int32_t n_items_gen = 0;
  sf::FastPlan fast;            // MFMA-path plan over items_fast (empty if there are none)
  sf::FastPlan fast_persistent; // persistent launch of a single-shape batch (built on request)
  // equality-only QP layer: sample chunks per problem (built on first use)
  sf::WorkItem* d_eq_chunks = nullptr;
  int32_t* d_eq_chunk_first = nullptr;
  int32_t n_eq_chunks = 0;
  struct GraphEntry {
    std::vector<uintptr_t> key;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<GraphEntry> graphs;       // captured launches, most recent first
};

}  // namespace

struct sf_handle_s {
  int device = 0;
  void* scratch = nullptr;       // adjoint recompute states, grown on demand
  size_t scratch_bytes = 0;
  void* eq_part = nullptr;       // per-chunk partial sums of the equality layer's reverse mode
  size_t eq_part_bytes = 0;
  std::vector<HostCfg> cfgs;
  sf::DevCfg* d_cfgs = nullptr;
  double* d_tab64 = nullptr;
  float* d_tab32 = nullptr;
  void* d_a16 = nullptr;         // 16-bit S1 basis operands of the MFMA kernels
  hipStream_t cap_stream = nullptr;   // stream used to capture launch graphs
  std::vector<Plan*> plans;
  std::mutex mu;
};

namespace {

void free_plan(Plan* p) {
  if (!p) return;
  for (auto& g : p->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (p->d_probs) (void)hipFree(p->d_probs);
  if (p->d_items_fast && p->d_items_fast != p->d_items) (void)hipFree(p->d_items_fast);
  if (p->d_items_gen) (void)hipFree(p->d_items_gen);
  if (p->d_items) (void)hipFree(p->d_items);
  if (p->d_eq_chunks) (void)hipFree(p->d_eq_chunks);
  if (p->d_eq_chunk_first) (void)hipFree(p->d_eq_chunk_first);
  sf::fast_plan_free(p->fast);
  sf::fast_plan_free(p->fast_persistent);
  delete p;
}

sf_status get_plan(sf_handle h, const sf_batch* batch, Plan** out) {
  if (!batch) return fail(SF_EINVAL, "batch is NULL");
  if (batch->n_problems < 1) return fail(SF_EINVAL, "batch has no problems");
  if (!batch->cfg_slot || !batch->sample_count) return fail(SF_EINVAL, "batch arrays are NULL");
  std::vector<int32_t> key(2 * (size_t)batch->n_problems);
  for (int p = 0; p < batch->n_problems; ++p) {
    const int32_t s = batch->cfg_slot[p], cnt = batch->sample_count[p];
    if (s < 0 || s >= (int)h->cfgs.size()) return fail(SF_EINVAL, "cfg_slot out of range");
    if (cnt < 1) return fail(SF_EINVAL, "sample_count must be >= 1");
    key[2 * p] = s;
    key[2 * p + 1] = cnt;
  }
  for (size_t i = 0; i < h->plans.size(); ++i)
    if (h->plans[i]->key == key) {
      Plan* p = h->plans[i];
      h->plans.erase(h->plans.begin() + i);
      h->plans.insert(h->plans.begin(), p);   // most recently used first
      *out = p;
      return SF_OK;
    }
  Plan* p = new Plan();
  p->key = key;
  std::vector<sf::WorkItem> items;
  std::vector<bool> used(h->cfgs.size(), false);
  int64_t coef = 0, bnd = 0, smp = 0;
  for (int q = 0; q < batch->n_problems; ++q) {
    const sf::DevCfg& c = h->cfgs[key[2 * q]].dev;
    sf::DevProblem pr;
    pr.cfg = key[2 * q];
    pr.count = key[2 * q + 1];
    pr.coef_off = coef;
    pr.bnd_off = bnd;
    pr.sample_base = smp;
    p->probs.push_back(pr);
    used[pr.cfg] = true;
    for (int s = 0; s < pr.count; ++s) items.push_back(sf::WorkItem{q, s, 1, 0});
    coef += (int64_t)pr.count * c.n * c.D * c.m;
    bnd += (int64_t)c.n * c.D * sf::kNFix;
    smp += pr.count;
  }
  for (size_t s = 0; s < used.size(); ++s)
    if (used[s]) p->slots_used.push_back((int32_t)s);
  if (items.size() > (size_t)INT32_MAX) {
    free_plan(p);
    return fail(SF_EUNSUPPORTED, "too many samples in one batch");
  }
  p->n_items = (int32_t)items.size();
  p->total_samples = smp;
  p->total_coef = coef;
  p->total_bnd = bnd;
  hipError_t e = hipMalloc(&p->d_probs, p->probs.size() * sizeof(sf::DevProblem));
  if (e == hipSuccess) e = hipMalloc(&p->d_items, items.size() * sizeof(sf::WorkItem));
  if (e == hipSuccess)
    e = hipMemcpy(p->d_probs, p->probs.data(), p->probs.size() * sizeof(sf::DevProblem), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(p->d_items, items.data(), items.size() * sizeof(sf::WorkItem), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_plan(p);
    return hip_fail(e, "plan upload");
  }
  std::vector<sf::DevCfg> cfgs;
  for (auto& hc : h->cfgs) cfgs.push_back(hc.dev);
  p->items = items;
  // split by kernel: problems the MFMA kernels cover, and the others (generic kernel)
  std::vector<sf::WorkItem> gen;
  for (const sf::WorkItem& w : items)
    (sf::fast_cfg_covered(cfgs[p->probs[w.problem].cfg]) ? p->items_fast : gen).push_back(w);
  p->n_items_fast = (int32_t)p->items_fast.size();
  p->n_items_gen = (int32_t)gen.size();
  if (gen.empty()) {
    p->d_items_fast = p->d_items;
  } else {
    e = hipMalloc(&p->d_items_gen, gen.size() * sizeof(sf::WorkItem));
    if (e == hipSuccess)
      e = hipMemcpy(p->d_items_gen, gen.data(), gen.size() * sizeof(sf::WorkItem), hipMemcpyHostToDevice);
    if (e == hipSuccess && !p->items_fast.empty()) {
      e = hipMalloc(&p->d_items_fast, p->items_fast.size() * sizeof(sf::WorkItem));
      if (e == hipSuccess)
        e = hipMemcpy(p->d_items_fast, p->items_fast.data(), p->items_fast.size() * sizeof(sf::WorkItem),
                      hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
      free_plan(p);
      return hip_fail(e, "plan upload");
    }
  }
  sf_status st = sf::fast_plan_build(cfgs, p->probs, p->items_fast, false, p->fast);
  if (st != SF_OK) {
    free_plan(p);
    return fail(st, "fast plan: " + sf::fast_last_error());
  }
  if (h->plans.size() >= 8) {
    free_plan(h->plans.back());
    h->plans.pop_back();
  }
  h->plans.insert(h->plans.begin(), p);
  *out = p;
  return SF_OK;
}

// Time tile of the generic kernels (one workgroup of kBlock threads per work item): the largest
// tile of at most 32 steps whose LDS plan fits 80 KB (a one-step tile may take up to 160 KB), unless
// a smaller one of at least 16 steps keeps more work items resident at once (more workgroups per CU:
// 16 robots x 1024 samples in fp32 run 75 ms with 32-step tiles, two workgroups per CU, and 46 ms with
// 16-step tiles, four per CU).  Smaller tiles than that cost more per sample than they gain.
sf_status pick_tile(sf_handle h, const Plan* p, size_t elem, size_t (*bytes)(const sf::DevCfg&, int, size_t),
                    int* tile, size_t* lds) {
  int maxH = 1;
  for (int32_t s : p->slots_used) maxH = std::max(maxH, h->cfgs[s].dev.H);
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess || ncu < 1)
    ncu = 256;
  int best = 0;
  size_t best_lds = 0;
  int64_t best_res = -1;
  for (int TT = std::min(32, maxH); TT >= 1; TT = (TT > 4 ? TT / 2 : TT - 1)) {
    size_t worst = 0;
    for (int32_t s : p->slots_used) worst = std::max(worst, bytes(h->cfgs[s].dev, TT, elem));
    if (!(worst <= 80 * 1024 || (TT == 1 && worst <= 160 * 1024))) continue;
    const int64_t per_cu = std::max<int64_t>(1, (int64_t)(160 * 1024) / (int64_t)std::max<size_t>(worst, 1));
    const int64_t res = std::min<int64_t>(p->n_items, per_cu * ncu);
    if (best == 0 || (TT >= std::min(16, maxH) && res > best_res)) {
      best = TT;
      best_lds = worst;
      best_res = res;
    }
    if (TT <= std::min(16, maxH)) break;
  }
  if (best == 0) return fail(SF_EUNSUPPORTED, "problem does not fit the LDS plan");
  *tile = best;
  *lds = best_lds;
  return SF_OK;
}

size_t generic_bytes(const sf::DevCfg& c, int tile, size_t elem) { return sf::generic_lds_bytes(c, tile, elem); }
size_t feas_bytes(const sf::DevCfg& c, int tile, size_t) { return sf::feasibility_lds_bytes(c, tile); }
size_t adj_bytes(const sf::DevCfg& c, int tile, size_t elem) { return sf::adjoint_lds_bytes(c, tile, elem); }

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

sf_status check_device(sf_handle h) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != h->device) return fail(SF_EINVAL, "current device differs from the handle's device");
  return SF_OK;
}

// ------------------------------------------------------------------------------------
// Autotuner of the persistent launch: times candidate grid sizes on the caller's batch and
// buffers, keeps the fastest per (device, batch, shapes, precision) in a JSON-lines cache.
// ------------------------------------------------------------------------------------

std::string tune_cache_path() {
  if (const char* e = std::getenv("SWARMSF_TUNE_CACHE")) return e;
  if (const char* home = std::getenv("HOME")) return std::string(home) + "/.cache/swarmsf_tune.jsonl";
  return "";
}

std::string tune_signature(sf_handle h, const Plan* p, int precision) {
  uint64_t f = 1469598103934665603ull;
  auto mix = [&](uint64_t v) {
    for (int i = 0; i < 8; ++i) {
      f ^= (v >> (8 * i)) & 0xff;
      f *= 1099511628211ull;
    }
  };
  for (int32_t v : p->key) mix((uint64_t)(uint32_t)v);
  for (int32_t s : p->slots_used) {
    const sf::DevCfg& c = h->cfgs[s].dev;
    mix(c.n); mix(c.m); mix(c.H); mix(c.D);
    if (c.ws_on) mix(0x7773);   // workspace instances are other kernels
  }
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) arch = prop.gcnArchName;
  char buf[160];
  std::snprintf(buf, sizeof(buf), "%s:p%d:%016llx", arch.c_str(), precision, (unsigned long long)f);
  return buf;
}

bool tune_lookup(const std::string& sig, int* waves, int* grid) {
  const std::string path = tune_cache_path();
  if (path.empty()) return false;
  FILE* fp = std::fopen(path.c_str(), "r");
  if (!fp) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof(line), fp)) {
    char key[256];
    int w = 0, g = 0;
    if (std::sscanf(line, "{\"key\": \"%255[^\"]\", \"waves\": %d, \"grid\": %d", key, &w, &g) == 3 &&
        sig == key && w >= 2 && w <= 4) {
      *waves = w;
      *grid = g;
      found = true;
    }
  }
  std::fclose(fp);
  return found;
}

void tune_store(const std::string& sig, int waves, int grid, double ms) {
  const std::string path = tune_cache_path();
  if (path.empty()) return;
  FILE* fp = std::fopen(path.c_str(), "a");
  if (!fp) return;
  std::fprintf(fp, "{\"key\": \"%s\", \"waves\": %d, \"grid\": %d, \"ms\": %.4f}\n", sig.c_str(), waves, grid, ms);
  std::fclose(fp);
}

sf_status autotune(sf_handle h, const Plan* p, sf::FastPlan& fp, const sf::LaunchArgs& a, int precision) {
  const int pi = precision & 3;
  if (fp.batched ? fp.tuned_wc[pi][0] > 0 : fp.tuned_w[pi] > 0) return SF_OK;
  // a single-shape plan is tuned as a whole; a persistent plan per robot-tile class (each class is its
  // own kernel with its own register budget, so each gets its own waves per workgroup and grid)
  const std::string base = tune_signature(h, p, precision) + (fp.batched ? ":persistent" : ":single");
  const int nsub = fp.batched ? fp.n_cls : 1;
  auto sig_of = [&](int sub) { return fp.batched ? base + ":c" + std::to_string(sub) : base; };
  int cw[2] = {0, 0}, cg[2] = {0, 0};
  bool cached = true;
  for (int sub = 0; sub < nsub; ++sub) cached = cached && tune_lookup(sig_of(sub), &cw[sub], &cg[sub]);
  if (cached) {
    if (fp.batched)
      for (int sub = 0; sub < nsub; ++sub) {
        fp.tuned_wc[pi][sub] = cw[sub];
        fp.tuned_gc[pi][sub] = cg[sub];
      }
    else
      fp.tuned_w[pi] = cw[0];
    return SF_OK;
  }
  // trial launches: single-shape plans are cheap, so they get longer trials, two warm-ups (the first
  // launches of a kernel also grow its scratch backing) and the best of three; persistent classes over
  // large ragged batches the best of two 30-iteration runs
  sf::LaunchArgs t = a;
  t.iters = std::max(1, std::min(a.iters, fp.batched ? 30 : 50));
  t.status_out = nullptr;   // trial launches read and write no status
  const int warm = fp.batched ? 1 : 2, reps = fp.batched ? 2 : 3;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return fail(SF_EDEVICE, "events");
  for (int sub = 0; sub < nsub; ++sub) {
    // candidates: waves per workgroup x (persistent only) workgroups in flight
    std::vector<std::pair<int, int>> cand;
    for (int W : {2, 3, 4}) {
      if (fp.ws && W > 3) continue;   // the workspace instances have 2 or 3 waves per workgroup
      if (!fp.batched) {
        cand.push_back({W, 0});
        continue;
      }
      std::vector<int> grids;
      for (int k = 1; k <= 6; ++k) grids.push_back(std::min(fp.ncu * k, fp.cls[sub].n_items));
      std::sort(grids.begin(), grids.end());
      grids.erase(std::unique(grids.begin(), grids.end()), grids.end());
      for (int g : grids) cand.push_back({W, g});
    }
    auto run = [&](const std::pair<int, int>& c) {
      if (!fp.batched) return sf::fast_launch_single(fp, t, h->d_tab32, h->d_a16, precision, c.first);
      int W2[2] = {2, 2}, G2[2] = {0, 0};
      W2[sub] = c.first;
      G2[sub] = c.second;
      return sf::fast_launch_batched(fp, t, h->d_tab32, h->d_a16, precision, G2, W2, 1 << sub);
    };
    std::pair<int, int> best = cand[0];
    float best_ms = 1e30f;
    for (const auto& c : cand) {
      hipError_t e = hipSuccess;
      for (int i = 0; i < warm && e == hipSuccess; ++i) e = run(c);
      float ms = 1e30f;
      for (int rep = 0; rep < reps && e == hipSuccess; ++rep) {
        e = hipEventRecord(e0, a.stream);
        if (e == hipSuccess) e = run(c);
        if (e == hipSuccess) e = hipEventRecord(e1, a.stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float one = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&one, e0, e1);
        ms = std::min(ms, one);
      }
      if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return hip_fail(e, "autotune");
      }
      if (ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
    if (fp.batched) {
      fp.tuned_wc[pi][sub] = best.first;
      fp.tuned_gc[pi][sub] = best.second;
    } else {
      fp.tuned_w[pi] = best.first;
    }
    tune_store(sig_of(sub), best.first, best.second, best_ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return SF_OK;
}

// Sample chunks of the equality-only QP layer: each problem's samples in runs of about 32K
// coefficients (one workgroup each), and the first chunk of every problem.
sf_status get_eq_chunks(sf_handle h, Plan* p) {
  if (p->d_eq_chunks) return SF_OK;
  std::vector<sf::WorkItem> ch;
  std::vector<int32_t> first;
  for (size_t q = 0; q < p->probs.size(); ++q) {
    const sf::DevProblem& pr = p->probs[q];
    const sf::DevCfg& c = h->cfgs[pr.cfg].dev;
    const int per = std::max(1, 32768 / (c.n * c.D * c.m));
    first.push_back((int32_t)ch.size());
    for (int s = 0; s < pr.count; s += per) ch.push_back(sf::WorkItem{(int32_t)q, s, std::min(per, pr.count - s), 0});
  }
  first.push_back((int32_t)ch.size());
  if (ch.size() > (size_t)INT32_MAX) return fail(SF_EUNSUPPORTED, "too many sample chunks");
  hipError_t e = hipMalloc(&p->d_eq_chunks, ch.size() * sizeof(sf::WorkItem));
  if (e == hipSuccess) e = hipMalloc(&p->d_eq_chunk_first, first.size() * sizeof(int32_t));
  if (e == hipSuccess)
    e = hipMemcpy(p->d_eq_chunks, ch.data(), ch.size() * sizeof(sf::WorkItem), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(p->d_eq_chunk_first, first.data(), first.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (p->d_eq_chunks) (void)hipFree(p->d_eq_chunks);
    if (p->d_eq_chunk_first) (void)hipFree(p->d_eq_chunk_first);
    p->d_eq_chunks = nullptr;
    p->d_eq_chunk_first = nullptr;
    return hip_fail(e, "equality layer chunk table");
  }
  p->n_eq_chunks = (int32_t)ch.size();
  return SF_OK;
}

// Reverse mode on the matrix cores (fp32; batches the MFMA forward kernels cover, up to 16 robots,
// no workspace rows).  Per checkpoint segment, last first: the forward MFMA kernel recomputes the
// segment's states from its checkpoint (with checkpoints every iteration into the scratch), the
// final-residual term is formed once from the last two states, and the reverse sweep carries the
// cotangents of (xi, lambda, xi_bar) to the segment's start.
sf_status adjoint_fast_path(sf_handle h, Plan* p, int32_t precision, const void* xi_bar, const void* bvals,
                            int32_t iters, const float* ckpt, int32_t ckpt_every, const void* g_xi_out,
                            const void* g_lam_out, const void* g_resid, const void* w_fpr, void* g_xi0, void* g_lam0,
                            void* g_xi_bar, void* stream) {
  const int64_t stride = p->total_coef;
  // final-residual term: one workgroup per (sample, time tile of kResidTile steps), per-tile partials
  constexpr int kResidTile = 16;
  int max_h = 1;
  size_t rlds = 0;
  for (int32_t sl : p->slots_used) {
    max_h = std::max(max_h, h->cfgs[sl].dev.H);
    rlds = std::max(rlds, sf::adjoint_resid_tile_lds_bytes(h->cfgs[sl].dev, kResidTile));
  }
  const int n_rtiles = g_resid ? (max_h + kResidTile - 1) / kResidTile : 0;
  // states, carries, pend, and the residual term's per-tile partials
  const size_t need = ((size_t)2 * (ckpt_every + 1) + 4 + 2 * (size_t)n_rtiles) * stride * sizeof(float);
  if (need > h->scratch_bytes) {
    if (h->scratch) (void)hipFree(h->scratch);
    h->scratch = nullptr;
    h->scratch_bytes = 0;
    if (hipMalloc(&h->scratch, need) != hipSuccess) return fail(SF_ENOMEM, "adjoint scratch allocation failed");
    h->scratch_bytes = need;
  }
  float* states = static_cast<float*>(h->scratch);
  float* carry = states + (size_t)2 * (ckpt_every + 1) * stride;
  float* pend = carry + 3 * stride;
  float* rpart = pend + stride;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  size_t lds = 0;
  for (int32_t sl : p->slots_used) lds = std::max(lds, sf::adjoint_fast_lds_bytes(h->cfgs[sl].dev));
  const int nseg = (iters + ckpt_every - 1) / ckpt_every;
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int s0 = seg * ckpt_every, len = std::min(ckpt_every, iters - s0);
    sf::LaunchArgs la{};
    la.cfgs = h->d_cfgs;
    la.probs = p->d_probs;
    la.items = p->d_items;
    la.n_items = p->n_items;
    la.xi_bar = xi_bar;
    la.bvals = bvals;
    la.xi0 = ckpt + (size_t)seg * 2 * stride;
    la.lam0 = ckpt + (size_t)seg * 2 * stride + stride;
    la.iters = len;
    la.xi_out = states + (size_t)len * 2 * stride;
    la.lam_out = states + (size_t)len * 2 * stride + stride;
    la.ckpt = states;
    la.ckpt_every = 1;
    la.ckpt_stride = stride;
    la.stream = s;
    hipError_t e = sf::fast_launch(p->fast, la, h->d_tab32, h->d_a16, precision);
    if (e != hipSuccess) return hip_fail(e, "sf_project_backward recompute");
    bool init = false;
    const float* pendp = nullptr;
    if (seg == nseg - 1) {
      if (g_resid) {
        sf::AdjointArgs ra{};
        ra.cfgs = h->d_cfgs;
        ra.tab = h->d_tab32;
        ra.probs = p->d_probs;
        ra.items = p->d_items;
        ra.n_items = p->n_items;
        ra.g_xi_out = g_xi_out;
        ra.g_lam_out = g_lam_out;
        ra.g_resid = g_resid;
        ra.stream = s;
        ra.tile = kResidTile;
        ra.lds_bytes = rlds;
        e = sf::launch_adjoint_resid_tiles(ra, states, stride, len - 1, rpart, n_rtiles, carry, pend);
        if (e != hipSuccess) return hip_fail(e, "sf_project_backward final-residual term");
        pendp = pend;
      } else {
        init = true;
      }
    }
    sf::AdjFastArgs f{};
    f.cfgs = h->d_cfgs;
    f.tab = h->d_tab32;
    f.a32 = h->d_a16;
    f.probs = p->d_probs;
    f.items = p->d_items;
    f.n_items = p->n_items;
    f.states = states;
    f.stride = stride;
    f.s0 = s0;
    f.len = len;
    f.iters = iters;
    f.w_fpr = static_cast<const float*>(w_fpr);
    f.g_xi_out = static_cast<const float*>(g_xi_out);
    f.g_lam_out = static_cast<const float*>(g_lam_out);
    f.init = init;
    f.carry = carry;
    f.pend = pendp;
    f.last = seg == 0;
    f.g_xi0 = static_cast<float*>(g_xi0);
    f.g_lam0 = static_cast<float*>(g_lam0);
    f.g_xi_bar = static_cast<float*>(g_xi_bar);
    f.lds_bytes = lds;
    f.stream = s;
    e = sf::launch_adjoint_fast(f, p->fast.KS);
    if (e != hipSuccess) return hip_fail(e, "sf_project_backward reverse sweep");
  }
  return SF_OK;
}

}  // namespace

// ------------------------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------------------------

extern "C" {

const char* sf_last_error(void) { return g_err.c_str(); }

sf_status sf_factor_table(const sf_config* cfg, double* out, int64_t capacity, int64_t* needed) {
  g_err.clear();
  if (!cfg || !needed) return fail(SF_EINVAL, "cfg/needed is NULL");
  HostCfg hc;
  sf_status st = build_cfg(*cfg, hc);
  if (st != SF_OK) return st;
  const int64_t header = 16;
  *needed = header + (int64_t)hc.tab.size();
  if (!out) return SF_OK;
  if (capacity < *needed) return fail(SF_EINVAL, "capacity too small");
  const sf::DevCfg& d = hc.dev;
  const double hdr[16] = {(double)d.m, (double)d.mf, (double)d.H, (double)d.n,
                          (double)d.off_basis, (double)d.off_X1, (double)d.off_X01, (double)d.off_Bmap,
                          (double)d.off_Gfx, (double)d.off_Rfx, 0, 0, 0, 0, 0, 0};
  std::memcpy(out, hdr, sizeof(hdr));
  std::memcpy(out + header, hc.tab.data(), hc.tab.size() * sizeof(double));
  return SF_OK;
}

sf_status sf_setup(const sf_config* cfgs, int32_t n_cfgs, sf_handle* out) {
  g_err.clear();
  if (!cfgs || !out || n_cfgs < 1) return fail(SF_EINVAL, "sf_setup: bad arguments");
  *out = nullptr;
  sf_handle h = new sf_handle_s();
  hipError_t e = hipGetDevice(&h->device);
  if (e != hipSuccess) {
    delete h;
    return hip_fail(e, "hipGetDevice");
  }
  std::vector<double> all;
  std::vector<sf::DevCfg> devs;
  for (int i = 0; i < n_cfgs; ++i) {
    HostCfg hc;
    sf_status st = build_cfg(cfgs[i], hc);
    if (st != SF_OK) {
      delete h;
      return fail(st, "config " + std::to_string(i) + ": " + g_err);
    }
    const int64_t base = all.size();
    sf::DevCfg d = hc.dev;
    d.off_basis += base; d.off_X1 += base; d.off_X01 += base;
    d.off_Bmap += base; d.off_Gfx += base; d.off_Rfx += base;
    all.insert(all.end(), hc.tab.begin(), hc.tab.end());
    hc.dev = d;
    devs.push_back(d);
    h->cfgs.push_back(std::move(hc));
  }
  std::vector<float> all32(all.begin(), all.end());
  // pre-split 16-bit basis operands (bf16 and fp16) of the MFMA kernels, 3D configs only
  std::vector<uint16_t> a16;
  for (size_t i = 0; i < devs.size(); ++i) {
    sf::DevCfg& d = devs[i];
    d.off_a16[0] = d.off_a16[1] = d.off_a32 = 0;
    if (d.D != 3 || d.m > 16) continue;
    {
      const int64_t e32 = sf::a32_entries(d);
      d.off_a32 = (int64_t)(a16.size() / 8);
      a16.resize(a16.size() + e32 * 8);
      sf::a32_fill(d, all.data() + d.off_basis, reinterpret_cast<float*>(a16.data() + d.off_a32 * 8));
    }
    const int64_t ent = sf::a16_entries(d);
    for (int pr = 0; pr < 2; ++pr) {
      d.off_a16[pr] = (int64_t)(a16.size() / 8);
      a16.resize(a16.size() + ent * 8);
      sf::a16_fill(d, all.data() + d.off_basis, pr == 0 ? SF_BF16 : SF_FP16,
                   a16.data() + d.off_a16[pr] * 8);
    }
    h->cfgs[i].dev.off_a16[0] = d.off_a16[0];
    h->cfgs[i].dev.off_a16[1] = d.off_a16[1];
    h->cfgs[i].dev.off_a32 = d.off_a32;
  }
  if (a16.empty()) a16.resize(8);
  e = hipMalloc(&h->d_cfgs, devs.size() * sizeof(sf::DevCfg));
  if (e == hipSuccess) e = hipMalloc(&h->d_tab64, all.size() * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&h->d_tab32, all32.size() * sizeof(float));
  if (e == hipSuccess) e = hipMemcpy(h->d_cfgs, devs.data(), devs.size() * sizeof(sf::DevCfg), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(h->d_tab64, all.data(), all.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(h->d_tab32, all32.data(), all32.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&h->d_a16, a16.size() * sizeof(uint16_t));
  if (e == hipSuccess) e = hipMemcpy(h->d_a16, a16.data(), a16.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    sf_destroy(h);
    return hip_fail(e, "sf_setup upload");
  }
  // device address of the allocation-free entry point's array on this device (once per device)
  e = sf::eq_noalloc_init(h->device);
  if (e != hipSuccess) {
    sf_destroy(h);
    return hip_fail(e, "sf_setup: hipGetSymbolAddress of the allocation-free scratch");
  }
  *out = h;
  return SF_OK;
}

void sf_destroy(sf_handle h) {
  if (!h) return;
  for (Plan* p : h->plans) free_plan(p);
  if (h->d_cfgs) (void)hipFree(h->d_cfgs);
  if (h->d_tab64) (void)hipFree(h->d_tab64);
  if (h->d_tab32) (void)hipFree(h->d_tab32);
  if (h->d_a16) (void)hipFree(h->d_a16);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->scratch) (void)hipFree(h->scratch);
  if (h->eq_part) (void)hipFree(h->eq_part);
  delete h;
}

sf_status sf_project(sf_handle h, const sf_batch* batch, int32_t precision, const void* xi_bar,
                     const void* bvals, const void* xi0, const void* lam0, int32_t iters, void* xi_out,
                     void* lam_out, void* resid_out, int32_t* status_out, int32_t flags, void* ckpt,
                     int32_t ckpt_every, void* stream) {
  g_err.clear();
  if (!h) return fail(SF_EINVAL, "handle is NULL");
  if (precision < SF_FP64 || precision > SF_FP16) return fail(SF_EINVAL, "unknown precision");
  if (!xi_bar || !bvals || !xi_out) return fail(SF_EINVAL, "xi_bar, bvals and xi_out are required");
  if (iters < 0) return fail(SF_EINVAL, "iters must be >= 0");
  const int32_t known = SF_RESID_HISTORY | SF_GENERIC_KERNEL | SF_USE_GRAPH | SF_AUTOTUNE | SF_PERSISTENT | SF_FP_RESIDUAL;
  if (flags & ~known) return fail(SF_EINVAL, "unknown flags");
  if ((flags & SF_FP_RESIDUAL) && (flags & SF_RESID_HISTORY))
    return fail(SF_EINVAL, "SF_FP_RESIDUAL and SF_RESID_HISTORY cannot be combined");
  if ((flags & SF_FP_RESIDUAL) && !resid_out) return fail(SF_EINVAL, "SF_FP_RESIDUAL needs resid_out");
  if (ckpt && ckpt_every < 1) return fail(SF_EINVAL, "ckpt_every must be >= 1 with a checkpoint buffer");
  const size_t elem = precision == SF_FP64 ? sizeof(double) : sizeof(float);
  const void* ptrs[] = {xi_bar, bvals, xi0, lam0, xi_out, lam_out, resid_out, ckpt};
  for (const void* q : ptrs)
    if (q && !aligned(q, elem)) return fail(SF_EINVAL, "misaligned array");
  if (status_out && !aligned(status_out, sizeof(int32_t))) return fail(SF_EINVAL, "misaligned status array");
  std::lock_guard<std::mutex> lock(h->mu);
  sf_status st = check_device(h);
  if (st != SF_OK) return st;
  Plan* p = nullptr;
  st = get_plan(h, batch, &p);
  if (st != SF_OK) return st;
  sf::LaunchArgs a{};
  a.cfgs = h->d_cfgs;
  a.probs = p->d_probs;
  a.items = p->d_items;
  a.n_items = p->n_items;
  a.xi_bar = xi_bar; a.bvals = bvals; a.xi0 = xi0; a.lam0 = lam0; a.iters = iters;
  a.xi_out = xi_out; a.lam_out = lam_out; a.resid_out = resid_out; a.status_out = status_out;
  a.flags = flags & (SF_RESID_HISTORY | SF_FP_RESIDUAL);
  a.ckpt = ckpt; a.ckpt_every = ckpt ? ckpt_every : 1; a.ckpt_stride = p->total_coef;
  a.stream = static_cast<hipStream_t>(stream);

  // choose the kernel path
  sf::FastPlan* fp = nullptr;
  if (precision != SF_FP64 && p->fast.ok && !(flags & (SF_RESID_HISTORY | SF_GENERIC_KERNEL))) {
    fp = &p->fast;
    if ((flags & SF_PERSISTENT) && !p->fast.batched) {
      if (!p->fast_persistent.ok) {
        std::vector<sf::DevCfg> cfgs;
        for (auto& hc : h->cfgs) cfgs.push_back(hc.dev);
        st = sf::fast_plan_build(cfgs, p->probs, p->items_fast, true, p->fast_persistent);
        if (st != SF_OK) return fail(st, "persistent plan: " + sf::fast_last_error());
      }
      if (p->fast_persistent.ok) fp = &p->fast_persistent;
    }
  }
  if (precision > SF_FP32 && !fp && (flags & (SF_RESID_HISTORY | SF_GENERIC_KERNEL)))
    return fail(SF_EUNSUPPORTED, "the MFMA precisions cannot be combined with SF_RESID_HISTORY or SF_GENERIC_KERNEL");
  // the generic kernel takes every work item without an MFMA plan, else the uncovered ones (if any)
  const bool gen_part = !fp || p->n_items_gen > 0;
  if (gen_part) {
    st = pick_tile(h, p, elem, generic_bytes, &a.tile, &a.lds_bytes);
    if (st != SF_OK) return st;
  }
  if (fp && (flags & SF_AUTOTUNE)) {
    sf::LaunchArgs af = a;
    af.items = p->d_items_fast;
    af.n_items = p->n_items_fast;
    st = autotune(h, p, *fp, af, precision);
    if (st != SF_OK) return st;
  }
  auto solve = [&](const sf::LaunchArgs& b0) -> hipError_t {
    sf::LaunchArgs b = b0;
    if (fp) {
      b.items = p->d_items_fast;
      b.n_items = p->n_items_fast;
      const hipError_t fe = sf::fast_launch(*fp, b, h->d_tab32, h->d_a16, precision);
      if (fe != hipSuccess || p->n_items_gen == 0) return fe;
      b.items = p->d_items_gen;   // the problems the MFMA kernels do not cover: generic kernel, FP32
      b.n_items = p->n_items_gen;
    }
    if (precision == SF_FP64) {
      b.tab = h->d_tab64;
      return sf::launch_generic_project<double>(b);
    }
    b.tab = h->d_tab32;
    return sf::launch_generic_project<float>(b);
  };
  // with status_out: input check before the solve, finiteness of the outputs after it
  auto launch = [&](hipStream_t s) -> hipError_t {
    sf::LaunchArgs b = a;
    b.stream = s;
    hipError_t le = hipSuccess;
    if (status_out) le = sf::launch_status_input(b, precision == SF_FP64);
    if (le == hipSuccess) le = solve(b);
    if (le == hipSuccess && status_out) le = sf::launch_status_output(b, precision == SF_FP64);
    return le;
  };
  hipError_t e;
  if (flags & SF_USE_GRAPH) {
    std::vector<uintptr_t> key = {(uintptr_t)precision, (uintptr_t)flags, (uintptr_t)iters, (uintptr_t)a.ckpt_every,
                                  (uintptr_t)fp, (uintptr_t)(fp ? fp->tuned_w[precision & 3] : 0),
                                  (uintptr_t)(fp ? fp->tuned_wc[precision & 3][0] : 0),
                                  (uintptr_t)(fp ? fp->tuned_wc[precision & 3][1] : 0),
                                  (uintptr_t)(fp ? fp->tuned_gc[precision & 3][0] : 0),
                                  (uintptr_t)(fp ? fp->tuned_gc[precision & 3][1] : 0),
                                  (uintptr_t)xi_bar, (uintptr_t)bvals, (uintptr_t)xi0, (uintptr_t)lam0,
                                  (uintptr_t)xi_out, (uintptr_t)lam_out, (uintptr_t)resid_out,
                                  (uintptr_t)status_out, (uintptr_t)ckpt};
    hipGraphExec_t exec = nullptr;
    for (auto& g : p->graphs)
      if (g.key == key) exec = g.exec;
    if (!exec) {
      if (!h->cap_stream) {
        e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "capture stream");
      }
      e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeRelaxed);
      if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
      const hipError_t le = launch(h->cap_stream);
      hipGraph_t graph = nullptr;
      e = hipStreamEndCapture(h->cap_stream, &graph);
      if (le != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(le, "sf_project launch (capture)");
      }
      if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
      if (p->graphs.size() >= 4) {
        (void)hipGraphExecDestroy(p->graphs.back().exec);
        p->graphs.pop_back();
      }
      p->graphs.insert(p->graphs.begin(), Plan::GraphEntry{key, exec});
    }
    e = hipGraphLaunch(exec, a.stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return SF_OK;
  }
  e = launch(a.stream);
  if (e != hipSuccess) return hip_fail(e, "sf_project launch");
  return SF_OK;
}

sf_status sf_project_backward(sf_handle h, const sf_batch* batch, int32_t precision, const void* xi_bar,
                              const void* bvals, int32_t iters, const void* ckpt, int32_t ckpt_every,
                              const void* g_xi_out, const void* g_lam_out, const void* g_resid,
                              const void* w_fpr, void* g_xi0, void* g_lam0, void* g_xi_bar, void* stream) {
  g_err.clear();
  if (!h) return fail(SF_EINVAL, "handle is NULL");
  if (precision < SF_FP64 || precision > SF_FP16) return fail(SF_EINVAL, "unknown precision");
  if (!xi_bar || !bvals || !ckpt) return fail(SF_EINVAL, "xi_bar, bvals and ckpt are required");
  if (iters < 0 || ckpt_every < 1) return fail(SF_EINVAL, "iters must be >= 0 and ckpt_every >= 1");
  const size_t elem = precision == SF_FP64 ? sizeof(double) : sizeof(float);
  const void* ptrs[] = {xi_bar, bvals, ckpt, g_xi_out, g_lam_out, g_resid, w_fpr, g_xi0, g_lam0, g_xi_bar};
  for (const void* q : ptrs)
    if (q && !aligned(q, elem)) return fail(SF_EINVAL, "misaligned array");
  std::lock_guard<std::mutex> lock(h->mu);
  sf_status st = check_device(h);
  if (st != SF_OK) return st;
  Plan* p = nullptr;
  st = get_plan(h, batch, &p);
  if (st != SF_OK) return st;
  int64_t max_ndm = 0;
  bool fast = precision != SF_FP64 && iters > 0 && p->fast.ok && p->n_items_gen == 0 && !(p->fast.ws);
  for (int32_t s : p->slots_used) {
    const sf::DevCfg& c = h->cfgs[s].dev;
    max_ndm = std::max<int64_t>(max_ndm, (int64_t)c.n * c.D * c.m);
    fast = fast && sf::adjoint_fast_supported(c);
  }
  if (fast) return adjoint_fast_path(h, p, precision, xi_bar, bvals, iters, static_cast<const float*>(ckpt), ckpt_every,
                                     g_xi_out, g_lam_out, g_resid, w_fpr, g_xi0, g_lam0, g_xi_bar, stream);
  sf::AdjointArgs a{};
  a.state_stride = (int64_t)2 * (ckpt_every + 1) * max_ndm;   // xi and lambda states of a segment
  const size_t need = (size_t)p->n_items * a.state_stride * elem;
  if (need > h->scratch_bytes) {
    if (h->scratch) (void)hipFree(h->scratch);
    h->scratch = nullptr;
    h->scratch_bytes = 0;
    hipError_t e = hipMalloc(&h->scratch, need);
    if (e != hipSuccess) return fail(SF_ENOMEM, "adjoint scratch allocation failed");
    h->scratch_bytes = need;
  }
  a.cfgs = h->d_cfgs;
  a.probs = p->d_probs;
  a.items = p->d_items;
  a.n_items = p->n_items;
  a.xi_bar = xi_bar; a.bvals = bvals; a.iters = iters; a.ckpt = ckpt; a.ckpt_every = ckpt_every;
  a.ckpt_stride = p->total_coef;
  a.g_xi_out = g_xi_out; a.g_lam_out = g_lam_out; a.g_resid = g_resid; a.w_fpr = w_fpr;
  a.g_xi0 = g_xi0; a.g_lam0 = g_lam0; a.g_xi_bar = g_xi_bar;
  a.states = h->scratch;
  a.stream = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (precision == SF_FP64) {
    a.tab = h->d_tab64;
    st = pick_tile(h, p, sizeof(double), adj_bytes, &a.tile, &a.lds_bytes);
    if (st != SF_OK) return st;
    e = sf::launch_adjoint<double>(a);
  } else {
    a.tab = h->d_tab32;
    st = pick_tile(h, p, sizeof(float), adj_bytes, &a.tile, &a.lds_bytes);
    if (st != SF_OK) return st;
    e = sf::launch_adjoint<float>(a);
  }
  if (e != hipSuccess) return hip_fail(e, "sf_project_backward launch");
  return SF_OK;
}

sf_status sf_feasibility(sf_handle h, const sf_batch* batch, int32_t precision, const void* xi,
                         const void* bvals, void* viol_out, void* stream) {
  g_err.clear();
  if (!h) return fail(SF_EINVAL, "handle is NULL");
  if (!xi || !bvals || !viol_out) return fail(SF_EINVAL, "xi, bvals and viol_out are required");
  if (precision < SF_FP64 || precision > SF_FP16) return fail(SF_EINVAL, "unknown precision");
  const size_t elem = precision == SF_FP64 ? sizeof(double) : sizeof(float);
  if (!aligned(xi, elem) || !aligned(bvals, elem) || !aligned(viol_out, sizeof(double)))
    return fail(SF_EINVAL, "misaligned array");
  std::lock_guard<std::mutex> lock(h->mu);
  sf_status st = check_device(h);
  if (st != SF_OK) return st;
  Plan* p = nullptr;
  st = get_plan(h, batch, &p);
  if (st != SF_OK) return st;
  int tile = 0;
  size_t lds = 0;
  st = pick_tile(h, p, sizeof(double), feas_bytes, &tile, &lds);
  if (st != SF_OK) return st;
  hipError_t e = sf::launch_feasibility(h->d_cfgs, h->d_tab64, p->d_probs, p->d_items, p->n_items, xi,
                                        precision == SF_FP64, bvals, static_cast<double*>(viol_out), tile, lds,
                                        static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "sf_feasibility launch");
  return SF_OK;
}

sf_status sf_qp_equality(sf_handle h, const sf_batch* batch, int32_t precision, const void* xi_in,
                         const void* bvals, void* xi_out, void* stream) {
  g_err.clear();
  if (!h) return fail(SF_EINVAL, "handle is NULL");
  if (!xi_in || !bvals || !xi_out) return fail(SF_EINVAL, "xi_in, bvals and xi_out are required");
  if (precision < SF_FP64 || precision > SF_FP16) return fail(SF_EINVAL, "unknown precision");
  const size_t elem = precision == SF_FP64 ? sizeof(double) : sizeof(float);
  if (!aligned(xi_in, elem) || !aligned(bvals, elem) || !aligned(xi_out, elem))
    return fail(SF_EINVAL, "misaligned array");
  std::lock_guard<std::mutex> lock(h->mu);
  sf_status st = check_device(h);
  if (st != SF_OK) return st;
  Plan* p = nullptr;
  st = get_plan(h, batch, &p);
  if (st == SF_OK) st = get_eq_chunks(h, p);
  if (st != SF_OK) return st;
  sf::EqArgs a{};
  a.cfgs = h->d_cfgs;
  a.probs = p->d_probs;
  a.n_probs = (int32_t)p->probs.size();
  a.chunks = p->d_eq_chunks;
  a.n_chunks = p->n_eq_chunks;
  a.forward = true;
  a.in = xi_in;
  a.bvals = bvals;
  a.out = xi_out;
  for (int32_t s : p->slots_used) a.lds_bytes = std::max(a.lds_bytes, sf::qp_equality_lds_bytes(h->cfgs[s].dev, elem));
  a.stream = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (precision == SF_FP64) {
    a.tab = h->d_tab64;
    e = sf::launch_qp_equality<double>(a);
  } else {
    a.tab = h->d_tab32;
    e = sf::launch_qp_equality<float>(a);
  }
  if (e != hipSuccess) return hip_fail(e, "sf_qp_equality launch");
  return SF_OK;
}

sf_status sf_qp_equality_backward(sf_handle h, const sf_batch* batch, int32_t precision, const void* g_out,
                                  void* g_xi_in, void* g_bvals, void* stream) {
  g_err.clear();
  if (!h) return fail(SF_EINVAL, "handle is NULL");
  if (!g_out) return fail(SF_EINVAL, "g_out is required");
  if (precision < SF_FP64 || precision > SF_FP16) return fail(SF_EINVAL, "unknown precision");
  const size_t elem = precision == SF_FP64 ? sizeof(double) : sizeof(float);
  if (!aligned(g_out, elem) || (g_xi_in && !aligned(g_xi_in, elem)) || (g_bvals && !aligned(g_bvals, elem)))
    return fail(SF_EINVAL, "misaligned array");
  if (!g_xi_in && !g_bvals) return SF_OK;
  std::lock_guard<std::mutex> lock(h->mu);
  sf_status st = check_device(h);
  if (st != SF_OK) return st;
  Plan* p = nullptr;
  st = get_plan(h, batch, &p);
  if (st == SF_OK) st = get_eq_chunks(h, p);
  if (st != SF_OK) return st;
  int32_t stride = 0;
  for (int32_t s : p->slots_used) stride = std::max(stride, h->cfgs[s].dev.n * h->cfgs[s].dev.D * sf::kNFix);
  if (g_bvals) {
    const size_t need = (size_t)p->n_eq_chunks * stride * elem;
    if (need > h->eq_part_bytes) {
      if (h->eq_part) (void)hipFree(h->eq_part);
      h->eq_part = nullptr;
      h->eq_part_bytes = 0;
      if (hipMalloc(&h->eq_part, need) != hipSuccess) return fail(SF_ENOMEM, "equality layer scratch allocation failed");
      h->eq_part_bytes = need;
    }
  }
  sf::EqArgs a{};
  a.cfgs = h->d_cfgs;
  a.probs = p->d_probs;
  a.n_probs = (int32_t)p->probs.size();
  a.chunks = p->d_eq_chunks;
  a.n_chunks = p->n_eq_chunks;
  a.chunk_first = p->d_eq_chunk_first;
  a.forward = false;
  a.in = g_out;
  a.out = g_xi_in;
  a.part = g_bvals ? h->eq_part : nullptr;
  a.part_stride = stride;
  a.max_rows = stride / sf::kNFix;
  a.g_bvals = g_bvals;
  for (int32_t s : p->slots_used) a.lds_bytes = std::max(a.lds_bytes, sf::qp_equality_lds_bytes(h->cfgs[s].dev, elem));
  a.stream = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (precision == SF_FP64) {
    a.tab = h->d_tab64;
    e = sf::launch_qp_equality<double>(a);
  } else {
    a.tab = h->d_tab32;
    e = sf::launch_qp_equality<float>(a);
  }
  if (e != hipSuccess) return hip_fail(e, "sf_qp_equality_backward launch");
  return SF_OK;
}

sf_status sf_qp_equality_backward_noalloc(sf_handle h, const sf_batch* batch, int32_t precision, const void* g_out,
                                          void* g_xi_in, void* g_bvals, void* stream) {
  g_err.clear();
  if (!h) return fail(SF_EINVAL, "handle is NULL");
  if (!g_out) return fail(SF_EINVAL, "g_out is required");
  if (precision < SF_FP64 || precision > SF_FP16) return fail(SF_EINVAL, "unknown precision");
  const size_t elem = precision == SF_FP64 ? sizeof(double) : sizeof(float);
  if (!aligned(g_out, elem) || (g_xi_in && !aligned(g_xi_in, elem)) || (g_bvals && !aligned(g_bvals, elem)))
    return fail(SF_EINVAL, "misaligned array");
  if (!batch) return fail(SF_EINVAL, "batch is NULL");
  if (batch->n_problems < 1) return fail(SF_EINVAL, "batch has no problems");
  if (!batch->cfg_slot || !batch->sample_count) return fail(SF_EINVAL, "batch arrays are NULL");
  if (batch->n_problems > sf::kEqNoAllocMaxProblems)
    return fail(SF_EUNSUPPORTED, "sf_qp_equality_backward_noalloc takes at most " +
                                     std::to_string(sf::kEqNoAllocMaxProblems) + " problems per call");
  if (!g_xi_in && !g_bvals) return SF_OK;
  std::lock_guard<std::mutex> lock(h->mu);
  sf_status st = check_device(h);
  if (st != SF_OK) return st;
  // the batch's sizes, chunk count and the most LDS any of its problems needs, without a plan
  // (building one allocates device memory)
  sf::EqNoAllocBatch b{};
  b.n_probs = batch->n_problems;
  int64_t n_chunks = 0;
  int32_t stride = 0;
  size_t lds = 0;
  for (int p = 0; p < batch->n_problems; ++p) {
    const int32_t slot = batch->cfg_slot[p], cnt = batch->sample_count[p];
    if (slot < 0 || slot >= (int)h->cfgs.size()) return fail(SF_EINVAL, "cfg_slot out of range");
    if (cnt < 1) return fail(SF_EINVAL, "sample_count must be >= 1");
    const sf::DevCfg& c = h->cfgs[slot].dev;
    const int per = std::max(1, 32768 / (c.n * c.D * c.m));
    n_chunks += (cnt + per - 1) / per;
    stride = std::max(stride, c.n * c.D * sf::kNFix);
    lds = std::max(lds, sf::qp_equality_lds_bytes(c, elem));
    b.slot[p] = slot;
    b.count[p] = cnt;
  }
  const sf::EqNoAllocLayout lay =
      sf::eq_noalloc_layout(b.n_probs, (int32_t)std::min<int64_t>(n_chunks, INT32_MAX), stride, elem);
  if (n_chunks > INT32_MAX || lay.total > sf::kEqNoAllocBytes)
    return fail(SF_EUNSUPPORTED, "batch needs " + std::to_string(lay.total) + " bytes of tables and partial sums; "
                                 "the allocation-free scratch holds " + std::to_string(sf::kEqNoAllocBytes));
  unsigned char* base = static_cast<unsigned char*>(sf::eq_noalloc_scratch(h->device));
  if (!base) return fail(SF_EDEVICE, "allocation-free scratch was not set up on this device");
  const hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = sf::launch_eq_noalloc_tables(h->d_cfgs, b, base, lay, s);
  if (e != hipSuccess) return hip_fail(e, "sf_qp_equality_backward_noalloc tables");
  sf::EqArgs a{};
  a.cfgs = h->d_cfgs;
  a.probs = reinterpret_cast<const sf::DevProblem*>(base + lay.probs);
  a.n_probs = b.n_probs;
  a.chunks = reinterpret_cast<const sf::WorkItem*>(base + lay.chunks);
  a.n_chunks = (int32_t)n_chunks;
  a.chunk_first = reinterpret_cast<const int32_t*>(base + lay.chunk_first);
  a.forward = false;
  a.in = g_out;
  a.out = g_xi_in;
  a.part = g_bvals ? base + lay.part : nullptr;
  a.part_stride = stride;
  a.max_rows = stride / sf::kNFix;
  a.g_bvals = g_bvals;
  a.lds_bytes = lds;
  a.stream = s;
  if (precision == SF_FP64) {
    a.tab = h->d_tab64;
    e = sf::launch_qp_equality<double>(a);
  } else {
    a.tab = h->d_tab32;
    e = sf::launch_qp_equality<float>(a);
  }
  if (e != hipSuccess) return hip_fail(e, "sf_qp_equality_backward_noalloc launch");
  return SF_OK;
}

}  // extern "C"
