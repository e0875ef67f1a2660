// Equality-only QP layer of the decoders (Sec. IV: the QP of eq. sf_form without its inequality
// rows, which has a closed form) and its reverse mode.
//
// xi_out = argmin 1/2 ||xi - xi_in||^2 subject to the boundary rows A xi = b of eq. boundary_con.
// Those rows touch only the three first and three last coefficients of each robot-axis (the
// Bernstein end conditions), and restricted to them A is the invertible 6 x 6 block whose inverse
// sf_setup stores as Bmap.  So the free coefficients pass through and the six pinned ones become
// Bmap b.  The kernels stream the coefficients (HBM-bound); the pinned values of a problem are
// formed once per workgroup in LDS, and an LDS table maps each position of a sample to its pinned
// value or to "pass".
#include "sf_eqqp.h"

#include <algorithm>
#include <mutex>

namespace sf {
namespace {

constexpr int kEqBlock = 256;

template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef float4 type; };
template <> struct Vec16<double> { typedef double2 type; };

// LDS per workgroup: pinned values [nD][6] (T) and the position table [nDm] (int).
template <typename T>
__device__ void eq_tables(const DevCfg& c, const T* __restrict__ Bmap, const T* __restrict__ bv, T* pin, int* tbl) {
  const int nD = c.n * c.D, m = c.m, nDm = nD * m;
  for (int q = threadIdx.x; q < nD * kNFix; q += kEqBlock) {
    const int row = q / kNFix, r = q - row * kNFix;
    T acc = T(0);
    for (int s = 0; s < kNFix; ++s) acc = fma(Bmap[r * kNFix + s], bv[row * kNFix + s], acc);
    pin[q] = acc;
  }
  for (int e = threadIdx.x; e < nDm; e += kEqBlock) {
    const int row = e / m, k = e - row * m;
    const int r = k < 3 ? k : (k >= m - 3 ? k - (m - kNFix) : -1);
    tbl[e] = r < 0 ? -1 : row * kNFix + r;
  }
}

// Forward: one workgroup per chunk of samples of one problem (grid-stride over the chunks).
template <typename T>
__global__ void __launch_bounds__(kEqBlock)
qp_equality_kernel(const DevCfg* __restrict__ cfgs, const T* __restrict__ tab, const DevProblem* __restrict__ probs,
                   const WorkItem* __restrict__ chunks, int n_chunks, const T* xin, const T* __restrict__ bvals,
                   T* xout) {
  extern __shared__ __align__(16) unsigned char eq_raw[];
  for (int it = blockIdx.x; it < n_chunks; it += gridDim.x) {
    const WorkItem w = chunks[it];
    const DevProblem pr = probs[w.problem];
    const DevCfg c = cfgs[pr.cfg];
    const int nDm = c.n * c.D * c.m;
    T* pin = reinterpret_cast<T*>(eq_raw);
    int* tbl = reinterpret_cast<int*>(pin + c.n * c.D * kNFix);
    eq_tables<T>(c, tab + c.off_Bmap, bvals + pr.bnd_off, pin, tbl);
    __syncthreads();
    const int64_t base = pr.coef_off + (int64_t)w.first * nDm;
    const int64_t total = (int64_t)w.count * nDm;
    constexpr int VW = 16 / sizeof(T);           // elements per 16-byte access
    const bool vec = (nDm % VW) == 0 && ((uintptr_t)(xin + base) % 16) == 0 && ((uintptr_t)(xout + base) % 16) == 0;
    if (vec) {
      // 16-byte accesses: VW consecutive positions of one sample per access
      typedef typename Vec16<T>::type V;
      const int nV = nDm / VW, stepV = kEqBlock % nV;
      int ev = threadIdx.x % nV;
      const V* xv = reinterpret_cast<const V*>(xin + base);
      V* ov = reinterpret_cast<V*>(xout + base);
      const int64_t nvt = total / VW;
      auto fix = [&](V& v, int at) {
        T* pv = reinterpret_cast<T*>(&v);
#pragma unroll
        for (int j = 0; j < VW; ++j) {
          const int p = tbl[at * VW + j];
          pv[j] = p < 0 ? pv[j] : pin[p < 0 ? 0 : p];
        }
      };
      int64_t idx = threadIdx.x;
      // four accesses in flight per thread: loads first, then the fix-ups and stores
      for (; idx + 3 * kEqBlock < nvt; idx += 4 * kEqBlock) {
        V v[4];
        int at[4];
        at[0] = ev;
#pragma unroll
        for (int u = 1; u < 4; ++u) {
          at[u] = at[u - 1] + stepV;
          if (at[u] >= nV) at[u] -= nV;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = xv[idx + u * kEqBlock];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          fix(v[u], at[u]);
          ov[idx + u * kEqBlock] = v[u];
        }
        ev = at[3] + stepV;
        if (ev >= nV) ev -= nV;
      }
      for (; idx < nvt; idx += kEqBlock) {
        V v = xv[idx];
        fix(v, ev);
        ov[idx] = v;
        ev += stepV;
        if (ev >= nV) ev -= nV;
      }
    } else {
      // position within the sample, advanced without a division per element
      const int step = kEqBlock % nDm;
      int e = threadIdx.x % nDm;
      for (int64_t idx = threadIdx.x; idx < total; idx += kEqBlock) {
        const T v = xin[base + idx];
        const int p = tbl[e];
        xout[base + idx] = p < 0 ? v : pin[p];
        e += step;
        if (e >= nDm) e -= nDm;
      }
    }
    __syncthreads();
  }
}

// Reverse mode, part 1: g_xi_in = g with the pinned positions zeroed (streamed like the forward).
template <typename T>
__global__ void __launch_bounds__(kEqBlock)
qp_equality_bwd_kernel(const DevCfg* __restrict__ cfgs, const DevProblem* __restrict__ probs,
                       const WorkItem* __restrict__ chunks, int n_chunks, const T* g, T* g_in) {
  extern __shared__ __align__(16) unsigned char eq_raw[];
  for (int it = blockIdx.x; it < n_chunks; it += gridDim.x) {
    const WorkItem w = chunks[it];
    const DevProblem pr = probs[w.problem];
    const DevCfg c = cfgs[pr.cfg];
    const int m = c.m, nDm = c.n * c.D * m;
    int* keep = reinterpret_cast<int*>(eq_raw);
    for (int e = threadIdx.x; e < nDm; e += kEqBlock) {
      const int k = e % m;
      keep[e] = (k < 3 || k >= m - 3) ? 0 : 1;
    }
    __syncthreads();
    const int64_t base = pr.coef_off + (int64_t)w.first * nDm;
    const int64_t total = (int64_t)w.count * nDm;
    constexpr int VW = 16 / sizeof(T);
    const bool vec = (nDm % VW) == 0 && ((uintptr_t)(g + base) % 16) == 0 && ((uintptr_t)(g_in + base) % 16) == 0;
    if (vec) {
      typedef typename Vec16<T>::type V;
      const int nV = nDm / VW, stepV = kEqBlock % nV;
      int ev = threadIdx.x % nV;
      const V* gv = reinterpret_cast<const V*>(g + base);
      V* ov = reinterpret_cast<V*>(g_in + base);
      for (int64_t idx = threadIdx.x; idx < total / VW; idx += kEqBlock) {
        V v = gv[idx];
        T* pv = reinterpret_cast<T*>(&v);
#pragma unroll
        for (int j = 0; j < VW; ++j) pv[j] = keep[ev * VW + j] ? pv[j] : T(0);
        ov[idx] = v;
        ev += stepV;
        if (ev >= nV) ev -= nV;
      }
    } else {
      const int step = kEqBlock % nDm;
      int e = threadIdx.x % nDm;
      for (int64_t idx = threadIdx.x; idx < total; idx += kEqBlock) {
        const T v = g[base + idx];
        g_in[base + idx] = keep[e] ? v : T(0);
        e += step;
        if (e >= nDm) e -= nDm;
      }
    }
    __syncthreads();
  }
}

// Reverse mode, part 2: per chunk and pinned slot (row, r), the sum over the chunk's samples of
// g at that slot (four accumulators, fixed order).  g_bvals is linear in these sums.
template <typename T>
__global__ void __launch_bounds__(kEqBlock)
qp_equality_part_kernel(const DevCfg* __restrict__ cfgs, const DevProblem* __restrict__ probs,
                        const WorkItem* __restrict__ chunks, int n_chunks, const T* __restrict__ g,
                        T* __restrict__ part, int part_stride) {
  for (int it = blockIdx.x; it < n_chunks; it += gridDim.x) {
    const WorkItem w = chunks[it];
    const DevProblem pr = probs[w.problem];
    const DevCfg c = cfgs[pr.cfg];
    const int m = c.m, nDm = c.n * c.D * m;
    const int64_t base = pr.coef_off + (int64_t)w.first * nDm;
    for (int q = threadIdx.x; q < c.n * c.D * kNFix; q += kEqBlock) {
      const int row = q / kNFix, r = q - row * kNFix;
      const T* gp = g + base + row * m + (r < 3 ? r : m - kNFix + r);
      T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
      int s = 0;
      for (; s + 4 <= w.count; s += 4) {
        a0 += gp[(int64_t)s * nDm];
        a1 += gp[(int64_t)(s + 1) * nDm];
        a2 += gp[(int64_t)(s + 2) * nDm];
        a3 += gp[(int64_t)(s + 3) * nDm];
      }
      for (; s < w.count; ++s) a0 += gp[(int64_t)s * nDm];
      part[(int64_t)it * part_stride + q] = (a0 + a1) + (a2 + a3);
    }
  }
}

// Reverse mode, part 3: one workgroup per (problem, robot-axis row); wave r sums slot (row, r)
// over the problem's chunks (lanes strided, then a fixed butterfly), and g_bvals[row][col] =
// sum_r Bmap[r][col] G[r].  Deterministic.
template <typename T>
__global__ void __launch_bounds__(64 * kNFix)
qp_equality_bsum_kernel(const DevCfg* __restrict__ cfgs, const T* __restrict__ tab,
                        const DevProblem* __restrict__ probs, int n_probs, const int* __restrict__ chunk_first,
                        const T* __restrict__ part, int part_stride, T* __restrict__ g_bvals) {
  __shared__ T G[kNFix];
  const int row = blockIdx.x;
  for (int p = blockIdx.y; p < n_probs; p += gridDim.y) {
    const DevProblem pr = probs[p];
    const DevCfg c = cfgs[pr.cfg];
    if (row >= c.n * c.D) continue;               // uniform over the workgroup
    const int lane = threadIdx.x & 63, r = threadIdx.x >> 6;
    T acc = T(0);
    for (int ch = chunk_first[p] + lane; ch < chunk_first[p + 1]; ch += 64)
      acc += part[(int64_t)ch * part_stride + row * kNFix + r];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) G[r] = acc;
    __syncthreads();
    if (threadIdx.x < kNFix) {
      const T* Bmap = tab + c.off_Bmap;
      T v = T(0);
      for (int q = 0; q < kNFix; ++q) v = fma(Bmap[q * kNFix + threadIdx.x], G[q], v);
      g_bvals[pr.bnd_off + row * kNFix + threadIdx.x] = v;
    }
    __syncthreads();
  }
}

// Allocation-free reverse mode: the tables of a batch, built on the device from its (config slot,
// sample count) list, in the layout and order of the host-built plan (get_plan / get_eq_chunks):
// problems packed in order, chunks of max(1, 32768 / (n D m)) samples.
__global__ void __launch_bounds__(256)
eq_noalloc_tables_kernel(const DevCfg* __restrict__ cfgs, EqNoAllocBatch b, DevProblem* __restrict__ probs,
                         WorkItem* __restrict__ chunks, int32_t* __restrict__ chunk_first) {
  __shared__ int32_t first[kEqNoAllocMaxProblems + 1], per[kEqNoAllocMaxProblems];
  if (threadIdx.x == 0) {
    int64_t coef = 0, bnd = 0, smp = 0;
    int32_t ch = 0;
    for (int p = 0; p < b.n_probs; ++p) {
      const DevCfg& c = cfgs[b.slot[p]];
      DevProblem pr;
      pr.cfg = b.slot[p];
      pr.count = b.count[p];
      pr.coef_off = coef;
      pr.bnd_off = bnd;
      pr.sample_base = smp;
      probs[p] = pr;
      per[p] = max(1, 32768 / (c.n * c.D * c.m));
      first[p] = ch;
      chunk_first[p] = ch;
      ch += (b.count[p] + per[p] - 1) / per[p];
      coef += (int64_t)b.count[p] * c.n * c.D * c.m;
      bnd += (int64_t)c.n * c.D * kNFix;
      smp += b.count[p];
    }
    first[b.n_probs] = ch;
    chunk_first[b.n_probs] = ch;
  }
  __syncthreads();
  for (int p = 0; p < b.n_probs; ++p)
    for (int q = threadIdx.x; q < first[p + 1] - first[p]; q += blockDim.x) {
      const int s = q * per[p];
      chunks[first[p] + q] = WorkItem{p, s, min(per[p], b.count[p] - s), 0};
    }
}

// The array itself.  Host code never uses its name as an address: hipGetSymbolAddress gives each
// device's copy, kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[kEqNoAllocBytes];

constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

}  // namespace

EqNoAllocLayout eq_noalloc_layout(int32_t n_probs, int32_t n_chunks, int32_t part_stride, size_t elem) {
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  EqNoAllocLayout l;
  l.probs = 0;
  l.chunks = up(l.probs + (size_t)n_probs * sizeof(DevProblem));
  l.chunk_first = up(l.chunks + (size_t)n_chunks * sizeof(WorkItem));
  l.part = up(l.chunk_first + (size_t)(n_probs + 1) * sizeof(int32_t));
  l.total = l.part + (size_t)n_chunks * part_stride * elem;
  return l;
}

hipError_t eq_noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

void* eq_noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

hipError_t launch_eq_noalloc_tables(const DevCfg* cfgs, const EqNoAllocBatch& b, void* base,
                                    const EqNoAllocLayout& lay, hipStream_t stream) {
  unsigned char* s = static_cast<unsigned char*>(base);
  hipLaunchKernelGGL(eq_noalloc_tables_kernel, dim3(1), dim3(256), 0, stream, cfgs, b,
                     reinterpret_cast<DevProblem*>(s + lay.probs), reinterpret_cast<WorkItem*>(s + lay.chunks),
                     reinterpret_cast<int32_t*>(s + lay.chunk_first));
  return hipGetLastError();
}

size_t qp_equality_lds_bytes(const DevCfg& c, size_t elem) {
  return (size_t)c.n * c.D * kNFix * elem + (size_t)c.n * c.D * c.m * sizeof(int);
}

template <typename T>
hipError_t launch_qp_equality(const EqArgs& a) {
  if (a.n_chunks == 0) return hipSuccess;
  const int grid = a.n_chunks;
  if (a.forward) {
    hipLaunchKernelGGL(qp_equality_kernel<T>, dim3(grid), dim3(kEqBlock), a.lds_bytes, a.stream, a.cfgs,
                       static_cast<const T*>(a.tab), a.probs, a.chunks, a.n_chunks, static_cast<const T*>(a.in),
                       static_cast<const T*>(a.bvals), static_cast<T*>(a.out));
    return hipGetLastError();
  }
  // the sums read g before g_in overwrites it (they may be the same array)
  if (a.g_bvals) {
    hipLaunchKernelGGL(qp_equality_part_kernel<T>, dim3(grid), dim3(kEqBlock), 0, a.stream, a.cfgs, a.probs,
                       a.chunks, a.n_chunks, static_cast<const T*>(a.in), static_cast<T*>(a.part), a.part_stride);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(qp_equality_bsum_kernel<T>, dim3(a.max_rows, std::min(a.n_probs, 65535)), dim3(64 * kNFix), 0,
                       a.stream, a.cfgs, static_cast<const T*>(a.tab), a.probs, a.n_probs, a.chunk_first,
                       static_cast<const T*>(a.part), a.part_stride, static_cast<T*>(a.g_bvals));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (a.out) {
    hipLaunchKernelGGL(qp_equality_bwd_kernel<T>, dim3(grid), dim3(kEqBlock), a.lds_bytes, a.stream, a.cfgs,
                       a.probs, a.chunks, a.n_chunks, static_cast<const T*>(a.in), static_cast<T*>(a.out));
    return hipGetLastError();
  }
  return hipSuccess;
}

template hipError_t launch_qp_equality<double>(const EqArgs&);
template hipError_t launch_qp_equality<float>(const EqArgs&);

}  // namespace sf
