// Small kernels: FP64 reduction of the absorbed-energy accumulators, point location and the
// Philox diagnostic.
#include "device.h"

using namespace rtd;

namespace {

// Sum the wavelength slots of each node (canonical order), optionally keep the
// per-(wavelength, node) values, and add the model total.
__global__ __launch_bounds__(256) void reduce_kernel(const ModelDev* __restrict__ models, int model,
                                                     const double* __restrict__ acc64,
                                                     int64_t slot_stride, int n_slots,
                                                     double* __restrict__ e_node,
                                                     double* __restrict__ e_lam_node,
                                                     double* __restrict__ e_total) {
  __shared__ double s_part[4];
  const ModelDev& m = models[model];
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double sum = 0.0;
  if (c < m.n_nodes) {
    const int64_t internal = m.base + (c < m.n_root ? c : c + (m.n_root_pad - m.n_root));
    for (int s = 0; s < n_slots; ++s) {
      const double v = acc64[s * slot_stride + internal];
      sum += v;
      if (e_lam_node) e_lam_node[m.lamnode_base + s * m.n_nodes + c] = v;
    }
    if (e_node) e_node[m.canon_base + c] = sum;
  }
  sum = wave_sum(sum);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += s_part[i];
    if (t != 0.0) unsafeAtomicAdd(e_total, t);
  }
}

__global__ void locate_kernel(const int32_t* __restrict__ child, const ModelDev* __restrict__ models,
                              int model, int64_t n, const double* __restrict__ xyz,
                              int32_t* __restrict__ lev_out, int64_t* __restrict__ node_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const ModelDev& m = models[model];
  const double P[3] = {xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]};
  int lev = -1;
  int32_t I[3];
  const int32_t node = locate_walk(dims_of(m), P, lev, I, ChildPlain{child});
  lev_out[i] = node < 0 ? -1 : lev;
  node_out[i] = node < 0 ? -1 : canon_of(m, node);
}

__global__ void philox_kernel(uint32_t k0, uint32_t k1, int64_t n, const uint32_t* __restrict__ ctr,
                              uint32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint4 r = philox(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1);
  out[4 * i] = r.x;
  out[4 * i + 1] = r.y;
  out[4 * i + 2] = r.z;
  out[4 * i + 3] = r.w;
}

__global__ void add_kernel(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                           double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] + b[i];
}

// Absorbed power balanced by the accelerated Lambda iteration (Sect. 3.1, Eq. 3) with a
// diagonal operator: lambda* = e_self / e_emit is the part of a cell's own emission it absorbs
// on its packets' first visit; E(T)(1 - lambda*) = A_stars + A_dust - e_self.
__global__ void ali_kernel(int64_t n, const double* __restrict__ a_stars, const double* __restrict__ a_dust,
                           const double* __restrict__ e_self, const double* __restrict__ e_emit,
                           double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double lam = e_emit[i] > 0.0 ? e_self[i] / e_emit[i] : 0.0;
  lam = lam < 1.0 - 1e-9 ? lam : 1.0 - 1e-9;
  out[i] = (a_stars[i] + a_dust[i] - e_self[i]) / (1.0 - lam);
}

// Mass-weighted mean relative temperature change over the leaves (Lambda-iteration stopping
// statistic): accumulates sum m |Tn - To| / To and sum m.
__global__ __launch_bounds__(256) void crit_kernel(const ModelDev* __restrict__ models, int model,
                                                   const int32_t* __restrict__ child,
                                                   const double* __restrict__ rho64,
                                                   const double* __restrict__ t_new,
                                                   const double* __restrict__ t_old,
                                                   double* __restrict__ out) {
  __shared__ double s_a[4], s_b[4];
  const ModelDev& m = models[model];
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double wa = 0.0, wb = 0.0;
  if (c < m.n_nodes) {
    const int64_t internal = m.base + (c < m.n_root ? c : c + (m.n_root_pad - m.n_root));
    if (child[internal] < 0) {
      int lev = 0;
      while (lev < m.nlev && c >= m.level_off[lev + 1]) ++lev;
      const double len = m.cell_cm * ldexp(1.0, -lev);
      const double mass = rho64[internal] * (len * len * len);
      wa = mass * (fabs(t_new[c] - t_old[c]) / t_old[c]);
      wb = mass;
    }
  }
  wa = wave_sum(wa);
  wb = wave_sum(wb);
  if ((threadIdx.x & 63) == 0) {
    s_a[threadIdx.x >> 6] = wa;
    s_b[threadIdx.x >> 6] = wb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, tb = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
      ta += s_a[i];
      tb += s_b[i];
    }
    if (tb != 0.0) {
      unsafeAtomicAdd(out, ta);
      unsafeAtomicAdd(out + 1, tb);
    }
  }
}

}  // namespace

hipError_t launch_ali_absorbed(int64_t n, const double* a_stars, const double* a_dust, const double* e_self,
                               const double* e_emit, double* out, hipStream_t s) {
  hipLaunchKernelGGL(ali_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, a_stars, a_dust, e_self,
                     e_emit, out);
  return hipGetLastError();
}

hipError_t launch_add(int64_t n, const double* a, const double* b, double* out, hipStream_t s) {
  hipLaunchKernelGGL(add_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, a, b, out);
  return hipGetLastError();
}

hipError_t launch_crit(const ModelDev* models, int model, int64_t n_nodes, const int32_t* child,
                       const double* rho64, const double* t_new, const double* t_old, double* out,
                       hipStream_t s) {
  hipLaunchKernelGGL(crit_kernel, dim3((unsigned)((n_nodes + 255) / 256)), dim3(256), 0, s, models,
                     model, child, rho64, t_new, t_old, out);
  return hipGetLastError();
}

hipError_t launch_reduce_model(const ModelDev* models_dev, int model, int64_t n_nodes,
                               const double* acc64, int64_t slot_stride,
                               int n_slots, double* e_node, double* e_lam_node, double* e_total,
                               hipStream_t s) {
  const int64_t grid = (n_nodes + 255) / 256;
  hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)grid), dim3(256), 0, s, models_dev, model, acc64, slot_stride, n_slots, e_node, e_lam_node, e_total);
  return hipGetLastError();
}

hipError_t launch_locate(const int32_t* child, const ModelDev* models, int model, int64_t n,
                         const double* xyz, int32_t* lev, int64_t* node, hipStream_t s) {
  const int64_t grid = (n + 255) / 256;
  hipLaunchKernelGGL(locate_kernel, dim3((unsigned)grid), dim3(256), 0, s, child, models, model, n,
                     xyz, lev, node);
  return hipGetLastError();
}

hipError_t launch_philox(uint32_t k0, uint32_t k1, int64_t n, const uint32_t* ctr, uint32_t* out,
                         hipStream_t s) {
  const int64_t grid = (n + 255) / 256;
  hipLaunchKernelGGL(philox_kernel, dim3((unsigned)grid), dim3(256), 0, s, k0, k1, n, ctr, out);
  return hipGetLastError();
}

// ---- small kernels of a captured iteration step (no memset or host copy inside a graph) ----
namespace {

__global__ void fill_u64_kernel(unsigned long long* __restrict__ a, int64_t n, unsigned long long v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

__global__ void copy_u64_kernel(const unsigned long long* __restrict__ a, unsigned long long* __restrict__ b,
                                int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

// The step's Philox key: the second word advances by one per step (key iteration n + 1).
__global__ void step_key_kernel(uint32_t* keys) {
  if (threadIdx.x == 0 && blockIdx.x == 0) keys[1] += 1u;
}

// What the host reads after a step: the stopping statistic (numerator, denominator), whether
// the sweeps drained, the step's crossings and its misplaced queue records (an invariant).
__global__ void step_report_kernel(const double* __restrict__ crit, const SweepState* __restrict__ st,
                                   const DevStats* __restrict__ stats, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  out[0] = crit[0];
  out[1] = crit[1];
  out[2] = st->done ? 1.0 : 0.0;
  out[3] = (double)stats->crossings;
  out[4] = (double)stats->misplaced;
}

}  // namespace

hipError_t launch_fill_u64(void* a, int64_t n_words, unsigned long long v, hipStream_t s) {
  if (n_words <= 0) return hipSuccess;
  const int64_t g = (n_words + 255) / 256;
  hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)(g < 4096 ? g : 4096)), dim3(256), 0, s,
                     static_cast<unsigned long long*>(a), n_words, v);
  return hipGetLastError();
}

hipError_t launch_copy_u64(const void* a, void* b, int64_t n_words, hipStream_t s) {
  if (n_words <= 0) return hipSuccess;
  const int64_t g = (n_words + 255) / 256;
  hipLaunchKernelGGL(copy_u64_kernel, dim3((unsigned)(g < 4096 ? g : 4096)), dim3(256), 0, s,
                     static_cast<const unsigned long long*>(a), static_cast<unsigned long long*>(b), n_words);
  return hipGetLastError();
}

hipError_t launch_step_key(uint32_t* keys, hipStream_t s) {
  hipLaunchKernelGGL(step_key_kernel, dim3(1), dim3(64), 0, s, keys);
  return hipGetLastError();
}

hipError_t launch_step_report(const double* crit, const SweepState* st, const DevStats* stats, double* out,
                              hipStream_t s) {
  hipLaunchKernelGGL(step_report_kernel, dim3(1), dim3(64), 0, s, crit, st, stats, out);
  return hipGetLastError();
}
