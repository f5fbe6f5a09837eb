// Dust model f(J) of the paper's Sect. 3.1 (one grain component at its equilibrium
// temperature, Sect. 4) and the per-leaf dust-emission luminosities used as a source.
#include "device.h"
#include "subiter.h"

using namespace rtd;

namespace {

constexpr double kK = 1.380649e-16;  // Boltzmann constant, erg/K

// sum_i kappa_abs_i B_i(T) dnu_i and its T derivative.
__device__ __forceinline__ void planck_sum(const LamConst* __restrict__ lc, int nl, double t,
                                           double& s, double& ds) {
  s = 0.0;
  ds = 0.0;
  const double kt = kK * t;
  for (int i = 0; i < nl; ++i) {
    const double x = lc[i].hnu / kt;
    const double em = expm1(x);
    const double b = lc[i].pre / em;
    const double kabs = (1.0 - lc[i].alb) * lc[i].kext;
    s += kabs * b * lc[i].dnu;
    if (em < INFINITY) ds += kabs * (b * x * ((em + 1.0) / em) / t) * lc[i].dnu;
  }
}

// Inverse table of the emission per unit mass, shared by every leaf of one solve: with
// S(T) = sum kappa_abs B(T) dnu, tab = {S(t_min), S(t_max), y0 = ln S(t_min), dy} followed by n
// pairs (u_i, du/dy at u_i), where u_i = ln T solves ln S = y0 + i dy (the same safeguarded
// Newton as the leaves, from a linear guess).  dy is left non-positive when S is not
// increasing and positive over [t_min, t_max]; the leaves then start from their linear guess.
__global__ __launch_bounds__(256) void planck_table_kernel(const LamConst* __restrict__ lc, int nl, double t_min,
                                                           double t_max, int n, double* __restrict__ tab) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double s0, d0, s1, d1;
  planck_sum(lc, nl, t_min, s0, d0);
  planck_sum(lc, nl, t_max, s1, d1);
  const bool ok = s0 > 0.0 && s1 > s0 && s1 < INFINITY;
  const double y0 = ok ? log(s0) : 0.0, y1 = ok ? log(s1) : 0.0;
  const double dy = ok ? (y1 - y0) / (double)(n - 1) : 0.0;
  if (i == 0) {
    tab[0] = s0;
    tab[1] = s1;
    tab[2] = y0;
    tab[3] = dy;
  }
  if (i >= n || !ok) return;
  const double y = i == n - 1 ? y1 : y0 + (double)i * dy;
  double lo = log(t_min), hi = log(t_max);
  double u = lo + (y - y0) / (y1 - y0) * (hi - lo);
  if (!(u > lo && u < hi)) u = 0.5 * (lo + hi);
  double s = 0.0, ds = 0.0, t = exp(u);
  for (int it = 0; it < 200; ++it) {
    t = exp(u);
    planck_sum(lc, nl, t, s, ds);
    const double g = log(s);
    if (g < y) lo = u;
    else hi = u;
    double un;
    if (s > 0.0 && ds > 0.0) {
      un = u - (g - y) / (t * ds / s);
      if (fabs(un - u) <= 1e-14) {  // converged (before the bracket test: see the leaves)
        u = un;
        break;
      }
      if (!(un > lo && un < hi)) un = 0.5 * (lo + hi);
    } else {
      un = 0.5 * (lo + hi);
    }
    const bool done = fabs(un - u) <= 1e-14 || hi - lo <= 1e-15;
    u = un;
    if (done) break;
  }
  t = exp(u);
  planck_sum(lc, nl, t, s, ds);
  tab[4 + 2 * i] = u;
  tab[5 + 2 * i] = (s > 0.0 && ds > 0.0) ? s / (t * ds) : 0.0;
}

// Per leaf: the temperature at which the emitted power 4 pi m sum kappa_abs B(T) dnu equals
// the absorbed power A.  With S increasing over the range, the inverse table's cubic Hermite
// interpolation in ln S is the root to rounding: its truncation error, h^4 / 384 times the fourth
// derivative of ln T in ln S, is of order 1e-16 at h = ln(S(t_max) / S(t_min)) / 65535 (about
// 7e-4 for the dust tables here, where the interpolated ln T is within 3e-15 of the root).
// Otherwise a Newton iteration on ln F(ln T), kept inside a shrinking bracket, from a linear
// guess.
__global__ __launch_bounds__(256) void temperature_kernel(
    const ModelDev* __restrict__ models, int model, const int32_t* __restrict__ child,
    const double* __restrict__ rho64, const double* __restrict__ a_node,
    const LamConst* __restrict__ lc, int nl, double t_min, double t_max, const double* __restrict__ tab,
    int n_tab, double* __restrict__ t_out) {
  const ModelDev& m = models[model];
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m.n_nodes) return;
  const int64_t internal = m.base + (c < m.n_root ? c : c + (m.n_root_pad - m.n_root));
  if (child[internal] >= 0) {
    t_out[c] = 0.0;
    return;
  }
  int lev = 0;
  while (lev < m.nlev && c >= m.level_off[lev + 1]) ++lev;
  const double len = m.cell_cm * ldexp(1.0, -lev);
  const double mass = rho64[internal] * (len * len * len);
  const double A = a_node[c];
  const double fpi = 4.0 * kPi;
  const double flo = fpi * mass * tab[0];
  if (A <= flo) {
    t_out[c] = t_min;
    return;
  }
  const double fhi = fpi * mass * tab[1];
  if (A >= fhi) {
    t_out[c] = t_max;
    return;
  }
  double lo = log(t_min), hi = log(t_max);
  const double la = log(A);
  double u;
  const double y0 = tab[2], dy = tab[3];
  if (dy > 0.0) {
    double q = (la - log(fpi * mass) - y0) / dy;
    // clamped into the table (a NaN absorbed power lands on entry 0)
    q = q >= 0.0 ? (q <= (double)(n_tab - 1) ? q : (double)(n_tab - 1)) : 0.0;
    int i = (int)q;
    if (i > n_tab - 2) i = n_tab - 2;
    const double f = q - (double)i;
    const double u0 = tab[4 + 2 * i], g0 = tab[5 + 2 * i] * dy;
    const double u1 = tab[6 + 2 * i], g1 = tab[7 + 2 * i] * dy;
    const double f2 = f * f, f3 = f2 * f;
    u = (2.0 * f3 - 3.0 * f2 + 1.0) * u0 + (f3 - 2.0 * f2 + f) * g0 + (3.0 * f2 - 2.0 * f3) * u1 + (f3 - f2) * g1;
    t_out[c] = exp(u < lo ? lo : (u > hi ? hi : u));
    return;
  } else {
    u = lo + (la - log(flo)) / (log(fhi) - log(flo)) * (hi - lo);
  }
  if (!(u > lo && u < hi)) u = 0.5 * (lo + hi);
  double s, ds;
  for (int it = 0; it < 200; ++it) {
    const double t = exp(u);
    planck_sum(lc, nl, t, s, ds);
    const double f = fpi * mass * s;
    if (f < A) lo = u;
    else hi = u;
    double un;
    if (f > 0.0 && ds > 0.0) {
      un = u - (log(f) - la) / (t * ds / s);
      // a Newton step below the tolerance ends the iteration.  Tested before the bracket:
      // where log(f) rounds to log(A) while f < A, the step is zero and un equals the new lower
      // end, which the bracket test would replace by the midpoint of a wide bracket
      if (fabs(un - u) <= 1e-14) {
        u = un;
        break;
      }
      if (!(un > lo && un < hi)) un = 0.5 * (lo + hi);
    } else {
      un = 0.5 * (lo + hi);
    }
    const bool done = fabs(un - u) <= 1e-14 || hi - lo <= 1e-15;
    u = un;
    if (done) break;
  }
  t_out[c] = exp(u);
}

// Dust luminosity of every leaf at one wavelength (paper Sect. 4.2: packets are started from
// a cell in proportion to its emission): 4 pi m kappa_abs B(T) dnu, and the maximum.
__global__ __launch_bounds__(256) void dust_lum_kernel(
    const ModelDev* __restrict__ models, int model, int64_t n_leaves,
    const int32_t* __restrict__ leaf_node, const uint8_t* __restrict__ leaf_level,
    const double* __restrict__ rho64, const double* __restrict__ t_node,
    const LamConst* __restrict__ lc, int lam, double* __restrict__ lum,
    unsigned long long* __restrict__ lmax_bits, const int32_t* __restrict__ leaf_coord, int sub_lev,
    int32_t s0, int32_t s1, int32_t s2) {
  const ModelDev& m = models[model];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double l = 0.0;
  if (k < n_leaves) {
    const int32_t node = leaf_node[m.leaf_base + k];
    const int lev = leaf_level[m.leaf_base + k];
    const double t = t_node[canon_of(m, node)];
    const double len = m.cell_cm * ldexp(1.0, -lev);
    const double mass = rho64[node] * (len * len * len);
    const double kabs = (1.0 - lc[lam].alb) * lc[lam].kext;
    double b = 0.0;
    if (t > 0.0) b = lc[lam].pre / expm1(lc[lam].hnu / (kK * t));
    l = 4.0 * kPi * mass * kabs * b * lc[lam].dnu;
    if (sub_lev >= 0) {  // a subiteration: only the leaves of the subtree emit
      const int32_t* xyz = leaf_coord + 3 * (m.leaf_base + k);
      const int32_t sI[3] = {s0, s1, s2};
      if (!in_subtree(sub_lev, sI, lev, xyz[0], xyz[1], xyz[2])) l = 0.0;
    }
    lum[k] = l;
  }
  // non-negative doubles order like their bit patterns
  unsigned long long bits = (unsigned long long)__double_as_longlong(l);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long other = __shfl_xor(bits, o, 64);
    bits = other > bits ? other : bits;
  }
  if ((threadIdx.x & 63) == 0 && bits) atomicMax(lmax_bits, bits);
}

// Quantise each leaf's share of the maximum to 32 bits: q = floor(L / Lmax * 2^32).
__global__ __launch_bounds__(256) void dust_quant_kernel(int64_t n, const double* __restrict__ lum,
                                                         const unsigned long long* __restrict__ lmax_bits,
                                                         uint64_t* __restrict__ q) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double lmax = __longlong_as_double((long long)*lmax_bits);
  q[k] = lmax > 0.0 ? (uint64_t)floor((lum[k] / lmax) * 4294967296.0) : 0ull;
}

// Exact exclusive prefix sum of the quantised luminosities on the device (the dust-emission
// table of a captured iteration step, whose total must stay on the device): tiles of
// kScanTile values are summed, the tile sums scanned by one block, then each tile is scanned
// from its offset.  Integer sums are exact, so the result equals any other summation order.
constexpr int kScanPer = 16;
constexpr int kScanTile = 256 * kScanPer;

__device__ __forceinline__ uint64_t block_exclusive_u64(uint64_t v, uint64_t* s_w, uint64_t& total) {
  // wave-inclusive scan, then across the 4 waves of a 256-thread block
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint64_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_w[wv] = x;
  __syncthreads();
  uint64_t off = 0;
  for (int k = 0; k < wv; ++k) off += s_w[k];
  total = s_w[0] + s_w[1] + s_w[2] + s_w[3];
  __syncthreads();
  return off + x - v;
}

__global__ __launch_bounds__(256) void scan_tile_sums_kernel(const uint64_t* __restrict__ q, int64_t n,
                                                             uint64_t* __restrict__ tile_sum) {
  __shared__ uint64_t s_w[4];
  const int64_t t0 = (int64_t)blockIdx.x * kScanTile;
  uint64_t v = 0;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    const int64_t i = t0 + (int64_t)j * 256 + threadIdx.x;
    if (i < n) v += q[i];
  }
  uint64_t total;
  (void)block_exclusive_u64(v, s_w, total);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

// One block: tile sums -> exclusive tile offsets (in place); the grand total to *total_out.
__global__ __launch_bounds__(256) void scan_tile_offsets_kernel(uint64_t* __restrict__ tile_sum, int64_t n_tiles,
                                                                uint64_t* __restrict__ total_out) {
  __shared__ uint64_t s_w[4];
  uint64_t carry = 0;
  for (int64_t t0 = 0; t0 < n_tiles; t0 += 256) {
    const int64_t i = t0 + threadIdx.x;
    const uint64_t v = i < n_tiles ? tile_sum[i] : 0ull;
    uint64_t total;
    const uint64_t ex = block_exclusive_u64(v, s_w, total);
    if (i < n_tiles) tile_sum[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) *total_out = carry;
}

__global__ __launch_bounds__(256) void scan_tiles_kernel(const uint64_t* __restrict__ q, int64_t n,
                                                         const uint64_t* __restrict__ tile_off,
                                                         uint64_t* __restrict__ qpre) {
  __shared__ uint64_t s_w[4];
  const int64_t t0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  uint64_t v[kScanPer], sum = 0;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    const int64_t i = t0 + j;
    v[j] = i < n ? q[i] : 0ull;
    sum += v[j];
  }
  uint64_t total;
  uint64_t run = tile_off[blockIdx.x] + block_exclusive_u64(sum, s_w, total);
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    const int64_t i = t0 + j;
    if (i < n) qpre[i] = run;
    run += v[j];
  }
}

// After a (sub)iteration step (App. B): for every leaf of the subtree, replace its arrays of
// levels >= lo by the step's deposits and record the energy imbalance |A - E(T_old)| / E(T_old)
// between what it now absorbs and what it emitted; for every leaf, A_tot = A_stars + the sum of
// its arrays (Eq. 9), from which the temperatures are solved.
__global__ __launch_bounds__(256) void subiter_update_kernel(
    const ModelDev* __restrict__ models, int model, int64_t n_leaves, const int32_t* __restrict__ leaf_node,
    const uint8_t* __restrict__ leaf_level, const int32_t* __restrict__ leaf_coord,
    const double* __restrict__ rho64, const LamConst* __restrict__ lc, int nl, int sub_lev, int32_t s0,
    int32_t s1, int32_t s2, int lo, const double* __restrict__ lvl_new, int64_t lvl_stride,
    double* __restrict__ arrays, const double* __restrict__ a_stars, const double* __restrict__ t_old,
    double* __restrict__ a_tot, double* __restrict__ imb) {
  const ModelDev& m = models[model];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_leaves) return;
  const int32_t node = leaf_node[m.leaf_base + k];
  const int lev = leaf_level[m.leaf_base + k];
  const int64_t c = canon_of(m, node);
  const int32_t* xyz = leaf_coord + 3 * (m.leaf_base + k);
  const int32_t sI[3] = {s0, s1, s2};
  const bool inside = sub_lev < 0 || in_subtree(sub_lev, sI, lev, xyz[0], xyz[1], xyz[2]);
  double sum = 0.0;
  for (int l = 0; l <= m.nlev; ++l) {
    double* a = arrays + (int64_t)l * m.n_nodes + c;
    if (inside && l >= lo) *a = lvl_new[(int64_t)l * lvl_stride + m.canon_base + c];
    sum += *a;
  }
  const double at = a_stars[c] + sum;
  a_tot[c] = at;
  if (inside) {
    const double len = m.cell_cm * ldexp(1.0, -lev);
    const double mass = rho64[node] * (len * len * len);
    double s, ds;
    planck_sum(lc, nl, t_old[c], s, ds);
    const double e = 4.0 * kPi * mass * s;
    imb[c] = e > 0.0 ? fabs(at - e) / e : 0.0;
  }
}

}  // namespace

hipError_t launch_subiter_update(const ModelDev* models, int model, int64_t n_leaves, const int32_t* leaf_node,
                                 const uint8_t* leaf_level, const int32_t* leaf_coord, const double* rho64,
                                 const LamConst* lc, int nl, int sub_lev, const int32_t sub_I[3], int lo,
                                 const double* lvl_new, int64_t lvl_stride, double* arrays, const double* a_stars,
                                 const double* t_old, double* a_tot, double* imb, hipStream_t s) {
  if (n_leaves == 0) return hipSuccess;
  hipLaunchKernelGGL(subiter_update_kernel, dim3((unsigned)((n_leaves + 255) / 256)), dim3(256), 0, s, models,
                     model, n_leaves, leaf_node, leaf_level, leaf_coord, rho64, lc, nl, sub_lev, sub_I[0], sub_I[1],
                     sub_I[2], lo, lvl_new, lvl_stride, arrays, a_stars, t_old, a_tot, imb);
  return hipGetLastError();
}

namespace {

// Leaf i of the subtree: a_solve (already a copy of a_tot) takes the balanced power.
__global__ __launch_bounds__(256) void subiter_ali_kernel(
    const ModelDev* __restrict__ models, int model, int64_t n_leaves,
    const int32_t* __restrict__ leaf_node, const uint8_t* __restrict__ leaf_level,
    const int32_t* __restrict__ leaf_coord, int sub_lev, int32_t s0, int32_t s1, int32_t s2,
    const double* __restrict__ a_tot, const double* __restrict__ e_self, const double* __restrict__ e_emit,
    double* __restrict__ a_solve) {
  const ModelDev& m = models[model];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_leaves) return;
  const int32_t node = leaf_node[m.leaf_base + i];
  const int lev = leaf_level[m.leaf_base + i];
  const int64_t c = canon_of(m, node);
  const int32_t* xyz = leaf_coord + 3 * (m.leaf_base + i);
  const int32_t sI[3] = {s0, s1, s2};
  if (!(sub_lev < 0 || in_subtree(sub_lev, sI, lev, xyz[0], xyz[1], xyz[2]))) return;
  double lam = e_emit[c] > 0.0 ? e_self[c] / e_emit[c] : 0.0;
  lam = lam < 1.0 - 1e-9 ? lam : 1.0 - 1e-9;
  a_solve[c] = (a_tot[c] - e_self[c]) / (1.0 - lam);
}

__global__ __launch_bounds__(256) void subiter_keep_kernel(
    const ModelDev* __restrict__ models, int model, int64_t n_leaves, const int32_t* __restrict__ leaf_node,
    const uint8_t* __restrict__ leaf_level, const int32_t* __restrict__ leaf_coord, int sub_lev, int32_t s0,
    int32_t s1, int32_t s2, const double* __restrict__ t_old, double* __restrict__ t_node) {
  const ModelDev& m = models[model];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_leaves || sub_lev < 0) return;
  const int32_t node = leaf_node[m.leaf_base + k];
  const int lev = leaf_level[m.leaf_base + k];
  const int32_t* xyz = leaf_coord + 3 * (m.leaf_base + k);
  const int32_t sI[3] = {s0, s1, s2};
  if (in_subtree(sub_lev, sI, lev, xyz[0], xyz[1], xyz[2])) return;
  const int64_t c = canon_of(m, node);
  t_node[c] = t_old[c];
}

}  // namespace

hipError_t launch_subiter_ali(const ModelDev* models, int model, int64_t n_nodes, int64_t n_leaves,
                              const int32_t* leaf_node, const uint8_t* leaf_level, const int32_t* leaf_coord,
                              int sub_lev, const int32_t sub_I[3], const double* a_tot, const double* e_self,
                              const double* e_emit, double* a_solve, hipStream_t s) {
  // every node first takes a_tot (the copy is ordered before the kernel on the stream, so the
  // subtree leaves' values are written last)
  hipError_t e = hipMemcpyAsync(a_solve, a_tot, 8 * (size_t)n_nodes, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess || n_leaves == 0) return e;
  hipLaunchKernelGGL(subiter_ali_kernel, dim3((unsigned)((n_leaves + 255) / 256)), dim3(256), 0, s, models, model,
                     n_leaves, leaf_node, leaf_level, leaf_coord, sub_lev, sub_I[0], sub_I[1], sub_I[2], a_tot,
                     e_self, e_emit, a_solve);
  return hipGetLastError();
}

hipError_t launch_subiter_keep(const ModelDev* models, int model, int64_t n_leaves, const int32_t* leaf_node,
                               const uint8_t* leaf_level, const int32_t* leaf_coord, int sub_lev,
                               const int32_t sub_I[3], const double* t_old, double* t_node, hipStream_t s) {
  if (n_leaves == 0 || sub_lev < 0) return hipSuccess;
  hipLaunchKernelGGL(subiter_keep_kernel, dim3((unsigned)((n_leaves + 255) / 256)), dim3(256), 0, s, models,
                     model, n_leaves, leaf_node, leaf_level, leaf_coord, sub_lev, sub_I[0], sub_I[1], sub_I[2],
                     t_old, t_node);
  return hipGetLastError();
}

hipError_t launch_temperature(const ModelDev* models, int model, int64_t n_nodes,
                              const int32_t* child, const double* rho64, const double* a_node,
                              const LamConst* lc, int nl, double t_min, double t_max, double* tab,
                              double* t_out, hipStream_t s) {
  hipLaunchKernelGGL(planck_table_kernel, dim3((kPlanckTable + 255) / 256), dim3(256), 0, s, lc, nl, t_min,
                     t_max, kPlanckTable, tab);
  hipLaunchKernelGGL(temperature_kernel, dim3((unsigned)((n_nodes + 255) / 256)), dim3(256), 0, s,
                     models, model, child, rho64, a_node, lc, nl, t_min, t_max, (const double*)tab,
                     kPlanckTable, t_out);
  return hipGetLastError();
}

hipError_t launch_dust_lum(const ModelDev* models, int model, int64_t n_leaves,
                           const int32_t* leaf_node, const uint8_t* leaf_level,
                           const double* rho64, const double* t_node, const LamConst* lc, int lam,
                           double* lum, unsigned long long* lmax_bits, const int32_t* leaf_coord,
                           int sub_lev, const int32_t sub_I[3], hipStream_t s) {
  hipLaunchKernelGGL(dust_lum_kernel, dim3((unsigned)((n_leaves + 255) / 256)), dim3(256), 0, s,
                     models, model, n_leaves, leaf_node, leaf_level, rho64, t_node, lc, lam, lum,
                     lmax_bits, leaf_coord, sub_lev, sub_I[0], sub_I[1], sub_I[2]);
  return hipGetLastError();
}

hipError_t launch_dust_quant(int64_t n_leaves, const double* lum,
                             const unsigned long long* lmax_bits, uint64_t* q, hipStream_t s) {
  hipLaunchKernelGGL(dust_quant_kernel, dim3((unsigned)((n_leaves + 255) / 256)), dim3(256), 0, s,
                     n_leaves, lum, lmax_bits, q);
  return hipGetLastError();
}

hipError_t launch_dust_scan(int64_t n, const uint64_t* q, uint64_t* qpre, uint64_t* tile_tmp, uint64_t* total_out,
                            hipStream_t s) {
  if (n <= 0) return hipErrorInvalidValue;
  const int64_t n_tiles = (n + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(scan_tile_sums_kernel, dim3((unsigned)n_tiles), dim3(256), 0, s, q, n, tile_tmp);
  hipLaunchKernelGGL(scan_tile_offsets_kernel, dim3(1), dim3(256), 0, s, tile_tmp, n_tiles, total_out);
  hipLaunchKernelGGL(scan_tiles_kernel, dim3((unsigned)n_tiles), dim3(256), 0, s, q, n, (const uint64_t*)tile_tmp,
                     qpre);
  return hipGetLastError();
}

int64_t dust_scan_tiles(int64_t n) { return (n + kScanTile - 1) / kScanTile; }
