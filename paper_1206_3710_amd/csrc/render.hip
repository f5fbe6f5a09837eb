// Surface-brightness maps through the tree (paper Sect. 4.1): one ray per pixel, orthographic
// view, I <- I exp(-dtau) + (1 - a) B(T) (1 - exp(-dtau)) cell by cell.  Up to NS wavelengths
// are carried in registers per pass (16 in FP64, 128 in FP32); the host splits longer selections
// into passes, each of which walks the ray again.
// Built with -ffp-contract=off like the FP64 trace.
//
// Two forms share the ray geometry (FP64, so both visit the same cells): the FP64 form
// evaluates the transfer in FP64; the FP32 form evaluates it per wavelength in FP32 (hardware
// exponentials, constants staged in LDS), which is where the work of a map is.
#include <mutex>

#include "device.h"

using namespace rtd;

namespace {

constexpr double kK = 1.380649e-16;
constexpr double kLog2e = 1.4426950408889634;
constexpr int kG = 8;  // wavelengths per group of the FP32 transfer

// e^x - 1 for x >= 0 in FP32, from y = x log2(e): below x = 1/32 the series to x^3
// (truncation below x^3 / 4! = 1.3e-6 relative), above it the hardware base-2 exponential
// (cancellation below 2 ulp / x = 7.6e-6 relative; inf for large x).
__device__ __forceinline__ float expm1_pos2(float y) {
  float p = 5.55041087e-2f;         // ln2^3 / 3!
  p = fmaf(p, y, 2.40226507e-1f);   // ln2^2 / 2!
  p = fmaf(p, y, 6.93147181e-1f);   // ln2
  const float small = p * y;
  const float large = __builtin_amdgcn_exp2f(y) - 1.0f;
  return y < 4.50842200e-2f ? small : large;  // log2(e) / 32
}

template <int NS, bool F32>
__global__ __launch_bounds__(256, NS > 32 ? 2 : 1) void render_kernel(
    const ModelDev* __restrict__ models, int model, const int32_t* __restrict__ child,
    const int32_t* __restrict__ up, const double* __restrict__ rho64,
    const double* __restrict__ t_node, const LamConst* __restrict__ lc,
    const int32_t* __restrict__ lam_idx, int n_sel, const double* __restrict__ view, int npix,
    double* __restrict__ image, unsigned long long* __restrict__ crossings) {
  const ModelDev& m = models[model];
  const Dims D = dims_of(m);
  const ChildPlain ch{child};
  // FP32 form: per-wavelength constants -kappa_ext * cell size * log2(e), (1 - albedo)
  // 2 h nu^3 / c^2, h nu / k * log2(e) (the base-2 exponentials then take them directly)
  // Wavelengths past n_sel (up to the next multiple of kG) are padded with kappa = 0 and no
  // source, which leaves their intensity at 0 and is never written out.
  __shared__ float s_kc[NS], s_ap[NS], s_hk[NS];
  if (F32) {
    if (threadIdx.x < NS) {
      const bool real = (int)threadIdx.x < n_sel;
      const LamConst& L = lc[lam_idx[real ? threadIdx.x : 0]];
      s_kc[threadIdx.x] = real ? (float)(-L.kext * m.cell_cm * kLog2e) : 0.0f;
      s_ap[threadIdx.x] = real ? (float)((1.0 - L.alb) * L.pre) : 0.0f;
      s_hk[threadIdx.x] = real ? (float)(L.hnu / kK * kLog2e) : 1.0f;
    }
    __syncthreads();
  }
  const int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long ncross = 0;
  if (pix < (int64_t)npix * npix) {
    const int i = (int)(pix % npix), j = (int)(pix / npix);
    const double n[3] = {view[0], view[1], view[2]};
    const double ox = (((double)i + 0.5) / (double)npix - 0.5) * view[12];
    const double oy = (((double)j + 0.5) / (double)npix - 0.5) * view[12];
    double Q[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) Q[a] = view[9 + a] + ox * view[3 + a] + oy * view[6 + a];
    double I[F32 ? 1 : NS];
    float I32[F32 ? NS : 1];
#pragma unroll
    for (int q = 0; q < (F32 ? 1 : NS); ++q) I[q] = 0.0;
#pragma unroll
    for (int q = 0; q < (F32 ? NS : 1); ++q) I32[q] = 0.0f;
    double tn = -INFINITY, tf = INFINITY;
    int ax = -1;
    bool miss = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double na = (double)D.na(a);
      if (n[a] != 0.0) {
        const double t1 = (0.0 - Q[a]) / n[a], t2 = (na - Q[a]) / n[a];
        const double lo = t1 < t2 ? t1 : t2, hi = t1 < t2 ? t2 : t1;
        if (lo > tn) {
          tn = lo;
          ax = a;
        }
        if (hi < tf) tf = hi;
      } else if (Q[a] < 0.0 || Q[a] >= na) {
        miss = true;
      }
    }
    if (!miss && ax >= 0 && tn < tf) {
      double P[3];
      const double nax = sel3(ax, n[0], n[1], n[2]);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double na = (double)D.na(a);
        double v = fma(tn, n[a], Q[a]);
        if (a == ax) v = nax > 0.0 ? 0.0 : na;
        v = v < 0.0 ? 0.0 : v;
        v = v > na ? na : v;
        P[a] = v;
      }
      int lev;
      int32_t Ic[3];
      int32_t node = locate_face(D, P, ax, nax > 0.0 ? 1 : -1, lev, Ic, ch);
      ncross = 1;
      for (;;) {
        // past 32 wavelengths the per-wavelength constants are read from LDS at every cell (a
        // compiler barrier keeps them from being hoisted into registers, which hold the
        // intensities)
        if (F32 && NS > 32) asm volatile("" ::: "memory");
        const double rho = rho64[node];
        const double h = ldexp(1.0, -lev);
        double texit = INFINITY, face_ax = 0.0;
        int cax = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          if (n[a] != 0.0) {
            const double face = n[a] > 0.0 ? (double)(Ic[a] + 1) * h : (double)Ic[a] * h;
            const double t = (face - P[a]) / n[a];
            if (t < texit) {
              texit = t;
              cax = a;
              face_ax = face;
            }
          }
        }
        const double s = texit;
        if (F32 && rho > 0.0 && s > 0.0) {
          // per wavelength: the segment's transmission e^-dtau, its emission weight 1 - e^-dtau
          // (series below 1/32, else from the transmission), and the source (1 - a) B(T)
          const float tc = (float)t_node[canon_of(m, node)];
          const float f = (float)(rho * s);
          // a cell without a temperature emits nothing: 1 / T = inf makes the source term 0
          const float inv_t = tc > 0.0f ? __builtin_amdgcn_rcpf(tc) : INFINITY;
          // groups of kG wavelengths: a group past the selection is skipped with a scalar
          // branch, the padded ones inside the last group are computed
#pragma unroll
          for (int q0 = 0; q0 < NS; q0 += kG) {
            if (NS <= kG || q0 < n_sel) {
#pragma unroll
              for (int q = q0; q < (q0 + kG < NS ? q0 + kG : NS); ++q) {
                const float z = s_kc[q] * f;  // -dtau log2(e)
                const float att = __builtin_amdgcn_exp2f(z);
                // 1 - e^-dtau: below dtau = 1/32 the series to dtau^3 in z
                float em = -5.55041087e-2f;
                em = fmaf(em, z, -2.40226507e-1f);
                em = fmaf(em, z, -6.93147181e-1f);
                em = z > -4.50842200e-2f ? em * z : 1.0f - att;
                const float src = s_ap[q] * __builtin_amdgcn_rcpf(expm1_pos2(s_hk[q] * inv_t));
                I32[q] = fmaf(I32[q], att, src * em);
              }
            }
          }
        } else if (!F32 && rho > 0.0 && s > 0.0) {
          const double tc = t_node[canon_of(m, node)];
#pragma unroll
          for (int q = 0; q < NS; ++q) {
            if (q < n_sel) {
              const LamConst& L = lc[lam_idx[q]];
              const double dtau = ((L.kext * rho) * m.cell_cm) * s;
              const double att = exp(-dtau);
              const double em = -expm1(-dtau);
              double b = 0.0;
              if (tc > 0.0) b = L.pre / expm1(L.hnu / (kK * tc));
              const double src = (1.0 - L.alb) * b;
              I[q] = I[q] * att + src * em;
            }
          }
        }
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          double v = fma(s, n[b], P[b]);
          const double lo = (double)Ic[b] * h, hi = (double)(Ic[b] + 1) * h;
          v = v < lo ? lo : v;
          v = v > hi ? hi : v;
          P[b] = b == cax ? face_ax : v;
        }
        const int sg = sel3(cax, n[0], n[1], n[2]) > 0.0 ? 1 : -1;
        int32_t raw;
        if (!cross_walk(D, up, cax, sg, node, lev, Ic, raw, ch)) break;
        int32_t c = raw;
        while (c >= 0) {
          const double hc = ldexp(1.0, -(lev + 1));
          int b = 0;
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            const int mid = (P[q] >= (double)(2 * Ic[q] + 1) * hc) ? 1 : 0;
            const int bit = q == cax ? (sg > 0 ? 0 : 1) : mid;
            Ic[q] = 2 * Ic[q] + bit;
            b |= bit << q;
          }
          node = c + b;
          ++lev;
          c = child[node];
        }
        ++ncross;
      }
    }
#pragma unroll
    for (int q = 0; q < NS; ++q)
      if (q < n_sel) image[((int64_t)q * npix + j) * npix + i] = F32 ? (double)I32[q] : I[F32 ? 0 : q];
  }
  if (crossings) {
    ncross = wave_sum_u64(ncross);
    if ((threadIdx.x & 63) == 0 && ncross) atomicAdd(crossings, ncross);
  }
}

}  // namespace

hipError_t launch_render(bool f32, const ModelDev* models, int model, const int32_t* child,
                         const int32_t* up, const double* rho64, const double* t_node,
                         const LamConst* lc, const int32_t* lam_idx, int n_sel,
                         const double* view, int npix, double* image,
                         unsigned long long* crossings, hipStream_t s) {
  const int64_t n = (int64_t)npix * npix;
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
#define RT_RENDER(NS, F)                                                                        \
  hipLaunchKernelGGL((render_kernel<NS, F>), grid, block, 0, s, models, model, child, up, rho64, \
                     t_node, lc, lam_idx, n_sel, view, npix, image, crossings)
  if (n_sel > (f32 ? kRenderPassF32 : kRenderPassF64)) return hipErrorInvalidValue;
  if (f32) {
    if (n_sel <= 4) RT_RENDER(4, true);
    else if (n_sel <= 8) RT_RENDER(8, true);
    else if (n_sel <= 16) RT_RENDER(16, true);
    else RT_RENDER(128, true);
  } else {
    if (n_sel <= 4) RT_RENDER(4, false);
    else if (n_sel <= 8) RT_RENDER(8, false);
    else RT_RENDER(16, false);
  }
#undef RT_RENDER
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Allocation-free maps: the per-call staging (view frame, wavelength list) and the crossing
// counter live in the file-scope device array `scratch` instead of context buffers.  Each
// device's copy is located once, when a context is created on it (rt_create); calls on one
// device share it, so calls that overlap on one device race.
// ------------------------------------------------------------------------------------------
namespace {

constexpr int kScrView = 0;       // 13 doubles: n, e1, e2, box centre, width
constexpr int kScrCount = 128;    // u64 crossing counter (cleared by every call)
constexpr int kScrLam = 256;      // int32 wavelength indices
constexpr int kScratchBytes = kScrLam + 4 * kRenderNoAllocMaxSel;
constexpr int kMaxDevices = 64;

struct RenderSetup {
  double view[13];
  int32_t n_sel;
  int32_t lam[kRenderNoAllocMaxSel];
};
static_assert(sizeof(RenderSetup) <= 4096, "kernel argument size");

// Writes one call's parameters into the scratch array and clears its counter (a kernel, not a
// memset, so that the call can also be recorded into a graph).
__global__ void render_setup_kernel(const RenderSetup a, unsigned char* __restrict__ scr) {
  double* v = reinterpret_cast<double*>(scr + kScrView);
  int32_t* li = reinterpret_cast<int32_t*>(scr + kScrLam);
  for (int i = threadIdx.x; i < 13; i += blockDim.x) v[i] = a.view[i];
  if (threadIdx.x == 0) *reinterpret_cast<unsigned long long*>(scr + kScrCount) = 0ull;
  for (int i = threadIdx.x; i < a.n_sel; i += blockDim.x) li[i] = a.lam[i];
}

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

hipError_t render_scratch_init(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

void* render_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return device >= 0 && device < kMaxDevices ? g_scratch_ptr[device] : nullptr;
}

hipError_t launch_render_noalloc(bool f32, const ModelDev* models, int model, const int32_t* child,
                                 const int32_t* up, const double* rho64, const double* t_node,
                                 const LamConst* lc, const int32_t* lam_idx_host, int n_sel,
                                 const double* view_host, int npix, double* image, void* scr,
                                 unsigned long long* crossings_host, hipStream_t s) {
  if (n_sel < 1 || n_sel > kRenderNoAllocMaxSel || !scr) return hipErrorInvalidValue;
  RenderSetup a;
  for (int i = 0; i < 13; ++i) a.view[i] = view_host[i];
  a.n_sel = n_sel;
  for (int i = 0; i < n_sel; ++i) a.lam[i] = lam_idx_host[i];
  unsigned char* base = static_cast<unsigned char*>(scr);
  hipLaunchKernelGGL(render_setup_kernel, dim3(1), dim3(256), 0, s, a, base);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const double* v = reinterpret_cast<const double*>(base + kScrView);
  const int32_t* li = reinterpret_cast<const int32_t*>(base + kScrLam);
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(base + kScrCount);
  const int pass = f32 ? kRenderPassF32 : kRenderPassF64;
  for (int q0 = 0; q0 < n_sel; q0 += pass) {
    const int nq = n_sel - q0 < pass ? n_sel - q0 : pass;
    e = launch_render(f32, models, model, child, up, rho64, t_node, lc, li + q0, nq, v, npix,
                      image + (size_t)q0 * npix * npix, q0 == 0 ? cnt : nullptr, s);
    if (e != hipSuccess) return e;
  }
  if (crossings_host) return hipMemcpyAsync(crossings_host, cnt, 8, hipMemcpyDeviceToHost, s);
  return hipSuccess;
}
