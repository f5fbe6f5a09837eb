// Surface-brightness maps through the tree (paper Sect. 4.1): one ray per pixel, orthographic
// view, I <- I exp(-dtau) + (1 - a) B(T) (1 - exp(-dtau)) cell by cell.  Up to NS wavelengths
// are carried in registers per pass; the host splits longer selections into passes.
// Built with -ffp-contract=off like the FP64 trace.
#include "device.h"

using namespace rtd;

namespace {

constexpr double kK = 1.380649e-16;

template <int NS>
__global__ __launch_bounds__(256) void render_fp64_kernel(
    const ModelDev* __restrict__ models, int model, const int32_t* __restrict__ child,
    const int32_t* __restrict__ up, const double* __restrict__ rho64,
    const double* __restrict__ t_node, const LamConst* __restrict__ lc,
    const int32_t* __restrict__ lam_idx, int n_sel, const double* __restrict__ view, int npix,
    double* __restrict__ image, unsigned long long* __restrict__ crossings) {
  const ModelDev& m = models[model];
  const Dims D = dims_of(m);
  const ChildPlain ch{child};
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
    double I[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) I[q] = 0.0;
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
        if (rho > 0.0 && s > 0.0) {
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
      if (q < n_sel) image[((int64_t)q * npix + j) * npix + i] = I[q];
  }
  if (crossings) {
    ncross = wave_sum_u64(ncross);
    if ((threadIdx.x & 63) == 0 && ncross) atomicAdd(crossings, ncross);
  }
}

}  // namespace

hipError_t launch_render_fp64(const ModelDev* models, int model, const int32_t* child,
                              const int32_t* up, const double* rho64, const double* t_node,
                              const LamConst* lc, const int32_t* lam_idx, int n_sel,
                              const double* view, int npix, double* image,
                              unsigned long long* crossings, hipStream_t s) {
  const int64_t n = (int64_t)npix * npix;
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  if (n_sel <= 4)
    hipLaunchKernelGGL(render_fp64_kernel<4>, grid, block, 0, s, models, model, child, up, rho64,
                       t_node, lc, lam_idx, n_sel, view, npix, image, crossings);
  else if (n_sel <= 8)
    hipLaunchKernelGGL(render_fp64_kernel<8>, grid, block, 0, s, models, model, child, up, rho64,
                       t_node, lc, lam_idx, n_sel, view, npix, image, crossings);
  else if (n_sel <= 16)
    hipLaunchKernelGGL(render_fp64_kernel<16>, grid, block, 0, s, models, model, child, up, rho64,
                       t_node, lc, lam_idx, n_sel, view, npix, image, crossings);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}
