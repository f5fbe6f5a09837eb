// Peel-off images of the scattered light with precomputed extinction tables (paper Sect. 2.4).
//
// The transport kernels keep every scattering event of a batch (position, incoming direction,
// weight before the event roulette, leaf, job) in a buffer; after each batch `peel_kernel`
// adds, for every event and observer direction n, w Phi_HG(d.n) exp(-tau) to the pixel the
// event projects onto, as surface brightness per Hz and steradian.  tau is kappa_ext times the
// column (density x length) from the event to the model border along n.  That column is
// either marched cell by cell through the tree, or, with extinction tables, marched only to
// the outer boundary of the refined root cell the event is in (through root leaves up to the
// first refined root cell, for events in a root leaf) and completed with the table value of
// the boundary tile the ray crosses: the column from that tile's centre to the border, built
// once per call by `peel_table_kernel`.  Geometry in FP64, as in the plain form: the march
// visits the cells the plain transport would.
#include "device.h"

using namespace rtd;

namespace {

// One step of a column march: density x length from P to the exit face of leaf (node, lev, I)
// along n (ties to the lowest axis); P moves onto that face.  Returns the exit axis.
__device__ __forceinline__ int march_step(const TraceParams& p, const double n[3], double P[3], int32_t node,
                                          int lev, const int32_t I[3], double& col, int& sg) {
  const double h = ldexp(1.0, -lev);
  double texit = INFINITY, face_ax = 0.0;
  int ax = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (n[a] != 0.0) {
      const double face = n[a] > 0.0 ? (double)(I[a] + 1) * h : (double)I[a] * h;
      const double t = (face - P[a]) / n[a];
      if (t < texit) {
        texit = t;
        ax = a;
        face_ax = face;
      }
    }
  }
  col += p.rho64[node] * texit;
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    double v = fma(texit, n[b], P[b]);
    const double lo = (double)I[b] * h, hi = (double)(I[b] + 1) * h;
    v = v < lo ? lo : v;
    v = v > hi ? hi : v;
    P[b] = v;
  }
#pragma unroll
  for (int b = 0; b < 3; ++b)
    if (b == ax) P[b] = face_ax;
  sg = sel3(ax, n[0], n[1], n[2]) > 0.0 ? 1 : -1;
  return ax;
}

// Across the face just reached: the neighbour leaf (near side on the crossing axis, midpoint
// rule on the others for a refined neighbour).  False when the ray leaves the model.
__device__ __forceinline__ bool cross(const TraceParams& p, Dims D, int ax, int sg, const double P[3], int32_t& node,
                                      int& lev, int32_t I[3]) {
  int32_t raw;
  if (!cross_walk(D, p.up, ax, sg, node, lev, I, raw, ChildPlain{p.child})) return false;
  int32_t c = raw;
  while (c >= 0) {
    const double hc = ldexp(1.0, -(lev + 1));
    int b = 0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int mid = (P[q] >= (double)(2 * I[q] + 1) * hc) ? 1 : 0;
      const int bit = q == ax ? (sg > 0 ? 0 : 1) : mid;
      I[q] = 2 * I[q] + bit;
      b |= bit << q;
    }
    node = c + b;
    ++lev;
    c = p.child[node];
  }
  return true;
}

__device__ double column_exact(const TraceParams& p, Dims D, const double n[3], const double P0[3], int32_t node,
                               int lev, const int32_t I0[3]) {
  double P[3] = {P0[0], P0[1], P0[2]}, col = 0.0;
  int32_t I[3] = {I0[0], I0[1], I0[2]};
  for (;;) {
    int sg;
    const int ax = march_step(p, n, P, node, lev, I, col, sg);
    if (!cross(p, D, ax, sg, P, node, lev, I)) return col;
  }
}

__device__ __forceinline__ int32_t root_linear(Dims D, const int32_t R[3]) { return R[0] + D.n0 * (R[1] + D.n1 * R[2]); }

// Tile of a face point: the two lateral axes in increasing order, [0, 1) of the root cell cut
// into `tiles` parts each.
__device__ __forceinline__ int64_t face_tile(const double P[3], const int32_t R[3], int a, int tiles) {
  const int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
  int64_t tx = (int64_t)floor((sel3(b1, P[0], P[1], P[2]) - (double)sel3(b1, R[0], R[1], R[2])) * tiles);
  int64_t ty = (int64_t)floor((sel3(b2, P[0], P[1], P[2]) - (double)sel3(b2, R[0], R[1], R[2])) * tiles);
  tx = tx < 0 ? 0 : (tx > tiles - 1 ? tiles - 1 : tx);
  ty = ty < 0 ? 0 : (ty > tiles - 1 ? tiles - 1 : ty);
  return ty * tiles + tx;
}

__device__ double column_tabled(const TraceParams& p, const PeelParams& q, int qi, Dims D, const double n[3],
                                const double P0[3], int32_t node, int lev, const int32_t I0[3]) {
  double P[3] = {P0[0], P0[1], P0[2]}, col = 0.0;
  int32_t I[3] = {I0[0], I0[1], I0[2]};
  const int T = q.tiles;
  const int64_t T2 = (int64_t)T * T;
  const int32_t R[3] = {I[0] >> lev, I[1] >> lev, I[2] >> lev};
  const int32_t t0 = q.root_tab[root_linear(D, R)];
  for (;;) {
    int sg;
    const int ax = march_step(p, n, P, node, lev, I, col, sg);
    const int32_t J = sel3(ax, I[0], I[1], I[2]) + sg;
    if (t0 >= 0) {
      if ((J >> lev) != sel3(ax, R[0], R[1], R[2])) {  // leaving the refined root cell
        const int64_t k = (((int64_t)qi * q.n_tab + t0) * 6 + 2 * ax + (sg > 0 ? 1 : 0)) * T2;
        return col + q.tab[k + face_tile(P, R, ax, T)];
      }
      cross(p, D, ax, sg, P, node, lev, I);
    } else {
      if (J < 0 || J >= D.na(ax)) return col;  // leaves the model
      int32_t Rn[3] = {I[0], I[1], I[2]};
      Rn[ax] = J;
      const int32_t tn = q.root_tab[root_linear(D, Rn)];
      if (tn >= 0) {  // enters a refined root cell through its face on the -sg side
        const int64_t k = (((int64_t)qi * q.n_tab + tn) * 6 + 2 * ax + (sg > 0 ? 0 : 1)) * T2;
        return col + q.tab[k + face_tile(P, Rn, ax, T)];
      }
      I[ax] = J;
      node = D.root(I[0], I[1], I[2]);
    }
  }
}

// Table entry (direction, refined root cell, face, tile): the column from the tile centre
// along n to the border; zero where n is parallel to the face or leaves the model through it.
__global__ __launch_bounds__(256) void peel_table_kernel(const TraceParams p, const PeelParams q) {
  const ModelDev& md = p.models[q.model];
  const Dims D = dims_of(md);
  const int T = q.tiles;
  const int64_t T2 = (int64_t)T * T;
  const int64_t total = (int64_t)q.n_dir * q.n_tab * 6 * T2;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t tile = i % T2;
    const int f = (int)((i / T2) % 6);
    const int64_t t = (i / (T2 * 6)) % q.n_tab;
    const int qi = (int)(i / (T2 * 6 * q.n_tab));
    const double* n = q.dir[qi].n;
    const int a = f >> 1, hi = f & 1;
    double v = 0.0;
    if (n[a] != 0.0) {
      const int sg = n[a] > 0.0 ? 1 : -1;
      const int32_t r = q.tab_root[t];
      const int32_t R[3] = {r % D.n0, (r / D.n0) % D.n1, r / (D.n0 * D.n1)};
      const int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
      const int tx = (int)(tile % T), ty = (int)(tile / T);
      double Q[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double rc = (double)R[c];
        Q[c] = c == a ? (double)(R[c] + hi)
                      : (c == b1 ? rc + ((double)tx + 0.5) / (double)T : rc + ((double)ty + 0.5) / (double)T);
      }
      (void)b2;
      const double qa = sel3(a, Q[0], Q[1], Q[2]);
      if (!((sg > 0 && qa >= (double)D.na(a)) || (sg < 0 && qa <= 0.0))) {
        int lev;
        int32_t I[3];
        const int32_t node = locate_face(D, Q, a, sg, lev, I, ChildPlain{p.child});
        v = column_exact(p, D, n, Q, node, lev, I);
      }
    }
    q.tab[i] = v;
  }
}

__global__ __launch_bounds__(256) void peel_kernel(const TraceParams p, const PeelParams q) {
  const unsigned long long n_ev = *q.count < q.cap ? *q.count : q.cap;
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n_ev;
       i += (unsigned long long)gridDim.x * blockDim.x) {
    const PeelEv e = q.ev[i];
    const JobDev& J = p.jobs[e.job];
    const ModelDev& md = p.models[J.model];
    const Dims D = dims_of(md);
    const double g = J.g;
    const double kc = J.kext * md.cell_cm;
    const double scale = q.dnu[J.lam] * q.pix_cm2;
    for (int qi = 0; qi < q.n_dir; ++qi) {
      const PeelDir& V = q.dir[qi];
      const double mu = e.d[0] * V.n[0] + e.d[1] * V.n[1] + e.d[2] * V.n[2];
      const double den = 1.0 + g * g - 2.0 * g * mu;
      const double phase = (1.0 - g * g) / (4.0 * kPi * den * sqrt(den));
      const double col = q.tiles > 0 ? column_tabled(p, q, qi, D, V.n, e.P, e.node, e.lev, e.I)
                                     : column_exact(p, D, V.n, e.P, e.node, e.lev, e.I);
      const double tau = kc * col;
      const double val = e.w * phase * exp(-tau) / scale;
      double u = 0.0, v = 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        u += (e.P[a] - q.C[a]) * V.e1[a];
        v += (e.P[a] - q.C[a]) * V.e2[a];
      }
      const int64_t ix = (int64_t)floor((u / q.W + 0.5) * q.npix);
      const int64_t iy = (int64_t)floor((v / q.W + 0.5) * q.npix);
      if (ix < 0 || iy < 0 || ix >= q.npix || iy >= q.npix) continue;
      unsafeAtomicAdd(q.image + (((int64_t)qi * md.nl + J.lam) * q.npix + iy) * q.npix + ix, val);
    }
  }
}

// After a batch: count what was peeled and what did not fit, empty the buffer.
__global__ void peel_reset_kernel(const PeelParams q) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const unsigned long long c = *q.count;
  *q.done += c < q.cap ? c : q.cap;
  if (c > q.cap) *q.lost += c - q.cap;
  *q.count = 0;
}

}  // namespace

hipError_t launch_peel_tables(const TraceParams& p, const PeelParams& q, hipStream_t s) {
  const int64_t total = (int64_t)q.n_dir * q.n_tab * 6 * q.tiles * q.tiles;
  if (total == 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 1 << 16);
  hipLaunchKernelGGL(peel_table_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, q);
  return hipGetLastError();
}

hipError_t launch_peel(const TraceParams& p, const PeelParams& q, int grid, hipStream_t s) {
  hipLaunchKernelGGL(peel_kernel, dim3(grid), dim3(256), 0, s, p, q);
  hipLaunchKernelGGL(peel_reset_kernel, dim3(1), dim3(64), 0, s, q);
  return hipGetLastError();
}
