// Device-side building blocks of the transport kernels: counter-based random numbers, packet
// emission, point location and the per-level face crossing of the oct-tree.
#pragma once

#include "internal.h"

namespace rtd {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;
constexpr float kTwoPiF = 6.28318530717958647692f;

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): 10 rounds of two 32x32->64 products
// with the published multipliers, key bumped by the Weyl constants between rounds.
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return make_uint4(c0, c1, c2, c3);
}

// Uniform in (0,1): (2 (x >> 9) + 1) 2^-24, exact in float and double alike.
__device__ __forceinline__ double unif64(uint32_t x) { return ((double)(x >> 9) * 2.0 + 1.0) * 0x1p-24; }
__device__ __forceinline__ float unif32(uint32_t x) { return (float)(((x >> 9) << 1) | 1u) * 0x1p-24f; }

// Node accessors.  raw(n) fetches the per-node word used for the subgrid lookup and
// child_of(r) turns it into the first child id (-1 for a leaf).
struct ChildPlain {
  const int32_t* __restrict__ child;
  __device__ __forceinline__ int32_t raw(int32_t n) const { return child[n]; }
  __device__ __forceinline__ static int32_t child_of(int32_t r) { return r; }
};
struct ChildWord {
  const int32_t* __restrict__ word;
  __device__ __forceinline__ int32_t raw(int32_t n) const { return word[n]; }
  __device__ __forceinline__ static int32_t child_of(int32_t r) { return r < 0 ? ~r : -1; }
};

// Root-grid shape and internal id of root cell 0, kept in registers.
struct Dims {
  int32_t n0, n1, n2, base;
  __device__ __forceinline__ int32_t na(int a) const { return a == 0 ? n0 : (a == 1 ? n1 : n2); }
  __device__ __forceinline__ int32_t root(int32_t i0, int32_t i1, int32_t i2) const {
    return base + i0 + n0 * (i1 + n1 * i2);
  }
};
__device__ __forceinline__ Dims dims_of(const ModelDev& m) { return Dims{m.n[0], m.n[1], m.n[2], m.base}; }

template <class T>
__device__ __forceinline__ T sel3(int a, T v0, T v1, T v2) { return a == 0 ? v0 : (a == 1 ? v1 : v2); }

// Half-open point location (paper Sect. 2.1: the subgrid identification entry is looked up
// level by level).
template <class CH>
__device__ int32_t locate_walk(Dims D, const double P[3], int& lev, int32_t I[3], CH ch) {
  if (!(P[0] >= 0.0) || !(P[0] < (double)D.n0) || !(P[1] >= 0.0) || !(P[1] < (double)D.n1) ||
      !(P[2] >= 0.0) || !(P[2] < (double)D.n2))
    return -1;
#pragma unroll
  for (int a = 0; a < 3; ++a) I[a] = (int32_t)floor(P[a]);
  int32_t node = D.root(I[0], I[1], I[2]);
  int l = 0;
  for (;;) {
    const int32_t c = CH::child_of(ch.raw(node));
    if (c < 0) break;
    int b = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int32_t f = (int32_t)floor(ldexp(P[a], l + 1));
      const int bit = f - 2 * I[a];
      I[a] = 2 * I[a] + bit;
      b |= bit << a;
    }
    node = c + b;
    ++l;
  }
  lev = l;
  return node;
}

// Location of a point on a root-box face entered along axis a in direction s: the near-side
// cell on axis a, the midpoint rule on the other axes.
template <class CH>
__device__ int32_t locate_face(Dims D, const double P[3], int a, int s, int& lev, int32_t I[3],
                               CH ch) {
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    int32_t v = (int32_t)floor(P[b]);
    const int32_t nb = D.na(b);
    v = v < 0 ? 0 : v;
    v = v > nb - 1 ? nb - 1 : v;
    const int32_t fa = s > 0 ? (int32_t)P[b] : (int32_t)P[b] - 1;
    I[b] = b == a ? fa : v;
  }
  int32_t node = D.root(I[0], I[1], I[2]);
  int l = 0;
  for (;;) {
    const int32_t c = CH::child_of(ch.raw(node));
    if (c < 0) break;
    const double hc = ldexp(1.0, -(l + 1));
    int b = 0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int mid = (P[q] >= (double)(2 * I[q] + 1) * hc) ? 1 : 0;
      const int bit = q == a ? (s > 0 ? 0 : 1) : mid;
      I[q] = 2 * I[q] + bit;
      b |= bit << q;
    }
    node = c + b;
    ++l;
  }
  lev = l;
  return node;
}

// Integer part of a face crossing (paper Sect. 2.3: a packet leaving a grid continues in the
// parent or enters a subgrid): from cell (node, lev, I) across axis a in direction s.  Ascends
// through parent octs only as far as the neighbour requires, then descends along the
// neighbour's own coordinate bits.  Returns false when the packet leaves the root grid.  On
// return node/lev/I are the neighbour cell where the descent along known bits stopped and raw
// is its node word; a cell that is still refined can only be at the original level, and the
// caller continues with the near-side / midpoint rule.
template <class CH>
__device__ __forceinline__ bool cross_walk(Dims D, const int32_t* __restrict__ up, int a, int s,
                                           int32_t& node, int& lev, int32_t I[3], int32_t& raw,
                                           CH ch) {
  const int L = lev;
  const int32_t Ia = sel3(a, I[0], I[1], I[2]);
  const int32_t Ja = Ia + s;
  if (Ja < 0 || Ja >= (D.na(a) << L)) return false;
  const int32_t J0 = a == 0 ? Ja : I[0];
  const int32_t J1 = a == 1 ? Ja : I[1];
  const int32_t J2 = a == 2 ? Ja : I[2];
  int32_t cur = node;
  int l = L;
  while (l > 0 && ((Ja >> (L - l + 1)) != (Ia >> (L - l + 1)))) {
    cur = up[cur >> 3];
    --l;
  }
  if (l == 0) cur = D.root(J0 >> L, J1 >> L, J2 >> L);
  else cur += s > 0 ? (1 << a) : -(1 << a);
  int32_t r = ch.raw(cur);
  while (l < L && CH::child_of(r) >= 0) {
    ++l;
    const int sh = L - l;
    cur = CH::child_of(r) + (((J0 >> sh) & 1) | (((J1 >> sh) & 1) << 1) | (((J2 >> sh) & 1) << 2));
    r = ch.raw(cur);
  }
  const int sh = L - l;
  I[0] = J0 >> sh;
  I[1] = J1 >> sh;
  I[2] = J2 >> sh;
  node = cur;
  lev = l;
  raw = r;
  return true;
}

// Energy flow from grids to their parents (Sect. 3.3): a package of weight w crossing from the
// leaf `node` (internal id, level L) across axis a, from level-L coordinate Ia to Ja (escaped:
// out of the model), leaves the subtree of every refined ancestor of the old leaf whose level-l
// coordinate on that axis differs from the neighbour's (the other axes are shared); those are
// the ancestors from level L - 1 up to the first that holds the neighbour.  w is added to each
// one's outflow, per canonical node.
__device__ __forceinline__ void flux_exits(const ModelDev& md, const int32_t* __restrict__ up,
                                           double* __restrict__ flux, int32_t node, int L, int32_t Ia,
                                           int32_t Ja, bool escaped, double w) {
  int32_t cur = node;
  for (int l = L - 1; l >= 0; --l) {
    const int sh = L - l;
    if (!escaped && (Ja >> sh) == (Ia >> sh)) break;
    cur = up[cur >> 3];
    const int32_t c = cur - md.base;
    unsafeAtomicAdd(flux + md.canon_base + (c < md.n_root ? c : c - (md.n_root_pad - md.n_root)), w);
  }
}

// ------------------------------------------------------------------------------------------
// Emission (FP64 in both forms)
// ------------------------------------------------------------------------------------------
struct Pk64 {
  double P[3], d[3];
  double w0, tau;
  int32_t node, lev;
  int32_t I[3];
};

__device__ __forceinline__ void iso_dir64(double mu_u, double phi_u, double d[3]) {
  const double mu = 2.0 * mu_u - 1.0;
  const double st = sqrt(1.0 - mu * mu);
  const double phi = kTwoPi * phi_u;
  double sp, cp;
  sincos(phi, &sp, &cp);
  d[0] = st * cp;
  d[1] = st * sp;
  d[2] = mu;
}

// Dust-emission cell pick: last leaf k with qpre[k] <= target.
__device__ __forceinline__ int64_t cdf_pick(const uint64_t* __restrict__ qpre, int64_t n,
                                            uint64_t target) {
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (qpre[mid] <= target) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Birth of packet j of a job (event 0, Philox blocks 0 and 1): position, direction, optical
// depth to the first scattering, start leaf and initial weight (paper Sect. 2.3: packets of
// internal sources and of the external field entering the root grid; Sect. 4.2: dust
// emission with cells picked in proportion to their emission, equal-energy packets).
template <class CH>
__device__ void emit64(const TraceParams& p, const JobDev& job, Dims D, int64_t n_leaves,
                       int64_t leaf_base, uint32_t j, Pk64& k, CH ch, uint32_t key0, uint32_t key1) {
  const uint4 b0 = philox(j, job.stream, 0u, 0u, key0, key1);
  const uint4 b1 = philox(j, job.stream, 0u, 1u, key0, key1);
  if (job.kind == RT_SRC_BACKGROUND) {
    const double n0 = (double)D.n0, n1 = (double)D.n1, n2 = (double)D.n2;
    const double area = 2.0 * (n0 * n1 + n1 * n2 + n0 * n2);
    const double target = unif64(b0.x) * area;
    double cum = 0.0;
    int f = 5;
    for (int f0 = 0; f0 < 6; ++f0) {
      cum += sel3(f0 >> 1, n1 * n2, n0 * n2, n0 * n1);
      if (target < cum) {
        f = f0;
        break;
      }
    }
    const int a = f >> 1;
    const int sg = (f & 1) == 0 ? 1 : -1;
    // tangential axes (lower index first)
    const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
    const double pa = sg > 0 ? 0.0 : sel3(a, n0, n1, n2);
    const double p1 = unif64(b0.y) * sel3(t1, n0, n1, n2);
    const double p2 = unif64(b0.z) * sel3(t2, n0, n1, n2);
    const double mu = sqrt(unif64(b0.w));
    const double st = sqrt(1.0 - mu * mu);
    const double phi = kTwoPi * unif64(b1.x);
    double sp, cp;
    sincos(phi, &sp, &cp);
    const double da = sg > 0 ? mu : -mu;
    const double d1 = st * cp, d2 = st * sp;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      k.P[q] = q == a ? pa : (q == t1 ? p1 : p2);
      k.d[q] = q == a ? da : (q == t1 ? d1 : d2);
    }
    k.tau = -log(unif64(b1.y));
    k.node = locate_face(D, k.P, a, sg, k.lev, k.I, ch);
    k.w0 = job.w0;
  } else if (job.kind == RT_SRC_POINT) {
    k.P[0] = job.pos[0];
    k.P[1] = job.pos[1];
    k.P[2] = job.pos[2];
    iso_dir64(unif64(b0.x), unif64(b0.y), k.d);
    k.tau = -log(unif64(b0.z));
    k.node = locate_walk(D, k.P, k.lev, k.I, ch);
    k.w0 = job.w0;
  } else if (job.kind == RT_SRC_BEAM) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      k.P[a] = job.pos[a];
      k.d[a] = job.dir[a];
    }
    k.tau = -log(unif64(b0.x));
    k.node = locate_walk(D, k.P, k.lev, k.I, ch);
    k.w0 = job.w0;
  } else {
    const uint64_t r = ((uint64_t)b0.x << 32) | (uint64_t)b0.y;
    const uint64_t target = __umul64hi(r, job.qtot);
    const int64_t leaf = cdf_pick(p.cdf_qpre + job.cdf_off, n_leaves, target);
    const int64_t gl = leaf_base + leaf;
    const int lev = p.leaf_level[gl];
    const double h = ldexp(1.0, -lev);
    const double u0 = unif64(b0.z), u1 = unif64(b0.w), u2 = unif64(b1.x);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      k.I[a] = p.leaf_coord[3 * gl + a];
      k.P[a] = ((double)k.I[a] + (a == 0 ? u0 : (a == 1 ? u1 : u2))) * h;
    }
    k.node = p.leaf_node[gl];
    k.lev = lev;
    iso_dir64(unif64(b1.y), unif64(b1.z), k.d);
    k.tau = -log(unif64(b1.w));
    const double lum = p.cdf_lum[job.cdf_off + leaf];
    const uint64_t q = p.cdf_q[job.cdf_off + leaf];
    k.w0 = lum * ((double)job.qtot / ((double)q * (double)job.n));
  }
}

// Henyey-Greenstein polar cosine by inverse CDF.
__device__ __forceinline__ double hg_mu64(double g, double u) {
  double mu;
  if (fabs(g) >= 1e-8) {
    const double gg = g * g;
    const double frac = (1.0 - gg) / (1.0 - g + 2.0 * g * u);
    mu = (1.0 + gg - frac * frac) / (2.0 * g);
  } else {
    mu = 2.0 * u - 1.0;
  }
  mu = mu < -1.0 ? -1.0 : mu;
  mu = mu > 1.0 ? 1.0 : mu;
  return mu;
}

// Direction change by polar cosine mu and azimuth phi (Wang, Jacques & Zheng 1995 form).
__device__ __forceinline__ void rotate64(double d[3], double mu, double phi) {
  const double st = sqrt(1.0 - mu * mu);
  double sp, cp;
  sincos(phi, &sp, &cp);
  double nx, ny, nz;
  if (fabs(d[2]) > 0.99999) {
    nx = st * cp;
    ny = st * sp;
    nz = d[2] > 0.0 ? mu : -mu;
  } else {
    const double tmp = sqrt(1.0 - d[2] * d[2]);
    nx = st * (d[0] * d[2] * cp - d[1] * sp) / tmp + d[0] * mu;
    ny = st * (d[1] * d[2] * cp + d[0] * sp) / tmp + d[1] * mu;
    nz = -st * cp * tmp + d[2] * mu;
  }
  const double nn = sqrt(nx * nx + ny * ny + nz * nz);
  d[0] = nx / nn;
  d[1] = ny / nn;
  d[2] = nz / nn;
}

// Branch identifier of child c of branch b split off at crossing number n (package splitting,
// Sect. 2.3): the MurmurHash3 32-bit finaliser of a mix of the three, 30 bits, never 0.  A
// branch's random numbers use Philox counter word 3 = (branch << 2) | block.
__device__ __forceinline__ uint32_t branch_id(uint32_t b, uint32_t n, uint32_t c) {
  uint32_t h = b * 0x9E3779B1u ^ n * 0x85EBCA77u ^ (c + 1u) * 0xC2B2AE3Du;
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  h &= 0x3FFFFFFFu;
  return h ? h : 1u;
}

// ---- FP32-local segment arithmetic (shared by both FP32-local schedules) ----
// Exit-distance coefficients of one axis: t = fma(x, n, c) is the distance, in local cell
// units, to the face the packet moves toward: (1 - x)/d for d > 0, -x/d for d < 0, infinite
// for d = 0 (components below 1e-30 count as 0, so the reciprocal stays finite).
__device__ __forceinline__ void exit_coef(float d, float& n, float& c) {
  const bool z = !(fabsf(d) >= 1e-30f);
  const float r = 1.0f / (z ? 1.0f : d);
  n = z ? 0.0f : -r;
  c = z ? INFINITY : (d > 0.0f ? r : 0.0f);
}

// 1 - exp(-q) for q >= 0 (the absorbed fraction of a segment).  Below 1/8 the Taylor
// polynomial to q^5 (truncation below q^5/6! = 4.2e-8 relative); above, the hardware base-2
// exponential, whose error of about one ulp of exp(-q) <= 0.89 is at most about 5e-7 relative
// of the result (at q = 1/8).
__device__ __forceinline__ float one_minus_exp(float q) {
  // 1 - e^-q = q (1 - q/2 + q^2/3! - q^3/4! + q^4/5!), in Horner form
  float p = 8.33333333e-3f;         // 1/5!
  p = fmaf(p, q, -4.16666667e-2f);  // -1/4!
  p = fmaf(p, q, 1.66666667e-1f);   // 1/3!
  p = fmaf(p, q, -0.5f);            // -1/2!
  p = fmaf(p, q, 1.0f);
  const float small = p * q;
  const float large = 1.0f - __builtin_amdgcn_exp2f(q * -1.44269504f);
  return q < 0.125f ? small : large;
}

// Henyey-Greenstein polar angle by inversion of its CDF (FP32), returned as its cosine and
// sine.  With a = 1 - g + 2 g u and t = (1 - g^2) / a, the inversion gives
//   1 - mu = (1 - g)(1 - u)(t + 1 - g) / a,   1 + mu = (1 + g) u (1 + g + t) / a,
// products of positive factors (a itself is formed as (1 - g)(1 - u) + (1 + g) u), so both keep
// full relative accuracy and sin = sqrt((1 - mu)(1 + mu)) stays accurate for near-forward and
// near-backward scattering, where sqrt(1 - mu^2) would carry an error of about 2^-24 / sin.
// 1 - u is exact for the uniforms of unif32.  g = 0 reduces to mu = 2u - 1 (isotropic).
__device__ __forceinline__ void hg_angle32(float g, float u, float& mu, float& st) {
  const float gm = 1.0f - g, gp = 1.0f + g, um = 1.0f - u;
  const float ra = 1.0f / (gm * um + gp * u);
  const float t = gm * gp * ra;
  const float om = gm * um * (t + gm) * ra;
  const float op = gp * u * (gp + t) * ra;
  mu = fminf(fmaxf(0.5f * (op - om), -1.0f), 1.0f);
  st = sqrtf(om * op);
}

// Direction change by polar angle (cosine mu, sine st) and azimuth phi (Wang, Jacques & Zheng
// 1995 form).  The sine of the old direction's polar angle is taken from its x and y components,
// which keeps its relative accuracy for directions close to the z axis.
__device__ __forceinline__ void rotate32(float& dx, float& dy, float& dz, float mu, float st, float phi) {
  float sp, cp;
  sincosf(phi, &sp, &cp);
  float nx, ny, nz;
  if (fabsf(dz) > 0.99999f) {
    nx = st * cp;
    ny = st * sp;
    nz = dz > 0.0f ? mu : -mu;
  } else {
    const float tmp = sqrtf(dx * dx + dy * dy);
    const float r = st / tmp;
    nx = r * (dx * dz * cp - dy * sp) + dx * mu;
    ny = r * (dy * dz * cp + dx * sp) + dy * mu;
    nz = -st * cp * tmp + dz * mu;
  }
  const float inv = 1.0f / sqrtf(nx * nx + ny * ny + nz * nz);
  dx = nx * inv;
  dy = ny * inv;
  dz = nz * inv;
}

// Canonical id of an internal id of model m.
__device__ __forceinline__ int64_t canon_of(const ModelDev& m, int32_t node) {
  const int32_t c = node - m.base;
  return c < m.n_root ? (int64_t)c : (int64_t)(c - (m.n_root_pad - m.n_root));
}

// Wave-wide sums (wave64).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace rtd
