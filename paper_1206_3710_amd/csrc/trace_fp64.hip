// Plain FP64 form of the Monte Carlo formal solution (paper Sect. 2.3): one packet per lane,
// global root-cell coordinates in FP64, FP64 atomics into the per-node absorbed energy.
// Built with -ffp-contract=off so every rounding step is the one written here.
#include "device.h"

using namespace rtd;

namespace {

__global__ __launch_bounds__(256) void trace_fp64_kernel(const TraceParams p, const int job_idx) {
  const JobDev& job = p.jobs[job_idx];
  const ModelDev& md = p.models[job.model];
  const Dims D = dims_of(md);
  const ChildPlain ch{p.child};
  const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;

  double t_esc = 0.0, t_emit = 0.0, t_kill = 0.0, t_gain = 0.0, t_trunc = 0.0;
  unsigned long long c_cross = 0, c_scat = 0, c_kill = 0, c_trunc = 0, c_pk = 0;

  if (j < job.n) {
    Pk64 k;
    emit64(p, job, D, md.n_leaves, md.leaf_base, (uint32_t)j, k, ch, p.key0, p.key1);
    const int32_t birth = k.node;
    double w = k.w0;
    const double w0 = k.w0;
    double tau = k.tau;
    c_pk = 1;
    t_emit = w0;
    if (p.emit_acc && job.kind == RT_SRC_DUST)
      unsafeAtomicAdd(p.emit_acc + md.canon_base + canon_of(md, k.node), w0);
    // shallowest level visited: the external field enters through the root grid
    int mlev = job.kind == RT_SRC_BACKGROUND ? 0 : k.lev;
    const double kext = job.kext, alb = job.alb, g = job.g, cm = md.cell_cm;
    double* __restrict__ acc = p.acc64 + job.acc_off;
    uint32_t crossings = 1, ev = 0, status = 0;
    for (;;) {
      const double rho = p.rho64[k.node];
      const double se = (kext * rho) * cm;
      const double ss = alb * se;
      const double sa = se - ss;
      const double h = ldexp(1.0, -k.lev);
      // exit distance through the leaf's faces; ties go to the lowest axis
      double texit = INFINITY, face_ax = 0.0;
      int ax = 0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (k.d[a] != 0.0) {
          const double face = k.d[a] > 0.0 ? (double)(k.I[a] + 1) * h : (double)k.I[a] * h;
          const double t = (face - k.P[a]) / k.d[a];
          if (t < texit) {
            texit = t;
            ax = a;
            face_ax = face;
          }
        }
      }
      // free path in scattering optical depth; continuous absorption along the segment
      bool event = false;
      double s;
      if (ss > 0.0 && tau <= ss * texit) {
        s = tau / ss;
        event = true;
      } else {
        s = texit;
        tau = tau - ss * texit;
      }
      if (sa > 0.0 && s > 0.0) {
        const double de = w * (-expm1(-(sa * s)));
        unsafeAtomicAdd(acc + k.node, de);
        // accelerated Lambda iteration: absorption in the birth cell before the first crossing
        if (p.self_acc && crossings == 1 && job.kind == RT_SRC_DUST)
          unsafeAtomicAdd(p.self_acc + md.canon_base + canon_of(md, k.node), de);
        if (p.lvl_acc)
          unsafeAtomicAdd(p.lvl_acc + (int64_t)mlev * p.lvl_stride + md.canon_base + canon_of(md, k.node), de);
        w = w - de;
      }
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        double v = fma(s, k.d[b], k.P[b]);
        const double lo = (double)k.I[b] * h, hi = (double)(k.I[b] + 1) * h;
        v = v < lo ? lo : v;
        v = v > hi ? hi : v;
        k.P[b] = v;
      }
      if (event) {
        ++ev;
        if ((int64_t)ev > p.max_events) {
          c_trunc = 1;
          t_trunc = w;
          status = 2;
          break;
        }
        ++c_scat;
        if (p.peel_ev) {
          // kept for the peel-off with the weight before the event roulette
          const unsigned long long idx = atomicAdd(p.peel_count, 1ull);
          if (idx < p.peel_cap) {
            PeelEv& e = p.peel_ev[idx];
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              e.P[b] = k.P[b];
              e.d[b] = k.d[b];
              e.I[b] = k.I[b];
            }
            e.w = w;
            e.node = k.node;
            e.job = job_idx;
            e.lev = k.lev;
          }
        }
        const uint4 x = philox((uint32_t)j, job.stream, ev, 0u, p.key0, p.key1);
        if (p.rr_p > 0.0 && w < p.rr_thr * w0) {
          if (unif64(x.x) < p.rr_p) {
            c_kill = 1;
            t_kill = w;
            status = 1;
            break;
          }
          const double nw = w / (1.0 - p.rr_p);
          t_gain += nw - w;
          w = nw;
        }
        const double mu = hg_mu64(g, unif64(x.y));
        rotate64(k.d, mu, kTwoPi * unif64(x.z));
        tau = -log(unif64(x.w));
        continue;
      }
#pragma unroll
      for (int b = 0; b < 3; ++b)
        if (b == ax) k.P[b] = face_ax;
      const int sg = sel3(ax, k.d[0], k.d[1], k.d[2]) > 0.0 ? 1 : -1;
      if (p.flux_acc) {
        // automatic iteration: the weight leaving each refined ancestor's subtree
        const int32_t Ia = k.I[ax], Ja = Ia + sg;
        flux_exits(md, p.up, p.flux_acc, k.node, k.lev, Ia, Ja, Ja < 0 || Ja >= (D.na(ax) << k.lev), w);
      }
      int32_t raw;
      if (!cross_walk(D, p.up, ax, sg, k.node, k.lev, k.I, raw, ch)) {
        t_esc = w;
        status = 0;
        break;
      }
      // a refined neighbour at the original level: near side on the crossing axis, midpoint
      // rule on the others
      int32_t c = raw;
      while (c >= 0) {
        const double hc = ldexp(1.0, -(k.lev + 1));
        int b = 0;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const int mid = (k.P[q] >= (double)(2 * k.I[q] + 1) * hc) ? 1 : 0;
          const int bit = q == ax ? (sg > 0 ? 0 : 1) : mid;
          k.I[q] = 2 * k.I[q] + bit;
          b |= bit << q;
        }
        k.node = c + b;
        ++k.lev;
        c = p.child[k.node];
      }
      if (p.sub_lev >= 0 && !in_subtree(p.sub_lev, p.sub_I, k.lev, k.I[0], k.I[1], k.I[2])) {
        // a subiteration follows packets only inside its subtree
        t_esc = w;
        status = 0;
        break;
      }
      if (k.lev < mlev) mlev = k.lev;
      if (++crossings >= (1u << 30)) {  // guards termination; never reached by valid input
        c_trunc = 1;
        t_trunc = w;
        status = 2;
        break;
      }
    }
    c_cross = crossings;
    if (p.rec_stride > 0 && (j % (uint64_t)p.rec_stride) == 0) {
      rt_record r;
      r.status = status;
      r.crossings = crossings;
      r.events = ev;
      r.pad = 0;
      r.node = status == 0 ? -1 : canon_of(md, k.node);
      r.birth = canon_of(md, birth);
      r.w = status == 0 ? t_esc : (status == 1 ? t_kill : t_trunc);
      p.rec[job.rec_base + (int64_t)(j / (uint64_t)p.rec_stride)] = r;
    }
  }
  // wave-level reduction of the tallies, one atomic per wave
  t_esc = wave_sum(t_esc);
  t_emit = wave_sum(t_emit);
  t_kill = wave_sum(t_kill);
  t_gain = wave_sum(t_gain);
  t_trunc = wave_sum(t_trunc);
  c_cross = wave_sum_u64(c_cross);
  c_scat = wave_sum_u64(c_scat);
  c_kill = wave_sum_u64(c_kill);
  c_trunc = wave_sum_u64(c_trunc);
  c_pk = wave_sum_u64(c_pk);
  if ((threadIdx.x & 63) == 0 && c_pk > 0) {
    unsafeAtomicAdd(p.esc + job.esc_slot, t_esc);
    unsafeAtomicAdd(&p.stats->e_emit, t_emit);
    if (t_kill != 0.0) unsafeAtomicAdd(&p.stats->e_killed, t_kill);
    if (t_gain != 0.0) unsafeAtomicAdd(&p.stats->e_rr_gain, t_gain);
    if (t_trunc != 0.0) unsafeAtomicAdd(&p.stats->e_trunc, t_trunc);
    atomicAdd(&p.stats->crossings, c_cross);
    atomicAdd(&p.stats->scatterings, c_scat);
    if (c_kill) atomicAdd(&p.stats->kills, c_kill);
    if (c_trunc) atomicAdd(&p.stats->truncated, c_trunc);
    atomicAdd(&p.stats->packets, c_pk);
  }
}

}  // namespace

hipError_t launch_trace_fp64(const TraceParams& p, int job, uint64_t n, int block, hipStream_t s) {
  const uint64_t grid = (n + block - 1) / block;
  hipLaunchKernelGGL(trace_fp64_kernel, dim3((unsigned)grid), dim3(block), 0, s, p, job);
  return hipGetLastError();
}
