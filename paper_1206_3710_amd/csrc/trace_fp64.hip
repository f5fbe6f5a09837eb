// Plain FP64 form of the Monte Carlo formal solution (paper Sect. 2.3): one packet per lane,
// global root-cell coordinates in FP64, FP64 atomics into the per-node absorbed energy.
// Built with -ffp-contract=off so every rounding step is the one written here.
//
// With package splitting (Sect. 2.3) a package entering a grid of a higher level continues with
// 1/N of its weight and appends N - 1 new packages to a queue; those are followed by later
// launches over the queue (launch_split_fp64), each with its own branch identifier in the
// counter of its random numbers.
#include "device.h"

using namespace rtd;

namespace {

// Tallies of the packages a lane follows, reduced per wave at the end of a kernel.
struct Tally64 {
  double esc = 0.0, kill = 0.0, gain = 0.0, trunc = 0.0, skilled = 0.0, sgain = 0.0;
  unsigned long long cross = 0, scat = 0, kills = 0, truncs = 0, splits = 0, skills = 0, sskips = 0;
};

// Follows one package (state k, weight w, free path tau, crossings and events so far, branch br
// of packet pid) to its end.  Returns the fate: 0 escaped, 1 killed by the event roulette,
// 2 truncated, 3 killed by the exit roulette of splitting.  SPLIT: package splitting is on
// (the instance without it keeps the registers of the plain walk).
template <bool SPLIT>
__device__ int follow64(const TraceParams& p, const int job_idx, const JobDev& job, const ModelDev& md,
                        const Dims& D, const ChildPlain& ch, const uint32_t pid, const uint32_t br, Pk64& k,
                        double& w, const double w0, double& tau, uint32_t& crossings, uint32_t& ev, int& mlev,
                        Tally64& T) {
  const double kext = job.kext, alb = job.alb, g = job.g, cm = md.cell_cm;
  double* __restrict__ acc = p.acc64 + job.acc_off;
  const int N = p.split_n;
  int status = 0;
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
      // (the package as emitted only: a split-off package starts its count in another cell)
      if (p.self_acc && crossings == 1 && br == 0 && job.kind == RT_SRC_DUST)
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
        status = 2;
        break;
      }
      ++T.scat;
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
      const uint4 x = philox(pid, job.stream, ev, br << 2, p.key0, p.key1);
      if (p.rr_p > 0.0 && w < p.rr_thr * w0) {
        if (unif64(x.x) < p.rr_p) {
          status = 1;
          break;
        }
        const double nw = w / (1.0 - p.rr_p);
        T.gain += nw - w;
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
    const int old_lev = k.lev;
    int32_t raw;
    if (!cross_walk(D, p.up, ax, sg, k.node, k.lev, k.I, raw, ch)) {
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
      status = 0;
      break;
    }
    if (k.lev < mlev) mlev = k.lev;
    if (++crossings >= (1u << 30)) {  // guards termination; never reached by valid input
      status = 2;
      break;
    }
    if (SPLIT && N > 1) {
      // splitting: the level of the grid the package is in (a grid holds the levels down to
      // split_depth below its top cell)
      const int gl_old = old_lev < p.split_depth ? old_lev : p.split_depth;
      const int gl_new = k.lev < p.split_depth ? k.lev : p.split_depth;
      if (gl_new > gl_old) {
        // entering a grid of a higher level: N packages of equal weight; this one continues,
        // the others draw their own free paths and wait in the queue
        const unsigned long long idx = atomicAdd(p.sq_count, (unsigned long long)(N - 1));
        if (idx + (unsigned long long)(N - 1) <= p.sq_cap) {
          const double wn = w / (double)N;
          for (int cc = 1; cc < N; ++cc) {
            const uint32_t bc = branch_id(br, crossings, (uint32_t)cc);
            const uint4 xs = philox(pid, job.stream, crossings, (bc << 2) | 2u, p.key0, p.key1);
            Split64& q = p.sq_out[idx + (unsigned long long)(cc - 1)];
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              q.P[b] = k.P[b];
              q.d[b] = k.d[b];
              q.I[b] = k.I[b];
            }
            q.w = wn;
            q.w0 = w0;
            q.tau = -log(unif64(xs.x));
            q.node = k.node;
            q.lev = k.lev;
            q.pid = pid;
            q.job = job_idx;
            q.ev = ev;
            q.br = bc;
            q.mlev = mlev;
          }
          w = wn;
          T.splits += 1;
        } else {
          // no room: the package continues whole (either is unbiased); the reserved slots that
          // are inside the queue are marked empty
          for (unsigned long long e = idx; e < idx + (unsigned long long)(N - 1) && e < p.sq_cap; ++e)
            p.sq_out[e].job = -1;
          T.sskips += 1;
        }
      } else if (gl_new < gl_old) {
        // leaving for a grid of a lower level: survives with probability 1/N, weight times N
        const uint4 xr = philox(pid, job.stream, crossings, (br << 2) | 3u, p.key0, p.key1);
        if (unif64(xr.x) < 1.0 / (double)N) {
          const double nw = w * (double)N;
          T.sgain += nw - w;
          w = nw;
        } else {
          status = 3;
          break;
        }
      }
    }
  }
  // the package's end, with its weight there
  if (status == 0) {
    T.esc += w;
  } else if (status == 1) {
    T.kills += 1;
    T.kill += w;
  } else if (status == 2) {
    T.truncs += 1;
    T.trunc += w;
  } else {
    T.skills += 1;
    T.skilled += w;
  }
  return status;
}

// Adds a wave's tallies to the totals.  followed: this lane followed a package (a split-off
// package may end, by the event roulette or an escape, before its first crossing, so neither
// the packet count nor the crossings tell whether a wave has something to add).
__device__ __forceinline__ void flush_tallies(const TraceParams& p, int esc_slot, Tally64& T, double t_emit,
                                              unsigned long long c_pk, bool followed) {
  const double t_esc = wave_sum(T.esc), e_emit = wave_sum(t_emit), t_kill = wave_sum(T.kill),
               t_gain = wave_sum(T.gain), t_trunc = wave_sum(T.trunc), t_sk = wave_sum(T.skilled),
               t_sg = wave_sum(T.sgain);
  const unsigned long long c_cross = wave_sum_u64(T.cross), c_scat = wave_sum_u64(T.scat),
                           c_kill = wave_sum_u64(T.kills), c_trunc = wave_sum_u64(T.truncs),
                           c_split = wave_sum_u64(T.splits), c_skill = wave_sum_u64(T.skills),
                           c_sskip = wave_sum_u64(T.sskips), n_pk = wave_sum_u64(c_pk);
  const bool any = __ballot(followed) != 0;  // every lane takes part in the vote
  if ((threadIdx.x & 63) == 0 && any) {
    unsafeAtomicAdd(p.esc + esc_slot, t_esc);
    if (e_emit != 0.0) unsafeAtomicAdd(&p.stats->e_emit, e_emit);
    if (t_kill != 0.0) unsafeAtomicAdd(&p.stats->e_killed, t_kill);
    if (t_gain != 0.0) unsafeAtomicAdd(&p.stats->e_rr_gain, t_gain);
    if (t_trunc != 0.0) unsafeAtomicAdd(&p.stats->e_trunc, t_trunc);
    if (t_sk != 0.0) unsafeAtomicAdd(&p.stats->e_split_killed, t_sk);
    if (t_sg != 0.0) unsafeAtomicAdd(&p.stats->e_split_gain, t_sg);
    atomicAdd(&p.stats->crossings, c_cross);
    atomicAdd(&p.stats->scatterings, c_scat);
    if (c_kill) atomicAdd(&p.stats->kills, c_kill);
    if (c_trunc) atomicAdd(&p.stats->truncated, c_trunc);
    if (c_split) atomicAdd(&p.stats->splits, c_split);
    if (c_skill) atomicAdd(&p.stats->split_kills, c_skill);
    if (c_sskip) atomicAdd(&p.stats->split_skips, c_sskip);
    if (n_pk) atomicAdd(&p.stats->packets, n_pk);
  }
}

template <bool SPLIT>
__global__ __launch_bounds__(256) void trace_fp64_kernel(const TraceParams p, const int job_idx) {
  const JobDev& job = p.jobs[job_idx];
  const ModelDev& md = p.models[job.model];
  const Dims D = dims_of(md);
  const ChildPlain ch{p.child};
  const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  Tally64 T;
  double t_emit = 0.0;
  unsigned long long c_pk = 0;
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
    uint32_t crossings = 1, ev = 0;
    const int status = follow64<SPLIT>(p, job_idx, job, md, D, ch, (uint32_t)j, 0u, k, w, w0, tau, crossings, ev, mlev, T);
    T.cross += crossings;
    if (p.rec_stride > 0 && (j % (uint64_t)p.rec_stride) == 0) {
      rt_record r;
      r.status = (uint32_t)status;
      r.crossings = crossings;
      r.events = ev;
      r.pad = 0;
      r.node = status == 0 ? -1 : canon_of(md, k.node);
      r.birth = canon_of(md, birth);
      r.w = w;  // at the package's end: escaped, killed or truncated with this weight
      p.rec[job.rec_base + (int64_t)(j / (uint64_t)p.rec_stride)] = r;
    }
  }
  flush_tallies(p, job.esc_slot, T, t_emit, c_pk, c_pk != 0);
}

// Packages split off in the FP64 form, one per lane, from where they were split.
__global__ __launch_bounds__(256) void split_fp64_kernel(const TraceParams p, const Split64* __restrict__ in,
                                                         const uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  Tally64 T;
  int esc_slot = 0;
  const bool followed = i < n && in[i].job >= 0;
  if (followed) {
    const Split64 q = in[i];
    const JobDev& job = p.jobs[q.job];
    const ModelDev& md = p.models[job.model];
    const Dims D = dims_of(md);
    const ChildPlain ch{p.child};
    Pk64 k;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      k.P[b] = q.P[b];
      k.d[b] = q.d[b];
      k.I[b] = q.I[b];
    }
    k.node = q.node;
    k.lev = q.lev;
    double w = q.w, tau = q.tau;
    // its cell was counted by the package it split from
    uint32_t crossings = 0, ev = q.ev;
    int mlev = q.mlev;
    (void)follow64<true>(p, q.job, job, md, D, ch, q.pid, q.br, k, w, q.w0, tau, crossings, ev, mlev, T);
    T.cross += crossings;
    esc_slot = job.esc_slot;
  }
  // a wave's packages may belong to different jobs: escapes are added lane by lane
  if (T.esc != 0.0) unsafeAtomicAdd(p.esc + esc_slot, T.esc);
  T.esc = 0.0;
  flush_tallies(p, esc_slot, T, 0.0, 0, followed);
}

}  // namespace

hipError_t launch_trace_fp64(const TraceParams& p, int job, uint64_t n, int block, hipStream_t s) {
  const uint64_t grid = (n + block - 1) / block;
  if (p.split_n > 1) hipLaunchKernelGGL(trace_fp64_kernel<true>, dim3((unsigned)grid), dim3(block), 0, s, p, job);
  else hipLaunchKernelGGL(trace_fp64_kernel<false>, dim3((unsigned)grid), dim3(block), 0, s, p, job);
  return hipGetLastError();
}

hipError_t launch_split_fp64(const TraceParams& p, const Split64* in, uint64_t n, int block, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint64_t grid = (n + block - 1) / block;
  hipLaunchKernelGGL(split_fp64_kernel, dim3((unsigned)grid), dim3(block), 0, s, p, in, n);
  return hipGetLastError();
}
