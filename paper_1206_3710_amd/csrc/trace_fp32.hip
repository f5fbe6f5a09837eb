// FP32-local form of the Monte Carlo formal solution (paper Sect. 2.3), batched over all jobs
// (sources x wavelengths x models) in one persistent launch.
//
// * Packet queue: each wave takes packet ids from one global counter with a single atomic
//   and refills only the lanes whose packets ended.
// * Wave-level compaction of divergent work: lanes that reach a scattering event or finish wait
//   while the others keep crossing cells; the wave services the waiting lanes together once
//   fewer than `refill_thr` of its live lanes are still crossing, so the expensive event and
//   emission code runs for many lanes at once instead of stalling every crossing step.
// * Positions are local coordinates x in [0,1]^3 of the current cell, in FP32: the paper's
//   Sect. 2.3 tracking "in local grid coordinates where a cell has size one", carried down to
//   single cells.  Descent x -> 2x - b is exact; when a crossing lands in a coarser cell the
//   lateral coordinates are recovered in FP64 from the segment origin O (kept in FP64 since
//   the last emission or scattering) and the exact face coordinate.
// * One 4-byte load per visited node: the density word doubles as the subgrid identification
//   entry (negative = refined).
// * Deposits go straight to FP64 accumulators (one per node, or per (wavelength, node) when
//   per-wavelength output is asked for); the final reduction to canonical order is a separate
//   pass.
#include "device.h"

using namespace rtd;

namespace {

enum : int { ST_EMIT = 0, ST_CROSS = 1, ST_EVENT = 2, ST_DEAD = 3 };

// Crossings after which a packet is retired as truncated (guards the kernel's termination).
constexpr uint32_t kMaxCrossings = 1u << 30;
// Ascents that start at this level or deeper re-derive the lateral coordinates in FP64.
constexpr int kRecoverLevel = 2;

__device__ __forceinline__ float pow2f(int e) { return __int_as_float((127 + e) << 23); }
__device__ __forceinline__ float clamp01(float v) { return fminf(fmaxf(v, 0.0f), 1.0f); }

template <int BS>
__global__ __launch_bounds__(BS) void trace_fp32_kernel(const TraceParams p) {
  __shared__ uint64_t s_start[RT_JOBS_LDS];
  __shared__ double s_esc[RT_ESC_LDS];
  __shared__ double s_misc[4];
  const int tid = threadIdx.x;
  const bool jobs_lds = p.n_jobs <= RT_JOBS_LDS;
  const bool esc_lds = p.n_esc <= RT_ESC_LDS;
  if (jobs_lds)
    for (int i = tid; i < p.n_jobs; i += BS) s_start[i] = p.jobs[i].start;
  if (esc_lds)
    for (int i = tid; i < p.n_esc; i += BS) s_esc[i] = 0.0;
  if (tid < 4) s_misc[tid] = 0.0;
  __syncthreads();

  const int lane = tid & 63;
  const ChildWord cw{p.word};
  const float rr_thr = (float)p.rr_thr, rr_p = (float)p.rr_p;
  const float rr_gain = rr_p > 0.0f ? 1.0f / (1.0f - rr_p) : 1.0f;

  int state = ST_EMIT;
  int32_t node = 0, lev = 0, I0 = 0, I1 = 0, I2 = 0, birth = 0;
  float x0 = 0.f, x1 = 0.f, x2 = 0.f, d0 = 0.f, d1 = 0.f, d2 = 1.f;
  float n0 = 0.f, n1 = 0.f, n2 = -1.f, c0 = INFINITY, c1 = INFINITY, c2 = 1.f;
  float w = 0.f, w0 = 0.f, tau = 0.f, rho = 0.f;
  double O0 = 0.0, O1 = 0.0, O2 = 0.0;
  uint32_t pid = 0, ev = 0, ncross = 0;
  int job = 0;
  float ks = 0.f, ka = 0.f, g = 0.f;  // scattering / absorption opacity per root-cell length per unit density
  uint32_t stream = 0;
  int64_t acc_off = 0;
  int esc_slot = 0;
  Dims D{1, 1, 1, 0};

  unsigned long long c_cross = 0;
  uint32_t c_scat = 0, c_kill = 0, c_trunc = 0, c_pk = 0;
  double t_emit = 0.0;

  for (;;) {
    // ---------------- refill: one atomic per wave ----------------
    const uint64_t need = __ballot(state == ST_EMIT);
    if (need) {
      uint32_t blo = 0, bhi = 0;
      if (lane == 0) {
        const unsigned long long b = atomicAdd(p.counter, (unsigned long long)__popcll(need));
        blo = (uint32_t)b;
        bhi = (uint32_t)(b >> 32);
      }
      blo = __shfl(blo, 0, 64);
      bhi = __shfl(bhi, 0, 64);
      if (state == ST_EMIT) {
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(need >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
        const uint64_t gid = (((uint64_t)bhi << 32) | blo) + rank;
        if (gid >= p.total_packets) {
          state = ST_DEAD;
        } else {
          int lo = 0, hi = p.n_jobs - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            const uint64_t st = jobs_lds ? s_start[mid] : p.jobs[mid].start;
            if (st <= gid) lo = mid;
            else hi = mid - 1;
          }
          job = lo;
          const JobDev& J = p.jobs[job];
          const ModelDev& md = p.models[J.model];
          pid = (uint32_t)(gid - J.start);
          D = dims_of(md);
          ks = J.kc32 * J.alb32;
          ka = J.kc32 - ks;
          g = J.g32;
          stream = J.stream;
          acc_off = J.acc_off;
          esc_slot = J.esc_slot;
          Pk64 k;
          emit64(p, J, D, md.n_leaves, md.leaf_base, pid, k, cw, p.key0, p.key1);
          node = k.node;
          lev = k.lev;
          I0 = k.I[0];
          I1 = k.I[1];
          I2 = k.I[2];
          birth = node;
          const double sc = ldexp(1.0, lev);
          x0 = clamp01((float)(k.P[0] * sc - (double)I0));
          x1 = clamp01((float)(k.P[1] * sc - (double)I1));
          x2 = clamp01((float)(k.P[2] * sc - (double)I2));
          O0 = k.P[0];
          O1 = k.P[1];
          O2 = k.P[2];
          d0 = (float)k.d[0];
          d1 = (float)k.d[1];
          d2 = (float)k.d[2];
          exit_coef(d0, n0, c0);
          exit_coef(d1, n1, c1);
          exit_coef(d2, n2, c2);
          w0 = (float)k.w0;
          w = w0;
          tau = (float)k.tau;
          t_emit += k.w0;
          ++c_pk;
          ev = 0;
          ncross = 1;
          rho = __int_as_float(p.word[node]);
          state = ST_CROSS;
        }
      }
    }
    const uint64_t live = __ballot(state != ST_DEAD);
    if (!live) break;
    const int want = max(1, (int)(p.refill_thr * (float)__popcll(live)));

    // ---------------- crossing phase ----------------
    for (;;) {
      if (state == ST_CROSS) {
        // density times the cell size in root-cell units (local lengths are in cell units)
        const float f = ldexpf(rho, -lev);
        const float ss = ks * f;
        const float sa = ka * f;
        const float tx = fmaf(x0, n0, c0);
        const float ty = fmaf(x1, n1, c1);
        const float tz = fmaf(x2, n2, c2);
        const float texit = fminf(tx, fminf(ty, tz));
        const int ax = tx == texit ? 0 : (ty == texit ? 1 : 2);  // ties to the lowest axis
        const float tsc = ss * texit;
        const bool event = ss > 0.0f && tau <= tsc;
        const float s = event ? tau * __builtin_amdgcn_rcpf(ss) : texit;
        if (!event) tau -= tsc;
        const float de = w * one_minus_exp(sa * s);
        if (de > 0.0f) {
          // FP64 accumulators: a point source deposits every packet's first segment in one
          // cell, far more terms than an FP32 running sum can add without stalling
          unsafeAtomicAdd(p.acc64 + acc_off + node, (double)de);
          w -= de;
        }
        x0 = clamp01(fmaf(s, d0, x0));
        x1 = clamp01(fmaf(s, d1, x1));
        x2 = clamp01(fmaf(s, d2, x2));
        if (event) {
          state = ST_EVENT;
        } else {
          const int sg = sel3(ax, d0, d1, d2) > 0.0f ? 1 : -1;
          const int L = lev;
          const int32_t Io0 = I0, Io1 = I1, Io2 = I2;
          int32_t I[3] = {I0, I1, I2};
          int32_t raw;
          if (!cross_walk(D, p.up, ax, sg, node, lev, I, raw, cw)) {
            // escape through the root boundary
            if (esc_lds) unsafeAtomicAdd(&s_esc[esc_slot], (double)w);
            else unsafeAtomicAdd(p.esc + esc_slot, (double)w);
            if (p.rec_stride > 0 && (pid % (uint32_t)p.rec_stride) == 0) {
              const JobDev& J = p.jobs[job];
              const ModelDev& md = p.models[J.model];
              rt_record r{0u, ncross, ev, 0u, -1, canon_of(md, birth), (double)w};
              p.rec[J.rec_base + pid / (uint32_t)p.rec_stride] = r;
            }
            c_cross += ncross;
            state = ST_EMIT;
          } else {
            I0 = I[0];
            I1 = I[1];
            I2 = I[2];
            const float nearf = sg > 0 ? 0.0f : 1.0f;
            if (lev < L) {
              // coarser neighbour: lateral coordinates scale into the bigger cell
              const int kk = L - lev;
              const int32_t mask = (1 << kk) - 1;
              const float scl = pow2f(-kk);
              x0 = ax == 0 ? nearf : (x0 + (float)(Io0 & mask)) * scl;
              x1 = ax == 1 ? nearf : (x1 + (float)(Io1 & mask)) * scl;
              x2 = ax == 2 ? nearf : (x2 + (float)(Io2 & mask)) * scl;
              if (L >= kRecoverLevel) {
                // FP64 recovery from the segment origin and the exact face coordinate
                const double hf = ldexp(1.0, -lev), inv = ldexp(1.0, lev);
                const double F = (double)(sel3(ax, I0, I1, I2) + (sg > 0 ? 0 : 1)) * hf;
                const double t = (F - sel3(ax, O0, O1, O2)) / (double)sel3(ax, d0, d1, d2);
                if (ax != 0) x0 = clamp01((float)(fma(t, (double)d0, O0) * inv - (double)I0));
                if (ax != 1) x1 = clamp01((float)(fma(t, (double)d1, O1) * inv - (double)I1));
                if (ax != 2) x2 = clamp01((float)(fma(t, (double)d2, O2) * inv - (double)I2));
              }
            } else {
              x0 = ax == 0 ? nearf : x0;
              x1 = ax == 1 ? nearf : x1;
              x2 = ax == 2 ? nearf : x2;
              int32_t c = ChildWord::child_of(raw);
              while (c >= 0) {
                // refined neighbour: near side on the crossing axis, midpoint elsewhere
                const int b0 = ax == 0 ? (sg > 0 ? 0 : 1) : (x0 >= 0.5f ? 1 : 0);
                const int b1 = ax == 1 ? (sg > 0 ? 0 : 1) : (x1 >= 0.5f ? 1 : 0);
                const int b2 = ax == 2 ? (sg > 0 ? 0 : 1) : (x2 >= 0.5f ? 1 : 0);
                x0 = 2.0f * x0 - (float)b0;
                x1 = 2.0f * x1 - (float)b1;
                x2 = 2.0f * x2 - (float)b2;
                I0 = 2 * I0 + b0;
                I1 = 2 * I1 + b1;
                I2 = 2 * I2 + b2;
                node = c + (b0 | (b1 << 1) | (b2 << 2));
                ++lev;
                raw = p.word[node];
                c = ChildWord::child_of(raw);
              }
            }
            rho = __int_as_float(raw);
            if (++ncross >= kMaxCrossings) {
              ev = (uint32_t)p.max_events;  // retire as truncated at the event stage
              state = ST_EVENT;
            }
          }
        }
      }
      if (__popcll(__ballot(state == ST_CROSS)) < want) break;
    }

    // ---------------- scattering events, serviced together ----------------
    if (state == ST_EVENT) {
      ++ev;
      if ((int64_t)ev > p.max_events) {
        ++c_trunc;
        unsafeAtomicAdd(&s_misc[2], (double)w);
        if (p.rec_stride > 0 && (pid % (uint32_t)p.rec_stride) == 0) {
          const JobDev& J = p.jobs[job];
          const ModelDev& md = p.models[J.model];
          rt_record r{2u, ncross, ev, 0u, canon_of(md, node), canon_of(md, birth), (double)w};
          p.rec[J.rec_base + pid / (uint32_t)p.rec_stride] = r;
        }
        c_cross += ncross;
        state = ST_EMIT;
      } else {
        ++c_scat;
        const double h = ldexp(1.0, -lev);
        O0 = ((double)I0 + (double)x0) * h;
        O1 = ((double)I1 + (double)x1) * h;
        O2 = ((double)I2 + (double)x2) * h;
        const uint4 xr = philox(pid, stream, ev, 0u, p.key0, p.key1);
        bool killed = false;
        if (rr_p > 0.0f && w < rr_thr * w0) {
          if (unif32(xr.x) < rr_p) {
            ++c_kill;
            unsafeAtomicAdd(&s_misc[0], (double)w);
            if (p.rec_stride > 0 && (pid % (uint32_t)p.rec_stride) == 0) {
              const JobDev& J = p.jobs[job];
              const ModelDev& md = p.models[J.model];
              rt_record r{1u, ncross, ev, 0u, canon_of(md, node), canon_of(md, birth), (double)w};
              p.rec[J.rec_base + pid / (uint32_t)p.rec_stride] = r;
            }
            c_cross += ncross;
            state = ST_EMIT;
            killed = true;
          } else {
            const float nw = w * rr_gain;
            unsafeAtomicAdd(&s_misc[1], (double)nw - (double)w);
            w = nw;
          }
        }
        if (!killed) {
          float mu, st;
          hg_angle32(g, unif32(xr.y), mu, st);
          rotate32(d0, d1, d2, mu, st, kTwoPiF * unif32(xr.z));
          exit_coef(d0, n0, c0);
          exit_coef(d1, n1, c1);
          exit_coef(d2, n2, c2);
          tau = -logf(unif32(xr.w));
          state = ST_CROSS;
        }
      }
    }
  }

  // ---------------- tallies: one atomic per wave, then the block's LDS slots ----------------
  const unsigned long long sc_cross = wave_sum_u64(c_cross);
  const unsigned long long sc_scat = wave_sum_u64(c_scat);
  const unsigned long long sc_kill = wave_sum_u64(c_kill);
  const unsigned long long sc_trunc = wave_sum_u64(c_trunc);
  const unsigned long long sc_pk = wave_sum_u64(c_pk);
  const double st_emit = wave_sum(t_emit);
  if (lane == 0 && sc_pk > 0) {
    atomicAdd(&p.stats->crossings, sc_cross);
    atomicAdd(&p.stats->scatterings, sc_scat);
    if (sc_kill) atomicAdd(&p.stats->kills, sc_kill);
    if (sc_trunc) atomicAdd(&p.stats->truncated, sc_trunc);
    atomicAdd(&p.stats->packets, sc_pk);
    unsafeAtomicAdd(&p.stats->e_emit, st_emit);
  }
  __syncthreads();
  if (esc_lds)
    for (int i = tid; i < p.n_esc; i += BS)
      if (s_esc[i] != 0.0) unsafeAtomicAdd(p.esc + i, s_esc[i]);
  if (tid == 0) {
    if (s_misc[0] != 0.0) unsafeAtomicAdd(&p.stats->e_killed, s_misc[0]);
    if (s_misc[1] != 0.0) unsafeAtomicAdd(&p.stats->e_rr_gain, s_misc[1]);
    if (s_misc[2] != 0.0) unsafeAtomicAdd(&p.stats->e_trunc, s_misc[2]);
  }
}

}  // namespace

hipError_t launch_trace_fp32(const TraceParams& p, int grid, int block, hipStream_t s) {
  switch (block) {
    case 64: hipLaunchKernelGGL(trace_fp32_kernel<64>, dim3(grid), dim3(64), 0, s, p); break;
    case 128: hipLaunchKernelGGL(trace_fp32_kernel<128>, dim3(grid), dim3(128), 0, s, p); break;
    case 256: hipLaunchKernelGGL(trace_fp32_kernel<256>, dim3(grid), dim3(256), 0, s, p); break;
    case 512: hipLaunchKernelGGL(trace_fp32_kernel<512>, dim3(grid), dim3(512), 0, s, p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t occupancy_trace_fp32(int block, int* blocks_per_cu) {
  switch (block) {
    case 64: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, trace_fp32_kernel<64>, 64, 0);
    case 128: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, trace_fp32_kernel<128>, 128, 0);
    case 256: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, trace_fp32_kernel<256>, 256, 0);
    case 512: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, trace_fp32_kernel<512>, 512, 0);
    default: return hipErrorInvalidValue;
  }
}
