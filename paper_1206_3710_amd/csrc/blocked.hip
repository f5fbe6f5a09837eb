// Grid-by-grid form of the FP32-local transport (paper Sect. 3.4 and App. A: the model is
// processed one grid at a time so that the grid's data stay in fast memory, and packets that
// leave a grid wait in the neighbouring grid's boundary array).
//
// On gfx950 a "grid" is a region: a brick of root cells and all their descendants, small enough
// that its node words and its absorbed-energy accumulators live in LDS.  A workgroup takes a
// work item (a region and a run of packets queued for it), loads the region into LDS, follows
// each packet with LDS lookups and LDS atomic deposits until the packet leaves the region,
// escapes or ends, and finally adds the LDS accumulators to the region-major FP32 accumulators
// with coalesced atomics.  Packets leaving the region are appended to the next sweep's queue
// (96-byte records); each sweep's queue is put in (wavelength slot, region) order on the device
// (sweep.hip) and sweeps repeat until the queue is empty, new packets streaming in at every
// sweep.
#include "device.h"

using namespace rtd;

namespace {

// lane states; B_SPLIT / B_ROUL: just crossed into a deeper / shallower leaf with package
// splitting on (Sect. 2.3), waiting for the split or the exit roulette; B_FAR: at a face whose
// neighbour is not in the leaf's own brick or oct, waiting for the phase that walks the tree
enum : int { B_EMPTY = 0, B_CROSS = 1, B_EVENT = 2, B_DONE = 3, B_EXIT = 4, B_SPLIT = 5, B_ROUL = 6, B_FAR = 7 };

constexpr uint32_t kMaxCrossings = 1u << 30;
constexpr int kRecoverLevel = 2;
constexpr int kEscLds = 256;

__device__ __forceinline__ float pow2f(int e) { return __int_as_float((127 + e) << 23); }
__device__ __forceinline__ float clamp01(float v) { return fminf(fmaxf(v, 0.0f), 1.0f); }

__device__ __forceinline__ int32_t child_of(int32_t w) { return w < 0 ? ~w : -1; }

__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Region holding the cell reached from the root along level-L coordinates J (a birth leaf,
// or the neighbour across a face).  Below level L (a coarse cell entering a split cell through
// face ax with sign sg) the child is picked as the landing picks it: the near side on the
// crossing axis, the midpoint on the others (y: local coordinates in the level-L cell).
__device__ __forceinline__ int32_t region_walk(const BlkParams& b, const Dims& D, int L, int32_t J0, int32_t J1,
                                               int32_t J2, int ax, int sg, float y0, float y1, float y2) {
  int32_t e = b.root_region[D.root(J0 >> L, J1 >> L, J2 >> L)];
  int l = 0;
  while (e < 0) {
    ++l;
    int oc;
    if (l <= L) {
      const int sh = L - l;
      oc = ((J0 >> sh) & 1) | (((J1 >> sh) & 1) << 1) | (((J2 >> sh) & 1) << 2);
    } else {
      const int b0 = ax == 0 ? (sg > 0 ? 0 : 1) : (y0 >= 0.5f ? 1 : 0);
      const int b1 = ax == 1 ? (sg > 0 ? 0 : 1) : (y1 >= 0.5f ? 1 : 0);
      const int b2 = ax == 2 ? (sg > 0 ? 0 : 1) : (y2 >= 0.5f ? 1 : 0);
      y0 = 2.0f * y0 - (float)b0;
      y1 = 2.0f * y1 - (float)b1;
      y2 = 2.0f * y2 - (float)b2;
      oc = b0 | (b1 << 1) | (b2 << 2);
    }
    e = b.split_tab[(size_t)(~e) * 8 + oc];
  }
  return e;
}

// ------------------------------------------------------------------------------------------
// emission into the queue (run by the pass kernel's blocks once the sweep's work items are
// taken: the births fill the tail of the pass)
// ------------------------------------------------------------------------------------------
// Birth of packet gid (global index over the trace's jobs) into record gid - g0 of the next
// queue, which the sweep reserved for its births.  s_start: the jobs' first packet indices in
// LDS when jobs_lds.
__device__ __forceinline__ void emit_one(const BlkParams& b, uint64_t gid, uint64_t g0,
                                         const uint64_t* s_start, bool jobs_lds, double& e_emit,
                                         unsigned long long& npk, uint32_t k0, uint32_t k1) {
  const TraceParams& p = b.t;
  int lo = 0, hi = p.n_jobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const uint64_t st = jobs_lds ? s_start[mid] : p.jobs[mid].start;
    if (st <= gid) lo = mid;
    else hi = mid - 1;
  }
  const JobDev& J = p.jobs[lo];
  const uint64_t idx = gid - g0;
  if (J.kind == RT_SRC_DUST && J.qtot == 0) {
    // a wavelength at which no cell emits (its table total is only known on the device in a
    // captured iteration step): no packet, and the record is skipped by the sort
    b.u_key[idx] = kInvalidKey;
    return;
  }
  const ModelDev& md = p.models[J.model];
  const Dims D = dims_of(md);
  const uint32_t pid = (uint32_t)(gid - J.start);
  Pk64 k;
  emit64(p, J, D, md.n_leaves, md.leaf_base, pid, k, ChildWord{p.word}, k0, k1);
  PRec r;
  const double sc = ldexp(1.0, k.lev);
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    r.I[q] = k.I[q];
    r.x[q] = clamp01((float)(k.P[q] * sc - (double)k.I[q]));
    r.d[q] = (float)k.d[q];
    r.O[q] = k.P[q];
  }
  r.lev = (uint8_t)k.lev;
  r.ax = 0;
  r.sg = 0;
  // subiterations: the shallowest level visited starts at the birth cell's (0 for the external
  // field, which enters through the root grid) and is the slot of the queue key
  const uint32_t mslot = b.lvl_slots > 0 ? (J.kind == RT_SRC_BACKGROUND ? 0u : (uint32_t)k.lev) : (uint32_t)J.slot;
  r.flag = b.lvl_slots > 0 ? (uint8_t)(mslot << 2) : 0;
  r.w0 = (float)k.w0;
  r.w = r.w0;
  r.tau = (float)k.tau;
  r.birth = k.node;
  r.pid = pid;
  r.job = lo;
  r.ev = 0;
  r.ncross = 1;
  const uint32_t key = mslot * (uint32_t)b.n_regions +
                       (uint32_t)region_walk(b, D, k.lev, k.I[0], k.I[1], k.I[2], -1, 1, 0.5f, 0.5f, 0.5f);
  e_emit += k.w0;
  ++npk;
  if (p.emit_acc && J.kind == RT_SRC_DUST)
    unsafeAtomicAdd(p.emit_acc + md.canon_base + canon_of(md, k.node), k.w0);
  b.u_out[idx] = r;
  b.u_key[idx] = key;
}

template <typename WF>
__device__ __forceinline__ void descend_loop(WF word_of, int ax, int sg, float& x0, float& x1, float& x2,
                                             int32_t& I0, int32_t& I1, int32_t& I2, int32_t& cur, int& l,
                                             int32_t& r);

// A queue record read as six 16-byte loads issued together (read field by field, the byte
// fields came as separate narrow loads, one of them only after the others had arrived).
__device__ __forceinline__ PRec load_rec(const PRec* __restrict__ src) {
  const uint4* __restrict__ v = reinterpret_cast<const uint4*>(src);
  uint4 t[sizeof(PRec) / 16];
#pragma unroll
  for (int k = 0; k < (int)(sizeof(PRec) / 16); ++k) t[k] = v[k];
  // (keeps the compiler from narrowing the loads to the fields each branch reads)
#pragma unroll
  for (int k = 0; k < (int)(sizeof(PRec) / 16); ++k)
    asm volatile("" : "+v"(t[k].x), "+v"(t[k].y), "+v"(t[k].z), "+v"(t[k].w));
  PRec r;
  __builtin_memcpy(&r, t, sizeof r);
  return r;
}

// Entering a neighbour at the packet's own level (word r of cell cur at level l): coordinate
// ax goes to the near face; while the cell is refined, step into the child on that face and,
// on the other axes, into the half holding the packet (the midpoint rule).
template <typename WF>
__device__ __forceinline__ void descend(WF word_of, int ax, int sg, float& x0, float& x1, float& x2,
                                        int32_t& I0, int32_t& I1, int32_t& I2, int32_t& cur, int& l,
                                        int32_t& r) {
  const float nearf = sg > 0 ? 0.0f : 1.0f;
  x0 = ax == 0 ? nearf : x0;
  x1 = ax == 1 ? nearf : x1;
  x2 = ax == 2 ? nearf : x2;
  descend_loop(word_of, ax, sg, x0, x1, x2, I0, I1, I2, cur, l, r);
}

// The walk of descend without the face reset: nothing happens while r is a leaf's word.
template <typename WF>
__device__ __forceinline__ void descend_loop(WF word_of, int ax, int sg, float& x0, float& x1, float& x2,
                                             int32_t& I0, int32_t& I1, int32_t& I2, int32_t& cur, int& l,
                                             int32_t& r) {
  int32_t c = child_of(r);
  while (c >= 0) {
    const int b0 = ax == 0 ? (sg > 0 ? 0 : 1) : (x0 >= 0.5f ? 1 : 0);
    const int b1 = ax == 1 ? (sg > 0 ? 0 : 1) : (x1 >= 0.5f ? 1 : 0);
    const int b2 = ax == 2 ? (sg > 0 ? 0 : 1) : (x2 >= 0.5f ? 1 : 0);
    x0 = 2.0f * x0 - (float)b0;
    x1 = 2.0f * x1 - (float)b1;
    x2 = 2.0f * x2 - (float)b2;
    I0 = 2 * I0 + b0;
    I1 = 2 * I1 + b1;
    I2 = 2 * I2 + b2;
    cur = c + (b0 | (b1 << 1) | (b2 << 2));
    ++l;
    r = word_of(cur);
    c = child_of(r);
  }
}


// Land in the neighbour after a face crossing: from cell `cur` at level l (an ancestor-level
// cell containing the neighbour J of the old cell Io at level L), descend along J's bits; a
// coarser landing cell rescales the lateral local coordinates (recovered in FP64 from the
// segment origin), a finer one descends by the near-side / midpoint rule.
template <class WF>
__device__ __forceinline__ void land(WF word_of, int ax, int sg, int L, int32_t Io0, int32_t Io1,
                                     int32_t Io2, int32_t J0, int32_t J1, int32_t J2, int32_t cur, int l,
                                     float& x0, float& x1, float& x2, double O0, double O1, double O2,
                                     float d0, float d1, float d2, int32_t& node, int32_t& lev,
                                     int32_t& I0, int32_t& I1, int32_t& I2, int32_t& raw) {
  int32_t r = word_of(cur);
  while (l < L && child_of(r) >= 0) {
    ++l;
    const int sh = L - l;
    cur = child_of(r) + (((J0 >> sh) & 1) | (((J1 >> sh) & 1) << 1) | (((J2 >> sh) & 1) << 2));
    r = word_of(cur);
  }
  const int sh = L - l;
  I0 = J0 >> sh;
  I1 = J1 >> sh;
  I2 = J2 >> sh;
  const float nearf = sg > 0 ? 0.0f : 1.0f;
  if (l < L) {
    const int kk = L - l;
    const int32_t mask = (1 << kk) - 1;
    const float scl = pow2f(-kk);
    x0 = ax == 0 ? nearf : (x0 + (float)(Io0 & mask)) * scl;
    x1 = ax == 1 ? nearf : (x1 + (float)(Io1 & mask)) * scl;
    x2 = ax == 2 ? nearf : (x2 + (float)(Io2 & mask)) * scl;
    if (L >= kRecoverLevel) {
      const double hf = ldexp(1.0, -l), inv = ldexp(1.0, l);
      const double F = (double)(sel3(ax, I0, I1, I2) + (sg > 0 ? 0 : 1)) * hf;
      const double t = (F - sel3(ax, O0, O1, O2)) / (double)sel3(ax, d0, d1, d2);
      if (ax != 0) x0 = clamp01((float)(fma(t, (double)d0, O0) * inv - (double)I0));
      if (ax != 1) x1 = clamp01((float)(fma(t, (double)d1, O1) * inv - (double)I1));
      if (ax != 2) x2 = clamp01((float)(fma(t, (double)d2, O2) * inv - (double)I2));
    }
  } else {
    descend(word_of, ax, sg, x0, x1, x2, I0, I1, I2, cur, l, r);
  }
  node = cur;
  lev = l;
  raw = r;
}

// One work item: follow every queued packet of the item through its region.  FITS: the whole
// region is in LDS (pure LDS lookups and deposits); otherwise nodes past the LDS capacity are
// read and deposited in global memory.  SPLIT: package splitting is on (split_n > 1); the
// unsplit instance carries none of its state or code.  PEEL: scattering events are kept for
// the peel-off.  ALI: the self-absorption of dust-emission packets is tallied for the
// accelerated Lambda iteration.  LVL: subiterations (Sect. 3.1, App. B): deposits go to the
// array of the shallowest level the package has visited (its `mlev`, which is also the slot of
// its queue key, so that a work item's LDS sums belong to one array), and with a subtree set a
// package that would cross out of it ends there as escaped.
template <bool FITS, bool SPLIT, bool PEEL, bool ALI, bool LVL>
__device__ __forceinline__ void run_item(const BlkParams& b, const WorkItem& it, const RegionDev& R,
                                         const ModelDev& md, const Dims D, int nloc, int nup,
                                         int32_t* s_word, float* s_acc, int32_t* s_up, uint32_t* s_next,
                                         double* s_esc, double* s_misc, bool esc_lds, int lane,
                                         unsigned long long& c_cross, uint32_t& c_scat, uint32_t& c_kill,
                                         uint32_t& c_trunc, uint32_t& c_split, uint32_t& c_skill,
                                         uint32_t& c_sskip, uint64_t& ch_base, uint32_t& ch_used,
                                         const uint32_t k0, const uint32_t k1) {
  const TraceParams& p = b.t;
  const float rr_thr = (float)p.rr_thr, rr_p = (float)p.rr_p;
  const float rr_gain = rr_p > 0.0f ? 1.0f / (1.0f - rr_p) : 1.0f;
  const int bx = R.hi[0] - R.lo[0], by = R.hi[1] - R.lo[1];
  // (opaque to the compiler, which would otherwise rebuild a brick-level stride as a multiply)
  const int bxy = __builtin_amdgcn_readfirstlane(bx * by);
  double* __restrict__ gacc64 = b.accb64 + (int64_t)it.slot * b.accb_stride + R.gbase;
  const int32_t* __restrict__ gword = b.rword + R.gbase;
  const int32_t* __restrict__ gup = b.rup + (R.gbase >> 3);
  auto word_of = [&](int32_t l) -> int32_t {
    if (FITS) return s_word[l];
    return l < nloc ? s_word[l] : gword[l];
  };
  auto up_of = [&](int32_t l) -> int32_t {
    if (FITS) return s_up[l >> 3];
    return (l >> 3) < nup ? s_up[l >> 3] : gup[l >> 3];
  };
  int mlev = 0;                // shallowest level visited (LVL)
  auto deposit = [&](int32_t l, float v) {
    // a package whose shallowest level dropped below the item's slot during the item deposits
    // straight into its own array
    if (LVL && mlev != it.slot) unsafeAtomicAdd(b.accb64 + (int64_t)mlev * b.accb_stride + R.gbase + l, (double)v);
    else if (FITS || l < nloc) atomicAdd(&s_acc[l], v);
    else unsafeAtomicAdd(gacc64 + l, (double)v);
  };
  int state = B_EMPTY;
  int32_t node = 0, lev = 0, I0 = 0, I1 = 0, I2 = 0, birth = 0, job = 0;
  float x0 = 0.f, x1 = 0.f, x2 = 0.f, d0 = 0.f, d1 = 0.f, d2 = 1.f;
  float n0 = 0.f, n1 = 0.f, n2 = -1.f, c0 = INFINITY, c1 = INFINITY, c2 = 1.f;
  float w = 0.f, w0 = 0.f, tau = 0.f, rho = 0.f;
  double O0 = 0.0, O1 = 0.0, O2 = 0.0;
  uint32_t pid = 0, ev = 0, ncross = 0, stream = 0;
  uint32_t br = 0;             // branch identifier (0: the package as emitted)
  bool dust_lane = false;      // the packet comes from dust emission
  constexpr bool self_on = ALI;
  constexpr bool splitting = SPLIT;
  // the grid of a cell (Sect. 2.3) is that of its ancestor at level sdep when it is deeper
  const int sdep = SPLIT ? p.split_depth : 0;
  float ks = 0.f, ka = 0.f, g = 0.f;  // scattering / absorption opacity per root-cell length per unit density
  int esc_slot = 0;
  int32_t xax = 0, xsg = 0;
  bool xpark = false;          // re-queued in this region without crossing a face
  bool pool_done = false;      // this item's packets are all taken (wave-uniform)
  int tail_it = 0;             // crossing rounds since then (wave-uniform)
  const uint32_t own_key = (uint32_t)it.slot * (uint32_t)b.n_regions + (uint32_t)it.region;

  // A crossing whose neighbour is not in the leaf's own brick or oct: ascend to the common
  // ancestor, leave the region or the model, or land in the neighbour (subiterations send every
  // crossing here: it tests the subtree and tallies the flow between levels).
  auto far_cross = [&](const int ax, const int sg) {
    const int32_t Ia = sel3(ax, I0, I1, I2);
    const int32_t Ja = Ia + sg;
    const int L = lev;
    // a subiteration follows packages only inside its subtree: crossing out of it ends
    // them as escaped (the test on the neighbour at the old level is exact, since the
    // subtree root is refined and the packet is below it)
    const bool sub_out = LVL && p.sub_lev >= 0 &&
                         !in_subtree(p.sub_lev, p.sub_I, L, ax == 0 ? Ja : I0, ax == 1 ? Ja : I1,
                                     ax == 2 ? Ja : I2);
    // automatic iteration: the weight leaving each refined ancestor's subtree (only when the
    // crossing leaves the leaf's oct), walked up the tree's global parent links
    if (LVL && p.flux_acc && (Ja >> 1) != (Ia >> 1) && L > 0) {
      const int32_t c = b.rcanon[R.gbase + node];
      const int32_t inode = md.base + (c < md.n_root ? c : c + (md.n_root_pad - md.n_root));
      flux_exits(md, p.up, p.flux_acc, inode, L, Ia, Ja, Ja < 0 || Ja >= (D.na(ax) << L), (double)w);
    }
    if (Ja < 0 || Ja >= (D.na(ax) << L) || sub_out) {
      // escape through the root boundary (or out of the subtree)
      // a region belongs to one model: its escapes are tallied per wavelength in LDS
      if (esc_lds) atomicAdd(&s_esc[esc_slot - (int)md.lam_base], (double)w);
      else unsafeAtomicAdd(p.esc + esc_slot, (double)w);
      if (p.rec_stride > 0 && br == 0 && (pid % (uint32_t)p.rec_stride) == 0) {
        const JobDev& J = p.jobs[job];
        rt_record rc{0u, ncross, ev, 0u, -1, canon_of(md, birth), (double)w};
        p.rec[J.rec_base + pid / (uint32_t)p.rec_stride] = rc;
      }
      c_cross += ncross;
      state = B_EMPTY;
    } else {
      int32_t cur = node;
      int l = L;
      while (l > R.rl && ((Ja >> (L - l + 1)) != (Ia >> (L - l + 1)))) {
        cur = up_of(cur);
        --l;
      }
      const int32_t J0 = ax == 0 ? Ja : I0, J1 = ax == 1 ? Ja : I1, J2 = ax == 2 ? Ja : I2;
      bool leave = false;
      if (l == R.rl) {
        const int sh = L - R.rl;
        const int32_t R0 = J0 >> sh, R1 = J1 >> sh, R2 = J2 >> sh;
        if (R0 < R.lo[0] || R0 >= R.hi[0] || R1 < R.lo[1] || R1 >= R.hi[1] || R2 < R.lo[2] ||
            R2 >= R.hi[2]) {
          // the neighbour lies in another region: its region is looked up when the record
          // is written, outside the crossing loop
          leave = true;
          xax = ax;
          xsg = sg;
          state = B_EXIT;
        } else {
          cur = (R0 - R.lo[0]) + bx * ((R1 - R.lo[1]) + by * (R2 - R.lo[2]));
        }
      } else {
        cur += sg > 0 ? (1 << ax) : -(1 << ax);
      }
      if (!leave) {
        int32_t raw;
        land(word_of, ax, sg, L, I0, I1, I2, J0, J1, J2, cur, l, x0, x1, x2, O0, O1, O2, d0, d1, d2,
             node, lev, I0, I1, I2, raw);
        rho = __int_as_float(raw);
        if (LVL && lev < mlev) mlev = lev;
        if (++ncross >= kMaxCrossings) {
          ev = (uint32_t)p.max_events;
          state = B_EVENT;
        } else if (splitting && min(lev, sdep) != min(L, sdep)) {
          state = lev > L ? B_SPLIT : B_ROUL;
        }
      }
    }
  };

  for (;;) {
    // ---------------- refill from this item's queue ----------------
    const uint64_t need = __ballot(state == B_EMPTY);
    if (need) {
      uint32_t base = 0;
      if (lane == 0) base = atomicAdd(s_next, (uint32_t)__popcll(need));
      base = __shfl(base, 0, 64);
      if (base + (uint32_t)__popcll(need) >= it.count) pool_done = true;
      if (state == B_EMPTY) {
        const uint32_t idx = base + lane_rank(need);
        if (idx >= it.count) {
          state = B_DONE;
        } else {
          const PRec rec = load_rec(b.q_in + b.q_perm[it.start + idx]);
          job = rec.job;
          const JobDev& J = p.jobs[job];
          ks = J.kc32 * J.alb32;
          ka = J.kc32 - ks;
          g = J.g32;
          stream = J.stream;
          esc_slot = J.esc_slot;
          dust_lane = J.kind == RT_SRC_DUST;
          x0 = rec.x[0];
          x1 = rec.x[1];
          x2 = rec.x[2];
          d0 = rec.d[0];
          d1 = rec.d[1];
          d2 = rec.d[2];
          exit_coef(d0, n0, c0);
          exit_coef(d1, n1, c1);
          exit_coef(d2, n2, c2);
          w = rec.w;
          w0 = rec.w0;
          tau = rec.tau;
          O0 = rec.O[0];
          O1 = rec.O[1];
          O2 = rec.O[2];
          pid = rec.pid;
          ev = rec.ev;
          ncross = rec.ncross;
          birth = rec.birth;
          br = (SPLIT && (rec.flag & 2)) ? (uint32_t)rec.birth : 0u;
          if (LVL) mlev = rec.flag >> 2;
          const bool crossing = rec.flag & 1;
          const int L = rec.lev;
          int32_t J0 = rec.I[0], J1 = rec.I[1], J2 = rec.I[2];
          int ax = 0, sg = 1;
          if (crossing) {
            ax = rec.ax;
            sg = rec.sg ? -1 : 1;
            if (ax == 0) J0 += sg;
            else if (ax == 1) J1 += sg;
            else J2 += sg;
          }
          // the cell of this region's brick (level R.rl) that holds the packet
          int Lj = L;  // level of J
          if (L < R.rl) {
            // entering a split cell from a coarser neighbour: descend to the brick's level as
            // the landing would (near side on the crossing axis, midpoint on the others)
            x0 = ax == 0 ? (sg > 0 ? 0.0f : 1.0f) : x0;
            x1 = ax == 1 ? (sg > 0 ? 0.0f : 1.0f) : x1;
            x2 = ax == 2 ? (sg > 0 ? 0.0f : 1.0f) : x2;
            for (int l = L + 1; l <= R.rl; ++l) {
              const int b0 = ax == 0 ? (sg > 0 ? 0 : 1) : (x0 >= 0.5f ? 1 : 0);
              const int b1 = ax == 1 ? (sg > 0 ? 0 : 1) : (x1 >= 0.5f ? 1 : 0);
              const int b2 = ax == 2 ? (sg > 0 ? 0 : 1) : (x2 >= 0.5f ? 1 : 0);
              x0 = 2.0f * x0 - (float)b0;
              x1 = 2.0f * x1 - (float)b1;
              x2 = 2.0f * x2 - (float)b2;
              J0 = 2 * J0 + b0;
              J1 = 2 * J1 + b1;
              J2 = 2 * J2 + b2;
            }
            Lj = R.rl;
          }
          const int shr = Lj - R.rl;
          const int32_t R0 = J0 >> shr, R1 = J1 >> shr, R2 = J2 >> shr;
          const int32_t rootl = (R0 - R.lo[0]) + bx * ((R1 - R.lo[1]) + by * (R2 - R.lo[2]));
          int32_t raw = 0;
          const bool misplaced = (L < R.rl && !crossing) || R0 < R.lo[0] || R0 >= R.hi[0] || R1 < R.lo[1] ||
                                 R1 >= R.hi[1] || R2 < R.lo[2] || R2 >= R.hi[2];
          if (misplaced) {
            // a record queued for the wrong region breaks the schedule's invariant: it is
            // dropped and counted, and the call reports the count as a device error
            atomicAdd(&s_misc[6], 1.0);
          } else if (crossing) {
            land(word_of, ax, sg, Lj, rec.I[0], rec.I[1], rec.I[2], J0, J1, J2, rootl, R.rl, x0, x1, x2, O0,
                 O1, O2, d0, d1, d2, node, lev, I0, I1, I2, raw);
            ++ncross;
          } else {
            // birth: walk down to the birth leaf along its coordinates
            int32_t cur = rootl;
            int32_t rr = word_of(cur);
            for (int l = R.rl + 1; l <= L && child_of(rr) >= 0; ++l) {
              const int sh = L - l;
              cur = child_of(rr) + (((J0 >> sh) & 1) | (((J1 >> sh) & 1) << 1) | (((J2 >> sh) & 1) << 2));
              rr = word_of(cur);
            }
            node = cur;
            lev = L;
            I0 = J0;
            I1 = J1;
            I2 = J2;
            raw = rr;
          }
          rho = __int_as_float(raw);
          if (LVL && lev < mlev) mlev = lev;
          state = misplaced ? B_EMPTY : B_CROSS;
          if (!misplaced && crossing && splitting && min(lev, sdep) != min(L, sdep))
            state = lev > L ? B_SPLIT : B_ROUL;
        }
      }
    }
    const uint64_t live = __ballot(state != B_DONE);
    if (!live) break;
    const int want = max(1, (int)(p.refill_thr * (float)__popcll(live)));

    // ---------------- crossing phase (LDS lookups, LDS deposits) ----------------
    for (;;) {
      if (state == B_CROSS) {
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
        if (FITS) {
          deposit(node, de);
          w -= de;
        } else if (de > 0.0f) {
          deposit(node, de);
          w -= de;
        }
        // accelerated Lambda iteration: what a dust-emission packet absorbs in its birth cell
        // before it first leaves it (a package split off later starts its count at 0 in another
        // cell, so only the package as emitted, branch 0, is counted)
        if (self_on && ncross == 1u && br == 0u && dust_lane && de > 0.0f)
          unsafeAtomicAdd(p.self_acc + md.canon_base + b.rcanon[R.gbase + node], (double)de);
        x0 = clamp01(fmaf(s, d0, x0));
        x1 = clamp01(fmaf(s, d1, x1));
        x2 = clamp01(fmaf(s, d2, x2));
        const int sg = sel3(ax, d0, d1, d2) > 0.0f ? 1 : -1;
        const int32_t Ia = sel3(ax, I0, I1, I2);
        const int32_t Ja = Ia + sg;
        // the common crossing: into the neighbour in the same brick (at the region's brick level)
        // or in the same oct (below it).  Its local id is one stride away, so no tree walk and no
        // brick lookup; a refined neighbour is descended as landing does.
        const bool at_brick = lev == R.rl;
        const bool in_brick = (Ja >= sel3(ax, R.lo[0], R.lo[1], R.lo[2])) & (Ja < sel3(ax, R.hi[0], R.hi[1], R.hi[2]));
        const bool in_oct = (Ja >> 1) == (Ia >> 1);
        const bool near_move = !LVL && (at_brick ? in_brick : in_oct);
        if (LVL) {
          if (event) state = B_EVENT;
          else far_cross(ax, sg);
        } else {
          // one path for every lane, with selects: a lane that moves (nm) takes the neighbour
          // and its word, the others keep their cell and re-read its word, which is a leaf's, so
          // the walk down does nothing for them
          const bool nm = !event && near_move;
          const int L = lev;
          const int32_t stride = at_brick ? sel3(ax, 1, bx, bxy) : (1 << ax);
          const float nearf = sg > 0 ? 0.0f : 1.0f;
          I0 = nm && ax == 0 ? Ja : I0;
          I1 = nm && ax == 1 ? Ja : I1;
          I2 = nm && ax == 2 ? Ja : I2;
          x0 = nm && ax == 0 ? nearf : x0;
          x1 = nm && ax == 1 ? nearf : x1;
          x2 = nm && ax == 2 ? nearf : x2;
          node += nm ? (sg > 0 ? stride : -stride) : 0;
          int32_t raw = word_of(node);
          descend_loop(word_of, ax, sg, x0, x1, x2, I0, I1, I2, node, lev, raw);
          rho = __int_as_float(raw);
          // (the guard on the crossing count is tested on the far crossings: between two of them
          // a packet crosses at most the cells of one brick along a straight line)
          ncross += nm ? 1u : 0u;
          xax = ax;
          xsg = sg;
          // a lane that does not move either stops at its event, or leaves the brick at its level
          // into the model (no tree walk: the record is written in the exit phase), or waits for
          // the far-crossing phase
          // (the root extent as sel3: written as D.na(ax) it compiled to a three-way branch here)
          const int s_exit = ((L == R.rl) & (Ja >= 0) & (Ja < (sel3(ax, D.n0, D.n1, D.n2) << L))) ? B_EXIT : B_FAR;
          const int s_near = splitting && min(lev, sdep) != min(L, sdep) ? B_SPLIT : B_CROSS;
          state = event ? B_EVENT : (nm ? s_near : s_exit);
        }
      }
      if (pool_done && ++tail_it >= b.tail_park) break;
      if (__popcll(__ballot(state == B_CROSS)) < want) break;
    }

    // ---------------- crossings that walk the tree, serviced together ----------------
    if (!LVL && __ballot(state == B_FAR)) {
      if (state == B_FAR) {
        state = B_CROSS;
        far_cross(xax, xsg);
      }
    }

    // ---------------- packets leaving the region: append to the next queue ----------------
    // the item's queue is empty and the wave has been finishing its last packets for a while:
    // re-queue the ones still crossing (for this same region, next sweep) so that the block
    // does not wait for a few long histories
    if (pool_done && tail_it >= b.tail_park && state == B_CROSS) {
      state = B_EXIT;
      xpark = true;
    }
    const uint64_t ex = __ballot(state == B_EXIT);
    if (ex) {
      // the wave writes into its own chunk of kExitChunk records of the next queue and takes a
      // new one from the shared counter only when the chunk runs out
      const uint32_t n_ex = (uint32_t)__popcll(ex);
      const uint32_t left = kExitChunk - ch_used;
      uint64_t nb = 0;
      if (n_ex > left) {
        uint32_t blo = 0, bhi = 0;
        if (lane == 0) {
          const unsigned long long base = atomicAdd(b.u_count, (unsigned long long)kExitChunk);
          blo = (uint32_t)base;
          bhi = (uint32_t)(base >> 32);
        }
        // lane 0 is active here (the phase is wave-uniform): the cursor stays in scalar registers
        blo = (uint32_t)__builtin_amdgcn_readfirstlane((int)blo);
        bhi = (uint32_t)__builtin_amdgcn_readfirstlane((int)bhi);
        nb = ((uint64_t)bhi << 32) | blo;
      }
      if (state == B_EXIT) {
        const uint32_t r = lane_rank(ex);
        const uint64_t idx = r < left ? ch_base + ch_used + r : nb + (r - left);
        PRec rc;
        rc.I[0] = I0;
        rc.I[1] = I1;
        rc.I[2] = I2;
        rc.lev = (uint8_t)lev;
        rc.ax = (uint8_t)xax;
        rc.sg = xsg > 0 ? 0 : 1;
        rc.flag = (xpark ? 0 : 1) | (br ? 2 : 0) | (LVL ? mlev << 2 : 0);
        rc.x[0] = x0;
        rc.x[1] = x1;
        rc.x[2] = x2;
        rc.d[0] = d0;
        rc.d[1] = d1;
        rc.d[2] = d2;
        rc.w = w;
        rc.w0 = w0;
        rc.tau = tau;
        rc.birth = br ? (int32_t)br : birth;
        rc.O[0] = O0;
        rc.O[1] = O1;
        rc.O[2] = O2;
        rc.pid = pid;
        rc.job = job;
        rc.ev = ev;
        rc.ncross = ncross;
        b.u_out[idx] = rc;
        const uint32_t kslot = LVL ? (uint32_t)mlev : (uint32_t)it.slot;
        uint32_t key = LVL ? kslot * (uint32_t)b.n_regions + (uint32_t)it.region : own_key;
        if (!xpark) {
          const int32_t K0 = I0 + (xax == 0 ? xsg : 0), K1 = I1 + (xax == 1 ? xsg : 0), K2 = I2 + (xax == 2 ? xsg : 0);
          key = kslot * (uint32_t)b.n_regions +
                (uint32_t)region_walk(b, D, lev, K0, K1, K2, xax, xsg, x0, x1, x2);
        }
        b.u_key[idx] = key;
        xpark = false;
        state = B_EMPTY;
      }
      if (n_ex > left) {
        ch_base = nb;
        ch_used = n_ex - left;
      } else {
        ch_used += n_ex;
      }
    }

    // ---------------- package splitting at subgrid entry, roulette at exit (Sect. 2.3) ----------------
    if (splitting && __ballot(state == B_SPLIT || state == B_ROUL)) {
      const uint32_t N = (uint32_t)p.split_n;
      if (state == B_ROUL) {
        // survives with probability 1/N: (2 m + 1) 2^-24 < 1/N  <=>  (2 m + 1) N < 2^24
        const uint4 xr = philox(pid, stream, ncross, (br << 2) | 3u, k0, k1);
        if ((2u * (xr.x >> 9) + 1u) * (uint64_t)N < (1ull << 24)) {
          const float nw = w * (float)N;
          atomicAdd(&s_misc[4], (double)nw - (double)w);
          w = nw;
          state = B_CROSS;
        } else {
          ++c_skill;
          atomicAdd(&s_misc[3], (double)w);
          if (p.rec_stride > 0 && br == 0 && (pid % (uint32_t)p.rec_stride) == 0) {
            const JobDev& J = p.jobs[job];
            rt_record rc{3u, ncross, ev, 0u, (int64_t)b.rcanon[R.gbase + node], canon_of(md, birth), (double)w};
            p.rec[J.rec_base + pid / (uint32_t)p.rec_stride] = rc;
          }
          c_cross += ncross;
          state = B_EMPTY;
        }
      }
      const uint64_t sm = __ballot(state == B_SPLIT);
      if (sm) {
        // N - 1 new packages per splitting lane, in the region's own queue for the next sweep;
        // a wave takes them from the sweep's split room, or skips splits that do not fit
        const uint32_t per = N - 1u;
        const uint32_t nsplit = (uint32_t)__popcll(sm);
        uint32_t n_ok = 0, blo = 0, bhi = 0;
        if (lane == 0) {
          const unsigned long long used = atomicAdd(b.split_used, (unsigned long long)nsplit * per);
          const unsigned long long room = *b.split_room;
          const unsigned long long fit = used < room ? (room - used) / per : 0ull;
          n_ok = fit < nsplit ? (uint32_t)fit : nsplit;
          if (n_ok) {
            const unsigned long long base = atomicAdd(b.u_count, (unsigned long long)n_ok * per);
            blo = (uint32_t)base;
            bhi = (uint32_t)(base >> 32);
          }
        }
        n_ok = __shfl(n_ok, 0, 64);
        blo = __shfl(blo, 0, 64);
        bhi = __shfl(bhi, 0, 64);
        if (state == B_SPLIT) {
          const uint32_t r = lane_rank(sm);
          if (r < n_ok) {
            const float wn = w / (float)N;
            uint64_t idx = (((uint64_t)bhi << 32) | blo) + (uint64_t)r * per;
            PRec rc;
            rc.I[0] = I0;
            rc.I[1] = I1;
            rc.I[2] = I2;
            rc.lev = (uint8_t)lev;
            rc.ax = 0;
            rc.sg = 0;
            rc.flag = (uint8_t)(2 | (LVL ? mlev << 2 : 0));
            rc.x[0] = x0;
            rc.x[1] = x1;
            rc.x[2] = x2;
            rc.d[0] = d0;
            rc.d[1] = d1;
            rc.d[2] = d2;
            rc.w = wn;
            rc.w0 = w0;
            rc.O[0] = O0;
            rc.O[1] = O1;
            rc.O[2] = O2;
            rc.pid = pid;
            rc.job = job;
            rc.ev = ev;
            rc.ncross = 0;
            for (uint32_t c = 1; c < N; ++c, ++idx) {
              const uint32_t bc = branch_id(br, ncross, c);
              const uint4 xr = philox(pid, stream, ncross, (bc << 2) | 2u, k0, k1);
              rc.tau = -logf(unif32(xr.x));
              rc.birth = (int32_t)bc;
              b.u_out[idx] = rc;
              // subiterations: a split-off package keeps the shallowest level of its parent
              b.u_key[idx] = LVL ? (uint32_t)mlev * (uint32_t)b.n_regions + (uint32_t)it.region : own_key;
            }
            w = wn;
            ++c_split;
          } else {
            ++c_sskip;
          }
          state = B_CROSS;
        }
      }
    }

    // ---------------- scattering events, serviced together ----------------
    if (state == B_EVENT) {
      ++ev;
      if ((int64_t)ev > p.max_events) {
        ++c_trunc;
        atomicAdd(&s_misc[2], (double)w);
        if (p.rec_stride > 0 && br == 0 && (pid % (uint32_t)p.rec_stride) == 0) {
          const JobDev& J = p.jobs[job];
          rt_record rc{2u, ncross, ev, 0u, (int64_t)b.rcanon[R.gbase + node], canon_of(md, birth), (double)w};
          p.rec[J.rec_base + pid / (uint32_t)p.rec_stride] = rc;
        }
        c_cross += ncross;
        state = B_EMPTY;
      } else {
        ++c_scat;
        const double h = ldexp(1.0, -lev);
        O0 = ((double)I0 + (double)x0) * h;
        O1 = ((double)I1 + (double)x1) * h;
        O2 = ((double)I2 + (double)x2) * h;
        if (PEEL) {
          // kept for the peel-off, with the weight before the event roulette (one reservation
          // per wave)
          const uint64_t pm = __ballot(1);
          const int leader = __builtin_ctzll(pm);
          uint32_t plo = 0, phi = 0;
          if (lane == leader) {
            const unsigned long long base = atomicAdd(p.peel_count, (unsigned long long)__popcll(pm));
            plo = (uint32_t)base;
            phi = (uint32_t)(base >> 32);
          }
          plo = __shfl(plo, leader, 64);
          phi = __shfl(phi, leader, 64);
          const uint64_t idx = (((uint64_t)phi << 32) | plo) + lane_rank(pm);
          if (idx < p.peel_cap) {
            PeelEv e;
            e.P[0] = O0;
            e.P[1] = O1;
            e.P[2] = O2;
            e.d[0] = (double)d0;
            e.d[1] = (double)d1;
            e.d[2] = (double)d2;
            e.w = (double)w;
            const int32_t c = b.rcanon[R.gbase + node];
            e.node = md.base + (c < md.n_root ? c : c + (md.n_root_pad - md.n_root));
            e.job = job;
            e.I[0] = I0;
            e.I[1] = I1;
            e.I[2] = I2;
            e.lev = lev;
            p.peel_ev[idx] = e;
          }
        }
        const uint4 xr = philox(pid, stream, ev, br << 2, k0, k1);
        bool killed = false;
        if (rr_p > 0.0f && w < rr_thr * w0) {
          if (unif32(xr.x) < rr_p) {
            ++c_kill;
            atomicAdd(&s_misc[0], (double)w);
            if (p.rec_stride > 0 && br == 0 && (pid % (uint32_t)p.rec_stride) == 0) {
              const JobDev& J = p.jobs[job];
              rt_record rc{1u, ncross, ev, 0u, (int64_t)b.rcanon[R.gbase + node], canon_of(md, birth), (double)w};
              p.rec[J.rec_base + pid / (uint32_t)p.rec_stride] = rc;
            }
            c_cross += ncross;
            state = B_EMPTY;
            killed = true;
          } else {
            const float nw = w * rr_gain;
            atomicAdd(&s_misc[1], (double)nw - (double)w);
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
          state = B_CROSS;
        }
      }
    }
  }
}

template <int BS, bool SPLIT, bool PEEL, bool ALI, bool LVL>
__global__ __launch_bounds__(BS) void blk_pass_kernel(const BlkParams b) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int cap = b.cap;
  int32_t* s_word = reinterpret_cast<int32_t*>(smem);
  float* s_acc = reinterpret_cast<float*>(smem + 4 * (size_t)cap);
  int32_t* s_up = reinterpret_cast<int32_t*>(smem + 8 * (size_t)cap);
  __shared__ int s_item;
  __shared__ uint32_t s_next;
  __shared__ double s_misc[7];  // killed, roulette gain, truncated, split-killed, split gain,
                                // emitted, misplaced records (a count)
  __shared__ unsigned long long s_npk;
  __shared__ double s_esc[kEscLds];
  const TraceParams& p = b.t;
  const int tid = threadIdx.x, lane = tid & 63;
  if (tid < 7) s_misc[tid] = 0.0;
  if (tid == 0) s_npk = 0;
  unsigned long long c_cross = 0;
  uint32_t c_scat = 0, c_kill = 0, c_trunc = 0, c_split = 0, c_skill = 0, c_sskip = 0;
  uint64_t ch_base = 0;          // this wave's chunk of next-queue records (none yet: full)
  uint32_t ch_used = kExitChunk;
  // Philox key: from the parameters, or from device memory in a captured iteration step (whose
  // key changes from step to step)
  const uint32_t k0 = p.keys ? p.keys[0] : p.key0;
  const uint32_t k1 = p.keys ? p.keys[1] : p.key1;

  for (;;) {
    __syncthreads();
    if (tid == 0) s_item = (int)atomicAdd(b.item_counter, 1u);
    __syncthreads();
    const uint32_t item = (uint32_t)s_item;
    if (item >= *b.n_items) break;
    const WorkItem it = b.items[item];
    const RegionDev R = b.regions[it.region];
    const ModelDev& md = p.models[R.model];
    const Dims D = dims_of(md);
    const int nloc = min(R.n, cap);
    const int nup = (nloc + 7) >> 3;
    const bool esc_lds = md.nl <= kEscLds;
    // the region's words and parent links: U loads per thread are issued before their LDS
    // stores, so a region costs a few global latencies instead of one per element
    {
      constexpr int U = 8;
      const int32_t* __restrict__ gw = b.rword + R.gbase;
      const int32_t* __restrict__ gu = b.rup + (R.gbase >> 3);
      for (int i0 = tid; i0 < nloc; i0 += BS * U) {
        int32_t v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = i0 + u * BS < nloc ? gw[i0 + u * BS] : 0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (i0 + u * BS < nloc) {
            s_word[i0 + u * BS] = v[u];
            s_acc[i0 + u * BS] = 0.0f;
          }
        }
      }
      for (int i0 = tid; i0 < nup; i0 += BS * U) {
        int32_t v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = i0 + u * BS < nup ? gu[i0 + u * BS] : 0;
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (i0 + u * BS < nup) s_up[i0 + u * BS] = v[u];
      }
    }
    if (esc_lds)
      for (int i = tid; i < md.nl; i += BS) s_esc[i] = 0.0;
    if (tid == 0) s_next = 0;
    __syncthreads();
    if (R.n <= cap)
      run_item<true, SPLIT, PEEL, ALI, LVL>(b, it, R, md, D, nloc, nup, s_word, s_acc, s_up, &s_next, s_esc, s_misc, esc_lds, lane,
                     c_cross, c_scat, c_kill, c_trunc, c_split, c_skill, c_sskip, ch_base, ch_used, k0, k1);
    else
      run_item<false, SPLIT, PEEL, ALI, LVL>(b, it, R, md, D, nloc, nup, s_word, s_acc, s_up, &s_next, s_esc, s_misc, esc_lds, lane,
                      c_cross, c_scat, c_kill, c_trunc, c_split, c_skill, c_sskip, ch_base, ch_used, k0, k1);
    __syncthreads();
    {
      double* __restrict__ gacc64 = b.accb64 + (int64_t)it.slot * b.accb_stride + R.gbase;
      for (int i = tid; i < nloc; i += BS) {
        const float v = s_acc[i];
        if (v != 0.0f) unsafeAtomicAdd(gacc64 + i, (double)v);
      }
    }
    if (esc_lds)
      for (int i = tid; i < md.nl; i += BS)
        if (s_esc[i] != 0.0) unsafeAtomicAdd(p.esc + md.lam_base + i, s_esc[i]);
  }

  // this sweep's births, in chunks of BS packets, once every work item is taken
  {
    const uint64_t g0 = b.sweep->e0, g1 = g0 + b.sweep->ne;
    if (g1 > g0) {
      uint64_t* s_start = reinterpret_cast<uint64_t*>(smem);  // the region's LDS is free now
      const bool jobs_lds = p.n_jobs <= RT_JOBS_LDS && p.n_jobs <= b.cap;
      __syncthreads();
      if (jobs_lds)
        for (int i = tid; i < p.n_jobs; i += BS) s_start[i] = p.jobs[i].start;
      double e_emit = 0.0;
      unsigned long long npk = 0;
      for (;;) {
        __syncthreads();
        if (tid == 0) s_item = (int)atomicAdd(b.emit_counter, 1u);
        __syncthreads();
        const uint64_t base = g0 + (uint64_t)(uint32_t)s_item * BS;
        if (base >= g1) break;
        if (base + (uint64_t)tid < g1) emit_one(b, base + (uint64_t)tid, g0, s_start, jobs_lds, e_emit, npk, k0, k1);
      }
      e_emit = wave_sum(e_emit);
      npk = wave_sum_u64(npk);
      if (lane == 0 && npk) {
        atomicAdd(&s_misc[5], e_emit);
        atomicAdd(&s_npk, npk);
      }
    }
  }

  // the unused end of the wave's chunk holds no packets: the next sweep's sort skips it
  for (uint32_t j = ch_used + (uint32_t)lane; j < kExitChunk; j += 64) b.u_key[ch_base + j] = kInvalidKey;

  const unsigned long long sc_cross = wave_sum_u64(c_cross);
  const unsigned long long sc_scat = wave_sum_u64(c_scat);
  const unsigned long long sc_kill = wave_sum_u64(c_kill);
  const unsigned long long sc_trunc = wave_sum_u64(c_trunc);
  if (lane == 0) {
    if (sc_cross) atomicAdd(&p.stats->crossings, sc_cross);
    if (sc_scat) atomicAdd(&p.stats->scatterings, sc_scat);
    if (sc_kill) atomicAdd(&p.stats->kills, sc_kill);
    if (sc_trunc) atomicAdd(&p.stats->truncated, sc_trunc);
  }
  if (SPLIT) {
    const unsigned long long sc_split = wave_sum_u64(c_split);
    const unsigned long long sc_skill = wave_sum_u64(c_skill);
    const unsigned long long sc_sskip = wave_sum_u64(c_sskip);
    if (lane == 0) {
      if (sc_split) atomicAdd(&p.stats->splits, sc_split);
      if (sc_skill) atomicAdd(&p.stats->split_kills, sc_skill);
      if (sc_sskip) atomicAdd(&p.stats->split_skips, sc_sskip);
    }
  }
  __syncthreads();
  if (tid == 0) {
    if (s_misc[0] != 0.0) unsafeAtomicAdd(&p.stats->e_killed, s_misc[0]);
    if (s_misc[1] != 0.0) unsafeAtomicAdd(&p.stats->e_rr_gain, s_misc[1]);
    if (s_misc[2] != 0.0) unsafeAtomicAdd(&p.stats->e_trunc, s_misc[2]);
    if (s_misc[3] != 0.0) unsafeAtomicAdd(&p.stats->e_split_killed, s_misc[3]);
    if (s_misc[4] != 0.0) unsafeAtomicAdd(&p.stats->e_split_gain, s_misc[4]);
    if (s_misc[6] != 0.0) atomicAdd(&p.stats->misplaced, (unsigned long long)s_misc[6]);
    if (s_npk) {
      unsafeAtomicAdd(&p.stats->e_emit, s_misc[5]);
      atomicAdd(&p.stats->packets, s_npk);
    }
  }
}

// Region-major FP64 accumulators -> canonical outputs (one block row per region).  Slots: one
// (wavelength-integrated), one per wavelength of the model (per-wavelength output, also written
// to e_lam_node), or one per level (subiterations: the level arrays go to lvl_out).  Each node's
// slots are summed into e_node.
__global__ __launch_bounds__(256) void blk_reduce_kernel(const ModelDev* __restrict__ models,
                                                         const RegionDev* __restrict__ regions,
                                                         const int32_t* __restrict__ rcanon,
                                                         const double* __restrict__ accb64, int64_t stride,
                                                         int n_slots, double* __restrict__ e_node,
                                                         double* __restrict__ e_lam_node,
                                                         double* __restrict__ lvl_out, int64_t lvl_stride,
                                                         double* __restrict__ e_total) {
  __shared__ double s_part[4];
  const RegionDev& R = regions[blockIdx.y];
  const ModelDev& m = models[R.model];
  const int32_t l = blockIdx.x * 256 + threadIdx.x;
  double sum = 0.0;
  if (l < R.n) {
    const int64_t gidx = R.gbase + l;
    const int32_t c = rcanon[gidx];
    if (c >= 0) {
      const int ns = lvl_out ? n_slots : (n_slots > 1 ? m.nl : 1);
      for (int s = 0; s < ns; ++s) {
        const double v = accb64[s * stride + gidx];
        sum += v;
        if (lvl_out) lvl_out[s * lvl_stride + m.canon_base + c] = v;
        if (e_lam_node) e_lam_node[m.lamnode_base + (int64_t)s * m.n_nodes + c] = v;
      }
      if (e_node) e_node[m.canon_base + c] = sum;
    }
  }
  sum = wave_sum(sum);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double t = s_part[0] + s_part[1] + s_part[2] + s_part[3];
    if (t != 0.0) unsafeAtomicAdd(e_total, t);
  }
}

}  // namespace

// Instances: any combination of splitting and peel-off, the accelerated-iteration tally with or
// without splitting (the peel-off never runs inside a Lambda iteration), and the per-level
// arrays of subiterations on their own.
template <bool SPLIT, bool PEEL, bool ALI, bool LVL>
static const void* pass_fn(int block) {
  switch (block) {
    case 256: return (const void*)blk_pass_kernel<256, SPLIT, PEEL, ALI, LVL>;
    case 512: return (const void*)blk_pass_kernel<512, SPLIT, PEEL, ALI, LVL>;
    case 768: return (const void*)blk_pass_kernel<768, SPLIT, PEEL, ALI, LVL>;
    case 1024: return (const void*)blk_pass_kernel<1024, SPLIT, PEEL, ALI, LVL>;
    default: return nullptr;
  }
}

hipError_t attr_blk_pass(int block, int lds_bytes) {
  for (const void* f : {pass_fn<false, false, false, false>(block), pass_fn<true, false, false, false>(block),
                        pass_fn<false, true, false, false>(block), pass_fn<true, true, false, false>(block),
                        pass_fn<false, false, true, false>(block), pass_fn<true, false, true, false>(block),
                        pass_fn<false, false, false, true>(block), pass_fn<true, false, false, true>(block),
                        pass_fn<false, false, true, true>(block), pass_fn<true, false, true, true>(block)}) {
    if (!f) return hipErrorInvalidValue;
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <bool SPLIT, bool PEEL, bool ALI, bool LVL>
static hipError_t launch_pass(const BlkParams& b, int grid, int block, int lds_bytes, hipStream_t s) {
  switch (block) {
    case 256: hipLaunchKernelGGL((blk_pass_kernel<256, SPLIT, PEEL, ALI, LVL>), dim3(grid), dim3(256), lds_bytes, s, b); break;
    case 512: hipLaunchKernelGGL((blk_pass_kernel<512, SPLIT, PEEL, ALI, LVL>), dim3(grid), dim3(512), lds_bytes, s, b); break;
    case 768: hipLaunchKernelGGL((blk_pass_kernel<768, SPLIT, PEEL, ALI, LVL>), dim3(grid), dim3(768), lds_bytes, s, b); break;
    case 1024: hipLaunchKernelGGL((blk_pass_kernel<1024, SPLIT, PEEL, ALI, LVL>), dim3(grid), dim3(1024), lds_bytes, s, b); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_blk_pass(const BlkParams& b, int grid, int block, int lds_bytes, hipStream_t s) {
  const bool split = b.t.split_n > 1, peel = b.t.peel_ev != nullptr, ali = b.t.self_acc != nullptr;
  if (b.lvl_slots > 0) {
    // the per-level arrays need one FP64 accumulator slot per level; splitting and the
    // accelerated tally ride along
    if (peel || !b.accb64) return hipErrorInvalidValue;
    if (ali)
      return split ? launch_pass<true, false, true, true>(b, grid, block, lds_bytes, s)
                   : launch_pass<false, false, true, true>(b, grid, block, lds_bytes, s);
    return split ? launch_pass<true, false, false, true>(b, grid, block, lds_bytes, s)
                 : launch_pass<false, false, false, true>(b, grid, block, lds_bytes, s);
  }
  if (ali) {
    if (peel) return hipErrorInvalidValue;
    return split ? launch_pass<true, false, true, false>(b, grid, block, lds_bytes, s)
                 : launch_pass<false, false, true, false>(b, grid, block, lds_bytes, s);
  }
  if (split) return peel ? launch_pass<true, true, false, false>(b, grid, block, lds_bytes, s)
                         : launch_pass<true, false, false, false>(b, grid, block, lds_bytes, s);
  return peel ? launch_pass<false, true, false, false>(b, grid, block, lds_bytes, s)
              : launch_pass<false, false, false, false>(b, grid, block, lds_bytes, s);
}

hipError_t launch_blk_reduce(const ModelDev* models, const RegionDev* regions, int n_regions,
                             int32_t max_region_nodes, const int32_t* rcanon, const double* accb64,
                             int64_t stride, int n_slots, double* e_node, double* e_lam_node,
                             double* lvl_out, int64_t lvl_stride, double* e_total, hipStream_t s) {
  if (n_regions == 0) return hipSuccess;
  hipLaunchKernelGGL(blk_reduce_kernel, dim3((max_region_nodes + 255) / 256, n_regions), dim3(256), 0, s, models,
                     regions, rcanon, accb64, stride, n_slots, e_node, e_lam_node, lvl_out, lvl_stride, e_total);
  return hipGetLastError();
}
