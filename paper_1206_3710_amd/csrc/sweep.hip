// Device-driven sweeps of the region schedule (grid-by-grid processing, paper Sect. 3.4 and
// App. A).  Every size a sweep needs (queue lengths, the packets still to be emitted, the
// number of work items) lives in device memory, so a run of sweeps is a fixed sequence of
// launches: it is captured once as a HIP graph and replayed until the queues drain.
//
// One sweep, on queue buffer `in` (its records were appended during the previous sweep):
//   begin    pick this sweep's emission range and reserve its records in the other buffer
//   hist     count the records per key (slot * n_regions + region); with few enough keys each
//            block counts a contiguous range of records in LDS and writes its counts, and a
//            column scan turns them into the block's offsets within each key (no global atomic)
//   scan     exclusive offsets per key; cut each key's run into work items
//   scatter  record index -> its place in key order (the permutation the pass reads through)
//   pass     the region pass (blocked.hip) appends leaving packets to the other buffer, in
//            per-wave chunks (unused chunk ends carry kInvalidKey and are skipped here); its
//            blocks then write the sweep's births to the records begin reserved.
#include "device.h"

using namespace rtd;

namespace {

constexpr int kHistLds = kSortLdsKeys;  // keys counted in LDS (larger key sets use global atomics)
constexpr int kSortBS = 1024;            // threads per block of the block-histogram sort
constexpr int kSortPer = 8;              // records per thread per round of its loops
constexpr int kAgg = 4;          // distinct keys per wave counted with one atomic each (global counters)

// Add 1 per valid lane to cnt[key]; returns each lane's rank among the lanes (and earlier
// callers) with its key.  Lanes sharing one of the first AGG distinct keys of the wave are
// counted with a single atomic per key (queues are often dominated by a few regions, whose
// global counters would otherwise serialise); the remaining lanes use one atomic each.  LDS
// counters take AGG = 0: one LDS atomic per lane is cheaper than the wave's ballot rounds.
template <int AGG = kAgg>
__device__ __forceinline__ uint32_t agg_count(uint32_t* cnt, uint32_t key, bool valid) {
  if (AGG == 0) return valid ? atomicAdd(&cnt[key], 1u) : 0u;
  const int lane = threadIdx.x & 63;
  uint64_t todo = __ballot(valid);
  uint32_t rank = 0;
  bool done = !valid;
  for (int it = 0; it < AGG && todo; ++it) {
    const int leader = __builtin_ctzll(todo);
    const uint32_t kl = (uint32_t)__builtin_amdgcn_readlane((int)key, leader);
    const uint64_t same = __ballot(valid && key == kl) & todo;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(&cnt[kl], (uint32_t)__popcll(same));
    base = (uint32_t)__builtin_amdgcn_readlane((int)base, leader);
    if ((same >> lane) & 1ull) {
      rank = base + (uint32_t)__popcll(same & ((1ull << lane) - 1ull));
      done = true;
    }
    todo &= ~same;
  }
  if (!done) rank = atomicAdd(&cnt[key], 1u);
  return rank;
}

__global__ void sw_begin_kernel(SweepState* st, int in, int slot, uint64_t batch, uint64_t capq) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int out = 1 - in;
  const unsigned long long n_in = st->count[in];
  st->item_counter = 0;
  st->emit_counter = 0;
  st->n_items = 0;
  const unsigned long long rem = st->total - st->emitted;
  unsigned long long ne = rem < batch ? rem : batch;
  const unsigned long long room = capq > n_in ? capq - n_in : 0;
  if (ne > room) ne = room;
  // this sweep's births own the first ne records of the output buffer (packet e0 + i at i);
  // packets leaving their regions are appended after them
  st->count[out] = ne;
  st->e0 = st->emitted;
  st->ne = ne;
  st->emitted += ne;
  // split-off packages may use what the worst case of exits (every input packet) and this
  // sweep's births leave of the other buffer
  const unsigned long long need = n_in + ne;
  st->split_room = st->cap_all > need ? st->cap_all - need : 0;
  st->split_used = 0;
  st->n_in = n_in;
  st->log_in[slot] = n_in;
  if (n_in == 0 && ne == 0) st->done = 1u;
  if (n_in > 0) st->sweeps += 1u;
}

// The sweep state at the start of a trace: nothing queued or emitted yet (a kernel, so that a
// captured iteration step contains no host copy).
__global__ void sw_init_kernel(SweepState* st, unsigned long long total, unsigned long long cap_all) {
  unsigned long long* w = reinterpret_cast<unsigned long long*>(st);
  for (int i = threadIdx.x; i < (int)(sizeof(SweepState) / 8); i += blockDim.x) w[i] = 0ull;
  __syncthreads();
  if (threadIdx.x == 0) {
    st->total = total;
    st->cap_all = cap_all;
  }
}

__global__ void sw_zero_kernel(uint32_t* __restrict__ a, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) a[i] = 0u;
}

// Key counts with global atomics (key sets too large for LDS).
__global__ __launch_bounds__(256) void sw_hist_kernel(const uint32_t* __restrict__ keys,
                                                      const SweepState* __restrict__ st,
                                                      uint32_t* __restrict__ hist) {
  const uint64_t n = st->n_in;
  // whole waves iterate together (agg_count needs every lane of the wave); kPerH keys per
  // thread are loaded before any is counted, so that the loads overlap
  constexpr int kPerH = 8;
  const uint64_t span = (uint64_t)gridDim.x * 256 * kPerH;
  for (uint64_t t0 = (uint64_t)blockIdx.x * 256 * kPerH; t0 < n; t0 += span) {
    uint32_t kk[kPerH];
#pragma unroll
    for (int j = 0; j < kPerH; ++j) {
      const uint64_t i = t0 + (uint64_t)j * 256 + threadIdx.x;
      kk[j] = i < n ? keys[i] : kInvalidKey;
    }
#pragma unroll
    for (int j = 0; j < kPerH; ++j) {
      const bool v = kk[j] != kInvalidKey;  // unused records of a pass wave's last chunk
      (void)agg_count(hist, v ? kk[j] : 0u, v);
    }
  }
}

// One block: exclusive key offsets (written as scatter cursors) and the work items.
__global__ __launch_bounds__(1024) void sw_scan_kernel(const uint32_t* __restrict__ hist, int n_keys,
                                                       int n_regions, int chunk, uint32_t* __restrict__ kfill,
                                                       WorkItem* __restrict__ items, SweepState* st) {
  __shared__ uint32_t s_a[1024], s_b[1024];
  uint32_t carry_r = 0, carry_i = 0;
  const int t = threadIdx.x;
  for (int k0 = 0; k0 < n_keys; k0 += 1024) {
    const int k = k0 + t;
    const uint32_t cnt = k < n_keys ? hist[k] : 0u;
    const uint32_t nch = (cnt + (uint32_t)chunk - 1u) / (uint32_t)chunk;
    s_a[t] = cnt;
    s_b[t] = nch;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const uint32_t va = t >= o ? s_a[t - o] : 0u;
      const uint32_t vb = t >= o ? s_b[t - o] : 0u;
      __syncthreads();
      s_a[t] += va;
      s_b[t] += vb;
      __syncthreads();
    }
    const uint32_t start = carry_r + s_a[t] - cnt;
    const uint32_t ifirst = carry_i + s_b[t] - nch;
    if (k < n_keys) {
      kfill[k] = start;
      for (uint32_t c = 0; c < nch; ++c) {
        WorkItem w;
        w.region = k % n_regions;
        w.slot = k / n_regions;
        w.start = start + c * (uint32_t)chunk;
        w.count = min((uint32_t)chunk, cnt - c * (uint32_t)chunk);
        items[ifirst + c] = w;
      }
    }
    carry_r += s_a[1023];
    carry_i += s_b[1023];
    __syncthreads();
  }
  if (t == 0) st->n_items = carry_i;
}

// Record index -> position in key order, with global cursors (key sets too large for LDS).
__global__ __launch_bounds__(256) void sw_scatter_kernel(const uint32_t* __restrict__ keys,
                                                         const SweepState* __restrict__ st,
                                                         uint32_t* __restrict__ kfill,
                                                         uint32_t* __restrict__ perm) {
  const uint64_t n = st->n_in;
  const uint64_t span = (uint64_t)gridDim.x * 256;
  for (uint64_t i0 = (uint64_t)blockIdx.x * 256; i0 < n; i0 += span) {
    const uint64_t i = i0 + threadIdx.x;
    const uint32_t k = i < n ? keys[i] : kInvalidKey;
    const bool v = k != kInvalidKey;
    const uint32_t pos = agg_count(kfill, v ? k : 0u, v);
    if (v) perm[pos] = (uint32_t)i;
  }
}

// Records [lo, hi) of block b: whole rounds of kSortBS * kSortPer records, split evenly over the
// blocks.  The counting and the scatter kernels take the same ranges, so each block's counts
// are exactly the records it places.
__device__ __forceinline__ void block_range(uint64_t n, int b, int nb, uint64_t& lo, uint64_t& hi) {
  constexpr uint64_t kRound = (uint64_t)kSortBS * kSortPer;
  const uint64_t rounds = (n + kRound - 1) / kRound;
  const uint64_t per = (rounds + (uint64_t)nb - 1) / (uint64_t)nb;
  lo = min(n, (uint64_t)b * per * kRound);
  hi = min(n, (uint64_t)(b + 1) * per * kRound);
}

// Per-block key counts of the block's record range, written as row b of bh.
__global__ __launch_bounds__(kSortBS) void sw_bhist_kernel(const uint32_t* __restrict__ keys,
                                                           const SweepState* __restrict__ st,
                                                           uint32_t* __restrict__ bh, int n_keys) {
  __shared__ uint32_t s_h[kHistLds];
  for (int k = threadIdx.x; k < n_keys; k += kSortBS) s_h[k] = 0u;
  __syncthreads();
  uint64_t lo, hi;
  block_range(st->n_in, blockIdx.x, gridDim.x, lo, hi);
  for (uint64_t t0 = lo; t0 < hi; t0 += (uint64_t)kSortBS * kSortPer) {
    uint32_t kk[kSortPer];
#pragma unroll
    for (int j = 0; j < kSortPer; ++j) {
      const uint64_t i = t0 + (uint64_t)j * kSortBS + threadIdx.x;
      kk[j] = i < hi ? keys[i] : kInvalidKey;
    }
#pragma unroll
    for (int j = 0; j < kSortPer; ++j) {
      const bool v = kk[j] != kInvalidKey;
      (void)agg_count<0>(s_h, v ? kk[j] : 0u, v);
    }
  }
  __syncthreads();
  uint32_t* __restrict__ row = bh + (size_t)blockIdx.x * n_keys;
  for (int k = threadIdx.x; k < n_keys; k += kSortBS) row[k] = s_h[k];
}

// Per key: the blocks' counts become their exclusive offsets within the key, and hist the key's
// total.
__global__ __launch_bounds__(256) void sw_colscan_kernel(uint32_t* __restrict__ bh, int nb, int n_keys,
                                                         uint32_t* __restrict__ hist) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= n_keys) return;
  uint32_t run = 0;
  int b = 0;
  for (; b + 8 <= nb; b += 8) {
    uint32_t v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = bh[(size_t)(b + j) * n_keys + k];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      bh[(size_t)(b + j) * n_keys + k] = run;
      run += v[j];
    }
  }
  for (; b < nb; ++b) {
    const uint32_t v = bh[(size_t)b * n_keys + k];
    bh[(size_t)b * n_keys + k] = run;
    run += v;
  }
  hist[k] = run;
}

// Record index -> position in key order: the block's cursor for key k starts at the key's start
// plus the block's offset within it, and is advanced in LDS.
__global__ __launch_bounds__(kSortBS) void sw_bscatter_kernel(const uint32_t* __restrict__ keys,
                                                              const SweepState* __restrict__ st,
                                                              const uint32_t* __restrict__ kfill,
                                                              const uint32_t* __restrict__ bh,
                                                              uint32_t* __restrict__ perm, int n_keys) {
  __shared__ uint32_t s_c[kHistLds];
  const uint32_t* __restrict__ row = bh + (size_t)blockIdx.x * n_keys;
  for (int k = threadIdx.x; k < n_keys; k += kSortBS) s_c[k] = kfill[k] + row[k];
  __syncthreads();
  uint64_t lo, hi;
  block_range(st->n_in, blockIdx.x, gridDim.x, lo, hi);
  for (uint64_t t0 = lo; t0 < hi; t0 += (uint64_t)kSortBS * kSortPer) {
    uint32_t kk[kSortPer];
#pragma unroll
    for (int j = 0; j < kSortPer; ++j) {
      const uint64_t i = t0 + (uint64_t)j * kSortBS + threadIdx.x;
      kk[j] = i < hi ? keys[i] : kInvalidKey;
    }
#pragma unroll
    for (int j = 0; j < kSortPer; ++j) {
      const uint64_t i = t0 + (uint64_t)j * kSortBS + threadIdx.x;
      const bool v = kk[j] != kInvalidKey;
      const uint32_t pos = agg_count<0>(s_c, v ? kk[j] : 0u, v);
      if (v) perm[pos] = (uint32_t)i;
    }
  }
}

}  // namespace

hipError_t launch_sweep_sort(SweepState* st, int in, int slot, uint64_t batch, uint64_t capq, const uint32_t* keys,
                             int n_keys, int n_regions, int chunk, uint32_t* hist, uint32_t* kfill,
                             uint32_t* bhist, uint32_t* perm, WorkItem* items, int grid, hipStream_t s) {
  hipLaunchKernelGGL(sw_begin_kernel, dim3(1), dim3(64), 0, s, st, in, slot, batch, capq);
  if (n_keys <= kHistLds) {
    const int nb = kSortBlocks(grid);
    hipLaunchKernelGGL(sw_bhist_kernel, dim3(nb), dim3(kSortBS), 0, s, keys, (const SweepState*)st, bhist, n_keys);
    hipLaunchKernelGGL(sw_colscan_kernel, dim3((n_keys + 255) / 256), dim3(256), 0, s, bhist, nb, n_keys, hist);
    hipLaunchKernelGGL(sw_scan_kernel, dim3(1), dim3(1024), 0, s, (const uint32_t*)hist, n_keys, n_regions, chunk,
                       kfill, items, st);
    hipLaunchKernelGGL(sw_bscatter_kernel, dim3(nb), dim3(kSortBS), 0, s, keys, (const SweepState*)st,
                       (const uint32_t*)kfill, (const uint32_t*)bhist, perm, n_keys);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(sw_zero_kernel, dim3((n_keys + 255) / 256 < 1024 ? (n_keys + 255) / 256 : 1024), dim3(256),
                     0, s, hist, n_keys);
  hipLaunchKernelGGL(sw_hist_kernel, dim3(grid), dim3(256), 0, s, keys, (const SweepState*)st, hist);
  hipLaunchKernelGGL(sw_scan_kernel, dim3(1), dim3(1024), 0, s, (const uint32_t*)hist, n_keys, n_regions, chunk,
                     kfill, items, st);
  hipLaunchKernelGGL(sw_scatter_kernel, dim3(grid), dim3(256), 0, s, keys, (const SweepState*)st, kfill, perm);
  return hipGetLastError();
}

hipError_t launch_sweep_init(SweepState* st, uint64_t total, uint64_t cap_all, hipStream_t s) {
  static_assert(sizeof(SweepState) % 8 == 0, "sweep state of whole words");
  hipLaunchKernelGGL(sw_init_kernel, dim3(1), dim3(64), 0, s, st, (unsigned long long)total,
                     (unsigned long long)cap_all);
  return hipGetLastError();
}
