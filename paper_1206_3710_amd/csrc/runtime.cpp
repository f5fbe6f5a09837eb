// Host runtime behind the C ABI of include/rt.h: validation, the device layout of the
// oct-tree, the job table, accumulator management and the calls into the gfx950 kernels.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <array>
#include <cfloat>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "subiter.h"

namespace {

constexpr double kH = 6.62607015e-27;
constexpr double kC = 2.99792458e10;
constexpr double kPi = 3.14159265358979323846;

thread_local std::string g_create_error;

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t want) {
    if (want <= bytes && p) return hipSuccess;
    if (p) {
      hipError_t e = hipFree(p);
      if (e != hipSuccess) return e;
      p = nullptr;
      bytes = 0;
    }
    size_t sz = std::max<size_t>(want, 256);
    hipError_t e = hipMalloc(&p, sz);
    if (e == hipSuccess) bytes = sz;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

struct HostModel {
  int32_t n[3];
  double cell_cm;
  int32_t nlev;
  int64_t n_root, n_root_pad, n_nodes, n_leaves, n_int, base, leaf_base;
  std::vector<int64_t> level_off;
  // dust
  int32_t nl = 0;
  std::vector<double> lam, kext, alb, g, nu, dnu;
  std::vector<LamConst> lc;
  DevBuf d_lc;
  DevBuf d_T;
  bool has_T = false;
  // subiterations (App. B): constant-source absorption, per-level arrays, last imbalance
  DevBuf sub_astars, sub_arrays, sub_imb;
  double sub_tmin = 0.0, sub_tmax = 0.0;
  bool sub_ready = false;
  bool sub_ali = false;  // steps use the accelerated iteration inside their subtree
  // automatic iteration (Sect. 3.3): canonical parent of each node (-1: a root cell), the outflow
  // of each refined node's subtree as last measured with its parent grid in the step, and the
  // grids tagged for the next step because the flow from a child changed (tag_root: the root
  // grid, i.e. the whole model)
  double sub_flux_frac = 0.0;
  std::vector<int64_t> sub_parent;
  std::vector<double> sub_flux_ref;
  std::vector<char> sub_tag;
  bool sub_tag_root = false;
};

// Launch configuration of one trace in the region schedule: what its sweeps need.
constexpr int kSweepBlock = 16;  // sweeps enqueued (or captured) as one unit; even, so that
                                 // queue buffer 0 is always the input of the first
struct RegionLaunch {
  BlkParams b;
  SweepState* st = nullptr;
  int64_t batch = 0, capq = 0, cap_all = 0, n_keys = 0;
  int n_regions = 0, chunk = 0, grid_sort = 0, grid_pass = 0, grid_peel = 0, bs = 0, reg_lds = 0;
  const PeelParams* peel = nullptr;
};

}  // namespace

struct rt_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int n_cu = 0;
  std::string err;
  std::vector<HostModel> models;
  // host mirrors of the device layout
  std::vector<int32_t> h_word, h_child, h_up, h_leaf_node, h_leaf_coord;
  std::vector<double> h_rho64;
  std::vector<uint8_t> h_leaf_level;
  int64_t total_int = 0, total_leaves = 0;
  bool tree_dirty = true, table_dirty = true;
  // device layout
  DevBuf d_word, d_child, d_up, d_rho64, d_leaf_node, d_leaf_coord, d_leaf_level, d_models;
  std::vector<ModelDev> h_models;
  // work buffers
  DevBuf acc, esc, stats, counter, jobs, records, out_node, out_lamnode, out_esc, e_total;
  DevBuf t_tab;  // inverse table of the emission per unit mass (temperature solves)
  DevBuf last_node;          // absorbed power per node of the last rt_trace_packets call
  int64_t last_nodes = -1;   // node total when it was written (-1: none yet)
  DevBuf cdf_lum, cdf_q, cdf_qpre, lmax, scan_tmp;
  DevBuf tmp_in, tmp_out, tmp_out2, view, lamidx;
  DevBuf it_astars, it_adust, it_sum, it_told, it_crit, it_self, it_emit;
  DevBuf it_aself, it_aemit, it_asolve;  // accelerated subiteration steps
  // peel-off
  DevBuf peel_ev, peel_ctr, peel_tab, peel_roottab, peel_tabroot, peel_dnu, peel_img;
  // grid-by-grid schedule: region-major copy of the trees
  int32_t reg_cap = 0;
  bool reg_dirty = true;
  std::vector<RegionDev> h_regions;
  int64_t reg_G = 0;
  int32_t reg_maxn = 0;
  DevBuf d_regions, d_rword, d_rup, d_rcanon, d_root_region, d_split;
  DevBuf q_rec[2], q_key[2], q_perm, q_hist, q_kfill, q_bhist, q_items, q_state;
  DevBuf sq[2], sq_cnt;  // plain FP64 form with splitting: queues of split-off packages
  int64_t q_capacity = 0;
  // sweep graph: kSweepBlock sweeps captured once per trace configuration, replayed
  hipGraphExec_t sweep_exec = nullptr;
  std::vector<char> sweep_sig;             // launch parameters the graph was captured with
  std::vector<hipEvent_t> sweep_ev;        // 2 per sweep of the block: around each pass
  std::vector<int32_t> h_reg_nodes;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;
  hipEvent_t ev_c = nullptr;
  hipStream_t work = nullptr;  // the sweeps of the region schedule (capturable: never the null stream)
  DevBuf g_jobs, g_keys, g_scan, g_report;  // captured iteration step: job table, Philox key,
                                            // scan scratch, what the host reads per step
  uint32_t g_keys_host[2] = {0, 0};
  int64_t last_sweep_blocks = 0;  // blocks of kSweepBlock sweeps the last region trace needed
  RegionLaunch rl_saved;          // its launch configuration (when the caller asked to keep it)
};

namespace {

rt_status fail(rt_ctx* c, rt_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  else g_create_error = buf;
  return code;
}

#define HIPCHK(x)                                                                        \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess)                                                                \
      return fail(ctx, e_ == hipErrorOutOfMemory ? RT_ENOMEM : RT_EDEVICE, "%s: %s", #x, \
                  hipGetErrorString(e_));                                                \
  } while (0)

#define GUARD(...)                                                             \
  try {                                                                        \
    __VA_ARGS__                                                                \
  } catch (const std::bad_alloc&) {                                            \
    return fail(ctx, RT_ENOMEM, "host allocation failed");                     \
  } catch (...) {                                                              \
    return fail(ctx, RT_EDEVICE, "unexpected host exception");                 \
  }

bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// Device view of a caller array: the pointer itself when on the device, else a staged copy.
rt_status stage_in(rt_ctx* ctx, const void* p, size_t bytes, DevBuf& tmp, const void** out) {
  if (is_device_ptr(p)) {
    *out = p;
    return RT_OK;
  }
  HIPCHK(tmp.ensure(bytes));
  if (bytes) HIPCHK(hipMemcpyAsync(tmp.p, p, bytes, hipMemcpyHostToDevice, ctx->stream));
  *out = tmp.p;
  return RT_OK;
}

// Device destination for a caller output; copy_back is set when it must be copied to the host.
rt_status stage_out(rt_ctx* ctx, void* p, size_t bytes, DevBuf& tmp, void** out, bool* copy_back) {
  *copy_back = false;
  if (!p) {
    *out = nullptr;
    return RT_OK;
  }
  if (is_device_ptr(p)) {
    *out = p;
    return RT_OK;
  }
  HIPCHK(tmp.ensure(bytes));
  *out = tmp.p;
  *copy_back = true;
  return RT_OK;
}

int64_t round8(int64_t v) { return (v + 7) & ~int64_t(7); }

template <class T>
rt_status upload(rt_ctx* ctx, DevBuf& b, const std::vector<T>& v) {
  HIPCHK(b.ensure(v.size() * sizeof(T)));
  if (!v.empty())
    HIPCHK(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, ctx->stream));
  return RT_OK;
}

rt_status check_model(rt_ctx* ctx, int32_t model) {
  if (model < 0 || model >= (int32_t)ctx->models.size())
    return fail(ctx, RT_EINVAL, "model %d does not exist", model);
  return RT_OK;
}

// Bring the device copies of the trees and the model table up to date.
rt_status sync_device(rt_ctx* ctx) {
  HIPCHK(hipSetDevice(ctx->device));
  if (ctx->tree_dirty) {
    rt_status s;
    if ((s = upload(ctx, ctx->d_word, ctx->h_word)) || (s = upload(ctx, ctx->d_child, ctx->h_child)) ||
        (s = upload(ctx, ctx->d_up, ctx->h_up)) || (s = upload(ctx, ctx->d_rho64, ctx->h_rho64)) ||
        (s = upload(ctx, ctx->d_leaf_node, ctx->h_leaf_node)) ||
        (s = upload(ctx, ctx->d_leaf_coord, ctx->h_leaf_coord)) ||
        (s = upload(ctx, ctx->d_leaf_level, ctx->h_leaf_level)))
      return s;
    ctx->tree_dirty = false;
    ctx->table_dirty = true;
    ctx->reg_dirty = true;
  }
  if (ctx->table_dirty) {
    ctx->h_models.assign(ctx->models.size(), ModelDev{});
    int64_t canon = 0, lam = 0, lamnode = 0;
    for (size_t i = 0; i < ctx->models.size(); ++i) {
      const HostModel& h = ctx->models[i];
      ModelDev& m = ctx->h_models[i];
      m.n[0] = h.n[0];
      m.n[1] = h.n[1];
      m.n[2] = h.n[2];
      m.nlev = h.nlev;
      m.base = (int32_t)h.base;
      m.n_root = (int32_t)h.n_root;
      m.n_root_pad = (int32_t)h.n_root_pad;
      m.n_int = (int32_t)h.n_int;
      m.cell_cm = h.cell_cm;
      m.canon_base = canon;
      m.lam_base = lam;
      m.lamnode_base = lamnode;
      m.leaf_base = h.leaf_base;
      m.n_leaves = h.n_leaves;
      m.n_nodes = h.n_nodes;
      m.nl = h.nl;
      for (int l = 0; l < RT_MAX_LEVELS + 2; ++l)
        m.level_off[l] = l < (int)h.level_off.size() ? h.level_off[l] : h.n_nodes;
      canon += h.n_nodes;
      lam += h.nl;
      lamnode += (int64_t)h.nl * h.n_nodes;
    }
    rt_status s = upload(ctx, ctx->d_models, ctx->h_models);
    if (s) return s;
    ctx->table_dirty = false;
  }
  return RT_OK;
}

// Partition every model into regions for the grid-by-grid schedule: bricks of root cells,
// bisected along their longest side until the brick's nodes (root cells padded to 8 plus all
// descendants) fit in `cap` or the brick is a single root cell; then renumber region-major.
rt_status build_regions(rt_ctx* ctx, int32_t cap) {
  if (!ctx->reg_dirty && ctx->reg_cap == cap) return RT_OK;
  std::vector<RegionDev> regs;
  std::vector<int32_t> rword, rup, rcanon, root_region(ctx->total_int, INT32_MIN);
  std::vector<int32_t> split_tab;  // 8 entries per split cell: region id, or ~(split index)
  int64_t G = 0;
  int32_t maxn = 0;
  for (size_t mi = 0; mi < ctx->models.size(); ++mi) {
    const HostModel& h = ctx->models[mi];
    const int nx = h.n[0], ny = h.n[1], nz = h.n[2];
    const int64_t nn = h.n_nodes, n_root = h.n_root;
    const int64_t pad0 = h.n_root_pad - n_root;
    auto internal = [&](int64_t c) { return h.base + (c < n_root ? c : c + pad0); };
    // subtree sizes, bottom-up over levels (canonical order)
    std::vector<int64_t> sz(nn, 1);
    for (int l = h.nlev - 1; l >= 0; --l)
      for (int64_t c = h.level_off[l]; c < h.level_off[l + 1]; ++c) {
        const int32_t fc = ctx->h_child[internal(c)];
        if (fc >= 0) {
          const int64_t cc = (int64_t)fc - h.base - pad0;  // canonical first child
          int64_t s = 1;
          for (int b = 0; b < 8; ++b) s += sz[cc + b];
          sz[c] = s;
        }
      }
    // 3D prefix sums of the root-cell subtree sizes
    const int64_t sx = nx + 1, sy = ny + 1;
    std::vector<int64_t> P((size_t)(nx + 1) * (ny + 1) * (nz + 1), 0);
    auto pidx = [&](int x, int y, int z) { return (size_t)x + sx * ((size_t)y + sy * (size_t)z); };
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
          P[pidx(x + 1, y + 1, z + 1)] = sz[x + (int64_t)nx * (y + (int64_t)ny * z)] + P[pidx(x, y + 1, z + 1)] +
                                         P[pidx(x + 1, y, z + 1)] + P[pidx(x + 1, y + 1, z)] - P[pidx(x, y, z + 1)] -
                                         P[pidx(x, y + 1, z)] - P[pidx(x + 1, y, z)] + P[pidx(x, y, z)];
    auto box_sum = [&](const int lo[3], const int hi[3]) {
      return P[pidx(hi[0], hi[1], hi[2])] - P[pidx(lo[0], hi[1], hi[2])] - P[pidx(hi[0], lo[1], hi[2])] -
             P[pidx(hi[0], hi[1], lo[2])] + P[pidx(lo[0], lo[1], hi[2])] + P[pidx(lo[0], hi[1], lo[2])] +
             P[pidx(hi[0], lo[1], lo[2])] - P[pidx(lo[0], lo[1], lo[2])];
    };
    // Bricks of cells at one level: root-grid bricks by bisection of the longest axis until
    // the subtree nodes fit `cap`; a single cell whose subtree is still too large is split,
    // and the brick of its 8 children (one level down) is bisected in turn.
    struct Box {
      int level;
      int64_t parent;  // canonical id of the split cell whose children the brick holds (-1: root)
      int32_t split;   // that cell's split-table index
      int lo[3], hi[3];
    };
    auto cell_of = [&](const Box& bx, int x, int y, int z) -> int64_t {
      if (bx.level == 0) return x + (int64_t)nx * (y + (int64_t)ny * z);
      const int64_t fc = (int64_t)ctx->h_child[internal(bx.parent)] - h.base - pad0;
      return fc + ((x & 1) | ((y & 1) << 1) | ((z & 1) << 2));
    };
    auto nodes_of = [&](const Box& bx) -> int64_t {
      const int64_t nb = (int64_t)(bx.hi[0] - bx.lo[0]) * (bx.hi[1] - bx.lo[1]) * (bx.hi[2] - bx.lo[2]);
      int64_t s = 0;
      if (bx.level == 0) {
        s = box_sum(bx.lo, bx.hi);
      } else {
        for (int z = bx.lo[2]; z < bx.hi[2]; ++z)
          for (int y = bx.lo[1]; y < bx.hi[1]; ++y)
            for (int x = bx.lo[0]; x < bx.hi[0]; ++x) s += sz[cell_of(bx, x, y, z)];
      }
      return round8(nb) + (s - nb);
    };
    std::vector<Box> stack{{0, -1, -1, {0, 0, 0}, {nx, ny, nz}}}, boxes;
    while (!stack.empty()) {
      Box bx = stack.back();
      stack.pop_back();
      const int64_t nb = (int64_t)(bx.hi[0] - bx.lo[0]) * (bx.hi[1] - bx.lo[1]) * (bx.hi[2] - bx.lo[2]);
      const int64_t nodes = nodes_of(bx);
      if (nodes <= cap) {
        boxes.push_back(bx);
        continue;
      }
      if (nb > 1) {
        int a = 0;
        for (int q = 1; q < 3; ++q)
          if (bx.hi[q] - bx.lo[q] > bx.hi[a] - bx.lo[a]) a = q;
        const int mid = (bx.lo[a] + bx.hi[a]) / 2;
        Box b1 = bx, b2 = bx;
        b1.hi[a] = mid;
        b2.lo[a] = mid;
        stack.push_back(b2);
        stack.push_back(b1);
        continue;
      }
      // one cell with too large a subtree: split it (its refined children keep their own data)
      const int64_t c = cell_of(bx, bx.lo[0], bx.lo[1], bx.lo[2]);
      if (ctx->h_child[internal(c)] < 0) {  // a single leaf always fits; guard anyway
        boxes.push_back(bx);
        continue;
      }
      const int32_t s = (int32_t)(split_tab.size() / 8);
      split_tab.resize(split_tab.size() + 8, INT32_MIN);
      if (bx.level == 0) {
        root_region[internal(c)] = ~s;
      } else {
        const int b = (bx.lo[0] & 1) | ((bx.lo[1] & 1) << 1) | ((bx.lo[2] & 1) << 2);
        split_tab[(size_t)bx.split * 8 + b] = ~s;
      }
      // the brick of its children, in coordinates one level down
      Box kid{bx.level + 1, c, s, {2 * bx.lo[0], 2 * bx.lo[1], 2 * bx.lo[2]},
              {2 * bx.lo[0] + 2, 2 * bx.lo[1] + 2, 2 * bx.lo[2] + 2}};
      stack.push_back(kid);
    }
    for (const auto& bx : boxes) {
      RegionDev R;
      R.model = (int32_t)mi;
      R.rl = bx.level;
      for (int q = 0; q < 3; ++q) {
        R.lo[q] = bx.lo[q];
        R.hi[q] = bx.hi[q];
      }
      const int bxn = R.hi[0] - R.lo[0], byn = R.hi[1] - R.lo[1];
      const int64_t nb = (int64_t)bxn * byn * (R.hi[2] - R.lo[2]);
      R.gbase = G;
      const int32_t rid = (int32_t)regs.size();
      // local numbering: the brick's cells, then octs level by level
      std::vector<std::pair<int64_t, int32_t>> cur;  // (canonical, local)
      cur.reserve(nb);
      for (int z = R.lo[2]; z < R.hi[2]; ++z)
        for (int y = R.lo[1]; y < R.hi[1]; ++y)
          for (int x = R.lo[0]; x < R.hi[0]; ++x) {
            const int64_t c = cell_of(bx, x, y, z);
            const int32_t l = (int32_t)((x - R.lo[0]) + bxn * ((y - R.lo[1]) + byn * (z - R.lo[2])));
            cur.emplace_back(c, l);
            if (bx.level == 0) root_region[internal(c)] = rid;
            else split_tab[(size_t)bx.split * 8 + ((x & 1) | ((y & 1) << 1) | ((z & 1) << 2))] = rid;
          }
      int64_t next = round8(nb);
      std::vector<int32_t> lw, lc;  // local words, canonical ids
      std::vector<std::pair<int32_t, int32_t>> lup;  // (first child local, parent local)
      lw.assign(next, 0);
      lc.assign(next, -1);
      while (!cur.empty()) {
        std::vector<std::pair<int64_t, int32_t>> nxt;
        for (const auto& e : cur) {
          const int64_t c = e.first;
          const int32_t l = e.second;
          const int32_t fc = ctx->h_child[internal(c)];
          lc[l] = (int32_t)c;
          if (fc < 0) {
            lw[l] = ctx->h_word[internal(c)];
          } else {
            const int32_t first = (int32_t)next;
            lw[l] = ~first;
            lup.emplace_back(first, l);
            next += 8;
            lw.resize(next, 0);
            lc.resize(next, -1);
            const int64_t cc = (int64_t)fc - h.base - pad0;
            for (int b = 0; b < 8; ++b) nxt.emplace_back(cc + b, first + b);
          }
        }
        cur.swap(nxt);
      }
      R.n = (int32_t)next;
      maxn = std::max(maxn, R.n);
      rword.insert(rword.end(), lw.begin(), lw.end());
      rcanon.insert(rcanon.end(), lc.begin(), lc.end());
      rup.resize((G + next) / 8, -1);
      for (const auto& u : lup) rup[(G + u.first) / 8] = u.second;
      G += next;
      regs.push_back(R);
    }
  }
  ctx->h_regions = regs;
  ctx->reg_G = G;
  ctx->reg_maxn = maxn;
  rt_status s;
  if ((s = upload(ctx, ctx->d_regions, regs)) || (s = upload(ctx, ctx->d_rword, rword)) ||
      (s = upload(ctx, ctx->d_rup, rup)) || (s = upload(ctx, ctx->d_rcanon, rcanon)) ||
      (s = upload(ctx, ctx->d_root_region, root_region)))
    return s;
  // every root cell has a region or a split entry; every split entry is a region or a split
  // created after its parent (so a walk down the table always ends)
  for (size_t mi = 0; mi < ctx->models.size(); ++mi) {
    const HostModel& h = ctx->models[mi];
    for (int64_t c = 0; c < h.n_root; ++c) {
      const int32_t e = root_region[h.base + c];
      if (e == INT32_MIN) return fail(ctx, RT_EDEVICE, "region layout: root cell without region");
      if (e < 0 && (size_t)(~e) * 8 >= split_tab.size())
        return fail(ctx, RT_EDEVICE, "region layout: bad split index");
    }
  }
  for (size_t i = 0; i < split_tab.size(); ++i) {
    const int32_t e = split_tab[i];
    if (e == INT32_MIN || (e >= 0 && e >= (int32_t)regs.size()) ||
        (e < 0 && ((size_t)(~e) <= i / 8 || (size_t)(~e) * 8 >= split_tab.size())))
      return fail(ctx, RT_EDEVICE, "region layout: bad split table entry");
  }
  if (split_tab.empty()) split_tab.assign(8, -1);
  if ((s = upload(ctx, ctx->d_split, split_tab)))
    return s;
  ctx->reg_cap = cap;
  ctx->reg_dirty = false;
  return RT_OK;
}

void totals(const rt_ctx* ctx, int64_t* nodes, int64_t* lams, int64_t* lamnodes) {
  int64_t a = 0, b = 0, c = 0;
  for (const HostModel& h : ctx->models) {
    a += h.n_nodes;
    b += h.nl;
    c += (int64_t)h.nl * h.n_nodes;
  }
  if (nodes) *nodes = a;
  if (lams) *lams = b;
  if (lamnodes) *lamnodes = c;
}

}  // namespace

// =========================================================================================
// C ABI
// =========================================================================================
extern "C" {

const char* rt_last_error(const rt_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

rt_status rt_create(rt_ctx** out, int32_t device, void* hip_stream) {
  rt_ctx* ctx = nullptr;
  if (!out) return fail(nullptr, RT_EINVAL, "null output pointer");
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
    (void)hipGetLastError();
    return fail(nullptr, RT_EDEVICE, "no HIP device available");
  }
  if (device < 0 || device >= count) return fail(nullptr, RT_EINVAL, "device %d out of range", device);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess)
    return fail(nullptr, RT_EDEVICE, "cannot query device %d", device);
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(nullptr, RT_EDEVICE, "device %d is %s; this library is built for gfx950", device,
                prop.gcnArchName);
  try {
    ctx = new rt_ctx();
  } catch (...) {
    return fail(nullptr, RT_ENOMEM, "host allocation failed");
  }
  ctx->device = device;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  ctx->n_cu = prop.multiProcessorCount;
  if (hipSetDevice(device) != hipSuccess || hipEventCreate(&ctx->ev0) != hipSuccess ||
      hipEventCreate(&ctx->ev1) != hipSuccess || hipEventCreate(&ctx->ev2) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_c, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&ctx->work, hipStreamNonBlocking) != hipSuccess) {
    delete ctx;
    return fail(nullptr, RT_EDEVICE, "cannot initialise device %d", device);
  }
  // the allocation-free maps' scratch array: its address on this device, once per device
  if (render_scratch_init(device) != hipSuccess) {
    (void)hipGetLastError();
    rt_destroy(ctx);
    return fail(nullptr, RT_EDEVICE, "cannot locate the scratch array on device %d", device);
  }
  *out = ctx;
  return RT_OK;
}

rt_status rt_destroy(rt_ctx* ctx) {
  if (!ctx) return RT_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  DevBuf* bufs[] = {&ctx->d_word, &ctx->d_child, &ctx->d_up, &ctx->d_rho64, &ctx->d_leaf_node,
                    &ctx->d_leaf_coord, &ctx->d_leaf_level, &ctx->d_models, &ctx->acc, &ctx->esc,
                    &ctx->stats, &ctx->counter, &ctx->jobs, &ctx->records, &ctx->out_node,
                    &ctx->out_lamnode, &ctx->out_esc, &ctx->e_total, &ctx->cdf_lum, &ctx->cdf_q,
                    &ctx->cdf_qpre, &ctx->lmax, &ctx->scan_tmp, &ctx->tmp_in, &ctx->tmp_out,
                    &ctx->tmp_out2, &ctx->view, &ctx->lamidx, &ctx->it_astars, &ctx->it_adust,
                    &ctx->it_sum, &ctx->it_told, &ctx->it_crit, &ctx->d_regions, &ctx->d_rword,
                    &ctx->d_rup, &ctx->d_rcanon, &ctx->d_root_region, &ctx->d_split, &ctx->q_rec[0], &ctx->q_rec[1],
                    &ctx->q_key[0], &ctx->q_key[1], &ctx->q_perm, &ctx->q_hist, &ctx->q_kfill, &ctx->q_bhist,
                    &ctx->sq[0], &ctx->sq[1], &ctx->sq_cnt,
                    &ctx->q_items, &ctx->q_state, &ctx->last_node, &ctx->t_tab, &ctx->it_self,
                    &ctx->it_emit, &ctx->peel_ev, &ctx->peel_ctr, &ctx->peel_tab, &ctx->peel_roottab,
                    &ctx->peel_tabroot, &ctx->peel_dnu, &ctx->peel_img, &ctx->g_jobs, &ctx->g_keys,
                    &ctx->g_scan, &ctx->g_report, &ctx->it_aself, &ctx->it_aemit, &ctx->it_asolve};
  for (DevBuf* b : bufs) b->release();
  for (HostModel& m : ctx->models) {
    m.d_lc.release();
    m.d_T.release();
    m.sub_astars.release();
    m.sub_arrays.release();
    m.sub_imb.release();
  }
  if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
  if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
  if (ctx->ev2) (void)hipEventDestroy(ctx->ev2);
  if (ctx->sweep_exec) (void)hipGraphExecDestroy(ctx->sweep_exec);
  for (hipEvent_t e : ctx->sweep_ev) (void)hipEventDestroy(e);
  if (ctx->ev_c) (void)hipEventDestroy(ctx->ev_c);
  if (ctx->work) (void)hipStreamDestroy(ctx->work);
  delete ctx;
  return RT_OK;
}

rt_status rt_build_tree(rt_ctx* ctx, const rt_tree_desc* d, int32_t* model_out, int64_t* n_nodes_out) {
  if (!ctx) return fail(nullptr, RT_EINVAL, "null context");
  GUARD({
    if (!d || !model_out) return fail(ctx, RT_EINVAL, "null argument");
    if (d->nx < 1 || d->ny < 1 || d->nz < 1) return fail(ctx, RT_EINVAL, "root dimensions must be >= 1");
    if (!(d->root_cell_cm > 0.0) || !std::isfinite(d->root_cell_cm))
      return fail(ctx, RT_EINVAL, "root cell size must be finite and > 0");
    if (d->n_levels < 0 || d->n_levels > RT_MAX_LEVELS)
      return fail(ctx, RT_EINVAL, "n_levels must be in [0, %d]", RT_MAX_LEVELS);
    if (!d->root_rho) return fail(ctx, RT_EINVAL, "null root densities");
    if (d->n_levels > 0 && (!d->n_refined || !d->refined || !d->child_rho))
      return fail(ctx, RT_EINVAL, "null refinement arrays");
    if (ctx->models.size() >= 4096) return fail(ctx, RT_EINVAL, "at most 4096 models per context");
    const int64_t nmax = std::max<int64_t>(d->nx, std::max<int64_t>(d->ny, d->nz));
    if ((nmax << d->n_levels) >= (int64_t(1) << 30))
      return fail(ctx, RT_EINVAL, "root size times 2^levels must stay below 2^30");
    const int64_t n_root = (int64_t)d->nx * d->ny * d->nz;
    std::vector<int64_t> off(d->n_levels + 2, 0);
    int64_t cells = n_root;
    for (int l = 0; l <= d->n_levels; ++l) {
      off[l + 1] = off[l] + cells;
      if (l < d->n_levels) {
        const int64_t nr = d->n_refined[l];
        if (nr < 0 || nr > cells) return fail(ctx, RT_EINVAL, "bad refined count at level %d", l);
        if (nr > 0 && (!d->refined[l] || !d->child_rho[l]))
          return fail(ctx, RT_EINVAL, "null refined list at level %d", l);
        for (int64_t i = 0; i < nr; ++i) {
          const int64_t v = d->refined[l][i];
          if (v < 0 || v >= cells) return fail(ctx, RT_EINVAL, "refined index out of range at level %d", l);
          if (i > 0 && v <= d->refined[l][i - 1])
            return fail(ctx, RT_EINVAL, "refined list not strictly ascending at level %d", l);
        }
        cells = 8 * nr;
      }
    }
    const int64_t n_nodes = off[d->n_levels + 1];
    const int64_t base = round8(ctx->total_int);
    const int64_t n_root_pad = round8(n_root);
    const int64_t pad0 = n_root_pad - n_root;
    const int64_t n_int = n_root_pad + (n_nodes - n_root);
    if (base + n_int >= (int64_t(1) << 31) - 8)
      return fail(ctx, RT_EINVAL, "total node count exceeds the 32-bit node index");
    auto rho_of = [&](int64_t canon) -> double {
      if (canon < n_root) return d->root_rho[canon];
      int l = 0;
      while (canon >= off[l + 2]) ++l;
      return d->child_rho[l][canon - off[l + 1]];
    };
    for (int64_t i = 0; i < n_root; ++i) {
      const double r = d->root_rho[i];
      if (!(r >= 0.0) || !std::isfinite(r) || r > (double)FLT_MAX)
        return fail(ctx, RT_EINVAL, "root density %lld must be finite, >= 0 and <= FLT_MAX", (long long)i);
    }
    for (int l = 0; l < d->n_levels; ++l)
      for (int64_t i = 0; i < 8 * d->n_refined[l]; ++i) {
        const double r = d->child_rho[l][i];
        if (!(r >= 0.0) || !std::isfinite(r) || r > (double)FLT_MAX)
          return fail(ctx, RT_EINVAL, "density at level %d must be finite, >= 0 and <= FLT_MAX", l + 1);
      }
    (void)rho_of;
    // ---- all checks passed: build the device layout (host mirror) ----
    HostModel hm;
    hm.n[0] = d->nx;
    hm.n[1] = d->ny;
    hm.n[2] = d->nz;
    hm.cell_cm = d->root_cell_cm;
    hm.nlev = d->n_levels;
    hm.n_root = n_root;
    hm.n_root_pad = n_root_pad;
    hm.n_nodes = n_nodes;
    hm.n_int = n_int;
    hm.base = base;
    hm.level_off = off;
    const int64_t end = base + n_int;
    ctx->h_word.resize(end, 0);
    ctx->h_child.resize(end, -1);
    ctx->h_rho64.resize(end, 0.0);
    ctx->h_up.resize(end / 8 + 1, -1);
    auto internal = [&](int64_t canon) { return base + (canon < n_root ? canon : canon + pad0); };
    auto set_leaf = [&](int64_t canon, double r) {
      const int64_t i = internal(canon);
      float f = (float)r;
      if (f == 0.0f) f = 0.0f;  // +0
      int32_t bits;
      std::memcpy(&bits, &f, 4);
      ctx->h_word[i] = bits;
      ctx->h_rho64[i] = r;
      ctx->h_child[i] = -1;
    };
    for (int64_t c = 0; c < n_root; ++c) set_leaf(c, d->root_rho[c]);
    for (int l = 0; l < d->n_levels; ++l)
      for (int64_t i = 0; i < 8 * d->n_refined[l]; ++i) set_leaf(off[l + 1] + i, d->child_rho[l][i]);
    // coordinates at each node's own level, for the leaf table
    std::vector<int32_t> coord(3 * n_nodes);
    std::vector<uint8_t> level(n_nodes, 0);
    for (int64_t c = 0; c < n_root; ++c) {
      coord[3 * c] = (int32_t)(c % d->nx);
      coord[3 * c + 1] = (int32_t)((c / d->nx) % d->ny);
      coord[3 * c + 2] = (int32_t)(c / ((int64_t)d->nx * d->ny));
    }
    std::vector<char> refined(n_nodes, 0);
    for (int l = 0; l < d->n_levels; ++l) {
      for (int64_t o = 0; o < d->n_refined[l]; ++o) {
        const int64_t pc = off[l] + d->refined[l][o];
        const int64_t fc = off[l + 1] + 8 * o;
        const int64_t pi = internal(pc), fi = internal(fc);
        ctx->h_word[pi] = ~(int32_t)fi;
        ctx->h_child[pi] = (int32_t)fi;
        ctx->h_up[fi >> 3] = (int32_t)pi;
        refined[pc] = 1;
        for (int b = 0; b < 8; ++b) {
          const int64_t cc = fc + b;
          level[cc] = (uint8_t)(l + 1);
          for (int a = 0; a < 3; ++a) coord[3 * cc + a] = 2 * coord[3 * pc + a] + ((b >> a) & 1);
        }
      }
    }
    hm.leaf_base = ctx->total_leaves;
    int64_t nleaf = 0;
    for (int64_t c = 0; c < n_nodes; ++c) {
      if (refined[c]) continue;
      ctx->h_leaf_node.push_back((int32_t)internal(c));
      ctx->h_leaf_level.push_back(level[c]);
      for (int a = 0; a < 3; ++a) ctx->h_leaf_coord.push_back(coord[3 * c + a]);
      ++nleaf;
    }
    hm.n_leaves = nleaf;
    ctx->total_leaves += nleaf;
    ctx->total_int = end;
    ctx->models.push_back(std::move(hm));
    ctx->tree_dirty = true;
    ctx->table_dirty = true;
    *model_out = (int32_t)ctx->models.size() - 1;
    if (n_nodes_out) *n_nodes_out = n_nodes;
    return RT_OK;
  })
}

rt_status rt_get_model_info(rt_ctx* ctx, int32_t model, rt_model_info* out) {
  if (!ctx) return fail(nullptr, RT_EINVAL, "null context");
  if (rt_status s = check_model(ctx, model)) return s;
  if (!out) return fail(ctx, RT_EINVAL, "null output");
  const HostModel& h = ctx->models[model];
  std::memset(out, 0, sizeof *out);
  out->n_nodes = h.n_nodes;
  out->n_leaves = h.n_leaves;
  out->n_levels = h.nlev;
  out->n_lambda = h.nl;
  for (int l = 0; l < RT_MAX_LEVELS + 2; ++l)
    out->level_offset[l] = l < (int)h.level_off.size() ? h.level_off[l] : h.n_nodes;
  for (int32_t i = 0; i < model; ++i) {
    out->node_base += ctx->models[i].n_nodes;
    out->lambda_base += ctx->models[i].nl;
    out->lambda_node_base += (int64_t)ctx->models[i].nl * ctx->models[i].n_nodes;
  }
  return RT_OK;
}

rt_status rt_get_sizes(rt_ctx* ctx, int64_t* nodes, int64_t* lambdas, int64_t* lambda_nodes) {
  if (!ctx) return fail(nullptr, RT_EINVAL, "null context");
  totals(ctx, nodes, lambdas, lambda_nodes);
  return RT_OK;
}

rt_status rt_locate(rt_ctx* ctx, int32_t model, int64_t n, const double* xyz, int32_t* level_out,
                    int64_t* node_out) {
  if (!ctx) return fail(nullptr, RT_EINVAL, "null context");
  GUARD({
    if (rt_status s = check_model(ctx, model)) return s;
    if (n < 0) return fail(ctx, RT_EINVAL, "negative point count");
    if (n == 0) return RT_OK;
    if (!xyz || !level_out || !node_out) return fail(ctx, RT_EINVAL, "null array");
    if (rt_status s = sync_device(ctx)) return s;
    const void* dx;
    if (rt_status s = stage_in(ctx, xyz, 24 * n, ctx->tmp_in, &dx)) return s;
    void *dl, *dn;
    bool cl, cn;
    if (rt_status s = stage_out(ctx, level_out, 4 * n, ctx->tmp_out, &dl, &cl)) return s;
    if (rt_status s = stage_out(ctx, node_out, 8 * n, ctx->tmp_out2, &dn, &cn)) return s;
    HIPCHK(launch_locate(ctx->d_child.as<int32_t>(), ctx->d_models.as<ModelDev>(), model, n,
                         static_cast<const double*>(dx), static_cast<int32_t*>(dl),
                         static_cast<int64_t*>(dn), ctx->stream));
    if (cl) HIPCHK(hipMemcpyAsync(level_out, dl, 4 * n, hipMemcpyDeviceToHost, ctx->stream));
    if (cn) HIPCHK(hipMemcpyAsync(node_out, dn, 8 * n, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RT_OK;
  })
}

rt_status rt_set_dust(rt_ctx* ctx, int32_t model, int32_t nl, const double* lam, const double* kappa,
                      const double* albedo, const double* g) {
  if (!ctx) return fail(nullptr, RT_EINVAL, "null context");
  GUARD({
    if (rt_status s = check_model(ctx, model)) return s;
    if (nl < 1 || nl > 4096) return fail(ctx, RT_EINVAL, "n_lambda must be in [1, 4096]");
    if (!lam || !kappa || !albedo || !g) return fail(ctx, RT_EINVAL, "null dust array");
    for (int i = 0; i < nl; ++i) {
      if (!(lam[i] > 0.0) || !std::isfinite(lam[i])) return fail(ctx, RT_EINVAL, "wavelength %d invalid", i);
      if (i > 0 && !(lam[i] > lam[i - 1])) return fail(ctx, RT_EINVAL, "wavelengths must ascend strictly");
      if (!(kappa[i] > 0.0) || !std::isfinite(kappa[i])) return fail(ctx, RT_EINVAL, "kappa %d must be > 0", i);
      if (!(albedo[i] >= 0.0 && albedo[i] <= 1.0)) return fail(ctx, RT_EINVAL, "albedo %d outside [0,1]", i);
      if (!(std::fabs(g[i]) < 1.0)) return fail(ctx, RT_EINVAL, "|g| must be < 1 (entry %d)", i);
    }
    HostModel& h = ctx->models[model];
    h.nl = nl;
    h.lam.assign(lam, lam + nl);
    h.kext.assign(kappa, kappa + nl);
    h.alb.assign(albedo, albedo + nl);
    h.g.assign(g, g + nl);
    h.nu.resize(nl);
    h.dnu.resize(nl);
    for (int i = 0; i < nl; ++i) h.nu[i] = kC / (lam[i] * 1e-4);
    if (nl == 1) {
      h.dnu[0] = 1.0;
    } else {
      h.dnu[0] = std::fabs(h.nu[1] - h.nu[0]) * 0.5;
      h.dnu[nl - 1] = std::fabs(h.nu[nl - 1] - h.nu[nl - 2]) * 0.5;
      for (int i = 1; i < nl - 1; ++i) h.dnu[i] = std::fabs(h.nu[i + 1] - h.nu[i - 1]) * 0.5;
    }
    h.lc.resize(nl);
    for (int i = 0; i < nl; ++i) {
      const double nu = h.nu[i];
      h.lc[i].kext = h.kext[i];
      h.lc[i].alb = h.alb[i];
      h.lc[i].dnu = h.dnu[i];
      h.lc[i].kabs_dnu = (1.0 - h.alb[i]) * h.kext[i] * h.dnu[i];
      h.lc[i].pre = 2.0 * kH * nu * nu * nu / (kC * kC);
      h.lc[i].hnu = kH * nu;
    }
    HIPCHK(hipSetDevice(ctx->device));
    if (rt_status s = upload(ctx, h.d_lc, h.lc)) return s;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->table_dirty = true;
    return RT_OK;
  })
}

rt_status rt_set_temperature(rt_ctx* ctx, int32_t model, const double* t_node) {
  if (!ctx) return fail(nullptr, RT_EINVAL, "null context");
  GUARD({
    if (rt_status s = check_model(ctx, model)) return s;
    if (!t_node) return fail(ctx, RT_EINVAL, "null temperatures");
    HostModel& h = ctx->models[model];
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(h.d_T.ensure(8 * h.n_nodes));
    HIPCHK(hipMemcpyAsync(h.d_T.p, t_node, 8 * h.n_nodes,
                          is_device_ptr(t_node) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    h.has_T = true;
    return RT_OK;
  })
}

}  // extern "C"

// -----------------------------------------------------------------------------------------
// tracing
// -----------------------------------------------------------------------------------------
namespace {

// Dust-emission tables of one (model, wavelength): luminosity, 32-bit quantised share of the
// maximum and its exact 64-bit exclusive prefix sum; returns the total.
rt_status build_dust_cdf(rt_ctx* ctx, int32_t model, int lam, int64_t off, uint64_t* qtot, int sub_lev,
                         const int32_t sub_I[3]) {
  HostModel& h = ctx->models[model];
  const int64_t n = h.n_leaves;
  double* lum = ctx->cdf_lum.as<double>() + off;
  uint64_t* q = ctx->cdf_q.as<uint64_t>() + off;
  uint64_t* qpre = ctx->cdf_qpre.as<uint64_t>() + off;
  HIPCHK(ctx->lmax.ensure(16));
  HIPCHK(hipMemsetAsync(ctx->lmax.p, 0, 16, ctx->stream));
  HIPCHK(launch_dust_lum(ctx->d_models.as<ModelDev>(), model, n, ctx->d_leaf_node.as<int32_t>(),
                         ctx->d_leaf_level.as<uint8_t>(), ctx->d_rho64.as<double>(),
                         h.d_T.as<double>(), h.d_lc.as<LamConst>(), lam, lum,
                         ctx->lmax.as<unsigned long long>(), ctx->d_leaf_coord.as<int32_t>(), sub_lev, sub_I,
                         ctx->stream));
  HIPCHK(launch_dust_quant(n, lum, ctx->lmax.as<unsigned long long>(), q, ctx->stream));
  size_t tmp = 0;
  HIPCHK(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp, q, qpre, (int)n, ctx->stream));
  HIPCHK(ctx->scan_tmp.ensure(tmp));
  HIPCHK(hipcub::DeviceScan::ExclusiveSum(ctx->scan_tmp.p, tmp, q, qpre, (int)n, ctx->stream));
  uint64_t last[2];
  HIPCHK(hipMemcpyAsync(&last[0], qpre + n - 1, 8, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipMemcpyAsync(&last[1], q + n - 1, 8, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  *qtot = last[0] + last[1];
  return RT_OK;
}

struct TraceOut {
  double* e_node = nullptr;      // device [total nodes] or null
  double* e_lamnode = nullptr;   // device [total lamnodes] or null
  double* e_esc = nullptr;       // device [total lambdas]
  const PeelParams* peel = nullptr;  // peel-off after every batch (rt_peel_map)
  double* self_acc = nullptr;        // accelerated Lambda iteration tallies (device, total nodes)
  double* emit_acc = nullptr;
  double* lvl_acc = nullptr;         // subiterations: per-level deposits (device, [levels][total nodes])
  int64_t lvl_stride = 0;
  int32_t sub_lev = -1;              // subtree root (level, coordinates); -1 = whole model
  int32_t sub_I[3] = {0, 0, 0};
  double* flux_acc = nullptr;        // automatic iteration: outflow of each refined node's subtree
  bool save_launch = false;          // keep the region schedule's launch configuration in the ctx
};

// Queue buffers, sort scratch and the pass kernel's parameters of one region-schedule trace.
rt_status region_launch_setup(rt_ctx* ctx, const rt_trace_opts* o, const TraceParams& p, const TraceOut& out,
                              uint64_t start, int bs, int reg_per_cu, int reg_lds, int key_slots, int n_lvl,
                              RegionLaunch* L) {
  const int n_regions = (int)ctx->h_regions.size();
  const int64_t n_keys = (int64_t)key_slots * n_regions;
  if (n_keys > (int64_t(1) << 28)) return fail(ctx, RT_EINVAL, "too many (wavelength, region) keys");
  // up to 2^27 records per buffer (13 GB of 96-byte records, 2^26 with splitting, whose buffers
  // hold two capacities): a trace of 1e9 packets keeps ~1e8 in flight, and a smaller capacity
  // would cut each sweep's births short and multiply the sweeps
  const int64_t cap_max = int64_t(1) << (p.split_n > 1 ? 26 : 27);
  const int64_t capq = std::min<int64_t>(cap_max, std::max<int64_t>((int64_t)start, 4096));
  const int64_t batch = std::min<int64_t>(o->batch_packets > 0 ? o->batch_packets : int64_t(1) << 23, capq);
  const int32_t chunk = o->chunk_packets > 0 ? o->chunk_packets : 16 * bs;
  // records per queue buffer: emission keeps each sweep's input + births within capq; with
  // package splitting a second capq holds the packages split off during a sweep
  const int64_t cap_all = p.split_n > 1 ? 2 * capq : capq;
  // plus the unused ends of the pass waves' last chunks of records (at most one chunk each)
  const int64_t cap_rec = cap_all + (int64_t)ctx->n_cu * reg_per_cu * (bs / 64) * (int64_t)kExitChunk;
  if (ctx->q_capacity < cap_rec) {
    for (int k = 0; k < 2; ++k) {
      HIPCHK(ctx->q_rec[k].ensure(sizeof(PRec) * cap_rec));
      HIPCHK(ctx->q_key[k].ensure(4 * cap_rec));
    }
    HIPCHK(ctx->q_perm.ensure(4 * cap_rec));
    ctx->q_capacity = cap_rec;
  }
  HIPCHK(ctx->q_hist.ensure(4 * n_keys));
  HIPCHK(ctx->q_kfill.ensure(4 * n_keys));
  if (n_keys <= kSortLdsKeys) HIPCHK(ctx->q_bhist.ensure(4 * n_keys * (int64_t)kSortBlocks(ctx->n_cu * 4)));
  HIPCHK(ctx->q_items.ensure(sizeof(WorkItem) * (cap_all / chunk + n_keys + 1)));
  HIPCHK(ctx->q_state.ensure(sizeof(SweepState)));
  SweepState* st = ctx->q_state.as<SweepState>();
  BlkParams& b = L->b;
  std::memset(&b, 0, sizeof b);
  b.t = p;
  b.regions = ctx->d_regions.as<RegionDev>();
  b.n_regions = n_regions;
  b.cap = ctx->reg_cap;
  b.rword = ctx->d_rword.as<int32_t>();
  b.rup = ctx->d_rup.as<int32_t>();
  b.rcanon = ctx->d_rcanon.as<int32_t>();
  b.root_region = ctx->d_root_region.as<int32_t>();
  b.split_tab = ctx->d_split.as<int32_t>();
  b.accb64 = ctx->acc.as<double>();
  b.accb_stride = ctx->reg_G;
  b.lvl_slots = n_lvl;
  b.q_perm = ctx->q_perm.as<uint32_t>();
  b.items = ctx->q_items.as<WorkItem>();
  b.n_items = &st->n_items;
  b.item_counter = &st->item_counter;
  b.sweep = st;
  b.emit_counter = &st->emit_counter;
  b.split_room = &st->split_room;
  b.split_used = &st->split_used;
  b.n_slots_key = key_slots;
  b.chunk = chunk;
  b.tail_park = o->tail_park < 0 ? INT32_MAX : (o->tail_park > 0 ? o->tail_park : 16);
  L->st = st;
  L->batch = batch;
  L->capq = capq;
  L->cap_all = cap_all;
  L->n_keys = n_keys;
  L->n_regions = n_regions;
  L->chunk = chunk;
  L->grid_pass = ctx->n_cu * reg_per_cu;
  L->grid_sort = ctx->n_cu * 4;
  L->grid_peel = ctx->n_cu * 8;
  L->bs = bs;
  L->reg_lds = reg_lds;
  L->peel = out.peel;
  return RT_OK;
}

// kSweepBlock sweeps of a region-schedule trace on stream s; with ev, the pass of sweep k is
// bracketed by events 2k and 2k + 1 (not while capturing a graph).
hipError_t enqueue_sweeps(rt_ctx* ctx, const RegionLaunch& L, hipStream_t s, const std::vector<hipEvent_t>* ev) {
  for (int k = 0; k < kSweepBlock; ++k) {
    const int in = k & 1, out = 1 - in;
    hipError_t e = launch_sweep_sort(L.st, in, k, (uint64_t)L.batch, (uint64_t)L.capq, ctx->q_key[in].as<uint32_t>(),
                                     (int)L.n_keys, L.n_regions, L.chunk, ctx->q_hist.as<uint32_t>(),
                                     ctx->q_kfill.as<uint32_t>(), ctx->q_bhist.as<uint32_t>(),
                                     ctx->q_perm.as<uint32_t>(), ctx->q_items.as<WorkItem>(), L.grid_sort, s);
    if (e != hipSuccess) return e;
    BlkParams bk = L.b;
    bk.q_in = ctx->q_rec[in].as<PRec>();
    bk.u_out = ctx->q_rec[out].as<PRec>();
    bk.u_key = ctx->q_key[out].as<uint32_t>();
    bk.u_count = &L.st->count[out];
    // the pass kernel's blocks also write this sweep's births, once its work items are taken
    if (ev && (e = hipEventRecord((*ev)[2 * k], s)) != hipSuccess) return e;
    if ((e = launch_blk_pass(bk, L.grid_pass, L.bs, L.reg_lds, s)) != hipSuccess) return e;
    if (ev && (e = hipEventRecord((*ev)[2 * k + 1], s)) != hipSuccess) return e;
    if (L.peel && (e = launch_peel(bk.t, *L.peel, L.grid_peel, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

rt_status trace_impl(rt_ctx* ctx, int32_t n_src, const rt_source* src, const rt_trace_opts* o,
                     const TraceOut& out, rt_trace_stats* st_out) {
  // ---- validation (no state changes before this block ends) ----
  if (n_src < 1 || n_src > 255) return fail(ctx, RT_EINVAL, "n_src must be in [1, 255]");
  if (!src || !o) return fail(ctx, RT_EINVAL, "null sources or options");
  if (o->precision != RT_FP64 && o->precision != RT_FP32_LOCAL)
    return fail(ctx, RT_EINVAL, "precision must be RT_FP64 or RT_FP32_LOCAL");
  if (!(o->rr_threshold >= 0.0) || !std::isfinite(o->rr_threshold))
    return fail(ctx, RT_EINVAL, "rr_threshold must be finite and >= 0");
  if (!(o->rr_prob >= 0.0 && o->rr_prob < 1.0)) return fail(ctx, RT_EINVAL, "rr_prob must be in [0, 1)");
  if (o->max_events < 0 || o->max_events > 0x7fffffff) return fail(ctx, RT_EINVAL, "bad max_events");
  const bool region_sched = o->precision == RT_FP32_LOCAL && o->schedule == RT_SCHED_REGIONS;
  // defaults from tuning on the molecular-cloud workload
  const int bs = o->block_size ? o->block_size : (region_sched ? 768 : 256);
  const bool bs_ok = region_sched ? (bs == 256 || bs == 512 || bs == 768 || bs == 1024)
                    : o->precision == RT_FP32_LOCAL ? (bs == 64 || bs == 128 || bs == 256 || bs == 512)
                                                     : (bs == 64 || bs == 128 || bs == 256);
  if (!bs_ok)
    return fail(ctx, RT_EINVAL,
                "block_size must be 64, 128 or 256 (FP64), 64-512 (FP32-local, one queue) or "
                "256, 512, 768, 1024 (FP32-local, regions)");
  if (o->blocks_per_cu < 0 || o->blocks_per_cu > 64) return fail(ctx, RT_EINVAL, "bad blocks_per_cu");
  if (!(o->refill_threshold >= 0.0f && o->refill_threshold <= 1.0f))
    return fail(ctx, RT_EINVAL, "refill_threshold must be in [0, 1]");
  if (o->schedule != RT_SCHED_REGIONS && o->schedule != RT_SCHED_GLOBAL)
    return fail(ctx, RT_EINVAL, "schedule must be RT_SCHED_REGIONS or RT_SCHED_GLOBAL");
  if (o->precision == RT_FP32_LOCAL && o->schedule == RT_SCHED_REGIONS && o->block_size &&
      o->block_size != 256 && o->block_size != 512 && o->block_size != 768 && o->block_size != 1024)
    return fail(ctx, RT_EINVAL, "the region schedule needs block_size 256, 512, 768 or 1024");
  if (o->chunk_packets < 0 || o->batch_packets < 0)
    return fail(ctx, RT_EINVAL, "chunk_packets and batch_packets must be >= 0");
  if (o->split_n < 0 || o->split_n > 64) return fail(ctx, RT_EINVAL, "split_n must be in [0, 64]");
  if (o->split_depth < 0) return fail(ctx, RT_EINVAL, "split_depth must be >= 0");
  if (o->split_n > 1 && !region_sched && o->precision != RT_FP64)
    return fail(ctx, RT_EINVAL, "package splitting runs in the region schedule or the RT_FP64 form");
  if (o->rec_stride < 0 || (o->rec_stride > 0 && !o->records))
    return fail(ctx, RT_EINVAL, "records needed when rec_stride > 0");
  for (int s = 0; s < n_src; ++s) {
    const rt_source& S = src[s];
    if (rt_status e = check_model(ctx, S.model)) return e;
    const HostModel& h = ctx->models[S.model];
    if (h.nl < 1) return fail(ctx, RT_ESTATE, "rt_set_dust not called for model %d", S.model);
    if (S.kind < 0 || S.kind > 3) return fail(ctx, RT_EINVAL, "source %d: bad kind", s);
    if (S.packets_per_lambda < 1 || S.packets_per_lambda > (int64_t(1) << 32))
      return fail(ctx, RT_EINVAL, "source %d: packets_per_lambda must be in [1, 2^32]", s);
    if (S.kind != RT_SRC_DUST) {
      if (!S.power) return fail(ctx, RT_EINVAL, "source %d: null power", s);
      for (int i = 0; i < h.nl; ++i)
        if (!(S.power[i] >= 0.0) || !std::isfinite(S.power[i]))
          return fail(ctx, RT_EINVAL, "source %d: power must be finite and >= 0", s);
    } else if (!h.has_T) {
      return fail(ctx, RT_ESTATE, "source %d: dust emission needs temperatures", s);
    }
    if (S.kind == RT_SRC_POINT || S.kind == RT_SRC_BEAM)
      for (int a = 0; a < 3; ++a)
        if (!(S.pos[a] >= 0.0 && S.pos[a] < (double)h.n[a]))
          return fail(ctx, RT_EINVAL, "source %d: position outside the root grid", s);
    if (S.kind == RT_SRC_BEAM) {
      const double nb = std::sqrt(S.dir[0] * S.dir[0] + S.dir[1] * S.dir[1] + S.dir[2] * S.dir[2]);
      if (!(nb > 0.0) || !std::isfinite(nb)) return fail(ctx, RT_EINVAL, "source %d: bad direction", s);
    }
  }
  // ---- setup ----
  if (rt_status e = sync_device(ctx)) return e;
  int64_t tot_nodes, tot_lam, tot_lamnode;
  totals(ctx, &tot_nodes, &tot_lam, &tot_lamnode);
  int max_nl = 1;
  for (const HostModel& h : ctx->models) max_nl = std::max(max_nl, h.nl);
  const bool fp32 = o->precision == RT_FP32_LOCAL;
  // FP64 accumulators in every form: one slot per node, or one per (wavelength, node) when
  // per-wavelength output is requested
  const int n_slots = out.e_lamnode ? max_nl : 1;
  const size_t elem = 8;
  const int64_t stride = ctx->total_int;
  HIPCHK(ctx->acc.ensure((size_t)n_slots * stride * elem));
  HIPCHK(hipMemsetAsync(ctx->acc.p, 0, (size_t)n_slots * stride * elem, ctx->stream));
  HIPCHK(ctx->stats.ensure(sizeof(DevStats)));
  HIPCHK(hipMemsetAsync(ctx->stats.p, 0, sizeof(DevStats), ctx->stream));
  HIPCHK(ctx->counter.ensure(8));
  HIPCHK(hipMemsetAsync(ctx->counter.p, 0, 8, ctx->stream));
  HIPCHK(ctx->e_total.ensure(8));
  HIPCHK(hipMemsetAsync(ctx->e_total.p, 0, 8, ctx->stream));
  HIPCHK(hipMemsetAsync(out.e_esc, 0, 8 * tot_lam, ctx->stream));

  // job table: source-major, then wavelength
  std::vector<JobDev> jobs;
  int64_t cdf_total = 0;
  for (int s = 0; s < n_src; ++s)
    if (src[s].kind == RT_SRC_DUST) cdf_total += ctx->models[src[s].model].n_leaves * ctx->models[src[s].model].nl;
  if (cdf_total > 0) {
    HIPCHK(ctx->cdf_lum.ensure(8 * cdf_total));
    HIPCHK(ctx->cdf_q.ensure(8 * cdf_total));
    HIPCHK(ctx->cdf_qpre.ensure(8 * cdf_total));
  }
  uint64_t start = 0;
  int64_t rec_base = 0, cdf_off = 0;
  for (int s = 0; s < n_src; ++s) {
    const rt_source& S = src[s];
    const HostModel& h = ctx->models[S.model];
    const ModelDev& md = ctx->h_models[S.model];
    double bd[3] = {0.0, 0.0, 1.0};
    if (S.kind == RT_SRC_BEAM) {
      const double nb = std::sqrt(S.dir[0] * S.dir[0] + S.dir[1] * S.dir[1] + S.dir[2] * S.dir[2]);
      for (int a = 0; a < 3; ++a) bd[a] = S.dir[a] / nb;
    }
    for (int i = 0; i < h.nl; ++i) {
      JobDev J;
      std::memset(&J, 0, sizeof J);
      const uint64_t N = (uint64_t)S.packets_per_lambda;
      J.start = start;
      J.n = N;
      J.model = S.model;
      J.kind = S.kind;
      J.lam = i;
      J.src = s;
      J.stream = ((uint32_t)S.model << 20) | ((uint32_t)s << 12) | (uint32_t)i;
      J.esc_slot = (int32_t)(md.lam_base + i);
      if (S.kind == RT_SRC_BACKGROUND) {
        const double area = 2.0 * ((double)h.n[0] * h.n[1] + (double)h.n[1] * h.n[2] +
                                   (double)h.n[0] * h.n[2]);
        const double pin = kPi * S.power[i] * h.dnu[i] * (area * h.cell_cm * h.cell_cm);
        J.w0 = pin / (double)N;
      } else if (S.kind == RT_SRC_POINT || S.kind == RT_SRC_BEAM) {
        J.w0 = S.power[i] * h.dnu[i] / (double)N;
      }
      for (int a = 0; a < 3; ++a) {
        J.pos[a] = S.pos[a];
        J.dir[a] = bd[a];
      }
      J.kext = h.kext[i];
      J.alb = h.alb[i];
      J.g = h.g[i];
      J.kc32 = (float)(h.kext[i] * h.cell_cm);
      J.alb32 = (float)h.alb[i];
      J.g32 = (float)h.g[i];
      J.acc_off = (n_slots > 1 ? (int64_t)i : 0) * stride;
      J.slot = n_slots > 1 ? i : 0;
      J.rec_base = rec_base;
      if (o->rec_stride > 0) rec_base += (int64_t)((N + o->rec_stride - 1) / o->rec_stride);
      if (S.kind == RT_SRC_DUST) {
        J.cdf_off = cdf_off;
        uint64_t qtot = 0;
        if (rt_status e = build_dust_cdf(ctx, S.model, i, cdf_off, &qtot, out.sub_lev, out.sub_I)) return e;
        J.qtot = qtot;
        cdf_off += h.n_leaves;
        if (qtot == 0) J.n = 0;  // nothing emits at this wavelength
      }
      start += J.n;
      jobs.push_back(J);
    }
  }
  if (rt_status e = upload(ctx, ctx->jobs, jobs)) return e;
  void* rec_dev = nullptr;
  bool rec_copy = false;
  if (o->rec_stride > 0) {
    if (rt_status e = stage_out(ctx, o->records, sizeof(rt_record) * rec_base, ctx->records, &rec_dev, &rec_copy))
      return e;
    HIPCHK(hipMemsetAsync(rec_dev, 0, sizeof(rt_record) * std::max<int64_t>(rec_base, 1), ctx->stream));
  }

  TraceParams p;
  std::memset(&p, 0, sizeof p);
  p.word = ctx->d_word.as<int32_t>();
  p.rho64 = ctx->d_rho64.as<double>();
  p.child = ctx->d_child.as<int32_t>();
  p.up = ctx->d_up.as<int32_t>();
  p.models = ctx->d_models.as<ModelDev>();
  p.jobs = ctx->jobs.as<JobDev>();
  p.n_jobs = (int32_t)jobs.size();
  p.n_esc = (int32_t)tot_lam;
  p.total_packets = start;
  p.counter = ctx->counter.as<unsigned long long>();
  p.acc64 = ctx->acc.as<double>();
  p.esc = out.e_esc;
  p.stats = ctx->stats.as<DevStats>();
  p.rec = static_cast<rt_record*>(rec_dev);
  p.rec_stride = o->rec_stride;
  p.key0 = (uint32_t)(o->seed & 0xffffffffu);
  p.key1 = (uint32_t)(o->seed >> 32) + o->iteration;
  p.rr_thr = o->rr_threshold;
  p.rr_p = o->rr_prob;
  p.max_events = o->max_events > 0 ? o->max_events : 1000000;
  p.refill_thr = o->refill_threshold > 0.0f ? o->refill_threshold : (region_sched ? 0.6f : 0.5f);
  p.split_n = o->split_n > 1 ? o->split_n : 1;
  p.split_depth = o->split_depth > 0 ? o->split_depth : 127;
  p.cdf_qpre = ctx->cdf_qpre.as<uint64_t>();
  p.cdf_q = ctx->cdf_q.as<uint64_t>();
  p.cdf_lum = ctx->cdf_lum.as<double>();
  p.leaf_node = ctx->d_leaf_node.as<int32_t>();
  p.leaf_coord = ctx->d_leaf_coord.as<int32_t>();
  p.leaf_level = ctx->d_leaf_level.as<uint8_t>();
  p.self_acc = out.self_acc;
  p.emit_acc = out.emit_acc;
  p.lvl_acc = out.lvl_acc;
  p.lvl_stride = out.lvl_stride;
  p.sub_lev = out.sub_lev;
  for (int a = 0; a < 3; ++a) p.sub_I[a] = out.sub_I[a];
  p.flux_acc = out.flux_acc;
  if ((out.lvl_acc || out.sub_lev >= 0) && fp32) {
    if (o->schedule != RT_SCHED_REGIONS)
      return fail(ctx, RT_EINVAL, "subiterations run in the RT_FP64 form or the region schedule");
    if (!out.lvl_acc || out.peel || out.e_lamnode)
      return fail(ctx, RT_EINVAL, "subiterations in the region schedule take no peel-off or per-wavelength "
                                  "output");
  }
  if (out.peel) {
    p.peel_ev = const_cast<PeelEv*>(out.peel->ev);
    p.peel_count = out.peel->count;
    p.peel_cap = out.peel->cap;
  }
  const int grid_peel = ctx->n_cu * 8;

  const bool regions = fp32 && o->schedule == RT_SCHED_REGIONS;
  // subiterations in the region schedule: the key slots are the shallowest level visited
  int n_lvl = 0;
  if (regions && out.lvl_acc)
    for (const HostModel& h : ctx->models) n_lvl = std::max(n_lvl, h.nlev + 1);
  const int key_slots = n_lvl > 0 ? n_lvl : n_slots;
  int reg_lds = 0, reg_per_cu = 0;
  if (regions) {
    // LDS per block: node words + accumulators (4 + 4 B per node) + parent links (4 B per oct)
    reg_per_cu = o->blocks_per_cu ? o->blocks_per_cu : (bs <= 256 ? 2 : 1);
    const int budget = 160 * 1024 / reg_per_cu - 4 * 1024;  // leave room for the static LDS
    int32_t cap = (int32_t)((budget * 8 / 68) & ~7);
    if (cap < 64) return fail(ctx, RT_EINVAL, "too many blocks per CU for the region schedule");
    reg_lds = 8 * cap + 4 * (cap / 8);
    if (rt_status e = build_regions(ctx, cap)) return e;
    HIPCHK(attr_blk_pass(bs, reg_lds));
    // region-major FP64 accumulators: one per node, per (wavelength, node) for per-wavelength
    // output, per (level, node) for subiterations
    const size_t racc = (size_t)key_slots * ctx->reg_G * 8;
    HIPCHK(ctx->acc.ensure(racc));
    HIPCHK(hipMemsetAsync(ctx->acc.p, 0, racc, ctx->stream));
  }
  double main_ms = 0.0;
  uint64_t main_launches = 0;
  HIPCHK(hipEventRecord(ctx->ev0, ctx->stream));
  if (start > 0 && regions) {
    RegionLaunch L;
    if (rt_status e = region_launch_setup(ctx, o, p, out, start, bs, reg_per_cu, reg_lds, key_slots, n_lvl, &L))
      return e;
    SweepState* st = L.st;
    SweepState init;  // stays alive until the first synchronisation below
    {
      std::memset(&init, 0, sizeof init);
      init.total = start;
      init.cap_all = (unsigned long long)L.cap_all;
      HIPCHK(hipEventRecord(ctx->ev_c, ctx->stream));
      HIPCHK(hipStreamWaitEvent(ctx->work, ctx->ev_c, 0));
      HIPCHK(hipMemcpyAsync(st, &init, sizeof init, hipMemcpyHostToDevice, ctx->work));
    }
    if ((int)ctx->sweep_ev.size() < 2 * kSweepBlock) {
      while ((int)ctx->sweep_ev.size() < 2 * kSweepBlock) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        ctx->sweep_ev.push_back(e);
      }
    }
    // capture the block as a graph (once per set of launch parameters), replay it until a
    // sweep finds the queues empty and nothing left to emit
    std::vector<char> sig(sizeof L.b + 6 * sizeof(int64_t) + (out.peel ? sizeof(PeelParams) : 0));
    {
      const int64_t extra[6] = {L.batch, L.capq, L.n_keys, L.grid_pass, L.bs, L.reg_lds};  // b holds split_n
      std::memcpy(sig.data(), &L.b, sizeof L.b);
      std::memcpy(sig.data() + sizeof L.b, extra, sizeof extra);
      if (out.peel) std::memcpy(sig.data() + sizeof L.b + sizeof extra, out.peel, sizeof(PeelParams));
    }
    const bool use_graph = o->sweep_graph > 0;
    if (use_graph && (!ctx->sweep_exec || sig != ctx->sweep_sig)) {
      if (ctx->sweep_exec) {
        HIPCHK(hipGraphExecDestroy(ctx->sweep_exec));
        ctx->sweep_exec = nullptr;
      }
      hipGraph_t graph = nullptr;
      HIPCHK(hipStreamBeginCapture(ctx->work, hipStreamCaptureModeThreadLocal));
      const hipError_t ce = enqueue_sweeps(ctx, L, ctx->work, nullptr);
      const hipError_t ee = hipStreamEndCapture(ctx->work, &graph);
      HIPCHK(ce);
      HIPCHK(ee);
      const hipError_t ie = hipGraphInstantiate(&ctx->sweep_exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      HIPCHK(ie);
      ctx->sweep_sig = sig;
    }
    int64_t blk = 0;
    for (;; ++blk) {
      if (use_graph) HIPCHK(hipGraphLaunch(ctx->sweep_exec, ctx->work));
      else HIPCHK(enqueue_sweeps(ctx, L, ctx->work, &ctx->sweep_ev));
      SweepState hs;
      HIPCHK(hipMemcpyAsync(&hs, st, sizeof hs, hipMemcpyDeviceToHost, ctx->work));
      HIPCHK(hipStreamSynchronize(ctx->work));
      // passes of sweeps that had packets to follow (events recorded by a replayed graph are
      // not timed: graph replays report no per-launch durations)
      for (int k = 0; k < kSweepBlock; ++k) {
        if (hs.log_in[k] == 0) continue;
        ++main_launches;
        if (use_graph) continue;
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ctx->sweep_ev[2 * k], ctx->sweep_ev[2 * k + 1]));
        main_ms += ms;
      }
      if (hs.done) break;
      if (blk > 2000000 / kSweepBlock) return fail(ctx, RT_EDEVICE, "region schedule did not drain");
    }
    ctx->last_sweep_blocks = blk + 1;
    if (out.save_launch) ctx->rl_saved = L;
    // later work on the caller's stream (the reduction) follows the sweeps
    HIPCHK(hipEventRecord(ctx->ev_c, ctx->work));
    HIPCHK(hipStreamWaitEvent(ctx->stream, ctx->ev_c, 0));
  } else if (start > 0) {
    if (fp32) {
      int per_cu = o->blocks_per_cu;
      if (per_cu == 0) {
        HIPCHK(occupancy_trace_fp32(bs, &per_cu));
        per_cu = std::max(per_cu, 1);
      }
      HIPCHK(launch_trace_fp32(p, ctx->n_cu * per_cu, bs, ctx->stream));
      main_launches = 1;
    } else {
      // splitting: packages split off go to a queue, followed by launches over the queue (each
      // appending to the other one) until it is empty
      const unsigned long long sq_cap = (unsigned long long)std::min<int64_t>(int64_t(1) << 22,
                                                                            std::max<int64_t>(4 * (int64_t)start, 4096));
      unsigned long long* cnt = nullptr;
      if (p.split_n > 1) {
        for (int k = 0; k < 2; ++k) HIPCHK(ctx->sq[k].ensure(sizeof(Split64) * sq_cap));
        HIPCHK(ctx->sq_cnt.ensure(2 * sizeof(unsigned long long)));
        cnt = ctx->sq_cnt.as<unsigned long long>();
        HIPCHK(hipMemsetAsync(cnt, 0, 2 * sizeof(unsigned long long), ctx->stream));
        p.sq_out = ctx->sq[0].as<Split64>();
        p.sq_count = cnt;
        p.sq_cap = sq_cap;
      }
      // back-to-back launches on one stream: their summed durations are the span ev0 -> ev1
      for (size_t k = 0; k < jobs.size(); ++k)
        if (jobs[k].n > 0) {
          HIPCHK(launch_trace_fp64(p, (int)k, jobs[k].n, bs, ctx->stream));
          ++main_launches;
          if (out.peel) HIPCHK(launch_peel(p, *out.peel, grid_peel, ctx->stream));
        }
      for (int cur = 0, round = 0; p.split_n > 1; cur = 1 - cur, ++round) {
        unsigned long long n_q = 0;
        HIPCHK(hipMemcpyAsync(&n_q, cnt + cur, sizeof n_q, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        if (n_q == 0) break;
        if (round > 100000) return fail(ctx, RT_EDEVICE, "split packages did not drain");
        HIPCHK(hipMemsetAsync(cnt + (1 - cur), 0, sizeof(unsigned long long), ctx->stream));
        p.sq_out = ctx->sq[1 - cur].as<Split64>();
        p.sq_count = cnt + (1 - cur);
        HIPCHK(launch_split_fp64(p, ctx->sq[cur].as<Split64>(), std::min(n_q, sq_cap), bs, ctx->stream));
        ++main_launches;
        if (out.peel) HIPCHK(launch_peel(p, *out.peel, grid_peel, ctx->stream));
      }
    }
  }
  HIPCHK(hipEventRecord(ctx->ev1, ctx->stream));
  if (regions) {
    HIPCHK(launch_blk_reduce(ctx->d_models.as<ModelDev>(), ctx->d_regions.as<RegionDev>(),
                             (int)ctx->h_regions.size(), ctx->reg_maxn, ctx->d_rcanon.as<int32_t>(),
                             ctx->acc.as<double>(), ctx->reg_G, key_slots, out.e_node,
                             n_lvl == 0 ? out.e_lamnode : nullptr,
                             n_lvl > 0 ? out.lvl_acc : nullptr, out.lvl_stride, ctx->e_total.as<double>(),
                             ctx->stream));
  } else {
    for (size_t m = 0; m < ctx->models.size(); ++m) {
      const HostModel& h = ctx->models[m];
      const int ns = n_slots > 1 ? std::max(h.nl, 1) : 1;
      HIPCHK(launch_reduce_model(ctx->d_models.as<ModelDev>(), (int)m, h.n_nodes, ctx->acc.as<double>(),
                                 stride, ns, out.e_node, out.e_lamnode, ctx->e_total.as<double>(),
                                 ctx->stream));
    }
  }
  HIPCHK(hipEventRecord(ctx->ev2, ctx->stream));
  if (rec_copy)
    HIPCHK(hipMemcpyAsync(o->records, rec_dev, sizeof(rt_record) * rec_base, hipMemcpyDeviceToHost,
                          ctx->stream));
  DevStats ds;
  double etot = 0.0;
  std::vector<double> esc(tot_lam);
  HIPCHK(hipMemcpyAsync(&ds, ctx->stats.p, sizeof ds, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipMemcpyAsync(&etot, ctx->e_total.p, 8, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipMemcpyAsync(esc.data(), out.e_esc, 8 * tot_lam, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (ds.misplaced)
    return fail(ctx, RT_EDEVICE,
                "internal error: %llu packet records were queued for a region that does not hold "
                "their cell; their energy is missing from the results",
                (unsigned long long)ds.misplaced);
  if (st_out) {
    float k_ms = 0.f, r_ms = 0.f;
    HIPCHK(hipEventElapsedTime(&k_ms, ctx->ev0, ctx->ev1));
    HIPCHK(hipEventElapsedTime(&r_ms, ctx->ev1, ctx->ev2));
    st_out->crossings = ds.crossings;
    st_out->scatterings = ds.scatterings;
    st_out->kills = ds.kills;
    st_out->truncated = ds.truncated;
    st_out->packets = ds.packets;
    st_out->e_emit = ds.e_emit;
    st_out->e_abs = etot;
    double ee = 0.0;
    for (double v : esc) ee += v;
    st_out->e_esc = ee;
    st_out->e_killed = ds.e_killed;
    st_out->e_rr_gain = ds.e_rr_gain;
    st_out->e_trunc = ds.e_trunc;
    st_out->kernel_ms = k_ms;
    st_out->reduce_ms = r_ms;
    st_out->main_ms = regions ? main_ms : k_ms;
    st_out->main_launches = main_launches;
    st_out->splits = ds.splits;
    st_out->split_kills = ds.split_kills;
    st_out->split_skips = ds.split_skips;
    st_out->e_split_killed = ds.e_split_killed;
    st_out->e_split_gain = ds.e_split_gain;
  }
  return RT_OK;
}

// Orthographic view of the maps (Sect. 4.1): v = {n, e1, e2, box centre, width} with
// e1 = z x n / |z x n| (x when n is along z), e2 = n x e1; width <= 0 takes the largest root
// extent.  False for a zero or non-finite direction or a non-finite width.
bool render_view(const HostModel& h, const double n_obs[3], double width, double v[13]) {
  const double nn = std::sqrt(n_obs[0] * n_obs[0] + n_obs[1] * n_obs[1] + n_obs[2] * n_obs[2]);
  if (!(nn > 0.0) || !std::isfinite(nn) || !std::isfinite(width)) return false;
  const double n[3] = {n_obs[0] / nn, n_obs[1] / nn, n_obs[2] / nn};
  double e1[3], e2[3];
  if (n[0] == 0.0 && n[1] == 0.0) {
    e1[0] = 1.0;
    e1[1] = 0.0;
    e1[2] = 0.0;
  } else {
    const double ex = -n[1], ey = n[0];
    const double en = std::sqrt(ex * ex + ey * ey);
    e1[0] = ex / en;
    e1[1] = ey / en;
    e1[2] = 0.0;
  }
  e2[0] = n[1] * e1[2] - n[2] * e1[1];
  e2[1] = n[2] * e1[0] - n[0] * e1[2];
  e2[2] = n[0] * e1[1] - n[1] * e1[0];
  double W = width;
  if (!(W > 0.0)) W = std::max<double>(h.n[0], std::max<double>(h.n[1], h.n[2]));
  for (int a = 0; a < 3; ++a) {
    v[a] = n[a];
    v[3 + a] = e1[a];
    v[6 + a] = e2[a];
    v[9 + a] = 0.5 * h.n[a];
  }
  v[12] = W;
  return true;
}

rt_status solve_T_impl(rt_ctx* ctx, int32_t model, const double* a_dev, double t_min, double t_max) {
  HostModel& h = ctx->models[model];
  HIPCHK(h.d_T.ensure(8 * h.n_nodes));
  HIPCHK(ctx->t_tab.ensure(8 * (4 + 2 * (size_t)kPlanckTable)));
  HIPCHK(launch_temperature(ctx->d_models.as<ModelDev>(), model, h.n_nodes, ctx->d_child.as<int32_t>(),
                            ctx->d_rho64.as<double>(), a_dev, h.d_lc.as<LamConst>(), h.nl, t_min,
                            t_max, ctx->t_tab.as<double>(), h.d_T.as<double>(), ctx->stream));
  h.has_T = true;
  return RT_OK;
}

}  // namespace

extern "C" {

rt_status rt_trace_packets(rt_ctx* ctx, int32_t n_src, const rt_source* src, const rt_trace_opts* o,
                           double* e_abs_node, double* e_abs_lambda_node, double* e_esc_lambda,
                           rt_trace_stats* stats) {
  if (!ctx) return fail(nullptr, RT_EINVAL, "null context");
  GUARD({
    HIPCHK(hipSetDevice(ctx->device));
    int64_t tn, tl, tln;
    totals(ctx, &tn, &tl, &tln);
    TraceOut out;
    void* pn = nullptr;
    void* pln = nullptr;
    void* pe = nullptr;
    bool cn = false, cln = false, ce = false;
    if (rt_status s = stage_out(ctx, e_abs_node, 8 * tn, ctx->out_node, &pn, &cn)) return s;
    if (rt_status s = stage_out(ctx, e_abs_lambda_node, 8 * std::max<int64_t>(tln, 1), ctx->out_lamnode, &pln, &cln))
      return s;
    if (e_esc_lambda) {
      if (rt_status s = stage_out(ctx, e_esc_lambda, 8 * std::max<int64_t>(tl, 1), ctx->out_esc, &pe, &ce)) return s;
    } else {
      HIPCHK(ctx->out_esc.ensure(8 * std::max<int64_t>(tl, 1)));
      pe = ctx->out_esc.p;
    }
    HIPCHK(ctx->last_node.ensure(8 * std::max<int64_t>(tn, 1)));
    out.e_node = pn ? static_cast<double*>(pn) : ctx->last_node.as<double>();
    out.e_lamnode = static_cast<double*>(pln);
    out.e_esc = static_cast<double*>(pe);
    ctx->last_nodes = -1;
    if (rt_status s = trace_impl(ctx, n_src, src, o, out, stats)) return s;
    // kept for rt_solve_temperature(a_node = NULL)
    if (pn) HIPCHK(hipMemcpyAsync(ctx->last_node.p, pn, 8 * tn, hipMemcpyDeviceToDevice, ctx->stream));
    ctx->last_nodes = tn;
    if (cn) HIPCHK(hipMemcpyAsync(e_abs_node, pn, 8 * tn, hipMemcpyDeviceToHost, ctx->stream));
    if (cln) HIPCHK(hipMemcpyAsync(e_abs_lambda_node, pln, 8 * tln, hipMemcpyDeviceToHost, ctx->stream));
    if (ce) HIPCHK(hipMemcpyAsync(e_esc_lambda, pe, 8 * tl, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RT_OK;
  })
}

rt_status rt_solve_temperature(rt_ctx* ctx, int32_t model, const double* a_node, double t_min,
                               double t_max, double* t_node) {
  if (!ctx) return fail(nullptr, RT_EINVAL, "null context");
  GUARD({
    if (rt_status s = check_model(ctx, model)) return s;
    if (!(t_min > 0.0) || !(t_max > t_min) || !std::isfinite(t_max))
      return fail(ctx, RT_EINVAL, "need 0 < t_min < t_max");
    HostModel& h = ctx->models[model];
    if (h.nl < 1) return fail(ctx, RT_ESTATE, "rt_set_dust not called for model %d", model);
    int64_t tn = 0;
    totals(ctx, &tn, nullptr, nullptr);
    if (!a_node && ctx->last_nodes != tn)
      return fail(ctx, RT_ESTATE, "a_node is NULL but no rt_trace_packets result covers the current models");
    if (rt_status s = sync_device(ctx)) return s;
    const void* da;
    if (!a_node) da = ctx->last_node.as<double>() + ctx->h_models[model].canon_base;
    else if (rt_status s = stage_in(ctx, a_node, 8 * h.n_nodes, ctx->tmp_in, &da)) return s;
    if (rt_status s = solve_T_impl(ctx, model, static_cast<const double*>(da), t_min, t_max)) return s;
    if (t_node)
      HIPCHK(hipMemcpyAsync(t_node, h.d_T.p, 8 * h.n_nodes,
                            is_device_ptr(t_node) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                            ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RT_OK;
  })
}

// A Lambda-iteration step captured as one HIP graph (region schedule): T_old <- T; the dust
// emission tables of every wavelength with their totals kept on the device; the trace (zeroed
// accumulators and tallies, sweep state, n_blocks blocks of sweeps); the FP64 reduction;
// A = A_stars + A_dust (or the accelerated update); the temperature solve; the stopping
// statistic.  The Philox key advances on the device at the start of each replay.  Built from the
// launch configuration of a direct step of the same iteration (same buffers and parameters).
struct StepGraph {
  hipGraphExec_t exec = nullptr;
  int64_t n_blocks = 0;
  RegionLaunch L;   // the direct step's configuration with the device job table and key
  uint64_t total = 0;
  ~StepGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
  }
};

// The step's work after its sweeps, on stream s (also run directly when a replay's sweeps did not
// drain).
static hipError_t step_post(rt_ctx* ctx, int32_t model, const StepGraph& G, bool ali, double t_min, double t_max,
                            hipStream_t s) {
  const HostModel& h = ctx->models[model];
  const int64_t cb = ctx->h_models[model].canon_base;
  hipError_t e;
  if ((e = launch_blk_reduce(ctx->d_models.as<ModelDev>(), ctx->d_regions.as<RegionDev>(), (int)ctx->h_regions.size(),
                             ctx->reg_maxn, ctx->d_rcanon.as<int32_t>(), ctx->acc.as<double>(), ctx->reg_G, 1,
                             ctx->it_adust.as<double>(), nullptr, nullptr, 0, ctx->e_total.as<double>(), s)) !=
      hipSuccess)
    return e;
  double* astars = ctx->it_astars.as<double>() + cb;
  e = ali ? launch_ali_absorbed(h.n_nodes, astars, ctx->it_adust.as<double>() + cb, ctx->it_self.as<double>() + cb,
                                ctx->it_emit.as<double>() + cb, ctx->it_sum.as<double>(), s)
          : launch_add(h.n_nodes, astars, ctx->it_adust.as<double>() + cb, ctx->it_sum.as<double>(), s);
  if (e != hipSuccess) return e;
  if ((e = launch_temperature(ctx->d_models.as<ModelDev>(), model, h.n_nodes, ctx->d_child.as<int32_t>(),
                              ctx->d_rho64.as<double>(), ctx->it_sum.as<double>(), h.d_lc.as<LamConst>(), h.nl, t_min,
                              t_max, ctx->t_tab.as<double>(), h.d_T.as<double>(), s)) != hipSuccess)
    return e;
  if ((e = launch_fill_u64(ctx->it_crit.p, 2, 0ull, s)) != hipSuccess) return e;
  if ((e = launch_crit(ctx->d_models.as<ModelDev>(), model, h.n_nodes, ctx->d_child.as<int32_t>(),
                       ctx->d_rho64.as<double>(), h.d_T.as<double>(), ctx->it_told.as<double>(),
                       ctx->it_crit.as<double>(), s)) != hipSuccess)
    return e;
  return launch_step_report(ctx->it_crit.as<double>(), G.L.st, ctx->stats.as<DevStats>(),
                            ctx->g_report.as<double>(), s);
}

static hipError_t step_record(rt_ctx* ctx, int32_t model, const StepGraph& G, bool ali, double t_min, double t_max,
                              hipStream_t s) {
  const HostModel& h = ctx->models[model];
  int64_t tn, tl, tln;
  totals(ctx, &tn, &tl, &tln);
  hipError_t e;
  if ((e = launch_step_key(ctx->g_keys.as<uint32_t>(), s)) != hipSuccess) return e;
  if ((e = launch_copy_u64(h.d_T.p, ctx->it_told.p, h.n_nodes, s)) != hipSuccess) return e;
  if (ali) {
    if ((e = launch_fill_u64(ctx->it_self.p, tn, 0ull, s)) != hipSuccess) return e;
    if ((e = launch_fill_u64(ctx->it_emit.p, tn, 0ull, s)) != hipSuccess) return e;
  }
  const int32_t no_sub[3] = {0, 0, 0};
  JobDev* jobs = ctx->g_jobs.as<JobDev>();
  for (int i = 0; i < h.nl; ++i) {
    const int64_t off = (int64_t)i * h.n_leaves;
    double* lum = ctx->cdf_lum.as<double>() + off;
    uint64_t* q = ctx->cdf_q.as<uint64_t>() + off;
    if ((e = launch_fill_u64(ctx->lmax.p, 2, 0ull, s)) != hipSuccess) return e;
    if ((e = launch_dust_lum(ctx->d_models.as<ModelDev>(), model, h.n_leaves, ctx->d_leaf_node.as<int32_t>(),
                             ctx->d_leaf_level.as<uint8_t>(), ctx->d_rho64.as<double>(), h.d_T.as<double>(),
                             h.d_lc.as<LamConst>(), i, lum, ctx->lmax.as<unsigned long long>(),
                             ctx->d_leaf_coord.as<int32_t>(), -1, no_sub, s)) != hipSuccess)
      return e;
    if ((e = launch_dust_quant(h.n_leaves, lum, ctx->lmax.as<unsigned long long>(), q, s)) != hipSuccess) return e;
    if ((e = launch_dust_scan(h.n_leaves, q, ctx->cdf_qpre.as<uint64_t>() + off, ctx->g_scan.as<uint64_t>(),
                              &jobs[i].qtot, s)) != hipSuccess)
      return e;
  }
  if ((e = launch_fill_u64(ctx->acc.p, ctx->reg_G, 0ull, s)) != hipSuccess) return e;
  if ((e = launch_fill_u64(ctx->stats.p, sizeof(DevStats) / 8, 0ull, s)) != hipSuccess) return e;
  if ((e = launch_fill_u64(ctx->e_total.p, 1, 0ull, s)) != hipSuccess) return e;
  if ((e = launch_fill_u64(ctx->out_esc.p, tl, 0ull, s)) != hipSuccess) return e;
  if ((e = launch_sweep_init(G.L.st, G.total, (uint64_t)G.L.cap_all, s)) != hipSuccess) return e;
  for (int64_t k = 0; k < G.n_blocks; ++k)
    if ((e = enqueue_sweeps(ctx, G.L, s, nullptr)) != hipSuccess) return e;
  return step_post(ctx, model, G, ali, t_min, t_max, s);
}

// Capture the step graph after a direct step of the same iteration (which left its launch
// configuration in ctx->rl_saved and its job table in ctx->jobs).  key1_done: the second key
// word of the direct step; every replay advances it by one first.
static rt_status step_build(rt_ctx* ctx, int32_t model, StepGraph& G, int64_t n_blocks, int64_t dust_packets,
                            uint32_t key0, uint32_t key1_done, bool ali, double t_min, double t_max) {
  const HostModel& h = ctx->models[model];
  if (G.exec) {
    HIPCHK(hipGraphExecDestroy(G.exec));
    G.exec = nullptr;
  }
  // the job table with every wavelength present (a wavelength with no emission is skipped on
  // the device from its table total) and the key in device memory
  std::vector<JobDev> jobs(h.nl);
  HIPCHK(hipMemcpyAsync(jobs.data(), ctx->jobs.p, sizeof(JobDev) * h.nl, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  uint64_t start = 0;
  for (int i = 0; i < h.nl; ++i) {
    if (jobs[i].kind != RT_SRC_DUST || jobs[i].lam != i || jobs[i].cdf_off != (int64_t)i * h.n_leaves)
      return fail(ctx, RT_EDEVICE, "internal error: unexpected dust job table");
    jobs[i].start = start;
    jobs[i].n = (uint64_t)dust_packets;
    jobs[i].qtot = 0;
    start += jobs[i].n;
  }
  if (rt_status e = upload(ctx, ctx->g_jobs, jobs)) return e;
  HIPCHK(ctx->g_keys.ensure(8));
  HIPCHK(ctx->g_scan.ensure(8 * std::max<int64_t>(dust_scan_tiles(h.n_leaves), 1)));
  HIPCHK(ctx->g_report.ensure(8 * 8));
  HIPCHK(ctx->lmax.ensure(16));
  ctx->g_keys_host[0] = key0;
  ctx->g_keys_host[1] = key1_done;
  HIPCHK(hipMemcpyAsync(ctx->g_keys.p, ctx->g_keys_host, 8, hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  G.L = ctx->rl_saved;
  G.L.b.t.jobs = ctx->g_jobs.as<JobDev>();
  G.L.b.t.n_jobs = h.nl;
  G.L.b.t.total_packets = start;
  G.L.b.t.keys = ctx->g_keys.as<uint32_t>();
  G.total = start;
  G.n_blocks = n_blocks;
  hipGraph_t graph = nullptr;
  HIPCHK(hipStreamBeginCapture(ctx->work, hipStreamCaptureModeThreadLocal));
  const hipError_t ce = step_record(ctx, model, G, ali, t_min, t_max, ctx->work);
  const hipError_t ee = hipStreamEndCapture(ctx->work, &graph);
  HIPCHK(ce);
  HIPCHK(ee);
  const hipError_t ie = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  HIPCHK(ie);
  return RT_OK;
}

// One replay of the step graph; when its sweeps did not drain (more than the captured blocks
// were needed), the remaining sweeps and the work after them run directly.  report: the
// stopping statistic's numerator and denominator, whether the replayed sweeps drained, the
// step's crossings and misplaced queue records.
static rt_status step_replay(rt_ctx* ctx, int32_t model, StepGraph& G, bool ali, double t_min, double t_max,
                             double report[5], bool* drained) {
  HIPCHK(hipEventRecord(ctx->ev_c, ctx->stream));
  HIPCHK(hipStreamWaitEvent(ctx->work, ctx->ev_c, 0));
  HIPCHK(hipGraphLaunch(G.exec, ctx->work));
  HIPCHK(hipMemcpyAsync(report, ctx->g_report.p, 40, hipMemcpyDeviceToHost, ctx->work));
  HIPCHK(hipStreamSynchronize(ctx->work));
  *drained = report[2] != 0.0;
  if (!*drained) {
    for (int64_t blk = 0;; ++blk) {
      HIPCHK(enqueue_sweeps(ctx, G.L, ctx->work, nullptr));
      SweepState hs;
      HIPCHK(hipMemcpyAsync(&hs, G.L.st, sizeof hs, hipMemcpyDeviceToHost, ctx->work));
      HIPCHK(hipStreamSynchronize(ctx->work));
      if (hs.done) break;
      if (blk > 2000000 / kSweepBlock) return fail(ctx, RT_EDEVICE, "region schedule did not drain");
    }
    HIPCHK(step_post(ctx, model, G, ali, t_min, t_max, ctx->work));
    HIPCHK(hipMemcpyAsync(report, ctx->g_report.p, 40, hipMemcpyDeviceToHost, ctx->work));
    HIPCHK(hipStreamSynchronize(ctx->work));
  }
  if (report[4] != 0.0)
    return fail(ctx, RT_EDEVICE, "internal error: %.0f packet records were queued for the wrong region", report[4]);
  HIPCHK(hipEventRecord(ctx->ev_c, ctx->work));
  HIPCHK(hipStreamWaitEvent(ctx->stream, ctx->ev_c, 0));
  return RT_OK;
}

static rt_status lambda_iterate_impl(rt_ctx* ctx, int32_t model, int32_t n_src, const rt_source* src,
                                     const rt_trace_opts* opts, int64_t dust_packets, int32_t n_max,
                                     double tol, double t_min, double t_max, double* t_node,
                                     int32_t* n_done, double* crit, bool ali) {
  if (!ctx) return fail(nullptr, RT_EINVAL, "null context");
  GUARD({
    if (ali && opts && opts->precision == RT_FP32_LOCAL && opts->schedule != RT_SCHED_REGIONS)
      return fail(ctx, RT_EINVAL, "the accelerated iteration needs RT_FP64 or the region schedule");
    if (rt_status s = check_model(ctx, model)) return s;
    if (n_max < 0 || n_max > 100000) return fail(ctx, RT_EINVAL, "bad n_max");
    if (!(tol >= 0.0)) return fail(ctx, RT_EINVAL, "bad tol");
    if (dust_packets < 1 || dust_packets > (int64_t(1) << 32)) return fail(ctx, RT_EINVAL, "bad dust_packets");
    if (!(t_min > 0.0) || !(t_max > t_min)) return fail(ctx, RT_EINVAL, "need 0 < t_min < t_max");
    if (!opts) return fail(ctx, RT_EINVAL, "null options");
    for (int s = 0; s < n_src; ++s)
      if (src && (src[s].model != model || src[s].kind == RT_SRC_DUST))
        return fail(ctx, RT_EINVAL, "constant sources must belong to the model and not be dust");
    HostModel& h = ctx->models[model];
    if (h.nl < 1) return fail(ctx, RT_ESTATE, "rt_set_dust not called for model %d", model);
    HIPCHK(hipSetDevice(ctx->device));
    if (rt_status s = sync_device(ctx)) return s;
    int64_t tn, tl, tln;
    totals(ctx, &tn, &tl, &tln);
    const int64_t cb = ctx->h_models[model].canon_base;
    HIPCHK(ctx->it_astars.ensure(8 * tn));
    HIPCHK(ctx->it_adust.ensure(8 * tn));
    HIPCHK(ctx->it_sum.ensure(8 * h.n_nodes));
    HIPCHK(ctx->it_told.ensure(8 * h.n_nodes));
    HIPCHK(ctx->it_crit.ensure(16));
    if (ali) {
      HIPCHK(ctx->it_self.ensure(8 * tn));
      HIPCHK(ctx->it_emit.ensure(8 * tn));
    }
    HIPCHK(ctx->out_esc.ensure(8 * std::max<int64_t>(tl, 1)));
    TraceOut out;
    out.e_esc = ctx->out_esc.as<double>();
    rt_trace_opts o = *opts;
    double* astars = ctx->it_astars.as<double>() + cb;
    if (n_src > 0) {
      out.e_node = ctx->it_astars.as<double>();
      o.iteration = opts->iteration;
      if (rt_status s = trace_impl(ctx, n_src, src, &o, out, nullptr)) return s;
    } else {
      HIPCHK(hipMemsetAsync(ctx->it_astars.p, 0, 8 * tn, ctx->stream));
    }
    if (rt_status s = solve_T_impl(ctx, model, astars, t_min, t_max)) return s;
    // captured steps: the region schedule with sweep_graph > 0; the first step runs directly
    // and gives the launch configuration and the number of sweeps to capture
    const bool graph = opts->sweep_graph > 0 && opts->precision == RT_FP32_LOCAL && opts->schedule == RT_SCHED_REGIONS;
    StepGraph G;
    const uint32_t key0 = (uint32_t)(opts->seed & 0xffffffffu);
    const uint32_t key1_base = (uint32_t)(opts->seed >> 32) + opts->iteration;
    int32_t n = 0;
    for (int32_t it = 1; it <= n_max; ++it) {
      if (graph && G.exec) {
        double rep[5];
        bool drained = false;
        if (rt_status s = step_replay(ctx, model, G, ali, t_min, t_max, rep, &drained)) return s;
        const double cval = rep[1] > 0.0 ? rep[0] / rep[1] : 0.0;
        if (crit) crit[it - 1] = cval;
        n = it;
        // a replay whose sweeps did not drain was completed directly: capture more sweeps
        if (!drained && it < n_max)
          if (rt_status s = step_build(ctx, model, G, G.n_blocks + 2, dust_packets, key0,
                                       key1_base + (uint32_t)it, ali, t_min, t_max))
            return s;
        if (cval < tol) break;
        continue;
      }
      rt_source ds;
      std::memset(&ds, 0, sizeof ds);
      ds.kind = RT_SRC_DUST;
      ds.model = model;
      ds.packets_per_lambda = dust_packets;
      o.iteration = opts->iteration + (uint32_t)it;
      out.e_node = ctx->it_adust.as<double>();
      out.save_launch = graph;
      if (ali) {
        HIPCHK(hipMemsetAsync(ctx->it_self.p, 0, 8 * tn, ctx->stream));
        HIPCHK(hipMemsetAsync(ctx->it_emit.p, 0, 8 * tn, ctx->stream));
        out.self_acc = ctx->it_self.as<double>();
        out.emit_acc = ctx->it_emit.as<double>();
      }
      if (rt_status s = trace_impl(ctx, 1, &ds, &o, out, nullptr)) return s;
      if (ali)
        HIPCHK(launch_ali_absorbed(h.n_nodes, astars, ctx->it_adust.as<double>() + cb,
                                   ctx->it_self.as<double>() + cb, ctx->it_emit.as<double>() + cb,
                                   ctx->it_sum.as<double>(), ctx->stream));
      else
        HIPCHK(launch_add(h.n_nodes, astars, ctx->it_adust.as<double>() + cb, ctx->it_sum.as<double>(),
                          ctx->stream));
      HIPCHK(hipMemcpyAsync(ctx->it_told.p, h.d_T.p, 8 * h.n_nodes, hipMemcpyDeviceToDevice, ctx->stream));
      if (rt_status s = solve_T_impl(ctx, model, ctx->it_sum.as<double>(), t_min, t_max)) return s;
      HIPCHK(hipMemsetAsync(ctx->it_crit.p, 0, 16, ctx->stream));
      HIPCHK(launch_crit(ctx->d_models.as<ModelDev>(), model, h.n_nodes, ctx->d_child.as<int32_t>(),
                         ctx->d_rho64.as<double>(), h.d_T.as<double>(), ctx->it_told.as<double>(),
                         ctx->it_crit.as<double>(), ctx->stream));
      double c2[2];
      HIPCHK(hipMemcpyAsync(c2, ctx->it_crit.p, 16, hipMemcpyDeviceToHost, ctx->stream));
      HIPCHK(hipStreamSynchronize(ctx->stream));
      const double cval = c2[1] > 0.0 ? c2[0] / c2[1] : 0.0;
      if (crit) crit[it - 1] = cval;
      n = it;
      if (cval < tol) break;
      if (graph && it < n_max)
        if (rt_status s = step_build(ctx, model, G, ctx->last_sweep_blocks + 1, dust_packets, key0,
                                     key1_base + (uint32_t)it, ali, t_min, t_max))
          return s;
    }
    if (n_done) *n_done = n;
    if (t_node)
      HIPCHK(hipMemcpyAsync(t_node, h.d_T.p, 8 * h.n_nodes,
                            is_device_ptr(t_node) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                            ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RT_OK;
  })
}

rt_status rt_lambda_iterate(rt_ctx* ctx, int32_t model, int32_t n_src, const rt_source* src,
                            const rt_trace_opts* opts, int64_t dust_packets, int32_t n_max,
                            double tol, double t_min, double t_max, double* t_node,
                            int32_t* n_done, double* crit) {
  return lambda_iterate_impl(ctx, model, n_src, src, opts, dust_packets, n_max, tol, t_min, t_max, t_node,
                             n_done, crit, false);
}

rt_status rt_ali_iterate(rt_ctx* ctx, int32_t model, int32_t n_src, const rt_source* src,
                         const rt_trace_opts* opts, int64_t dust_packets, int32_t n_max, double tol,
                         double t_min, double t_max, double* t_node, int32_t* n_done, double* crit) {
  return lambda_iterate_impl(ctx, model, n_src, src, opts, dust_packets, n_max, tol, t_min, t_max, t_node,
                             n_done, crit, true);
}

}  // extern "C"

namespace {

// Nodes of the subtree below refined node `root` (root itself excluded; all nodes for -1), from
// the canonical parents (a parent precedes its children in canonical order).
std::vector<char> subtree_of(const HostModel& h, int64_t root) {
  std::vector<char> in(h.n_nodes, root < 0 ? 1 : 0);
  if (root >= 0)
    for (int64_t c = h.n_root; c < h.n_nodes; ++c) {
      const int64_t pc = h.sub_parent[c];
      in[c] = (pc == root || in[pc]) ? 1 : 0;
    }
  return in;
}

// After a step below `root` (Sect. 3.3): the energy flow from the root's subtree into its parent
// grid is compared with what it was when that parent grid last took part in a step; a change
// above flux_frac of the energy the parent grid absorbs tags the parent grid for the next step.
// The refined nodes below the root get their new reference flows (their parent grids took part),
// and every grid of this step loses its tag.
void subiter_flux_update(rt_ctx* ctx, int32_t model, int64_t root, const std::vector<double>& flux,
                         const std::vector<double>& a_tot) {
  HostModel& h = ctx->models[model];
  const int64_t pad0 = h.n_root_pad - h.n_root;
  auto refined = [&](int64_t c) { return ctx->h_child[h.base + (c < h.n_root ? c : c + pad0)] >= 0; };
  const std::vector<char> in = subtree_of(h, root);
  if (root >= 0) {
    const int64_t par = h.sub_parent[root];  // -1: the root grid
    const std::vector<char> in_par = subtree_of(h, par);
    double absorbed = 0.0;
    for (int64_t c = 0; c < h.n_nodes; ++c)
      if (in_par[c] && !refined(c)) absorbed += a_tot[c];
    if (std::fabs(flux[root] - h.sub_flux_ref[root]) > h.sub_flux_frac * absorbed) {
      if (par < 0) h.sub_tag_root = true;
      else h.sub_tag[par] = 1;
    }
  }
  for (int64_t c = 0; c < h.n_nodes; ++c)
    if (in[c] && refined(c)) {
      h.sub_flux_ref[c] = flux[c];
      h.sub_tag[c] = 0;
    }
  if (root >= 0) h.sub_tag[root] = 0;
  else h.sub_tag_root = false;
}

}  // namespace

extern "C" {

rt_status rt_subiter_begin(rt_ctx* ctx, int32_t model, int32_t n_src, const rt_source* src,
                           const rt_trace_opts* opts, double t_min, double t_max, double flux_frac,
                           int32_t ali) {
  if (!ctx) return fail(nullptr, RT_EINVAL, "null context");
  GUARD({
    if (rt_status s = check_model(ctx, model)) return s;
    if (!opts) return fail(ctx, RT_EINVAL, "null options");
    if (!(opts->precision == RT_FP64 || (opts->precision == RT_FP32_LOCAL && opts->schedule == RT_SCHED_REGIONS)))
      return fail(ctx, RT_EINVAL, "subiterations run in the RT_FP64 form or the region schedule");
    if (!(t_min > 0.0) || !(t_max > t_min)) return fail(ctx, RT_EINVAL, "need 0 < t_min < t_max");
    if (!(flux_frac >= 0.0) || !std::isfinite(flux_frac)) return fail(ctx, RT_EINVAL, "flux_frac must be >= 0");
    for (int s = 0; s < n_src; ++s)
      if (src && (src[s].model != model || src[s].kind == RT_SRC_DUST))
        return fail(ctx, RT_EINVAL, "constant sources must belong to the model and not be dust");
    HostModel& h = ctx->models[model];
    if (h.nl < 1) return fail(ctx, RT_ESTATE, "rt_set_dust not called for model %d", model);
    HIPCHK(hipSetDevice(ctx->device));
    if (rt_status s = sync_device(ctx)) return s;
    int64_t tn, tl, tln;
    totals(ctx, &tn, &tl, &tln);
    const int64_t cb = ctx->h_models[model].canon_base;
    HIPCHK(ctx->it_astars.ensure(8 * tn));
    HIPCHK(ctx->out_esc.ensure(8 * std::max<int64_t>(tl, 1)));
    // canonical parents (the flux bookkeeping of the automatic iteration)
    h.sub_parent.assign(h.n_nodes, -1);
    {
      const int64_t pad0 = h.n_root_pad - h.n_root;
      for (int64_t c = h.n_root; c < h.n_nodes; ++c) {
        const int64_t pi = ctx->h_up[(h.base + c + pad0) >> 3];
        const int64_t pc = pi - h.base;
        h.sub_parent[c] = pc < h.n_root ? pc : pc - pad0;
      }
    }
    h.sub_flux_frac = flux_frac;
    h.sub_ali = ali != 0;
    h.sub_flux_ref.assign(h.n_nodes, 0.0);
    h.sub_tag.assign(h.n_nodes, 0);
    h.sub_tag_root = false;
    if (n_src > 0) {
      TraceOut out;
      out.e_esc = ctx->out_esc.as<double>();
      out.e_node = ctx->it_astars.as<double>();
      if (rt_status s = trace_impl(ctx, n_src, src, opts, out, nullptr)) return s;
    } else {
      HIPCHK(hipMemsetAsync(ctx->it_astars.p, 0, 8 * tn, ctx->stream));
    }
    HIPCHK(h.sub_astars.ensure(8 * h.n_nodes));
    HIPCHK(hipMemcpyAsync(h.sub_astars.p, ctx->it_astars.as<double>() + cb, 8 * h.n_nodes,
                          hipMemcpyDeviceToDevice, ctx->stream));
    const size_t na = (size_t)(h.nlev + 1) * h.n_nodes;
    HIPCHK(h.sub_arrays.ensure(8 * na));
    HIPCHK(hipMemsetAsync(h.sub_arrays.p, 0, 8 * na, ctx->stream));
    HIPCHK(h.sub_imb.ensure(8 * h.n_nodes));
    HIPCHK(hipMemsetAsync(h.sub_imb.p, 0, 8 * h.n_nodes, ctx->stream));
    if (rt_status s = solve_T_impl(ctx, model, h.sub_astars.as<double>(), t_min, t_max)) return s;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    h.sub_tmin = t_min;
    h.sub_tmax = t_max;
    h.sub_ready = true;
    return RT_OK;
  })
}

rt_status rt_subiter_step(rt_ctx* ctx, int32_t model, int64_t root, int64_t dust_packets, uint32_t iteration,
                          const rt_trace_opts* opts, double* crit, double* t_node, rt_trace_stats* stats) {
  if (!ctx) return fail(nullptr, RT_EINVAL, "null context");
  GUARD({
    if (rt_status s = check_model(ctx, model)) return s;
    if (!opts) return fail(ctx, RT_EINVAL, "null options");
    if (!(opts->precision == RT_FP64 || (opts->precision == RT_FP32_LOCAL && opts->schedule == RT_SCHED_REGIONS)))
      return fail(ctx, RT_EINVAL, "subiterations run in the RT_FP64 form or the region schedule");
    HostModel& h = ctx->models[model];
    if (!h.sub_ready) return fail(ctx, RT_ESTATE, "rt_subiter_begin not called for model %d", model);
    if (dust_packets < 1 || dust_packets > (int64_t(1) << 32)) return fail(ctx, RT_EINVAL, "bad dust_packets");
    if (root < -1 || root >= h.n_nodes) return fail(ctx, RT_EINVAL, "bad subtree root");
    int32_t sub_lev = -1, sub_I[3] = {0, 0, 0};
    if (root >= 0) {
      // canonical -> internal, its level and coordinates; it must be refined
      const int64_t internal = h.base + (root < h.n_root ? root : root + (h.n_root_pad - h.n_root));
      if (ctx->h_child[internal] < 0) return fail(ctx, RT_EINVAL, "the subtree root must be a refined node");
      int lev = 0;
      while (lev < h.nlev && root >= h.level_off[lev + 1]) ++lev;
      int64_t li = root - h.level_off[lev];
      // coordinates: walk the level index back to the root (oct o, child b = bx + 2 by + 4 bz)
      int32_t I[3] = {0, 0, 0};
      int sh = 0;
      int64_t cur = internal;
      for (int l = lev; l > 0; --l) {
        const int b = (int)(cur & 7);
        I[0] |= (b & 1) << sh;
        I[1] |= ((b >> 1) & 1) << sh;
        I[2] |= ((b >> 2) & 1) << sh;
        ++sh;
        cur = ctx->h_up[cur >> 3];
      }
      const int64_t r = cur - h.base;
      I[0] |= (int32_t)(r % h.n[0]) << sh;
      I[1] |= (int32_t)((r / h.n[0]) % h.n[1]) << sh;
      I[2] |= (int32_t)(r / ((int64_t)h.n[0] * h.n[1])) << sh;
      (void)li;
      sub_lev = lev;
      for (int a = 0; a < 3; ++a) sub_I[a] = I[a];
    }
    HIPCHK(hipSetDevice(ctx->device));
    if (rt_status s = sync_device(ctx)) return s;
    int64_t tn, tl, tln;
    totals(ctx, &tn, &tl, &tln);
    const int64_t cb = ctx->h_models[model].canon_base;
    // level arrays for every level of every model on the device (the region schedule's
    // reduction writes one per level of the deepest model)
    size_t nlv = 1;
    for (const HostModel& hm : ctx->models) nlv = std::max(nlv, (size_t)(hm.nlev + 1));
    HIPCHK(ctx->it_adust.ensure(8 * tn));
    HIPCHK(ctx->it_sum.ensure(8 * h.n_nodes));
    HIPCHK(ctx->it_told.ensure(8 * h.n_nodes));
    HIPCHK(ctx->it_crit.ensure(16));
    HIPCHK(ctx->it_self.ensure(8 * nlv * tn));  // per-level deposits of this step
    HIPCHK(hipMemsetAsync(ctx->it_self.p, 0, 8 * nlv * tn, ctx->stream));
    HIPCHK(ctx->out_esc.ensure(8 * std::max<int64_t>(tl, 1)));
    HIPCHK(hipMemcpyAsync(ctx->it_told.p, h.d_T.p, 8 * h.n_nodes, hipMemcpyDeviceToDevice, ctx->stream));
    rt_source ds;
    std::memset(&ds, 0, sizeof ds);
    ds.kind = RT_SRC_DUST;
    ds.model = model;
    ds.packets_per_lambda = dust_packets;
    rt_trace_opts o = *opts;
    o.iteration = iteration;
    TraceOut out;
    out.e_esc = ctx->out_esc.as<double>();
    out.e_node = ctx->it_adust.as<double>();
    out.lvl_acc = ctx->it_self.as<double>();
    out.lvl_stride = tn;
    out.sub_lev = sub_lev;
    for (int a = 0; a < 3; ++a) out.sub_I[a] = sub_I[a];
    if (h.sub_flux_frac > 0.0) {
      HIPCHK(ctx->it_emit.ensure(8 * tn));
      HIPCHK(hipMemsetAsync(ctx->it_emit.p, 0, 8 * tn, ctx->stream));
      out.flux_acc = ctx->it_emit.as<double>();
    }
    if (h.sub_ali) {
      // the diagonal operator's tallies: what each leaf's own emission deposited in it before its
      // packets first left it, and what it emitted
      HIPCHK(ctx->it_aself.ensure(8 * tn));
      HIPCHK(ctx->it_aemit.ensure(8 * tn));
      HIPCHK(ctx->it_asolve.ensure(8 * h.n_nodes));
      HIPCHK(hipMemsetAsync(ctx->it_aself.p, 0, 8 * tn, ctx->stream));
      HIPCHK(hipMemsetAsync(ctx->it_aemit.p, 0, 8 * tn, ctx->stream));
      out.self_acc = ctx->it_aself.as<double>();
      out.emit_acc = ctx->it_aemit.as<double>();
    }
    if (rt_status s = trace_impl(ctx, 1, &ds, &o, out, stats)) return s;
    HIPCHK(launch_subiter_update(ctx->d_models.as<ModelDev>(), model, h.n_leaves, ctx->d_leaf_node.as<int32_t>(),
                                 ctx->d_leaf_level.as<uint8_t>(), ctx->d_leaf_coord.as<int32_t>(),
                                 ctx->d_rho64.as<double>(), h.d_lc.as<LamConst>(), h.nl, sub_lev, sub_I,
                                 sub_lev + 1, ctx->it_self.as<double>(), tn, h.sub_arrays.as<double>(),
                                 h.sub_astars.as<double>(), ctx->it_told.as<double>(), ctx->it_sum.as<double>(),
                                 h.sub_imb.as<double>(), ctx->stream));
    const double* a_solve = ctx->it_sum.as<double>();
    if (h.sub_ali) {
      HIPCHK(launch_subiter_ali(ctx->d_models.as<ModelDev>(), model, h.n_nodes, h.n_leaves,
                                ctx->d_leaf_node.as<int32_t>(), ctx->d_leaf_level.as<uint8_t>(),
                                ctx->d_leaf_coord.as<int32_t>(), sub_lev, sub_I, ctx->it_sum.as<double>(),
                                ctx->it_aself.as<double>() + cb, ctx->it_aemit.as<double>() + cb,
                                ctx->it_asolve.as<double>(), ctx->stream));
      a_solve = ctx->it_asolve.as<double>();
    }
    if (rt_status s = solve_T_impl(ctx, model, a_solve, h.sub_tmin, h.sub_tmax)) return s;
    if (h.sub_ali)
      HIPCHK(launch_subiter_keep(ctx->d_models.as<ModelDev>(), model, h.n_leaves, ctx->d_leaf_node.as<int32_t>(),
                                 ctx->d_leaf_level.as<uint8_t>(), ctx->d_leaf_coord.as<int32_t>(), sub_lev, sub_I,
                                 ctx->it_told.as<double>(), h.d_T.as<double>(), ctx->stream));
    HIPCHK(hipMemsetAsync(ctx->it_crit.p, 0, 16, ctx->stream));
    HIPCHK(launch_crit(ctx->d_models.as<ModelDev>(), model, h.n_nodes, ctx->d_child.as<int32_t>(),
                       ctx->d_rho64.as<double>(), h.d_T.as<double>(), ctx->it_told.as<double>(),
                       ctx->it_crit.as<double>(), ctx->stream));
    double c2[2];
    HIPCHK(hipMemcpyAsync(c2, ctx->it_crit.p, 16, hipMemcpyDeviceToHost, ctx->stream));
    if (t_node)
      HIPCHK(hipMemcpyAsync(t_node, h.d_T.p, 8 * h.n_nodes,
                            is_device_ptr(t_node) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, ctx->stream));
    std::vector<double> flux, a_tot;
    if (h.sub_flux_frac > 0.0) {
      flux.resize(h.n_nodes);
      a_tot.resize(h.n_nodes);
      HIPCHK(hipMemcpyAsync(flux.data(), ctx->it_emit.as<double>() + cb, 8 * h.n_nodes, hipMemcpyDeviceToHost,
                            ctx->stream));
      HIPCHK(hipMemcpyAsync(a_tot.data(), ctx->it_sum.p, 8 * h.n_nodes, hipMemcpyDeviceToHost, ctx->stream));
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (crit) *crit = c2[1] > 0.0 ? c2[0] / c2[1] : 0.0;
    if (h.sub_flux_frac > 0.0) subiter_flux_update(ctx, model, root, flux, a_tot);
    return RT_OK;
  })
}

rt_status rt_subiter_select(rt_ctx* ctx, int32_t model, double frac, int64_t* root, double* max_imbalance) {
  if (!ctx) return fail(nullptr, RT_EINVAL, "null context");
  GUARD({
    if (rt_status s = check_model(ctx, model)) return s;
    if (!root || !(frac > 0.0 && frac <= 1.0)) return fail(ctx, RT_EINVAL, "need frac in (0, 1] and root");
    HostModel& h = ctx->models[model];
    if (!h.sub_ready) return fail(ctx, RT_ESTATE, "rt_subiter_begin not called for model %d", model);
    HIPCHK(hipSetDevice(ctx->device));
    std::vector<double> imb(h.n_nodes);
    HIPCHK(hipMemcpyAsync(imb.data(), h.sub_imb.p, 8 * h.n_nodes, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    double mx = 0.0;
    for (double v : imb) mx = std::max(mx, v);
    if (max_imbalance) *max_imbalance = mx;
    // the lowest common ancestor of every leaf within frac of the largest imbalance; a common
    // ancestor above the root level means the whole model
    auto internal_of = [&](int64_t c) { return h.base + (c < h.n_root ? c : c + (h.n_root_pad - h.n_root)); };
    auto canon_of_h = [&](int64_t i) {
      const int64_t c = i - h.base;
      return c < h.n_root ? c : c - (h.n_root_pad - h.n_root);
    };
    auto level_of = [&](int64_t c) {
      int l = 0;
      while (l < h.nlev && c >= h.level_off[l + 1]) ++l;
      return l;
    };
    auto parent = [&](int64_t c) -> int64_t {  // canonical parent, -1 for a root cell
      if (c < h.n_root) return -1;
      const int64_t i = internal_of(c);
      return canon_of_h(ctx->h_up[i >> 3]);
    };
    // a grid tagged because the energy flowing into it from a child changed (Sect. 3.3) must be
    // in the next step too: the root grid's tag means the whole model
    int64_t lca = h.sub_tag_root ? -1 : -2;  // -2: none yet
    for (int64_t c = 0; c < h.n_nodes && lca != -1; ++c) {
      const bool tagged = h.sub_tag.size() == (size_t)h.n_nodes && h.sub_tag[c];
      if (!tagged && (!(mx > 0.0) || imb[c] < frac * mx)) continue;
      int64_t a = tagged ? c : parent(c);
      if (lca == -2) {
        lca = a;
        continue;
      }
      // walk both up to the same level, then together
      int64_t x = lca, y = a;
      while (x >= 0 && y >= 0 && x != y) {
        const int lx = level_of(x), ly = level_of(y);
        if (lx >= ly) x = parent(x);
        if (ly >= lx) y = parent(y);
      }
      lca = (x >= 0 && y >= 0) ? x : -1;
    }
    *root = lca < 0 ? -1 : lca;
    return RT_OK;
  })
}

rt_status rt_subiter_run(rt_ctx* ctx, int32_t model, int32_t n_steps, double frac, double stall,
                         int64_t dust_packets, uint32_t first_iteration, const rt_trace_opts* opts,
                         int64_t* roots, double* crit, uint64_t* crossings, double* t_node) {
  if (!ctx) return fail(nullptr, RT_EINVAL, "null context");
  if (n_steps < 1 || n_steps > 100000) return fail(ctx, RT_EINVAL, "bad n_steps");
  if (!(stall > 0.0 && stall <= 1.0)) return fail(ctx, RT_EINVAL, "stall must be in (0, 1]");
  int64_t prev_root = -2;
  double prev_max = 0.0;
  for (int32_t k = 0; k < n_steps; ++k) {
    int64_t root = -1;
    if (k > 0) {
      double mx = 0.0;
      if (rt_status s = rt_subiter_select(ctx, model, frac, &root, &mx)) return s;
      // the same subtree again without a clear drop of the largest imbalance: the noise limit
      // of that subtree; take the whole model instead (Sect. 3.3)
      if (root >= 0 && root == prev_root && mx > stall * prev_max) root = -1;
      prev_max = mx;
    }
    rt_trace_stats st;
    std::memset(&st, 0, sizeof st);
    double c = 0.0;
    if (rt_status s = rt_subiter_step(ctx, model, root, dust_packets, first_iteration + (uint32_t)k, opts, &c,
                                      k == n_steps - 1 ? t_node : nullptr, &st))
      return s;
    prev_root = root;
    if (roots) roots[k] = root;
    if (crit) crit[k] = c;
    if (crossings) crossings[k] = st.crossings;
  }
  return RT_OK;
}

rt_status rt_render_map(rt_ctx* ctx, int32_t model, const double n_obs[3], int32_t npix, double width,
                        int32_t n_sel, const int32_t* lambda_idx, int32_t precision, double* image,
                        uint64_t* crossings) {
  if (!ctx) return fail(nullptr, RT_EINVAL, "null context");
  GUARD({
    if (rt_status s = check_model(ctx, model)) return s;
    if (!n_obs || !lambda_idx || !image) return fail(ctx, RT_EINVAL, "null argument");
    if (npix < 1 || npix > 16384) return fail(ctx, RT_EINVAL, "npix must be in [1, 16384]");
    if (n_sel < 1) return fail(ctx, RT_EINVAL, "n_sel must be >= 1");
    if (precision != RT_FP64 && precision != RT_FP32_LOCAL)
      return fail(ctx, RT_EINVAL, "precision must be RT_FP64 or RT_FP32_LOCAL");
    HostModel& h = ctx->models[model];
    if (h.nl < 1) return fail(ctx, RT_ESTATE, "rt_set_dust not called for model %d", model);
    if (!h.has_T) return fail(ctx, RT_ESTATE, "model %d has no temperatures", model);
    for (int q = 0; q < n_sel; ++q)
      if (lambda_idx[q] < 0 || lambda_idx[q] >= h.nl) return fail(ctx, RT_EINVAL, "bad wavelength index");
    double v[13];
    if (!render_view(h, n_obs, width, v)) return fail(ctx, RT_EINVAL, "bad view direction or width");
    if (rt_status s = sync_device(ctx)) return s;
    HIPCHK(ctx->view.ensure(sizeof v));
    HIPCHK(hipMemcpyAsync(ctx->view.p, v, sizeof v, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx->lamidx.ensure(4 * n_sel));
    HIPCHK(hipMemcpyAsync(ctx->lamidx.p, lambda_idx, 4 * n_sel, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx->counter.ensure(8));
    HIPCHK(hipMemsetAsync(ctx->counter.p, 0, 8, ctx->stream));
    const size_t img_bytes = 8 * (size_t)n_sel * npix * npix;
    void* dimg;
    bool copy;
    if (rt_status s = stage_out(ctx, image, img_bytes, ctx->tmp_out, &dimg, &copy)) return s;
    const int pass = precision == RT_FP32_LOCAL ? kRenderPassF32 : kRenderPassF64;
    for (int q0 = 0; q0 < n_sel; q0 += pass) {
      const int nq = std::min(pass, n_sel - q0);
      HIPCHK(launch_render(precision == RT_FP32_LOCAL, ctx->d_models.as<ModelDev>(), model,
                           ctx->d_child.as<int32_t>(),
                                ctx->d_up.as<int32_t>(), ctx->d_rho64.as<double>(), h.d_T.as<double>(),
                                h.d_lc.as<LamConst>(), ctx->lamidx.as<int32_t>() + q0, nq,
                                ctx->view.as<double>(), npix,
                                static_cast<double*>(dimg) + (size_t)q0 * npix * npix,
                                q0 == 0 ? ctx->counter.as<unsigned long long>() : nullptr,
                                ctx->stream));
    }
    if (copy) HIPCHK(hipMemcpyAsync(image, dimg, img_bytes, hipMemcpyDeviceToHost, ctx->stream));
    unsigned long long cr = 0;
    HIPCHK(hipMemcpyAsync(&cr, ctx->counter.p, 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (crossings) *crossings = cr;
    return RT_OK;
  })
}

rt_status rt_render_map_noalloc(rt_ctx* ctx, int32_t model, const double n_obs[3], int32_t npix, double width,
                                int32_t n_sel, const int32_t* lambda_idx, int32_t precision, double* image,
                                uint64_t* crossings) {
  if (!ctx) return fail(nullptr, RT_EINVAL, "null context");
  GUARD({
    if (rt_status s = check_model(ctx, model)) return s;
    if (!n_obs || !lambda_idx || !image) return fail(ctx, RT_EINVAL, "null argument");
    if (npix < 1 || npix > 16384) return fail(ctx, RT_EINVAL, "npix must be in [1, 16384]");
    if (n_sel < 1 || n_sel > kRenderNoAllocMaxSel)
      return fail(ctx, RT_EINVAL, "n_sel must be in [1, %d] (the scratch array holds %d wavelength indices)",
                  kRenderNoAllocMaxSel, kRenderNoAllocMaxSel);
    if (precision != RT_FP64 && precision != RT_FP32_LOCAL)
      return fail(ctx, RT_EINVAL, "precision must be RT_FP64 or RT_FP32_LOCAL");
    HostModel& h = ctx->models[model];
    if (h.nl < 1) return fail(ctx, RT_ESTATE, "rt_set_dust not called for model %d", model);
    if (!h.has_T) return fail(ctx, RT_ESTATE, "model %d has no temperatures", model);
    for (int q = 0; q < n_sel; ++q)
      if (lambda_idx[q] < 0 || lambda_idx[q] >= h.nl) return fail(ctx, RT_EINVAL, "bad wavelength index");
    double v[13];
    if (!render_view(h, n_obs, width, v)) return fail(ctx, RT_EINVAL, "bad view direction or width");
    if (!is_device_ptr(image)) return fail(ctx, RT_EINVAL, "image must be device memory of the context's GPU");
    // uploading changed models would allocate: the device copies must already be current
    if (ctx->tree_dirty || ctx->table_dirty)
      return fail(ctx, RT_ESTATE, "the device copies of the models are out of date: one allocating call "
                                  "(e.g. rt_render_map or rt_trace_packets) is needed after rt_build_tree "
                                  "or rt_set_dust");
    void* scr = render_scratch(ctx->device);
    if (!scr) return fail(ctx, RT_ESTATE, "no scratch array on device %d", ctx->device);
    HIPCHK(hipSetDevice(ctx->device));
    unsigned long long cr = 0;
    HIPCHK(launch_render_noalloc(precision == RT_FP32_LOCAL, ctx->d_models.as<ModelDev>(), model,
                                 ctx->d_child.as<int32_t>(), ctx->d_up.as<int32_t>(), ctx->d_rho64.as<double>(),
                                 h.d_T.as<double>(), h.d_lc.as<LamConst>(), lambda_idx, n_sel, v, npix, image,
                                 scr, crossings ? &cr : nullptr, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (crossings) *crossings = cr;
    return RT_OK;
  })
}

// ---- peel-off (Sect. 2.4) ---------------------------------------------------------------
rt_status rt_peel_map(rt_ctx* ctx, int32_t n_src, const rt_source* src, const rt_trace_opts* o,
                      const rt_peel_opts* po, rt_trace_stats* stats) {
  if (!ctx) return fail(nullptr, RT_EINVAL, "null context");
  GUARD({
    HIPCHK(hipSetDevice(ctx->device));
    if (!po || !o || !src) return fail(ctx, RT_EINVAL, "null argument");
    if (po->n_dir < 1 || po->n_dir > RT_PEEL_MAXDIR) return fail(ctx, RT_EINVAL, "n_dir must be in [1, 16]");
    if (po->npix < 1 || po->npix > 16384) return fail(ctx, RT_EINVAL, "npix must be in [1, 16384]");
    if (po->tiles < 0 || po->tiles > 64) return fail(ctx, RT_EINVAL, "tiles must be in [0, 64]");
    if (po->event_buffer < 0) return fail(ctx, RT_EINVAL, "event_buffer must be >= 0");
    if (!po->n_obs || !po->image) return fail(ctx, RT_EINVAL, "null directions or image");
    if (!std::isfinite(po->width)) return fail(ctx, RT_EINVAL, "bad width");
    if (!(o->precision == RT_FP64 || (o->precision == RT_FP32_LOCAL && o->schedule == RT_SCHED_REGIONS)))
      return fail(ctx, RT_EINVAL, "peel-off needs RT_FP64 or the FP32-local region schedule");
    if (n_src < 1 || n_src > 255) return fail(ctx, RT_EINVAL, "n_src must be in [1, 255]");
    const int32_t model = src[0].model;
    if (rt_status s = check_model(ctx, model)) return s;
    for (int s = 1; s < n_src; ++s)
      if (src[s].model != model) return fail(ctx, RT_EINVAL, "peel-off sources must share one model");
    HostModel& h = ctx->models[model];
    if (h.nl < 1) return fail(ctx, RT_ESTATE, "rt_set_dust not called for model %d", model);
    PeelParams q;
    std::memset(&q, 0, sizeof q);
    q.n_dir = po->n_dir;
    for (int d = 0; d < po->n_dir; ++d) {
      const double* v = po->n_obs + 3 * d;
      const double nn = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
      if (!(nn > 0.0) || !std::isfinite(nn)) return fail(ctx, RT_EINVAL, "bad observer direction %d", d);
      PeelDir& V = q.dir[d];
      for (int a = 0; a < 3; ++a) V.n[a] = v[a] / nn;
      // image frame of the maps: e1 = z x n / |z x n| (x when n is along z), e2 = n x e1
      if (V.n[0] == 0.0 && V.n[1] == 0.0) {
        V.e1[0] = 1.0;
        V.e1[1] = 0.0;
        V.e1[2] = 0.0;
      } else {
        const double en = std::sqrt(V.n[1] * V.n[1] + V.n[0] * V.n[0]);
        V.e1[0] = -V.n[1] / en;
        V.e1[1] = V.n[0] / en;
        V.e1[2] = 0.0;
      }
      V.e2[0] = V.n[1] * V.e1[2] - V.n[2] * V.e1[1];
      V.e2[1] = V.n[2] * V.e1[0] - V.n[0] * V.e1[2];
      V.e2[2] = V.n[0] * V.e1[1] - V.n[1] * V.e1[0];
    }
    q.npix = po->npix;
    q.tiles = po->tiles;
    q.model = model;
    q.W = po->width > 0.0 ? po->width : (double)std::max(h.n[0], std::max(h.n[1], h.n[2]));
    for (int a = 0; a < 3; ++a) q.C[a] = 0.5 * h.n[a];
    const double side = q.W / (double)q.npix * h.cell_cm;
    q.pix_cm2 = side * side;
    if (rt_status s = sync_device(ctx)) return s;
    // refined root cells: table ordinals
    std::vector<int32_t> root_tab(h.n_root, -1), tab_root;
    for (int64_t r = 0; r < h.n_root; ++r)
      if (ctx->h_child[h.base + r] >= 0) {
        root_tab[r] = (int32_t)tab_root.size();
        tab_root.push_back((int32_t)r);
      }
    q.n_tab = (int64_t)tab_root.size();
    if (rt_status e = upload(ctx, ctx->peel_roottab, root_tab)) return e;
    if (rt_status e = upload(ctx, ctx->peel_tabroot, tab_root.empty() ? std::vector<int32_t>(1, 0) : tab_root))
      return e;
    if (rt_status e = upload(ctx, ctx->peel_dnu, h.dnu)) return e;
    q.root_tab = ctx->peel_roottab.as<int32_t>();
    q.tab_root = ctx->peel_tabroot.as<int32_t>();
    q.dnu = ctx->peel_dnu.as<double>();
    const size_t tab_n = (size_t)q.n_dir * q.n_tab * 6 * q.tiles * q.tiles;
    HIPCHK(ctx->peel_tab.ensure(8 * std::max<size_t>(tab_n, 1)));
    q.tab = ctx->peel_tab.as<double>();
    const size_t img_n = (size_t)q.n_dir * h.nl * q.npix * q.npix;
    HIPCHK(ctx->peel_img.ensure(8 * img_n));
    HIPCHK(hipMemsetAsync(ctx->peel_img.p, 0, 8 * img_n, ctx->stream));
    q.image = ctx->peel_img.as<double>();
    q.cap = po->event_buffer > 0 ? (unsigned long long)po->event_buffer : (1ull << 24);
    HIPCHK(ctx->peel_ev.ensure(sizeof(PeelEv) * q.cap));
    HIPCHK(ctx->peel_ctr.ensure(3 * sizeof(unsigned long long)));
    HIPCHK(hipMemsetAsync(ctx->peel_ctr.p, 0, 3 * sizeof(unsigned long long), ctx->stream));
    q.ev = ctx->peel_ev.as<PeelEv>();
    q.count = ctx->peel_ctr.as<unsigned long long>();
    q.lost = q.count + 1;
    q.done = q.count + 2;
    // extinction tables (device, FP64 marches from every tile centre)
    double table_ms = 0.0;
    if (tab_n > 0) {
      TraceParams tp;
      std::memset(&tp, 0, sizeof tp);
      tp.child = ctx->d_child.as<int32_t>();
      tp.up = ctx->d_up.as<int32_t>();
      tp.rho64 = ctx->d_rho64.as<double>();
      tp.models = ctx->d_models.as<ModelDev>();
      HIPCHK(hipEventRecord(ctx->ev0, ctx->stream));
      HIPCHK(launch_peel_tables(tp, q, ctx->stream));
      HIPCHK(hipEventRecord(ctx->ev1, ctx->stream));
      HIPCHK(hipEventSynchronize(ctx->ev1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
      table_ms = ms;
    }
    int64_t tn, tl, tln;
    totals(ctx, &tn, &tl, &tln);
    HIPCHK(ctx->out_esc.ensure(8 * std::max<int64_t>(tl, 1)));
    TraceOut out;
    out.e_esc = ctx->out_esc.as<double>();
    out.peel = &q;
    if (rt_status s = trace_impl(ctx, n_src, src, o, out, stats)) return s;
    unsigned long long ctr[3] = {0, 0, 0};
    HIPCHK(hipMemcpyAsync(ctr, q.count, sizeof ctr, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (ctr[1] > 0)
      return fail(ctx, RT_EDEVICE,
                  "peel-off event buffer too small: %llu events of a batch did not fit in %llu (raise "
                  "event_buffer or lower batch_packets)",
                  (unsigned long long)ctr[1], (unsigned long long)q.cap);
    HIPCHK(hipMemcpyAsync(po->image, q.image, 8 * img_n,
                          is_device_ptr(po->image) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (stats) {
      stats->peel_events = ctr[2];
      stats->table_ms = table_ms;
    }
    return RT_OK;
  })
}

// ---- autotuner ------------------------------------------------------------------------
// Coordinate search over the launch parameters of the requested form: every candidate value of
// one parameter is timed with the others held at the best so far (device time of the whole
// trace, HIP events, best of two runs) on a packet-id prefix of every source; parameters are
// visited in order of their measured influence.  Results are cached per workload signature.

static std::string tune_signature(rt_ctx* ctx, int32_t n_src, const rt_source* src, const rt_trace_opts* o,
                                  double frac) {
  char buf[256];
  std::string s;
  snprintf(buf, sizeof buf, "cu%d p%d s%d f%.6g", ctx->n_cu, o->precision, o->schedule, frac);
  s += buf;
  for (size_t m = 0; m < ctx->models.size(); ++m) {
    const HostModel& h = ctx->models[m];
    snprintf(buf, sizeof buf, " m%lld.%d.%d", (long long)h.n_nodes, h.nlev, h.nl);
    s += buf;
  }
  for (int32_t i = 0; i < n_src; ++i) {
    snprintf(buf, sizeof buf, " s%d.%d.%lld", (int)src[i].kind, src[i].model, (long long)src[i].packets_per_lambda);
    s += buf;
  }
  return s;
}

static bool tune_cache_lookup(const char* path, const std::string& sig, rt_trace_opts* t, double* rate) {
  if (!path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[4096];
  bool found = false;
  while (fgets(line, sizeof line, f)) {
    char* bar = strchr(line, '|');
    if (!bar) continue;
    *bar = 0;
    if (sig != line) continue;
    int bs, bpc, tail, chunk;
    float thr;
    long long batch;
    double rt_;
    if (sscanf(bar + 1, "%d %d %f %d %d %lld %lf", &bs, &bpc, &thr, &tail, &chunk, &batch, &rt_) == 7) {
      t->block_size = bs;
      t->blocks_per_cu = bpc;
      t->refill_threshold = thr;
      t->tail_park = tail;
      t->chunk_packets = chunk;
      t->batch_packets = batch;
      *rate = rt_;
      found = true;  // the last matching line wins
    }
  }
  fclose(f);
  return found;
}

rt_status rt_autotune(rt_ctx* ctx, int32_t n_src, const rt_source* src, const rt_trace_opts* base,
                      double sample_fraction, const char* cache_path, rt_trace_opts* best,
                      double* best_rate) {
  if (!ctx) return fail(nullptr, RT_EINVAL, "null context");
  GUARD({
    if (!base || !best || !src || n_src <= 0) return fail(ctx, RT_EINVAL, "null argument");
    if (!(sample_fraction > 0.0) || sample_fraction > 1.0)
      return fail(ctx, RT_EINVAL, "sample_fraction must be in (0, 1]");
    HIPCHK(hipSetDevice(ctx->device));
    const std::string sig = tune_signature(ctx, n_src, src, base, sample_fraction);
    rt_trace_opts cur = *base;
    cur.rec_stride = 0;
    cur.records = nullptr;
    double rate = 0.0;
    if (tune_cache_lookup(cache_path, sig, &cur, &rate)) {
      cur.rec_stride = base->rec_stride;
      cur.records = base->records;
      *best = cur;
      if (best_rate) *best_rate = rate;
      return RT_OK;
    }
    // packet-id prefix of every source (at least 2^16 packets per wavelength when available)
    std::vector<rt_source> sample(src, src + n_src);
    for (auto& s : sample) {
      const int64_t n = s.packets_per_lambda;
      int64_t k = (int64_t)std::ceil((double)n * sample_fraction);
      k = std::max<int64_t>(k, std::min<int64_t>(n, 65536));
      s.packets_per_lambda = std::max<int64_t>(1, std::min(n, k));
    }
    int64_t tn, tl, tln;
    totals(ctx, &tn, &tl, &tln);
    TraceOut out;
    HIPCHK(ctx->out_node.ensure(8 * std::max<int64_t>(tn, 1)));
    HIPCHK(ctx->out_esc.ensure(8 * std::max<int64_t>(tl, 1)));
    out.e_node = ctx->out_node.as<double>();
    out.e_esc = ctx->out_esc.as<double>();
    auto measure = [&](const rt_trace_opts& t, double* r) -> rt_status {
      double bestv = 0.0;
      for (int rep = 0; rep < 2; ++rep) {
        rt_trace_stats st;
        if (rt_status e = trace_impl(ctx, n_src, sample.data(), &t, out, &st)) return e;
        if (st.kernel_ms > 0.0) bestv = std::max(bestv, (double)st.crossings / (st.kernel_ms * 1e-3));
      }
      *r = bestv;
      return RT_OK;
    };
    // starting point: the library defaults made explicit
    const bool regions = base->precision == RT_FP32_LOCAL && base->schedule == RT_SCHED_REGIONS;
    const bool global32 = base->precision == RT_FP32_LOCAL && !regions;
    if (regions) {
      if (!cur.block_size) cur.block_size = 768;
      if (!cur.blocks_per_cu) cur.blocks_per_cu = 1;
      if (!(cur.refill_threshold > 0.0f)) cur.refill_threshold = 0.6f;
      if (!cur.tail_park) cur.tail_park = 16;
      if (!cur.chunk_packets) cur.chunk_packets = 16 * cur.block_size;
      if (!cur.batch_packets) cur.batch_packets = int64_t(1) << 23;
    } else if (global32) {
      if (!cur.block_size) cur.block_size = 256;
      if (!(cur.refill_threshold > 0.0f)) cur.refill_threshold = 0.5f;
    } else if (!cur.block_size) {
      cur.block_size = 256;
    }
    if (rt_status e = measure(cur, &rate)) return e;
    struct Axis {
      int kind;
      std::vector<double> v;
    };
    std::vector<Axis> axes;
    if (regions) {
      axes = {{0, {512, 768, 1024}},        {2, {0.15, 0.3, 0.4, 0.45, 0.6, 0.75}}, {4, {8, 12, 16, 24, 32}},
              {3, {4, 8, 12, 16, 24, 32, -1}}, {5, {22, 23, 24}}};
    } else if (global32) {
      axes = {{0, {64, 128, 256, 512}}, {2, {0.25, 0.5, 0.75}}, {1, {1, 2, 4}}};
    } else {
      axes = {{0, {64, 128, 256}}};
    }
    for (const Axis& ax : axes) {
      rt_trace_opts keep = cur;
      for (double v : ax.v) {
        rt_trace_opts t = keep;
        switch (ax.kind) {
          case 0: {
            const int old = t.block_size;
            t.block_size = (int)v;
            if (regions) t.chunk_packets = t.chunk_packets / old * t.block_size;
            break;
          }
          case 1: t.blocks_per_cu = (int)v; break;
          case 2: t.refill_threshold = (float)v; break;
          case 3: t.tail_park = (int)v; break;
          case 4: t.chunk_packets = (int)v * t.block_size; break;
          case 5: t.batch_packets = int64_t(1) << (int)v; break;
        }
        if (memcmp(&t, &keep, sizeof t) == 0) continue;
        double rv = 0.0;
        if (rt_status e = measure(t, &rv)) return e;
        if (rv > rate) {
          rate = rv;
          cur = t;
        }
      }
    }
    if (cache_path) {
      if (FILE* f = fopen(cache_path, "a")) {
        fprintf(f, "%s|%d %d %.6g %d %d %lld %.9g\n", sig.c_str(), cur.block_size, cur.blocks_per_cu,
                (double)cur.refill_threshold, cur.tail_park, cur.chunk_packets, (long long)cur.batch_packets, rate);
        fclose(f);
      }
    }
    cur.rec_stride = base->rec_stride;
    cur.records = base->records;
    *best = cur;
    if (best_rate) *best_rate = rate;
    return RT_OK;
  })
}

rt_status rt_philox(rt_ctx* ctx, uint32_t key0, uint32_t key1, int64_t n, const uint32_t* ctr, uint32_t* out) {
  if (!ctx) return fail(nullptr, RT_EINVAL, "null context");
  GUARD({
    if (n < 0) return fail(ctx, RT_EINVAL, "negative count");
    if (n == 0) return RT_OK;
    if (!ctr || !out) return fail(ctx, RT_EINVAL, "null array");
    HIPCHK(hipSetDevice(ctx->device));
    const void* dc;
    if (rt_status s = stage_in(ctx, ctr, 16 * n, ctx->tmp_in, &dc)) return s;
    void* dout;
    bool copy;
    if (rt_status s = stage_out(ctx, out, 16 * n, ctx->tmp_out, &dout, &copy)) return s;
    HIPCHK(launch_philox(key0, key1, n, static_cast<const uint32_t*>(dc), static_cast<uint32_t*>(dout),
                         ctx->stream));
    if (copy) HIPCHK(hipMemcpyAsync(out, dout, 16 * n, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RT_OK;
  })
}

}  // extern "C"
