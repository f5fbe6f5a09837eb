// Internal structures shared by the host runtime and the gfx950 kernels.
//
// Device node layout (all models of a context in one id space):
//   model m occupies internal ids [base, base + n_int), base a multiple of 8;
//   root cells at base + (ix + nx*(iy + ny*iz)); the root level is padded to a multiple of 8,
//   so every oct (8 children) starts at a multiple of 8 and its id >> 3 indexes `up`.
//   canonical id = internal - base                (root level)
//                = internal - base - pad0         (deeper levels), pad0 = n_root_pad - n_root.
// Per internal node:
//   word[i]  int32: a leaf stores the float32 bits of its density (>= +0, so the int is >= 0);
//            a refined cell stores ~first_child (negative): the subgrid identification entry
//            of the paper's Sect. 2.1 packed into the density word (Sect. 3.4 footnote);
//   rho64[i] FP64 density and child[i] first child or -1 (plain FP64 form);
//   up[i>>3] parent id of the oct that starts at i (i a multiple of 8, level >= 1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rt.h"

#define RT_JOBS_LDS 1024   // job starts staged in LDS when at most this many jobs
#define RT_ESC_LDS 1024    // escape tallies staged in LDS when at most this many slots

struct ModelDev {
  int32_t n[3];
  int32_t nlev;
  int32_t base;        // internal id of root cell 0
  int32_t n_root;      // nx*ny*nz
  int32_t n_root_pad;  // n_root rounded up to a multiple of 8
  int32_t n_int;       // internal ids used by this model (including padding)
  double cell_cm;
  int64_t canon_base;      // node-wise output offset
  int64_t lam_base;        // wavelength-wise output offset
  int64_t lamnode_base;    // per-(wavelength, node) output offset
  int64_t leaf_base;       // offset into the leaf tables
  int64_t n_leaves;
  int64_t n_nodes;         // canonical node count
  int32_t nl;
  int32_t pad;
  int64_t level_off[RT_MAX_LEVELS + 2];
};

struct JobDev {
  uint64_t start;      // first global packet index of this job
  uint64_t n;          // packets
  int32_t model, kind, lam, src;
  uint32_t stream;
  int32_t esc_slot;    // wavelength-wise slot for escape tallies
  double w0;           // initial weight (non-dust sources)
  double pos[3];
  double dir[3];
  double kext, alb, g; // FP64 dust constants at this wavelength
  float kc32, alb32, g32;  // FP32: kext * root_cell_cm, albedo, g
  int32_t slot;        // accumulator slot (wavelength, or 0 when wavelengths are summed)
  int64_t acc_off;     // element offset of this job's accumulator slot
  int64_t rec_base;    // first record index (rec_stride > 0)
  int64_t cdf_off;     // dust emission: offset of this (model, wavelength) table
  uint64_t qtot;       // dust emission: total quantised luminosity
};

struct DevStats {
  unsigned long long crossings, scatterings, kills, truncated, packets;
  double e_emit, e_killed, e_rr_gain, e_trunc;
  unsigned long long splits, split_kills, split_skips;
  double e_split_killed, e_split_gain;
  unsigned long long misplaced;  // queue records found outside the region they were queued for
                                 // (an internal invariant; the call fails when it is not 0)
};

// A scattering event kept for the peel-off (Sect. 2.4): position (root-cell units), incoming
// direction and weight before the event roulette, the leaf it is in (internal id, level,
// integer coordinates at that level) and its job.
struct PeelEv {
  double P[3];
  double d[3];
  double w;
  int32_t node;
  int32_t job;
  int32_t I[3];
  int32_t lev;
};

// A package split off in the plain FP64 form (Sect. 2.3), waiting in a queue to be followed from
// the cell where it was split: position, direction, weight and free path, the packet it came
// from, its job, event count and branch identifier (128 bytes).
struct Split64 {
  double P[3], d[3];
  double w, w0, tau;
  int32_t node, lev;
  int32_t I[3];
  uint32_t pid;
  int32_t job;
  uint32_t ev;
  uint32_t br;
  int32_t mlev;  // shallowest level visited by the package it split from (subiterations)
  int32_t pad[4];
};
static_assert(sizeof(Split64) == 128, "split package layout");

struct TraceParams {
  const int32_t* word;
  const double* rho64;
  const int32_t* child;
  const int32_t* up;
  const ModelDev* models;
  const JobDev* jobs;
  int32_t n_jobs;
  int32_t n_esc;
  uint64_t total_packets;
  unsigned long long* counter;
  double* acc64;             // FP64 accumulators [slots][internal ids] (plain and one-queue forms)
  double* esc;
  DevStats* stats;
  rt_record* rec;
  int64_t rec_stride;
  uint32_t key0, key1;
  const uint32_t* keys;      // region pass: the Philox key from device memory when set (a
                             // captured iteration step advances it on the device)
  double rr_thr, rr_p;
  int64_t max_events;
  float refill_thr;
  int32_t split_n;           // package splitting factor at subgrid entry (1: none)
  int32_t split_depth;       // levels past this one belong to the grid of their ancestor at it
                             // (a large value: every oct is a grid)
  // dust emission tables
  const uint64_t* cdf_qpre;
  const uint64_t* cdf_q;
  const double* cdf_lum;
  const int32_t* leaf_node;
  const int32_t* leaf_coord;
  const uint8_t* leaf_level;
  // accelerated Lambda iteration: absorption of dust-emission packets in their birth cell
  // before their first crossing, per canonical node (null when off)
  double* self_acc;
  double* emit_acc;          // energy emitted by dust-emission packets, per birth node
  // subiterations: every deposit also goes to the array of the shallowest level the packet
  // visited, lvl_acc[level * lvl_stride + canonical output index]; sub_lev >= 0 confines the
  // packets to the subtree below the refined cell (sub_lev, sub_I)
  double* lvl_acc;
  int64_t lvl_stride;
  int32_t sub_lev;
  int32_t sub_I[3];
  // automatic iteration (Sect. 3.3): per canonical node, the weight of the packages leaving each
  // refined cell's subtree (the energy flow from a grid to its parent); null when off
  double* flux_acc;
  // peel-off: scattering events of the current batch (null when off)
  PeelEv* peel_ev;
  unsigned long long* peel_count;
  unsigned long long peel_cap;
  // package splitting in the plain FP64 form: packages split off are appended here (a split
  // that does not fit is skipped and counted), and followed by launch_split_fp64
  Split64* sq_out;
  unsigned long long* sq_count;
  unsigned long long sq_cap;
};

#define RT_PEEL_MAXDIR 16

struct PeelDir {
  double n[3], e1[3], e2[3];
};

// Peel-off images and extinction tables of one model (Sect. 2.4).
struct PeelParams {
  PeelDir dir[RT_PEEL_MAXDIR];
  int32_t n_dir, npix, tiles, model;
  double W, C[3], pix_cm2;
  const double* dnu;            // [n_lambda of the model] bandwidths
  const int32_t* root_tab;      // [n_root] ordinal of a refined root cell, -1 for a root leaf
  const int32_t* tab_root;      // [n_tab] root index of each ordinal
  int64_t n_tab;
  double* tab;                  // [n_dir][n_tab][6][tiles^2]
  double* image;                // [n_dir][n_lambda][npix][npix]
  const PeelEv* ev;
  unsigned long long* count;    // events of the batch
  unsigned long long* lost;     // events beyond the buffer, all batches
  unsigned long long* done;     // events peeled, all batches
  unsigned long long cap;
};

// ------------------------------------------------------------------------------------------
// Grid-by-grid (region-blocked) form.  A region is a brick of cells [lo, hi) at one level rl
// (root cells, or children of a cell whose subtree is too large for one region) with all
// their descendants, renumbered region-major: local ids [0, nb_pad) are the brick's cells
// (x fastest), then the octs level by level, each oct 8-aligned.  Region-major global id =
// gbase + local.  rword: leaf -> float bits of the density, refined -> ~(local first child);
// rup[g >> 3]: local parent of the oct starting at g; rcanon[g]: canonical id (-1 = padding).
// ------------------------------------------------------------------------------------------
struct RegionDev {
  int32_t model;
  int32_t rl;       // level of the brick's cells (0: root cells; > 0: children of a split cell)
  int32_t lo[3], hi[3];  // the brick, in level-rl coordinates
  int32_t n;        // local ids used (including padding)
  int32_t pad;
  int64_t gbase;    // region-major global id of local 0 (multiple of 8)
};

// A packet waiting at a region boundary, just born, or re-queued inside its cell: 96 bytes.
struct PRec {
  int32_t I[3];          // integer coordinates of the cell it is in, at level lev
  uint8_t lev, ax, sg, flag;  // flag bit 0 clear: inside the cell (born, re-queued or split
                              // off, no crossing counted on resume); set: about to cross axis
                              // ax (sg 0: +, 1: -).  Bit 1: a split-off branch, `birth` holds
                              // its branch identifier
  float x[3], d[3];      // local coordinates in that cell, direction
  float w, w0, tau;
  int32_t birth;         // internal id of the birth leaf (records), or the branch id
  double O[3];           // FP64 segment origin (root-cell units)
  uint32_t pid;
  int32_t job;
  uint32_t ev, ncross;
};
static_assert(sizeof(PRec) == 96, "packet record layout");

struct WorkItem {
  int32_t region, slot;
  uint32_t start, count;
};

struct SweepState;

struct BlkParams {
  TraceParams t;
  const RegionDev* regions;
  int32_t n_regions;
  int32_t cap;               // node capacity of the LDS copy of a region
  const int32_t* rword;
  const int32_t* rup;
  const int32_t* rcanon;     // region-major id -> canonical id within its model (-1 = padding)
  const int32_t* root_region;  // per internal id of a root cell (old layout): its region, or
                               // ~s when the cell is split (split_tab entry s)
  const int32_t* split_tab;    // 8 per split cell, by child octant: region id, or ~s (split again)
  double* accb64;            // [slots][G] region-major FP64 accumulators: one slot (wavelength-
                             // integrated output), one per wavelength (per-wavelength output) or
                             // one per level (lvl_slots > 0); a key's slot selects the array
  int64_t accb_stride;       // G
  // queues
  PRec* u_out;               // append target
  uint32_t* u_key;           // its sort keys (slot * n_regions + region)
  unsigned long long* u_count;
  const PRec* q_in;          // records of this sweep, read through q_perm
  const uint32_t* q_perm;
  const WorkItem* items;
  const uint32_t* n_items;
  uint32_t* item_counter;
  const SweepState* sweep;   // this sweep's emission range [e0, e0 + ne)
  uint32_t* emit_counter;    // chunks of births taken
  int32_t n_slots_key;       // accumulator slots (wavelengths, or levels) in the key
  int32_t lvl_slots;         // > 0: subiterations; the slots are the shallowest level visited
                             // (levels 0..lvl_slots-1), accumulated in FP64 (accb64)
  int32_t chunk;             // packets per work item
  int32_t tail_park;         // crossing rounds after an item's queue runs dry before the
                             // packets still in flight are re-queued (INT32_MAX = never)
  const unsigned long long* split_room;  // queue room for split-off packages in this sweep
  unsigned long long* split_used;        // records reserved for them so far
};

// Device-resident state of the sweeps of one trace (all sizes the sweep launches need).
// Queue records: each wave of the region pass takes kExitChunk records of the next queue at a
// time for the packets leaving its regions; the part of its last chunk it does not fill keeps
// kInvalidKey and is skipped by the sort.
constexpr uint32_t kExitChunk = 128;
constexpr uint32_t kInvalidKey = 0xFFFFFFFFu;

struct SweepState {
  unsigned long long count[2];  // records appended to queue buffer 0 / 1
  unsigned long long emitted;   // packets emitted so far (global packet index)
  unsigned long long total;     // packets to emit
  unsigned long long e0, ne;    // this sweep's emission range [e0, e0 + ne)
  unsigned long long n_in;      // records in this sweep's input buffer
  uint32_t n_items, item_counter;
  uint32_t done;                // a sweep found nothing queued and nothing left to emit
  uint32_t emit_counter;        // chunks of births taken by the pass kernel's blocks
  uint32_t sweeps;              // sweeps that had packets to follow
  unsigned long long split_room;  // queue room for split-off packages in this sweep
  unsigned long long split_used;  // records reserved for them so far
  unsigned long long cap_all;     // allocated records per queue buffer
  unsigned long long log_in[16];  // records in the input of each sweep of the current block
};

// Is the cell (lev, I) inside the subtree below the refined cell (sub_lev, sub_I)?
__host__ __device__ inline bool in_subtree(int sub_lev, const int32_t sub_I[3], int lev, int32_t I0, int32_t I1,
                                           int32_t I2) {
  if (lev <= sub_lev) return false;
  const int sh = lev - sub_lev;
  return (I0 >> sh) == sub_I[0] && (I1 >> sh) == sub_I[1] && (I2 >> sh) == sub_I[2];
}

hipError_t launch_ali_absorbed(int64_t n, const double* a_stars, const double* a_dust, const double* e_self,
                               const double* e_emit, double* out, hipStream_t s);
hipError_t launch_peel_tables(const TraceParams& p, const PeelParams& q, hipStream_t s);
hipError_t launch_peel(const TraceParams& p, const PeelParams& q, int grid, hipStream_t s);
// Sort of one sweep's queue by key.  With at most kSortLdsKeys keys the counts are kept per
// block (bhist: kSortBlocks(grid) x n_keys) and no global atomic is used; otherwise hist and the
// cursors are counted with global atomics.
constexpr int kSortLdsKeys = 16384;
inline int kSortBlocks(int grid) { return grid / 4 > 0 ? grid / 4 : 1; }
hipError_t launch_sweep_sort(SweepState* st, int in, int slot, uint64_t batch, uint64_t capq, const uint32_t* keys,
                             int n_keys, int n_regions, int chunk, uint32_t* hist, uint32_t* kfill,
                             uint32_t* bhist, uint32_t* perm, WorkItem* items, int grid, hipStream_t s);
hipError_t launch_blk_pass(const BlkParams& b, int grid, int block, int lds_bytes, hipStream_t s);
hipError_t attr_blk_pass(int block, int lds_bytes);
hipError_t launch_blk_reduce(const ModelDev* models, const RegionDev* regions, int n_regions,
                             int32_t max_region_nodes, const int32_t* rcanon, const double* accb64,
                             int64_t stride, int n_slots, double* e_node, double* e_lam_node,
                             double* lvl_out, int64_t lvl_stride, double* e_total, hipStream_t s);

// Launch wrappers (defined in the .hip files)
hipError_t launch_trace_fp64(const TraceParams& p, int job, uint64_t n, int block, hipStream_t s);
// Follows the n packages in `in` (split off in the plain FP64 form); packages they split off in
// turn go to p.sq_out.
hipError_t launch_split_fp64(const TraceParams& p, const Split64* in, uint64_t n, int block, hipStream_t s);
hipError_t launch_trace_fp32(const TraceParams& p, int grid, int block, hipStream_t s);
hipError_t occupancy_trace_fp32(int block, int* blocks_per_cu);
hipError_t launch_reduce_model(const ModelDev* models_dev, int model, int64_t n_nodes,
                               const double* acc64, int64_t slot_stride,
                               int n_slots, double* e_node, double* e_lam_node, double* e_total,
                               hipStream_t s);
hipError_t launch_locate(const int32_t* child, const ModelDev* models, int model, int64_t n,
                         const double* xyz, int32_t* lev, int64_t* node, hipStream_t s);
hipError_t launch_philox(uint32_t k0, uint32_t k1, int64_t n, const uint32_t* ctr, uint32_t* out,
                         hipStream_t s);
hipError_t launch_add(int64_t n, const double* a, const double* b, double* out, hipStream_t s);
hipError_t launch_crit(const ModelDev* models, int model, int64_t n_nodes, const int32_t* child,
                       const double* rho64, const double* t_new, const double* t_old, double* out,
                       hipStream_t s);

// Planck constants of one wavelength for the temperature solve, dust emission and maps.
struct LamConst {
  double kext, alb;
  double kabs_dnu;   // (1 - albedo) * kappa_ext * dnu
  double pre;        // 2 h nu^3 / c^2
  double hnu;        // h nu
  double dnu;
};
// Temperatures of every leaf (tab: scratch of 4 + 2 kPlanckTable doubles for the inverse table
// of the emission per unit mass, rebuilt by each call; dense enough that its cubic Hermite
// interpolation is the root to rounding).
constexpr int kPlanckTable = 65536;
hipError_t launch_temperature(const ModelDev* models, int model, int64_t n_nodes,
                              const int32_t* child, const double* rho64, const double* a_node,
                              const LamConst* lc, int nl, double t_min, double t_max, double* tab,
                              double* t_out, hipStream_t s);
hipError_t launch_dust_lum(const ModelDev* models, int model, int64_t n_leaves,
                           const int32_t* leaf_node, const uint8_t* leaf_level,
                           const double* rho64, const double* t_node, const LamConst* lc, int lam,
                           double* lum, unsigned long long* lmax_bits, const int32_t* leaf_coord,
                           int sub_lev, const int32_t sub_I[3], hipStream_t s);
hipError_t launch_subiter_update(const ModelDev* models, int model, int64_t n_leaves, const int32_t* leaf_node,
                                 const uint8_t* leaf_level, const int32_t* leaf_coord, const double* rho64,
                                 const LamConst* lc, int nl, int sub_lev, const int32_t sub_I[3], int lo,
                                 const double* lvl_new, int64_t lvl_stride, double* arrays, const double* a_stars,
                                 const double* t_old, double* a_tot, double* imb, hipStream_t s);
hipError_t launch_dust_quant(int64_t n_leaves, const double* lum,
                             const unsigned long long* lmax_bits, uint64_t* q, hipStream_t s);
// Wavelengths per pass of the map kernel (registers per ray): FP64 and FP32 transfer.
constexpr int kRenderPassF64 = 16;
constexpr int kRenderPassF32 = 128;
hipError_t launch_render(bool f32, const ModelDev* models, int model, const int32_t* child,
                         const int32_t* up, const double* rho64, const double* t_node,
                         const LamConst* lc, const int32_t* lam_idx, int n_sel,
                         const double* view /* n, e1, e2, centre, W */, int npix,
                         double* image, unsigned long long* crossings, hipStream_t s);

// Allocation-free maps (render.hip): wavelengths per call, the per-device scratch array's
// location (found once per device when a context is created) and the launch.
constexpr int kRenderNoAllocMaxSel = 512;
hipError_t render_scratch_init(int device);
void* render_scratch(int device);
hipError_t launch_render_noalloc(bool f32, const ModelDev* models, int model, const int32_t* child,
                                 const int32_t* up, const double* rho64, const double* t_node,
                                 const LamConst* lc, const int32_t* lam_idx_host, int n_sel,
                                 const double* view_host, int npix, double* image, void* scr,
                                 unsigned long long* crossings_host, hipStream_t s);

// A captured iteration step (Lambda iteration in the region schedule): device-only pieces.
hipError_t launch_dust_scan(int64_t n, const uint64_t* q, uint64_t* qpre, uint64_t* tile_tmp, uint64_t* total_out,
                            hipStream_t s);
int64_t dust_scan_tiles(int64_t n);
hipError_t launch_fill_u64(void* a, int64_t n_words, unsigned long long v, hipStream_t s);
hipError_t launch_copy_u64(const void* a, void* b, int64_t n_words, hipStream_t s);
hipError_t launch_step_key(uint32_t* keys, hipStream_t s);
hipError_t launch_step_report(const double* crit, const SweepState* st, const DevStats* stats, double* out,
                              hipStream_t s);
hipError_t launch_sweep_init(SweepState* st, uint64_t total, uint64_t cap_all, hipStream_t s);
