/* rt.h — C ABI of the MI355X (gfx950) Monte Carlo continuum radiative-transfer library for
 * hierarchical (oct-tree) grids.
 *
 * The operations follow Lunttila & Juvela, "Radiative transfer on hierarchial grids":
 *   rt_build_tree         the nested-grid hierarchy of Sect. 2.1 (refinement ratio one half);
 *   rt_set_dust           the single-component dust model of Sect. 4 (opacity, albedo, and a
 *                         Henyey-Greenstein asymmetry parameter for the phase function);
 *   rt_trace_packets      the Monte Carlo formal solution of Sect. 2.3 (internal sources and the
 *                         external field, continuous absorption, Russian roulette);
 *   rt_solve_temperature  the dust model f(J) of Sect. 3.1 Eq. (1)-(2): equilibrium temperature
 *                         of one grain component (Sect. 4);
 *   rt_lambda_iterate     the Lambda iteration of Sect. 3.1 Eq. (2) with the constant-source
 *                         field kept (Sect. 3.2);
 *   rt_ali_iterate        the same with the accelerated iteration (Sect. 3.1 Eq. 3);
 *   rt_subiter_*          subiterations on complete subtrees (Sect. 3.1, 3.3, App. B);
 *   rt_render_map         surface-brightness maps toward chosen directions (Sect. 4.1);
 *   rt_peel_map           images of the scattered light by peel-off, with precomputed
 *                         extinction tables (Sect. 2.4).
 *
 * Conventions
 *   - Every call validates all of its arguments before it changes any state; on error it
 *     returns a negative status, leaves the context unchanged and records a message that
 *     rt_last_error() returns.  No C++ exception crosses this interface.
 *   - Array arguments marked "host or device" may point to host memory or to device memory of
 *     the context's GPU (for example torch tensors); the library classifies them itself.
 *     Device outputs are written in order on the context's stream; calls return after the
 *     stream has completed the work unless stated otherwise.
 *   - The context owns every device buffer it allocates; the caller owns all arrays it passes.
 *   - One context per host thread.
 */
#ifndef RT_H
#define RT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rt_status;
#define RT_OK 0
#define RT_EINVAL (-1)   /* invalid argument */
#define RT_ENOMEM (-2)   /* device or host allocation failed */
#define RT_EDEVICE (-3)  /* HIP runtime error, or no usable gfx950 device */
#define RT_ESTATE (-4)   /* call out of order (e.g. tracing before rt_set_dust) */

#define RT_MAX_LEVELS 24

typedef struct rt_ctx rt_ctx;

/* Message describing the last failing call on ctx ("" if none).  Valid until the next call. */
const char* rt_last_error(const rt_ctx* ctx);

/* Create a context on HIP device `device`, issuing work on `hip_stream` (a hipStream_t; NULL =
 * the null stream).  Fails with RT_EDEVICE if the device is absent or not gfx950. */
rt_status rt_create(rt_ctx** out, int32_t device, void* hip_stream);
rt_status rt_destroy(rt_ctx* ctx);

/* ---------------------------------------------------------------------------------------- */
/* Tree (Sect. 2.1).  Root grid of nx*ny*nz cells (x fastest); each refined cell is replaced by
 * one oct of 8 cells of half its size.  Canonical order: level-0 index ix + nx*(iy + ny*iz);
 * the octs of level l+1 follow the ascending level-l index of their parent, and cell
 * b = bx + 2by + 4bz of oct o has level index 8o + b; node id = level offset + level index.
 * Host arrays are read during the call only.                                                */
typedef struct {
  int32_t nx, ny, nz;            /* root cells per axis, >= 1 */
  double root_cell_cm;           /* physical edge of a root cell (cm), > 0 */
  int32_t n_levels;              /* refinement levels below the root, 0..RT_MAX_LEVELS */
  const double* root_rho;        /* [nx*ny*nz] density (g cm^-3), finite, >= 0 */
  const int64_t* n_refined;      /* [n_levels] number of refined cells at level l */
  const int64_t* const* refined; /* [n_levels][n_refined[l]] strictly ascending level-l indices */
  const double* const* child_rho;/* [n_levels][8*n_refined[l]] densities of level l+1 cells */
} rt_tree_desc;

/* Validates and uploads a tree; returns its model id and canonical node count.  Several
 * models may live in one context (they are traced together by rt_trace_packets). */
rt_status rt_build_tree(rt_ctx* ctx, const rt_tree_desc* desc, int32_t* model_out,
                        int64_t* n_nodes_out);

typedef struct {
  int64_t n_nodes, n_leaves;
  int32_t n_levels, n_lambda;
  int64_t level_offset[RT_MAX_LEVELS + 2]; /* canonical node offset of each level */
  int64_t node_base;        /* offset of this model in node-wise outputs (all models) */
  int64_t lambda_base;      /* offset of this model in wavelength-wise outputs */
  int64_t lambda_node_base; /* offset of this model in per-(wavelength, node) outputs */
} rt_model_info;
rt_status rt_get_model_info(rt_ctx* ctx, int32_t model, rt_model_info* out);

/* Totals over all models of the context: node-wise, wavelength-wise and per-(wavelength,
 * node) output lengths. */
rt_status rt_get_sizes(rt_ctx* ctx, int64_t* nodes, int64_t* lambdas, int64_t* lambda_nodes);

/* Point location with half-open cells [lo, hi): xyz [n][3] in root-cell units (host or
 * device); outputs level and canonical node (host or device), -1 for points outside the root
 * grid or NaN.  Bit-exact: no rounding is involved. */
rt_status rt_locate(rt_ctx* ctx, int32_t model, int64_t n, const double* xyz, int32_t* level_out,
                    int64_t* node_out);

/* ---------------------------------------------------------------------------------------- */
/* Dust (Sect. 4): per wavelength (strictly ascending, um) the extinction opacity (cm^2 g^-1,
 * > 0), albedo in [0, 1] and Henyey-Greenstein g in (-1, 1).  Frequency bandwidths are the
 * trapezoid weights in nu of this grid (a single wavelength has bandwidth 1).  Host arrays. */
rt_status rt_set_dust(rt_ctx* ctx, int32_t model, int32_t n_lambda, const double* lambda_um,
                      const double* kappa_ext, const double* albedo, const double* hg_g);

/* Per-leaf temperatures used by dust-emission sources and maps: canonical [n_nodes] (host or
 * device, values of refined nodes ignored).  rt_solve_temperature also sets them. */
rt_status rt_set_temperature(rt_ctx* ctx, int32_t model, const double* t_node);

/* ---------------------------------------------------------------------------------------- */
/* Sources (Sect. 2.3) */
#define RT_SRC_BACKGROUND 0 /* isotropic field I_nu outside the root box (power: I_nu, per sr) */
#define RT_SRC_POINT 1      /* isotropic point source L_nu at pos (power: L_nu, erg/s/Hz) */
#define RT_SRC_DUST 2       /* thermal dust emission of the model's current temperatures */
#define RT_SRC_BEAM 3       /* pencil beam from pos along dir (power: L_nu); test source */

typedef struct {
  int32_t kind;
  int32_t model;
  double pos[3];                /* POINT, BEAM: root-cell units, inside the root grid */
  double dir[3];                /* BEAM: direction (normalised by the library) */
  const double* power;          /* host [n_lambda of the model]; NULL for DUST */
  int64_t packets_per_lambda;   /* 1 .. 2^32 */
} rt_source;

#define RT_FP64 0        /* plain form: one packet per lane, global FP64 coordinates */
#define RT_FP32_LOCAL 1  /* packet queues, FP32 per-cell local coordinates */

#define RT_SCHED_REGIONS 0 /* grid by grid (paper Sect. 3.4, App. A) on LDS-sized regions */
#define RT_SCHED_GLOBAL 1  /* one persistent packet-queue kernel over the whole tree */

/* Per-packet end state, written for sampled packets (see rt_trace_opts.rec_stride). */
typedef struct {
  uint32_t status;     /* 0 escaped, 1 killed by roulette, 2 truncated at max_events,
                          3 killed by the roulette at a subgrid exit (package splitting) */
  uint32_t crossings;  /* leaf cells entered, including the birth cell */
  uint32_t events;     /* scattering events reached */
  uint32_t pad;
  int64_t node;        /* canonical node where it ended (-1 escaped) */
  int64_t birth;       /* canonical node where it started */
  double w;            /* weight at the end (escaped, killed or truncated energy) */
} rt_record;

typedef struct {
  uint64_t seed;            /* Philox key = (lo32(seed), hi32(seed) + iteration) */
  uint32_t iteration;
  int32_t precision;        /* RT_FP64 or RT_FP32_LOCAL */
  double rr_threshold;      /* roulette when w < rr_threshold * w0 (relative); 0 = off */
  double rr_prob;           /* kill probability p; survivors scaled by 1/(1-p) */
  int64_t max_events;       /* per-packet scattering cap; 0 = 1e6 */
  int32_t block_size;       /* threads per block; 0 = default.  FP64: 64, 128, 256 (default
                               256); FP32-local one queue: 64-512 (256); FP32-local regions:
                               256, 512, 768, 1024 (768) */
  int32_t blocks_per_cu;    /* persistent form: resident blocks per CU; 0 = default */
  float refill_threshold;   /* FP32-local form: service events/refills when fewer than this
                               fraction of live lanes are crossing; 0 = default */
  int32_t schedule;         /* FP32-local form: RT_SCHED_REGIONS (default) processes the tree
                               region by region with LDS-resident nodes and accumulators;
                               RT_SCHED_GLOBAL runs one persistent kernel over the whole tree
                               with global atomics */
  int32_t chunk_packets;    /* region schedule: packets per work item; 0 = 16 * block_size */
  int32_t tail_park;        /* region schedule: crossing rounds a wave keeps following its last
                               packets after its work item's queue is empty before it re-queues
                               them for the next sweep; 0 = default (16), < 0 = never */
  int64_t batch_packets;    /* region schedule: packets emitted per sweep; 0 = 2^23 */
  int64_t rec_stride;       /* > 0: record packet j of each (source, wavelength) when
                               j % rec_stride == 0 */
  rt_record* records;       /* host or device; job-major: job (source-major, then wavelength)
                               base = sum over earlier jobs of ceil(N/rec_stride) */
  int32_t sweep_graph;      /* region schedule: > 0 replays a captured HIP graph of 16 sweeps
                               until the queues drain (per-pass durations are then not
                               reported); <= 0 (default) launches the same kernels directly */
  int32_t split_n;          /* package splitting (paper Sect. 2.3), in the RT_FP64 form and the
                               region schedule (RT_EINVAL in the one-queue FP32 form): at a
                               face crossing into a deeper leaf the package
                               becomes split_n packages of 1/split_n its weight (the new ones
                               draw their own free path); at a crossing into a shallower leaf
                               it survives with probability 1/split_n and its weight is
                               multiplied by split_n.  0 or 1 = off, at most 64.  Records
                               (rec_stride) follow the package as emitted (branch 0).  A split
                               that would overrun the sweep's queue room (the FP64 form's queue
                               of split-off packages, up to 2^22) is skipped (counted in
                               split_skips); either choice leaves every expectation unchanged */
  int32_t split_depth;      /* with split_n > 1, what a "grid" is (Sect. 2.3): 0 (default) every
                               oct, so every change of level splits or roulettes; d > 0 all
                               levels below d belong to the grid of their level-d ancestor (d = 1:
                               the root grid and one grid per refined root cell), and only a
                               change of min(level, d) splits or roulettes.  Must be >= 0 */
} rt_trace_opts;

typedef struct {
  uint64_t crossings, scatterings, kills, truncated, packets;
  double e_emit, e_abs, e_esc, e_killed, e_rr_gain, e_trunc;
  double kernel_ms;         /* device time from the first transport launch to the last (HIP
                               events on the context stream), emission and queue sorting
                               included */
  double reduce_ms;         /* device time of the final FP64 reduction */
  double main_ms;           /* summed durations of the launches of the dominant transport
                               kernel (FP64: the per-job kernel; FP32-local: the persistent
                               kernel, or the region pass of every sweep, which also writes
                               the sweep's new packets), HIP events recorded on the stream
                               each launch runs on */
  uint64_t main_launches;   /* number of those launches */
  uint64_t splits;          /* crossings at which a package was split */
  uint64_t split_kills;     /* packages ended by the roulette at a subgrid exit */
  uint64_t split_skips;     /* splits skipped for lack of queue room */
  double e_split_killed;    /* weight of those packages */
  double e_split_gain;      /* weight added to the survivors of that roulette; energy balance:
                               e_emit + e_rr_gain + e_split_gain = e_abs + e_esc + e_killed +
                               e_trunc + e_split_killed */
  uint64_t peel_events;     /* rt_peel_map: scattering events peeled off */
  double table_ms;          /* rt_peel_map: device time of the extinction-table build */
} rt_trace_stats;

/* Follow packets_per_lambda packets of every source at every wavelength of its model.  Packet
 * j of (source s, wavelength i, model m) uses Philox stream (m << 20 | s << 12 | i).
 * Outputs (host or device; NULL to skip):
 *   e_abs_node         [total nodes] absorbed power per canonical node, all wavelengths;
 *   e_abs_lambda_node  [total lambda_nodes] per (wavelength, node), model-major;
 *   e_esc_lambda       [total lambdas] escaped power per wavelength.
 * Deposits are accumulated in FP64 in both precisions (the region schedule first sums each work
 * item's deposits in FP32 in LDS), then reduced to canonical order in a final pass.  A broken
 * internal invariant of the region schedule (a queued packet record outside the region it was
 * queued for) fails the call with RT_EDEVICE after the trace, naming the count. */
rt_status rt_trace_packets(rt_ctx* ctx, int32_t n_src, const rt_source* src,
                           const rt_trace_opts* opts, double* e_abs_node,
                           double* e_abs_lambda_node, double* e_esc_lambda,
                           rt_trace_stats* stats);

/* Equilibrium temperature per leaf (FP64): 4 pi m sum_i kappa_abs_i B_i(T) dnu_i = A, with A
 * the absorbed power per canonical node of the model (host or device).  a_node = NULL takes
 * the model's part of the e_abs_node result of the last rt_trace_packets call on this context
 * (RT_ESTATE if there is none, or if models were added since).  A at or below the emission at
 * t_min gives t_min, at or above the emission at t_max gives t_max; refined nodes get 0.
 * Stores the result as the model's temperatures; t_node (host or device) may be NULL. */
rt_status rt_solve_temperature(rt_ctx* ctx, int32_t model, const double* a_node, double t_min,
                               double t_max, double* t_node);

/* Lambda iteration (Sect. 3.1 Eq. 2, constant sources kept per Sect. 3.2): trace the constant
 * sources once (key iteration 0) -> A_stars, T_0 = f(A_stars); for n >= 1 trace the dust
 * emission of T_{n-1} (key iteration n, dust_packets per wavelength) -> A_dust,
 * T_n = f(A_stars + A_dust); stop when the mass-weighted mean of |T_n - T_{n-1}| / T_{n-1} is
 * below tol or after n_max steps.  crit [n_max] (host, may be NULL) receives the statistic of
 * each step; t_node (host or device, may be NULL) the final temperatures. */
rt_status rt_lambda_iterate(rt_ctx* ctx, int32_t model, int32_t n_src, const rt_source* src,
                            const rt_trace_opts* opts, int64_t dust_packets, int32_t n_max,
                            double tol, double t_min, double t_max, double* t_node,
                            int32_t* n_done, double* crit);

/* Accelerated Lambda iteration with a diagonal operator (Sect. 3.1, Eq. 3), otherwise as
 * rt_lambda_iterate (same arguments, stopping rule and outputs).  Each dust-emission trace also
 * tallies, per cell, the energy its own packets deposit in it before they first leave it
 * (A_self) and the energy they start with (E_emit); lambda* = A_self / E_emit is the diagonal
 * operator, and T_n balances E(T_n) (1 - lambda*) = A_stars + A_dust - A_self, which has the
 * Lambda iteration's fixed point and converges faster where cells are optically thick.
 * RT_FP64, or RT_FP32_LOCAL with the region schedule. */
rt_status rt_ali_iterate(rt_ctx* ctx, int32_t model, int32_t n_src, const rt_source* src,
                         const rt_trace_opts* opts, int64_t dust_packets, int32_t n_max, double tol,
                         double t_min, double t_max, double* t_node, int32_t* n_done, double* crit);

/* Subiterations on complete subtrees (Sect. 3.1, Sect. 3.3, App. B), in the RT_FP64 form or the
 * RT_FP32_LOCAL region schedule (RT_EINVAL in the one-queue FP32 form), with or without package
 * splitting (a split-off package inherits the shallowest level visited of the package it split
 * from).
 * rt_subiter_begin traces the constant sources (key iteration opts->iteration) into A_stars,
 * solves T_0 and clears the model's per-level arrays (one absorbed-energy array per hierarchy
 * level at or above each cell's own).  flux_frac > 0 turns on the tracking of the energy flow
 * from each grid to its parent (Sect. 3.3): every step then also measures, per refined node,
 * the weight of the packages leaving its subtree; when a step below root r changes the flow out
 * of r's subtree by more than flux_frac times the energy absorbed in the subtree of r's parent
 * (the whole model for a root cell) since that parent last took part in a step, the parent is
 * tagged, and rt_subiter_select includes every tagged grid until a step includes it.
 * flux_frac = 0: no tracking.  ali != 0: every step uses the accelerated iteration with the
 * diagonal operator (Sect. 3.1 Eq. 3) inside its subtree: each subtree leaf's temperature balances (A - e_self) / (1 - lambda*), with A = A_stars
 * plus the leaf's arrays (Eq. 9) and e_self, lambda* = e_self / e_emit from the step's own
 * trace as in rt_ali_iterate; the recorded imbalances and the flows use A itself.
 * rt_subiter_step takes one step with the subtree below `root`, a refined canonical node of
 * the model, or the whole model (root = -1): the dust emission of the subtree's leaves at the
 * current temperatures is traced with key `iteration`; every deposit is filed under the
 * shallowest level its package has visited (0 for the external field), and a package leaving
 * the subtree is ended there.  The arrays of levels below the root's of the subtree's leaves
 * are replaced by the new deposits, each subtree leaf's energy imbalance |A - E(T_old)| /
 * E(T_old) is recorded, and the temperatures follow from A_stars plus the sum of each leaf's
 * arrays (Eq. 9).  crit (may be NULL): mass-weighted mean |T_new - T_old| / T_old over all
 * leaves; t_node (host or device, may be NULL): the temperatures after the step.
 * rt_subiter_select picks the next subtree (Sect. 3.3): the lowest common ancestor of every
 * leaf whose last recorded imbalance is within frac of the largest and of every tagged grid;
 * root = -1 when that is the whole model.  max_imbalance (may be NULL) receives the largest. */
rt_status rt_subiter_begin(rt_ctx* ctx, int32_t model, int32_t n_src, const rt_source* src,
                           const rt_trace_opts* opts, double t_min, double t_max, double flux_frac,
                           int32_t ali);
rt_status rt_subiter_step(rt_ctx* ctx, int32_t model, int64_t root, int64_t dust_packets,
                          uint32_t iteration, const rt_trace_opts* opts, double* crit,
                          double* t_node, rt_trace_stats* stats);
rt_status rt_subiter_select(rt_ctx* ctx, int32_t model, double frac, int64_t* root,
                            double* max_imbalance);
/* Automatic iteration (Sect. 3.3): n_steps steps after rt_subiter_begin, the first on the whole
 * model, each later one on the subtree rt_subiter_select(frac) picks; when it picks the subtree
 * of the step before and the largest imbalance has not dropped below stall times its previous
 * value (the Monte Carlo noise limit of that subtree), the step takes the whole model instead.
 * Key iterations first_iteration, first_iteration + 1, ...  roots, crit, crossings [n_steps]
 * (host, may be NULL): the subtree root, the stopping statistic and the cell crossings of each
 * step; t_node (host or device, may be NULL): the temperatures after the last step. */
rt_status rt_subiter_run(rt_ctx* ctx, int32_t model, int32_t n_steps, double frac, double stall,
                         int64_t dust_packets, uint32_t first_iteration, const rt_trace_opts* opts,
                         int64_t* roots, double* crit, uint64_t* crossings, double* t_node);

/* Surface-brightness map (Sect. 4.1) of a model with its current temperatures: orthographic
 * view toward the observer direction n_obs; pixel (i, j) centre = box centre +
 * ((i+0.5)/npix - 0.5) W e1 + ((j+0.5)/npix - 0.5) W e2 with e1 = z x n / |z x n| (x if n is
 * along z), e2 = n x e1, W = width (<= 0: largest root extent).  Along each ray
 * I <- I exp(-dtau) + (1 - a) B(T) (1 - exp(-dtau)).  image [n_sel][npix][npix] (host or
 * device) in erg s^-1 cm^-2 Hz^-1 sr^-1; crossings (may be NULL) counts leaf entries.
 * precision: RT_FP64, or RT_FP32_LOCAL (the same FP64 ray geometry, hence the same cells;
 * the transfer per wavelength evaluated in FP32). */
rt_status rt_render_map(rt_ctx* ctx, int32_t model, const double n_obs[3], int32_t npix,
                        double width, int32_t n_sel, const int32_t* lambda_idx,
                        int32_t precision, double* image, uint64_t* crossings);

/* Allocation-free variant of rt_render_map, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same map,
 * same kernels and arguments, except: image must be device memory of the context's GPU;
 * lambda_idx is a host array of at most 512 entries (RT_EINVAL beyond: the per-call staging
 * lives in a fixed 2.3 KB device array, not in context buffers); crossings (host, may be NULL).
 * The call allocates nothing (no hipMalloc, hipFree or allocating library routine): the view
 * frame, the wavelength list and the crossing counter are written into a file-scope device
 * array, located on each device once when a context is created there, and cleared by every
 * call.  Every call on one GPU shares that array, so calls that overlap on one GPU (several
 * contexts or threads on one device) race and must be serialised by the caller.  The
 * context's device copies of the models must be current (RT_ESTATE otherwise): after
 * rt_build_tree or rt_set_dust, one allocating call such as rt_render_map or
 * rt_trace_packets uploads them. */
rt_status rt_render_map_noalloc(rt_ctx* ctx, int32_t model, const double n_obs[3], int32_t npix,
                                double width, int32_t n_sel, const int32_t* lambda_idx,
                                int32_t precision, double* image, uint64_t* crossings);

/* Peel-off images of the scattered light (Sect. 2.4).  The sources (all of one model) are
 * traced as by rt_trace_packets with the same options (RT_FP64, or RT_FP32_LOCAL with the
 * region schedule); at every scattering event, before the event roulette, the part of the
 * packet scattered toward each observer direction n and escaping, w Phi_HG(d.n) exp(-tau),
 * is added to the pixel the event position projects onto (the map geometry of
 * rt_render_map), divided by the wavelength's bandwidth and the pixel area: the image is the
 * scattered surface brightness in erg s^-1 cm^-2 Hz^-1 sr^-1.  tau = kappa_ext times the
 * column density from the event to the model border along n:
 *   tiles = 0  marched cell by cell to the border;
 *   tiles > 0  extinction tables on the six faces of every refined root cell, tiles x tiles
 *              per face, each entry the column from the tile centre to the border: a ray from
 *              inside a refined root cell is marched to that cell's boundary, a ray from a root
 *              leaf through root leaves until it enters a refined root cell or leaves the
 *              model, and the table entry of the tile it crosses completes the column (the
 *              paper's accelerated peel-off; an approximation of the order of a tile).
 * Events are kept per batch (a sweep of the region schedule, a (source, wavelength) job of the
 * FP64 form) in a device buffer of event_buffer entries (80 B each); a batch with more events
 * than that fails the call with RT_EDEVICE, naming the count, after the trace (lower
 * batch_packets or raise event_buffer).  The absorbed energy is not returned. */
typedef struct {
  int32_t n_dir;            /* observer directions, 1..16 */
  int32_t npix;             /* pixels per image side, 1..16384 */
  const double* n_obs;      /* [n_dir][3] host: direction toward each observer, any length > 0 */
  double width;             /* image side in root-cell units; <= 0: the largest root extent */
  int32_t tiles;            /* tiles per face side of the extinction tables, 0..64 */
  int32_t pad;
  int64_t event_buffer;     /* events kept per batch; 0 = 2^24 */
  double* image;            /* [n_dir][n_lambda of the model][npix][npix] host or device,
                               overwritten */
} rt_peel_opts;

rt_status rt_peel_map(rt_ctx* ctx, int32_t n_src, const rt_source* src, const rt_trace_opts* opts,
                      const rt_peel_opts* peel, rt_trace_stats* stats);

/* Autotuner for the launch parameters of rt_trace_packets (the FP32-local form's block size,
 * blocks per CU, refill threshold, tail rounds, packets per work item and packets emitted
 * per sweep; the FP64 form's block size).  Traces a packet-id prefix of every source
 * (sample_fraction of its packets, at least 2^16 per wavelength where available) for each
 * candidate of one parameter at a time, holding the others at the best so far, and keeps
 * the configuration with the most crossings per second of device time (best of two runs).
 * base: the options to start from (precision and schedule select what is tuned; zero fields
 * start at the library defaults); best receives base with the tuned fields filled in;
 * best_rate (may be NULL) the crossings per second of the sample.  cache_path (may be NULL):
 * a text file of earlier results keyed by the workload signature (device CU count, form,
 * sample fraction, model sizes, sources); a hit returns the cached result without tracing,
 * a miss appends the new result.  Uses the context's trace buffers; models, dust and
 * temperatures are unchanged. */
rt_status rt_autotune(rt_ctx* ctx, int32_t n_src, const rt_source* src, const rt_trace_opts* base,
                      double sample_fraction, const char* cache_path, rt_trace_opts* best,
                      double* best_rate);

/* Diagnostic: Philox4x32-10 blocks for explicit counters ctr[n][4] -> out[n][4] (host or
 * device), computed on the GPU with the transport kernels' generator. */
rt_status rt_philox(rt_ctx* ctx, uint32_t key0, uint32_t key1, int64_t n, const uint32_t* ctr,
                    uint32_t* out);

#ifdef __cplusplus
}
#endif
#endif
