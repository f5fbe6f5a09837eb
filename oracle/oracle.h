/* FP64 CPU oracle for Monte Carlo continuum radiative transfer on an oct-tree.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, single-threaded C; shares no source with the GPU
 * library.  Only the tests, the smoke check and the benchmark's CPU-baseline leg may load it.
 *
 * What it follows (Lunttila & Juvela, "Radiative transfer on hierarchial grids"):
 *   - Sect. 2.1: nested-grid hierarchy, subgrid identification looked up at every crossing;
 *   - Sect. 2.3: packets from internal sources and from the external field, continuous
 *     absorption, Russian roulette with threshold n and probability p;
 *   - Sect. 3.1 Eq. (2): Lambda iteration J_{n+1} = Lambda S_n + J_0, S_{n+1} = f(J_{n+1});
 *   - Sect. 4: one dust component at its equilibrium temperature, frequencies one by one;
 *   - Sect. 4.1: surface-brightness maps toward chosen directions.
 * The in-grid tracking itself is not described in the paper (it defers to earlier work);
 * the readings used here are listed in the header comment of oracle.c.
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct om_model om_model;

/* Build a model from a tree description (root grid + per-level refined-cell lists + child
 * densities, canonical order).  Returns NULL on invalid input (message in om_error()). */
om_model* om_build(int32_t nx, int32_t ny, int32_t nz, double root_cell_cm, int32_t n_levels,
                   const double* root_rho, const int64_t* n_refined,
                   const int64_t* const* refined, const double* const* child_rho);
void om_free(om_model* m);
const char* om_error(void);

int64_t om_n_nodes(const om_model* m);
int32_t om_n_levels(const om_model* m);
void om_level_offsets(const om_model* m, int64_t* off /* n_levels+2 */);
void om_child(const om_model* m, int64_t* child /* n_nodes: oct index or -1 */);
void om_node_rho(const om_model* m, double* rho);

/* Point location: half-open cells.  level_out/node_out receive -1 outside. */
void om_locate(const om_model* m, int64_t n, const double* xyz, int32_t* level_out,
               int64_t* node_out);

/* Philox4x32-10 blocks for explicit counters: ctr[4n] -> out[4n]. */
void om_philox(uint32_t k0, uint32_t k1, int64_t n, const uint32_t* ctr, uint32_t* out);

int om_set_dust(om_model* m, int32_t n_lambda, const double* lambda_um, const double* kappa,
                const double* albedo, const double* hg_g);
void om_dnu(const om_model* m, double* dnu);

/* Source kinds */
#define OM_BACKGROUND 0
#define OM_POINT 1
#define OM_DUST 2
#define OM_BEAM 3

typedef struct {
  uint64_t crossings, scatterings, kills, truncated, packets, dropped_zero_q;
  double e_emit, e_abs, e_esc, e_killed, e_rr_gain, e_trunc;
  uint64_t splits, split_kills;
  double e_split_killed, e_split_gain;
} om_stats;

/* One packet's end state (for sampled-history comparison). status: 0 escaped, 1 killed,
   2 truncated, 3 killed leaving a subgrid (package splitting).  node: canonical node where the
   packet ended (-1 if escaped); birth: node where
   it started; w: its weight at the end. */
typedef struct {
  uint32_t status, crossings, events, pad;
  int64_t node, birth;
  double w;
} om_record;

/* Trace the packets of n_src sources.  For each source s and each wavelength i, packets
 * 0..packets[s]-1 of stream (model<<20 | s<<12 | i) are followed.  power[s*n_lambda + i]
 * is the background intensity times nothing (I_nu, per Hz) or the source luminosity L_nu;
 * DUST sources take the temperatures t_node (canonical, leaves) instead.
 * e_abs: [n_nodes] (lambda-integrated) or [n_lambda*n_nodes] if per_lambda; NULL to only
 * total the deposits in stats (single-packet replays on large trees).
 * e_esc: [n_lambda].  rec (optional): one record per sampled packet, packet index j of
 * (source s, wavelength i) is sampled when j % rec_stride == 0 and stored at
 * (s*n_lambda + i)*nrec + (j-pid_begin)/rec_stride with nrec = ceil((pid_end-pid_begin)/rec_stride);
 * only packets j in [pid_begin, min(pid_end, packets[s])) are traced, and only wavelength
 * lam_sel unless it is negative.  split_n > 1 turns on package splitting at subgrid entry
 * (Sect. 2.3): a package whose crossing lands in a deeper leaf continues with 1/split_n of its
 * weight and split_n - 1 packages of the same weight start there (each a new branch, with its
 * own free path); a package whose crossing lands in a shallower leaf survives with probability
 * 1/split_n, its weight multiplied by split_n.  A record follows the emitted package's main
 * line (the branch that keeps its identifier). */
/* Peel-off (Sect. 2.4): at every scattering event (before the event roulette) the part of
 * the packet scattered toward each observer direction and escaping, w Phi_HG(d.n)
 * exp(-tau(P -> border along n)), is added as surface brightness (per Hz, per pixel area in
 * cm^2, per steradian) to the pixel the event position projects onto (the map geometry of
 * om_render).  tiles > 0: tau from extinction tables on the faces of every refined root cell
 * (tiles x tiles per face, the column from each tile centre): a ray from inside a refined root
 * cell is marched to that cell's boundary, a ray from a root leaf through root leaves until it
 * enters a refined root cell or leaves the model, and the table value of the tile it crosses is
 * added.  tiles = 0: the column is marched to the border. */
typedef struct {
  int32_t n_dir;          /* 1..16 */
  const double* n_obs;    /* [n_dir][3], any length > 0 */
  int32_t npix;
  double width;           /* root-cell units; <= 0: largest root extent */
  int32_t tiles;
  double* image;          /* [n_dir][n_lambda][npix][npix], added to */
} om_peel_opts;

int om_trace(om_model* m, int32_t model_index, int32_t n_src, const int32_t* kind,
             const double* pos /*3n*/, const double* dir /*3n*/, const double* power,
             const int64_t* packets, const double* t_node, uint64_t seed, uint32_t iteration,
             double rr_threshold, double rr_prob, int64_t max_events, int32_t per_lambda,
             int64_t pid_begin, int64_t pid_end, int32_t lam_sel,
             double* e_abs, double* e_esc, om_stats* stats, int64_t rec_stride, om_record* rec,
             int32_t split_n, const om_peel_opts* peel, double* e_self, double* e_emit_node,
             double* e_lvl, int64_t sub_node, double* e_flux, int32_t split_depth);

/* e_self, e_emit_node ([n_nodes], added to; NULL = off): for the accelerated Lambda iteration
 * (Sect. 3.1 Eq. 3, diagonal operator), the energy that dust-emission packets deposit in their
 * birth cell before their first crossing, and the energy they start with, per birth cell. */

/* Subiterations (Sect. 3.1, App. B).  e_lvl ([n_levels + 1][n_nodes], added to; NULL = off):
 * every deposit also goes to the array of the shallowest hierarchy level the package has
 * visited (0 for the external field, which enters through the root grid; otherwise the birth
 * level, lowered at every crossing into a shallower cell).  sub_node >= 0 (a refined node):
 * only the leaves of its subtree emit dust, and a package leaving the subtree is ended there
 * (tallied as escaped). */

/* e_flux ([n_nodes], added to; NULL = off): for the automatic iteration (Sect. 3.3), the energy
 * flowing from each grid to its parent: per refined node, the weight of the packages leaving its
 * subtree (to a neighbour outside it, out of the model, or out of the iterated subtree). */

/* Equilibrium temperature per leaf: 4 pi m sum_i kappa_abs_i B_i(T) dnu_i = A. */
void om_solve_temperature(const om_model* m, const double* a_node, double t_min, double t_max,
                          double* t_node);
/* Emitted power of a leaf at temperature T (the left-hand side above). */
double om_emission(const om_model* m, int64_t node, double t);

/* Surface-brightness map along rays toward the observer direction n. */
int om_render(const om_model* m, const double n_obs[3], int32_t npix, double width,
              int32_t n_sel, const int32_t* lambda_idx, const double* t_node, double* image,
              uint64_t* crossings);

/* Test hooks exposing single steps for the pins. */
double om_hg_mu(double g, double u);
void om_rotate(double* d, double mu, double phi);
double om_uniform(uint32_t x);
int64_t om_cdf_pick(const uint64_t* q, int64_t n, uint64_t r);
uint32_t om_branch_id(uint32_t b, uint32_t n, uint32_t c);
double om_hg_phase(double g, double mu);
/* Emitted power of every leaf at t_node (0 for refined nodes). */
void om_emission_all(const om_model* m, const double* t_node, double* out);
/* Integer coordinates of every node at its own level: out[3 n_nodes]. */
void om_node_coords(const om_model* m, int32_t* out);
/* Peel-off column (density x length, root-cell units) from each point toward n_obs, marched
 * to the border (tiles = 0) or with the extinction tables. */
int om_peel_column(const om_model* m, const double n_obs[3], int32_t tiles, int64_t npts,
                   const double* xyz, double* col);

#ifdef __cplusplus
}
#endif
#endif
