/*
 * mcc.h -- C ABI of libmcc_hip.so: the weighted, moment-preserving
 * binary-pairing Monte-Carlo Coulomb collision step on MI355X (gfx950).
 *
 * Method: J. R. Angus, Y. Fu, V. Geyko, D. Grote, D. Larson,
 * "Moment-preserving Monte-Carlo Coulomb collision method for particle codes"
 * (arXiv 2407.19151).  One call applies one time step of the paper's
 * Algorithm 1 to every cell: random binary pairing (Fig. 1, Sec. 3.2; or
 * N x N, Sec. 3.1; or Higginson et al.'s duplicity), weighted TA77/N97
 * scatter with w_min/w_max acceptance (Eq. (12), Secs. 3.1-3.2; or the
 * hard-sphere process, a non-Coulomb case of Sec. 2), momentum restore
 * (Eq. (17)), energy-violation partition
 * (Eqs. (18), (24)) and zero-angle inelastic pair energy correction
 * (Eqs. (19)-(23)); relativistic variant of Appendix A; failure fallback of
 * Sec. 6.2.
 *
 * Conventions for every entry point:
 *  - Pointers marked "device" are HIP device (or managed) pointers; the
 *    caller owns them; the library never frees or retains them past the call.
 *  - Work is enqueued on the context's stream and the call returns without
 *    waiting; outputs are valid after the stream is synchronized.
 *  - Velocities are FP64 structure-of-arrays and are updated in place in all
 *    precision modes.  In relativistic mode they hold the proper velocity
 *    u = gamma v.
 *  - Errors are returned as mcc_status; nothing is thrown across the ABI.
 *    Host-checkable arguments are checked on every call.  Data-dependent
 *    checks (offsets monotone, ids in range, cell sizes within the supported
 *    maximum) run on the device; a violating cell is skipped, never read out
 *    of bounds, and the first such code is latched in the context; read it
 *    with mcc_device_error.  With the environment variable MCC_VALIDATE=1 the
 *    collide calls synchronize and return that code themselves.
 *  - An energy-correction failure is not an error: it is handled by
 *    on_failure and counted in mcc_stats.failed.
 *  - Random numbers are Philox4x32-10 keyed by seed, with counters built from
 *    (index, cell, step, collision, purpose); results do not depend on how
 *    cells are split across calls or GPUs.
 */
#ifndef MCC_H
#define MCC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MCC_OK = 0,
  MCC_ERR_INVALID = -1,     /* bad argument (host check) */
  MCC_ERR_OOM = -2,         /* device allocation failed */
  MCC_ERR_DEVICE = -3,      /* HIP runtime error */
  MCC_ERR_UNSUPPORTED = -4, /* valid but not supported combination */
  MCC_ERR_DATA = -5         /* device-side data check failed (see mcc_device_error) */
} mcc_status;

/* Scattering process of a pair, given its normalized path length s.
 * TA77, N97: small-angle Coulomb scattering; s of Eq. (12) (Eq. (10) for
 * N x N pairing) sets the spread of the centre-of-mass angle (Sec. 3.2).
 * HARD_SPHERE: a non-Coulomb process of the collision integral of Sec. 2,
 * the extension the paper's summary names: elastic scattering with the
 * collision's constant total cross-section and isotropic angles.
 * s = sigma n_eff |u| dt, n_eff the density factor the pairing gives the
 * Coulomb s (w_max N_min / dV, w_max / dV, or w_max (N_max / D) / dV), is
 * read as the expected number of collisions: the pair collides with
 * probability 1 - exp(-s).  Weighting, acceptance and moment correction are
 * the Coulomb ones.  Charges, the Coulomb logarithm and eps0 are unused.
 * FP64 precision and non-relativistic only (otherwise MCC_ERR_UNSUPPORTED);
 * not available to mcc_collide_sorted_jvp. */
typedef enum { MCC_TA77 = 0, MCC_N97 = 1, MCC_HARD_SPHERE = 2 } mcc_method;
typedef enum { MCC_FP64 = 0, MCC_FP32_KINEMATICS = 1 } mcc_precision;
typedef enum { MCC_FAIL_RESET = 0, MCC_FAIL_KEEP = 1 } mcc_fail_policy;
/* Binary pairing of the scatter.  ORDER_N: the TA77 random pairs of Fig. 1
 * (Sec. 3.2), s of Eq. (12) with w_max N_min / dV.  NXN: every pair of
 * the collision once (Sec. 3.1), s of Eq. (10) with w_max / dV and
 * the same w_min/w_max acceptance; the pairs run in rounds of disjoint pairs
 * over the shuffled lists (intra-species: the circle schedule on N rounded
 * up to even, N - 1 or N rounds; inter-species: round r pairs list-a entry i
 * with list-b entry (i + r) mod N_max, N_max rounds).  O(N^2) pairs per cell.
 * DUPLICITY: the order-N pairs with the s of Higginson et al. that the paper
 * describes after Sec. 3.2: an inter-species pair takes N_max / D in place
 * of N_min, D the number of pairs its fewer-population particle takes in the
 * step (intra-species pairs are unchanged).  The momentum restore and energy
 * correction are the same for all three. */
typedef enum {
  MCC_PAIRING_ORDER_N = 0,
  MCC_PAIRING_NXN = 1,
  MCC_PAIRING_DUPLICITY = 2
} mcc_pairing;

#define MCC_MAX_SPECIES 8
#define MCC_MAX_COLLISIONS 32
/* largest number of particles in one cell (all species) */
#define MCC_MAX_CELL 32768

/* Physical (unweighted) mass and charge of a species. */
typedef struct {
  double mass;
  double charge;
} mcc_species;

/* One collision of the step: species a with species b (a == b: intra-species).
 * Collisions are applied in list order; velocities carry over. */
typedef struct {
  int32_t a;
  int32_t b;
  double cross_section; /* MCC_HARD_SPHERE: total cross-section (area, caller's units),
                           finite and >= 0; ignored by the Coulomb methods */
} mcc_collision;

typedef struct {
  int32_t method;            /* mcc_method: angle map from s (Sec. 3.2) */
  int32_t precision;         /* mcc_precision: FP32 pair kinematics, FP64 state/sums/correction */
  int32_t relativistic;      /* 1: arrays hold u = gamma v, Appendix A; needs c */
  int32_t moment_correction; /* 1: Eqs. (17)-(24) after the scatter */
  int32_t sort_by_weight;    /* 1: descending-weight order for the energy pairs (Alg. 1) */
  int32_t max_passes;        /* passes of the energy-pair loop, >= 1 (default 1) */
  int32_t on_failure;        /* mcc_fail_policy (Sec. 6.2) */
  int32_t diagnostics;       /* 1: measure residual momentum/energy per collision into stats */
  int32_t pairing;           /* mcc_pairing (default ORDER_N) */
  double f_E;                /* energy-correction factor, 0 < f_E < 1 (Eq. (23); default 0.05) */
  double eps0;               /* vacuum permittivity in the caller's units (default 1) */
  double c;                  /* speed of light (relativistic only) */
} mcc_params;

/* Step counters; lives in DEVICE memory, accumulated by the kernels.  The
 * collide calls zero it first. */
typedef struct {
  unsigned long long pairs;      /* binary scatter pairs formed */
  unsigned long long corr_pairs; /* energy-correction pairs with U != 0 */
  unsigned long long failed;     /* (cell, collision) energy-correction failures */
  unsigned long long collisions; /* (cell, collision) applications with pairs */
  double max_rel_dP;             /* diagnostics: max residual |dP| / sum m w |v| */
  double max_rel_dE;             /* diagnostics: max residual |dE| / KE */
} mcc_stats;

typedef struct mcc_ctx mcc_ctx;
typedef struct mcc_plan mcc_plan;

/* Defaults: N97, FP64, non-relativistic, correction on, sort on, one pass,
 * reset on failure, no diagnostics, order-N pairing, f_E = 0.05, eps0 = 1,
 * c = 0. */
void mcc_default_params(mcc_params *p);

const char *mcc_status_string(mcc_status s);

/* Create a context on `device` enqueuing on `hip_stream` (NULL: the default
 * stream).  The context owns its workspace (cell work lists, error word,
 * large-cell scratch, the collide kernels' cell-queue counters), grown on
 * demand.  Work enqueued through one context must run in order: the calls of
 * one context share that workspace, so they must not overlap on the device.
 * The context also creates one side stream (default priority) on which the
 * sorted step runs the kernel of its 2049-4096-particle cells beside the
 * 1025-2048 one; it forks from and joins back to the context's stream by
 * events within the call, so callers see one stream. */
mcc_status mcc_create(mcc_ctx **ctx, int device, void *hip_stream);
/* Enqueue later calls on `hip_stream`.  Work already enqueued on the previous
 * stream must be complete (or ordered before the next call) first, since it
 * shares the context's workspace. */
mcc_status mcc_set_stream(mcc_ctx *ctx, void *hip_stream);
void mcc_destroy(mcc_ctx *ctx);

/* Synchronize the context's stream and return the first device-side data
 * error code latched since the last call (0 if none), then clear it.
 * Codes: 1 offsets not monotone or out of [0, n]; 2 cell larger than
 * MCC_MAX_CELL; 3 cell or species id out of range (unsorted entry,
 * re-binning); 4 a weight not positive and finite (the sorted entries check
 * every call, a plan once when it is created). */
mcc_status mcc_device_error(mcc_ctx *ctx, int32_t *code);

/*
 * Kernel variant used for cells of size bucket `bucket` (0..6: cells with at
 * most 128, 256, 512, 1024, 2048, 4096, MCC_MAX_CELL particles) by the
 * non-plan entry points.  `variant` indexes the compiled (threads per cell,
 * capacity) table: 0 (64,128), 1 (64,256), 2 (128,256), 3 (128,512),
 * 4 (256,512), 5 (256,1024), 6 (512,1024), 7 (512,2048), 8 (1024,2048),
 * 9 (1024,4096), 10 (64,32768, one wave with global scratch), 11 (256,2048),
 * 12 (512,4096), 13 (256,4096), 14 (256,32768) and 15 (512,32768) (four and
 * eight waves with global scratch; the diagnostic and tangent forms run them
 * as 10).  In relativistic mode 9, 12 and 13 run in
 * global scratch: as (256,4096), four waves, in the order-N step, and as
 * (64,4096), one wave, in its diagnostic, N x N and duplicity forms.  -1 restores the default, which depends on
 * the precision mode (built-in table, the fastest measured on lognormal
 * cell-size mixes).  The variant's capacity must hold the bucket's largest cell,
 * else MCC_ERR_INVALID.  Results agree between variants to rounding (the
 * order of the per-cell sums depends on the threads per cell).
 */
mcc_status mcc_set_variant(mcc_ctx *ctx, int32_t bucket, int32_t variant);

/*
 * The device's polar-angle sampler alone (Sec. 3.2: the map from the
 * normalized scattering length s to the centre-of-mass angle), for testing
 * it against a reference: for i < n, with uniforms from the 32-bit words
 * a0[i], a1[i] (the same conversion as the collision step), writes
 * oc[i] = 1 - cos(theta) and st[i] = sin(theta), and for N97 A[i] (Nanbu's
 * A(s); may be NULL).  All pointers are device memory; precision selects the
 * FP64 or FP32 kinematics code.
 */
mcc_status mcc_sample_angles(mcc_ctx *ctx, int32_t method, int32_t precision, int64_t n,
                             const double *s, const uint32_t *a0, const uint32_t *a1,
                             double *oc, double *st, double *A);

/*
 * One step on particles grouped by (cell, species) -- Algorithm 1.
 *  n            number of particles
 *  n_cells, n_species (1..MCC_MAX_SPECIES)
 *  offsets      device int64[n_cells*n_species + 1]; particles of cell c and
 *               species s are [offsets[c*S+s], offsets[c*S+s+1])
 *  weights      device double[n], w > 0 (Eq. (4): density w / dV)
 *  vx, vy, vz   device double[n], in/out
 *  cell_volume  device double[n_cells] or NULL to use cell_volume_scalar
 *  species      host mcc_species[n_species]
 *  coll         host mcc_collision[n_coll], n_coll <= MCC_MAX_COLLISIONS
 *  dt, coulomb_log  time step and lnL of Eq. (12)
 *  seed, step   Philox key and step counter
 *  p            host parameters
 *  stats        device mcc_stats* or NULL
 *  cell_corr_pairs  device int32[n_cells] or NULL: energy-correction pairs
 *               used per cell this step (the count of Sec. 5.1)
 */
mcc_status mcc_collide_sorted(mcc_ctx *ctx, int64_t n, int32_t n_cells,
                              int32_t n_species, const int64_t *offsets,
                              const double *weights, double *vx, double *vy,
                              double *vz, const double *cell_volume,
                              double cell_volume_scalar,
                              const mcc_species *species, int32_t n_coll,
                              const mcc_collision *coll, double dt,
                              double coulomb_log, uint64_t seed, uint64_t step,
                              const mcc_params *p, mcc_stats *stats,
                              int32_t *cell_corr_pairs);

/*
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The step
 * of mcc_collide_sorted (same arguments, same results bit for bit) with its
 * cell work lists and size-bucket counters in a fixed device array of the
 * library instead of context workspace; it calls no hipMalloc, hipFree or
 * allocating routine (the context, created beforehand, supplies its error
 * word, angle table and queue counters, all allocated by mcc_create).
 * Limits: n_cells <= 262144 (MCC_ERR_INVALID above); cells of at most 4096
 * particles: a larger cell is left unchanged and latched as data error 2;
 * non-relativistic forms only (MCC_ERR_UNSUPPORTED).  The array (7.3 MB)
 * exists once per device, is held until the process ends and keeps the
 * last call's contents; every call on a device shares it, so calls that
 * overlap on one device race (as calls of one context must not overlap).
 */
mcc_status mcc_collide_sorted_noalloc(mcc_ctx *ctx, int64_t n, int32_t n_cells,
                                      int32_t n_species, const int64_t *offsets,
                                      const double *weights, double *vx, double *vy, double *vz,
                                      const double *cell_volume, double cell_volume_scalar,
                                      const mcc_species *species, int32_t n_coll,
                                      const mcc_collision *coll, double dt, double coulomb_log,
                                      uint64_t seed, uint64_t step, const mcc_params *p,
                                      mcc_stats *stats, int32_t *cell_corr_pairs);

/*
 * One step on particles in any order: cells, species_id are device
 * int32[n].  Particles are grouped by (cell, species) keeping ascending
 * index order inside each group, the sorted step is applied, and the
 * velocities are written back in place.  Same other arguments.  The context
 * grows scratch of about 68 bytes per particle for it (the grouping, the
 * payload in grouped order and in 32-byte records) plus 16 for the binning.
 */
mcc_status mcc_collide(mcc_ctx *ctx, int64_t n, const int32_t *cells,
                       const int32_t *species_id, int32_t n_cells,
                       int32_t n_species, const double *weights, double *vx,
                       double *vy, double *vz, const double *cell_volume,
                       double cell_volume_scalar, const mcc_species *species,
                       int32_t n_coll, const mcc_collision *coll, double dt,
                       double coulomb_log, uint64_t seed, uint64_t step,
                       const mcc_params *p, mcc_stats *stats,
                       int32_t *cell_corr_pairs);

/*
 * Forward-mode derivative of one step (the differentiated form): the same
 * step as mcc_collide_sorted (FP64, non-relativistic), carrying the tangent
 * (tx, ty, tz) of the velocities, device double[n] in/out, and the tangent
 * coulomb_log_tangent of ln(Lambda) (Eq. (12): s is proportional to it).  On
 * return (tx, ty, tz) hold J (t, dlnL) where J is the Jacobian of the step
 * with every random number and every discrete choice of the primal fixed:
 * the pairing, the acceptances, the correction order, the cut pair of
 * Eq. (23) and the failure decision.  The N97 parameter is differentiated as
 * the root of Nanbu's equation (dA/ds = -exp(-s)/L'(A)).  update_primal = 0
 * leaves (vx, vy, vz) unchanged (several tangents of one state); 1 also
 * writes the primal step.  Diagnostics and per-cell counts are not
 * produced; stats (nullable) counts as for mcc_collide_sorted.
 * Errors: MCC_ERR_UNSUPPORTED for the relativistic or FP32 forms or a pairing
 * other than ORDER_N;
 * MCC_ERR_INVALID for a nonzero lnL tangent with lnL <= 0.
 */
mcc_status mcc_collide_sorted_jvp(mcc_ctx *ctx, int64_t n, int32_t n_cells,
                                  int32_t n_species, const int64_t *offsets,
                                  const double *weights, double *vx, double *vy,
                                  double *vz, double *tx, double *ty, double *tz,
                                  const double *cell_volume,
                                  double cell_volume_scalar,
                                  const mcc_species *species, int32_t n_coll,
                                  const mcc_collision *coll, double dt,
                                  double coulomb_log, double coulomb_log_tangent,
                                  uint64_t seed, uint64_t step, const mcc_params *p,
                                  int32_t update_primal, mcc_stats *stats);

/*
 * Reverse-mode derivative of one step (the vector-Jacobian product): for the
 * step of mcc_collide_sorted from the state (vx, vy, vz), device double[n]
 * (read only; not stepped), and an adjoint g of its output velocities,
 * (gx, gy, gz) device double[n] in/out, returns g J in place, J the Jacobian
 * of the step with every random number and every discrete choice of the step
 * fixed: the pairing, the acceptances, the correction order, the cut pair of
 * Eq. (23) and the failure decision.  Through the cut pair, whose U is
 * Delta E_s minus the f_E K of the pairs before it, the derivative reaches
 * the energy violation of Eq. (18), its partition (Eq. (24)) and the
 * momentum restore of Eq. (17).  The N97 parameter is differentiated as the
 * root of Nanbu's equation (dA/ds = -exp(-s)/L'(A)); s is proportional to
 * lnL (Eq. (12)).
 *  g_coulomb_log  device double* or NULL: receives g dv'/dlnL (zero when
 *                 lnL = 0, where no pair scatters)
 * FP32 kinematics: the step is recomputed in that form, so the derivative
 * is taken at its states and with its discrete choices and 23-bit uniforms;
 * the pair Jacobians are evaluated in FP64.  A reset (Sec. 6.2) collision
 * passes the adjoint through unchanged.
 * Scratch: per workgroup, 228 B per particle of capacity (4096, or
 * MCC_MAX_CELL for the cells above 4096): about 0.5 GB on 256 compute units
 * for cells up to 4096, 1.9 GB more once a cell above 4096 occurs; owned by
 * the context.  The call waits once on the context's stream (to read the
 * cell counts per size bucket) before it enqueues the kernels.
 * Errors: MCC_ERR_UNSUPPORTED for the relativistic form, a pairing other
 * than ORDER_N, hard spheres or max_passes > 1.
 */
mcc_status mcc_collide_adjoint(mcc_ctx *ctx, int64_t n, int32_t n_cells, int32_t n_species,
                               const int64_t *offsets, const double *weights, const double *vx,
                               const double *vy, const double *vz, double *gx, double *gy,
                               double *gz, const double *cell_volume,
                               double cell_volume_scalar, const mcc_species *species,
                               int32_t n_coll, const mcc_collision *coll, double dt,
                               double coulomb_log, uint64_t seed, uint64_t step,
                               const mcc_params *p, double *g_coulomb_log);

/*
 * Cell binning alone (the grouping used by mcc_collide, the particles of a
 * cell of Sec. 2): a stable sort of the particles by the group key
 * cell * n_species + species.
 *  offsets_out  device int64[n_cells*n_species + 1]
 *  perm_out     device int32[n]: perm_out[j] = original index of the j-th
 *               particle in grouped order (ascending within each group)
 * A particle whose cell or species id is out of range is latched as data
 * error 3 and placed after every group, in index order (offsets_out[end]
 * then counts the particles with valid ids).  Cost: ceil(b/9) passes of a
 * radix sort over 9-bit digits, b the bits of n_cells * n_species, each
 * reading and writing 8 B per particle.  Scratch: 16 B per particle plus
 * 12 B per 4096 particles per digit bin (512 bins), owned by the context.
 * Errors: MCC_ERR_UNSUPPORTED above 2^31 - 1 particles or groups.
 */
mcc_status mcc_bin(mcc_ctx *ctx, int64_t n, const int32_t *cells,
                   const int32_t *species_id, int32_t n_cells,
                   int32_t n_species, int64_t *offsets_out, int32_t *perm_out);

/*
 * Incremental re-binning: the regrouping of a grouped population after its
 * particles moved to new cells (a particle push between collision steps).
 * The grouping by cell is the one every collision step starts from (the
 * particles of a cell, Sec. 2); when few particles change cell, it is
 * updated in a few streaming passes instead of being rebuilt.
 *  offsets      device int64[n_cells*n_species + 1]: the current grouping
 *               (offsets[0] = 0, monotone, offsets[end] = n)
 *  cells_new    device int32[n]: the new cell of the particle at each
 *               grouped position (its species does not change)
 *  offsets_out  device int64[n_cells*n_species + 1]
 *  perm_out     device int32[n]: perm_out[j] = current position of the
 *               particle that goes to position j; ascending inside every
 *               new group, i.e. what mcc_bin returns for cells_new and the
 *               species of each position
 *  weights, vx, vy, vz  device double[n], all or none (NULL): permuted in
 *               place to the new order
 * Cost: two streaming passes over cells_new (the second also writes
 * perm_out) and work on the movers only: each group's arrivals are sorted
 * by position (a sorting network: one thread for up to 32, a wave beyond).
 * Meant for partial moves; rebuild a wholesale reshuffle with mcc_bin.
 * Context scratch: about 12 bytes per particle and 36 per group.  Data errors (cell id out of range, inconsistent
 * offsets) are latched as for the collide calls; such a particle keeps its
 * cell.  Errors: MCC_ERR_INVALID for bad arguments (some payload pointers
 * only), MCC_ERR_UNSUPPORTED above 2^31 - 1 particles or groups.
 */
mcc_status mcc_rebin(mcc_ctx *ctx, int64_t n, int32_t n_cells, int32_t n_species,
                     const int64_t *offsets, const int32_t *cells_new, int64_t *offsets_out,
                     int32_t *perm_out, double *weights, double *vx, double *vy, double *vz);
/* The same regrouping with the payload gathered out of place, for callers
 * that keep two sets of particle arrays and swap them: weights, vx, vy, vz
 * (read) go to weights_out, vx_out, vy_out, vz_out (written) in the new
 * order, with no scratch arrays and no copy back.  All eight are required
 * when n > 0.  An output array must not overlap an input array (the same
 * pointer is rejected with MCC_ERR_INVALID; partial overlap is not
 * detected).  Other arguments and errors as for mcc_rebin. */
mcc_status mcc_rebin_out(mcc_ctx *ctx, int64_t n, int32_t n_cells, int32_t n_species,
                         const int64_t *offsets, const int32_t *cells_new, int64_t *offsets_out,
                         int32_t *perm_out, const double *weights, const double *vx,
                         const double *vy, const double *vz, double *weights_out,
                         double *vx_out, double *vy_out, double *vz_out);

/*
 * Batched form: a plan binds the sorted arrays of one particle population
 * (same pointers every step), sorts its cells into size buckets on the
 * device and each bucket's cells largest first (on the host: the offsets and
 * the lists are copied there once, so the last cells a bucket's persistent
 * grid claims are its smallest), picks threads-per-cell for each bucket
 * (autotune = 1 times the candidates on this population; 0 uses the
 * built-in table), and captures one step into a HIP graph.  mcc_plan_run replays it n_steps times with
 * steps first_step, first_step+1, ...  The plan holds the offsets and the
 * weights by pointer: if they change, destroy and re-create it.  With the
 * moment correction on, it also computes once what depends on the weights
 * alone (per cell and species: sum w, sum w^2, the weight range, and the
 * descending-weight order of Algorithm 1), owning 40 B per (cell, species)
 * and 2 B per particle of device memory for it.  A plan whose cells need the
 * large-cell kernels (above 4096 particles, or above 2048 in relativistic
 * mode) owns their global scratch too, 2.75 MB per compute unit for cells
 * above 4096 particles (0.34 MB up to 4096), held until mcc_plan_destroy:
 * its graph replays against that scratch, so later calls on the context
 * (which grow the context's own scratch) never move it.  A plan shares the
 * context's cell-queue counters and error word, so its replays must not
 * overlap other work of the same context either.
 */
mcc_status mcc_plan_create(mcc_ctx *ctx, mcc_plan **plan, int64_t n,
                           int32_t n_cells, int32_t n_species,
                           const int64_t *offsets, const double *weights,
                           double *vx, double *vy, double *vz,
                           const double *cell_volume, double cell_volume_scalar,
                           const mcc_species *species, int32_t n_coll,
                           const mcc_collision *coll, double dt,
                           double coulomb_log, uint64_t seed,
                           const mcc_params *p, mcc_stats *stats,
                           int32_t *cell_corr_pairs, int32_t autotune);
mcc_status mcc_plan_run(mcc_plan *plan, uint64_t first_step, int32_t n_steps);
/* The cells of one size bucket only (0..6, as for mcc_set_variant), one step
 * `step`, launched directly rather than from the graph: for timing one kernel
 * of the step.  Stats and per-cell counts accumulate without a reset. */
mcc_status mcc_plan_run_bucket(mcc_plan *plan, int32_t bucket, uint64_t step);
/* Text (JSON) description of the buckets: cell and particle counts, the
 * chosen kernel variants and the autotuner's timings. */
mcc_status mcc_plan_describe(mcc_plan *plan, char *buf, size_t len);
void mcc_plan_destroy(mcc_plan *plan);

#ifdef __cplusplus
}
#endif

#endif /* MCC_H */
