/*
 * md.h - C ABI of libmdx, an MI355X (gfx950) molecular-dynamics hot path:
 * Lennard-Jones / Kob-Andersen pair forces over Verlet neighbour lists built
 * from a particle sort by cell, and velocity-Verlet integration with the
 * position and velocity updates in double-single (FP32-pair) arithmetic.
 *
 * The method is that of Colberg & Hoefling, "Highly accelerated simulations
 * of glassy dynamics using GPUs: caveats on limited floating-point precision"
 * (arXiv:0912.3824):
 *   - Sec. 2.2 (the MD integration step): velocity Verlet, Verlet lists with
 *     a skin, cell binning by a sort on the 1-D cell index, rebuild when the
 *     maximum displacement since the last build demands it;
 *   - Sec. 2.4 and Alg. 1 (double-single arithmetic): the velocity-Verlet
 *     update and the force summation in double-single, the pair force itself
 *     in single precision;
 *   - Sec. 3: LJ 12-6 potential cut off at rc = 2.5 sigma, dt* = 0.001;
 *   - Sec. 5: the Kob-Andersen pair table (eps_AB = 1.5, eps_BB = 0.5,
 *     sigma_AB = 0.8, sigma_BB = 0.88, equal masses).
 *
 * Conventions shared by every entry point
 *   - Units are reduced LJ units (sigma_AA, eps_AA, m).  Boxes are cubic and
 *     periodic.  Energies are shifted to vanish at the cutoff, forces are not.
 *   - A system is a pool of `max_slots` replica slots over one particle arena;
 *     a single system is a pool with one attached replica.  Replicas are
 *     independent: the trajectory of a replica does not depend on which other
 *     replicas share the pool (bitwise).
 *   - Memory: the CALLER owns all device memory.  It passes one device
 *     workspace of md_workspace_bytes() bytes and a hipStream_t (as void*);
 *     the library never allocates or frees device memory.  The library owns
 *     only the host handle (freed by md_destroy) and its host-side mirrors.
 *   - Host arrays passed in are read before the call returns; host arrays
 *     passed out are written before the call returns.
 *   - Asynchrony: calls that only launch work (md_step, md_advance,
 *     md_rebuild_neighbours, md_forces with NULL outputs) return before the
 *     GPU finishes.  Calls that return data to the host synchronise the stream.
 *   - Errors: no exception crosses the ABI.  Every call returns an md_status;
 *     md_last_error() holds a human-readable description of the last failure
 *     on that handle.  Device-side failures (list overflow, non-finite
 *     coordinates) set sticky per-replica status bits.  A replica with such
 *     a bit stops on the device at once (the next step launch leaves it
 *     where it is, so no step runs on a truncated list); the other replicas
 *     of the pool go on unaffected.  md_poll() and md_observables() report
 *     the bits and return MD_E_CAPACITY or MD_E_NONFINITE; after that, the
 *     launching calls (md_step, md_advance) return the same code without
 *     launching until the replica is detached or restored.  The library
 *     does not regrow a list: the capacity is fixed by the workspace.
 *   - Threading: one handle must not be used from two host threads at once.
 */
#ifndef MDX_MD_H
#define MDX_MD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MD_ABI_VERSION 5

typedef struct md_system md_system;

typedef enum {
    MD_OK = 0,
    MD_E_ARG = -1,       /* invalid argument or configuration */
    MD_E_BOX = -2,       /* box shorter than twice the largest list radius */
    MD_E_WORKSPACE = -3, /* workspace missing, misaligned or too small */
    MD_E_CAPACITY = -4,  /* particle/cell arena full or neighbour list overflow */
    MD_E_NONFINITE = -5, /* a coordinate or force became NaN/Inf */
    MD_E_HIP = -6,       /* a HIP runtime call failed */
    MD_E_NOSLOT = -7,    /* slot index out of range, busy or empty */
    MD_E_STATE = -8      /* call not valid in the current state */
} md_status;

/* Arithmetic of the path (Sec. 2.4 defines the double-single split). */
typedef enum {
    MD_FP32 = 0,    /* FP32 pair force, FP32 force sum, FP32 velocity Verlet */
    MD_DS = 1,      /* FP32 pair force, double-single force sum (error-free
                       transformations), double-single velocity Verlet (Alg. 1) */
    MD_MIXED64 = 2, /* FP32 pair force, FP64 force sum, FP64 velocity Verlet */
    MD_FP64 = 3     /* everything in FP64 */
} md_precision;

/* Order of the cells in the particle sort.  Sec. 2.2 reorders particles
 * along a Hilbert curve for the locality of neighbour reads; here the sort
 * is by cell (each species separately), and the cells follow one of these
 * orders.  For nd^3 cells, the Morton and Hilbert orders are those of the
 * enclosing 2^b grid with the cells outside nd^3 skipped. */
typedef enum {
    MD_ORDER_ROW = 0,     /* rank = x + nd (y + nd z) */
    MD_ORDER_MORTON = 1,  /* Z-order: coordinate bits interleaved (x lowest) */
    MD_ORDER_HILBERT = 2  /* Hilbert curve (Skilling's transposed index):
                             consecutive cells are face neighbours on 2^b grids */
} md_cell_order_kind;

/* Per-replica status bits (sticky until md_detach / md_restore). */
#define MD_ST_LIST_OVERFLOW 1 /* a particle had more neighbours than nbr_capacity */
#define MD_ST_NONFINITE 2     /* a position became NaN/Inf */
#define MD_ST_LOST 4          /* cell counting lost particles (follows NONFINITE) */
#define MD_ST_NO_PAD 8        /* a list could not be padded: every particle of the
                                 replica lies within the list radius of another */
#define MD_ST_AT_FULL_STEP 256 /* not an error: velocities are at a full step
                                  (reported by md_poll only) */

/*
 * Pool configuration.  Pair parameters are a symmetric 2x2 table indexed
 * [a*2+b] for species a, b in {0 (A), 1 (B)}; with n_species == 1 only [0]
 * is used.  rcut holds absolute cutoffs (the KA reading is 2.5 sigma_ab).
 * The list radius of a pair is rcut[ab] + skin (Sec. 2.2).
 */
typedef struct {
    int32_t n_species;     /* 1 or 2 */
    int32_t precision;     /* md_precision */
    double eps[4];
    double sigma[4];
    double rcut[4];
    double mass;           /* equal masses (Sec. 5); > 0 */
    double dt;             /* time step; > 0 */
    double skin;           /* Verlet skin; > 0 */
    int32_t nbr_capacity;  /* list entries per particle, rounded up to a multiple of 16;
                              0 = derive from max_density */
    int32_t max_slots;     /* replicas attachable at once; >= 1 */
    int64_t max_particles; /* particle arena capacity: 1 .. 2^28 - 256 (Verlet-list
                              entries are 32-bit byte offsets of 16-byte records) */
    int64_t max_cells;     /* cell arena capacity; 0 = derive from max_particles */
    double max_density;    /* density used to derive capacities; 0 = 1.2 */
    int32_t lanes_per_particle; /* lanes summing one particle's list: 1, 2 or 4
                                   (0 = 2).  Part of the arithmetic: the force
                                   sum is split into this many partial sums,
                                   combined in a fixed order, so results are
                                   bitwise reproducible for a given value. */
    int32_t cell_order;    /* md_cell_order_kind: the order of the cells in the particle
                              sort (Sec. 2.2 orders particles along a Hilbert curve);
                              part of the arithmetic (it fixes the list order) */
    double smooth;         /* h of the C2 smoothing of Sec. 4: the truncated-and-
                              shifted potential times g(x) = x^4 / (1 + x^4),
                              x = (r - rc_ab) / (h sigma_ab); 0 = no smoothing;
                              >= 0 and finite.  (WCA is rcut = 2^(1/6) sigma.) */
    int32_t rebuild_every; /* 0, or K >= 2: a replica also rebuilds its lists after
                              a step whose count is a multiple of K once its largest
                              displacement since the last build exceeds
                              rebuild_early * skin / 2 (besides the skin / 2 rule of
                              Sec. 2.2).  Replicas of a pool whose step counts are
                              aligned then rebuild together, at a few launches, so a
                              batch pays the rebuild kernels' latency once for many
                              replicas.  The rule reads only the replica's own state
                              (a replica rebuilds at the same steps alone and in a
                              pool); it is part of the arithmetic (it moves the
                              rebuild steps, hence the sort and sum order). */
    int32_t reserved0;
    double rebuild_early;  /* the fraction in (0, 1] for rebuild_every; else ignored */
} md_config;

/* One replica: N particles in a cubic box of edge `box`. */
typedef struct {
    int32_t n;
    int32_t reserved;
    double box;
} md_replica;

/* Observables of one replica at its current (full) step, FP64 sums over the
 * per-particle values in a fixed order. */
typedef struct {
    double epot;        /* sum_i e_i, e_i = 1/2 sum_j V_ts(r_ij) */
    double ekin;        /* 1/2 m sum_i v_i^2 */
    double etot;
    double temperature; /* 2 E_kin / (3 N) */
    double virial;      /* W = sum_{i<j} r_ij . F_ij */
    double pressure;    /* (2 E_kin + W) / (3 V) */
    double momentum[3]; /* m sum_i v_i */
    int64_t step;       /* steps completed since attach */
    int64_t n_rebuilds; /* neighbour-list builds since attach (incl. the first) */
    int64_t list_entries; /* sum of the Verlet-list lengths of the replica */
    int32_t status;     /* MD_ST_* bits */
    int32_t n;          /* particles (0 if the slot is empty) */
} md_obs;

/* Launch shapes (the autotuner's knobs).  None changes any result bit. */
typedef struct {
    int32_t step_block;    /* threads per block of the fused step kernel: 64..1024, multiple of 64 */
    int32_t build_width;   /* cells per row segment staged in LDS by the list build: 1..16 */
    int32_t build_block;   /* threads per block of the list build: 64..1024, multiple of 64 */
    int32_t graph_steps;   /* steps per captured hipGraph (even, 2..256); 0 = no graphs */
    int32_t xcd_remap;     /* 1 = map consecutive particle tiles to one XCD (8 XCDs) */
    int32_t build_lanes;   /* lanes that build one particle's list together: 1, 2, 4, .., 64;
                            * 0 = automatic: one lane for replicas with >= 256 row segments;
                            * smaller replicas split each segment's members over several
                            * work items, each using the most lanes that keep one group per
                            * member (16 for single-cell replicas) */
    int32_t build_split;   /* most list-build work items one row segment is split into (the
                            * members of a small replica's segments are shared out): 0 =
                            * automatic (up to 256 / segments per replica), 1 = no split,
                            * up to 256 */
    int32_t build_bulk;    /* a step's list build in which at least this many replicas rebuild
                            * uses one lane per member and unsplit row segments for every
                            * replica of more than one cell, whatever build_lanes and
                            * build_split say (the shape that suits many simultaneous
                            * rebuilds, as aligned rebuilds make); 0 = never.  Changes no
                            * list entry. */
} md_launch;

/* ---- sizing and lifetime ------------------------------------------------ */

/* Bytes of device workspace a pool with this configuration needs (>= 0), or
 * a negative md_status if the configuration is invalid.  Host only; no GPU
 * call. */
int64_t md_workspace_bytes(const md_config *cfg);

/* Validate a configuration and a replica against it without touching the
 * GPU: returns MD_OK, MD_E_ARG, MD_E_BOX (the box is shorter than twice the
 * largest list radius, so the minimum image of Sec. 2.2 would be ambiguous)
 * or MD_E_CAPACITY (the replica would not fit even an empty pool of this
 * configuration: more particles than max_particles, or more cells than the
 * cell arena holds).  `rep` may be NULL. */
md_status md_validate(const md_config *cfg, const md_replica *rep);

/* Create an empty pool over the caller's workspace (device pointer,
 * 256-byte aligned, ws_bytes >= md_workspace_bytes(cfg)) and stream
 * (hipStream_t as void*, must not be the legacy NULL stream when graphs are
 * used).  Clears the control words on the stream.  On success *out owns a
 * host handle. */
md_status md_create(const md_config *cfg, void *workspace, int64_t ws_bytes,
                    void *hip_stream, md_system **out);

/* md_init (the one-call form): md_create, then md_attach of replicas
 * 0..n_rep-1 into slots 0..n_rep-1.  species/pos/vel are host arrays of the
 * concatenated replicas (sum of n entries; pos and vel [n][3] FP64).  The
 * problem it sets up is the paper's: N particles of one or two species with
 * equal masses in a periodic cubic box, pair parameters per species pair,
 * a cutoff, a time step and a list skin (Sec. 2.2 and Sec. 3; the KA table
 * of Sec. 5).  On an error after md_create succeeded, *out stays valid so
 * the caller can read md_last_error and call md_destroy. */
md_status md_init(const md_config *cfg, const md_replica *reps, int32_t n_rep,
                  const int32_t *species, const double *pos, const double *vel,
                  void *workspace, int64_t ws_bytes, void *hip_stream,
                  md_system **out);

/* Free the host handle.  Device memory stays with the caller.  Safe on NULL. */
void md_destroy(md_system *sys);

/* ---- replicas (serving pool) --------------------------------------------- */

/* Attach a replica to an empty slot: host FP64 positions (any image; they
 * are wrapped into [0, box)), velocities and species (0/1) are converted to
 * the pool's precision (double-single: hi = fl32(x), lo = fl32(x - hi),
 * Sec. 2.4), sorted by cell on the host (the cell binning of Sec. 2.2),
 * uploaded, and the replica's first Verlet list is built (Sec. 2.2).  The replica starts at step 0 with full-step velocities.
 * Synchronises the stream.  Errors: MD_E_NOSLOT, MD_E_BOX, MD_E_CAPACITY
 * (arena full or list overflow), MD_E_ARG. */
md_status md_attach(md_system *sys, int32_t slot, const md_replica *rep,
                    const int32_t *species, const double *pos, const double *vel);

/* Release a slot and its arena ranges.  Pending work on the stream that
 * still advances the replica must have finished (call md_poll first). */
md_status md_detach(md_system *sys, int32_t slot);

/* ---- the MD step ---------------------------------------------------------- */

/* Rebuild (re-sort by cell, then Verlet lists) every attached replica now,
 * at its current positions (Sec. 2.2).  Asynchronous. */
md_status md_rebuild_neighbours(md_system *sys);

/* Evaluate forces, per-particle energies and virials at the current
 * positions of every attached replica (no state change): the pair force of
 * Sec. 3 (12-6 LJ, truncated at the pair's cutoff, energy shifted) over each
 * particle's Verlet list, the pair term in FP32 and the sum in the pool's
 * precision (Sec. 2.4), or all in FP64.  If f_host (n x 3)
 * or e_host (n) are non-NULL, synchronises and copies the values of `slot`
 * in particle-id order (input order of md_attach).  Asynchronous when both
 * are NULL (slot is then ignored). */
md_status md_forces(md_system *sys, int32_t slot, double *f_host, double *e_host);

/* Advance every attached replica by n_steps velocity-Verlet steps (Sec. 2.2;
 * refused with MD_E_CAPACITY / MD_E_NONFINITE while a replica reported as
 * stopped by md_poll or md_observables is attached):
 * per step one fused launch (force, second half-kick, first half-kick of the
 * next step, drift, displacement check) plus the rebuild kernels, which do
 * work only for replicas whose maximum displacement since their last build
 * exceeds skin/2.  Replays captured hipGraphs where possible.  Replicas end
 * at full-step velocities.  Asynchronous.
 *
 * The launch that brings a replica to its full step keeps its forces, and the
 * next call's first launch uses them instead of evaluating forces again at
 * the same positions, so n calls of one step cost as many force passes as one
 * call of n steps, with bitwise the same trajectory.  md_rebuild_neighbours,
 * md_thermostat and, in double-single mode, md_forces and md_observables
 * (which overwrite the rows that hold them) drop the kept forces; the next
 * call then evaluates them. */
md_status md_step(md_system *sys, int64_t n_steps);

/* Serving form: set the absolute step at which a replica stops
 * (>= its current step).  Takes effect for launches issued afterwards. */
md_status md_set_target(md_system *sys, int32_t slot, int64_t target_step);

/* Serving form: issue n_launch step launches for the whole pool; each
 * replica advances until it reaches its target, then finalises (full-step
 * velocities) and idles.  Asynchronous. */
md_status md_advance(md_system *sys, int64_t n_launch);

/* Synchronise and read every slot's completed step count (steps[max_slots],
 * -1 for empty slots) and status bits (status[max_slots]); either may be
 * NULL.  The outputs are always written.  Returns MD_OK, or MD_E_CAPACITY /
 * MD_E_NONFINITE if an attached replica has stopped with an error bit
 * (md_last_error names the first such slot). */
md_status md_poll(md_system *sys, int64_t *steps, int32_t *status);

/* Synchronise and compute the observables of every slot (out[max_slots]):
 * the reductions of Sec. 2.2 (potential energy, kinetic energy and
 * temperature, momentum, virial and pressure), as FP64 sums in a fixed
 * order.  Replicas must be at full steps (true after md_step, or once
 * md_advance reached their target).  `out` is always written; returns
 * MD_E_CAPACITY / MD_E_NONFINITE like md_poll if a replica has stopped. */
md_status md_observables(md_system *sys, md_obs *out);

/* Multiply the velocities of a replica by `factor` (velocity rescaling for
 * host-driven equilibration).  Asynchronous. */
md_status md_scale_velocities(md_system *sys, int32_t slot, double factor);

/* Modified Andersen thermostat (Sec. 2.3): assign every particle of the
 * replica at `slot` a Maxwell-Boltzmann velocity at `temperature` (mass from
 * the configuration), subtract the mean velocity if remove_mean != 0, and
 * rescale all velocities so that 2 E_kin / (3 N) equals `temperature`
 * exactly.  Random numbers: rand48 (x -> 0x5DEECE66D x + 0xB mod 2^48)
 * started from the state srand48(seed) sets (low 32 bits of seed); particle
 * id i at call `call` uses stream elements i + n (4 call + r), r = 0..3 (a
 * leap-frog of stride n), turned into three normals by Box-Muller.  Calling
 * it every (mu dt)^-1 steps with call = 0, 1, 2, ... is the paper's heat
 * bath of collision rate mu.  The replica must be at a full step.
 * Asynchronous.  Errors: MD_E_NOSLOT, MD_E_ARG, MD_E_HIP. */
md_status md_thermostat(md_system *sys, int32_t slot, double temperature, uint64_t seed, int64_t call,
                        int32_t remove_mean);

/* md_thermostat for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, same arithmetic and bitwise the same velocities as
 * md_thermostat, but it neither allocates nor touches the pool's scratch
 * rows (which md_forces results occupy): its per-call partial sums live in
 * a static device array inside the library, one per GPU, of at most 16384
 * chunks of 4096 particles, so a replica may hold at most 67,108,864
 * particles (else MD_E_CAPACITY, nothing launched).  The array is shared by
 * every call on a GPU: calls that overlap on one GPU (two streams, two host
 * threads) race and must not be issued.  Asynchronous.  Errors as
 * md_thermostat, plus MD_E_CAPACITY and MD_E_STATE. */
md_status md_thermostat_noalloc(md_system *sys, int32_t slot, double temperature, uint64_t seed,
                                int64_t call, int32_t remove_mean);

/* Benchmark helper: advance every attached replica by n_steps like md_step
 * but with eager launches, timing each step's fused kernel and its group of
 * rebuild kernels with hipEvents recorded on the pool's stream.  The launches
 * are issued back to back (no host synchronisation between steps; per-step
 * rebuild counters are copied to pinned host memory on the stream), so the
 * kernels run as they do in md_step.  n_steps in [1, 65536].  out[5]:
 * [0] mean fused-kernel ms, [1] mean rebuild-group ms over all steps,
 * [2] mean rebuild-group ms over steps in which a replica rebuilt,
 * [3] number of such steps, [4] total GPU ms of the n_steps.  Synchronises.
 * Allocates pinned host memory for the duration of the call. */
md_status md_profile_steps(md_system *sys, int64_t n_steps, double *out);

/* Block until all work on the pool's stream has finished. */
md_status md_sync(md_system *sys);

/* ---- state access ---------------------------------------------------------- */

/* Copy a replica's state to the host in particle-id order: positions folded
 * into [0, box) (FP64; double-single as hi + lo, the value Sec. 2.4 defines),
 * velocities, and the image counters such that pos + image * box is the
 * unwrapped trajectory.  pos, vel and image are host arrays of [n][3]
 * (caller-owned); any pointer may be NULL.  Synchronises.  Errors:
 * MD_E_NOSLOT, MD_E_HIP, MD_E_STATE (corrupt particle ids). */
md_status md_get_state(md_system *sys, int32_t slot, double *pos, double *vel,
                       int32_t *image);

/* Size in bytes of a bit-exact checkpoint of a slot (> 0), or < 0 on error. */
int64_t md_checkpoint_bytes(md_system *sys, int32_t slot);

/* Write a bit-exact checkpoint of a slot (state words incl. double-single lo
 * words, particle order, list reference positions, image counters, step and
 * phase) into a host buffer of md_checkpoint_bytes() bytes.  Synchronises. */
md_status md_save(md_system *sys, int32_t slot, void *blob, int64_t bytes);

/* Attach a checkpoint to an empty slot of a pool with the same precision,
 * pair table, dt and skin.  The continued trajectory is bitwise identical to
 * the uninterrupted one.  Synchronises. */
md_status md_restore(md_system *sys, int32_t slot, const void *blob, int64_t bytes);

/* Neighbour lists of a replica in particle-id order (tests): counts[n] and
 * ids[n][cap] (unused entries -1).  Synchronises. */
md_status md_debug_neighbours(md_system *sys, int32_t slot, int32_t *counts,
                              int32_t *ids, int32_t cap);

/* ---- launch shapes ----------------------------------------------------------- */

md_status md_get_launch(const md_system *sys, md_launch *out);
/* Changes take effect for later launches; captured graphs are dropped. */
md_status md_set_launch(md_system *sys, const md_launch *in);

/* ---- time-correlation functions (Sec. 2.5, blocking scheme) -------------------- */

typedef struct md_tcf md_tcf;

/* Bytes of device workspace of a blocking scheme of `levels` blocks of
 * `block` entries for a replica of n particles, or MD_E_ARG (levels in
 * [1, 16], block in [2, 33]).  Host only. */
int64_t md_tcf_workspace_bytes(int32_t n, int32_t levels, int32_t block);

/* Bind a blocking scheme (Sec. 2.5) to the replica attached at `slot`:
 * samples fill `levels` blocks of `block` entries, block n holding every
 * block^n-th sample; a full block correlates its oldest entry with the
 * others (time lags j block^n samples, j = 1 .. block-1) and drops it.  Per
 * species it accumulates the tagged-particle means of the mean-square
 * displacement (unwrapped positions), the velocity autocorrelation and the
 * self-intermediate scattering function F_s(q, t) = <cos(q dx)>, averaged
 * over the three box axes at wave number q (> 0).  The workspace (device,
 * 256-byte aligned, md_tcf_workspace_bytes) is caller-owned and must stay
 * valid until md_tcf_destroy; the replica must stay attached.  Errors:
 * MD_E_NOSLOT, MD_E_ARG, MD_E_WORKSPACE, MD_E_HIP. */
md_status md_tcf_create(md_system *sys, int32_t slot, int32_t levels, int32_t block, double q,
                        void *workspace, int64_t ws_bytes, md_tcf **out);

/* Record the replica's current state as the next sample.  The replica must
 * be at a full step (as after md_step, or once md_advance reached its
 * target).  Asynchronous on the pool's stream. */
md_status md_tcf_sample(md_tcf *tcf);

/* Synchronise and read, for k = level * (block - 1) + (j - 1):
 * lags[k] = j block^level (in samples), terms[k] = correlation passes so
 * far, values[6k .. 6k+5] = (MSD, VACF, F_s) of species A then B, each the
 * mean over passes of the species mean (NaN before the first pass).  Any
 * output may be NULL. */
md_status md_tcf_read(md_tcf *tcf, int64_t *lags, double *values, int64_t *terms);

/* Release the host handle (the workspace belongs to the caller). */
void md_tcf_destroy(md_tcf *tcf);

/* ---- double-single arithmetic self-test (Sec. 2.4, Alg. 1) -------------------- */

/* Element-wise double-single operation on device arrays of n (hi, lo) float
 * pairs, on the given stream: op 0 = add (Alg. 1), 1 = subtract,
 * 2 = multiply (exact FMA product of the high words plus cross terms),
 * 3 = compensated sum of a[k].hi over k (out[0] only; Sum2-style error-free
 * accumulation as used for the force sum).  Asynchronous. */
md_status md_ds_eval(int32_t op, int64_t n, const float *a, const float *b, float *out,
                     void *hip_stream);

/* ---- errors --------------------------------------------------------------------- */

const char *md_strerror(md_status st);
/* Last error text of a handle ("" if none); valid until the next call. */
const char *md_last_error(const md_system *sys);
int32_t md_abi_version(void);

/* Host-only: rank[c] (c = x + nd (y + nd z), nd^3 entries, caller-owned) of
 * every cell of an nd^3 grid in the cell order `order` (md_cell_order_kind),
 * the table the library uses for replicas with nd cells per edge.  Touches
 * no device.  Errors: MD_E_ARG (nd outside 1..1024, bad order, null rank). */
md_status md_cell_order(int32_t nd, int32_t order, int32_t *rank);

#ifdef __cplusplus
}
#endif
#endif /* MDX_MD_H */
