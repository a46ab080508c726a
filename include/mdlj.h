/*
 * mdlj.h -- C ABI of libmdlj: short-range Lennard-Jones 12-6 forces on one
 * MI355X (gfx950) over linked cells, Verlet lists and Verlet cluster lists,
 * with a runtime choice of the particle interaction order.
 *
 * Method: "Tuning of Vectorization Parameters for Molecular Dynamics
 * Simulations in AutoPas" (arXiv 2512.03565).
 *   - pair force sum F_i = sum_j F_ij over pairs inside the cutoff, with
 *     F_ij = -F_ji (section 2.1, Eq. 1 and the cutoff/Newton-3 paragraphs);
 *   - neighbour identification by linked cells, Verlet lists with a skin and
 *     Verlet cluster lists (section 2.1.1);
 *   - containers own particles and neighbour structures, a traversal hands
 *     two particle lists to the force functor (section 2.3, Fig. "flow");
 *   - interaction orders 1/VL, VL/1, 2/(VL/2), (VL/2)/2 (section 4.1,
 *     Fig. "vec_patterns") -- here: wave-per-i, i-per-lane, cluster tiles;
 *   - full-search auto-tuning over the Cartesian product of options,
 *     several samples per configuration reduced to one value
 *     (section 2.3.2), extended by the interaction order (section 4);
 *   - a data-driven tuner, the paper's future-work item (section 6).
 * The 12-6 law (which the paper names but does not print) is
 *   u(r) = 4 eps [(sig/r)^12 - (sig/r)^6] - shift,
 *   F_ij = 24 eps s6 (2 s6 - 1) / r^2 * (x_i - x_j),  s6 = (sig/r)^6,
 * force truncated at rc (a pair interacts iff r^2 < rc^2), energy shifted
 * by default so u(rc) = 0, Lorentz-Berthelot mixing of species.
 *
 * Conventions for every entry point:
 *   - Every call returns an mdlj_status; nothing aborts or exits.  On error
 *     mdlj_last_error(ctx) holds a message (valid until the next call on ctx).
 *   - Pointers are borrowed for the duration of the call only.  mem_kind says
 *     whether they are host (MDLJ_MEM_HOST) or device (MDLJ_MEM_DEVICE)
 *     memory; the library copies what it needs into memory it owns.
 *   - Per-particle arrays are indexed in the caller's order: outputs are
 *     written back in the order the particles were given to mdlj_create.
 *   - All device work is enqueued on the stream given to mdlj_create.  Calls
 *     that return host scalars (epot, virial, counts, tuning results)
 *     synchronise that stream before returning.
 *   - One context per host thread; a context must not be used by two threads
 *     at once.  Contexts are independent.
 */
#ifndef MDLJ_H
#define MDLJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mdlj_ctx mdlj_ctx;

typedef enum {
    MDLJ_OK = 0,
    MDLJ_ERR_ARG = -1,       /* a NULL pointer, a size or an enum out of range */
    MDLJ_ERR_STATE = -2,     /* box, cutoff or species not set yet */
    MDLJ_ERR_HIP = -3,       /* a HIP runtime call failed (message in last_error) */
    MDLJ_ERR_NOMEM = -4,     /* device allocation failed */
    MDLJ_ERR_OVERFLOW = -5,  /* a neighbour structure exceeded its capacity and
                                growth is disabled */
    MDLJ_ERR_NONFINITE = -6, /* a position is NaN or infinite */
    MDLJ_ERR_GEOMETRY = -7,  /* box edge < 2 x interaction range, or fewer than
                                3 linked cells along an axis */
    MDLJ_ERR_NOTFOUND = -8   /* file or symbol missing (network weights) */
} mdlj_status;

enum { MDLJ_MEM_HOST = 0, MDLJ_MEM_DEVICE = 1 };

/* Neighbour identification algorithm (section 2.1.1). */
enum { MDLJ_NBR_LC = 0, MDLJ_NBR_VL = 1, MDLJ_NBR_VCL = 2 };

/* Particle interaction order (section 4.1).  I_PER_LANE is VectorLength/1
 * (distinct i per lane, one j broadcast to all lanes); CLUSTER_TILE covers
 * the split patterns 2/(VL/2) and (VL/2)/2 as a tile_i x tile_j lane grid;
 * WAVE_PER_I is 1/VectorLength (j across lanes, reduction over lanes). */
enum { MDLJ_ORD_I_PER_LANE = 0, MDLJ_ORD_CLUSTER_TILE = 1, MDLJ_ORD_WAVE_PER_I = 2 };

/* Arithmetic: FP32 pair arithmetic with FP64 accumulation, or all FP64. */
enum { MDLJ_PREC_F32PAIR_F64ACC = 0, MDLJ_PREC_F64 = 1 };

/* What the tuner minimises: time per MD step, or energy per MD step
 * (section 2.3.3; read from the GPU's energy counter). */
enum { MDLJ_METRIC_TIME = 0, MDLJ_METRIC_ENERGY = 1 };

/* Tuning strategy (section 2.3.2 full search; section 6 data-driven and
 * cheaper searches). */
enum { MDLJ_TUNE_FIXED = 0, MDLJ_TUNE_EXHAUSTIVE = 1, MDLJ_TUNE_LEARNED = 2,
       MDLJ_TUNE_EARLY_STOP = 3 };

/*
 * One point of the search space.  Meaning of tile_i / tile_j per order:
 *   I_PER_LANE   LC: tile_i = linked cells per i-tile along x (1, 2, 4);
 *                VL/VCL: unused (0).
 *   CLUSTER_TILE tile_i x tile_j = 64 lanes of one wavefront, tile_i i's and
 *                tile_j j's per step (LC: 16x4, 8x8; VCL: cluster_size x
 *                64/cluster_size), or for VCL also cluster_size x 4 lanes
 *                per cluster pair with 64/(4 cluster_size) cluster pairs
 *                (each its own cluster I) per wavefront: 4x4 x 4 pairs for
 *                cluster size 4, 8x4 x 2 pairs for cluster size 8 (the
 *                4 j-lanes then take half of a j-cluster per step).
 *   WAVE_PER_I   tile_i = g, the i-particles per wavefront (LC: 1, 2, 4;
 *                VL: 1, 2, 4, 8, 16); each gets 64/g lanes.  tile_j = 64/g,
 *                except for staged VL, where tile_j = v, the list entries
 *                each lane reads per trip (2, 4 or 8: one 4-, 8- or 16-byte
 *                load); staged VL takes (g, v) in {(8,2), (8,4), (16,2),
 *                (16,4), (4,8)}.
 * cluster_size is 4 or 8 for VCL, 0 otherwise.  newton3 = 1 computes each
 * pair once and applies F_ji = -F_ij with atomics (section 4.1.3).
 * staged = 1 (full lists only): the particles a workgroup's i's can reach
 * are first copied into LDS with coalesced loads and j-particles are then
 * read from LDS.  LC cluster-tile / wave-per-i: a workgroup owns one cell
 * and stages its 27-cell neighbourhood.  VL wave-per-i: a workgroup owns 4
 * consecutive cells along x and stages the 9 rows of 6 cells around them;
 * the Verlet list then holds 16-bit indices into that staged set; with
 * FP32 pair arithmetic its records are kept as 32-bit fixed-point words of
 * one frame centred on the box (12 bytes, the species apart, in global
 * memory and in LDS; separations exact to within the grid 1/s, 5.8e-8
 * sigma for a box of 175 sigma), with all-FP64 as FP64 (24 bytes).  A scene
 * whose neighbourhoods do not fit the 64 KB staging budget rejects staged
 * configurations with MDLJ_ERR_ARG, and so does a box whose fixed-point
 * step would exceed 1e-7 of the smallest sigma (beyond about 310 sigma)
 * for the FP32-pair staged ones.  staged = 0 reads
 * every j-particle from global memory.
 * Linked cells with newton3 = 1 (staged = 1): a wavefront per cell pairs
 * its own particles with those of its 13 forward neighbour cells (a half
 * shell) and with each other, every pair once; both forces are added in LDS
 * and flushed with one atomic per staged record.  swap chooses which side
 * of those cell pairs is the i-list (the traversal's choice, section 5):
 * swap = 0, the cell's own particles (WAVE_PER_I 1x64, CLUSTER_TILE 4x16 or
 * 16x4: tile_i i's per step, tile_j lanes each over its partners); swap =
 * 1, the partners (I_PER_LANE, tile_i = 1: each lane one partner, the own
 * particles broadcast to all lanes).  VCL CLUSTER_TILE: swap = 0 runs the
 * lanes of a cluster pair over j fastest (the 2/(VL/2) fill widened), swap
 * = 1 over i fastest (the (VL/2)/2 fill), both cluster_size i's by tile_j
 * j's.  swap is 0 for every other configuration.
 */
typedef struct {
    int32_t nbr_algo;
    int32_t order;
    int32_t tile_i;
    int32_t tile_j;
    int32_t cluster_size;
    int32_t newton3;
    int32_t staged;
    int32_t swap;
} mdlj_config;

/*
 * A context is the container of section 2.3: it owns the particles and the
 * neighbour structure built over them; positions are handed over as
 * separate x, y, z arrays (structure of arrays, the layout section 2.3.1
 * prefers for vector loads).
 * Create a context holding n particles (n >= 1) of n_species species
 * (1..8).  x, y, z: positions (float64, length n); type: species index per
 * particle (int32 in [0, n_species), or NULL for all zero).  mem_kind says
 * where the arrays live.  hip_stream: a hipStream_t (NULL = default stream)
 * on which all work of this context is enqueued.  On success *out owns all
 * device memory of the context.  Defaults: energy shift on, FP32 pair
 * arithmetic, rebuild every 10 steps, skin 0, config LC / I_PER_LANE / 1.
 */
mdlj_status mdlj_create(mdlj_ctx **out, int64_t n, const double *x, const double *y,
                        const double *z, const int32_t *type, int32_t n_species,
                        int32_t mem_kind, void *hip_stream);

/* Free the context and all its device memory.  NULL is accepted. */
mdlj_status mdlj_destroy(mdlj_ctx *ctx);

/* Orthorhombic periodic box [0,lx) x [0,ly) x [0,lz); edges > 0. */
mdlj_status mdlj_set_box(mdlj_ctx *ctx, double lx, double ly, double lz);

/* Cutoff radius rc > 0 (section 2.1): pairs interact iff r^2 < rc^2. */
mdlj_status mdlj_set_cutoff(mdlj_ctx *ctx, double rc);

/* Verlet skin >= 0 and the rebuild interval (>= 1 force evaluations) of the
 * Verlet and cluster lists (section 2.1.1).  Lists hold pairs within rc+skin
 * and are also rebuilt early once any particle has moved more than skin/2. */
mdlj_status mdlj_set_skin(mdlj_ctx *ctx, double skin, int32_t rebuild_every);

/* Pruned inner list of the staged Verlet-list kernels: on (1) or off (0,
 * default).  The Verlet lists of section 2.1.1 hold the pairs within
 * rc + skin; the list build also keeps, per particle and in list order, the
 * entries closer than rc + 2 skin / 3, and force evaluations read that
 * shorter list while no particle has moved more than skin / 3 since the
 * build (the skin/2 argument with the smaller skin), then the full one until
 * the next build.  Forces agree with the unpruned ones up to the order of
 * the FP64 sums.  Only tiled builds of the staged kernels' lists write it.
 * Changing the setting marks the lists for rebuilding.
 * Validity is kept per tile (four cells along x, the staged kernels' unit
 * of work): a tile falls back to the full list once a particle in it or in
 * one of the 26 tiles around it has crossed the bound.
 * mdlj_pruning_state (synchronises the stream): 0 no inner list for the
 * current lists, 1 valid in every tile, 2 given up in some tiles, 3 given up
 * in every tile; the count of tiles that gave it up into *tiles_out when not
 * null. */
mdlj_status mdlj_set_pruning(mdlj_ctx *ctx, int32_t on);
mdlj_status mdlj_pruning_state(mdlj_ctx *ctx, int32_t *state, int64_t *tiles_out);

/* Parameters of species s for the Lennard-Jones 12-6 pair law (section 4.1
 * names the potential, section 2.1 Eq. 1 sums it over pairs): epsilon > 0,
 * sigma > 0.  Unlike species mix by the Lorentz-Berthelot rule (the paper
 * gives no rule).  Every species must be set before forces are computed. */
mdlj_status mdlj_set_species(mdlj_ctx *ctx, int32_t s, double epsilon, double sigma);

/* Energy shift so that u(rc) = 0: on (1, default) or off (0).  Forces are
 * never shifted. */
mdlj_status mdlj_set_energy_shift(mdlj_ctx *ctx, int32_t on);

/* MDLJ_PREC_F32PAIR_F64ACC (default) or MDLJ_PREC_F64. */
mdlj_status mdlj_set_precision(mdlj_ctx *ctx, int32_t prec);

/* Replace all positions (caller order, float64, length n).  Non-finite
 * values give MDLJ_ERR_NONFINITE (checked on the device for device input;
 * the check synchronises the stream). */
mdlj_status mdlj_set_positions(mdlj_ctx *ctx, const double *x, const double *y,
                               const double *z, int32_t mem_kind);

/* Copy current positions (wrapped into the box, caller order) out. */
mdlj_status mdlj_get_positions(mdlj_ctx *ctx, double *x, double *y, double *z,
                               int32_t mem_kind);

/* Select the configuration used by compute_forces.  An invalid combination
 * gives MDLJ_ERR_ARG and leaves the current one in place. */
mdlj_status mdlj_set_config(mdlj_ctx *ctx, const mdlj_config *cfg);
mdlj_status mdlj_get_config(const mdlj_ctx *ctx, mdlj_config *cfg);

/* Number of valid configurations (the tuner's search space) and the k-th. */
mdlj_status mdlj_config_count(const mdlj_ctx *ctx, int32_t *count);
mdlj_status mdlj_config_at(const mdlj_ctx *ctx, int32_t k, mdlj_config *cfg);

/* Rebuild the neighbour structure of the current configuration now
 * (binning, Verlet or cluster lists).  compute_forces does this itself when
 * needed. */
mdlj_status mdlj_rebuild_neighbors(mdlj_ctx *ctx);

/*
 * The force on every particle as the sum of its pair forces inside the
 * cutoff (section 2.1, Eq. 1), computed with the current configuration.
 * Forces on every particle (caller order) into fx, fy, fz (float64, length
 * n; mem_kind says where).  epot (total potential energy U = sum over pairs
 * of u) and virial (W = sum over pairs of r_ij . F_ij) are host float64
 * pointers and may be NULL; when either is given the call synchronises.
 * Rebuilds the neighbour structure first when it is due.
 */
mdlj_status mdlj_compute_forces(mdlj_ctx *ctx, double *fx, double *fy, double *fz,
                                int32_t mem_kind, double *epot, double *virial);

/*
 * mdlj_compute_forces for callers that cannot allocate memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * fx, fy, fz: device float64 arrays (length n, caller order); epot and
 * virial as for mdlj_compute_forces (host, may be NULL; given, the call
 * synchronises).  The call computes exactly what mdlj_compute_forces
 * computes, with the same kernels, but allocates nothing: the force
 * kernels' per-workgroup energy/virial partials go to a static device array
 * of 2^22 doubles (32 MiB, one per GPU, held until the process ends), and
 * every other buffer is the context's own.  When the call would have to
 * create or grow one of those (the first force call of a context, a rebuild
 * that needs more list, record or cell memory than earlier calls sized, a
 * timing event) it returns MDLJ_ERR_NOMEM and allocates nothing; one
 * mdlj_compute_forces call sizes the context, after which the neighbour
 * structure is rebuilt on the next call.  A configuration whose energy
 * partials exceed the scratch array (contexts beyond about two million
 * particles) gives MDLJ_ERR_ARG.  Every call on one GPU uses that GPU's
 * array, and each launch writes all the partials it reads, so nothing has
 * to be cleared between calls; calls that overlap on one GPU (two streams
 * or threads at once) race on the array.
 */
mdlj_status mdlj_compute_forces_noalloc(mdlj_ctx *ctx, double *fx, double *fy, double *fz,
                                        double *epot, double *virial);

/* Number of unordered pairs with r < rc (the pairs inside the cutoff of
 * section 2.1 that contribute to Eq. 1: the useful pairs), counted on the
 * device from the current positions (by a linked-cell binning at rc, which
 * replaces the current neighbour structure).  Synchronises. */
mdlj_status mdlj_count_pairs(mdlj_ctx *ctx, int64_t *n_useful_pairs);

/*
 * Size of the current neighbour structure (section 2.1.1), for traffic
 * accounting: *list_entries = stored Verlet-list entries including the
 * padding of each row to a multiple of 8 (0 unless the structure is a
 * Verlet list), *entry_bytes = bytes per entry (2 for the 16-bit lists of
 * staged configurations, 4 otherwise, 0 without lists), *records = sorted
 * records including halo images (0 before the first build).  Host
 * pointers, all required.  Synchronises.  MDLJ_ERR_STATE before the first
 * force call.
 */
mdlj_status mdlj_neighbor_stats(mdlj_ctx *ctx, int64_t *list_entries, int32_t *entry_bytes,
                                int64_t *records);

/*
 * Which pair each lane computes in one step of an interaction order
 * (section 4.1.1, the register fills of Fig. "vec_patterns"), as offsets
 * (*i, *j) from the step's first i and first j.  Pure host functions.
 *   lane_map: a vector of `width` lanes holding ai i's (ai divides width).
 *     layout 0 (j fastest): lane -> (lane / (width/ai), lane % (width/ai));
 *     ai = 1 is 1/VectorLength, ai = 2 is 2/VectorLengthDiv2.
 *     layout 1 (i fastest): lane -> (lane % ai, lane / ai); ai = width is
 *     VectorLength/1, ai = width/2 is VectorLengthDiv2/2.
 *   config_lane_map: the map the kernel of configuration *cfg uses on its
 *     64-lane wavefronts (*layout receives 0 or 1): i-per-lane orders take
 *     layout 1 with 64 i's; wave-per-i and the linked-cell tiles layout 0
 *     with tile_i i's; the VCL cluster tiles layout swap with cluster_size
 *     i's, and with several cluster pairs per wavefront the lanes in groups
 *     of tile_i x tile_j, group q mapped like one pair's lanes with i and j
 *     offset by q tile_i and q tile_j.  The kernels take their lane offsets
 *     from the same function.
 */
mdlj_status mdlj_lane_map(int32_t layout, int32_t ai, int32_t width, int32_t lane, int32_t *i,
                          int32_t *j);
mdlj_status mdlj_config_lane_map(const mdlj_config *cfg, int32_t lane, int32_t *layout,
                                 int32_t *i, int32_t *j);

/*
 * Index views of the neighbour structure, for checking it against a plain
 * neighbour search (section 2.1.1).  Host arrays; both calls synchronise
 * the stream.
 *   get_cells   the linked cell of every particle in the last binning
 *               (caller order), numbered cx + nx (cy + ny cz) over the
 *               nx x ny x nz cells of the box (ncell3 = {nx, ny, nz}):
 *               n = floor(L / r) cells of edge L / n >= r per axis (r = rc
 *               for linked cells, rc + skin for Verlet lists; for cluster
 *               lists the xy columns and z slabs), c = (int)(x_w n / L)
 *               clamped to n - 1, x_w = x - L floor(x / L), each operation
 *               rounded on its own.  MDLJ_ERR_STATE before the first
 *               binning.  cell has length n.
 *   get_pairs   the particle pairs the current list hands to the force
 *               kernels, as caller indices (pi[k], pj[k]).  Verlet lists:
 *               one pair per stored entry (full lists hold each pair in
 *               both directions, Newton-3 lists once, with pi < pj).
 *               Cluster lists: every pair of real particles (i in I, j in
 *               J) of every stored cluster pair, a particle with itself
 *               under the zero image shift left out.  *count receives the
 *               number of pairs; with pi and pj NULL nothing else is done,
 *               otherwise up to cap pairs are written and MDLJ_ERR_OVERFLOW
 *               is returned when *count > cap.  An entry that names no
 *               record gives pj = -2.  MDLJ_ERR_STATE for linked cells or
 *               before a list was built.  Allocates temporary device
 *               memory.
 */
mdlj_status mdlj_get_cells(mdlj_ctx *ctx, int32_t *cell, int32_t *ncell3);
mdlj_status mdlj_get_pairs(mdlj_ctx *ctx, int64_t cap, int32_t *pi, int32_t *pj,
                           int64_t *count);

/*
 * Choose a configuration by the cost of one MD step as mdlj_step_vv runs it
 * (force kernel, integrator step, list upkeep, and a rebuild every
 * rebuild_every steps or re-binning every step), measured on the current
 * positions with HIP events: one sample is a cycle of rebuild_every (at most
 * 50) velocity-Verlet steps with time step 0 from zero velocities, so the
 * positions keep their values bit for bit while every kernel does its usual
 * work; the first cycle (which also builds the structure) is a warm-up.
 * FIXED keeps the current configuration; EXHAUSTIVE (section 2.3.2's full
 * search) times every valid configuration `samples` cycles, drops the
 * first and averages the rest, the lower index winning ties; LEARNED asks
 * the network and falls back to EXHAUSTIVE when its confidence is below the
 * threshold set by mdlj_mlp_set_threshold (default 0.6) or no network is
 * loaded (a network of K classes chooses among the first K configurations
 * of config_at order; its fallback searches them all); EARLY_STOP is the full search with early stopping (the decision
 * rule of mdlj_tune_select_early with warm_factor +inf, i.e. the warm-up
 * cycle is not scored, and margin 0.1), the
 * configurations visited by descending network probability when a network
 * is loaded (configurations beyond its K classes last, in config_at order),
 * else in config_at order.  The chosen
 * configuration is made current; *chosen and *step_us (microseconds per MD
 * step of the chosen one, may be NULL) are written.  The context's kernel
 * timing (mdlj_set_timing) does not count the tuning steps.
 */
mdlj_status mdlj_tune(mdlj_ctx *ctx, int32_t mode, int32_t samples, mdlj_config *chosen,
                      double *step_us);

/* Per-configuration results of the last EXHAUSTIVE or EARLY_STOP search:
 * up to cap entries of microseconds per step in config_at order (+inf where
 * a configuration cannot run; for a configuration EARLY_STOP dropped, its
 * last sample); *count = number of configurations.  mdlj_tune_taken: the
 * samples each configuration used. */
mdlj_status mdlj_tune_results(const mdlj_ctx *ctx, double *us, int32_t cap, int32_t *count);
mdlj_status mdlj_tune_taken(const mdlj_ctx *ctx, int32_t *taken, int32_t cap, int32_t *count);

/*
 * Energy as the tuning metric (section 2.3.3).  set_tune_metric: TIME
 * (default) or ENERGY for the following mdlj_tune calls.  Under ENERGY a
 * configuration's value is microjoules per MD step: its steps run (as for
 * the time metric, time step 0) while the GPU's energy counter, which the
 * firmware refreshes about once a second, is read between runs of at least
 * 5 ms; `samples` is then the number of refresh intervals the measured
 * window spans (>= 1, so about `samples` seconds per configuration), and
 * the value is the mean power over that window times the mean step time
 * of the steps run in it.  FIXED and EXHAUSTIVE measure by energy; LEARNED
 * falls back to EXHAUSTIVE (the network predicts the fastest
 * configuration); EARLY_STOP gives MDLJ_ERR_ARG.  mdlj_tune_results then
 * reports microjoules per step and mdlj_tune_power the mean watts of each
 * configuration (NaN under TIME).  The counter is read through AMD SMI
 * (libamd_smi, loaded on first use): MDLJ_ERR_NOTFOUND without it, and
 * MDLJ_ERR_STATE when the counter is not refreshed.
 * mdlj_gpu_energy: the counter now, in joules, and the time of its last
 * refresh in seconds (the firmware's clock).
 * mdlj_tune_select_energy (pure host function): energy per step
 * us[q] * watts[q] (microjoules; +inf where either is not a positive
 * number) into uj[q] and the smallest, lower index on ties (-1 if none):
 * a configuration that runs faster but draws more power can lose.
 */
mdlj_status mdlj_set_tune_metric(mdlj_ctx *ctx, int32_t metric);
mdlj_status mdlj_tune_power(const mdlj_ctx *ctx, double *watts, int32_t cap, int32_t *count);
mdlj_status mdlj_gpu_energy(mdlj_ctx *ctx, double *joules, double *seconds);
mdlj_status mdlj_tune_select_energy(const double *us, const double *watts, int32_t k, double *uj,
                                    int32_t *chosen);

/*
 * Decision rules of the tuner, as pure host functions (no context, no
 * device work), usable by drivers that time configurations themselves.
 *   tune_select: samples is row-major [k][s] (microseconds; +inf or NaN for
 *     a configuration that cannot run).  mode 0 reduces each row to its mean
 *     with the first sample dropped as warm-up (all samples when s == 1),
 *     mode 1 to its minimum (section 2.3.2 allows either).  values[k]
 *     receives the reduced values; *chosen the index of the smallest finite
 *     one, the lower index on ties, or -1 if none is finite.
 *   retune_needed: *needed = 1 when the density (feature 1) or the
 *     cell-occupancy spread (feature 5) of mdlj_features changed by more
 *     than `threshold` relative to `before8` (the optimum moves with the
 *     particle distribution, section 5).
 */
mdlj_status mdlj_tune_select(const double *samples, int32_t k, int32_t s, int32_t mode,
                             double *values, int32_t *chosen);
/*
 * The early-stopping search as a pure host function over a table of
 * samples [k][s] (row-major, microseconds; sample 0 is the warm-up cycle;
 * +inf or NaN where a configuration cannot run), visiting configurations
 * in `order` (a permutation of 0..k-1, or NULL for index order).  Once a
 * configuration has been fully measured, a later one is dropped when its
 * warm-up sample exceeds warm_factor (>= 1, +inf allowed) times the best mean so far or
 * its first timed sample exceeds (1 + margin) times it (margin >= 0).
 * values[q] = mean of samples 1..s-1 of a fully measured configuration (all
 * s when s == 1), else its last sample taken (+inf if it cannot run);
 * taken[q] = samples used; *chosen = the smallest fully measured mean,
 * lower index on ties, or -1.
 */
mdlj_status mdlj_tune_select_early(const double *samples, int32_t k, int32_t s,
                                   const int32_t *order, double warm_factor, double margin,
                                   double *values, int32_t *taken, int32_t *chosen);
mdlj_status mdlj_retune_needed(const float *before8, const float *now8, double threshold,
                               int32_t *needed);

/*
 * nsteps velocity-Verlet steps (mass per species, default 1; time step dt):
 * v += F dt/2m; x += v dt; wrap; F = F(x); v += F dt/2m.  vx, vy, vz are
 * device float64 arrays in caller order, updated in place.  The forces of
 * the current positions must have been computed once before (they are kept
 * in the context).  With Verlet lists the steps keep positions and
 * velocities in the context in sorted order (the velocities also across
 * list rebuilds); the caller's arrays and the context's positions are
 * brought up to date before the call returns (also when it returns an
 * error).  With a staged Verlet-list configuration the force kernel takes
 * the integrator step between rebuilds itself; the trajectory is the same,
 * bit for bit, and the time of those force calls (mdlj_get_timing)
 * includes it.
 */
mdlj_status mdlj_step_vv(mdlj_ctx *ctx, double *vx, double *vy, double *vz, double dt,
                         int32_t nsteps);
mdlj_status mdlj_set_mass(mdlj_ctx *ctx, int32_t s, double mass);

/* Kernel timing with HIP events on the context's stream.  on = 1 enables
 * and resets the totals.  Events (timing only: no system-scope fence) are
 * recorded around the force kernel of every force evaluation and, when it
 * rebuilds, from the start of the rebuild; they are read when get_timing is
 * called (which synchronises the stream) or recycled once they are 64
 * evaluations old.  get_timing returns
 * the summed force-kernel and rebuild (binning + list build, or the
 * per-step re-binning of linked cells) microseconds and how many of each
 * were timed.  Outputs may be NULL. */
mdlj_status mdlj_set_timing(mdlj_ctx *ctx, int32_t on);
mdlj_status mdlj_get_timing(mdlj_ctx *ctx, double *force_us, double *build_us,
                            int64_t *n_force, int64_t *n_build);
/* Of the timed force kernels, those that took the velocity-Verlet step too
 * (staged Verlet lists inside mdlj_step_vv): summed microseconds and count
 * since mdlj_set_timing.  Synchronises the stream like mdlj_get_timing.
 * Outputs may be NULL; MDLJ_ERR_ARG for a NULL context. */
mdlj_status mdlj_get_timing_fused(mdlj_ctx *ctx, double *fused_us, int64_t *n_fused);

/* Eight scene features the learned tuner reads (log10 N, density,
 * rc / sigma_max, species count, expected neighbours within rc, cell
 * occupancy coefficient of variation, empty-cell fraction, max/mean cell
 * occupancy), computed on the device from the current positions. */
mdlj_status mdlj_features(mdlj_ctx *ctx, float *features8);

/*
 * Learned tuner (data-driven tuning, section 6): a network 8 -> 64 -> 64 ->
 * K (ReLU, softmax over the first K configurations of config_at order: a
 * network trained before configurations were added to the end of the
 * search space keeps choosing among those it knows), FP32,
 * trained and evaluated on the device by the library's own kernels.
 * Parameters are one flat float array W1[64][8] b1[64] W2[64][64] b2[64]
 * W3[K][64] b3[K] (row-major [out][in]); inputs are z-scored with a stored
 * mean and deviation per feature (set_norm; init sets 0 and 1).
 *   init        He-normal weights from `seed`, zero biases, K classes (1..256).
 *   set_norm    per-feature mean and standard deviation (> 0), 8 each.
 *   get/set_params  copy the flat parameter array (count must match K).
 *   predict     softmax probabilities [n][K] for n raw feature rows (host).
 *   loss_grad   mean cross-entropy over n rows (used as network input as
 *               given, no z-scoring) and its gradient [n_params] (host).
 *   train       `epochs` passes of Adam (lr, beta 0.9/0.999, eps 1e-8) over
 *               full minibatches of `batch` rows in a seeded shuffled order;
 *               rows are raw features, z-scored with the stored values;
 *               *final_loss = mean loss of the last epoch.
 *   load/save   file "MDLJMLP1", int32 K, 8, 64, 64, float mean[8], std[8],
 *               params (little-endian); MDLJ_ERR_NOTFOUND if unreadable.
 *   set_threshold  confidence (largest probability) below which LEARNED
 *               tuning falls back to full search; default 0.6.
 *   stats       confidence of the last LEARNED decision and the number of
 *               fallbacks so far.
 * All feature/label/probability arrays are host memory.
 */
mdlj_status mdlj_mlp_init(mdlj_ctx *ctx, int32_t k, uint64_t seed);
mdlj_status mdlj_mlp_set_norm(mdlj_ctx *ctx, const float *mean8, const float *std8);
mdlj_status mdlj_mlp_get_params(const mdlj_ctx *ctx, float *w, int64_t cap, int64_t *count,
                                int32_t *k);
mdlj_status mdlj_mlp_set_params(mdlj_ctx *ctx, const float *w, int64_t count, int32_t k);
mdlj_status mdlj_mlp_predict(mdlj_ctx *ctx, const float *x, int32_t n, float *probs);
mdlj_status mdlj_mlp_loss_grad(mdlj_ctx *ctx, const float *x, const int32_t *labels, int32_t n,
                               float *grad, float *loss);
mdlj_status mdlj_mlp_train(mdlj_ctx *ctx, const float *x, const int32_t *labels, int32_t n,
                           int32_t epochs, int32_t batch, double lr, uint64_t seed,
                           double *final_loss);
mdlj_status mdlj_mlp_load(mdlj_ctx *ctx, const char *path);
mdlj_status mdlj_mlp_save(const mdlj_ctx *ctx, const char *path);
mdlj_status mdlj_mlp_set_threshold(mdlj_ctx *ctx, double threshold);
mdlj_status mdlj_mlp_stats(const mdlj_ctx *ctx, double *last_confidence, int64_t *fallbacks);

/* Human-readable message of the last failing call on ctx ("" if none). */
const char *mdlj_last_error(const mdlj_ctx *ctx);

/* Library version string. */
const char *mdlj_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MDLJ_H */
