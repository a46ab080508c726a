// internal.h -- shared declarations of libmdlj (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <deque>
#include <string>
#include <vector>

#include "mdlj.h"

#define MDLJ_MAX_SPECIES 8
#define MDLJ_WAVE 64

// Sorted particle record: FP64 position, species and the caller index of
// the particle (for a halo image: of the particle it copies).  32 bytes, so
// a j-load is two 16-byte loads.
struct __attribute__((aligned(32))) PosT {
    double x, y, z;
    int32_t t;
    int32_t orig;
};

// Uniform grid over the box plus h halo layers per side.  Cell coordinate
// c in [-h, n + h) maps to the extended index sum_a (c_a + h_a) * stride_a.
// Halo cells hold periodic images of interior cells (shifted by +-L).
struct Grid {
    int n[3];
    int h[3];
    int e[3];
    double L[3];
    double inv[3];   // n / L, for the cell index
    double edge[3];  // L / n
    int64_t stride[3];
    int64_t ncell_ext;
    int64_t ncell_int;
};

// Pair-law table in the arithmetic type of the pair loop.  For pair type
// index k = ti * ns + tj: sig2 = sigma^2, eps24 = 24 eps, eps4 = 4 eps,
// shift = energy shift; rc2 = cutoff^2.
template <typename T>
struct LJTable {
    T sig2[MDLJ_MAX_SPECIES * MDLJ_MAX_SPECIES];
    T eps24[MDLJ_MAX_SPECIES * MDLJ_MAX_SPECIES];
    T eps4[MDLJ_MAX_SPECIES * MDLJ_MAX_SPECIES];
    T shift[MDLJ_MAX_SPECIES * MDLJ_MAX_SPECIES];
    T rc2;
    double rc2d;  // cutoff^2 in FP64: the in/out decision is taken on FP64 r^2
    int ns;
};

// Output of a force kernel in sorted order: FP64 forces per slot and, when
// energies are requested, one (U, W) pair per workgroup.
struct ForceOut {
    double *fx, *fy, *fz;
    double *partial;  // [2 * nblocks] or nullptr
};

// Fixed-point word of a coordinate for the FP32-pair staged kernel: the
// coordinate relative to the frame centre c times the scale s, rounded,
// plus 2^31.  Paired with the high word 0x43300000 a word is the binary64
// number 2^52 + word, so the difference of two words is their exact integer
// separation.  Particles occupy words within FX_RANGE of the centre (the
// scale is chosen so), which leaves at least 2^29 steps on every axis to
// the padding record at word 0; the clamp keeps the conversion defined, and
// that gap intact, for a particle that has run far off (the force call is
// then repeated after a rebuild).
#define FX_RANGE 1610612736.0  // 1.5 * 2^30
__device__ __forceinline__ unsigned to_fx(double v, double c, double s)
{
    const double q = fmin(fmax(rint((v - c) * s), -FX_RANGE), FX_RANGE);
    return (unsigned)(int)q ^ 0x80000000u;
}

// The fixed-point words of one record's x, y and z (12 bytes).
struct FxWords {
    unsigned x, y, z;
};

// The velocity-Verlet step fused into the staged Verlet-list force kernel.
// From the forces of x(t) the kernel finishes v(t) and starts the next step
// for its own particles (half kick, half kick, drift: the arithmetic of the
// separate sorted-order integrator kernel) and tests their displacement
// since the list build.  Records and velocities go to second buffers: other
// workgroups of the same launch still stage the old positions.
struct KickArgs {
    PosT *rec_out;          // records after the drift, same slots as the input
    const double *vs_in;    // velocities by compact index, (x, y, z) triples
    double *vs_out;
    const double *xrs;      // list-build reference positions by compact index, SoA
    int32_t *flag;          // set to 1 when a particle moved more than sqrt(thr2)
    double im[MDLJ_MAX_SPECIES];  // 1 / mass per species
    double dt, thr2;
    int64_t pad_slot;       // the padding record, copied to rec_out as it is
    // FP32-pair kernel: fixed-point words of the new positions (frame fx_c,
    // fx_s) to a second word array; null otherwise
    FxWords *fxr_out;
    double fx_c[3], fx_s;
    // the pruned inner list's squared displacement bound (InnerList)
    double thr_in2;
};

// Staged Verlet-list kernels: a tile is STAGE_K consecutive cells along x
// of one (y, z) cell row (tiles_x = ceil(n_x / STAGE_K) per row, numbered
// x-fastest); its workgroup stages the nine cell rows around it.
constexpr int STAGE_K = 4;

// The pruned inner Verlet list of the staged kernels, written by the list
// build: the entries of each row whose pair was closer than r_in at the
// build, in list order (same row layout and capacity as the list, rows
// padded to 8 with the padding entry).  A tile's inner rows hold every pair
// inside the cutoff while no particle of its staged neighbourhood has moved
// more than (r_in - rc) / 2 since the build.  One validity word per tile, in
// two copies that take turns: a launch reads one (cur) and anything that
// moves particles writes the other (next), so that no launch reads a word it
// also writes.  Both are cleared at the build and only ever set afterwards:
// a particle that crosses the bound sets the words of the 27 tiles around
// its own (every tile whose staged rows include its cell), and each mover
// carries the words already set over.  A tile reads the inner rows while its
// word is clear.
struct InnerList {
    const uint16_t *nbr;
    const int2 *lo;           // per row: length, start less t cap
    const int32_t *tile_cur;  // null: no inner list
    int32_t *tile_next;       // written by the fused integrator step
};

// What a kernel that moves particles outside the force kernel needs to
// keep the tile words: cur / next as above (null: no inner list), the
// extended cell of each caller index at the build (the cell its record is
// staged in), the grid and the bound.
struct InnerMark {
    const int32_t *cur;
    int32_t *next;
    const int32_t *cell_of;
    Grid g;
    int tiles_x;
    int64_t ntiles;
    double thr2;
};

// Set the words of the 27 tiles around tile (tx, ty, tz), periodically (the
// fused force kernel does the same with one thread per tile).
__device__ __forceinline__ void inner_mark_tiles(int32_t *next, int tx, int ty, int tz,
                                                 int tiles_x, const Grid &g)
{
    for (int k = 0; k < 27; ++k) {
        const int nx = (tx + k % 3 - 1 + tiles_x) % tiles_x;
        const int ny = (ty + (k / 3) % 3 - 1 + g.n[1]) % g.n[1];
        const int nz = (tz + k / 9 - 1 + g.n[2]) % g.n[2];
        int32_t *w = next + nx + (int64_t)tiles_x * (ny + (int64_t)g.n[1] * nz);
        if (*w == 0) atomicOr(w, 1);
    }
}

// Caller particle i moved d2 (squared) since the build: past the bound, the
// tiles around its record's tile give the inner list up.
__device__ __forceinline__ void inner_mark(const InnerMark &m, int64_t i, double d2)
{
    if (!m.next || d2 <= m.thr2) return;
    const int32_t e = m.cell_of[i];
    int c[3];
    for (int a = 0; a < 3; ++a) c[a] = (int)((e / m.g.stride[a]) % m.g.e[a]) - m.g.h[a];
    inner_mark_tiles(m.next, c[0] / STAGE_K, c[1], c[2], m.tiles_x, m.g);
}

// The words already set carried over to the next copy (grid-stride over
// the tiles; every thread of the launch takes part).
__device__ __forceinline__ void inner_carry(const InnerMark &m)
{
    if (!m.next) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m.ntiles; k += stride)
        if (m.cur[k]) atomicOr(m.next + k, 1);
}

// Device buffers that grow on demand.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct mdlj_ctx {
    hipStream_t stream = nullptr;
    int64_t n = 0;
    int nspec = 1;
    double eps[MDLJ_MAX_SPECIES] = {0};
    double sig[MDLJ_MAX_SPECIES] = {0};
    double mass[MDLJ_MAX_SPECIES] = {1, 1, 1, 1, 1, 1, 1, 1};
    bool species_set[MDLJ_MAX_SPECIES] = {false};
    double box[3] = {0, 0, 0};
    bool box_set = false;
    double rc = 0;
    double skin = 0;
    int rebuild_every = 10;
    int shift_on = 1;
    int prec = MDLJ_PREC_F32PAIR_F64ACC;
    mdlj_config cfg = {MDLJ_NBR_LC, MDLJ_ORD_I_PER_LANE, 1, 1, 0, 0, 0, 0};
    std::string err;

    // caller-order particle state (device)
    double *x = nullptr, *y = nullptr, *z = nullptr;  // wrapped positions
    int32_t *type = nullptr;
    double *fx = nullptr, *fy = nullptr, *fz = nullptr;  // last forces, caller order
    bool forces_valid = false;
    bool pos_changed = true;      // positions changed since the last force call
    // the integrator already wrote the interior sorted records and the skin/2
    // displacement flag for the current positions (Verlet lists only)
    bool upkeep_fused = false;
    // Between Verlet-list rebuilds the integrator keeps its state in sorted
    // order: positions in the interior sorted records, velocities (x, y, z
    // triples) and the list-build reference positions (SoA) by compact
    // sorted index (b_vsort, b_xrsort).  While sorted_active the
    // caller-order positions and the velocity arrays of the running step
    // call (vv_v) are behind.  A rebuild gets caller-order positions and
    // tinv (caller index -> compact index); the velocities stay in the old
    // compact order (vs_old_order) until the next sorted step carries them
    // into the new one.  The call brings the caller's arrays up to date
    // before it returns.
    bool sorted_active = false;
    bool vs_old_order = false;
    double *vv_v[3] = {nullptr, nullptr, nullptr};
    // the interior sorted records still hold the positions of the last list
    // build (equal to the saved reference positions)
    bool rec_at_build = false;

    // neighbour structure state
    bool built = false;           // structure matches cfg/positions
    mdlj_config built_cfg = {-1, -1, -1, -1, -1, -1, -1, -1};
    int steps_since_build = 0;
    double built_box[3] = {0, 0, 0};
    double built_rc = -1, built_skin = -1;
    Grid grid{};
    int64_t n_ext = 0;            // real + halo slots
    int32_t max_cell = 0;         // most particles in one cell of the last binning
    int32_t max_nbhd = 0;         // most particles in one 27-cell neighbourhood (VL build)
    // largest staged neighbourhood and candidate-list total of one tile in the
    // last tiled list build, and the grid (n, trim) they belong to: sizes
    // the next build's LDS without a pre-pass
    int32_t tile_c_hint = 0, tile_nc_hint = 0;
    int tile_hint_key[4] = {0, 0, 0, -1};
    int64_t nbr_cap = 0;          // Verlet list capacity per particle
    int64_t vl_max = 0;           // longest list of the last build
    int64_t vcl_cap = 0;          // cluster-pair list capacity per cluster

    // named device buffers
    DevBuf b_pos, b_type, b_force;  // caller-order state above
    DevBuf b_cell_of, b_rank, b_count, b_start, b_slot_of, b_sorted, b_scan_part, b_fsorted,
        b_partial, b_flags, b_nbr, b_nlen, b_ref, b_disp, b_misc, b_clu, b_cpair, b_cstart,
        b_fold, b_cnt_ext, b_img, b_icnt, b_ilist, b_xref, b_mlp, b_feat, b_halo, b_hstart, b_vsort,
        b_vsort2, b_xrsort, b_tinv, b_sorted2, b_fxrec, b_fxrec2, b_fxspec, b_tunev, b_nbr_in,
        b_nlo_in, b_tilebad, b_nlo;
    int64_t nhalo = 0;            // entries of b_halo
    int halo_key[6] = {0, 0, 0, 0, 0, 0};  // grid (n, h) the halo list was made for

    // tuner state
    std::vector<mdlj_config> space;
    std::vector<double> tune_us;
    std::vector<int> tune_taken;  // samples each configuration used in the last search
    std::vector<double> tune_watts;  // mean power per configuration (energy metric)
    int tune_metric = MDLJ_METRIC_TIME;
    // learned tuner
    std::vector<float> mlp_w, mlp_m, mlp_v;
    float mlp_mean[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    float mlp_std[8] = {1, 1, 1, 1, 1, 1, 1, 1};
    int mlp_k = 0;
    int mlp_adam_t = 0;
    double mlp_threshold = 0.6;
    double mlp_last_conf = 0.0;
    int64_t mlp_fallbacks = 0;
    bool mlp_loaded = false;

    // reusable host scratch
    std::vector<double> h_partial;

    // kernel timing (HIP events on the context's stream), read lazily
    struct Timed {
        hipEvent_t e0, e1, e2;
        bool rebuilt;
        bool fused;  // the force kernel took the integrator step too
    };
    bool timing = false;
    // inside a timed force call: rebuild() records build_mark at its start
    bool want_build_mark = false;
    hipEvent_t build_mark = nullptr;
    std::vector<hipEvent_t> ev_pool;
    std::deque<Timed> ev_pending;
    // host words written by small kernels (pinned host memory, d_hflag its
    // device address): the displacement flag with its sequence number, the
    // binning results and the list-build maxima; dflag_zero: the
    // device-side flag is known to hold 0
    int32_t *h_flag = nullptr;
    int32_t *d_hflag = nullptr;
    // sequence numbers of publications to the host words: the last one
    // handed out, and that of the last displacement flag
    uint32_t flag_seq = 0, flag_seq_disp = 0;
    bool dflag_zero = false;
    // fused integrator step: kd_req is set by the integrator around a force
    // call whose step continues in sorted order (kd_dt its time step);
    // kd_go is the decision taken for the current configuration after the
    // structure was made current, kd_done that the force kernel ran fused
    bool kd_req = false, kd_go = false, kd_done = false, kd_fx = false;
    double kd_dt = 0.0;
    // fixed-point words of the records (b_fxrec, frame centre fx_c and scale
    // fx_s; the species per record in b_fxspec) for the FP32-pair staged
    // kernel; fx_valid: they match the records (writers of the records that
    // do not keep them clear it)
    bool fx_valid = false;
    double fx_c[3] = {0, 0, 0}, fx_s = 0.0;
    // pruned inner list of the staged Verlet-list kernels (b_nbr_in,
    // b_nlo_in; two copies of inner_ntiles tile words in b_tilebad): prune
    // enables it; inner: 1 when the list build wrote one for the current
    // lists; inner_par: the copy launches read now
    bool prune = false;
    int inner = 0, inner_par = 0;
    int64_t inner_ntiles = 0;
    // allocation-free calls (mdlj_compute_forces_noalloc): no device buffer,
    // pinned word or timing event may be created or grown (ensure() and the
    // others refuse), and the energy/virial partials of the force kernels go
    // to partial_ext (partial_ext_cap doubles, the library's static scratch
    // array) instead of b_partial
    bool no_alloc = false;
    double *partial_ext = nullptr;
    int64_t partial_ext_cap = 0;
    double t_force_us = 0, t_build_us = 0, t_fused_us = 0;
    int64_t t_nforce = 0, t_nbuild = 0, t_nfused = 0;
    double last_force_us = 0, last_build_us = 0;
};

// --- helpers implemented in api.cpp --------------------------------------
mdlj_status set_err(mdlj_ctx *ctx, mdlj_status st, const std::string &msg);
mdlj_status hip_check(mdlj_ctx *ctx, hipError_t e, const char *what);
mdlj_status ensure(mdlj_ctx *ctx, DevBuf &b, size_t bytes);
// Buffer for nvals doubles of per-workgroup (U, W) partials: the context's
// b_partial, or in an allocation-free call the static scratch array (an
// error when nvals exceeds it).
mdlj_status partial_buffer(mdlj_ctx *ctx, int64_t nvals, double **out);

#define HIPCHK(ctx, call)                                      \
    do {                                                       \
        hipError_t _e = (call);                                \
        if (_e != hipSuccess) return hip_check(ctx, _e, #call); \
    } while (0)

#define STCHK(call)                       \
    do {                                  \
        mdlj_status _s = (call);          \
        if (_s != MDLJ_OK) return _s;     \
    } while (0)

// --- pruned inner list (vl.hip) -------------------------------------------
// The tile words for a kernel that moves particles (cur/next null when
// there is no inner list).  The caller calls inner_flip after queueing it.
InnerMark inner_marker(mdlj_ctx *ctx);
void inner_flip(mdlj_ctx *ctx);

// --- binning (bin.hip) ----------------------------------------------------
// Bins the caller-order positions into g (wrapping them in place), writes
// the sorted real + halo records and slot_of[i] (slot of caller particle i).
// interior_list: also the compact interior order (build_ilist), queued
// before the host waits for the binning's sizes.
mdlj_status bin_particles(mdlj_ctx *ctx, const Grid &g, bool interior_list = false);
// Halo slots carry forces applied to images by Newton-3 kernels: add them
// onto the slot of the particle they copy.
mdlj_status fold_forces(mdlj_ctx *ctx, const ForceOut &fo);
// Sorted FP64 forces back to caller order.
mdlj_status unpermute_forces(mdlj_ctx *ctx, const ForceOut &fo, double *ox, double *oy, double *oz);
mdlj_status zero_forces(mdlj_ctx *ctx, const ForceOut &fo, int64_t nslots);
// Sum of per-block (U, W) partials.
mdlj_status reduce_partials(mdlj_ctx *ctx, const double *partial, int64_t nblocks,
                            double *UW_host);
mdlj_status check_types(mdlj_ctx *ctx, bool *ok);
// Exclusive scan of n int32 counts; out[n] receives the total.
mdlj_status exclusive_scan(mdlj_ctx *ctx, const int32_t *in, int32_t *out, int64_t n);
// Compact list (length n) of the slots of real particles in sorted order,
// for grid g (binned, its cell starts written).
mdlj_status build_ilist(mdlj_ctx *ctx, const Grid &g);
mdlj_status check_finite(mdlj_ctx *ctx, const double *x, const double *y, const double *z,
                         int64_t n, bool *ok);

// --- integrator and record upkeep (integrate.hip) ---------------------------
mdlj_status save_reference(mdlj_ctx *ctx);
// Pinned host words ctx->h_flag (16 int32) and their device address
// ctx->d_hflag: [0] the displacement flag and [1] its sequence number,
// [4..6] binning results and [7] their sequence number, [8..11] Verlet-list
// build maxima and [12] their sequence number.
mdlj_status ensure_host_flag(mdlj_ctx *ctx);
mdlj_status moved_too_far(mdlj_ctx *ctx, bool *too_far);
// Enqueue the skin/2 displacement check; its result lands in pinned host
// memory with the sequence number flag_seq_disp (read with check_result).
mdlj_status launch_displacement_check(mdlj_ctx *ctx);
mdlj_status check_result(mdlj_ctx *ctx, bool *too_far);
// Wait until h_flag[at] holds seq: written (release, system scope) by a
// small kernel after the host words it publishes.  Spins, then falls back
// to a stream synchronisation.
mdlj_status wait_host_words(mdlj_ctx *ctx, int at, uint32_t seq);
mdlj_status refresh_records(mdlj_ctx *ctx);
// After a fused integrator step: refresh the halo records from their
// sources; the same kernel hands the displacement flag to the host (with
// the sequence number flag_seq_disp) and clears it for the next step.
mdlj_status finish_fused_upkeep(mdlj_ctx *ctx);
// (halo cell, source cell) pairs of the current grid, for the halo refresh.
mdlj_status build_halo_list(mdlj_ctx *ctx);
mdlj_status vv_steps(mdlj_ctx *ctx, double *vx, double *vy, double *vz, double dt, int nsteps);
// Write the sorted-order integrator state back to the caller-order
// positions and velocities (no-op without such state).
mdlj_status leave_sorted(mdlj_ctx *ctx);
// Before a rebuild: caller-order positions from the sorted state, the
// velocities kept for the next sorted step (no-op without such state).
mdlj_status positions_for_rebuild(mdlj_ctx *ctx);
// Before a force call that may fuse the integrator step: decide (kd_go)
// and, if the state is still in caller order, carry it into sorted order.
mdlj_status kd_prepare(mdlj_ctx *ctx, const mdlj_config &c, bool energy);
// Inside the integrator, after the records of a staged Verlet-list build
// are made: carry the velocities into the new sorted order now (the step
// continues in sorted order), so that it runs while the host waits for the
// build's sizes.  Nothing otherwise.
mdlj_status enter_sorted_early(mdlj_ctx *ctx, const mdlj_config &c);
// Arguments of the fused step from the context's current buffers.
mdlj_status kd_args(mdlj_ctx *ctx, KickArgs *ka);

// --- force evaluation (api.cpp) ---------------------------------------------
// Bring the neighbour structure of c up to date for the current positions.
mdlj_status prepare(mdlj_ctx *ctx, const mdlj_config &c, bool positions_changed, bool *rebuilt);
mdlj_status run_force_kernel(mdlj_ctx *ctx, const mdlj_config &c, bool energy, ForceOut &fo,
                             int64_t *nblocks);
// Full evaluation with the current configuration.  Sorted forces (halo
// images folded) are returned in *fo when fo is given; when to_caller is set
// they are also written to ctx->fx/fy/fz in caller order.  UW (host, may be
// null) receives U and W (this synchronises).
mdlj_status forces_internal(mdlj_ctx *ctx, bool positions_changed, double *UW, ForceOut *fo = nullptr,
                            bool to_caller = true);
// Sum up timed calls whose events have completed (synchronises).
mdlj_status collect_timing(mdlj_ctx *ctx);
bool needs_fold(const mdlj_config &c);

// --- tuning (tune.cpp, mlp.hip) ---------------------------------------------
mdlj_status tune_exhaustive(mdlj_ctx *ctx, int samples, mdlj_config *chosen, double *best_us);
mdlj_status tune_measure_current(mdlj_ctx *ctx, int samples, double *us);
mdlj_status tune_learned(mdlj_ctx *ctx, int samples, mdlj_config *chosen, double *us);
mdlj_status tune_early(mdlj_ctx *ctx, int samples, mdlj_config *chosen, double *us);
// The GPU's energy counter (AMD SMI): joules and the refresh timestamp (ns).
mdlj_status energy_read(mdlj_ctx *ctx, double *joules, uint64_t *ts_ns);
// Configuration indices by descending network probability for the current
// scene; empty when no network for this search space is loaded.
mdlj_status mlp_rank(mdlj_ctx *ctx, std::vector<int> &order);

// --- force kernels ----------------------------------------------------------
mdlj_status lc_forces(mdlj_ctx *ctx, const mdlj_config &cfg, bool energy, ForceOut &fo,
                      int64_t *nblocks);
mdlj_status vl_build(mdlj_ctx *ctx, const mdlj_config &cfg);
mdlj_status vl_forces(mdlj_ctx *ctx, const mdlj_config &cfg, bool energy, ForceOut &fo,
                      int64_t *nblocks);
// Stored list entries (rows padded to a multiple of 8) of the current lists.
mdlj_status vl_list_entries(mdlj_ctx *ctx, int64_t *entries);
mdlj_status vcl_build(mdlj_ctx *ctx, const mdlj_config &cfg);
mdlj_status vcl_forces(mdlj_ctx *ctx, const mdlj_config &cfg, bool energy, ForceOut &fo,
                       int64_t *nblocks);
mdlj_status count_pairs_dev(mdlj_ctx *ctx, int64_t *out);
// Caller-index views of the current lists (mdlj_get_pairs): *count pairs,
// written to host arrays pi, pj when given (MDLJ_ERR_OVERFLOW if over cap).
mdlj_status vl_pairs(mdlj_ctx *ctx, int64_t cap, int32_t *pi, int32_t *pj, int64_t *count);
mdlj_status vcl_pairs(mdlj_ctx *ctx, int64_t cap, int32_t *pi, int32_t *pj, int64_t *count);

// grid set-up shared by the containers: edge >= r_min per axis, h halo layers
bool make_grid(const double *L, const double *r_min, const int *h, bool z_fastest, Grid *g);

template <typename T>
void fill_table(const mdlj_ctx *ctx, LJTable<T> *t);

__host__ __device__ static inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
