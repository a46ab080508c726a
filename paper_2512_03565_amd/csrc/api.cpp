// api.cpp -- the C ABI of libmdlj: context, settings, neighbour-structure
// life cycle and dispatch of the force kernel of the current configuration.
//
// The container/traversal/functor split follows section 2.3 (Fig. "flow"):
// the context owns particles and neighbour structures (linked cells,
// Verlet lists, Verlet cluster lists, section 2.1.1), and compute_forces
// hands them to the force kernel of the chosen interaction order
// (section 4.1).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>

#include "internal.h"
#include "lanemap.h"

#define MDLJ_VERSION_STR "mdlj 0.1 gfx950"

mdlj_status set_err(mdlj_ctx *ctx, mdlj_status st, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return st;
}

mdlj_status hip_check(mdlj_ctx *ctx, hipError_t e, const char *what)
{
    char buf[512];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    return set_err(ctx, e == hipErrorOutOfMemory ? MDLJ_ERR_NOMEM : MDLJ_ERR_HIP, buf);
}

mdlj_status ensure(mdlj_ctx *ctx, DevBuf &b, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    if (b.bytes >= bytes) return MDLJ_OK;
    if (ctx->no_alloc)
        return set_err(ctx, MDLJ_ERR_NOMEM,
                       "the allocation-free call would have to grow a device buffer to " +
                           std::to_string(bytes) + " bytes (call mdlj_compute_forces first)");
    if (b.p) {
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        HIPCHK(ctx, hipFree(b.p));
        b.p = nullptr;
        b.bytes = 0;
    }
    size_t want = bytes + bytes / 8;  // grow with headroom
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        b.p = nullptr;
        return hip_check(ctx, e, "hipMalloc");
    }
    b.bytes = want;
    return MDLJ_OK;
}

mdlj_status partial_buffer(mdlj_ctx *ctx, int64_t nvals, double **out)
{
    if (ctx->partial_ext) {
        if (nvals > ctx->partial_ext_cap)
            return set_err(ctx, MDLJ_ERR_ARG,
                           "energy partials of " + std::to_string(nvals) +
                               " doubles exceed the allocation-free scratch of " +
                               std::to_string(ctx->partial_ext_cap));
        *out = ctx->partial_ext;
        return MDLJ_OK;
    }
    STCHK(ensure(ctx, ctx->b_partial, sizeof(double) * nvals));
    *out = (double *)ctx->b_partial.p;
    return MDLJ_OK;
}

static void free_buf(DevBuf &b)
{
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

template <typename T>
void fill_table(const mdlj_ctx *ctx, LJTable<T> *t)
{
    memset(t, 0, sizeof *t);
    int ns = ctx->nspec;
    t->ns = ns;
    t->rc2 = (T)(ctx->rc * ctx->rc);
    t->rc2d = ctx->rc * ctx->rc;
    for (int a = 0; a < ns; ++a)
        for (int b = 0; b < ns; ++b) {
            // Lorentz-Berthelot mixing
            double sig = 0.5 * (ctx->sig[a] + ctx->sig[b]);
            double eps = sqrt(ctx->eps[a] * ctx->eps[b]);
            double sr = sig / ctx->rc;
            double sr6 = sr * sr * sr * sr * sr * sr;
            int k = a * ns + b;
            t->sig2[k] = (T)(sig * sig);
            t->eps24[k] = (T)(24.0 * eps);
            t->eps4[k] = (T)(4.0 * eps);
            t->shift[k] = ctx->shift_on ? (T)(4.0 * eps * (sr6 * sr6 - sr6)) : (T)0;
        }
}
template void fill_table<float>(const mdlj_ctx *, LJTable<float> *);
template void fill_table<double>(const mdlj_ctx *, LJTable<double> *);

// ------------------------------------------------------------------ configs

static bool cfg_eq(const mdlj_config &a, const mdlj_config &b)
{
    return a.nbr_algo == b.nbr_algo && a.order == b.order && a.tile_i == b.tile_i &&
           a.tile_j == b.tile_j && a.cluster_size == b.cluster_size && a.newton3 == b.newton3 &&
           a.staged == b.staged && a.swap == b.swap;
}

// The search space: neighbour algorithm x interaction order x tile shape x
// Newton-3, the Cartesian product of section 2.3.2 extended by the order
// (section 4), restricted to the combinations that exist.
static std::vector<mdlj_config> build_space()
{
    std::vector<mdlj_config> v;
    // linked cells (rebinned every step; full shell, no Newton-3)
    for (int k : {1, 2, 4}) v.push_back({MDLJ_NBR_LC, MDLJ_ORD_I_PER_LANE, k, 1, 0, 0, 0});
    for (int st : {0, 1}) {
        for (int ai : {8, 16})
            v.push_back({MDLJ_NBR_LC, MDLJ_ORD_CLUSTER_TILE, ai, 64 / ai, 0, 0, st});
        for (int g : {1, 2, 4})
            v.push_back({MDLJ_NBR_LC, MDLJ_ORD_WAVE_PER_I, g, 64 / g, 0, 0, st});
    }
    // linked cells, Newton 3 over a half shell of neighbour cells: the own
    // particles as the i-list (three lane grids) or the partners (swap)
    v.push_back({MDLJ_NBR_LC, MDLJ_ORD_WAVE_PER_I, 1, 64, 0, 1, 1, 0});
    for (int ai : {4, 16}) v.push_back({MDLJ_NBR_LC, MDLJ_ORD_CLUSTER_TILE, ai, 64 / ai, 0, 1, 1, 0});
    v.push_back({MDLJ_NBR_LC, MDLJ_ORD_I_PER_LANE, 1, 1, 0, 1, 1, 1});
    // Verlet lists
    for (int n3 : {0, 1}) {
        v.push_back({MDLJ_NBR_VL, MDLJ_ORD_I_PER_LANE, 0, 0, 0, n3, 0});
        for (int g : {1, 2, 4, 8, 16})
            v.push_back({MDLJ_NBR_VL, MDLJ_ORD_WAVE_PER_I, g, 64 / g, 0, n3, 0});
    }
    // staged: tile_i = i's per wavefront, tile_j = list entries per lane per trip
    for (int gv : {802, 804, 1602, 1604, 408})
        v.push_back({MDLJ_NBR_VL, MDLJ_ORD_WAVE_PER_I, gv / 100, gv % 100, 0, 0, 1});
    // Verlet cluster lists
    for (int m : {4, 8})
        for (int n3 : {0, 1}) {
            v.push_back({MDLJ_NBR_VCL, MDLJ_ORD_I_PER_LANE, 0, 0, m, n3, 0});
            v.push_back({MDLJ_NBR_VCL, MDLJ_ORD_CLUSTER_TILE, m, 64 / m, m, n3, 0});
            // the same tile with the lanes running over i fastest
            v.push_back({MDLJ_NBR_VCL, MDLJ_ORD_CLUSTER_TILE, m, 64 / m, m, n3, 0, 1});
        }
    // Verlet cluster lists, a second tile shape: cluster_size x 4 lanes per
    // cluster pair, 64 / (4 cluster_size) cluster pairs per wavefront (after
    // the shapes above, so that their indices stay as they were)
    for (int m : {4, 8})
        for (int n3 : {0, 1})
            for (int sw : {0, 1}) v.push_back({MDLJ_NBR_VCL, MDLJ_ORD_CLUSTER_TILE, m, 4, m, n3, 0, sw});
    return v;
}

static bool cfg_valid(const mdlj_ctx *ctx, const mdlj_config &c)
{
    for (const auto &s : ctx->space)
        if (cfg_eq(s, c)) return true;
    return false;
}

// ------------------------------------------------------------------ helpers

static bool ready(const mdlj_ctx *ctx, std::string *why)
{
    if (!ctx->box_set) { *why = "box not set"; return false; }
    if (!(ctx->rc > 0)) { *why = "cutoff not set"; return false; }
    for (int s = 0; s < ctx->nspec; ++s)
        if (!ctx->species_set[s]) { *why = "species parameters not set"; return false; }
    return true;
}

// Interaction range a configuration needs from its neighbour structure.
static double range_of(const mdlj_ctx *ctx, const mdlj_config &c)
{
    return c.nbr_algo == MDLJ_NBR_LC ? ctx->rc : ctx->rc + ctx->skin;
}

static mdlj_status check_geometry(mdlj_ctx *ctx, const mdlj_config &c)
{
    double r = range_of(ctx, c);
    for (int a = 0; a < 3; ++a) {
        if (ctx->box[a] < 2.0 * r)
            return set_err(ctx, MDLJ_ERR_GEOMETRY, "box edge shorter than twice the interaction range");
        if (c.nbr_algo != MDLJ_NBR_VCL && floor(ctx->box[a] / r) < 3)
            return set_err(ctx, MDLJ_ERR_GEOMETRY, "fewer than 3 linked cells along an axis");
    }
    return MDLJ_OK;
}

static mdlj_status copy_in(mdlj_ctx *ctx, double *dst, const double *src, int mem_kind)
{
    hipMemcpyKind k = mem_kind == MDLJ_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIPCHK(ctx, hipMemcpyAsync(dst, src, sizeof(double) * ctx->n, k, ctx->stream));
    return MDLJ_OK;
}

static mdlj_status copy_out(mdlj_ctx *ctx, double *dst, const double *src, int mem_kind)
{
    hipMemcpyKind k = mem_kind == MDLJ_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    HIPCHK(ctx, hipMemcpyAsync(dst, src, sizeof(double) * ctx->n, k, ctx->stream));
    return MDLJ_OK;
}

static void invalidate(mdlj_ctx *ctx)
{
    ctx->built = false;
    ctx->forces_valid = false;
    ctx->inner = 0;
}

// ------------------------------------------------------------------ build

// (Re)build the neighbour structure of configuration c.
static mdlj_status take_event(mdlj_ctx *ctx, hipEvent_t *e);

static mdlj_status rebuild(mdlj_ctx *ctx, const mdlj_config &c)
{
    // a timed force call marks where its rebuild starts (its build time)
    if (ctx->want_build_mark && !ctx->build_mark) {
        STCHK(take_event(ctx, &ctx->build_mark));
        HIPCHK(ctx, hipEventRecord(ctx->build_mark, ctx->stream));
    }
    // binning reads the caller-order positions
    STCHK(positions_for_rebuild(ctx));
    // a build that fails part-way (a buffer that cannot grow) leaves nothing
    // marked as current
    ctx->built = false;
    ctx->inner = 0;
    STCHK(check_geometry(ctx, c));
    if (c.nbr_algo == MDLJ_NBR_VCL) {
        STCHK(vcl_build(ctx, c));
    } else {
        double r = range_of(ctx, c);
        double rmin[3] = {r, r, r};
        int h[3] = {1, 1, 1};
        Grid g;
        if (!make_grid(ctx->box, rmin, h, false, &g))
            return set_err(ctx, MDLJ_ERR_GEOMETRY, "grid set-up failed");
        STCHK(bin_particles(ctx, g, c.nbr_algo == MDLJ_NBR_VL));
        if (c.nbr_algo == MDLJ_NBR_VL) {
            // the reference positions (wrapped by the binning) are queued
            // before the build, which waits for its sizes
            STCHK(save_reference(ctx));
            STCHK(vl_build(ctx, c));
            STCHK(build_halo_list(ctx));
        }
    }
    if (c.nbr_algo == MDLJ_NBR_VCL) STCHK(save_reference(ctx));
    ctx->rec_at_build = c.nbr_algo == MDLJ_NBR_VL;
    ctx->built = true;
    ctx->built_cfg = c;
    ctx->steps_since_build = 0;
    memcpy(ctx->built_box, ctx->box, sizeof ctx->box);
    ctx->built_rc = ctx->rc;
    ctx->built_skin = ctx->skin;
    return MDLJ_OK;
}

static bool structure_current(const mdlj_ctx *ctx, const mdlj_config &c)
{
    if (!ctx->built) return false;
    const mdlj_config &b = ctx->built_cfg;
    // the VL/VCL structures differ per layout; LC grids only by range
    if (b.nbr_algo != c.nbr_algo) return false;
    if (c.nbr_algo == MDLJ_NBR_VL &&
        (b.order != c.order || b.newton3 != c.newton3 || b.staged != c.staged))
        return false;
    if (c.nbr_algo == MDLJ_NBR_VCL && (b.cluster_size != c.cluster_size || b.newton3 != c.newton3))
        return false;
    if (memcmp(ctx->built_box, ctx->box, sizeof ctx->box) != 0) return false;
    if (ctx->built_rc != ctx->rc || ctx->built_skin != ctx->skin) return false;
    return true;
}

// Make the structure valid for the current positions: LC re-bins whenever
// positions changed; lists are rebuilt when stale (interval reached).  When
// the lists are reused, the skin/2 displacement check is only enqueued
// (*check_pending); its result is read after the force kernel is queued.
mdlj_status prepare(mdlj_ctx *ctx, const mdlj_config &c, bool positions_changed, bool *rebuilt,
                    bool *check_pending)
{
    *rebuilt = false;
    *check_pending = false;
    const bool fused = ctx->upkeep_fused;
    ctx->upkeep_fused = false;
    bool need = !structure_current(ctx, c);
    if (!need && positions_changed) {
        if (c.nbr_algo == MDLJ_NBR_LC) {
            need = true;
        } else if (ctx->steps_since_build >= ctx->rebuild_every) {
            need = true;
        } else if (fused && c.nbr_algo == MDLJ_NBR_VL) {
            // the integrator moved the interior records and tested the
            // displacements; only the halo images are left
            STCHK(finish_fused_upkeep(ctx));
            *check_pending = true;
        } else {
            // lists stay exact while every particle moved less than skin/2
            STCHK(launch_displacement_check(ctx));
            STCHK(refresh_records(ctx));
            *check_pending = true;
        }
    }
    if (need) {
        STCHK(rebuild(ctx, c));
        *rebuilt = true;
    }
    return MDLJ_OK;
}

mdlj_status prepare(mdlj_ctx *ctx, const mdlj_config &c, bool positions_changed, bool *rebuilt)
{
    bool pending = false;
    STCHK(prepare(ctx, c, positions_changed, rebuilt, &pending));
    if (pending) {
        bool far = false;
        STCHK(check_result(ctx, &far));
        if (far) {
            STCHK(rebuild(ctx, c));
            *rebuilt = true;
        }
    }
    return MDLJ_OK;
}

// Add one timed force call to the totals and return its events to the pool.
static mdlj_status account(mdlj_ctx *ctx, const mdlj_ctx::Timed &t)
{
    float tf = 0;
    HIPCHK(ctx, hipEventElapsedTime(&tf, t.e1, t.e2));
    ctx->last_force_us = 1e3 * tf;
    ctx->t_force_us += 1e3 * tf;
    ctx->t_nforce++;
    if (t.fused) {
        ctx->t_fused_us += 1e3 * tf;
        ctx->t_nfused++;
    }
    if (t.e0) {
        float tb = 0;
        HIPCHK(ctx, hipEventElapsedTime(&tb, t.e0, t.e1));
        ctx->t_build_us += 1e3 * tb;
        ctx->t_nbuild++;
        ctx->ev_pool.push_back(t.e0);
    }
    ctx->ev_pool.push_back(t.e1);
    ctx->ev_pool.push_back(t.e2);
    return MDLJ_OK;
}

// An event for a timed force call: from the pool, refilled first from
// timed calls at least 64 calls old, which the device finished long ago (the
// wait on them returns at once), so a long timed run cycles a few hundred
// events instead of creating three per call.
static mdlj_status take_event(mdlj_ctx *ctx, hipEvent_t *e)
{
    while (ctx->ev_pool.empty() && ctx->ev_pending.size() > 64) {
        HIPCHK(ctx, hipEventSynchronize(ctx->ev_pending.front().e2));
        STCHK(account(ctx, ctx->ev_pending.front()));
        ctx->ev_pending.pop_front();
    }
    if (ctx->ev_pool.empty()) {
        if (ctx->no_alloc)
            return set_err(ctx, MDLJ_ERR_NOMEM,
                           "the allocation-free call would have to create a timing event");
        // timing only: no system-scope fence when recorded (no cache
        // write-back between the timed kernels)
        HIPCHK(ctx, hipEventCreateWithFlags(e, hipEventDisableSystemFence));
    } else {
        *e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
    }
    return MDLJ_OK;
}

mdlj_status collect_timing(mdlj_ctx *ctx)
{
    if (ctx->ev_pending.empty()) return MDLJ_OK;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (const auto &t : ctx->ev_pending) STCHK(account(ctx, t));
    ctx->ev_pending.clear();
    return MDLJ_OK;
}

// Run the force kernel of c into the sorted force buffers.
mdlj_status run_force_kernel(mdlj_ctx *ctx, const mdlj_config &c, bool energy, ForceOut &fo,
                             int64_t *nblocks)
{
    // one slot per record plus the padding record (Newton-3 kernels add
    // zero to it); the padding slot is never read back
    const int64_t stride = ctx->n_ext + 1;
    ctx->kd_done = false;
    STCHK(ensure(ctx, ctx->b_fsorted, sizeof(double) * 3 * stride));
    double *f = (double *)ctx->b_fsorted.p;
    fo.fx = f;
    fo.fy = f + stride;
    fo.fz = f + 2 * stride;
    fo.partial = nullptr;
    switch (c.nbr_algo) {
    case MDLJ_NBR_LC: return lc_forces(ctx, c, energy, fo, nblocks);
    case MDLJ_NBR_VL: return vl_forces(ctx, c, energy, fo, nblocks);
    case MDLJ_NBR_VCL: return vcl_forces(ctx, c, energy, fo, nblocks);
    }
    return set_err(ctx, MDLJ_ERR_ARG, "unknown neighbour algorithm");
}

// Newton-3 kernels over halo images leave forces on the images; cluster
// lists use shift codes instead of images and need no fold.
bool needs_fold(const mdlj_config &c)
{
    return c.newton3 != 0 && c.nbr_algo != MDLJ_NBR_VCL;
}

// The whole force evaluation for the current configuration into the
// context's caller-order force arrays; optional totals.
mdlj_status forces_internal(mdlj_ctx *ctx, bool positions_changed, double *UW, ForceOut *fo_out,
                            bool to_caller)
{
    std::string why;
    if (!ready(ctx, &why)) return set_err(ctx, MDLJ_ERR_STATE, why);
    const mdlj_config c = ctx->cfg;
    bool rebuilt = false, pending = false;
    mdlj_ctx::Timed tm = {nullptr, nullptr, nullptr, false, false};
    if (ctx->timing) {
        // e0 only when the call rebuilds (recorded by rebuild()); a mark
        // left by a call that failed goes back to the pool
        if (ctx->build_mark) ctx->ev_pool.push_back(ctx->build_mark);
        ctx->build_mark = nullptr;
        STCHK(take_event(ctx, &tm.e1));
        STCHK(take_event(ctx, &tm.e2));
        ctx->want_build_mark = true;
    }
    STCHK(prepare(ctx, c, positions_changed, &rebuilt, &pending));
    ForceOut fo;
    int64_t nb = 0;
    const bool energy = UW != nullptr;
    STCHK(kd_prepare(ctx, c, energy));
    if (ctx->timing) HIPCHK(ctx, hipEventRecord(tm.e1, ctx->stream));
    STCHK(run_force_kernel(ctx, c, energy, fo, &nb));
    if (ctx->timing) HIPCHK(ctx, hipEventRecord(tm.e2, ctx->stream));
    if (pending) {
        // the host waits for the check while the force kernel runs; on a
        // violation the lists are rebuilt and the forces computed again
        bool far = false;
        STCHK(check_result(ctx, &far));
        if (far) {
            // a fused integrator step wrote only the second record and
            // velocity buffers, which are not taken: the step is redone
            STCHK(rebuild(ctx, c));
            rebuilt = true;
            STCHK(kd_prepare(ctx, c, energy));
            if (ctx->timing) HIPCHK(ctx, hipEventRecord(tm.e1, ctx->stream));
            STCHK(run_force_kernel(ctx, c, energy, fo, &nb));
            if (ctx->timing) HIPCHK(ctx, hipEventRecord(tm.e2, ctx->stream));
        }
    }
    if (ctx->timing) {
        tm.rebuilt = rebuilt;
        tm.fused = ctx->kd_done;
        tm.e0 = ctx->build_mark;
        ctx->build_mark = nullptr;
        ctx->want_build_mark = false;
        ctx->ev_pending.push_back(tm);
    }
    if (needs_fold(c)) STCHK(fold_forces(ctx, fo));
    if (to_caller) STCHK(unpermute_forces(ctx, fo, ctx->fx, ctx->fy, ctx->fz));
    if (energy) STCHK(reduce_partials(ctx, fo.partial, nb, UW));
    ctx->steps_since_build++;
    ctx->forces_valid = to_caller;
    if (fo_out) *fo_out = fo;
    return MDLJ_OK;
}

// ------------------------------------------------- allocation-free scratch

// Device scratch of mdlj_compute_forces_noalloc: the per-workgroup (U, W)
// partials of the force kernels, 2^22 doubles (32 MiB), enough for every
// configuration of a context of up to about two million particles.  Each GPU
// holds its own copy for the life of the process.  Host code never uses the
// name itself (a host-side stand-in): the device address of each GPU's copy
// is taken once with hipGetSymbolAddress while that GPU is current.
#define MDLJ_SCRATCH_DOUBLES (1 << 22)
#define MDLJ_SCRATCH_MAX_DEVICES 64
static __device__ __align__(256) double scratch[MDLJ_SCRATCH_DOUBLES];
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[MDLJ_SCRATCH_MAX_DEVICES] = {};

static mdlj_status scratch_address(mdlj_ctx *ctx, double **out)
{
    int dev = -1;
    HIPCHK(ctx, hipGetDevice(&dev));
    if (dev < 0 || dev >= MDLJ_SCRATCH_MAX_DEVICES)
        return set_err(ctx, MDLJ_ERR_ARG, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIPCHK(ctx, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return set_err(ctx, MDLJ_ERR_HIP, "no device address for the scratch array");
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return MDLJ_OK;
}

// ------------------------------------------------------------------ ABI

extern "C" {

const char *mdlj_version(void) { return MDLJ_VERSION_STR; }

const char *mdlj_last_error(const mdlj_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

mdlj_status mdlj_create(mdlj_ctx **out, int64_t n, const double *x, const double *y,
                        const double *z, const int32_t *type, int32_t n_species,
                        int32_t mem_kind, void *hip_stream)
{
    if (!out) return MDLJ_ERR_ARG;
    *out = nullptr;
    if (n < 1 || n >= ((int64_t)1 << 30) || !x || !y || !z) return MDLJ_ERR_ARG;
    if (n_species < 1 || n_species > MDLJ_MAX_SPECIES) return MDLJ_ERR_ARG;
    if (mem_kind != MDLJ_MEM_HOST && mem_kind != MDLJ_MEM_DEVICE) return MDLJ_ERR_ARG;
    if (mem_kind == MDLJ_MEM_HOST) {
        for (int64_t i = 0; i < n; ++i)
            if (!isfinite(x[i]) || !isfinite(y[i]) || !isfinite(z[i])) return MDLJ_ERR_NONFINITE;
        if (type)
            for (int64_t i = 0; i < n; ++i)
                if (type[i] < 0 || type[i] >= n_species) return MDLJ_ERR_ARG;
    }
    mdlj_ctx *ctx = new (std::nothrow) mdlj_ctx();
    if (!ctx) return MDLJ_ERR_NOMEM;
    ctx->stream = (hipStream_t)hip_stream;
    ctx->n = n;
    ctx->nspec = n_species;
    ctx->space = build_space();
    mdlj_status st = MDLJ_OK;
    DevBuf pos, typ, frc;
    do {
        if ((st = ensure(ctx, pos, sizeof(double) * 3 * n)) != MDLJ_OK) break;
        if ((st = ensure(ctx, typ, sizeof(int32_t) * n)) != MDLJ_OK) break;
        if ((st = ensure(ctx, frc, sizeof(double) * 3 * n)) != MDLJ_OK) break;
        ctx->x = (double *)pos.p;
        ctx->y = ctx->x + n;
        ctx->z = ctx->x + 2 * n;
        ctx->type = (int32_t *)typ.p;
        ctx->fx = (double *)frc.p;
        ctx->fy = ctx->fx + n;
        ctx->fz = ctx->fx + 2 * n;
        if ((st = copy_in(ctx, ctx->x, x, mem_kind)) != MDLJ_OK) break;
        if ((st = copy_in(ctx, ctx->y, y, mem_kind)) != MDLJ_OK) break;
        if ((st = copy_in(ctx, ctx->z, z, mem_kind)) != MDLJ_OK) break;
        hipError_t e;
        if (type) {
            e = hipMemcpyAsync(ctx->type, type, sizeof(int32_t) * n,
                               mem_kind == MDLJ_MEM_DEVICE ? hipMemcpyDeviceToDevice
                                                           : hipMemcpyHostToDevice,
                               ctx->stream);
        } else {
            e = hipMemsetAsync(ctx->type, 0, sizeof(int32_t) * n, ctx->stream);
        }
        if (e != hipSuccess) { st = hip_check(ctx, e, "type copy"); break; }
        if (mem_kind == MDLJ_MEM_DEVICE) {
            bool ok = true;
            if ((st = check_finite(ctx, ctx->x, ctx->y, ctx->z, n, &ok)) != MDLJ_OK) break;
            if (!ok) { st = MDLJ_ERR_NONFINITE; break; }
            if (type) {
                if ((st = check_types(ctx, &ok)) != MDLJ_OK) break;
                if (!ok) { st = MDLJ_ERR_ARG; break; }
            }
        }
        e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) { st = hip_check(ctx, e, "create sync"); break; }
    } while (0);
    if (st != MDLJ_OK) {
        free_buf(pos);
        free_buf(typ);
        free_buf(frc);
        mdlj_destroy(ctx);
        return st;
    }
    ctx->b_pos = pos;
    ctx->b_type = typ;
    ctx->b_force = frc;
    *out = ctx;
    return MDLJ_OK;
}

mdlj_status mdlj_destroy(mdlj_ctx *ctx)
{
    if (!ctx) return MDLJ_OK;
    (void)hipStreamSynchronize(ctx->stream);
    for (const auto &t : ctx->ev_pending) {
        if (t.e0) ctx->ev_pool.push_back(t.e0);
        ctx->ev_pool.push_back(t.e1);
        ctx->ev_pool.push_back(t.e2);
    }
    if (ctx->build_mark) ctx->ev_pool.push_back(ctx->build_mark);
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    if (ctx->h_flag) (void)hipHostFree(ctx->h_flag);
    DevBuf *bufs[] = {&ctx->b_cell_of, &ctx->b_rank,    &ctx->b_count,   &ctx->b_start,
                      &ctx->b_slot_of, &ctx->b_sorted,  &ctx->b_scan_part, &ctx->b_fsorted,
                      &ctx->b_partial, &ctx->b_flags,   &ctx->b_nbr,     &ctx->b_nlen,
                      &ctx->b_ref,     &ctx->b_disp,    &ctx->b_misc,    &ctx->b_clu,
                      &ctx->b_cpair,   &ctx->b_cstart,  &ctx->b_fold,
                      &ctx->b_pos,     &ctx->b_type,    &ctx->b_force,
                      &ctx->b_cnt_ext, &ctx->b_img,     &ctx->b_icnt,    &ctx->b_ilist,
                      &ctx->b_xref,    &ctx->b_mlp,     &ctx->b_feat,    &ctx->b_halo,    &ctx->b_hstart,
                      &ctx->b_vsort,   &ctx->b_vsort2,  &ctx->b_xrsort,  &ctx->b_tinv,
                      &ctx->b_sorted2, &ctx->b_fxrec, &ctx->b_fxrec2, &ctx->b_fxspec,
                      &ctx->b_tunev,   &ctx->b_nbr_in,  &ctx->b_nlo_in,  &ctx->b_tilebad,
                      &ctx->b_nlo};
    for (DevBuf *b : bufs) free_buf(*b);
    delete ctx;
    return MDLJ_OK;
}

mdlj_status mdlj_set_box(mdlj_ctx *ctx, double lx, double ly, double lz)
{
    if (!ctx) return MDLJ_ERR_ARG;
    if (!(lx > 0 && ly > 0 && lz > 0) || !isfinite(lx) || !isfinite(ly) || !isfinite(lz))
        return set_err(ctx, MDLJ_ERR_ARG, "box edges must be positive and finite");
    ctx->box[0] = lx;
    ctx->box[1] = ly;
    ctx->box[2] = lz;
    ctx->box_set = true;
    invalidate(ctx);
    return MDLJ_OK;
}

mdlj_status mdlj_set_cutoff(mdlj_ctx *ctx, double rc)
{
    if (!ctx) return MDLJ_ERR_ARG;
    if (!(rc > 0) || !isfinite(rc)) return set_err(ctx, MDLJ_ERR_ARG, "cutoff must be positive");
    ctx->rc = rc;
    invalidate(ctx);
    return MDLJ_OK;
}

mdlj_status mdlj_set_skin(mdlj_ctx *ctx, double skin, int32_t rebuild_every)
{
    if (!ctx) return MDLJ_ERR_ARG;
    if (!(skin >= 0) || !isfinite(skin) || rebuild_every < 1)
        return set_err(ctx, MDLJ_ERR_ARG, "skin must be >= 0 and rebuild_every >= 1");
    ctx->skin = skin;
    ctx->rebuild_every = rebuild_every;
    invalidate(ctx);
    return MDLJ_OK;
}

mdlj_status mdlj_set_pruning(mdlj_ctx *ctx, int32_t on)
{
    if (!ctx) return MDLJ_ERR_ARG;
    if (on != 0 && on != 1) return set_err(ctx, MDLJ_ERR_ARG, "pruning is 0 or 1");
    ctx->prune = on != 0;
    ctx->inner = 0;
    invalidate(ctx);
    return MDLJ_OK;
}

mdlj_status mdlj_pruning_state(mdlj_ctx *ctx, int32_t *state, int64_t *tiles_out)
{
    if (!ctx || !state) return MDLJ_ERR_ARG;
    *state = 0;
    if (tiles_out) *tiles_out = 0;
    if (ctx->inner != 1) return MDLJ_OK;
    std::vector<int32_t> tw((size_t)ctx->inner_ntiles);
    HIPCHK(ctx, hipMemcpyAsync(tw.data(), (const int32_t *)ctx->b_tilebad.p +
                                              ctx->inner_par * ctx->inner_ntiles,
                               sizeof(int32_t) * tw.size(), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    int64_t bad = 0;
    for (int32_t v : tw) bad += v != 0;
    if (tiles_out) *tiles_out = bad;
    *state = bad == 0 ? 1 : (bad < (int64_t)tw.size() ? 2 : 3);
    return MDLJ_OK;
}

mdlj_status mdlj_set_species(mdlj_ctx *ctx, int32_t s, double epsilon, double sigma)
{
    if (!ctx) return MDLJ_ERR_ARG;
    if (s < 0 || s >= ctx->nspec) return set_err(ctx, MDLJ_ERR_ARG, "species index out of range");
    if (!(epsilon > 0) || !(sigma > 0) || !isfinite(epsilon) || !isfinite(sigma))
        return set_err(ctx, MDLJ_ERR_ARG, "epsilon and sigma must be positive");
    ctx->eps[s] = epsilon;
    ctx->sig[s] = sigma;
    ctx->species_set[s] = true;
    ctx->forces_valid = false;
    return MDLJ_OK;
}

mdlj_status mdlj_set_mass(mdlj_ctx *ctx, int32_t s, double mass)
{
    if (!ctx) return MDLJ_ERR_ARG;
    if (s < 0 || s >= ctx->nspec || !(mass > 0) || !isfinite(mass))
        return set_err(ctx, MDLJ_ERR_ARG, "bad species index or mass");
    ctx->mass[s] = mass;
    return MDLJ_OK;
}

mdlj_status mdlj_set_energy_shift(mdlj_ctx *ctx, int32_t on)
{
    if (!ctx) return MDLJ_ERR_ARG;
    if (on != 0 && on != 1) return set_err(ctx, MDLJ_ERR_ARG, "shift flag must be 0 or 1");
    ctx->shift_on = on;
    return MDLJ_OK;
}

mdlj_status mdlj_set_precision(mdlj_ctx *ctx, int32_t prec)
{
    if (!ctx) return MDLJ_ERR_ARG;
    if (prec != MDLJ_PREC_F32PAIR_F64ACC && prec != MDLJ_PREC_F64)
        return set_err(ctx, MDLJ_ERR_ARG, "unknown precision");
    ctx->prec = prec;
    ctx->forces_valid = false;
    return MDLJ_OK;
}

mdlj_status mdlj_set_positions(mdlj_ctx *ctx, const double *x, const double *y, const double *z,
                               int32_t mem_kind)
{
    if (!ctx) return MDLJ_ERR_ARG;
    if (!x || !y || !z || (mem_kind != MDLJ_MEM_HOST && mem_kind != MDLJ_MEM_DEVICE))
        return set_err(ctx, MDLJ_ERR_ARG, "bad positions");
    if (mem_kind == MDLJ_MEM_HOST) {
        for (int64_t i = 0; i < ctx->n; ++i)
            if (!isfinite(x[i]) || !isfinite(y[i]) || !isfinite(z[i]))
                return set_err(ctx, MDLJ_ERR_NONFINITE, "non-finite particle position");
    }
    STCHK(copy_in(ctx, ctx->x, x, mem_kind));
    STCHK(copy_in(ctx, ctx->y, y, mem_kind));
    STCHK(copy_in(ctx, ctx->z, z, mem_kind));
    if (mem_kind == MDLJ_MEM_DEVICE) {
        bool ok = true;
        STCHK(check_finite(ctx, ctx->x, ctx->y, ctx->z, ctx->n, &ok));
        if (!ok) return set_err(ctx, MDLJ_ERR_NONFINITE, "non-finite particle position");
    } else {
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    }
    ctx->forces_valid = false;
    ctx->pos_changed = true;
    ctx->upkeep_fused = false;
    return MDLJ_OK;
}

mdlj_status mdlj_get_positions(mdlj_ctx *ctx, double *x, double *y, double *z, int32_t mem_kind)
{
    if (!ctx) return MDLJ_ERR_ARG;
    if (!x || !y || !z || (mem_kind != MDLJ_MEM_HOST && mem_kind != MDLJ_MEM_DEVICE))
        return set_err(ctx, MDLJ_ERR_ARG, "bad output pointers");
    STCHK(copy_out(ctx, x, ctx->x, mem_kind));
    STCHK(copy_out(ctx, y, ctx->y, mem_kind));
    STCHK(copy_out(ctx, z, ctx->z, mem_kind));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return MDLJ_OK;
}

mdlj_status mdlj_set_config(mdlj_ctx *ctx, const mdlj_config *cfg)
{
    if (!ctx) return MDLJ_ERR_ARG;
    if (!cfg || !cfg_valid(ctx, *cfg)) return set_err(ctx, MDLJ_ERR_ARG, "invalid configuration");
    if (!cfg_eq(ctx->cfg, *cfg)) ctx->forces_valid = false;
    ctx->cfg = *cfg;
    return MDLJ_OK;
}

mdlj_status mdlj_get_config(const mdlj_ctx *ctx, mdlj_config *cfg)
{
    if (!ctx || !cfg) return MDLJ_ERR_ARG;
    *cfg = ctx->cfg;
    return MDLJ_OK;
}

mdlj_status mdlj_config_count(const mdlj_ctx *ctx, int32_t *count)
{
    if (!ctx || !count) return MDLJ_ERR_ARG;
    *count = (int32_t)ctx->space.size();
    return MDLJ_OK;
}

mdlj_status mdlj_config_at(const mdlj_ctx *ctx, int32_t k, mdlj_config *cfg)
{
    if (!ctx || !cfg || k < 0 || k >= (int32_t)ctx->space.size()) return MDLJ_ERR_ARG;
    *cfg = ctx->space[k];
    return MDLJ_OK;
}

mdlj_status mdlj_rebuild_neighbors(mdlj_ctx *ctx)
{
    if (!ctx) return MDLJ_ERR_ARG;
    std::string why;
    if (!ready(ctx, &why)) return set_err(ctx, MDLJ_ERR_STATE, why);
    STCHK(rebuild(ctx, ctx->cfg));
    ctx->pos_changed = false;
    return MDLJ_OK;
}

mdlj_status mdlj_compute_forces(mdlj_ctx *ctx, double *fx, double *fy, double *fz,
                                int32_t mem_kind, double *epot, double *virial)
{
    if (!ctx) return MDLJ_ERR_ARG;
    if (!fx || !fy || !fz || (mem_kind != MDLJ_MEM_HOST && mem_kind != MDLJ_MEM_DEVICE))
        return set_err(ctx, MDLJ_ERR_ARG, "bad output pointers");
    double UW[2] = {0, 0};
    bool want = epot || virial;
    STCHK(forces_internal(ctx, ctx->pos_changed, want ? UW : nullptr));
    ctx->pos_changed = false;
    STCHK(copy_out(ctx, fx, ctx->fx, mem_kind));
    STCHK(copy_out(ctx, fy, ctx->fy, mem_kind));
    STCHK(copy_out(ctx, fz, ctx->fz, mem_kind));
    if (mem_kind == MDLJ_MEM_HOST) HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (epot) *epot = UW[0];
    if (virial) *virial = UW[1];
    return MDLJ_OK;
}

mdlj_status mdlj_compute_forces_noalloc(mdlj_ctx *ctx, double *fx, double *fy, double *fz,
                                        double *epot, double *virial)
{
    if (!ctx) return MDLJ_ERR_ARG;
    if (!fx || !fy || !fz) return set_err(ctx, MDLJ_ERR_ARG, "bad output pointers");
    double *scr = nullptr;
    STCHK(scratch_address(ctx, &scr));
    ctx->no_alloc = true;
    ctx->partial_ext = scr;
    ctx->partial_ext_cap = MDLJ_SCRATCH_DOUBLES;
    double UW[2] = {0, 0};
    const bool want = epot || virial;
    mdlj_status st = forces_internal(ctx, ctx->pos_changed, want ? UW : nullptr);
    if (st == MDLJ_OK) {
        ctx->pos_changed = false;
        st = copy_out(ctx, fx, ctx->fx, MDLJ_MEM_DEVICE);
        if (st == MDLJ_OK) st = copy_out(ctx, fy, ctx->fy, MDLJ_MEM_DEVICE);
        if (st == MDLJ_OK) st = copy_out(ctx, fz, ctx->fz, MDLJ_MEM_DEVICE);
    }
    ctx->no_alloc = false;
    ctx->partial_ext = nullptr;
    ctx->partial_ext_cap = 0;
    if (st != MDLJ_OK) return st;
    if (epot) *epot = UW[0];
    if (virial) *virial = UW[1];
    return MDLJ_OK;
}

mdlj_status mdlj_set_timing(mdlj_ctx *ctx, int32_t on)
{
    if (!ctx) return MDLJ_ERR_ARG;
    STCHK(collect_timing(ctx));
    ctx->timing = on != 0;
    ctx->t_force_us = ctx->t_build_us = ctx->t_fused_us = 0;
    ctx->t_nforce = ctx->t_nbuild = ctx->t_nfused = 0;
    return MDLJ_OK;
}

mdlj_status mdlj_get_timing_fused(mdlj_ctx *ctx, double *fused_us, int64_t *n_fused)
{
    if (!ctx) return MDLJ_ERR_ARG;
    STCHK(collect_timing(ctx));
    if (fused_us) *fused_us = ctx->t_fused_us;
    if (n_fused) *n_fused = ctx->t_nfused;
    return MDLJ_OK;
}

mdlj_status mdlj_get_timing(mdlj_ctx *ctx, double *force_us, double *build_us,
                            int64_t *n_force, int64_t *n_build)
{
    if (!ctx) return MDLJ_ERR_ARG;
    STCHK(collect_timing(ctx));
    if (force_us) *force_us = ctx->t_force_us;
    if (build_us) *build_us = ctx->t_build_us;
    if (n_force) *n_force = ctx->t_nforce;
    if (n_build) *n_build = ctx->t_nbuild;
    return MDLJ_OK;
}

mdlj_status mdlj_step_vv(mdlj_ctx *ctx, double *vx, double *vy, double *vz, double dt,
                         int32_t nsteps)
{
    if (!ctx) return MDLJ_ERR_ARG;
    if (!vx || !vy || !vz || nsteps < 0 || !(dt > 0) || !isfinite(dt))
        return set_err(ctx, MDLJ_ERR_ARG, "bad velocities, time step or step count");
    std::string why;
    if (!ready(ctx, &why)) return set_err(ctx, MDLJ_ERR_STATE, why);
    return vv_steps(ctx, vx, vy, vz, dt, nsteps);
}

mdlj_status mdlj_count_pairs(mdlj_ctx *ctx, int64_t *n_useful_pairs)
{
    if (!ctx || !n_useful_pairs) return MDLJ_ERR_ARG;
    std::string why;
    if (!ready(ctx, &why)) return set_err(ctx, MDLJ_ERR_STATE, why);
    return count_pairs_dev(ctx, n_useful_pairs);
}

mdlj_status mdlj_neighbor_stats(mdlj_ctx *ctx, int64_t *list_entries, int32_t *entry_bytes,
                                int64_t *records)
{
    if (!ctx || !list_entries || !entry_bytes || !records) return MDLJ_ERR_ARG;
    if (!ctx->built) return set_err(ctx, MDLJ_ERR_STATE, "no neighbour structure built yet");
    const mdlj_config &b = ctx->built_cfg;
    *list_entries = 0;
    *entry_bytes = 0;
    *records = ctx->n_ext;
    if (b.nbr_algo == MDLJ_NBR_VL) {
        STCHK(vl_list_entries(ctx, list_entries));
        *entry_bytes = b.staged ? 2 : 4;
    }
    return MDLJ_OK;
}

mdlj_status mdlj_lane_map(int32_t layout, int32_t ai, int32_t width, int32_t lane, int32_t *i,
                          int32_t *j)
{
    if (!i || !j || (layout != LANE_I_MAJOR && layout != LANE_J_MAJOR) || width < 1 || ai < 1 ||
        ai > width || width % ai != 0 || lane < 0 || lane >= width)
        return MDLJ_ERR_ARG;
    const LanePair p = lane_pair(layout, ai, width, lane);
    *i = p.i;
    *j = p.j;
    return MDLJ_OK;
}

mdlj_status mdlj_config_lane_map(const mdlj_config *cfg, int32_t lane, int32_t *layout,
                                 int32_t *i, int32_t *j)
{
    if (!cfg || !layout || !i || !j || lane < 0 || lane >= MDLJ_WAVE) return MDLJ_ERR_ARG;
    int lay = LANE_I_MAJOR, ai = 1;
    const bool ipl = cfg->order == MDLJ_ORD_I_PER_LANE;
    if (ipl) {
        // every lane its own i, one j for all (within a cluster for VCL)
        lay = LANE_J_MAJOR;
        ai = MDLJ_WAVE;
    } else if (cfg->nbr_algo == MDLJ_NBR_VCL) {
        lay = cfg->swap ? LANE_J_MAJOR : LANE_I_MAJOR;
        ai = cfg->cluster_size;
        // several cluster pairs per wavefront: lane groups of tile_i x
        // tile_j lanes, group q with its own cluster (i offset q tile_i)
        // and its own j-lanes (offset q tile_j)
        const int w = cfg->tile_i * cfg->tile_j;
        if (cfg->tile_i == ai && cfg->tile_j >= 1 && w < MDLJ_WAVE && w >= 1 && MDLJ_WAVE % w == 0) {
            const int q = lane / w;
            const LanePair p = lane_pair(lay, ai, w, lane % w);
            *layout = lay;
            *i = q * cfg->tile_i + p.i;
            *j = q * cfg->tile_j + p.j;
            return MDLJ_OK;
        }
    } else {
        ai = cfg->tile_i;
    }
    if (ai < 1 || ai > MDLJ_WAVE || MDLJ_WAVE % ai != 0) return MDLJ_ERR_ARG;
    const LanePair p = lane_pair(lay, ai, MDLJ_WAVE, lane);
    *layout = lay;
    *i = p.i;
    *j = p.j;
    return MDLJ_OK;
}

mdlj_status mdlj_get_cells(mdlj_ctx *ctx, int32_t *cell, int32_t *ncell3)
{
    if (!ctx || !cell || !ncell3) return MDLJ_ERR_ARG;
    const Grid &g = ctx->grid;
    if (!ctx->b_cell_of.p || g.ncell_int <= 0)
        return set_err(ctx, MDLJ_ERR_STATE, "no binning yet");
    const int64_t n = ctx->n;
    std::vector<int32_t> e(n);
    HIPCHK(ctx, hipMemcpyAsync(e.data(), ctx->b_cell_of.p, sizeof(int32_t) * n,
                               hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (int64_t i = 0; i < n; ++i) {
        // extended index -> interior cell coordinates -> x-fastest number
        int c[3];
        for (int a = 0; a < 3; ++a) c[a] = (int)((e[i] / g.stride[a]) % g.e[a]) - g.h[a];
        cell[i] = c[0] + g.n[0] * (c[1] + g.n[1] * c[2]);
    }
    for (int a = 0; a < 3; ++a) ncell3[a] = g.n[a];
    return MDLJ_OK;
}

mdlj_status mdlj_get_pairs(mdlj_ctx *ctx, int64_t cap, int32_t *pi, int32_t *pj, int64_t *count)
{
    if (!ctx || !count || (pi == nullptr) != (pj == nullptr) || cap < 0) return MDLJ_ERR_ARG;
    if (!ctx->built) return set_err(ctx, MDLJ_ERR_STATE, "no neighbour structure built");
    if (ctx->built_cfg.nbr_algo == MDLJ_NBR_VL) return vl_pairs(ctx, cap, pi, pj, count);
    if (ctx->built_cfg.nbr_algo == MDLJ_NBR_VCL) return vcl_pairs(ctx, cap, pi, pj, count);
    return set_err(ctx, MDLJ_ERR_STATE, "linked cells keep no pair list");
}

}  // extern "C"
