// integrate.hip -- velocity Verlet (the integrator the paper's background
// names for turning forces into motion, section 2.1) and the upkeep of the
// sorted records between neighbour-list rebuilds.
//
// Verlet and cluster lists stay valid while no particle has moved more
// than skin/2 since they were built (section 2.1.1).  Between rebuilds the
// sorted records keep their slots; only their coordinates are refreshed
// from the caller-order positions, halo images with the same +-L shift as
// at build time.  Positions are left unwrapped until the next rebuild.
#include <string.h>

#include <utility>
#include <vector>

#include "internal.h"

namespace {

struct InvMass {
    double v[MDLJ_MAX_SPECIES];
};

// v += F dt / (2m); x += v dt
__global__ void k_kick_drift(int64_t n, double *__restrict__ x, double *__restrict__ y,
                             double *__restrict__ z, double *__restrict__ vx,
                             double *__restrict__ vy, double *__restrict__ vz,
                             const double *__restrict__ fx, const double *__restrict__ fy,
                             const double *__restrict__ fz, const int32_t *__restrict__ type,
                             InvMass im, double dt)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double h = 0.5 * dt * im.v[type[i]];
    const double ux = vx[i] + h * fx[i];
    const double uy = vy[i] + h * fy[i];
    const double uz = vz[i] + h * fz[i];
    vx[i] = ux;
    vy[i] = uy;
    vz[i] = uz;
    x[i] += dt * ux;
    y[i] += dt * uy;
    z[i] += dt * uz;
}

// Sorted records from current positions: rec[k] = x[orig] + image * L.
// Padding records (orig < 0) are left as they are.
__global__ void k_refresh(int64_t n_ext, PosT *__restrict__ rec, const char4 *__restrict__ img,
                          const double *__restrict__ x, const double *__restrict__ y,
                          const double *__restrict__ z, double lx, double ly, double lz)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_ext) return;
    const int32_t o = rec[k].orig;
    if (o < 0) return;
    const char4 c = img[k];
    rec[k].x = x[o] + (double)c.x * lx;
    rec[k].y = y[o] + (double)c.y * ly;
    rec[k].z = z[o] + (double)c.z * lz;
}

// Sorted forces (read through slot_of) drive the kicks, so no separate
// un-permute pass is needed between steps.
// v += F dt / m; x += v dt  (the second half kick of one step fused with the
// first half kick and the drift of the next)
__global__ void k_kick_drift_sorted(int64_t n, double *__restrict__ x, double *__restrict__ y,
                                    double *__restrict__ z, double *__restrict__ vx,
                                    double *__restrict__ vy, double *__restrict__ vz,
                                    const double *__restrict__ fx, const double *__restrict__ fy,
                                    const double *__restrict__ fz,
                                    const int32_t *__restrict__ slot_of,
                                    const int32_t *__restrict__ type, InvMass im, double dt)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t s = slot_of[i];
    const double h = 0.5 * dt * im.v[type[i]];
    // two half kicks, rounded as the unfused form would round them
    const double ux = (vx[i] + h * fx[s]) + h * fx[s];
    const double uy = (vy[i] + h * fy[s]) + h * fy[s];
    const double uz = (vz[i] + h * fz[s]) + h * fz[s];
    vx[i] = ux;
    vy[i] = uy;
    vz[i] = uz;
    x[i] += dt * ux;
    y[i] += dt * uy;
    z[i] += dt * uz;
}

// The same step for Verlet lists between rebuilds, in sorted order: thread
// t takes the t-th interior record (ilist), its sorted force and its
// velocity and list-build reference position by compact index, so every
// access is coalesced.  The new position goes to the record (the list
// upkeep of the next force call), and a particle that has now moved more
// than sqrt(thr2) since the list build sets *flag.  Same arithmetic as
// k_kick_drift_sorted.
__global__ void k_kick_drift_compact(int64_t n, const int32_t *__restrict__ ilist,
                                     PosT *__restrict__ rec, double *__restrict__ vs,
                                     const double *__restrict__ fx,
                                     const double *__restrict__ fy,
                                     const double *__restrict__ fz, InvMass im, double dt,
                                     const double *__restrict__ xrs, double thr2,
                                     int32_t *__restrict__ flag, InnerMark imk)
{
    inner_carry(imk);
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int32_t s = ilist[t];
    PosT r = rec[s];
    const double h = 0.5 * dt * im.v[r.t];
    const double ux = (vs[3 * t] + h * fx[s]) + h * fx[s];
    const double uy = (vs[3 * t + 1] + h * fy[s]) + h * fy[s];
    const double uz = (vs[3 * t + 2] + h * fz[s]) + h * fz[s];
    vs[3 * t] = ux;
    vs[3 * t + 1] = uy;
    vs[3 * t + 2] = uz;
    r.x += dt * ux;
    r.y += dt * uy;
    r.z += dt * uz;
    // the whole 32-byte record, so no partially written sectors
    rec[s] = r;
    const double dx = r.x - xrs[t], dy = r.y - xrs[n + t], dz = r.z - xrs[2 * n + t];
    const double d2 = dx * dx + dy * dy + dz * dz;
    if (!(d2 <= thr2)) atomicOr(flag, 1);
    inner_mark(imk, r.orig, d2);
}

// The step before a list rebuild, from the sorted-order state: the same
// kick and drift as k_kick_drift_compact.  Positions go to caller order (the
// rebuild bins from there); velocities stay by compact index, and
// tinv[caller index] = compact index lets the first sorted step after the
// rebuild carry them into the new order.
__global__ void k_kick_leave(int64_t n, const int32_t *__restrict__ ilist,
                             const PosT *__restrict__ rec, double *__restrict__ vs,
                             const double *__restrict__ fx, const double *__restrict__ fy,
                             const double *__restrict__ fz, InvMass im, double dt,
                             double *__restrict__ x, double *__restrict__ y,
                             double *__restrict__ z, int32_t *__restrict__ tinv)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int32_t s = ilist[t];
    const PosT r = rec[s];
    const double h = 0.5 * dt * im.v[r.t];
    const double ux = (vs[3 * t] + h * fx[s]) + h * fx[s];
    const double uy = (vs[3 * t + 1] + h * fy[s]) + h * fy[s];
    const double uz = (vs[3 * t + 2] + h * fz[s]) + h * fz[s];
    vs[3 * t] = ux;
    vs[3 * t + 1] = uy;
    vs[3 * t + 2] = uz;
    const int32_t o = r.orig;
    x[o] = r.x + dt * ux;
    y[o] = r.y + dt * uy;
    z[o] = r.z + dt * uz;
    tinv[o] = (int32_t)t;
}

// For a rebuild while the sorted-order state is current: caller-order
// positions from the records and tinv as in k_kick_leave.
__global__ void k_leave_positions(int64_t n, const int32_t *__restrict__ ilist,
                                  const PosT *__restrict__ rec, double *__restrict__ x,
                                  double *__restrict__ y, double *__restrict__ z,
                                  int32_t *__restrict__ tinv)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const PosT r = rec[ilist[t]];
    const int32_t o = r.orig;
    x[o] = r.x;
    y[o] = r.y;
    z[o] = r.z;
    tinv[o] = (int32_t)t;
}

// Reference positions of a list build: xr = (x, y, z) in one pass.
__global__ void k_save_reference(int64_t n, const double *__restrict__ x,
                                 const double *__restrict__ y, const double *__restrict__ z,
                                 double *__restrict__ xr)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    xr[i] = x[i];
    xr[n + i] = y[i];
    xr[2 * n + i] = z[i];
}

// Into sorted order: velocities and list-build reference positions of the
// interior records by compact index (velocities as x, y, z triples).
// Velocities come from caller order (vx, vy, vz) or, after a rebuild, from
// the previous compact order through tinv (vprev).  from_rec: the records
// still hold the build positions, which then serve as the reference (no
// gather).
__global__ void k_enter_sorted(int64_t n, const int32_t *__restrict__ ilist,
                               const PosT *__restrict__ rec, const double *__restrict__ vx,
                               const double *__restrict__ vy, const double *__restrict__ vz,
                               const int32_t *__restrict__ tinv,
                               const double *__restrict__ vprev, const double *__restrict__ xr,
                               int from_rec, double *__restrict__ vs, double *__restrict__ xrs)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const PosT r = rec[ilist[t]];
    const int32_t o = r.orig;
    if (vprev) {
        const int64_t q = tinv[o];
        vs[3 * t] = vprev[3 * q];
        vs[3 * t + 1] = vprev[3 * q + 1];
        vs[3 * t + 2] = vprev[3 * q + 2];
    } else {
        vs[3 * t] = vx[o];
        vs[3 * t + 1] = vy[o];
        vs[3 * t + 2] = vz[o];
    }
    xrs[t] = from_rec ? r.x : xr[o];
    xrs[n + t] = from_rec ? r.y : xr[n + o];
    xrs[2 * n + t] = from_rec ? r.z : xr[2 * n + o];
}

// Back to caller order: positions from the interior records, velocities
// from their compact-index copies.
__global__ void k_leave_sorted(int64_t n, const int32_t *__restrict__ ilist,
                               const PosT *__restrict__ rec, const double *__restrict__ vs,
                               double *__restrict__ x, double *__restrict__ y,
                               double *__restrict__ z, double *__restrict__ vx,
                               double *__restrict__ vy, double *__restrict__ vz)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const PosT r = rec[ilist[t]];
    const int32_t o = r.orig;
    x[o] = r.x;
    y[o] = r.y;
    z[o] = r.z;
    vx[o] = vs[3 * t];
    vy[o] = vs[3 * t + 1];
    vz[o] = vs[3 * t + 2];
}

// Back to caller order from the previous compact order (the positions are
// there already): v[o] = vs[tinv[o]].
__global__ void k_leave_velocities(int64_t n, const int32_t *__restrict__ tinv,
                                   const double *__restrict__ vs, double *__restrict__ vx,
                                   double *__restrict__ vy, double *__restrict__ vz)
{
    int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n) return;
    const int64_t q = tinv[o];
    vx[o] = vs[3 * q];
    vy[o] = vs[3 * q + 1];
    vz[o] = vs[3 * q + 2];
}

// The displacement flag of the last integrator step goes to the host word
// (system scope, so the host sees it once the kernel has finished) and is
// cleared for the next step.  The integrator kernel that set it has
// finished: it ran before on the same stream.
// The value goes to the host together with the publication's sequence
// number in one 64-bit store, so the host knows the word it reads is this
// publication's without a system-scope fence on the stream.
__device__ __forceinline__ void publish_flag(int32_t *flag, int32_t *host, uint32_t seq)
{
    const int32_t v = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t w = ((uint64_t)seq << 32) | (uint32_t)v;
    __hip_atomic_store((uint64_t *)host, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(flag, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_publish_flag(int32_t *flag, int32_t *host, uint32_t seq)
{
    if (threadIdx.x == 0) publish_flag(flag, host, seq);
}

// Halo records from their source records, a group of lanes per halo cell:
// rec = source + image * L (the same sum the full refresh forms from the
// caller-order positions).  hl holds (halo cell, source cell) pairs.  The
// first thread also publishes the displacement flag.
constexpr int HALO_LANES = 16;

__global__ __launch_bounds__(256) void k_refresh_halo(int64_t nh, const int2 *__restrict__ hl,
                                                      const int32_t *__restrict__ start,
                                                      const char4 *__restrict__ img,
                                                      PosT *__restrict__ rec, double lx, double ly,
                                                      double lz, int32_t *flag, int32_t *host,
                                                      uint32_t seq, FxWords *__restrict__ fxr,
                                                      double cx, double cy, double cz, double fs)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) publish_flag(flag, host, seq);
    // HALO_LANES lanes per halo cell (cells hold ~17 records at liquid
    // densities, so a whole wavefront per cell would idle most lanes)
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / HALO_LANES;
    const int sub = threadIdx.x & (HALO_LANES - 1);
    if (w >= nh) return;
    const int2 p = hl[w];
    const int32_t b = start[p.x], cnt = start[p.x + 1] - b, sb = start[p.y];
    for (int32_t m = sub; m < cnt; m += HALO_LANES) {
        const char4 c = img[b + m];
        PosT q = rec[sb + m];
        q.x += (double)c.x * lx;
        q.y += (double)c.y * ly;
        q.z += (double)c.z * lz;
        rec[b + m] = q;
        // the images' fixed-point words, when the records have them
        if (fxr)
            fxr[b + m] = FxWords{to_fx(q.x, cx, fs), to_fx(q.y, cy, fs), to_fx(q.z, cz, fs)};
    }
}

// v += F dt / (2m) from sorted forces; also writes the caller-order forces
__global__ void k_kick_sorted(int64_t n, double *__restrict__ vx, double *__restrict__ vy,
                              double *__restrict__ vz, const double *__restrict__ fx,
                              const double *__restrict__ fy, const double *__restrict__ fz,
                              const int32_t *__restrict__ slot_of,
                              const int32_t *__restrict__ type, InvMass im, double dt,
                              double *__restrict__ ox, double *__restrict__ oy,
                              double *__restrict__ oz)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t s = slot_of[i];
    const double h = 0.5 * dt * im.v[type[i]];
    const double gx = fx[s], gy = fy[s], gz = fz[s];
    vx[i] += h * gx;
    vy[i] += h * gy;
    vz[i] += h * gz;
    ox[i] = gx;
    oy[i] = gy;
    oz[i] = gz;
}

// flag := 1 if any particle moved more than sqrt(thr2) since the reference
__global__ void k_displacement(int64_t n, const double *__restrict__ x,
                               const double *__restrict__ y, const double *__restrict__ z,
                               const double *__restrict__ xr, double thr2,
                               int32_t *__restrict__ flag, InnerMark imk)
{
    inner_carry(imk);
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double dx = x[i] - xr[i], dy = y[i] - xr[n + i], dz = z[i] - xr[2 * n + i];
    const double d2 = dx * dx + dy * dy + dz * dz;
    if (!(d2 <= thr2)) atomicOr(flag, 1);
    inner_mark(imk, i, d2);
}

}  // namespace

mdlj_status save_reference(mdlj_ctx *ctx)
{
    const int64_t n = ctx->n;
    STCHK(ensure(ctx, ctx->b_xref, sizeof(double) * 3 * n));
    double *xr = (double *)ctx->b_xref.p;
    k_save_reference<<<ceil_div(n, 256), 256, 0, ctx->stream>>>(n, ctx->x, ctx->y, ctx->z, xr);
    HIPCHK(ctx, hipGetLastError());
    return MDLJ_OK;
}

mdlj_status ensure_host_flag(mdlj_ctx *ctx)
{
    if (ctx->h_flag) return MDLJ_OK;
    if (ctx->no_alloc)
        return set_err(ctx, MDLJ_ERR_NOMEM,
                       "the allocation-free call would have to allocate pinned host words");
    // coherent: the kernel's store reaches host memory without a cache
    // write-back
    HIPCHK(ctx, hipHostMalloc((void **)&ctx->h_flag, 64, hipHostMallocCoherent));
    memset(ctx->h_flag, 0, 64);
    ctx->flag_seq = ctx->flag_seq_disp = 0;
    HIPCHK(ctx, hipHostGetDevicePointer((void **)&ctx->d_hflag, ctx->h_flag, 0));
    return MDLJ_OK;
}

mdlj_status launch_displacement_check(mdlj_ctx *ctx)
{
    const int64_t n = ctx->n;
    STCHK(ensure_host_flag(ctx));
    int32_t *flag = (int32_t *)ctx->b_flags.p + 13;
    if (!ctx->dflag_zero) HIPCHK(ctx, hipMemsetAsync(flag, 0, sizeof(int32_t), ctx->stream));
    const double h = 0.5 * ctx->skin;
    k_displacement<<<ceil_div(n, 256), 256, 0, ctx->stream>>>(n, ctx->x, ctx->y, ctx->z,
                                                             (const double *)ctx->b_xref.p, h * h,
                                                             flag, inner_marker(ctx));
    HIPCHK(ctx, hipGetLastError());
    inner_flip(ctx);
    ctx->flag_seq_disp = ++ctx->flag_seq;
    k_publish_flag<<<1, 64, 0, ctx->stream>>>(flag, ctx->d_hflag, ctx->flag_seq_disp);
    HIPCHK(ctx, hipGetLastError());
    ctx->dflag_zero = true;
    return MDLJ_OK;
}

mdlj_status wait_host_words(mdlj_ctx *ctx, int at, uint32_t seq)
{
    const uint32_t *w = (const uint32_t *)ctx->h_flag + at;
    for (int k = 0; k < (1 << 24); ++k)
        if (__atomic_load_n(w, __ATOMIC_ACQUIRE) == seq) return MDLJ_OK;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (__atomic_load_n(w, __ATOMIC_ACQUIRE) == seq) return MDLJ_OK;
    return set_err(ctx, MDLJ_ERR_HIP, "host words were not published");
}

mdlj_status check_result(mdlj_ctx *ctx, bool *too_far)
{
    // the publishing kernel's store to host memory carries the sequence
    // number: spin on it (no event between the kernels, which would stall
    // the stream), and in the end wait for the whole stream
    const uint64_t *w = (const uint64_t *)ctx->h_flag;
    uint64_t v = __atomic_load_n(w, __ATOMIC_ACQUIRE);
    for (int k = 0; (uint32_t)(v >> 32) != ctx->flag_seq_disp && k < (1 << 24); ++k)
        v = __atomic_load_n(w, __ATOMIC_ACQUIRE);
    if ((uint32_t)(v >> 32) != ctx->flag_seq_disp) {
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        v = __atomic_load_n(w, __ATOMIC_ACQUIRE);
        if ((uint32_t)(v >> 32) != ctx->flag_seq_disp)
            return set_err(ctx, MDLJ_ERR_HIP, "displacement flag was not published");
    }
    *too_far = (int32_t)(uint32_t)v != 0;
    return MDLJ_OK;
}

mdlj_status moved_too_far(mdlj_ctx *ctx, bool *too_far)
{
    STCHK(launch_displacement_check(ctx));
    return check_result(ctx, too_far);
}

mdlj_status finish_fused_upkeep(mdlj_ctx *ctx)
{
    int32_t *flag = (int32_t *)ctx->b_flags.p + 13;
    ctx->flag_seq_disp = ++ctx->flag_seq;
    if (ctx->nhalo > 0) {
        k_refresh_halo<<<ceil_div(ctx->nhalo, 256 / HALO_LANES), 256, 0, ctx->stream>>>(
            ctx->nhalo, (const int2 *)ctx->b_halo.p, (const int32_t *)ctx->b_start.p,
            (const char4 *)ctx->b_img.p, (PosT *)ctx->b_sorted.p, ctx->box[0], ctx->box[1],
            ctx->box[2], flag, ctx->d_hflag, ctx->flag_seq_disp,
            ctx->fx_valid ? (FxWords *)ctx->b_fxrec.p : nullptr,
            ctx->fx_c[0], ctx->fx_c[1], ctx->fx_c[2], ctx->fx_s);
    } else {
        k_publish_flag<<<1, 64, 0, ctx->stream>>>(flag, ctx->d_hflag, ctx->flag_seq_disp);
    }
    HIPCHK(ctx, hipGetLastError());
    ctx->dflag_zero = true;
    return MDLJ_OK;
}

mdlj_status build_halo_list(mdlj_ctx *ctx)
{
    const Grid &g = ctx->grid;
    const int key[6] = {g.n[0], g.n[1], g.n[2], g.h[0], g.h[1], g.h[2]};
    if (ctx->b_halo.p && memcmp(key, ctx->halo_key, sizeof key) == 0) return MDLJ_OK;
    std::vector<int2> hl;
    hl.reserve((size_t)(g.ncell_ext - g.ncell_int));
    for (int cz = -g.h[2]; cz < g.n[2] + g.h[2]; ++cz)
        for (int cy = -g.h[1]; cy < g.n[1] + g.h[1]; ++cy)
            for (int cx = -g.h[0]; cx < g.n[0] + g.h[0]; ++cx) {
                const int c[3] = {cx, cy, cz};
                bool halo = false;
                int64_t e = 0, src = 0;
                for (int a = 0; a < 3; ++a) {
                    int s = c[a];
                    if (s < 0) { s += g.n[a]; halo = true; }
                    if (s >= g.n[a]) { s -= g.n[a]; halo = true; }
                    e += (int64_t)(c[a] + g.h[a]) * g.stride[a];
                    src += (int64_t)(s + g.h[a]) * g.stride[a];
                }
                if (halo) hl.push_back(make_int2((int)e, (int)src));
            }
    ctx->nhalo = (int64_t)hl.size();
    memcpy(ctx->halo_key, key, sizeof key);
    if (hl.empty()) return MDLJ_OK;
    STCHK(ensure(ctx, ctx->b_halo, sizeof(int2) * hl.size()));
    HIPCHK(ctx, hipMemcpyAsync(ctx->b_halo.p, hl.data(), sizeof(int2) * hl.size(),
                               hipMemcpyHostToDevice, ctx->stream));
    // the host vector is released on return
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return MDLJ_OK;
}

mdlj_status refresh_records(mdlj_ctx *ctx)
{
    ctx->rec_at_build = false;
    ctx->fx_valid = false;
    k_refresh<<<ceil_div(ctx->n_ext, 256), 256, 0, ctx->stream>>>(
        ctx->n_ext, (PosT *)ctx->b_sorted.p, (const char4 *)ctx->b_img.p, ctx->x, ctx->y, ctx->z,
        ctx->box[0], ctx->box[1], ctx->box[2]);
    HIPCHK(ctx, hipGetLastError());
    return MDLJ_OK;
}

static InvMass inv_mass(const mdlj_ctx *ctx)
{
    InvMass im;
    for (int s = 0; s < MDLJ_MAX_SPECIES; ++s) im.v[s] = 1.0 / ctx->mass[s];
    return im;
}

static mdlj_status enter_sorted(mdlj_ctx *ctx)
{
    const int64_t n = ctx->n;
    STCHK(ensure(ctx, ctx->b_vsort, sizeof(double) * 3 * n));
    STCHK(ensure(ctx, ctx->b_vsort2, sizeof(double) * 3 * n));
    STCHK(ensure(ctx, ctx->b_xrsort, sizeof(double) * 3 * n));
    const bool carry = ctx->vs_old_order;
    k_enter_sorted<<<ceil_div(n, 256), 256, 0, ctx->stream>>>(
        n, (const int32_t *)ctx->b_ilist.p, (const PosT *)ctx->b_sorted.p, ctx->vv_v[0],
        ctx->vv_v[1], ctx->vv_v[2], (const int32_t *)ctx->b_tinv.p,
        carry ? (const double *)ctx->b_vsort.p : nullptr, (const double *)ctx->b_xref.p,
        ctx->rec_at_build ? 1 : 0, (double *)ctx->b_vsort2.p, (double *)ctx->b_xrsort.p);
    HIPCHK(ctx, hipGetLastError());
    std::swap(ctx->b_vsort, ctx->b_vsort2);
    ctx->vs_old_order = false;
    ctx->sorted_active = true;
    return MDLJ_OK;
}

mdlj_status leave_sorted(mdlj_ctx *ctx)
{
    const int64_t n = ctx->n;
    if (ctx->sorted_active) {
        ctx->sorted_active = false;
        k_leave_sorted<<<ceil_div(n, 256), 256, 0, ctx->stream>>>(
            n, (const int32_t *)ctx->b_ilist.p, (const PosT *)ctx->b_sorted.p,
            (const double *)ctx->b_vsort.p, ctx->x, ctx->y, ctx->z, ctx->vv_v[0], ctx->vv_v[1],
            ctx->vv_v[2]);
        HIPCHK(ctx, hipGetLastError());
    } else if (ctx->vs_old_order) {
        ctx->vs_old_order = false;
        k_leave_velocities<<<ceil_div(n, 256), 256, 0, ctx->stream>>>(
            n, (const int32_t *)ctx->b_tinv.p, (const double *)ctx->b_vsort.p, ctx->vv_v[0],
            ctx->vv_v[1], ctx->vv_v[2]);
        HIPCHK(ctx, hipGetLastError());
    }
    return MDLJ_OK;
}

mdlj_status enter_sorted_early(mdlj_ctx *ctx, const mdlj_config &c)
{
    if (!ctx->kd_req || ctx->sorted_active || c.nbr_algo != MDLJ_NBR_VL || !c.staged ||
        c.newton3 || ctx->rebuild_every < 2)
        return MDLJ_OK;
    // the records were just made from the positions the lists are built for
    ctx->rec_at_build = true;
    return enter_sorted(ctx);
}

mdlj_status positions_for_rebuild(mdlj_ctx *ctx)
{
    if (!ctx->sorted_active) return MDLJ_OK;
    const int64_t n = ctx->n;
    STCHK(ensure(ctx, ctx->b_tinv, sizeof(int32_t) * n));
    ctx->sorted_active = false;
    k_leave_positions<<<ceil_div(n, 256), 256, 0, ctx->stream>>>(
        n, (const int32_t *)ctx->b_ilist.p, (const PosT *)ctx->b_sorted.p, ctx->x, ctx->y, ctx->z,
        (int32_t *)ctx->b_tinv.p);
    HIPCHK(ctx, hipGetLastError());
    ctx->vs_old_order = true;
    return MDLJ_OK;
}

mdlj_status kd_prepare(mdlj_ctx *ctx, const mdlj_config &c, bool energy)
{
    const int64_t n = ctx->n;
    // as for the separate sorted-order step: lists kept for the next step
    // (the force call counts as a step since the build), and the forces
    // alone are asked for
    ctx->kd_go = ctx->kd_req && !energy && c.nbr_algo == MDLJ_NBR_VL && c.staged &&
                 !c.newton3 && ctx->built && ctx->built_cfg.nbr_algo == MDLJ_NBR_VL &&
                 ctx->built_cfg.staged && ctx->steps_since_build + 1 < ctx->rebuild_every &&
                 ctx->b_xref.bytes >= sizeof(double) * 3 * n;
    if (!ctx->kd_go) return MDLJ_OK;
    STCHK(ensure_host_flag(ctx));
    if (!ctx->sorted_active) STCHK(enter_sorted(ctx));
    return MDLJ_OK;
}

mdlj_status kd_args(mdlj_ctx *ctx, KickArgs *ka)
{
    STCHK(ensure(ctx, ctx->b_sorted2, sizeof(PosT) * (ctx->n_ext + 1)));
    int32_t *flag = (int32_t *)ctx->b_flags.p + 13;
    if (!ctx->dflag_zero) HIPCHK(ctx, hipMemsetAsync(flag, 0, sizeof(int32_t), ctx->stream));
    ctx->dflag_zero = false;
    ka->rec_out = (PosT *)ctx->b_sorted2.p;
    ka->vs_in = (const double *)ctx->b_vsort.p;
    ka->vs_out = (double *)ctx->b_vsort2.p;
    ka->xrs = (const double *)ctx->b_xrsort.p;
    ka->flag = flag;
    const InvMass im = inv_mass(ctx);
    for (int s = 0; s < MDLJ_MAX_SPECIES; ++s) ka->im[s] = im.v[s];
    ka->dt = ctx->kd_dt;
    const double h = 0.5 * ctx->skin;
    ka->thr2 = h * h;
    ka->pad_slot = ctx->n_ext;
    ka->thr_in2 = 0.0;  // set by the launch
    return MDLJ_OK;
}

static mdlj_status vv_loop(mdlj_ctx *ctx, double *vx, double *vy, double *vz, double dt,
                           int nsteps);

mdlj_status vv_steps(mdlj_ctx *ctx, double *vx, double *vy, double *vz, double dt, int nsteps)
{
    ctx->vv_v[0] = vx;
    ctx->vv_v[1] = vy;
    ctx->vv_v[2] = vz;
    const mdlj_status st = vv_loop(ctx, vx, vy, vz, dt, nsteps);
    ctx->kd_req = ctx->kd_go = ctx->kd_done = false;
    // on an error mid-loop the caller-order state is still made whole
    const mdlj_status st2 = leave_sorted(ctx);
    ctx->vv_v[0] = ctx->vv_v[1] = ctx->vv_v[2] = nullptr;
    return st != MDLJ_OK ? st : st2;
}

static mdlj_status vv_loop(mdlj_ctx *ctx, double *vx, double *vy, double *vz, double dt,
                           int nsteps)
{
    const int64_t n = ctx->n;
    const InvMass im = inv_mass(ctx);
    const int TB = 256;
    const int64_t nb = ceil_div(n, TB);
    if (nsteps == 0) return MDLJ_OK;
    if (!ctx->forces_valid) STCHK(forces_internal(ctx, ctx->pos_changed, nullptr));
    ctx->pos_changed = false;
    // first half kick and drift from the caller-order forces of x(t)
    k_kick_drift<<<nb, TB, 0, ctx->stream>>>(n, ctx->x, ctx->y, ctx->z, vx, vy, vz, ctx->fx,
                                             ctx->fy, ctx->fz, ctx->type, im, dt);
    HIPCHK(ctx, hipGetLastError());
    ctx->forces_valid = false;
    for (int s = 0; s < nsteps; ++s) {
        ForceOut fo;
        // all but the last step may continue in sorted order; the staged
        // Verlet-list kernel then takes the integrator step itself
        ctx->kd_req = s + 1 < nsteps;
        ctx->kd_dt = dt;
        STCHK(forces_internal(ctx, true, nullptr, &fo, false));
        ctx->kd_req = ctx->kd_go = false;
        if (ctx->kd_done) {
            ctx->kd_done = false;
            std::swap(ctx->b_sorted, ctx->b_sorted2);
            std::swap(ctx->b_vsort, ctx->b_vsort2);
            // the FP32-pair kernel wrote the interior records' fixed-point
            // words too (the halo refresh adds the images'); the FP64 one
            // did not
            if (ctx->kd_fx)
                std::swap(ctx->b_fxrec, ctx->b_fxrec2);
            else
                ctx->fx_valid = false;
            ctx->upkeep_fused = true;
            ctx->rec_at_build = false;
            continue;
        }
        const int32_t *slot_of = (const int32_t *)ctx->b_slot_of.p;
        // lists kept for the next step (and a context with the fused
        // upkeep state): positions, sorted records and the displacement test
        // in one pass
        const bool fuse = ctx->built && ctx->built_cfg.nbr_algo == MDLJ_NBR_VL &&
                          ctx->cfg.nbr_algo == MDLJ_NBR_VL &&
                          ctx->steps_since_build < ctx->rebuild_every && ctx->h_flag &&
                          ctx->b_xref.bytes >= sizeof(double) * 3 * n;
        if (s + 1 < nsteps && fuse) {
            if (!ctx->sorted_active) STCHK(enter_sorted(ctx));
            int32_t *flag = (int32_t *)ctx->b_flags.p + 13;
            const double h = 0.5 * ctx->skin;
            if (!ctx->dflag_zero) HIPCHK(ctx, hipMemsetAsync(flag, 0, sizeof(int32_t), ctx->stream));
            ctx->dflag_zero = false;
            k_kick_drift_compact<<<nb, TB, 0, ctx->stream>>>(
                n, (const int32_t *)ctx->b_ilist.p, (PosT *)ctx->b_sorted.p,
                (double *)ctx->b_vsort.p, fo.fx, fo.fy, fo.fz, im, dt,
                (const double *)ctx->b_xrsort.p, h * h, flag, inner_marker(ctx));
            inner_flip(ctx);
            ctx->upkeep_fused = true;
            ctx->rec_at_build = false;
            ctx->fx_valid = false;
            HIPCHK(ctx, hipGetLastError());
            continue;
        }
        if (s + 1 < nsteps && ctx->sorted_active) {
            // the next force call rebuilds the lists from caller-order
            // positions; the velocities wait in the old compact order
            STCHK(ensure(ctx, ctx->b_tinv, sizeof(int32_t) * n));
            ctx->sorted_active = false;
            k_kick_leave<<<nb, TB, 0, ctx->stream>>>(
                n, (const int32_t *)ctx->b_ilist.p, (const PosT *)ctx->b_sorted.p,
                (double *)ctx->b_vsort.p, fo.fx, fo.fy, fo.fz, im, dt, ctx->x, ctx->y, ctx->z,
                (int32_t *)ctx->b_tinv.p);
            HIPCHK(ctx, hipGetLastError());
            ctx->vs_old_order = true;
            continue;
        }
        STCHK(leave_sorted(ctx));
        if (s + 1 < nsteps) {
            k_kick_drift_sorted<<<nb, TB, 0, ctx->stream>>>(n, ctx->x, ctx->y, ctx->z, vx, vy, vz,
                                                            fo.fx, fo.fy, fo.fz, slot_of,
                                                            ctx->type, im, dt);
        } else {
            k_kick_sorted<<<nb, TB, 0, ctx->stream>>>(n, vx, vy, vz, fo.fx, fo.fy, fo.fz, slot_of,
                                                      ctx->type, im, dt, ctx->fx, ctx->fy,
                                                      ctx->fz);
        }
        HIPCHK(ctx, hipGetLastError());
    }
    ctx->forces_valid = true;
    return MDLJ_OK;
}
