// bin.hip -- counting-sort cell binning with periodic halo images.
//
// The linked-cell container (section 2.1.1: equal cells, a particle
// interacts with its own and the neighbouring cells) is stored as one
// sorted array of particle records.  Interior cells hold the particles of
// the box; the h outer layers of cells hold periodic images (shifted by
// +-L) of the interior cells they mirror, so force kernels read every
// neighbour cell as plain memory and never apply a minimum image.
//
// Steps: wrap + cell index + per-cell rank (atomics) -> exclusive scan of
// the extended cell counts -> scatter caller indices -> order each cell by
// caller index (so results do not depend on atomic order) -> fill records
// of interior and halo cells.
#include "atomics.h"
#include "internal.h"

namespace {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

// x - L floor(x / L), every operation rounded on its own (no FMA), so the
// cell decision is the same as a plain binary64 evaluation of the formula.
__device__ __forceinline__ double wrap_coord(double x, double L)
{
#pragma clang fp contract(off)
    double q = floor(x / L);
    double m = L * q;
    return x - m;
}

__device__ __forceinline__ int cell_coord(double xw, double inv, int n)
{
#pragma clang fp contract(off)
    double s = xw * inv;
    int c = (int)s;
    c = c >= n ? n - 1 : c;
    c = c < 0 ? 0 : c;
    return c;
}

// Interior source cell of an extended cell (identity for interior cells).
__device__ __forceinline__ int64_t source_cell(int64_t e, const Grid &g)
{
    int64_t src = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int c = (int)(((uint32_t)e / (uint32_t)g.stride[a]) % (uint32_t)g.e[a]) - g.h[a];
        int s = c % g.n[a];
        s = s < 0 ? s + g.n[a] : s;
        src += (int64_t)(s + g.h[a]) * g.stride[a];
    }
    return src;
}

// Also the binning flags (words 0-3) and the list build's maxima (12-15,
// which the build's publishing kernel clears again after each build).
__global__ void k_clear_bins(int32_t *__restrict__ count, int64_t ncell, int32_t *__restrict__ flags)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < ncell) count[e] = 0;
    if (e < 4 || (e >= 12 && e < 16)) flags[e] = 0;
}

__global__ void k_bin_count(int64_t n, double *__restrict__ x, double *__restrict__ y,
                            double *__restrict__ z, Grid g, int32_t *__restrict__ cell_of,
                            int32_t *__restrict__ rank, int32_t *__restrict__ count,
                            int32_t *__restrict__ flags)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & (MDLJ_WAVE - 1);
    bool valid = i < n;
    int32_t e = 0;
    if (valid) {
        double p[3] = {x[i], y[i], z[i]};
        if (!isfinite(p[0]) || !isfinite(p[1]) || !isfinite(p[2])) {
            atomicOr(&flags[0], 1);
            cell_of[i] = -1;
            rank[i] = 0;
            valid = false;
        } else {
            int64_t ee = 0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                double xw = wrap_coord(p[a], g.L[a]);
                int c = cell_coord(xw, g.inv[a], g.n[a]);
                ee += (int64_t)(c + g.h[a]) * g.stride[a];
                p[a] = xw;
            }
            x[i] = p[0];
            y[i] = p[1];
            z[i] = p[2];
            e = (int32_t)ee;
            cell_of[i] = e;
        }
    }
    // Lanes of a wavefront in the same cell take one atomic: the lowest lane
    // of a group adds the group's size and hands out the base (particles in
    // spatial order put a wavefront into a few cells).  Up to 16 groups are
    // formed; lanes left over add 1 each.  Ranks within a cell are a set of
    // distinct numbers in any order (the fill sorts each cell by its key).
    uint64_t todo = __builtin_amdgcn_ballot_w64(valid);
    int leader = lane, sub = 0, size = 1;
    for (int it = 0; it < 16 && todo != 0; ++it) {
        const int ld = __builtin_ctzll(todo);
        const int32_t el = __builtin_amdgcn_readlane(e, ld);
        const uint64_t grp = __builtin_amdgcn_ballot_w64(valid && e == el);
        if ((grp >> lane) & 1) {
            leader = ld;
            sub = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(grp >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)grp, 0u));
            size = __builtin_popcountll(grp);
        }
        todo &= ~grp;
    }
    int32_t base = 0;
    if (valid && leader == lane) base = atomicAdd(&count[e], size);
    base = __shfl(base, leader);
    if (valid) rank[i] = base + sub;
}

// Extended-cell counts: a halo cell holds as many records as its source.
// Also the largest occupancy, into flags[2] (one atomic per workgroup).
__global__ __launch_bounds__(256) void k_ext_counts(Grid g, const int32_t *__restrict__ count,
                                                    int32_t *__restrict__ cnt_ext,
                                                    int32_t *__restrict__ flags)
{
    __shared__ int32_t red[256 / MDLJ_WAVE];
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t m = 0;
    if (e < g.ncell_ext) {
        m = count[source_cell(e, g)];
        cnt_ext[e] = m;
    }
    for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o));
    if ((threadIdx.x & (MDLJ_WAVE - 1)) == 0) red[threadIdx.x / MDLJ_WAVE] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)blockDim.x / MDLJ_WAVE; ++w) m = max(m, red[w]);
        if (m > 0) atomic_max_rare(&flags[2], m);
    }
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_reduce(int64_t n,
                                                            const int32_t *__restrict__ in,
                                                            int32_t *__restrict__ part)
{
    __shared__ int32_t red[SCAN_BLOCK / MDLJ_WAVE];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t e = base + (int64_t)k * SCAN_BLOCK + threadIdx.x;
        if (e < n) s += in[e];
    }
    for (int o = MDLJ_WAVE / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & (MDLJ_WAVE - 1)) == 0) red[threadIdx.x / MDLJ_WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int w = 0; w < SCAN_BLOCK / MDLJ_WAVE; ++w) t += red[w];
        part[blockIdx.x] = t;
    }
}

// Exclusive scan of the per-tile sums in one workgroup; writes the total.
// Each thread sums a run of consecutive tiles; the 1024 run sums are
// scanned in parallel (lane prefix sums, then the 16 wavefront totals).
__global__ __launch_bounds__(1024) void k_scan_parts(int64_t nparts, int32_t *__restrict__ part,
                                                     int32_t *__restrict__ total)
{
    constexpr int NWV = 1024 / MDLJ_WAVE;
    __shared__ int32_t wsum[NWV];
    const int64_t per = ceil_div(nparts, 1024);
    const int64_t b = threadIdx.x * per;
    const int64_t e = b + per < nparts ? b + per : nparts;
    int32_t s = 0;
    for (int64_t k = b; k < e; ++k) s += part[k];
    const int lane = threadIdx.x & (MDLJ_WAVE - 1), wv = threadIdx.x / MDLJ_WAVE;
    int32_t inc = s;
    for (int o = 1; o < MDLJ_WAVE; o <<= 1) {
        const int32_t t = __shfl_up(inc, o);
        if (lane >= o) inc += t;
    }
    if (lane == MDLJ_WAVE - 1) wsum[wv] = inc;
    __syncthreads();
    int32_t woff = 0, all = 0;
    for (int w = 0; w < NWV; ++w) {
        const int32_t v = wsum[w];
        woff += w < wv ? v : 0;
        all += v;
    }
    if (threadIdx.x == 0) *total = all;
    int32_t run = woff + inc - s;
    for (int64_t k = b; k < e; ++k) {
        const int32_t v = part[k];
        part[k] = run;
        run += v;
    }
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_down(int64_t n,
                                                          const int32_t *__restrict__ in,
                                                          const int32_t *__restrict__ part,
                                                          int32_t *__restrict__ out)
{
    __shared__ int32_t wsum[SCAN_BLOCK / MDLJ_WAVE];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    int32_t v[SCAN_ITEMS];
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t e = base + k;
        v[k] = e < n ? in[e] : 0;
        s += v[k];
    }
    int lane = threadIdx.x & (MDLJ_WAVE - 1);
    int32_t inc = s;
    for (int o = 1; o < MDLJ_WAVE; o <<= 1) {
        int32_t t = __shfl_up(inc, o);
        if (lane >= o) inc += t;
    }
    if (lane == MDLJ_WAVE - 1) wsum[threadIdx.x / MDLJ_WAVE] = inc;
    __syncthreads();
    int32_t woff = 0;
    for (int w = 0; w < (int)(threadIdx.x / MDLJ_WAVE); ++w) woff += wsum[w];
    int32_t run = part[blockIdx.x] + woff + inc - s;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t e = base + k;
        if (e < n) out[e] = run;
        run += v[k];
    }
}

// Both kernels below write records up to the total *total (the end of the
// cell starts); when it exceeds cap, the records their buffers hold, they
// write nothing (the host grows the buffers and runs them again).
__global__ void k_scatter(int64_t n, const int32_t *__restrict__ cell_of,
                          const int32_t *__restrict__ rank, const int32_t *__restrict__ start,
                          int32_t *__restrict__ sorted_orig, const int32_t *__restrict__ total,
                          int64_t cap)
{
    if ((int64_t)*total > cap) return;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t e = cell_of[i];
    if (e < 0) return;
    sorted_orig[start[e] + rank[i]] = (int32_t)i;
}

// FILL_LANES lanes per extended cell (cells hold ~17 records at liquid
// densities, so a whole wavefront per cell would idle most lanes): interior
// cells gather their records, halo cells copy the records of their source
// cell shifted by +-L.  Within a cell records are ordered by the key
// (x half, caller index): first the particles in the lower half of the cell
// along x, then the upper half, each by caller index.  The order does not
// depend on the order in which the counting atomics were served: element m
// of the source cell's unordered list goes to slot b + (number of elements
// with a smaller key).  Halo cells rank their source's list the same way, so
// every image has the order of its source.  hstart[e] = first slot of the
// upper half (the list build uses the halves to drop candidates more than
// one cell away in x).
constexpr int FILL_LANES = 16;

__global__ __launch_bounds__(256) void k_fill(Grid g, const int32_t *__restrict__ start,
                                              const int32_t *__restrict__ unordered,
                                              const double *__restrict__ x,
                                              const double *__restrict__ y,
                                              const double *__restrict__ z,
                                              const int32_t *__restrict__ type,
                                              PosT *__restrict__ rec,
                                              int32_t *__restrict__ slot_of,
                                              char4 *__restrict__ img,
                                              int32_t *__restrict__ hstart, int64_t cap)
{
    if ((int64_t)start[g.ncell_ext] > cap) return;
    const int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / FILL_LANES;
    const int sub = threadIdx.x & (FILL_LANES - 1);
    // a group of lanes past the last cell has no records: every lane of a
    // group runs the same trips, so the shuffles below read only lanes of
    // the own group, all active
    const bool live = e < g.ncell_ext;
    int32_t b = 0, cnt = 0, sb = 0;
    double sh[3] = {0.0, 0.0, 0.0};
    signed char code[3] = {0, 0, 0};
    bool interior = true;
    int sx_cell = 0;
    if (live) {
        b = start[e];
        cnt = start[e + 1] - b;
        int64_t src = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            int c = (int)(((uint32_t)e / (uint32_t)g.stride[a]) % (uint32_t)g.e[a]) - g.h[a];
            int s = c;
            if (c < 0) { s = c + g.n[a]; sh[a] = -g.L[a]; code[a] = -1; interior = false; }
            if (c >= g.n[a]) { s = c - g.n[a]; sh[a] = g.L[a]; code[a] = 1; interior = false; }
            src += (int64_t)(s + g.h[a]) * g.stride[a];
            if (a == 0) sx_cell = s;
        }
        sb = start[src];
    }
    // caller indices are below 2^30: key = upper-half bit 31 | caller index
    const double xmid = ((double)sx_cell + 0.5) * g.edge[0];
    auto key_of = [&](int32_t i) {
        return (uint32_t)i | (x[i] < xmid ? 0u : 0x80000000u);
    };
    int32_t nlow = 0;
    for (int32_t m0 = 0; m0 < cnt; m0 += FILL_LANES) {
        const int32_t m = m0 + sub;
        const int32_t i = m < cnt ? unordered[sb + m] : 0;
        const uint32_t ki = m < cnt ? key_of(i) : 0xffffffffu;
        int32_t rank = 0;
        for (int32_t q0 = 0; q0 < cnt; q0 += FILL_LANES) {
            const int32_t vi = q0 + sub < cnt ? unordered[sb + q0 + sub] : 0;
            const uint32_t v = q0 + sub < cnt ? key_of(vi) : 0xffffffffu;
            const int32_t nq = min(cnt - q0, FILL_LANES);
            for (int32_t q = 0; q < nq; ++q) rank += __shfl(v, q, FILL_LANES) < ki;
        }
        if (m < cnt) {
            nlow += ki < 0x80000000u ? 1 : 0;
            const int32_t k = b + rank;
            PosT r;
            r.x = x[i] + sh[0];
            r.y = y[i] + sh[1];
            r.z = z[i] + sh[2];
            r.t = type[i];
            r.orig = i;
            rec[k] = r;
            img[k] = make_char4(code[0], code[1], code[2], 0);
            if (interior) slot_of[i] = k;
        }
    }
    // the group's count of lower-half records
#pragma unroll
    for (int o = FILL_LANES / 2; o > 0; o >>= 1) nlow += __shfl_xor(nlow, o, FILL_LANES);
    if (live && sub == 0) hstart[e] = b + nlow;
    // the padding record at slot n_ext, after the last cell: far outside the
    // box, no particle
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        PosT p;
        p.x = p.y = p.z = 1.0e7;
        p.t = 0;
        p.orig = -1;
        rec[start[g.ncell_ext]] = p;
    }
}


__global__ void k_unpermute(int64_t n, const int32_t *__restrict__ slot_of,
                            const double *__restrict__ fx, const double *__restrict__ fy,
                            const double *__restrict__ fz, double *__restrict__ ox,
                            double *__restrict__ oy, double *__restrict__ oz)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t s = slot_of[i];
    ox[i] = fx[s];
    oy[i] = fy[s];
    oz[i] = fz[s];
}

// Halo slots carry forces applied to images (Newton-3 kernels); add them
// onto the slot of the particle they copy.
__global__ void k_fold(int64_t n_ext, const PosT *__restrict__ rec,
                       const int32_t *__restrict__ slot_of, double *__restrict__ fx,
                       double *__restrict__ fy, double *__restrict__ fz)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_ext) return;
    const int32_t o = rec[k].orig;
    if (o < 0) return;
    int32_t s = slot_of[o];
    if (s == k) return;
    atomicAdd(&fx[s], fx[k]);
    atomicAdd(&fy[s], fy[k]);
    atomicAdd(&fz[s], fz[k]);
}

__global__ void k_zero3(int64_t n, double *__restrict__ a, double *__restrict__ b,
                        double *__restrict__ c)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    a[i] = 0.0;
    b[i] = 0.0;
    c[i] = 0.0;
}

__global__ __launch_bounds__(256) void k_reduce_partials(int64_t nb,
                                                         const double *__restrict__ part,
                                                         double *__restrict__ out)
{
    __shared__ double su[256], sw[256];
    double u = 0, w = 0;
    for (int64_t k = threadIdx.x; k < nb; k += 256) {
        u += part[2 * k];
        w += part[2 * k + 1];
    }
    su[threadIdx.x] = u;
    sw[threadIdx.x] = w;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            su[threadIdx.x] += su[threadIdx.x + o];
            sw[threadIdx.x] += sw[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = su[0];
        out[1] = sw[0];
    }
}

__global__ void k_finite(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                         const double *__restrict__ z, int32_t *__restrict__ flag)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (!isfinite(x[i]) || !isfinite(y[i]) || !isfinite(z[i])) atomicOr(flag, 1);
}

__global__ void k_types(int64_t n, const int32_t *__restrict__ t, int32_t ns,
                        int32_t *__restrict__ flag)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (t[i] < 0 || t[i] >= ns) atomicOr(flag, 1);
}

// Compact list of the real slots in sorted order (interior cells only).
__global__ void k_int_counts(Grid g, const int32_t *__restrict__ count, int32_t *__restrict__ icnt)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncell_int) return;
    int cx = (int)((uint32_t)c % (uint32_t)g.n[0]);
    int cy = (int)(((uint32_t)c / (uint32_t)g.n[0]) % (uint32_t)g.n[1]);
    int cz = (int)((uint32_t)c / ((uint32_t)g.n[0] * (uint32_t)g.n[1]));
    int64_t e = (int64_t)(cx + g.h[0]) * g.stride[0] + (int64_t)(cy + g.h[1]) * g.stride[1] +
                (int64_t)(cz + g.h[2]) * g.stride[2];
    icnt[c] = count[e];
}

// host[0] = non-finite flag, host[1] = records with halo images,
// host[2] = largest cell occupancy (system-scope stores to pinned memory)
__global__ void k_publish_bin(const int32_t *__restrict__ flags, const int32_t *__restrict__ total,
                              int32_t *host, uint32_t seq)
{
    if (threadIdx.x == 0) {
        __hip_atomic_store(host, flags[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(host + 1, *total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(host + 2, flags[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        // after the values: the host waits for this word
        __hip_atomic_store((uint32_t *)host + 3, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

__global__ void k_ilist(Grid g, const int32_t *__restrict__ start, const int32_t *__restrict__ ibase,
                        int32_t *__restrict__ ilist)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncell_int) return;
    int cx = (int)((uint32_t)c % (uint32_t)g.n[0]);
    int cy = (int)(((uint32_t)c / (uint32_t)g.n[0]) % (uint32_t)g.n[1]);
    int cz = (int)((uint32_t)c / ((uint32_t)g.n[0] * (uint32_t)g.n[1]));
    int64_t e = (int64_t)(cx + g.h[0]) * g.stride[0] + (int64_t)(cy + g.h[1]) * g.stride[1] +
                (int64_t)(cz + g.h[2]) * g.stride[2];
    int32_t b = start[e], en = start[e + 1], o = ibase[c];
    for (int32_t k = b; k < en; ++k) ilist[o + (k - b)] = k;
}

}  // namespace

mdlj_status exclusive_scan(mdlj_ctx *ctx, const int32_t *in, int32_t *out, int64_t n)
{
    int64_t nparts = ceil_div(n, SCAN_TILE);
    STCHK(ensure(ctx, ctx->b_scan_part, sizeof(int32_t) * (nparts > 0 ? nparts : 1)));
    int32_t *part = (int32_t *)ctx->b_scan_part.p;
    hipStream_t s = ctx->stream;
    if (n > 0) k_scan_reduce<<<nparts, SCAN_BLOCK, 0, s>>>(n, in, part);
    k_scan_parts<<<1, 1024, 0, s>>>(nparts, part, out + n);
    if (n > 0) k_scan_down<<<nparts, SCAN_BLOCK, 0, s>>>(n, in, part, out);
    HIPCHK(ctx, hipGetLastError());
    return MDLJ_OK;
}

mdlj_status build_ilist(mdlj_ctx *ctx, const Grid &g)
{
    STCHK(ensure(ctx, ctx->b_icnt, sizeof(int32_t) * (g.ncell_int + 1) * 2));
    STCHK(ensure(ctx, ctx->b_ilist, sizeof(int32_t) * ctx->n));
    int32_t *icnt = (int32_t *)ctx->b_icnt.p;
    int32_t *ibase = icnt + g.ncell_int + 1;
    const int TB = 256;
    k_int_counts<<<ceil_div(g.ncell_int, TB), TB, 0, ctx->stream>>>(g, (const int32_t *)ctx->b_count.p,
                                                                    icnt);
    STCHK(exclusive_scan(ctx, icnt, ibase, g.ncell_int));
    k_ilist<<<ceil_div(g.ncell_int, TB), TB, 0, ctx->stream>>>(g, (const int32_t *)ctx->b_start.p,
                                                               ibase, (int32_t *)ctx->b_ilist.p);
    HIPCHK(ctx, hipGetLastError());
    return MDLJ_OK;
}

mdlj_status check_types(mdlj_ctx *ctx, bool *ok)
{
    STCHK(ensure(ctx, ctx->b_flags, sizeof(int32_t) * 64));
    int32_t *flag = (int32_t *)ctx->b_flags.p + 9;
    HIPCHK(ctx, hipMemsetAsync(flag, 0, sizeof(int32_t), ctx->stream));
    k_types<<<ceil_div(ctx->n, 256), 256, 0, ctx->stream>>>(ctx->n, ctx->type, ctx->nspec, flag);
    HIPCHK(ctx, hipGetLastError());
    int32_t h = 0;
    HIPCHK(ctx, hipMemcpyAsync(&h, flag, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    *ok = (h == 0);
    return MDLJ_OK;
}

bool make_grid(const double *L, const double *r_min, const int *h, bool z_fastest, Grid *g)
{
    for (int a = 0; a < 3; ++a) {
        int n = (int)floor(L[a] / r_min[a]);
        if (n < 1) return false;
        g->n[a] = n;
        g->h[a] = h[a];
        g->e[a] = n + 2 * h[a];
        g->L[a] = L[a];
        g->inv[a] = (double)n / L[a];
        g->edge[a] = L[a] / (double)n;
    }
    if (z_fastest) {
        g->stride[2] = 1;
        g->stride[0] = g->e[2];
        g->stride[1] = (int64_t)g->e[2] * g->e[0];
    } else {
        g->stride[0] = 1;
        g->stride[1] = g->e[0];
        g->stride[2] = (int64_t)g->e[0] * g->e[1];
    }
    g->ncell_ext = (int64_t)g->e[0] * g->e[1] * g->e[2];
    g->ncell_int = (int64_t)g->n[0] * g->n[1] * g->n[2];
    return true;
}

mdlj_status bin_particles(mdlj_ctx *ctx, const Grid &g, bool interior_list)
{
    const int64_t n = ctx->n;
    if (g.ncell_ext >= (int64_t)1 << 31) return set_err(ctx, MDLJ_ERR_GEOMETRY, "too many cells");
    STCHK(ensure(ctx, ctx->b_cell_of, sizeof(int32_t) * n));
    STCHK(ensure(ctx, ctx->b_rank, sizeof(int32_t) * n));
    STCHK(ensure(ctx, ctx->b_count, sizeof(int32_t) * g.ncell_ext));
    STCHK(ensure(ctx, ctx->b_start, sizeof(int32_t) * (g.ncell_ext + 1)));
    STCHK(ensure(ctx, ctx->b_slot_of, sizeof(int32_t) * n));
    STCHK(ensure(ctx, ctx->b_flags, sizeof(int32_t) * 64));
    STCHK(ensure(ctx, ctx->b_cnt_ext, sizeof(int32_t) * g.ncell_ext));
    int32_t *count = (int32_t *)ctx->b_count.p;
    int32_t *start = (int32_t *)ctx->b_start.p;
    int32_t *flags = (int32_t *)ctx->b_flags.p;
    hipStream_t s = ctx->stream;
    // cell counts and the four binning flags cleared in one launch
    k_clear_bins<<<ceil_div(g.ncell_ext, 256), 256, 0, s>>>(count, g.ncell_ext, flags);
    const int TB = 256;
    k_bin_count<<<ceil_div(n, TB), TB, 0, s>>>(n, ctx->x, ctx->y, ctx->z, g,
                                                 (int32_t *)ctx->b_cell_of.p,
                                                 (int32_t *)ctx->b_rank.p, count, flags);
    k_ext_counts<<<ceil_div(g.ncell_ext, TB), TB, 0, s>>>(g, count, (int32_t *)ctx->b_cnt_ext.p,
                                                  flags);
    HIPCHK(ctx, hipGetLastError());
    STCHK(exclusive_scan(ctx, (const int32_t *)ctx->b_cnt_ext.p, start, g.ncell_ext));
    HIPCHK(ctx, hipGetLastError());
    // the compact interior order needs only the counts and cell starts:
    // queued before the wait below, so that it runs while the host waits
    if (interior_list) STCHK(build_ilist(ctx, g));
    // the records' scatter and fill, queued before the wait below when the
    // buffers of the last binning hold at least the particles and their
    // earlier number of images (they check the actual total themselves);
    // the halo starts and slot map have sizes known here
    STCHK(ensure(ctx, ctx->b_hstart, sizeof(int32_t) * g.ncell_ext));
    int64_t cap = std::min<int64_t>({(int64_t)(ctx->b_sorted.bytes / sizeof(PosT)) - 1,
                                     (int64_t)(ctx->b_misc.bytes / sizeof(int32_t)),
                                     (int64_t)(ctx->b_img.bytes / sizeof(char4))});
    const int32_t *total = start + g.ncell_ext;
    auto scatter_fill = [&]() -> mdlj_status {
        k_scatter<<<ceil_div(n, TB), TB, 0, s>>>(n, (int32_t *)ctx->b_cell_of.p,
                                                  (int32_t *)ctx->b_rank.p, start,
                                                  (int32_t *)ctx->b_misc.p, total, cap);
        k_fill<<<ceil_div(g.ncell_ext, TB / FILL_LANES), TB, 0, s>>>(
            g, start, (const int32_t *)ctx->b_misc.p, ctx->x, ctx->y, ctx->z, ctx->type,
            (PosT *)ctx->b_sorted.p, (int32_t *)ctx->b_slot_of.p, (char4 *)ctx->b_img.p,
            (int32_t *)ctx->b_hstart.p, cap);
        HIPCHK(ctx, hipGetLastError());
        return MDLJ_OK;
    };
    // non-finite flag, record total and largest occupancy to the host in
    // one small kernel, ahead of the scatter and fill, so that the host
    // can go on while they run
    STCHK(ensure_host_flag(ctx));
    const uint32_t seq = ++ctx->flag_seq;
    k_publish_bin<<<1, 64, 0, s>>>(flags, start + g.ncell_ext, ctx->d_hflag + 4, seq);
    HIPCHK(ctx, hipGetLastError());
    const bool early = cap >= n;
    if (early) STCHK(scatter_fill());
    STCHK(wait_host_words(ctx, 7, seq));
    const int32_t host[3] = {ctx->h_flag[4], ctx->h_flag[5], ctx->h_flag[6]};
    if (host[0]) return set_err(ctx, MDLJ_ERR_NONFINITE, "non-finite particle position");
    const int64_t n_ext = host[1];
    if (n_ext < n) return set_err(ctx, MDLJ_ERR_HIP, "binning lost particles");
    ctx->max_cell = host[2];
    if (!early || n_ext > cap) {
        STCHK(ensure(ctx, ctx->b_sorted, sizeof(PosT) * (n_ext + 1)));
        STCHK(ensure(ctx, ctx->b_misc, sizeof(int32_t) * n_ext));
        STCHK(ensure(ctx, ctx->b_img, sizeof(char4) * n_ext));
        cap = n_ext;
        STCHK(scatter_fill());
    }
    ctx->fx_valid = false;
    HIPCHK(ctx, hipGetLastError());
    ctx->grid = g;
    ctx->n_ext = n_ext;
    return MDLJ_OK;
}

mdlj_status fold_forces(mdlj_ctx *ctx, const ForceOut &fo)
{
    const int TB = 256;
    k_fold<<<ceil_div(ctx->n_ext, TB), TB, 0, ctx->stream>>>(
        ctx->n_ext, (const PosT *)ctx->b_sorted.p, (const int32_t *)ctx->b_slot_of.p, fo.fx, fo.fy,
        fo.fz);
    HIPCHK(ctx, hipGetLastError());
    return MDLJ_OK;
}

mdlj_status unpermute_forces(mdlj_ctx *ctx, const ForceOut &fo, double *ox, double *oy, double *oz)
{
    const int TB = 256;
    k_unpermute<<<ceil_div(ctx->n, TB), TB, 0, ctx->stream>>>(ctx->n, (const int32_t *)ctx->b_slot_of.p,
                                                              fo.fx, fo.fy, fo.fz, ox, oy, oz);
    HIPCHK(ctx, hipGetLastError());
    return MDLJ_OK;
}

mdlj_status zero_forces(mdlj_ctx *ctx, const ForceOut &fo, int64_t nslots)
{
    const int TB = 256;
    k_zero3<<<ceil_div(nslots, TB), TB, 0, ctx->stream>>>(nslots, fo.fx, fo.fy, fo.fz);
    HIPCHK(ctx, hipGetLastError());
    return MDLJ_OK;
}

mdlj_status reduce_partials(mdlj_ctx *ctx, const double *partial, int64_t nblocks,
                            double *UW_host)
{
    double *out = (double *)ctx->b_flags.p + 16;  // bytes 128..143 of the flag block
    k_reduce_partials<<<1, 256, 0, ctx->stream>>>(nblocks, partial, out);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipMemcpyAsync(UW_host, out, 2 * sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return MDLJ_OK;
}

mdlj_status check_finite(mdlj_ctx *ctx, const double *x, const double *y, const double *z,
                         int64_t n, bool *ok)
{
    STCHK(ensure(ctx, ctx->b_flags, sizeof(int32_t) * 64));
    int32_t *flag = (int32_t *)ctx->b_flags.p + 8;
    HIPCHK(ctx, hipMemsetAsync(flag, 0, sizeof(int32_t), ctx->stream));
    k_finite<<<ceil_div(n, 256), 256, 0, ctx->stream>>>(n, x, y, z, flag);
    HIPCHK(ctx, hipGetLastError());
    int32_t h = 0;
    HIPCHK(ctx, hipMemcpyAsync(&h, flag, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    *ok = (h == 0);
    return MDLJ_OK;
}
