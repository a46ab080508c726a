// vl.hip -- Verlet lists (section 2.1.1): per-particle lists of partners
// within rc + skin, built from linked cells of edge >= rc + skin and reused
// for several steps.  With Newton-3 (section 2.1) a pair is stored once
// (on the particle with the smaller caller index) and F_ji = -F_ij is
// applied with atomics.
//
// Two layouts, one per interaction order:
//   i-per-lane (VectorLength/1): lane t owns i; entry k of every list is
//     stored at nbr[k * n + t] so the 64 lanes of a wavefront read one
//     coalesced row per step.
//   wave-per-i (1/VectorLength): 64/g lanes share one i and stride along
//     its list, stored contiguously at nbr[t * cap + k]; the lanes' partial
//     forces are then summed over the segment.
// Lists index the sorted records, halo images included, so no minimum
// image is applied in the force loop.
#include "pair.h"

namespace {

// candidates per trip of the force loops
constexpr int UNROLL = 4;

// One lane per particle: walk the nine rows of three cells around its cell
// and append every partner within rc + skin.  Lanes of a wavefront are
// consecutive sorted particles (one or two cells), so their j-reads overlap.
__global__ __launch_bounds__(256) void k_vl_build(const PosT *__restrict__ rec,
                                                  const int32_t *__restrict__ start,
                                                  const int32_t *__restrict__ ilist,
                                                  const int32_t *__restrict__ cell_of, Grid g,
                                                  int64_t n, double rl2, int half, int64_t sk,
                                                  int64_t st, int32_t cap,
                                                  int32_t *__restrict__ nbr,
                                                  int32_t *__restrict__ len,
                                                  int32_t *__restrict__ maxlen)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t cnt = 0;
    if (t < n) {
        const int32_t i = ilist[t];
        const PosT pi = rec[i];
        const int64_t e = cell_of[pi.orig];
        int32_t *out = nbr + t * st;
        for (int r = 0; r < 9; ++r) {
            const int dy = r % 3 - 1, dz = r / 3 - 1;
            const int64_t ej = e + dy * g.stride[1] + dz * g.stride[2] - 1;
            const int32_t jb = start[ej], je = start[ej + 3];
            for (int32_t j = jb; j < je; ++j) {
                const PosT pj = rec[j];
                const double dx = pi.x - pj.x, dyy = pi.y - pj.y, dzz = pi.z - pj.z;
                const bool in = (j != i) && (dx * dx + dyy * dyy + dzz * dzz < rl2) &&
                                (!half || pj.orig > pi.orig);
                if (in) {
                    if (cnt < cap) out[(int64_t)cnt * sk] = j;
                    ++cnt;
                }
            }
        }
        len[t] = cnt;
    }
    // longest list of the wavefront, one atomic per wavefront
    for (int o = 32; o > 0; o >>= 1) cnt = max(cnt, __shfl_xor(cnt, o));
    if ((threadIdx.x & (MDLJ_WAVE - 1)) == 0 && cnt > 0) atomicMax(maxlen, cnt);
}

// i-per-lane over ELL lists.
template <typename T, bool E, bool MS, bool N3>
__global__ __launch_bounds__(256) void k_vl_ipl(const PosT *__restrict__ rec,
                                                const int32_t *__restrict__ ilist,
                                                const int32_t *__restrict__ nbr,
                                                const int32_t *__restrict__ len, int64_t n,
                                                LJTable<T> tab, ForceOut fo, int remap)
{
    __shared__ LdsTable<T> lt;
    const double rc2 = tab.rc2d;
    if (MS) {
        lds_table_load(lt, tab, threadIdx.x, blockDim.x);
        __syncthreads();
    }
    const int64_t b = remap ? xcd_remap(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    const int64_t t = b * blockDim.x + threadIdx.x;
    Acc a;
    acc_zero(a);
    if (t < n) {
        const int32_t i = ilist[t];
        const PosT pi = rec[i];
        const int32_t L = len[t];
        // U candidates per trip: their index and record loads are in flight together
        for (int32_t k0 = 0; k0 < L; k0 += UNROLL) {
            int32_t jj[UNROLL];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u)
                jj[u] = k0 + u < L ? nbr[(int64_t)(k0 + u) * n + t] : -1;
            PosT pj[UNROLL];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) pj[u] = rec[jj[u] >= 0 ? jj[u] : i];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                const PairP<T> p = pair_params<T, MS>(tab, lt, pi.t, pj[u].t);
                double fxp, fyp, fzp;
                lj_pair<T, E>(pi.x, pi.y, pi.z, pj[u].x, pj[u].y, pj[u].z, jj[u] >= 0, p, rc2, a,
                              fxp, fyp, fzp);
                if (N3 && jj[u] >= 0) {
                    atomicAdd(&fo.fx[jj[u]], -fxp);
                    atomicAdd(&fo.fy[jj[u]], -fyp);
                    atomicAdd(&fo.fz[jj[u]], -fzp);
                }
            }
        }
        if (N3) {
            atomicAdd(&fo.fx[i], a.fx);
            atomicAdd(&fo.fy[i], a.fy);
            atomicAdd(&fo.fz[i], a.fz);
        } else {
            fo.fx[i] = a.fx;
            fo.fy[i] = a.fy;
            fo.fz[i] = a.fz;
        }
    }
    if (E)
        wave_partial(a.u, a.w, N3 ? 1.0 : 0.5, fo.partial,
                     (int64_t)blockIdx.x * (blockDim.x / MDLJ_WAVE) + threadIdx.x / MDLJ_WAVE);
}

// g i's per wavefront, 64/g lanes per i, row-major lists.
template <typename T, bool E, bool MS, bool N3, int G>
__global__ __launch_bounds__(256) void k_vl_wpi(const PosT *__restrict__ rec,
                                                const int32_t *__restrict__ ilist,
                                                const int32_t *__restrict__ nbr,
                                                const int32_t *__restrict__ len, int64_t n,
                                                int32_t cap, LJTable<T> tab, ForceOut fo,
                                                int remap)
{
    constexpr int SEG = MDLJ_WAVE / G;
    __shared__ LdsTable<T> lt;
    const double rc2 = tab.rc2d;
    if (MS) {
        lds_table_load(lt, tab, threadIdx.x, blockDim.x);
        __syncthreads();
    }
    const int64_t b = remap ? xcd_remap(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    const int lane = threadIdx.x & (MDLJ_WAVE - 1);
    const int64_t wave = b * (blockDim.x / MDLJ_WAVE) + threadIdx.x / MDLJ_WAVE;
    const int64_t t = wave * G + lane / SEG;
    const int l = lane % SEG;
    Acc a;
    acc_zero(a);
    int32_t i = 0;
    if (t < n) {
        i = ilist[t];
        const PosT pi = rec[i];
        const int32_t L = len[t];
        const int32_t *row = nbr + t * cap;
        for (int32_t k0 = l; k0 < L; k0 += UNROLL * SEG) {
            int32_t jj[UNROLL];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) jj[u] = k0 + u * SEG < L ? row[k0 + u * SEG] : -1;
            PosT pj[UNROLL];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) pj[u] = rec[jj[u] >= 0 ? jj[u] : i];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                const PairP<T> p = pair_params<T, MS>(tab, lt, pi.t, pj[u].t);
                double fxp, fyp, fzp;
                lj_pair<T, E>(pi.x, pi.y, pi.z, pj[u].x, pj[u].y, pj[u].z, jj[u] >= 0, p, rc2, a,
                              fxp, fyp, fzp);
                if (N3 && jj[u] >= 0) {
                    atomicAdd(&fo.fx[jj[u]], -fxp);
                    atomicAdd(&fo.fy[jj[u]], -fyp);
                    atomicAdd(&fo.fz[jj[u]], -fzp);
                }
            }
        }
    }
    a.fx = seg_sum(a.fx, SEG);
    a.fy = seg_sum(a.fy, SEG);
    a.fz = seg_sum(a.fz, SEG);
    if (t < n && l == 0) {
        if (N3) {
            atomicAdd(&fo.fx[i], a.fx);
            atomicAdd(&fo.fy[i], a.fy);
            atomicAdd(&fo.fz[i], a.fz);
        } else {
            fo.fx[i] = a.fx;
            fo.fy[i] = a.fy;
            fo.fz[i] = a.fz;
        }
    }
    if (E)
        wave_partial(a.u, a.w, N3 ? 1.0 : 0.5, fo.partial,
                     (int64_t)blockIdx.x * (blockDim.x / MDLJ_WAVE) + threadIdx.x / MDLJ_WAVE);
}

template <typename T, bool E, bool MS, bool N3>
int64_t launch_vl(mdlj_ctx *ctx, const mdlj_config &cfg, const LJTable<T> &tab, ForceOut &fo,
                  int remap)
{
    const int64_t n = ctx->n;
    const PosT *rec = (const PosT *)ctx->b_sorted.p;
    const int32_t *ilist = (const int32_t *)ctx->b_ilist.p;
    const int32_t *nbr = (const int32_t *)ctx->b_nbr.p;
    const int32_t *len = (const int32_t *)ctx->b_nlen.p;
    hipStream_t s = ctx->stream;
    const int TB = 256;
    if (cfg.order == MDLJ_ORD_I_PER_LANE) {
        const int64_t nb = ceil_div(n, TB);
        k_vl_ipl<T, E, MS, N3><<<nb, TB, 0, s>>>(rec, ilist, nbr, len, n, tab, fo, remap);
        return nb * (TB / MDLJ_WAVE);
    }
    const int32_t cap = (int32_t)ctx->nbr_cap;
    const int64_t waves = ceil_div(n, cfg.tile_i);
    const int64_t nb = ceil_div(waves, TB / MDLJ_WAVE);
    switch (cfg.tile_i) {
    case 1: k_vl_wpi<T, E, MS, N3, 1><<<nb, TB, 0, s>>>(rec, ilist, nbr, len, n, cap, tab, fo, remap); break;
    case 2: k_vl_wpi<T, E, MS, N3, 2><<<nb, TB, 0, s>>>(rec, ilist, nbr, len, n, cap, tab, fo, remap); break;
    case 4: k_vl_wpi<T, E, MS, N3, 4><<<nb, TB, 0, s>>>(rec, ilist, nbr, len, n, cap, tab, fo, remap); break;
    case 8: k_vl_wpi<T, E, MS, N3, 8><<<nb, TB, 0, s>>>(rec, ilist, nbr, len, n, cap, tab, fo, remap); break;
    default: return -1;
    }
    return nb * (TB / MDLJ_WAVE);
}

template <typename T, bool E, bool MS>
int64_t launch_vl_n3(mdlj_ctx *ctx, const mdlj_config &cfg, const LJTable<T> &tab, ForceOut &fo,
                     int remap)
{
    if (cfg.newton3) return launch_vl<T, E, MS, true>(ctx, cfg, tab, fo, remap);
    return launch_vl<T, E, MS, false>(ctx, cfg, tab, fo, remap);
}

template <typename T>
mdlj_status vl_forces_t(mdlj_ctx *ctx, const mdlj_config &cfg, bool energy, ForceOut &fo,
                        int64_t *nblocks)
{
    LJTable<T> tab;
    fill_table<T>(ctx, &tab);
    const bool ms = ctx->nspec > 1;
    const int remap = 1;
    if (cfg.newton3) STCHK(zero_forces(ctx, fo, ctx->n_ext));
    int64_t nw;
    if (energy) {
        const int64_t maxw = ctx->n + 64;  // >= waves of every launch shape
        STCHK(ensure(ctx, ctx->b_partial, sizeof(double) * 2 * maxw));
        fo.partial = (double *)ctx->b_partial.p;
        nw = ms ? launch_vl_n3<T, true, true>(ctx, cfg, tab, fo, remap)
                : launch_vl_n3<T, true, false>(ctx, cfg, tab, fo, remap);
    } else {
        nw = ms ? launch_vl_n3<T, false, true>(ctx, cfg, tab, fo, remap)
                : launch_vl_n3<T, false, false>(ctx, cfg, tab, fo, remap);
    }
    if (nw < 0) return set_err(ctx, MDLJ_ERR_ARG, "unsupported Verlet-list shape");
    HIPCHK(ctx, hipGetLastError());
    *nblocks = nw;
    return MDLJ_OK;
}

}  // namespace

mdlj_status vl_build(mdlj_ctx *ctx, const mdlj_config &cfg)
{
    const Grid &g = ctx->grid;
    const int64_t n = ctx->n;
    STCHK(build_ilist(ctx));
    const double rl = ctx->rc + ctx->skin;
    const double vol = ctx->box[0] * ctx->box[1] * ctx->box[2];
    const double est = (double)n / vol * 4.18879020478639 * rl * rl * rl * (cfg.newton3 ? 0.5 : 1.0);
    int64_t cap = (int64_t)(1.3 * est) + 16;
    if (ctx->nbr_cap > cap && ctx->built_cfg.newton3 == cfg.newton3) cap = ctx->nbr_cap;
    cap = (cap + 3) & ~(int64_t)3;
    STCHK(ensure(ctx, ctx->b_nlen, sizeof(int32_t) * n));
    int32_t *maxlen = (int32_t *)ctx->b_flags.p + 12;
    const bool rowmajor = cfg.order != MDLJ_ORD_I_PER_LANE;
    for (int attempt = 0; attempt < 3; ++attempt) {
        if ((double)cap * (double)n * 4.0 > 64e9) return set_err(ctx, MDLJ_ERR_OVERFLOW, "Verlet lists too large");
        STCHK(ensure(ctx, ctx->b_nbr, sizeof(int32_t) * n * cap));
        HIPCHK(ctx, hipMemsetAsync(maxlen, 0, sizeof(int32_t), ctx->stream));
        const int64_t sk = rowmajor ? 1 : n;
        const int64_t st = rowmajor ? cap : 1;
        k_vl_build<<<ceil_div(n, 256), 256, 0, ctx->stream>>>(
            (const PosT *)ctx->b_sorted.p, (const int32_t *)ctx->b_start.p,
            (const int32_t *)ctx->b_ilist.p, (const int32_t *)ctx->b_cell_of.p, g, n, rl * rl,
            cfg.newton3 ? 1 : 0, sk, st, (int32_t)cap, (int32_t *)ctx->b_nbr.p,
            (int32_t *)ctx->b_nlen.p, maxlen);
        HIPCHK(ctx, hipGetLastError());
        int32_t hmax = 0;
        HIPCHK(ctx, hipMemcpyAsync(&hmax, maxlen, sizeof hmax, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        ctx->vl_max = hmax;
        if (hmax <= cap) {
            ctx->nbr_cap = cap;
            return MDLJ_OK;
        }
        cap = ((int64_t)(hmax * 1.1) + 8 + 3) & ~(int64_t)3;
    }
    return set_err(ctx, MDLJ_ERR_OVERFLOW, "Verlet list capacity could not be grown");
}

mdlj_status vl_forces(mdlj_ctx *ctx, const mdlj_config &cfg, bool energy, ForceOut &fo,
                      int64_t *nblocks)
{
    if (ctx->prec == MDLJ_PREC_F64) return vl_forces_t<double>(ctx, cfg, energy, fo, nblocks);
    return vl_forces_t<float>(ctx, cfg, energy, fo, nblocks);
}
