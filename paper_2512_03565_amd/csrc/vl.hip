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
#include <algorithm>

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
                                                  int64_t st, int32_t cap, int32_t pad,
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
            for (int32_t j0 = jb; j0 < je; j0 += UNROLL) {
                PosT pj[UNROLL];
#pragma unroll
                for (int u = 0; u < UNROLL; ++u) pj[u] = rec[j0 + u < je ? j0 + u : jb];
#pragma unroll
                for (int u = 0; u < UNROLL; ++u) {
                    const int32_t j = j0 + u;
                    const double dx = pi.x - pj[u].x, dyy = pi.y - pj[u].y, dzz = pi.z - pj[u].z;
                    const bool in = j < je && (j != i) &&
                                    (dx * dx + dyy * dyy + dzz * dzz < rl2) &&
                                    (!half || pj[u].orig > pi.orig);
                    if (in) {
                        if (cnt < cap) out[(int64_t)cnt * sk] = j;
                        ++cnt;
                    }
                }
            }
        }
        // pad to a multiple of 8 with the padding record (slot pad)
        for (int32_t k = cnt; k < ((cnt + 7) & ~7) && k < cap; ++k) out[(int64_t)k * sk] = pad;
        len[t] = cnt;
    }
    // longest list of the wavefront, one atomic per wavefront
    for (int o = 32; o > 0; o >>= 1) cnt = max(cnt, __shfl_xor(cnt, o));
    if ((threadIdx.x & (MDLJ_WAVE - 1)) == 0 && cnt > 0) atomicMax(maxlen, cnt);
}

// Lists for the staged kernel: entry = index of j in the concatenation of
// the nine neighbour rows of i's x-tile (STAGE_K consecutive cells along x
// and one halo cell either side), the order in which the force kernel
// stages them into LDS; 16 bits, row-major per i, padded to a multiple of 8
// with the index one past the staged particles (a far-away padding entry).
constexpr int STAGE_K = 4;

__global__ __launch_bounds__(256) void k_vl_build_local(const PosT *__restrict__ rec,
                                                        const int32_t *__restrict__ start,
                                                        const int32_t *__restrict__ ilist,
                                                        const int32_t *__restrict__ cell_of,
                                                        Grid g, int64_t n, double rl2,
                                                        int32_t cap, uint16_t *__restrict__ nbr,
                                                        int32_t *__restrict__ len,
                                                        int32_t *__restrict__ maxlen,
                                                        int32_t *__restrict__ maxnb)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t cnt = 0, base = 0;
    if (t < n) {
        const int32_t i = ilist[t];
        const PosT pi = rec[i];
        const int64_t e = cell_of[pi.orig];
        // x-tile of i's cell
        const int cx = (int)(e % g.stride[1]) - g.h[0];
        const int cx0 = (cx / STAGE_K) * STAGE_K;
        const int ncx = min(STAGE_K, g.n[0] - cx0);
        const int64_t erow = e - (cx + g.h[0]);  // first cell of i's x-row
        uint16_t *out = nbr + t * cap;
        for (int r = 0; r < 9; ++r) {
            const int dy = r % 3 - 1, dz = r / 3 - 1;
            const int64_t et = erow + dy * g.stride[1] + dz * g.stride[2] + cx0 - 1 + g.h[0];
            const int32_t tb = start[et], te = start[et + ncx + 2];
            // only i's own 3 cells of this row can hold partners
            const int64_t ej = e + dy * g.stride[1] + dz * g.stride[2] - 1;
            const int32_t jb = start[ej], je = start[ej + 3];
            for (int32_t j0 = jb; j0 < je; j0 += UNROLL) {
                PosT pj[UNROLL];
#pragma unroll
                for (int u = 0; u < UNROLL; ++u) pj[u] = rec[j0 + u < je ? j0 + u : jb];
#pragma unroll
                for (int u = 0; u < UNROLL; ++u) {
                    const int32_t j = j0 + u;
                    const double dx = pi.x - pj[u].x, dyy = pi.y - pj[u].y, dzz = pi.z - pj[u].z;
                    if (j < je && j != i && dx * dx + dyy * dyy + dzz * dzz < rl2) {
                        if (cnt < cap) out[cnt] = (uint16_t)(base + (j - tb));
                        ++cnt;
                    }
                }
            }
            base += te - tb;
        }
        for (int32_t k = cnt; k < ((cnt + 7) & ~7) && k < cap; ++k) out[k] = (uint16_t)base;
        len[t] = cnt;
    }
    for (int o = 32; o > 0; o >>= 1) {
        cnt = max(cnt, __shfl_xor(cnt, o));
        base = max(base, __shfl_xor(base, o));
    }
    if ((threadIdx.x & (MDLJ_WAVE - 1)) == 0) {
        if (cnt > 0) atomicMax(maxlen, cnt);
        if (base > 0) atomicMax(maxnb, base);
    }
}

// Staged wave-per-i: a workgroup of 4 wavefronts owns STAGE_K consecutive
// cells along x and copies their common neighbourhood (nine rows of
// STAGE_K + 2 cells) into LDS; its wavefronts then take g i's at a time,
// 64/g lanes per i, each lane reading V list entries per trip (one 16-, 8-
// or 4-byte load) and the j-particles from LDS.
template <typename T, bool E, bool MS, int G, int V>
__global__ __launch_bounds__(256) void k_vl_lds(const PosT *__restrict__ rec,
                                                const int32_t *__restrict__ start,
                                                const int32_t *__restrict__ ibase, Grid g,
                                                int tiles_x, const uint16_t *__restrict__ nbr,
                                                const int32_t *__restrict__ len, int32_t cap,
                                                int cmax, LJTable<T> tab, ForceOut fo, int remap)
{
    constexpr int SEG = MDLJ_WAVE / G;
    constexpr int NW = 4;
    extern __shared__ double stage[];
    __shared__ int seg_b[9];
    __shared__ int seg_c[10];
    __shared__ LdsTable<T> lt;
    __shared__ double red[2 * NW];
    const double rc2 = tab.rc2d;
    const int tid = threadIdx.x;
    const int lane = tid & (MDLJ_WAVE - 1), wv = tid / MDLJ_WAVE;
    if (MS) lds_table_load(lt, tab, tid, blockDim.x);
    const int64_t tile = remap ? xcd_remap(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    const int tx = (int)(tile % tiles_x);
    const int64_t rr = tile / tiles_x;
    const int cy = (int)(rr % g.n[1]);
    const int cz = (int)(rr / g.n[1]);
    const int cx0 = tx * STAGE_K;
    const int ncx = min(STAGE_K, g.n[0] - cx0);
    const int64_t ei = (int64_t)(cy + g.h[1]) * g.stride[1] + (int64_t)(cz + g.h[2]) * g.stride[2] +
                       cx0 + g.h[0];
    const int ib = start[ei], ie = start[ei + ncx];
    if (tid < 9) {
        const int dy = tid % 3 - 1, dz = tid / 3 - 1;
        const int64_t ej = (int64_t)(cy + dy + g.h[1]) * g.stride[1] +
                           (int64_t)(cz + dz + g.h[2]) * g.stride[2] + cx0 - 1 + g.h[0];
        seg_b[tid] = start[ej];
        seg_c[tid + 1] = start[ej + ncx + 2] - start[ej];
    }
    __syncthreads();
    if (tid == 0) {
        seg_c[0] = 0;
        for (int r = 0; r < 9; ++r) seg_c[r + 1] += seg_c[r];
    }
    __syncthreads();
    const int C = seg_c[9];
    double *sx = stage, *sy = stage + cmax, *sz = stage + 2 * cmax;
    int *st = (int *)(stage + 3 * cmax);
    stage_rows(rec, seg_b, seg_c, C, sx, sy, sz, st, MS, tid, blockDim.x);
    if (tid == 0) {
        sx[C] = sy[C] = sz[C] = PAD_COORD;
        if (MS) st[C] = 0;
    }
    __syncthreads();
    // compact index of the tile's first particle (cells of a tile are consecutive)
    const int64_t c0 = (int64_t)cx0 + (int64_t)g.n[0] * (cy + (int64_t)g.n[1] * cz);
    const int64_t t0 = ibase[c0];
    const int l = lane % SEG;
    double bu = 0.0, bw = 0.0;
    for (int i0 = ib + wv * G; i0 < ie; i0 += NW * G) {
        const int i = i0 + lane / SEG;
        const bool act = i < ie;
        const PosT pi = rec[act ? i : ib];
        const int64_t t = t0 + (act ? i - ib : 0);
        const int32_t L = act ? len[t] : 0;
        const uint16_t *row = nbr + t * cap;
        Acc a;
        acc_zero(a);
        for (int32_t k0 = V * l; k0 < L; k0 += V * SEG) {
            uint32_t w[4];
            if (V == 8) {
                const uint4 q = ((const uint4 *)row)[k0 >> 3];
                w[0] = q.x; w[1] = q.y; w[2] = q.z; w[3] = q.w;
            } else if (V == 4) {
                const uint2 q = ((const uint2 *)row)[k0 >> 2];
                w[0] = q.x; w[1] = q.y;
            } else {
                w[0] = ((const uint32_t *)row)[k0 >> 1];
            }
#pragma unroll
            for (int u = 0; u < V; ++u) {
                const int k = (int)((w[u >> 1] >> (16 * (u & 1))) & 0xffffu);
                const PairP<T> p = pair_params<T, MS>(tab, lt, pi.t, MS ? st[k] : 0);
                double fxp, fyp, fzp;
                lj_pair<T, E>(pi.x, pi.y, pi.z, sx[k], sy[k], sz[k], true, p, rc2, a, fxp, fyp, fzp);
            }
        }
        a.fx = seg_sum(a.fx, SEG);
        a.fy = seg_sum(a.fy, SEG);
        a.fz = seg_sum(a.fz, SEG);
        if (act && l == 0) {
            fo.fx[i] = a.fx;
            fo.fy[i] = a.fy;
            fo.fz[i] = a.fz;
        }
        if (E) {
            bu += a.u;
            bw += a.w;
        }
    }
    if (E) {
        bu = seg_sum(bu, MDLJ_WAVE);
        bw = seg_sum(bw, MDLJ_WAVE);
        if (lane == 0) {
            red[2 * wv] = bu;
            red[2 * wv + 1] = bw;
        }
        __syncthreads();
        if (tid == 0) {
            double u = 0, w = 0;
            for (int q = 0; q < NW; ++q) {
                u += red[2 * q];
                w += red[2 * q + 1];
            }
            fo.partial[2 * blockIdx.x] = 0.5 * u;
            fo.partial[2 * blockIdx.x + 1] = 0.5 * w;
        }
    }
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
                                                int32_t cap, int64_t nrec, LJTable<T> tab,
                                                ForceOut fo, int remap)
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
        // lane l takes entries [4l, 4l+3] of each window of 4*SEG, read as one
        // 16-byte load; rows are 16-byte aligned and padded to a multiple of
        // 8 with the padding record, so every loaded index is valid
        const int4 *row = (const int4 *)(nbr + t * cap);
        const __amdgpu_buffer_rsrc_t rr = records_rsrc(rec, nrec);
        for (int32_t k0 = 4 * l; k0 < L; k0 += 4 * SEG) {
            const int4 q = row[k0 >> 2];
            const int32_t jj[4] = {q.x, q.y, q.z, q.w};
            double xj[4], yj[4], zj[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) load_xyz(rr, jj[u], xj[u], yj[u], zj[u]);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const PairP<T> p = pair_params<T, MS>(tab, lt, pi.t, MS ? rec[jj[u]].t : 0);
                double fxp, fyp, fzp;
                lj_pair<T, E>(pi.x, pi.y, pi.z, xj[u], yj[u], zj[u], true, p, rc2, a, fxp, fyp,
                              fzp);
                if (N3) {
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
    const int64_t nrec = ctx->n_ext + 1;  // records + the padding record
    if (cfg.staged) {
        const Grid &g = ctx->grid;
        const int cmax = ctx->max_nbhd + 1;  // + the padding entry
        const size_t lds = (size_t)cmax * (3 * sizeof(double) + (MS ? sizeof(int) : 0));
        if (lds > (size_t)STAGE_LDS_BYTES || N3) return -2;
        const int tiles_x = (int)ceil_div(g.n[0], STAGE_K);
        const int64_t nbt = (int64_t)tiles_x * g.n[1] * g.n[2];
        const int32_t *ibase = (const int32_t *)ctx->b_icnt.p + g.ncell_int + 1;
        const uint16_t *nbr16 = (const uint16_t *)ctx->b_nbr.p;
        const int32_t *start = (const int32_t *)ctx->b_start.p;
#define VL_LDS(GG, VV)                                                                        \
    k_vl_lds<T, E, MS, GG, VV><<<nbt, 256, lds, s>>>(rec, start, ibase, g, tiles_x, nbr16, len, \
                                                     cap, cmax, tab, fo, remap)
        const int key = cfg.tile_i * 100 + cfg.tile_j;
        switch (key) {
        case 802: VL_LDS(8, 2); break;
        case 804: VL_LDS(8, 4); break;
        case 1602: VL_LDS(16, 2); break;
        case 1604: VL_LDS(16, 4); break;
        case 408: VL_LDS(4, 8); break;
        default: return -1;
        }
#undef VL_LDS
        return nbt;
    }
    // 32-bit buffer offsets: records must stay under 2 GiB
    if (nrec * (int64_t)sizeof(PosT) >= ((int64_t)1 << 31)) return -3;
    const int64_t waves = ceil_div(n, cfg.tile_i);
    const int64_t nb = ceil_div(waves, TB / MDLJ_WAVE);
    switch (cfg.tile_i) {
    case 1: k_vl_wpi<T, E, MS, N3, 1><<<nb, TB, 0, s>>>(rec, ilist, nbr, len, n, cap, nrec, tab, fo, remap); break;
    case 2: k_vl_wpi<T, E, MS, N3, 2><<<nb, TB, 0, s>>>(rec, ilist, nbr, len, n, cap, nrec, tab, fo, remap); break;
    case 4: k_vl_wpi<T, E, MS, N3, 4><<<nb, TB, 0, s>>>(rec, ilist, nbr, len, n, cap, nrec, tab, fo, remap); break;
    case 8: k_vl_wpi<T, E, MS, N3, 8><<<nb, TB, 0, s>>>(rec, ilist, nbr, len, n, cap, nrec, tab, fo, remap); break;
    case 16: k_vl_wpi<T, E, MS, N3, 16><<<nb, TB, 0, s>>>(rec, ilist, nbr, len, n, cap, nrec, tab, fo, remap); break;
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
    if (cfg.newton3) STCHK(zero_forces(ctx, fo, ctx->n_ext + 1));
    int64_t nw;
    if (energy) {
        const int64_t maxw = std::max<int64_t>(ctx->n + 64, ctx->grid.ncell_int);
        STCHK(ensure(ctx, ctx->b_partial, sizeof(double) * 2 * maxw));
        fo.partial = (double *)ctx->b_partial.p;
        nw = ms ? launch_vl_n3<T, true, true>(ctx, cfg, tab, fo, remap)
                : launch_vl_n3<T, true, false>(ctx, cfg, tab, fo, remap);
    } else {
        nw = ms ? launch_vl_n3<T, false, true>(ctx, cfg, tab, fo, remap)
                : launch_vl_n3<T, false, false>(ctx, cfg, tab, fo, remap);
    }
    if (nw == -2) return set_err(ctx, MDLJ_ERR_ARG, "neighbourhood too large for LDS staging");
    if (nw == -3) return set_err(ctx, MDLJ_ERR_ARG, "too many records for 32-bit buffer offsets");
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
    cap = (cap + 7) & ~(int64_t)7;
    STCHK(ensure(ctx, ctx->b_nlen, sizeof(int32_t) * n));
    int32_t *maxlen = (int32_t *)ctx->b_flags.p + 12;
    int32_t *maxnb = (int32_t *)ctx->b_flags.p + 14;
    const bool rowmajor = cfg.order != MDLJ_ORD_I_PER_LANE;
    const bool local = cfg.staged != 0;
    const size_t esize = local ? sizeof(uint16_t) : sizeof(int32_t);
    for (int attempt = 0; attempt < 3; ++attempt) {
        if ((double)cap * (double)n * (double)esize > 64e9)
            return set_err(ctx, MDLJ_ERR_OVERFLOW, "Verlet lists too large");
        STCHK(ensure(ctx, ctx->b_nbr, esize * n * cap));
        HIPCHK(ctx, hipMemsetAsync(maxlen, 0, 4 * sizeof(int32_t), ctx->stream));
        if (local) {
            k_vl_build_local<<<ceil_div(n, 256), 256, 0, ctx->stream>>>(
                (const PosT *)ctx->b_sorted.p, (const int32_t *)ctx->b_start.p,
                (const int32_t *)ctx->b_ilist.p, (const int32_t *)ctx->b_cell_of.p, g, n, rl * rl,
                (int32_t)cap, (uint16_t *)ctx->b_nbr.p, (int32_t *)ctx->b_nlen.p, maxlen, maxnb);
        } else {
            const int64_t sk = rowmajor ? 1 : n;
            const int64_t st = rowmajor ? cap : 1;
            k_vl_build<<<ceil_div(n, 256), 256, 0, ctx->stream>>>(
                (const PosT *)ctx->b_sorted.p, (const int32_t *)ctx->b_start.p,
                (const int32_t *)ctx->b_ilist.p, (const int32_t *)ctx->b_cell_of.p, g, n, rl * rl,
                cfg.newton3 ? 1 : 0, sk, st, (int32_t)cap, (int32_t)ctx->n_ext,
                (int32_t *)ctx->b_nbr.p, (int32_t *)ctx->b_nlen.p, maxlen);
        }
        HIPCHK(ctx, hipGetLastError());
        int32_t hmax[3] = {0, 0, 0};
        HIPCHK(ctx, hipMemcpyAsync(hmax, maxlen, 3 * sizeof(int32_t), hipMemcpyDeviceToHost,
                                   ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        ctx->vl_max = hmax[0];
        ctx->max_nbhd = hmax[2];
        if (local && hmax[2] > 65535)
            return set_err(ctx, MDLJ_ERR_ARG, "neighbourhood too large for 16-bit local lists");
        if (hmax[0] <= cap) {
            ctx->nbr_cap = cap;
            return MDLJ_OK;
        }
        cap = ((int64_t)(hmax[0] * 1.1) + 8 + 7) & ~(int64_t)7;
    }
    return set_err(ctx, MDLJ_ERR_OVERFLOW, "Verlet list capacity could not be grown");
}

mdlj_status vl_forces(mdlj_ctx *ctx, const mdlj_config &cfg, bool energy, ForceOut &fo,
                      int64_t *nblocks)
{
    if (ctx->prec == MDLJ_PREC_F64) return vl_forces_t<double>(ctx, cfg, energy, fo, nblocks);
    return vl_forces_t<float>(ctx, cfg, energy, fo, nblocks);
}
