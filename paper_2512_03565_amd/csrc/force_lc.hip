// force_lc.hip -- force kernels over linked cells (section 2.1.1) with the
// interaction orders of section 4.1, mapped onto 64-lane wavefronts.
//
// Cells have edge >= rc, so a particle's partners lie in the 3x3x3 block
// of cells around its own (halo cells included).  Cells are numbered x
// fastest, so the three cells cx-1..cx+1 of one (dy, dz) row are one
// contiguous run of sorted records: the candidate set of a cell is nine
// contiguous runs.  Every pair is evaluated from both sides (no Newton-3),
// which needs no atomics and no colouring of the domain.
//
// Orders:
//   k_lc_ipl   VectorLength/1 (i-per-lane): each lane owns one i of an
//              i-tile of K consecutive cells along x; the j-candidates of
//              the tile (nine runs of K+2 cells) are staged 64 at a time in
//              LDS and every lane reads the same j (LDS broadcast).  No
//              reduction: each lane stores its own i (section 4.1.2).
//   k_lc_tile  a_i x a_j lane grid, a_i * a_j = 64: a_i i's of one cell
//              per step, a_j lanes per i striding over the concatenated
//              nine runs; the a_j partial forces of an i are summed over
//              their lanes at the end.  a_i = 1 is 1/VectorLength
//              (wave-per-i), a_i = 2, 4 its split variants, a_i = 8, 16
//              the cluster tiles (2/(VL/2)-, (VL/2)/2-like).
#include "pair.h"

namespace {

// candidates per trip of the tile loops
constexpr int UNROLL = 4;

template <typename T, bool E, bool MS>
__global__ __launch_bounds__(64) void k_lc_ipl(const PosT *__restrict__ rec,
                                               const int32_t *__restrict__ start, Grid g, int K,
                                               int tiles_x, LJTable<T> tab, ForceOut fo,
                                               int remap)
{
    __shared__ PosT js[MDLJ_WAVE];
    __shared__ LdsTable<T> lt;
    const double rc2 = tab.rc2d;
    const int lane = threadIdx.x;
    if (MS) lds_table_load(lt, tab, lane, MDLJ_WAVE);
    const int64_t nb = gridDim.x;
    const int64_t t = remap ? xcd_remap(blockIdx.x, nb) : (int64_t)blockIdx.x;
    const int tx = (int)((uint32_t)t % (uint32_t)tiles_x);
    const uint32_t rr = (uint32_t)t / (uint32_t)tiles_x;
    const int cy = (int)(rr % (uint32_t)g.n[1]);
    const int cz = (int)(rr / (uint32_t)g.n[1]);
    const int cx0 = tx * K;
    const int ncx = min(K, g.n[0] - cx0);
    const int64_t ei = (int64_t)(cy + g.h[1]) * g.stride[1] + (int64_t)(cz + g.h[2]) * g.stride[2] +
                       cx0 + g.h[0];
    const int ib = start[ei], ie = start[ei + ncx];
    double bu = 0.0, bw = 0.0;
    __syncthreads();
    for (int i0 = ib; i0 < ie; i0 += MDLJ_WAVE) {
        // every lane its own i, one j for all (VectorLength/1)
        const int i = i0 + lane_pair(LANE_J_MAJOR, MDLJ_WAVE, MDLJ_WAVE, lane).i;
        const bool act = i < ie;
        const PosT pi = rec[act ? i : ib];
        Acc a;
        acc_zero(a);
        for (int r = 0; r < 9; ++r) {
            const int dy = r % 3 - 1, dz = r / 3 - 1;
            const int64_t ej = (int64_t)(cy + dy + g.h[1]) * g.stride[1] +
                               (int64_t)(cz + dz + g.h[2]) * g.stride[2] + cx0 - 1 + g.h[0];
            const int jb = start[ej], je = start[ej + ncx + 2];
            for (int j0 = jb; j0 < je; j0 += MDLJ_WAVE) {
                const int jn = min(MDLJ_WAVE, je - j0);
                __syncthreads();
                if (lane < jn) js[lane] = rec[j0 + lane];
                __syncthreads();
                for (int jj = 0; jj < jn; ++jj) {
                    const PosT pj = js[jj];
                    const PairP<T> p = pair_params<T, MS>(tab, lt, pi.t, pj.t);
                    double fxp, fyp, fzp;
                    lj_pair<T, E>(pi.x, pi.y, pi.z, pj.x, pj.y, pj.z, act && (j0 + jj) != i, p,
                                  rc2, a, fxp, fyp, fzp);
                }
            }
        }
        if (act) {
            fo.fx[i] = a.fx;
            fo.fy[i] = a.fy;
            fo.fz[i] = a.fz;
        }
        if (E) {
            bu += a.u;
            bw += a.w;
        }
    }
    if (E) wave_partial(bu, bw, 0.5, fo.partial, blockIdx.x);
}

template <typename T, bool E, bool MS, int AI, bool STAGED>
__global__ __launch_bounds__(64) void k_lc_tile(const PosT *__restrict__ rec,
                                                const int32_t *__restrict__ start, Grid g,
                                                LJTable<T> tab, ForceOut fo, int remap,
                                                int cmax)
{
    extern __shared__ double stage[];
    constexpr int AJ = MDLJ_WAVE / AI;
    __shared__ int seg_b[9];
    __shared__ int seg_c[10];
    __shared__ LdsTable<T> lt;
    const double rc2 = tab.rc2d;
    const int lane = threadIdx.x;
    if (MS) lds_table_load(lt, tab, lane, MDLJ_WAVE);
    const int64_t nb = gridDim.x;
    const int64_t c = remap ? xcd_remap(blockIdx.x, nb) : (int64_t)blockIdx.x;
    const int cx = (int)((uint32_t)c % (uint32_t)g.n[0]);
    const int cy = (int)(((uint32_t)c / (uint32_t)g.n[0]) % (uint32_t)g.n[1]);
    const int cz = (int)((uint32_t)c / ((uint32_t)g.n[0] * (uint32_t)g.n[1]));
    const int64_t ei = (int64_t)(cy + g.h[1]) * g.stride[1] + (int64_t)(cz + g.h[2]) * g.stride[2] +
                       cx + g.h[0];
    const int ib = start[ei], ie = start[ei + 1];
    if (lane < 9) {
        const int dy = lane % 3 - 1, dz = lane / 3 - 1;
        const int64_t ej = (int64_t)(cy + dy + g.h[1]) * g.stride[1] +
                           (int64_t)(cz + dz + g.h[2]) * g.stride[2] + cx - 1 + g.h[0];
        seg_b[lane] = start[ej];
        seg_c[lane + 1] = start[ej + 3] - start[ej];
    }
    __syncthreads();
    if (lane == 0) {
        seg_c[0] = 0;
        for (int r = 0; r < 9; ++r) seg_c[r + 1] += seg_c[r];
    }
    __syncthreads();
    const int C = seg_c[9];
    double *sx = stage, *sy = stage + cmax, *sz = stage + 2 * cmax;
    int *st = (int *)(stage + 3 * cmax);
    if (STAGED) {
        stage_rows_simple(rec, seg_b, seg_c, C, sx, sy, sz, st, MS, lane, MDLJ_WAVE);
        __syncthreads();
    }
    // local index of the cell's own first particle in the staged order
    const int own0 = seg_c[4] + (ib - seg_b[4]);
    // AI i's, AJ lanes each striding over the candidates, j fastest
    const LanePair lp = lane_pair(LANE_I_MAJOR, AI, MDLJ_WAVE, lane);
    const int ii = lp.i, jl = lp.j;
    double bu = 0.0, bw = 0.0;
    for (int i0 = ib; i0 < ie; i0 += AI) {
        const int i = i0 + ii;
        const bool act = i < ie;
        const PosT pi = rec[act ? i : ib];
        const int iloc = own0 + (i - ib);
        Acc a;
        acc_zero(a);
        if (STAGED) {
            for (int k0 = jl; k0 < C; k0 += UNROLL * AJ) {
#pragma unroll
                for (int u = 0; u < UNROLL; ++u) {
                    const int k = k0 + u * AJ;
                    const bool ok = k < C;
                    const int kk = ok ? k : 0;
                    const PairP<T> p = pair_params<T, MS>(tab, lt, pi.t, MS ? st[kk] : 0);
                    double fxp, fyp, fzp;
                    lj_pair<T, E>(pi.x, pi.y, pi.z, sx[kk], sy[kk], sz[kk],
                                  act && ok && k != iloc, p, rc2, a, fxp, fyp, fzp);
                }
            }
        } else {
        int r = 0;
        // U candidates per trip: their record loads are in flight together
        for (int k0 = jl; k0 < C; k0 += UNROLL * AJ) {
            int jj[UNROLL];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                const int k = k0 + u * AJ;
                jj[u] = -1;
                if (k < C) {
                    while (k >= seg_c[r + 1]) ++r;
                    jj[u] = seg_b[r] + (k - seg_c[r]);
                }
            }
            PosT pj[UNROLL];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) pj[u] = rec[jj[u] >= 0 ? jj[u] : ib];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                const PairP<T> p = pair_params<T, MS>(tab, lt, pi.t, pj[u].t);
                double fxp, fyp, fzp;
                lj_pair<T, E>(pi.x, pi.y, pi.z, pj[u].x, pj[u].y, pj[u].z,
                              act && jj[u] >= 0 && jj[u] != i, p, rc2, a, fxp, fyp, fzp);
            }
        }
        }
        a.fx = seg_sum(a.fx, AJ);
        a.fy = seg_sum(a.fy, AJ);
        a.fz = seg_sum(a.fz, AJ);
        if (act && jl == 0) {
            fo.fx[i] = a.fx;
            fo.fy[i] = a.fy;
            fo.fz[i] = a.fz;
        }
        if (E) {
            bu += a.u;
            bw += a.w;
        }
    }
    if (E) wave_partial(bu, bw, 0.5, fo.partial, blockIdx.x);
}

// Newton 3 over linked cells (section 2.1's F_ji = -F_ij; section 4.1.3):
// a cell pairs its own particles with those of its 13 forward neighbour
// cells -- the half of the 26 with dz = +1, or dz = 0 and dy = +1, or
// dz = dy = 0 and dx = +1 -- and with each other, so that every pair inside
// the cutoff is computed once.  One wavefront per cell stages its own
// records followed by those of the forward cells in LDS (five runs of sorted
// records: the own cell with its right neighbour, the row dy = +1, dz = 0,
// and the three rows dz = +1), with an FP64 force accumulator per staged
// record.  The pairs are (a, b) with a an own record and b > a any staged
// one.  Both forces of a pair are added in LDS; at the end every staged
// record adds its force to the sorted force array with one atomic per
// component (forces on halo images are folded onto their particles
// afterwards).
// Two assignments of the cell pair's roles (the traversal's choice of
// which cell provides the i-list):
//   SWAP = false  the own particles are the i's: AI of them per step, AJ
//                 lanes per i striding over its partners b; F_i is summed
//                 over the AJ lanes, F_b added to LDS per lane.
//   SWAP = true   the partners are the i's: a lane takes one b and walks
//                 the own particles a < b as j, read from LDS by every lane
//                 at once (a broadcast); F_b stays in the lane, F_a is summed
//                 over the wavefront and added by one lane.
constexpr int HALF_RUNS = 5;

template <typename T, bool E, bool MS, int AI, bool SWAP>
__global__ __launch_bounds__(64) void k_lc_half(const PosT *__restrict__ rec,
                                                const int32_t *__restrict__ start, Grid g,
                                                LJTable<T> tab, ForceOut fo, int remap, int cmax)
{
    extern __shared__ double stage[];
    constexpr int AJ = MDLJ_WAVE / AI;
    __shared__ int seg_b[HALF_RUNS];
    __shared__ int seg_c[HALF_RUNS + 1];
    __shared__ LdsTable<T> lt;
    const double rc2 = tab.rc2d;
    const int lane = threadIdx.x;
    if (MS) lds_table_load(lt, tab, lane, MDLJ_WAVE);
    const int64_t nb = gridDim.x;
    const int64_t c = remap ? xcd_remap(blockIdx.x, nb) : (int64_t)blockIdx.x;
    const int cx = (int)((uint32_t)c % (uint32_t)g.n[0]);
    const int cy = (int)(((uint32_t)c / (uint32_t)g.n[0]) % (uint32_t)g.n[1]);
    const int cz = (int)((uint32_t)c / ((uint32_t)g.n[0] * (uint32_t)g.n[1]));
    const int64_t ei = (int64_t)(cy + g.h[1]) * g.stride[1] + (int64_t)(cz + g.h[2]) * g.stride[2] +
                       cx + g.h[0];
    if (lane < HALF_RUNS) {
        // run 0: the own cell and its right neighbour; run 1: row dy = +1,
        // dz = 0; runs 2..4: rows dz = +1, dy = -1, 0, +1 (cells cx-1..cx+1)
        int64_t b, e;
        if (lane == 0) {
            b = ei;
            e = ei + 2;
        } else {
            const int dy = lane == 1 ? 1 : lane - 3, dz = lane == 1 ? 0 : 1;
            b = ei + dy * g.stride[1] + dz * g.stride[2] - 1;
            e = b + 3;
        }
        seg_b[lane] = start[b];
        seg_c[lane + 1] = start[e] - start[b];
    }
    __syncthreads();
    if (lane == 0) {
        seg_c[0] = 0;
        for (int r = 0; r < HALF_RUNS; ++r) seg_c[r + 1] += seg_c[r];
    }
    __syncthreads();
    const int C = seg_c[HALF_RUNS];
    const int nown = start[ei + 1] - start[ei];
    double *sx = stage, *sy = stage + cmax, *sz = stage + 2 * cmax;
    double *sfx = stage + 3 * cmax, *sfy = stage + 4 * cmax, *sfz = stage + 5 * cmax;
    int *st = (int *)(stage + 6 * cmax);
    for (int k = lane; k < C; k += MDLJ_WAVE) {
        int r = 0;
        while (k >= seg_c[r + 1]) ++r;
        const PosT p = rec[seg_b[r] + (k - seg_c[r])];
        sx[k] = p.x;
        sy[k] = p.y;
        sz[k] = p.z;
        if (MS) st[k] = p.t;
        sfx[k] = 0.0;
        sfy[k] = 0.0;
        sfz[k] = 0.0;
    }
    __syncthreads();
    double bu = 0.0, bw = 0.0;
    if constexpr (!SWAP) {
        const LanePair lp = lane_pair(LANE_I_MAJOR, AI, MDLJ_WAVE, lane);
        const int ii = lp.i, jl = lp.j;
        for (int a0 = 0; a0 < nown; a0 += AI) {
            const int a = a0 + ii;
            const bool act = a < nown;
            const int aa = act ? a : 0;
            const double xa = sx[aa], ya = sy[aa], za = sz[aa];
            const int ta = MS ? st[aa] : 0;
            Acc acc;
            acc_zero(acc);
            for (int b = aa + 1 + jl; b < C; b += AJ) {
                const PairP<T> p = pair_params<T, MS>(tab, lt, ta, MS ? st[b] : 0);
                double fxp, fyp, fzp;
                if (lj_pair<T, E>(xa, ya, za, sx[b], sy[b], sz[b], act, p, rc2, acc, fxp, fyp,
                                  fzp)) {
                    atomicAdd(&sfx[b], -fxp);
                    atomicAdd(&sfy[b], -fyp);
                    atomicAdd(&sfz[b], -fzp);
                }
            }
            acc.fx = seg_sum(acc.fx, AJ);
            acc.fy = seg_sum(acc.fy, AJ);
            acc.fz = seg_sum(acc.fz, AJ);
            if (act && jl == 0) {
                atomicAdd(&sfx[a], acc.fx);
                atomicAdd(&sfy[a], acc.fy);
                atomicAdd(&sfz[a], acc.fz);
            }
            if (E) {
                bu += acc.u;
                bw += acc.w;
            }
        }
    } else {
        for (int b0 = 0; b0 < C; b0 += MDLJ_WAVE) {
            const int b = b0 + lane;
            const bool act = b < C;
            const int bb = act ? b : 0;
            const double xb = sx[bb], yb = sy[bb], zb = sz[bb];
            const int tb = MS ? st[bb] : 0;
            Acc acc;
            acc_zero(acc);
            // own particles a < b: every lane walks the same a
            const int amax = min(nown, b0 + MDLJ_WAVE);
            for (int a = 0; a < amax; ++a) {
                const PairP<T> p = pair_params<T, MS>(tab, lt, tb, MS ? st[a] : 0);
                double fxp, fyp, fzp;
                lj_pair<T, E>(xb, yb, zb, sx[a], sy[a], sz[a], act && a < b, p, rc2, acc, fxp,
                              fyp, fzp);
                // F_a = -sum over the lanes' F_b contributions
                fxp = seg_sum(fxp, MDLJ_WAVE);
                fyp = seg_sum(fyp, MDLJ_WAVE);
                fzp = seg_sum(fzp, MDLJ_WAVE);
                if (lane == 0) {
                    sfx[a] -= fxp;
                    sfy[a] -= fyp;
                    sfz[a] -= fzp;
                }
            }
            if (act) {
                atomicAdd(&sfx[b], acc.fx);
                atomicAdd(&sfy[b], acc.fy);
                atomicAdd(&sfz[b], acc.fz);
            }
            if (E) {
                bu += acc.u;
                bw += acc.w;
            }
        }
    }
    __syncthreads();
    // one atomic per component of every staged record that took a force
    for (int k = lane; k < C; k += MDLJ_WAVE) {
        const double fx = sfx[k], fy = sfy[k], fz = sfz[k];
        if (fx != 0.0 || fy != 0.0 || fz != 0.0) {
            int r = 0;
            while (k >= seg_c[r + 1]) ++r;
            const int slot = seg_b[r] + (k - seg_c[r]);
            atomicAdd(&fo.fx[slot], fx);
            atomicAdd(&fo.fy[slot], fy);
            atomicAdd(&fo.fz[slot], fz);
        }
    }
    if (E) wave_partial(bu, bw, 1.0, fo.partial, blockIdx.x);
}

// Unordered pairs {i, j} with r < rc, each counted once (from the particle
// with the smaller caller index), in FP64.
__global__ __launch_bounds__(64) void k_lc_count(const PosT *__restrict__ rec,
                                                 const int32_t *__restrict__ start, Grid g,
                                                 double rc2,
                                                 unsigned long long *__restrict__ out)
{
    __shared__ int seg_b[9];
    __shared__ int seg_c[10];
    const int lane = threadIdx.x;
    const int64_t c = blockIdx.x;
    const int cx = (int)((uint32_t)c % (uint32_t)g.n[0]);
    const int cy = (int)(((uint32_t)c / (uint32_t)g.n[0]) % (uint32_t)g.n[1]);
    const int cz = (int)((uint32_t)c / ((uint32_t)g.n[0] * (uint32_t)g.n[1]));
    const int64_t ei = (int64_t)(cy + g.h[1]) * g.stride[1] + (int64_t)(cz + g.h[2]) * g.stride[2] +
                       cx + g.h[0];
    const int ib = start[ei], ie = start[ei + 1];
    if (lane < 9) {
        const int dy = lane % 3 - 1, dz = lane / 3 - 1;
        const int64_t ej = (int64_t)(cy + dy + g.h[1]) * g.stride[1] +
                           (int64_t)(cz + dz + g.h[2]) * g.stride[2] + cx - 1 + g.h[0];
        seg_b[lane] = start[ej];
        seg_c[lane + 1] = start[ej + 3] - start[ej];
    }
    __syncthreads();
    if (lane == 0) {
        seg_c[0] = 0;
        for (int r = 0; r < 9; ++r) seg_c[r + 1] += seg_c[r];
    }
    __syncthreads();
    const int C = seg_c[9];
    unsigned long long cnt = 0;
    for (int i = ib; i < ie; ++i) {
        const PosT pi = rec[i];
        int r = 0;
        for (int k = lane; k < C; k += MDLJ_WAVE) {
            while (k >= seg_c[r + 1]) ++r;
            const PosT pj = rec[seg_b[r] + (k - seg_c[r])];
            if (pj.orig <= pi.orig) continue;
            const double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
            if (dx * dx + dy * dy + dz * dz < rc2) ++cnt;
        }
    }
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
    if (lane == 0 && cnt) atomicAdd(out, cnt);
}

template <typename T, bool E, bool MS>
void launch_lc(mdlj_ctx *ctx, const mdlj_config &cfg, const LJTable<T> &tab, ForceOut &fo,
               int64_t *nblocks, int remap)
{
    const Grid &g = ctx->grid;
    const PosT *rec = (const PosT *)ctx->b_sorted.p;
    const int32_t *start = (const int32_t *)ctx->b_start.p;
    hipStream_t s = ctx->stream;
    if (cfg.newton3) {
        const int64_t nb = g.ncell_int;
        *nblocks = nb;
        // own + 13 forward cells, x, y, z, three force sums and the species
        const int cmax = 14 * ctx->max_cell;
        const size_t lds = (size_t)cmax * (6 * sizeof(double) + (MS ? sizeof(int) : 0));
        if (lds > (size_t)STAGE_LDS_BYTES) {
            *nblocks = -2;
            return;
        }
        if (cfg.swap) {
            if (cfg.order != MDLJ_ORD_I_PER_LANE) {
                *nblocks = -1;
                return;
            }
            k_lc_half<T, E, MS, 64, true><<<nb, 64, lds, s>>>(rec, start, g, tab, fo, remap, cmax);
            return;
        }
        switch (cfg.tile_i) {
        case 1: k_lc_half<T, E, MS, 1, false><<<nb, 64, lds, s>>>(rec, start, g, tab, fo, remap, cmax); break;
        case 4: k_lc_half<T, E, MS, 4, false><<<nb, 64, lds, s>>>(rec, start, g, tab, fo, remap, cmax); break;
        case 16: k_lc_half<T, E, MS, 16, false><<<nb, 64, lds, s>>>(rec, start, g, tab, fo, remap, cmax); break;
        default: *nblocks = -1;
        }
        return;
    }
    if (cfg.order == MDLJ_ORD_I_PER_LANE) {
        const int K = cfg.tile_i;
        const int tiles_x = (int)ceil_div(g.n[0], K);
        const int64_t nb = (int64_t)tiles_x * g.n[1] * g.n[2];
        *nblocks = nb;
        k_lc_ipl<T, E, MS><<<nb, 64, 0, s>>>(rec, start, g, K, tiles_x, tab, fo, remap);
        return;
    }
    const int64_t nb = g.ncell_int;
    *nblocks = nb;
    if (cfg.staged) {
        const int cmax = 27 * ctx->max_cell;
        const size_t lds = (size_t)cmax * (3 * sizeof(double) + (MS ? sizeof(int) : 0));
        if (lds > (size_t)STAGE_LDS_BYTES) {
            *nblocks = -2;
            return;
        }
        switch (cfg.tile_i) {
        case 1: k_lc_tile<T, E, MS, 1, true><<<nb, 64, lds, s>>>(rec, start, g, tab, fo, remap, cmax); break;
        case 2: k_lc_tile<T, E, MS, 2, true><<<nb, 64, lds, s>>>(rec, start, g, tab, fo, remap, cmax); break;
        case 4: k_lc_tile<T, E, MS, 4, true><<<nb, 64, lds, s>>>(rec, start, g, tab, fo, remap, cmax); break;
        case 8: k_lc_tile<T, E, MS, 8, true><<<nb, 64, lds, s>>>(rec, start, g, tab, fo, remap, cmax); break;
        case 16: k_lc_tile<T, E, MS, 16, true><<<nb, 64, lds, s>>>(rec, start, g, tab, fo, remap, cmax); break;
        default: *nblocks = -1;
        }
        return;
    }
    switch (cfg.tile_i) {
    case 1: k_lc_tile<T, E, MS, 1, false><<<nb, 64, 0, s>>>(rec, start, g, tab, fo, remap, 0); break;
    case 2: k_lc_tile<T, E, MS, 2, false><<<nb, 64, 0, s>>>(rec, start, g, tab, fo, remap, 0); break;
    case 4: k_lc_tile<T, E, MS, 4, false><<<nb, 64, 0, s>>>(rec, start, g, tab, fo, remap, 0); break;
    case 8: k_lc_tile<T, E, MS, 8, false><<<nb, 64, 0, s>>>(rec, start, g, tab, fo, remap, 0); break;
    case 16: k_lc_tile<T, E, MS, 16, false><<<nb, 64, 0, s>>>(rec, start, g, tab, fo, remap, 0); break;
    default: *nblocks = -1;
    }
}

template <typename T>
mdlj_status lc_forces_t(mdlj_ctx *ctx, const mdlj_config &cfg, bool energy, ForceOut &fo,
                        int64_t *nblocks)
{
    LJTable<T> tab;
    fill_table<T>(ctx, &tab);
    const bool ms = ctx->nspec > 1;
    const int remap = 1;
    int64_t nb = 0;
    // Newton-3 kernels add both forces of a pair with atomics
    if (cfg.newton3) STCHK(zero_forces(ctx, fo, ctx->n_ext + 1));
    if (energy) {
        // partial buffer sized by the launch: one (U, W) per workgroup
        const Grid &g = ctx->grid;
        int64_t maxb = g.ncell_int;
        STCHK(partial_buffer(ctx, 2 * maxb, &fo.partial));
        if (ms) launch_lc<T, true, true>(ctx, cfg, tab, fo, &nb, remap);
        else launch_lc<T, true, false>(ctx, cfg, tab, fo, &nb, remap);
    } else {
        if (ms) launch_lc<T, false, true>(ctx, cfg, tab, fo, &nb, remap);
        else launch_lc<T, false, false>(ctx, cfg, tab, fo, &nb, remap);
    }
    if (nb == -2) return set_err(ctx, MDLJ_ERR_ARG, "cell neighbourhood too large for LDS staging");
    if (nb < 0) return set_err(ctx, MDLJ_ERR_ARG, "unsupported linked-cell tile shape");
    HIPCHK(ctx, hipGetLastError());
    *nblocks = nb;
    return MDLJ_OK;
}

}  // namespace

mdlj_status lc_forces(mdlj_ctx *ctx, const mdlj_config &cfg, bool energy, ForceOut &fo,
                      int64_t *nblocks)
{
    if (ctx->grid.h[0] != 1 || ctx->grid.stride[0] != 1)
        return set_err(ctx, MDLJ_ERR_STATE, "linked-cell grid not built");
    if (ctx->prec == MDLJ_PREC_F64) return lc_forces_t<double>(ctx, cfg, energy, fo, nblocks);
    return lc_forces_t<float>(ctx, cfg, energy, fo, nblocks);
}

mdlj_status count_pairs_dev(mdlj_ctx *ctx, int64_t *out)
{
    // bin at the cutoff (as linked cells do) and count from the smaller index
    double r = ctx->rc;
    for (int a = 0; a < 3; ++a)
        if (ctx->box[a] < 2.0 * r || floor(ctx->box[a] / r) < 3)
            return set_err(ctx, MDLJ_ERR_GEOMETRY, "box too small for linked cells");
    double rmin[3] = {r, r, r};
    int h[3] = {1, 1, 1};
    Grid g;
    if (!make_grid(ctx->box, rmin, h, false, &g)) return set_err(ctx, MDLJ_ERR_GEOMETRY, "grid");
    STCHK(bin_particles(ctx, g));
    ctx->built = false;  // the current structure was replaced
    STCHK(ensure(ctx, ctx->b_partial, sizeof(unsigned long long)));
    unsigned long long *d = (unsigned long long *)ctx->b_partial.p;
    HIPCHK(ctx, hipMemsetAsync(d, 0, sizeof(unsigned long long), ctx->stream));
    k_lc_count<<<g.ncell_int, 64, 0, ctx->stream>>>((const PosT *)ctx->b_sorted.p,
                                                   (const int32_t *)ctx->b_start.p, g, r * r, d);
    HIPCHK(ctx, hipGetLastError());
    unsigned long long h_cnt = 0;
    HIPCHK(ctx, hipMemcpyAsync(&h_cnt, d, sizeof h_cnt, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    *out = (int64_t)h_cnt;
    return MDLJ_OK;
}
