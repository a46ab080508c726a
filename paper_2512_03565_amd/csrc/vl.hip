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
#include <limits.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "pair.h"

namespace {

// Pruned inner list: r_in = rc + PRUNE_FRACTION skin; it stays valid while
// no particle has moved more than PRUNE_FRACTION skin / 2 since the build
constexpr double PRUNE_FRACTION = 2.0 / 3.0;

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
    if ((threadIdx.x & (MDLJ_WAVE - 1)) == 0 && cnt > 0) atomic_max_rare(maxlen, cnt);
}

// Lists for the staged kernel: entry = index of j in the concatenation of
// the nine neighbour rows of i's x-tile (STAGE_K consecutive cells along x
// and one halo cell either side), the order in which the force kernel
// stages them into LDS; 16 bits, row-major per i, padded to a multiple of 8
// with the index one past the staged particles (a far-away padding entry).
// The staged kernel reads each row's length and start from lo[t] = {len[t],
// start of row t less t cap}: the tiled build packs the rows of a tile,
// this per-particle build leaves each at t cap.

__global__ __launch_bounds__(256) void k_vl_build_local(const PosT *__restrict__ rec,
                                                        const int32_t *__restrict__ start,
                                                        const int32_t *__restrict__ ilist,
                                                        const int32_t *__restrict__ cell_of,
                                                        Grid g, int64_t n, double rl2,
                                                        int32_t cap, uint16_t *__restrict__ nbr,
                                                        int32_t *__restrict__ len,
                                                        int2 *__restrict__ lo,
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
        const int cx = (int)((uint32_t)e % (uint32_t)g.stride[1]) - g.h[0];
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
        lo[t] = make_int2(cnt, 0);
    }
    for (int o = 32; o > 0; o >>= 1) {
        cnt = max(cnt, __shfl_xor(cnt, o));
        base = max(base, __shfl_xor(base, o));
    }
    if ((threadIdx.x & (MDLJ_WAVE - 1)) == 0) {
        if (cnt > 0) atomic_max_rare(maxlen, cnt);
        if (base > 0) atomic_max_rare(maxnb, base);
    }
}

// Tiled build: one workgroup per x-tile (the tiles of the staged force
// kernel) copies the tile's neighbourhood into LDS and lists, for each cell
// of the tile, the staged indices of its 27 cells (nine runs of three
// cells).  A wavefront then takes one i at a time: its 64 lanes test 64
// candidates per trip and the hits are packed in candidate order with a
// ballot and a lane prefix count, so each list row is written as one
// contiguous run.  The lists equal those of the per-particle builds above
// entry for entry (a partner at distance zero, which only the particle
// itself can be, is left out by the distance test).
//
// Local rows are packed: the rows a wavefront writes (its i's, every NW-th
// of the tile) follow one another, each from where the last one ended
// (its length rounded up to 8 entries, at most cap), inside a region of
// cap entries per row that follows the regions of the lower wavefronts; a
// tile's rows then fill one run of the array from t0 cap on, and a reader
// fetches no unused row capacity.  lo[t] holds the row's length and its
// start less t cap.  Which wavefront takes which i is fixed, so the layout is the same
// on every build of the same lists.
//
// LOCAL: 16-bit staged indices, rows padded with C (the staged count);
// otherwise sorted-record slots at nbr[t * st + k * sk], padded with `pad`.
// HALF keeps partners with a larger caller index only.
// A tile whose neighbourhood exceeds cmax records its size in maxnb and
// builds nothing; the host then falls back to the per-particle build.
constexpr int BUILD_TB = 512;
// Each candidate list is padded to a multiple of a trip (2 x 64 lanes) with
// the index of a far-away padding record staged after the neighbourhood, so
// lanes past a list need no test of their own: CAND_PAD bounds the padding
// of a tile's lists, CAND_SLACK the entries after the last one.
constexpr int CAND_TRIP = 2 * MDLJ_WAVE;
constexpr int CAND_PAD = 2 * STAGE_K * (CAND_TRIP - 1);
constexpr int CAND_SLACK = 2 * MDLJ_WAVE;

// Candidate runs of the tiled build.  Records in a cell are ordered lower x
// half first (hstart = first upper-half slot).  With cells at least rl + a
// margin wide along x, a particle in the lower half of its cell cannot
// reach the upper half of the cell to its right (and an upper-half one the
// lower half of the cell to its left): more than one cell edge apart in x.
// So each tile cell has two candidate lists, one per half, each nine
// contiguous runs:  lower: [start(c-1), hstart(c+1)),  upper:
// [hstart(c-1), end(c+1)).  Without the margin both are the full runs.
__device__ __forceinline__ void half_runs(const int (*rs)[STAGE_K + 3],
                                          const int (*hs)[STAGE_K + 2], int r, int c, int h,
                                          bool trim, int &b, int &e)
{
    // row cells c .. c + 2 are the left neighbour, the cell and the right one
    b = (trim && h == 1) ? hs[r][c] : rs[r][c];
    e = (trim && h == 0) ? hs[r][c + 2] : rs[r][c + 3];
}

// host[0..3] = src[0..3] (system-scope stores to pinned memory)
__global__ void k_publish4(int32_t *__restrict__ src, int32_t *host, uint32_t seq)
{
    if (threadIdx.x == 0) {
        for (int k = 0; k < 4; ++k) {
            __hip_atomic_store(host + k, src[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            src[k] = 0;  // cleared for the next build
        }
        // after the values: the host waits for this word
        __hip_atomic_store((uint32_t *)host + 4, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// Staged records and candidate-list entries of the largest tile, for the
// LDS size of the tiled build: one thread per tile.
__global__ void k_tile_sizes(const int32_t *__restrict__ start,
                             const int32_t *__restrict__ hstart, Grid g, int tiles_x,
                             int64_t ntiles, int trim, int32_t *__restrict__ out)
{
    const int64_t tile = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t C = 0, NC = 0;
    if (tile < ntiles) {
        const int tx = (int)((uint32_t)tile % (uint32_t)tiles_x);
        const uint32_t rr = (uint32_t)tile / (uint32_t)tiles_x;
        const int cy = (int)(rr % (uint32_t)g.n[1]);
        const int cz = (int)(rr / (uint32_t)g.n[1]);
        const int cx0 = tx * STAGE_K;
        const int ncx = min(STAGE_K, g.n[0] - cx0);
        for (int r = 0; r < 9; ++r) {
            const int dy = r % 3 - 1, dz = r / 3 - 1;
            const int64_t ej = (int64_t)(cy + dy + g.h[1]) * g.stride[1] +
                               (int64_t)(cz + dz + g.h[2]) * g.stride[2] + cx0 - 1 + g.h[0];
            C += start[ej + ncx + 2] - start[ej];
            for (int c = 0; c < ncx; ++c) {
                NC += (trim ? hstart[ej + c + 2] : start[ej + c + 3]) - start[ej + c];
                NC += start[ej + c + 3] - (trim ? hstart[ej + c] : start[ej + c]);
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        C = max(C, __shfl_xor(C, o));
        NC = max(NC, __shfl_xor(NC, o));
    }
    if ((threadIdx.x & (MDLJ_WAVE - 1)) == 0) {
        atomic_max_rare(out, C);
        atomic_max_rare(out + 1, NC);
    }
}

// the tiled build's set-up: cell starts of the nine rows by threads
// 0 .. 9 (STAGE_K + 3) - 1, half starts by the third wavefront on, and the
// (cell, half) list offsets scanned over 16 lanes of the first wavefront
static_assert(9 * (STAGE_K + 3) <= 2 * MDLJ_WAVE, "tile too wide for the set-up");
static_assert(2 * MDLJ_WAVE + 9 * (STAGE_K + 2) <= BUILD_TB, "tile too wide for the set-up");
static_assert(2 * STAGE_K <= 16, "tile too wide for the set-up");

// INNER (local lists only): the pruned inner list too, the entries closer
// than sqrt(rin2) in list order, into rows of in_nbr (same layout, packed
// the same way, with lengths and starts in in_lo).
template <bool LOCAL, bool HALF, bool ELL, bool INNER>
__global__ __launch_bounds__(BUILD_TB) void k_vl_build_tile(
    const PosT *__restrict__ rec, const int32_t *__restrict__ start,
    const int32_t *__restrict__ hstart, const int32_t *__restrict__ ibase, Grid g, int tiles_x,
    double rl2, int trim, int cmax, int ccand, int64_t n, int32_t cap, int32_t pad,
    void *__restrict__ nbr_out, int32_t *__restrict__ len, int32_t *__restrict__ maxlen,
    int32_t *__restrict__ maxnb, int32_t *__restrict__ maxnc, int remap,
    uint16_t *__restrict__ in_nbr, double rin2,
    int2 *__restrict__ lo, int2 *__restrict__ in_lo)
{
    static_assert(!INNER || (LOCAL && !HALF && !ELL), "inner lists are local full lists");
    constexpr int NW = BUILD_TB / MDLJ_WAVE;
    constexpr int RC = STAGE_K + 3;  // cell starts per row: STAGE_K + 2 cells and the end
    // staged record: x, y, z (a stride of 6 dwords keeps 64-bit LDS reads of
    // consecutive records free of bank conflicts); slot lists also stage
    // each record's slot and caller index in arrays of their own
    constexpr int RW = 3;
    extern __shared__ double stage[];
    __shared__ int rs[9][RC];            // start[] of the cells of each row
    __shared__ int hs[9][RC - 1];        // hstart[] of the cells of each row
    __shared__ int seg_c[10];            // staged offset of each row
    __shared__ int nc[2 * STAGE_K + 1];  // offsets of the (tile cell, half) candidate lists
    __shared__ int qlen[2 * STAGE_K];    // their lengths before the padding
    __shared__ int roff[2 * STAGE_K][9]; // offset of row r's run inside list q
    __shared__ int wmx[NW];
    const int tid = threadIdx.x;
    // the wavefront index as a uniform value: the per-i addressing below
    // then stays in scalar registers
    const int lane = tid & (MDLJ_WAVE - 1), wv = __builtin_amdgcn_readfirstlane(tid / MDLJ_WAVE);
    const int64_t tile = remap ? xcd_remap(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    const int tx = (int)((uint32_t)tile % (uint32_t)tiles_x);
    const uint32_t rr = (uint32_t)tile / (uint32_t)tiles_x;
    const int cy = (int)(rr % (uint32_t)g.n[1]);
    const int cz = (int)(rr / (uint32_t)g.n[1]);
    const int cx0 = tx * STAGE_K;
    const int ncx = min(STAGE_K, g.n[0] - cx0);
    // all cell starts of the nine rows in one round of loads
    if (tid < 9 * (ncx + 3)) {
        const int r = tid / (ncx + 3), c = tid % (ncx + 3);
        const int dy = r % 3 - 1, dz = r / 3 - 1;
        const int64_t ej = (int64_t)(cy + dy + g.h[1]) * g.stride[1] +
                           (int64_t)(cz + dz + g.h[2]) * g.stride[2] + cx0 - 1 + g.h[0];
        rs[r][c] = start[ej + c];
    } else if (tid >= 2 * MDLJ_WAVE && tid < 2 * MDLJ_WAVE + 9 * (ncx + 2)) {
        const int q = tid - 2 * MDLJ_WAVE;
        const int r = q / (ncx + 2), c = q % (ncx + 2);
        const int dy = r % 3 - 1, dz = r / 3 - 1;
        const int64_t ej = (int64_t)(cy + dy + g.h[1]) * g.stride[1] +
                           (int64_t)(cz + dz + g.h[2]) * g.stride[2] + cx0 - 1 + g.h[0];
        hs[r][c] = hstart[ej + c];
    }
    const int64_t c0 = (int64_t)cx0 + (int64_t)g.n[0] * (cy + (int64_t)g.n[1] * cz);
    const int64_t t0 = ibase[c0];
    __syncthreads();
    if (wv == 0) {
        // lanes 0..8: row lengths; lanes 16..16+2ncx-1: candidates of list
        // q = 2 * (tile cell) + half
        int v = 0;
        if (lane < 9) v = rs[lane][ncx + 2] - rs[lane][0];
        const int q = lane - 16;
        if (q >= 0 && q < 2 * ncx) {
            for (int r = 0; r < 9; ++r) {
                int b, e;
                half_runs(rs, hs, r, q >> 1, q & 1, trim, b, e);
                roff[q][r] = v;
                v += e - b;
            }
            qlen[q] = v;
            v = (v + CAND_TRIP - 1) & ~(CAND_TRIP - 1);
        }
        // inclusive scans over lanes 0..15 and 16..31
        for (int o = 1; o < 16; o <<= 1) {
            const int u = __shfl_up(v, o, 16);
            if ((lane & 15) >= o) v += u;
        }
        if (lane < 9) seg_c[lane + 1] = v;
        if (lane == 0) seg_c[0] = 0;
        if (q >= 0 && q < 2 * ncx) nc[q + 1] = v;
        if (lane == 16) nc[0] = 0;
    }
    __syncthreads();
    const int C = seg_c[9];
    // candidates before the padding, for the host's sizing
    int ncu = 0;
    for (int q = 0; q < 2 * ncx; ++q) ncu += qlen[q];
    if (C > cmax || ncu > ccand) {  // block-uniform: report the sizes, build nothing
        if (tid == 0) {
            atomicMax(maxnb, max(C, cmax + 1));
            atomicMax(maxnc, ncu);
        }
        return;
    }
    // cmax + 1 staged records: the neighbourhood and the padding record C
    const int cm1 = cmax + 1;
    double *srec = stage;
    int32_t *sslot = (int32_t *)(stage + (size_t)RW * cm1);
    int32_t *sorig = sslot + (LOCAL ? 0 : cm1);
    uint16_t *cand = (uint16_t *)(sorig + (HALF ? cm1 : 0));
    {
        // two records per thread in flight; rows found without branches and
        // loads unconditional (past the end record C - 1 is read, not stored)
        int cb[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) cb[q] = seg_c[q + 1];
        for (int k0 = tid; k0 < C; k0 += 2 * BUILD_TB) {
            double x[2], y[2], z[2];
            int32_t sl[2], org[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int k = min(k0 + u * BUILD_TB, C - 1);
                int r = 0;
#pragma unroll
                for (int q = 0; q < 8; ++q) r += k >= cb[q];
                sl[u] = rs[r][0] + (k - seg_c[r]);
                const PosT *p = rec + sl[u];
                x[u] = p->x;
                y[u] = p->y;
                z[u] = p->z;
                org[u] = HALF ? p->orig : 0;
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int k = k0 + u * BUILD_TB;
                if (k < C) {
                    double *d = srec + RW * k;
                    d[0] = x[u];
                    d[1] = y[u];
                    d[2] = z[u];
                    if (!LOCAL) sslot[k] = sl[u];
                    if (HALF) sorig[k] = org[u];
                }
            }
        }
    }
    // candidate runs: list q (tile cell q / 2, half q % 2), row r; then
    // each list's padding
    for (int w = wv; w < 9 * 2 * ncx; w += NW) {
        const int q = w / 9, r = w % 9;
        const int off = nc[q] + roff[q][r];
        int rb, re;
        half_runs(rs, hs, r, q >> 1, q & 1, trim, rb, re);
        const int b = seg_c[r] + rb - rs[r][0], m = re - rb;
        for (int u = lane; u < m; u += MDLJ_WAVE) cand[off + u] = (uint16_t)(b + u);
    }
    for (int q = wv; q < 2 * ncx; q += NW)
        for (int u = nc[q] + qlen[q] + lane; u < nc[q + 1]; u += MDLJ_WAVE) cand[u] = (uint16_t)C;
    if (tid < CAND_SLACK) cand[nc[2 * ncx] + tid] = (uint16_t)C;
    if (tid == 0) {
        double *d = srec + RW * C;
        d[0] = d[1] = d[2] = PAD_COORD;
    }
    __syncthreads();
    const int ib = rs[4][1], ie = rs[4][ncx + 1];
    // starts of tile cells 1 .. STAGE_K - 1 (row 4, row cells 2 ..), for a
    // branch-free search of i's cell
    int cs[STAGE_K - 1];
#pragma unroll
    for (int q = 0; q < STAGE_K - 1; ++q) cs[q] = q + 1 < ncx ? rs[4][q + 2] : INT_MAX;
    int32_t wmax = 0;
    // local rows: the start of the wavefront's region (rows of the lower
    // wavefronts, cap entries each) and of its next row, from t0 cap on
    int64_t ro = 0, rio = 0;
    if constexpr (LOCAL) {
        const int m = ie - ib;
        int rows = 0;
        for (int w = 0; w < wv; ++w) rows += w < m ? (m - 1 - w) / NW + 1 : 0;
        ro = rio = (int64_t)rows * cap;
    }
    // The wavefront's i's are ib + wv + NW k.  Their set-up (staged index,
    // candidate list, coordinates) is done for up to 64 of them at once, one
    // per lane, and read back one i at a time with readlane.
    for (int i0 = ib + wv; i0 < ie; i0 += NW * MDLJ_WAVE) {
        const int il = i0 + NW * lane;
        int own_l = 0, pb_l = 0, pe_l = 0, oi_l = 0;
        double xl = 0.0, yl = 0.0, zl = 0.0;
        if (il < ie) {
            own_l = seg_c[4] + (il - rs[4][0]);
            int c = 0;
#pragma unroll
            for (int q = 0; q < STAGE_K - 1; ++q) c += il >= cs[q];
            // i's half of its cell (row 4, row cell c + 1)
            const int hq = 2 * c + ((trim && il >= hs[4][c + 1]) ? 1 : 0);
            const double *di = srec + RW * own_l;
            xl = di[0];
            yl = di[1];
            zl = di[2];
            oi_l = HALF ? sorig[own_l] : 0;
            pb_l = nc[hq];
            pe_l = nc[hq + 1];
        }
        auto bcast = [](double v, int k) {
            return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), k),
                                    __builtin_amdgcn_readlane(__double2loint(v), k));
        };
        const int mi = min(MDLJ_WAVE, (ie - i0 + NW - 1) / NW);
        for (int k = 0; k < mi; ++k) {
            const int i = i0 + NW * k;
            const double xi = bcast(xl, k), yi = bcast(yl, k), zi = bcast(zl, k);
            const int32_t oi = HALF ? __builtin_amdgcn_readlane(oi_l, k) : 0;
            const int pb = __builtin_amdgcn_readlane(pb_l, k);
            const int pe = __builtin_amdgcn_readlane(pe_l, k);
            const int64_t t = t0 + (i - ib);
            uint16_t *row16 = (uint16_t *)nbr_out + t0 * cap + ro;
            int32_t *row32 = (int32_t *)nbr_out + (ELL ? t : t * cap);
            uint16_t *irow = INNER ? in_nbr + t0 * cap + rio : nullptr;
            uint32_t cnt = 0, icnt = 0;
            // two trips of 64 candidates in flight; the list is padded to
            // whole trips with the padding record, which no test passes
            for (int p0 = pb; p0 < pe; p0 += CAND_TRIP) {
                const int ka = cand[p0 + lane];
                const int kb = cand[p0 + MDLJ_WAVE + lane];
                const double *da = srec + RW * ka;
                const double *db = srec + RW * kb;
                const double ax = xi - da[0], ay = yi - da[1], az = zi - da[2];
                const double bx = xi - db[0], by = yi - db[1], bz = zi - db[2];
                // 0 < r^2 < rl2 in one unsigned compare of the bit patterns
                // (positive doubles order like their bits; r^2 = 0, i
                // itself, wraps to the largest value): a single compare
                // feeds the ballot directly
                const uint64_t lim = (uint64_t)__double_as_longlong(rl2) - 1;
                const uint64_t ra = (uint64_t)__double_as_longlong(ax * ax + ay * ay + az * az) - 1;
                const uint64_t rb = (uint64_t)__double_as_longlong(bx * bx + by * by + bz * bz) - 1;
                bool ha = ra < lim;
                bool hb = rb < lim;
                if constexpr (INNER) {
                    // the same order over the candidates, the smaller radius
                    const uint64_t lin = (uint64_t)__double_as_longlong(rin2) - 1;
                    const bool ia = ra < lin, ib = rb < lin;
                    const uint64_t ma = __builtin_amdgcn_ballot_w64(ia);
                    const uint64_t mb = __builtin_amdgcn_ballot_w64(ib);
                    const uint32_t na = (uint32_t)__builtin_popcountll(ma);
                    const uint32_t qa = __builtin_amdgcn_mbcnt_hi(
                        (uint32_t)(ma >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)ma, icnt));
                    const uint32_t qb = __builtin_amdgcn_mbcnt_hi(
                        (uint32_t)(mb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mb, icnt + na));
                    if (ia) *(uint16_t *)((char *)irow + 2u * qa) = (uint16_t)ka;
                    if (ib) *(uint16_t *)((char *)irow + 2u * qb) = (uint16_t)kb;
                    icnt += na + (uint32_t)__builtin_popcountll(mb);
                }
                if (HALF) {
                    ha &= sorig[ka] > oi;
                    hb &= sorig[kb] > oi;
                }
                const uint64_t ma = __builtin_amdgcn_ballot_w64(ha);
                const uint64_t mb = __builtin_amdgcn_ballot_w64(hb);
                const uint32_t na = (uint32_t)__builtin_popcountll(ma);
                const uint32_t qa = __builtin_amdgcn_mbcnt_hi((uint32_t)(ma >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((uint32_t)ma, cnt));
                const uint32_t qb = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(mb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mb, cnt + na));
                // row-major rows have slack after the last row, so an overlong row
                // only spills into its neighbours (the host then rebuilds with a
                // larger capacity); column-major rows must stop at cap
                if (LOCAL) {
                    // 32-bit byte offsets from the row's (scalar) address
                    if (ha) *(uint16_t *)((char *)row16 + 2u * qa) = (uint16_t)ka;
                    if (hb) *(uint16_t *)((char *)row16 + 2u * qb) = (uint16_t)kb;
                } else if (!ELL) {
                    if (ha) row32[qa] = sslot[ka];
                    if (hb) row32[qb] = sslot[kb];
                } else {
                    if (ha && qa < (uint32_t)cap) row32[(int64_t)qa * n] = sslot[ka];
                    if (hb && qb < (uint32_t)cap) row32[(int64_t)qb * n] = sslot[kb];
                }
                cnt += na + (uint32_t)__builtin_popcountll(mb);
            }
            // padding up to a multiple of 8 entries: at most 7, one per lane
            const int32_t pe8 = min((int32_t)((cnt + 7) & ~7u), cap);
            const int32_t q = (int32_t)cnt + lane;
            if (q < pe8) {
                if (LOCAL)
                    row16[q] = (uint16_t)C;
                else
                    row32[ELL ? (int64_t)q * n : q] = pad;
            }
            if (lane == 0) len[t] = (int32_t)cnt;
            if constexpr (LOCAL) {
                if (lane == 0) lo[t] = make_int2((int)cnt, (int)(ro - (int64_t)(i - ib) * cap));
                ro += pe8;
            }
            if constexpr (INNER) {
                const int32_t ie8 = min((int32_t)((icnt + 7) & ~7u), cap);
                const int32_t qi = (int32_t)icnt + lane;
                if (qi < ie8) irow[qi] = (uint16_t)C;
                if (lane == 0) in_lo[t] = make_int2((int)icnt, (int)(rio - (int64_t)(i - ib) * cap));
                rio += ie8;
            }
            wmax = max(wmax, (int32_t)cnt);
        }
    }
    if (lane == 0) wmx[wv] = wmax;
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < NW; ++w) wmax = max(wmax, wmx[w]);
        if (wmax > 0) atomic_max_rare(maxlen, wmax);
        atomic_max_rare(maxnb, C);
        atomic_max_rare(maxnc, ncu);
    }
}

// Staged wave-per-i: a workgroup of 4 wavefronts owns STAGE_K consecutive
// cells along x and copies their common neighbourhood (nine rows of
// STAGE_K + 2 cells) into LDS; its wavefronts then take g i's at a time,
// 64/g lanes per i, each lane reading V list entries per trip (one 16-, 8-
// or 4-byte load) and the j-particles from LDS.
constexpr int VL_LDS_TB = 256;

// V list entries (16-bit) at byte offset vo of the tile's list rows: one
// 16-, 8- or 4-byte buffer load, entries in the low halves first.  The
// resource's range check returns zeros for reads past the end of the list
// array, so the prefetch of trips beyond a row needs no clamp.
template <int V>
__device__ __forceinline__ uint4 list_words(__amdgpu_buffer_rsrc_t r, uint32_t vo)
{
    if (V == 8) {
        const auto q = __builtin_amdgcn_raw_buffer_load_b128(r, vo, 0, 0);
        return make_uint4(q[0], q[1], q[2], q[3]);
    }
    if (V == 4) {
        const auto q = __builtin_amdgcn_raw_buffer_load_b64(r, vo, 0, 0);
        return make_uint4(q[0], q[1], 0u, 0u);
    }
    return make_uint4(__builtin_amdgcn_raw_buffer_load_b32(r, vo, 0, 0), 0u, 0u, 0u);
}

// Word 3 of a raw buffer resource on this architecture (32-bit dwords,
// range-checked against num_records bytes).
constexpr int BUF_RSRC_W3 = 0x00020000;

// base + S * (low or high 16 bits of w) in one v_mad_u32_u16: the LDS
// address of a staged record (S = 24) or of its species (S = 4) straight
// from a packed pair of 16-bit list entries.
template <bool HI, int S>
__device__ __forceinline__ uint32_t mad16(uint32_t w, uint32_t base)
{
    uint32_t a;
    if (HI)
        asm("v_mad_u32_u16 %0, %1, %2, %3 op_sel:[1,0,0,0]" : "=v"(a) : "v"(w), "i"(S), "v"(base));
    else
        asm("v_mad_u32_u16 %0, %1, %2, %3" : "=v"(a) : "v"(w), "i"(S), "v"(base));
    return a;
}

typedef __attribute__((address_space(3))) const double lds_cdouble;
typedef __attribute__((address_space(3))) const int lds_cint;
typedef __attribute__((address_space(3))) const unsigned lds_cuint;

// Fixed-point layout of the FP32-pair staged kernel: a staged record is
// {x, y, z} as 32-bit words (to_fx) of one frame for the whole grid, its
// species apart.  The separation of two records is the exact integer
// difference of their words, formed by the same FP64 subtraction as for
// FP64 coordinates and with no conversion instruction.  What is given up is
// the rounding of each coordinate to the grid 1/s (s is chosen so that every
// record, halo images included, stays within 1.5 2^30 steps of the centre:
// 1/s is 5.8e-8 sigma for a box of 175 sigma), below the FP32 pair law's
// own rounding.  The words are kept in global memory (12 bytes per record, the
// species apart), so that staging reads 12 bytes per record instead of the
// 32 of the FP64 records, and a staged record takes 12 bytes of LDS instead
// of 24.
__device__ __forceinline__ double fx_value(unsigned w)
{
    return __hiloint2double(0x43300000, (int)w);
}

// Fixed-point copy of the records for the FP32-pair staged kernel: x, y, z
// as words of one frame for the whole grid (centre c, scale s), 12 bytes per
// record, and the species apart.
__global__ void k_fx_records(int64_t nrec, const PosT *__restrict__ rec, double cx, double cy,
                             double cz, double s, FxWords *__restrict__ fxr,
                             int32_t *__restrict__ spec)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nrec) return;
    const PosT p = rec[k];
    fxr[k] = FxWords{to_fx(p.x, cx, s), to_fx(p.y, cy, s), to_fx(p.z, cz, s)};
    spec[k] = p.t;
}

// the padding record: word 0 on every axis (coordinate -2^31), at least
// sqrt(3) 2^29 / s from any staged particle (whose coordinates stay within
// FX_RANGE = 1.5 2^30 steps); with s = FX_RANGE / reach that is 0.58 reach,
// and reach is at least 3.5 (rc + skin), so beyond the cutoff
constexpr unsigned FX_PAD = 0u;

// Staging of the fixed-point layout: record k of the nine concatenated rows
// from the fixed-point record array (four per thread in flight, rows found
// without branches as in stage_rows).
__device__ __forceinline__ void stage_rows_fx(const FxWords *__restrict__ fxr,
                                              const int32_t *__restrict__ spec, const int *seg_b,
                                              const int *seg_c, int C, unsigned *sd, int *st,
                                              bool types, int tid, int nthr)
{
    constexpr int U = 4;
    int c[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) c[q] = seg_c[q + 1];
    for (int k0 = tid; k0 < C; k0 += U * nthr) {
        FxWords w[U];
        int t[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = min(k0 + u * nthr, C - 1);
            int r = 0;
#pragma unroll
            for (int q = 0; q < 8; ++q) r += k >= c[q];
            const int j = seg_b[r] + (k - seg_c[r]);
            w[u] = fxr[j];
            t[u] = types ? spec[j] : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u * nthr;
            if (k < C) {
                sd[3 * k] = w[u].x;
                sd[3 * k + 1] = w[u].y;
                sd[3 * k + 2] = w[u].z;
                if (types) st[k] = t[u];
            }
        }
    }
}

// The fused integrator step of one particle (record slot s, compact index
// t) along axis k from its force component f, given the axis coordinate x,
// velocity v and list-build reference xr and the species sp: v += f dt / (2m)
// twice (the end of this step and the start of the next) and x += v dt, the
// expressions of the separate sorted-order step, so trajectories agree bit
// for bit.  Returns the displacement from the reference.
template <bool FX>
__device__ __forceinline__ double kick_drift_axis(const KickArgs &ka, int s, int64_t t, int k,
                                                  double f, double x, double v, double xr, int sp)
{
    // 1/m of the species by selects (no dynamic index into the argument)
    double im = ka.im[0];
#pragma unroll
    for (int q = 1; q < MDLJ_MAX_SPECIES; ++q) im = sp == q ? ka.im[q] : im;
    const double h = 0.5 * ka.dt * im;
    const double u = (v + h * f) + h * f;
    ka.vs_out[3 * t + k] = u;
    const double y = x + ka.dt * u;
    (&ka.rec_out[s].x)[k] = y;
    if (FX) ((unsigned *)&ka.fxr_out[s])[k] = to_fx(y, ka.fx_c[k], ka.fx_s);
    return y - xr;
}

template <typename T, bool E, bool MS, int G, int V, bool KD>
__device__ __forceinline__ void vl_lds_body(const PosT *__restrict__ rec,
                                            const int32_t *__restrict__ start,
                                            const int32_t *__restrict__ ibase, const Grid &g,
                                            int tiles_x, const uint16_t *__restrict__ nbr_full,
                                            const int2 *__restrict__ lo_full, int32_t cap,
                                            int64_t n, int cmax, const LJTable<T> &tab,
                                            const ForceOut &fo, int remap, double fxs,
                                            const FxWords *__restrict__ fxr,
                                            const int32_t *__restrict__ fxspec, const KickArgs &ka,
                                            const InnerList &il)
{
    // FP32 pair law: fixed-point staged records; fxs is their scale and tab
    // holds sig^2 fxs^2, 24 eps fxs and rc^2 fxs^2, so that every pair
    // quantity comes out in its own units.  FP64 law: FP64 coordinates.
    constexpr bool FX = sizeof(T) == sizeof(float);
    constexpr int SEG = MDLJ_WAVE / G;
    constexpr int NW = VL_LDS_TB / MDLJ_WAVE;
    constexpr int KS = V * SEG;  // entries of one i per trip
    extern __shared__ __attribute__((aligned(16))) double stage[];
    __shared__ int seg_b[9];
    __shared__ int seg_c[10];
    __shared__ LdsTable<T> lt;
    __shared__ double red[2 * NW];
    __shared__ int s_moved;  // fused step: a particle crossed the inner list's bound
    const double rc2 = tab.rc2d;
    const int tid = threadIdx.x;
    // the wavefront index as a uniform value (i-group bases in scalar registers)
    const int lane = tid & (MDLJ_WAVE - 1), wv = __builtin_amdgcn_readfirstlane(tid / MDLJ_WAVE);
    if (MS) lds_table_load(lt, tab, tid, blockDim.x);
    // fused step: the padding record is carried over to the new records
    if (KD && blockIdx.x == 0 && tid == 0) {
        ka.rec_out[ka.pad_slot] = rec[ka.pad_slot];
        if (FX) ka.fxr_out[ka.pad_slot] = fxr[ka.pad_slot];
    }
    const int64_t tile = remap ? xcd_remap(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    const int tx = (int)((uint32_t)tile % (uint32_t)tiles_x);
    const uint32_t rr = (uint32_t)tile / (uint32_t)tiles_x;
    const int cy = (int)(rr % (uint32_t)g.n[1]);
    const int cz = (int)(rr / (uint32_t)g.n[1]);
    const int cx0 = tx * STAGE_K;
    const int ncx = min(STAGE_K, g.n[0] - cx0);
    // the list this tile reads: the pruned inner rows while they hold every
    // pair inside the cutoff, else the full rows (a uniform decision, from
    // the tile's word, which earlier launches wrote)
    bool use_in = false;
    if (il.tile_cur) {
        use_in = __builtin_amdgcn_readfirstlane(il.tile_cur[tile]) == 0;
    }
    const uint16_t *__restrict__ nbr = use_in ? il.nbr : nbr_full;
    const int2 *__restrict__ lo = use_in ? il.lo : lo_full;
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
    if (KD && tid == 9) s_moved = 0;
    // compact index of the tile's first particle (cells of a tile are consecutive)
    const int64_t c0 = (int64_t)cx0 + (int64_t)g.n[0] * (cy + (int64_t)g.n[1] * cz);
    const int64_t t0 = ibase[c0];
    // G i's per wavefront, SEG lanes each over the i's list (j fastest)
    const LanePair lp = lane_pair(LANE_I_MAJOR, G, MDLJ_WAVE, lane);
    const int l = lp.j;
    // list rows of the tile's particles (t0 onwards) through one buffer
    // resource; lane offsets in bytes
    const __amdgpu_buffer_rsrc_t lr = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(nbr + min(t0, n - 1) * cap), (short)0,
        (int)min((n - min(t0, n - 1)) * cap * 2, (int64_t)0x7fffffff), BUF_RSRC_W3);
    // The first i-group of this wavefront: its records, list lengths and the
    // first two trips of list entries are requested before the staging, so
    // their latency overlaps it.  The loads are unconditional (a branch
    // around a load makes the compiler wait for it at the merge): inactive
    // lanes read the tile's first row and list length; what those reads
    // return is never used.
    int i0 = ib + wv * G;
    int i = i0 + lp.i;
    bool act = i < ie;
    int64_t t = t0 + (act ? i - ib : 0);
    // i's record: FP64 coordinates and species, or (fixed point) the words
    // and species
    PosT pi;
    FxWords qi;
    int qt = 0;
    auto load_i = [&](int k) {
        if constexpr (FX) {
            qi = fxr[k];
            if (MS) qt = fxspec[k];
        } else {
            pi = rec[k];
        }
    };
    load_i(act ? i : ib);
    // fused step: lane l of an i's segment needs word l & 3 of its record
    // (x, y, z, or species and caller index) and, for l < 3, that axis's
    // velocity and reference position; requested with the i-group's other
    // loads, so that their latency overlaps the pair loop
    double kx = 0.0, kv = 0.0, kr = 0.0;
    auto load_kd = [&]() {
        if constexpr (KD) {
            const int lk = l & 3, la = min(lk, 2);
            const int64_t ts = min(t, n - 1);
            kx = ((const double *)(rec + (act ? i : ib)))[lk];
            kv = ka.vs_in[3 * ts + la];
            kr = ka.xrs[la * n + ts];
        }
    };
    load_kd();
    // row t: its length and its start less t cap (tile-packed rows)
    const int2 q = lo[min(t, n - 1)];
    int32_t L = act ? q.x : 0;
    uint32_t vo = (uint32_t)(((t - t0) * cap + q.y + V * l) * 2);
    uint4 wa = list_words<V>(lr, vo);
    uint4 wb = list_words<V>(lr, vo + 2 * KS);
    __syncthreads();
    if (tid == 0) {
        seg_c[0] = 0;
        for (int r = 0; r < 9; ++r) seg_c[r + 1] += seg_c[r];
    }
    __syncthreads();
    const int C = seg_c[9];
    // FP64 layout: x, y, z of staged record k interleaved at sp[3k .. 3k+2]
    // (one LDS address per candidate), species in st[k]
    double *sp = stage;
    int *st = (int *)(stage + 3 * cmax);
    // fixed-point layout: x, y, z words of record k at sd[3k .. 3k+2] (a
    // 12-byte stride spreads random records over all LDS banks), species in
    // st2[k]
    unsigned *sd = (unsigned *)stage;
    int *st2 = (int *)(sd + 3 * cmax);
    if constexpr (FX) {
        stage_rows_fx(fxr, fxspec, seg_b, seg_c, C, sd, st2, MS, tid, blockDim.x);
        if (tid == 0) {
            sd[3 * C] = sd[3 * C + 1] = sd[3 * C + 2] = FX_PAD;
            if (MS) st2[C] = 0;
        }
    } else {
        stage_rows<3>(rec, seg_b, seg_c, C, sp, sp + 1, sp + 2, st, MS, tid, blockDim.x);
        if (tid == 0) {
            sp[3 * C] = sp[3 * C + 1] = sp[3 * C + 2] = PAD_COORD;
            if (MS) st[C] = 0;
        }
    }
    __syncthreads();
    // LDS byte addresses of the staged coordinates and species
    const uint32_t xb = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) double *)sp;
    const uint32_t tb = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) int *)(FX ? st2 : st);
    // i's coordinates in the frame of its staged partners, and its species
    auto frame = [&](double &x, double &y, double &z) {
        if constexpr (FX) {
            x = fx_value(qi.x);
            y = fx_value(qi.y);
            z = fx_value(qi.z);
        } else {
            x = pi.x;
            y = pi.y;
            z = pi.z;
        }
    };
    auto species_i = [&]() -> int {
        if constexpr (FX)
            return qt;
        else
            return pi.t;
    };
    double xi, yi, zi;
    frame(xi, yi, zi);
    double bu = 0.0, bw = 0.0;
    for (bool first = true; i0 < ie; i0 += NW * G, first = false) {
        if (!first) {
            i = i0 + lp.i;
            act = i < ie;
            t = t0 + (act ? i - ib : 0);
            load_i(act ? i : ib);
            load_kd();
            frame(xi, yi, zi);
            const int2 qn = lo[min(t, n - 1)];
            L = act ? qn.x : 0;
            vo = (uint32_t)(((t - t0) * cap + qn.y + V * l) * 2);
            wa = list_words<V>(lr, vo);
            wb = list_words<V>(lr, vo + 2 * KS);
        }
        Acc a;
        acc_zero(a);
        auto trip = [&](const uint4 q) {
            const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int u = 0; u < V; ++u) {
                double fxp, fyp, fzp;
                if constexpr (FX) {
                    const uint32_t ad = (u & 1) ? mad16<true, 12>(w[u >> 1], xb)
                                                : mad16<false, 12>(w[u >> 1], xb);
                    int tj = 0;
                    if (MS) {
                        const uint32_t at = (u & 1) ? mad16<true, 4>(w[u >> 1], tb)
                                                    : mad16<false, 4>(w[u >> 1], tb);
                        tj = *(lds_cint *)(uintptr_t)at;
                    }
                    lds_cuint *q = (lds_cuint *)(uintptr_t)ad;
                    const PairP<T> p = pair_params<T, MS>(tab, lt, species_i(), tj);
                    lj_pair<T, E>(xi, yi, zi, fx_value(q[0]), fx_value(q[1]), fx_value(q[2]),
                                  true, p, rc2, a, fxp, fyp, fzp);
                } else {
                    const uint32_t ad = (u & 1) ? mad16<true, 24>(w[u >> 1], xb)
                                                : mad16<false, 24>(w[u >> 1], xb);
                    int tj = 0;
                    if (MS) {
                        const uint32_t at = (u & 1) ? mad16<true, 4>(w[u >> 1], tb)
                                                    : mad16<false, 4>(w[u >> 1], tb);
                        tj = *(lds_cint *)(uintptr_t)at;
                    }
                    const PairP<T> p = pair_params<T, MS>(tab, lt, species_i(), tj);
                    lds_cdouble *q = (lds_cdouble *)(uintptr_t)ad;
                    lj_pair<T, E>(xi, yi, zi, q[0], q[1], q[2], true, p, rc2, a, fxp, fyp, fzp);
                }
            }
        };
        // two trips in flight.  Both reloads are unconditional, so every
        // path through the loop issues the same loads in the same order
        // and each wait covers only the load its trip needs (a load
        // inside the branch would make the loop head wait for all of
        // them).
        for (int32_t k0 = V * l; k0 < L; k0 += 2 * KS, vo += 4 * KS) {
            trip(wa);
            wa = list_words<V>(lr, vo + 4 * KS);
            if (k0 + KS < L) trip(wb);
            wb = list_words<V>(lr, vo + 6 * KS);
        }
        a.fx = seg_sum(a.fx, SEG);
        a.fy = seg_sum(a.fy, SEG);
        a.fz = seg_sum(a.fz, SEG);
        if constexpr (KD) {
            // lanes 0, 1, 2 of an i's segment step its x, y and z, lane 3
            // copies species and caller index: one 32-byte record store
            static_assert(SEG >= 4, "the fused step needs 4 lanes per i");
            double d = 0.0;
            if (act && l < 3)
                d = kick_drift_axis<FX>(ka, i, t, l, l == 0 ? a.fx : (l == 1 ? a.fy : a.fz), kx,
                                        kv, kr, species_i());
            if (act && l == 3) ((double *)(ka.rec_out + i))[3] = kx;
            const double dy = __shfl_down(d, 1, SEG), dz = __shfl_down(d, 2, SEG);
            const double d2 = d * d + dy * dy + dz * dz;
            if (act && l == 0 && !(d2 <= ka.thr2)) atomicOr(ka.flag, 1);
            // a particle of the tile crossed the inner list's bound
            if (act && l == 0 && !(d2 <= ka.thr_in2)) s_moved = 1;
        } else if (act && l == 0) {
            fo.fx[i] = a.fx;
            fo.fy[i] = a.fy;
            fo.fz[i] = a.fz;
        }
        if (E) {
            bu += a.u;
            // the fixed-point path sums 24 eps s6 (2 s6 - 1) fxs
            bw += FX ? a.w * (1.0 / fxs) : a.w;
        }
    }
    if constexpr (KD) {
        // the inner list's bound crossed in this tile: the next launch gives
        // up the inner rows in the 27 tiles around it (every tile whose
        // staged rows include cells of this one)
        if (il.tile_cur) {
            __syncthreads();
            // the tile's coordinates again (not kept live through the loop)
            const int64_t tl = remap ? xcd_remap(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
            if (s_moved && tid < 27) {
                const int ux = (int)((uint32_t)tl % (uint32_t)tiles_x);
                const uint32_t ur = (uint32_t)tl / (uint32_t)tiles_x;
                const int uy = (int)(ur % (uint32_t)g.n[1]), uz = (int)(ur / (uint32_t)g.n[1]);
                const int nx = (ux + tid % 3 - 1 + tiles_x) % tiles_x;
                const int ny = (uy + (tid / 3) % 3 - 1 + g.n[1]) % g.n[1];
                const int nz = (uz + tid / 9 - 1 + g.n[2]) % g.n[2];
                atomicOr(il.tile_next + nx + (int64_t)tiles_x * (ny + (int64_t)g.n[1] * nz), 1);
            }
            // a word already set stays set in the next copy
            if (tid == 32 && il.tile_cur[tl]) atomicOr(il.tile_next + tl, 1);
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

#define VL_LDS_PARAMS                                                                            \
    const PosT *__restrict__ rec, const int32_t *__restrict__ start,                            \
        const int32_t *__restrict__ ibase, Grid g, int tiles_x, const uint16_t *__restrict__ nbr, \
        const int2 *__restrict__ lo, int32_t cap, int64_t n, int cmax, LJTable<T> tab,          \
        ForceOut fo, int remap, double fxs, const FxWords *__restrict__ fxr,                     \
        const int32_t *__restrict__ fxspec, KickArgs ka, InnerList il

template <typename T, bool E, bool MS, int G, int V, bool KD>
__global__ __launch_bounds__(VL_LDS_TB) void k_vl_lds(VL_LDS_PARAMS)
{
    vl_lds_body<T, E, MS, G, V, KD>(rec, start, ibase, g, tiles_x, nbr, lo, cap, n, cmax, tab, fo,
                                    remap, fxs, fxr, fxspec, ka, il);
}

// The same, held to 64 registers so that eight wavefronts share a SIMD:
// for the FP32-pair fused step, whose prefetched operands would otherwise
// cost two of them (taken only where the cap causes no spills: one
// species, 8 or 16 i's per wavefront).
template <typename T, bool E, bool MS, int G, int V, bool KD>
__global__ __launch_bounds__(VL_LDS_TB) __attribute__((amdgpu_waves_per_eu(8, 8))) void
k_vl_lds_w8(VL_LDS_PARAMS)
{
    vl_lds_body<T, E, MS, G, V, KD>(rec, start, ibase, g, tiles_x, nbr, lo, cap, n, cmax, tab, fo,
                                    remap, fxs, fxr, fxspec, ka, il);
}
#undef VL_LDS_PARAMS

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
                const bool in = lj_pair<T, E>(pi.x, pi.y, pi.z, pj[u].x, pj[u].y, pj[u].z,
                                              jj[u] >= 0, p, rc2, a, fxp, fyp, fzp);
                // pairs in the skin (and list padding) add nothing to j
                if (N3 && in) {
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
    const LanePair lp = lane_pair(LANE_I_MAJOR, G, MDLJ_WAVE, lane);
    const int64_t t = wave * G + lp.i;
    const int l = lp.j;
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
                const bool in = lj_pair<T, E>(pi.x, pi.y, pi.z, xj[u], yj[u], zj[u], true, p, rc2,
                                              a, fxp, fyp, fzp);
                // pairs in the skin and the padding entries add nothing to j
                if (N3 && in) {
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

// The fixed-point words of the current records, converted when stale.  The
// frame is centred on the box; every record (halo images one cell beyond
// the box) plus rc + skin for particles that drift before a rebuild stays
// within FX_RANGE steps of the centre.  *scale receives s.
static mdlj_status fx_words(mdlj_ctx *ctx, double *scale)
{
    const Grid &g = ctx->grid;
    double reach = 0.0;
    for (int a = 0; a < 3; ++a) reach = std::max(reach, 0.5 * g.L[a] + g.h[a] * g.edge[a]);
    reach += ctx->rc + ctx->skin;
    const double fxs = FX_RANGE / reach;
    // Rounding each coordinate to the grid 1/s moves a force by up to about
    // 55 (1/s) / sigma relative to the scene's force scale (measured against
    // the FP64 oracle on dense liquids and lattices); with the FP32 pair
    // law's own 2.5e-6 the 1e-5 bar holds while 1/s <= 1e-7 of the smallest
    // sigma (boxes up to about 310 sigma); beyond, the kernel is refused
    double sig_min = ctx->sig[0];
    for (int k = 1; k < ctx->nspec; ++k) sig_min = std::min(sig_min, ctx->sig[k]);
    if (fxs * sig_min < 1.0e7)
        return set_err(ctx, MDLJ_ERR_ARG,
                       "box too large for the fixed-point frame of the FP32-pair staged kernel");
    const double c[3] = {0.5 * g.L[0], 0.5 * g.L[1], 0.5 * g.L[2]};
    *scale = fxs;
    if (ctx->fx_valid && ctx->fx_s == fxs && memcmp(ctx->fx_c, c, sizeof c) == 0) return MDLJ_OK;
    const int64_t nrec = ctx->n_ext + 1;  // records + the padding record
    STCHK(ensure(ctx, ctx->b_fxrec, sizeof(FxWords) * nrec));
    STCHK(ensure(ctx, ctx->b_fxspec, sizeof(int32_t) * nrec));
    k_fx_records<<<ceil_div(nrec, 256), 256, 0, ctx->stream>>>(
        nrec, (const PosT *)ctx->b_sorted.p, c[0], c[1], c[2], fxs, (FxWords *)ctx->b_fxrec.p,
        (int32_t *)ctx->b_fxspec.p);
    HIPCHK(ctx, hipGetLastError());
    ctx->fx_s = fxs;
    memcpy(ctx->fx_c, c, sizeof c);
    ctx->fx_valid = true;
    return MDLJ_OK;
}


template <typename T, bool E, bool MS, bool N3>
int64_t launch_vl(mdlj_ctx *ctx, const mdlj_config &cfg, const LJTable<T> &tab, ForceOut &fo,
                  int remap, const KickArgs *kdp)
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
        constexpr bool FX = sizeof(T) == sizeof(float);
        const size_t lds = (size_t)cmax * ((FX ? 3 * sizeof(unsigned) : 3 * sizeof(double)) +
                                           (MS ? sizeof(int) : 0));
        if (lds > (size_t)STAGE_LDS_BYTES || N3) return -2;
        double fxs = 1.0;
        if (FX) {
            const mdlj_status fst = fx_words(ctx, &fxs);
            if (fst != MDLJ_OK) return fst == MDLJ_ERR_ARG ? -5 : -4;
        }
        const FxWords *fxr = nullptr;
        const int32_t *fxspec = nullptr;
        KickArgs kk = {};
        if (kdp) kk = *kdp;
        if (FX) {
            fxr = (const FxWords *)ctx->b_fxrec.p;
            fxspec = (const int32_t *)ctx->b_fxspec.p;
            if (kdp && !E) {
                if (ensure(ctx, ctx->b_fxrec2, sizeof(FxWords) * nrec) != MDLJ_OK) return -4;
                kk.fxr_out = (FxWords *)ctx->b_fxrec2.p;
                memcpy(kk.fx_c, ctx->fx_c, sizeof kk.fx_c);
                kk.fx_s = fxs;
            }
        }
        LJTable<T> tx = tab;
        if (FX) {
            for (int k = 0; k < tab.ns * tab.ns; ++k) {
                tx.sig2[k] = (T)((double)tab.sig2[k] * fxs * fxs);
                tx.eps24[k] = (T)((double)tab.eps24[k] * fxs);
            }
            tx.rc2d = tab.rc2d * fxs * fxs;
            tx.rc2 = (T)tx.rc2d;
        }
        const int key = cfg.tile_i * 100 + cfg.tile_j;
        if (key != 802 && key != 804 && key != 1602 && key != 1604 && key != 408) return -1;
        const int tiles_x = (int)ceil_div(g.n[0], STAGE_K);
        const int64_t nbt = (int64_t)tiles_x * g.n[1] * g.n[2];
        const int32_t *ibase = (const int32_t *)ctx->b_icnt.p + g.ncell_int + 1;
        const uint16_t *nbr16 = (const uint16_t *)ctx->b_nbr.p;
        const int2 *lo = (const int2 *)ctx->b_nlo.p;
        const int32_t *start = (const int32_t *)ctx->b_start.p;
        // the fused integrator step only with forces alone (no energies)
        const bool kd = kdp != nullptr && !E;
        // the pruned inner list, written by the list build, while valid
        InnerList il = {};
        if (ctx->inner == 1) {
            il.nbr = (uint16_t *)ctx->b_nbr_in.p;
            il.lo = (const int2 *)ctx->b_nlo_in.p;
            int32_t *tw = (int32_t *)ctx->b_tilebad.p;
            il.tile_cur = tw + ctx->inner_par * nbt;
            il.tile_next = tw + (ctx->inner_par ^ 1) * nbt;
            const double h = 0.5 * PRUNE_FRACTION * ctx->skin;
            kk.thr_in2 = h * h;
        }
        const KickArgs none = {};
#define VL_LDS(GG, VV)                                                                          \
    do {                                                                                        \
        bool done = false;                                                                      \
        if constexpr (FX && !MS && GG >= 8) {                                                   \
            if (kd) {                                                                           \
                k_vl_lds_w8<T, false, MS, GG, VV, true><<<nbt, VL_LDS_TB, lds, s>>>(            \
                    rec, start, ibase, g, tiles_x, nbr16, lo, cap, n, cmax, tx, fo, remap, fxs, \
                    fxr, fxspec, kk, il);                                                       \
                done = true;                                                                    \
            }                                                                                   \
        }                                                                                       \
        if (done) break;                                                                        \
        if (kd)                                                                                 \
            k_vl_lds<T, false, MS, GG, VV, true><<<nbt, VL_LDS_TB, lds, s>>>(                   \
                rec, start, ibase, g, tiles_x, nbr16, lo, cap, n, cmax, tx, fo, remap, fxs, fxr,   \
                fxspec, kk, il);                                                                \
        else                                                                                    \
            k_vl_lds<T, E, MS, GG, VV, false><<<nbt, VL_LDS_TB, lds, s>>>(                      \
                rec, start, ibase, g, tiles_x, nbr16, lo, cap, n, cmax, tx, fo, remap, fxs, fxr,   \
                fxspec, none, il);                                                              \
    } while (0)
        switch (key) {
        case 802: VL_LDS(8, 2); break;
        case 804: VL_LDS(8, 4); break;
        case 1602: VL_LDS(16, 2); break;
        case 1604: VL_LDS(16, 4); break;
        case 408: VL_LDS(4, 8); break;
        default: return -1;
        }
#undef VL_LDS
        if (kd) inner_flip(ctx);
        ctx->kd_done = kd;
        ctx->kd_fx = kd && FX;
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
                     int remap, const KickArgs *kdp)
{
    if (cfg.newton3) return launch_vl<T, E, MS, true>(ctx, cfg, tab, fo, remap, kdp);
    return launch_vl<T, E, MS, false>(ctx, cfg, tab, fo, remap, kdp);
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
    // the integrator step fused into the staged kernel (decided by kd_prepare)
    KickArgs ka;
    const KickArgs *kdp = nullptr;
    if (ctx->kd_go && cfg.staged && !cfg.newton3 && !energy) {
        STCHK(kd_args(ctx, &ka));
        kdp = &ka;
    }
    int64_t nw;
    if (energy) {
        const int64_t maxw = std::max<int64_t>(ctx->n + 64, ctx->grid.ncell_int);
        STCHK(partial_buffer(ctx, 2 * maxw, &fo.partial));
        nw = ms ? launch_vl_n3<T, true, true>(ctx, cfg, tab, fo, remap, nullptr)
                : launch_vl_n3<T, true, false>(ctx, cfg, tab, fo, remap, nullptr);
    } else {
        nw = ms ? launch_vl_n3<T, false, true>(ctx, cfg, tab, fo, remap, kdp)
                : launch_vl_n3<T, false, false>(ctx, cfg, tab, fo, remap, kdp);
    }
    if (nw == -2) return set_err(ctx, MDLJ_ERR_ARG, "neighbourhood too large for LDS staging");
    if (nw == -3) return set_err(ctx, MDLJ_ERR_ARG, "too many records for 32-bit buffer offsets");
    if (nw == -4) return MDLJ_ERR_NOMEM;
    if (nw == -5) return MDLJ_ERR_ARG;  // message set by fx_words
    if (nw < 0) return set_err(ctx, MDLJ_ERR_ARG, "unsupported Verlet-list shape");
    HIPCHK(ctx, hipGetLastError());
    *nblocks = nw;
    return MDLJ_OK;
}

size_t build_tile_lds(bool local, bool half, int cmax, int ccand)
{
    return (size_t)(cmax + 1) * (3 * sizeof(double) + (local ? 0 : sizeof(int32_t)) +
                                 (half ? sizeof(int32_t) : 0)) +
           (size_t)(ccand + CAND_PAD + CAND_SLACK) * sizeof(uint16_t);
}

mdlj_status launch_build_tile(mdlj_ctx *ctx, bool local, bool half, bool ell, double rl2,
                              bool trim, int cmax, int ccand, int32_t cap, bool inner, double rin2)
{
    const Grid &g = ctx->grid;
    const int tiles_x = (int)ceil_div(g.n[0], STAGE_K);
    const int64_t nbt = (int64_t)tiles_x * g.n[1] * g.n[2];
    const size_t lds = build_tile_lds(local, half, cmax, ccand);
    const PosT *rec = (const PosT *)ctx->b_sorted.p;
    const int32_t *start = (const int32_t *)ctx->b_start.p;
    const int32_t *hstart = (const int32_t *)ctx->b_hstart.p;
    const int32_t *ibase = (const int32_t *)ctx->b_icnt.p + g.ncell_int + 1;
    int32_t *maxlen = (int32_t *)ctx->b_flags.p + 12;
    int32_t *maxnb = (int32_t *)ctx->b_flags.p + 14;
    int32_t *maxnc = (int32_t *)ctx->b_flags.p + 15;
    int32_t *len = (int32_t *)ctx->b_nlen.p;
    void *nbr = ctx->b_nbr.p;
    const int32_t pad = (int32_t)ctx->n_ext;
    const int64_t n = ctx->n;
    hipStream_t s = ctx->stream;
    uint16_t *in_nbr = inner ? (uint16_t *)ctx->b_nbr_in.p : nullptr;
    int2 *lo = local ? (int2 *)ctx->b_nlo.p : nullptr;
    int2 *in_lo = inner ? (int2 *)ctx->b_nlo_in.p : nullptr;
#define VL_BT(L, H, E)                                                                          \
    k_vl_build_tile<L, H, E, false><<<nbt, BUILD_TB, lds, s>>>(                                 \
        rec, start, hstart, ibase, g, tiles_x, rl2, trim ? 1 : 0, cmax, ccand, n, cap, pad, nbr, \
        len, maxlen, maxnb, maxnc, 1, nullptr, 0.0, lo, nullptr)
    if (local) {
        if (half || ell) return set_err(ctx, MDLJ_ERR_ARG, "local lists are full row-major lists");
        if (inner)
            k_vl_build_tile<true, false, false, true><<<nbt, BUILD_TB, lds, s>>>(
                rec, start, hstart, ibase, g, tiles_x, rl2, trim ? 1 : 0, cmax, ccand, n, cap, pad,
                nbr, len, maxlen, maxnb, maxnc, 1, in_nbr, rin2, lo, in_lo);
        else
            VL_BT(true, false, false);
    } else if (ell) {
        if (half)
            VL_BT(false, true, true);
        else
            VL_BT(false, false, true);
    } else if (half) {
        VL_BT(false, true, false);
    } else {
        VL_BT(false, false, false);
    }
#undef VL_BT
    HIPCHK(ctx, hipGetLastError());
    return MDLJ_OK;
}

// Sum over rows of the row length rounded up to a multiple of 8.
__global__ __launch_bounds__(256) void k_list_entries(const int32_t *__restrict__ len, int64_t n,
                                                      unsigned long long *__restrict__ out)
{
    __shared__ unsigned long long red[256 / MDLJ_WAVE];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long v = t < n ? (unsigned long long)((len[t] + 7) & ~7) : 0ull;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & (MDLJ_WAVE - 1)) == 0) red[threadIdx.x / MDLJ_WAVE] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)blockDim.x / MDLJ_WAVE; ++w) v += red[w];
        atomicAdd(out, v);
    }
}

// Caller indices of the pairs a Verlet list holds, for checking the list:
// entry k of compact row t becomes (caller index of i, caller index of j)
// at off[t] + k.  layout 0: column-major slots (nbr[k n + t]); 1: row-major
// slots (nbr[t cap + k]); 2: 16-bit staged indices, decoded through the cell
// starts of the nine rows of i's x-tile, the order in which the force
// kernel stages them.  An entry that names no record gives j = -2.
__global__ __launch_bounds__(256) void k_vl_pairs(const PosT *__restrict__ rec,
                                                  const int32_t *__restrict__ start,
                                                  const int32_t *__restrict__ ilist,
                                                  const int32_t *__restrict__ cell_of, Grid g,
                                                  int64_t n, int64_t nrec, const void *nbr,
                                                  const int32_t *__restrict__ len,
                                                  const int2 *__restrict__ lo, int32_t cap,
                                                  int layout, const int64_t *__restrict__ off,
                                                  int32_t *__restrict__ pi,
                                                  int32_t *__restrict__ pj)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int32_t oi = rec[ilist[t]].orig;
    const int32_t L = len[t];
    int32_t *a = pi + off[t];
    int32_t *b = pj + off[t];
    int32_t rb[9], rl[9];
    if (layout == 2) {
        const int64_t e = cell_of[oi];
        const int cx = (int)(e % g.stride[1]) - g.h[0];
        const int cy = (int)((e / g.stride[1]) % g.e[1]) - g.h[1];
        const int cz = (int)(e / g.stride[2]) - g.h[2];
        const int cx0 = (cx / STAGE_K) * STAGE_K;
        const int ncx = min(STAGE_K, g.n[0] - cx0);
        for (int r = 0; r < 9; ++r) {
            const int dy = r % 3 - 1, dz = r / 3 - 1;
            const int64_t ej = (int64_t)(cy + dy + g.h[1]) * g.stride[1] +
                               (int64_t)(cz + dz + g.h[2]) * g.stride[2] + cx0 - 1 + g.h[0];
            rb[r] = start[ej];
            rl[r] = start[ej + ncx + 2] - start[ej];
        }
    }
    for (int32_t k = 0; k < L; ++k) {
        int64_t sj = -1;
        if (layout == 2) {
            int32_t q = ((const uint16_t *)nbr)[t * cap + lo[t].y + k];
            for (int r = 0; r < 9 && sj < 0; ++r) {
                if (q < rl[r]) sj = rb[r] + q;
                else q -= rl[r];
            }
        } else if (layout == 1) {
            sj = ((const int32_t *)nbr)[t * cap + k];
        } else {
            sj = ((const int32_t *)nbr)[(int64_t)k * n + t];
        }
        a[k] = oi;
        b[k] = (sj >= 0 && sj < nrec) ? rec[sj].orig : -2;
    }
}

}  // namespace

mdlj_status vl_list_entries(mdlj_ctx *ctx, int64_t *entries)
{
    STCHK(ensure(ctx, ctx->b_misc, sizeof(unsigned long long)));
    // b_misc is binning scratch, free between builds
    unsigned long long *d = (unsigned long long *)ctx->b_misc.p;
    HIPCHK(ctx, hipMemsetAsync(d, 0, sizeof *d, ctx->stream));
    k_list_entries<<<ceil_div(ctx->n, 256), 256, 0, ctx->stream>>>((const int32_t *)ctx->b_nlen.p,
                                                                  ctx->n, d);
    HIPCHK(ctx, hipGetLastError());
    unsigned long long h = 0;
    HIPCHK(ctx, hipMemcpyAsync(&h, d, sizeof h, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    *entries = (int64_t)h;
    return MDLJ_OK;
}

InnerMark inner_marker(mdlj_ctx *ctx)
{
    InnerMark m = {};
    if (ctx->inner != 1) return m;
    int32_t *tw = (int32_t *)ctx->b_tilebad.p;
    const int64_t nt = ctx->inner_ntiles;
    m.cur = tw + ctx->inner_par * nt;
    m.next = tw + (ctx->inner_par ^ 1) * nt;
    m.cell_of = (const int32_t *)ctx->b_cell_of.p;
    m.g = ctx->grid;
    m.tiles_x = (int)ceil_div(ctx->grid.n[0], STAGE_K);
    m.ntiles = nt;
    const double h = 0.5 * PRUNE_FRACTION * ctx->skin;
    m.thr2 = h * h;
    return m;
}

void inner_flip(mdlj_ctx *ctx)
{
    if (ctx->inner == 1) ctx->inner_par ^= 1;
}

mdlj_status vl_build(mdlj_ctx *ctx, const mdlj_config &cfg)
{
    const Grid &g = ctx->grid;
    const int64_t n = ctx->n;
    // the compact interior order (ilist, ibase) comes with the binning
    const double rl = ctx->rc + ctx->skin;
    const double vol = ctx->box[0] * ctx->box[1] * ctx->box[2];
    const double est = (double)n / vol * 4.18879020478639 * rl * rl * rl * (cfg.newton3 ? 0.5 : 1.0);
    int64_t cap = (int64_t)(1.3 * est) + 16;
    if (ctx->nbr_cap > cap && ctx->built_cfg.newton3 == cfg.newton3) cap = ctx->nbr_cap;
    cap = (cap + 7) & ~(int64_t)7;
    STCHK(ensure(ctx, ctx->b_nlen, sizeof(int32_t) * n));
    // local lists: each row's length and start for the staged kernel
    if (cfg.staged) STCHK(ensure(ctx, ctx->b_nlo, sizeof(int2) * n));
    int32_t *maxlen = (int32_t *)ctx->b_flags.p + 12;
    int32_t *maxnb = (int32_t *)ctx->b_flags.p + 14;
    const bool rowmajor = cfg.order != MDLJ_ORD_I_PER_LANE;
    const bool local = cfg.staged != 0;
    const size_t esize = local ? sizeof(uint16_t) : sizeof(int32_t);
    // LDS of the tiled build: staged records (x, y, z; slot unless local;
    // caller index for half lists) and the candidate lists.  Sized from the
    // maxima of the last tiled build on this grid (+1/8, the particles have
    // moved little since), else from a pre-pass over the tiles; a tile that
    // does not fit reports its sizes and the build is repeated with exact
    // ones.  Candidates are trimmed by cell halves only when cells are wider
    // than rc + skin by a margin far above rounding.
    const bool trim = g.edge[0] >= rl + 1e-9 * ctx->box[0];
    const int key[4] = {g.n[0], g.n[1], g.n[2], trim ? 1 : 0};
    bool hinted = ctx->tile_c_hint > 0 && memcmp(key, ctx->tile_hint_key, sizeof key) == 0;
    int cmax = 0, ccand = 0;
    auto exact_sizes = [&]() -> mdlj_status {
        int32_t *sz = (int32_t *)ctx->b_flags.p + 24;
        const int tiles_x = (int)ceil_div(g.n[0], STAGE_K);
        const int64_t nbt = (int64_t)tiles_x * g.n[1] * g.n[2];
        HIPCHK(ctx, hipMemsetAsync(sz, 0, 2 * sizeof(int32_t), ctx->stream));
        k_tile_sizes<<<ceil_div(nbt, 256), 256, 0, ctx->stream>>>(
            (const int32_t *)ctx->b_start.p, (const int32_t *)ctx->b_hstart.p, g, tiles_x, nbt,
            trim ? 1 : 0, sz);
        HIPCHK(ctx, hipGetLastError());
        int32_t h[2] = {0, 0};
        HIPCHK(ctx, hipMemcpyAsync(h, sz, sizeof h, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        cmax = h[0];
        ccand = h[1];
        return MDLJ_OK;
    };
    if (hinted) {
        cmax = ctx->tile_c_hint + ctx->tile_c_hint / 8 + 16;
        ccand = ctx->tile_nc_hint + ctx->tile_nc_hint / 8 + 64;
    } else {
        STCHK(exact_sizes());
    }
    bool tile_ok = cmax > 0 &&
                   build_tile_lds(local, cfg.newton3 != 0, cmax, ccand) <= (size_t)STAGE_LDS_BYTES;
    // a row of the tiled build may run past its capacity before the host
    // sees it (it then rebuilds): slack of the longest possible row
    const int64_t slack = rowmajor ? 27 * (int64_t)ctx->max_cell + 8 : 0;
    bool overlap = false;
    for (int attempt = 0; attempt < 3; ++attempt) {
        if ((double)cap * (double)n * (double)esize > 64e9)
            return set_err(ctx, MDLJ_ERR_OVERFLOW, "Verlet lists too large");
        STCHK(ensure(ctx, ctx->b_nbr, esize * (n * cap + slack)));
        // the four maxima start at zero: cleared by the binning and by the
        // publishing kernel after each build
        const int64_t sk = rowmajor ? 1 : n;
        const int64_t st = rowmajor ? cap : 1;
        const bool tiled = tile_ok;
        // the pruned inner list, written by the tiled build of the staged
        // kernels' lists (an allocation-free call goes without it rather
        // than grow its buffers)
        bool inner = false;
        const int64_t ntiles = ceil_div(g.n[0], STAGE_K) * g.n[1] * g.n[2];
        if (tiled && local && !cfg.newton3 && ctx->prune && ctx->skin > 0.0) {
            const size_t ib = esize * (size_t)(n * cap + slack), lb = sizeof(int2) * (size_t)n;
            const size_t tb = 2 * sizeof(int32_t) * (size_t)ntiles;
            if (!ctx->no_alloc || (ctx->b_nbr_in.bytes >= ib && ctx->b_nlo_in.bytes >= lb &&
                                   ctx->b_tilebad.bytes >= tb)) {
                STCHK(ensure(ctx, ctx->b_nbr_in, ib));
                STCHK(ensure(ctx, ctx->b_nlo_in, lb));
                STCHK(ensure(ctx, ctx->b_tilebad, tb));
                inner = true;
            }
        }
        const double rin = ctx->rc + PRUNE_FRACTION * ctx->skin;
        if (tiled) {
            STCHK(launch_build_tile(ctx, local, cfg.newton3 != 0, !rowmajor, rl * rl, trim, cmax,
                                    ccand, (int32_t)cap, inner, rin * rin));
        } else if (local) {
            k_vl_build_local<<<ceil_div(n, 256), 256, 0, ctx->stream>>>(
                (const PosT *)ctx->b_sorted.p, (const int32_t *)ctx->b_start.p,
                (const int32_t *)ctx->b_ilist.p, (const int32_t *)ctx->b_cell_of.p, g, n, rl * rl,
                (int32_t)cap, (uint16_t *)ctx->b_nbr.p, (int32_t *)ctx->b_nlen.p,
                (int2 *)ctx->b_nlo.p, maxlen, maxnb);
        } else {
            k_vl_build<<<ceil_div(n, 256), 256, 0, ctx->stream>>>(
                (const PosT *)ctx->b_sorted.p, (const int32_t *)ctx->b_start.p,
                (const int32_t *)ctx->b_ilist.p, (const int32_t *)ctx->b_cell_of.p, g, n, rl * rl,
                cfg.newton3 ? 1 : 0, sk, st, (int32_t)cap, (int32_t)ctx->n_ext,
                (int32_t *)ctx->b_nbr.p, (int32_t *)ctx->b_nlen.p, maxlen);
        }
        HIPCHK(ctx, hipGetLastError());
        // the four maxima to pinned host words in one small kernel
        STCHK(ensure_host_flag(ctx));
        const uint32_t seq = ++ctx->flag_seq;
        k_publish4<<<1, 64, 0, ctx->stream>>>(maxlen, ctx->d_hflag + 8, seq);
        HIPCHK(ctx, hipGetLastError());
        if (!overlap) {
            // work of the next force call that needs neither the lists nor
            // their sizes, queued before the host waits for the sizes: the
            // fixed-point words of the new records (an error there is left
            // to the force launch to report) and the integrator's move to
            // the new sorted order
            overlap = true;
            if (local && ctx->prec == MDLJ_PREC_F32PAIR_F64ACC) {
                double fxs;
                (void)fx_words(ctx, &fxs);
            }
            STCHK(enter_sorted_early(ctx, cfg));
        }
        STCHK(wait_host_words(ctx, 12, seq));
        const int32_t hmax[4] = {ctx->h_flag[8], ctx->h_flag[9], ctx->h_flag[10], ctx->h_flag[11]};
        if (tiled && (hmax[2] > cmax || hmax[3] > ccand)) {
            // a tile over the sizes built nothing: exact sizes, or (if those
            // do not fit the LDS budget) the per-particle build
            if (hinted) {
                hinted = false;
                STCHK(exact_sizes());
                tile_ok = build_tile_lds(local, cfg.newton3 != 0, cmax, ccand) <=
                          (size_t)STAGE_LDS_BYTES;
            } else {
                tile_ok = false;
            }
            --attempt;
            continue;
        }
        if (tiled) {
            ctx->tile_c_hint = hmax[2];
            ctx->tile_nc_hint = hmax[3];
            memcpy(ctx->tile_hint_key, key, sizeof key);
        }
        ctx->vl_max = hmax[0];
        ctx->max_nbhd = hmax[2];
        if (local && hmax[2] > 65535)
            return set_err(ctx, MDLJ_ERR_ARG, "neighbourhood too large for 16-bit local lists");
        if (hmax[0] <= cap) {
            ctx->nbr_cap = cap;
            if (inner) {
                HIPCHK(ctx, hipMemsetAsync(ctx->b_tilebad.p, 0, 2 * sizeof(int32_t) * ntiles,
                                           ctx->stream));
                ctx->inner = 1;
                ctx->inner_par = 0;
                ctx->inner_ntiles = ntiles;
            }
            return MDLJ_OK;
        }
        cap = ((int64_t)(hmax[0] * 1.1) + 8 + 7) & ~(int64_t)7;
    }
    return set_err(ctx, MDLJ_ERR_OVERFLOW, "Verlet list capacity could not be grown");
}

mdlj_status vl_pairs(mdlj_ctx *ctx, int64_t cap, int32_t *pi, int32_t *pj, int64_t *count)
{
    const int64_t n = ctx->n;
    const mdlj_config &b = ctx->built_cfg;
    std::vector<int32_t> hl(n);
    HIPCHK(ctx, hipMemcpyAsync(hl.data(), ctx->b_nlen.p, sizeof(int32_t) * n,
                               hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    std::vector<int64_t> off(n);
    int64_t total = 0;
    for (int64_t t = 0; t < n; ++t) {
        off[t] = total;
        total += hl[t];
    }
    *count = total;
    if (!pi) return MDLJ_OK;
    if (total > cap) return set_err(ctx, MDLJ_ERR_OVERFLOW, "pair arrays too short");
    const int layout = b.staged ? 2 : (b.order != MDLJ_ORD_I_PER_LANE ? 1 : 0);
    int64_t *d_off = nullptr;
    int32_t *d_out = nullptr;
    hipError_t e = hipMalloc((void **)&d_off, sizeof(int64_t) * n);
    if (e == hipSuccess) e = hipMalloc((void **)&d_out, sizeof(int32_t) * 2 * (total > 0 ? total : 1));
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_off, off.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice,
                           ctx->stream);
    if (e == hipSuccess) {
        k_vl_pairs<<<ceil_div(n, 256), 256, 0, ctx->stream>>>(
            (const PosT *)ctx->b_sorted.p, (const int32_t *)ctx->b_start.p,
            (const int32_t *)ctx->b_ilist.p, (const int32_t *)ctx->b_cell_of.p, ctx->grid, n,
            ctx->n_ext, ctx->b_nbr.p, (const int32_t *)ctx->b_nlen.p,
            layout == 2 ? (const int2 *)ctx->b_nlo.p : nullptr, (int32_t)ctx->nbr_cap, layout,
            d_off, d_out, d_out + total);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(pi, d_out, sizeof(int32_t) * total, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(pj, d_out + total, sizeof(int32_t) * total, hipMemcpyDeviceToHost,
                           ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    (void)hipFree(d_off);
    (void)hipFree(d_out);
    if (e != hipSuccess) return hip_check(ctx, e, "Verlet-list pair view");
    return MDLJ_OK;
}

mdlj_status vl_forces(mdlj_ctx *ctx, const mdlj_config &cfg, bool energy, ForceOut &fo,
                      int64_t *nblocks)
{
    if (ctx->prec == MDLJ_PREC_F64) return vl_forces_t<double>(ctx, cfg, energy, fo, nblocks);
    return vl_forces_t<float>(ctx, cfg, energy, fo, nblocks);
}
