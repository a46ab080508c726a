// vcl.hip -- Verlet cluster lists (section 2.1.1, after Pall & Hess): the
// particles are grouped into clusters of a fixed size M (4 or 8, cf. the
// cluster-size study of section 5), and every cluster keeps a list of the
// clusters whose bounding boxes lie within rc + skin, rebuilt every few
// steps.  Neighbour lists are thereby multiples of M long (section 5).
//
// Clusters: the box is cut into xy columns of edge ~(M/rho)^(1/3) and thin
// z slabs; binning sorts each column by slab, and each column is chunked
// into clusters of M consecutive particles.  The last cluster of a column
// is padded with dummy records placed far outside the box (distinct
// positions, so dummy pairs fall outside the cutoff).
//
// Periodic images are handled per cluster pair: a list entry packs J (low
// 26 bits) and an image code (high bits), the code naming the lattice shift (sx, sy, sz) in {-1,0,1}^3 that
// is added to J's coordinates.  With Newton-3 an entry is kept only for
// I < J, or I == J with a shift that is zero or lexicographically positive,
// so each particle pair is computed once (section 4.1.3).
//
// Kernels:
//   k_vcl_tile  cluster tile: 64 lanes = M i's of cluster I x (64/M) j's,
//               i.e. one J (M = 8, 8x8) or four consecutive list entries
//               (M = 4, 4x16) per step; i-forces summed over the j lanes at
//               the end, j-forces (Newton-3) over the i lanes every step.
//   k_vcl_ipl   i-per-lane: a lane owns one i; the M lanes of a cluster walk
//               its list and read the M j's of each J in turn, so the j is
//               the same for all lanes of the cluster (a broadcast load).
#include <vector>

#include "pair.h"

namespace {

constexpr int CODE_SHIFT = 26;
constexpr int32_t J_MASK = (1 << CODE_SHIFT) - 1;
constexpr double DUMMY_BASE = 1.0e7;
constexpr double DUMMY_STEP = 64.0;
// list steps per trip of the force loops
constexpr int UNROLL = 4;

__host__ __device__ inline int shift_code(int sx, int sy, int sz)
{
    return (sx + 1) + 3 * (sy + 1) + 9 * (sz + 1);
}

struct ClusterGeom {
    int M;
    int ncx, ncy, nz;   // columns in x and y, slabs in z
    double L[3];
    double slab;        // slab height
    int64_t nclu;
    int hx, hy;         // columns to search on each side
    double R2;          // (rc + skin)^2
};

// Per column: number of clusters.
__global__ void k_col_counts(Grid g, const int32_t *__restrict__ start, int M,
                             int32_t *__restrict__ ccount)
{
    int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= (int64_t)g.n[0] * g.n[1]) return;
    int cx = (int)((uint32_t)col % (uint32_t)g.n[0]), cy = (int)((uint32_t)col / (uint32_t)g.n[0]);
    int64_t e0 = (int64_t)cx * g.stride[0] + (int64_t)cy * g.stride[1];
    int32_t cnt = start[e0 + g.n[2]] - start[e0];
    ccount[col] = (cnt + M - 1) / M;
}

// Per column (one wavefront): copy records into clusters, pad, bounding
// boxes, slab range, column of each cluster and the particle -> slot map.
__global__ __launch_bounds__(64) void k_make_clusters(
    Grid g, const int32_t *__restrict__ start, const int32_t *__restrict__ cbase, int M,
    const PosT *__restrict__ rec, PosT *__restrict__ crec, int32_t *__restrict__ slot_of,
    double *__restrict__ bb, int32_t *__restrict__ slabr, int32_t *__restrict__ ccol)
{
    const int64_t col = blockIdx.x;
    const int lane = threadIdx.x;
    const int cx = (int)((uint32_t)col % (uint32_t)g.n[0]), cy = (int)((uint32_t)col / (uint32_t)g.n[0]);
    const int64_t e0 = (int64_t)cx * g.stride[0] + (int64_t)cy * g.stride[1];
    const int32_t b = start[e0], en = start[e0 + g.n[2]];
    const int32_t q0 = cbase[col], q1 = cbase[col + 1];
    for (int32_t q = q0; q < q1; ++q) {
        for (int m = lane; m < M; m += MDLJ_WAVE) {
            const int32_t src = b + (q - q0) * M + m;
            const int64_t dst = (int64_t)q * M + m;
            if (src < en) {
                const PosT r = rec[src];
                crec[dst] = r;
                slot_of[r.orig] = (int32_t)dst;
            } else {
                PosT d;
                d.x = d.y = d.z = DUMMY_BASE + DUMMY_STEP * (double)dst;
                d.t = 0;
                d.orig = -1;
                crec[dst] = d;
            }
        }
    }
    // bounding boxes and slab ranges: one lane per cluster
    for (int32_t q = q0 + lane; q < q1; q += MDLJ_WAVE) {
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        const int32_t s0 = b + (q - q0) * M;
        const int32_t s1 = min(s0 + M, en);
        for (int32_t k = s0; k < s1; ++k) {
            const PosT r = rec[k];
            lo[0] = fmin(lo[0], r.x); hi[0] = fmax(hi[0], r.x);
            lo[1] = fmin(lo[1], r.y); hi[1] = fmax(hi[1], r.y);
            lo[2] = fmin(lo[2], r.z); hi[2] = fmax(hi[2], r.z);
        }
        for (int a = 0; a < 3; ++a) {
            bb[6 * (int64_t)q + a] = lo[a];
            bb[6 * (int64_t)q + 3 + a] = hi[a];
        }
        // slab of the first and last member (records are sorted by slab)
        int slab_first = (int)(rec[s0].z * g.inv[2]);
        int slab_last = (int)(rec[s1 - 1].z * g.inv[2]);
        slab_first = max(0, min(g.n[2] - 1, slab_first));
        slab_last = max(0, min(g.n[2] - 1, slab_last));
        slabr[2 * (int64_t)q] = slab_first;
        slabr[2 * (int64_t)q + 1] = slab_last;
        ccol[q] = (int32_t)col;
    }
}

__device__ __forceinline__ double gap(double alo, double ahi, double blo, double bhi)
{
    const double d1 = blo - ahi, d2 = alo - bhi;
    const double d = d1 > d2 ? d1 : d2;
    return d > 0.0 ? d : 0.0;
}

// One thread per cluster I: all (J, shift) with bounding-box distance
// < rc + skin, into row I of the list (row-major, capacity cap).
__global__ void k_pair_search(ClusterGeom cg, const double *__restrict__ bb,
                              const int32_t *__restrict__ slabr,
                              const int32_t *__restrict__ ccol,
                              const int32_t *__restrict__ cbase, int half, int32_t cap,
                              int32_t *__restrict__ list, int32_t *__restrict__ len,
                              int32_t *__restrict__ maxlen)
{
    const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= cg.nclu) return;
    double ilo[3], ihi[3];
    for (int a = 0; a < 3; ++a) {
        ilo[a] = bb[6 * I + a];
        ihi[a] = bb[6 * I + 3 + a];
    }
    const int col = ccol[I];
    const int cx = col % cg.ncx, cy = col / cg.ncx;
    const double R = sqrt(cg.R2);
    int32_t cnt = 0;
    for (int dy = -cg.hy; dy <= cg.hy; ++dy) {
        int ny = cy + dy;
        int sy = 0;
        while (ny < 0) { ny += cg.ncy; --sy; }
        while (ny >= cg.ncy) { ny -= cg.ncy; ++sy; }
        if (sy < -1 || sy > 1) continue;
        for (int dx = -cg.hx; dx <= cg.hx; ++dx) {
            int nx = cx + dx;
            int sx = 0;
            while (nx < 0) { nx += cg.ncx; --sx; }
            while (nx >= cg.ncx) { nx -= cg.ncx; ++sx; }
            if (sx < -1 || sx > 1) continue;
            const int ncol = nx + cg.ncx * ny;
            const int32_t q0 = cbase[ncol], q1 = cbase[ncol + 1];
            if (q0 == q1) continue;
            for (int sz = -1; sz <= 1; ++sz) {
                const double shz = sz * cg.L[2];
                const double wlo = ilo[2] - R - shz, whi = ihi[2] + R - shz;
                if (whi < 0.0 || wlo > cg.L[2]) continue;
                // first cluster whose last slab reaches the window (monotone key)
                int32_t lo = q0, hi = q1;
                while (lo < hi) {
                    const int32_t mid = (lo + hi) >> 1;
                    if ((slabr[2 * (int64_t)mid + 1] + 1) * cg.slab < wlo) lo = mid + 1;
                    else hi = mid;
                }
                for (int32_t q = lo; q < q1; ++q) {
                    if (slabr[2 * (int64_t)q] * cg.slab > whi) break;
                    const double shx = sx * cg.L[0], shy = sy * cg.L[1];
                    const double gx = gap(ilo[0], ihi[0], bb[6 * (int64_t)q] + shx, bb[6 * (int64_t)q + 3] + shx);
                    const double gy = gap(ilo[1], ihi[1], bb[6 * (int64_t)q + 1] + shy, bb[6 * (int64_t)q + 4] + shy);
                    const double gz = gap(ilo[2], ihi[2], bb[6 * (int64_t)q + 2] + shz, bb[6 * (int64_t)q + 5] + shz);
                    if (gx * gx + gy * gy + gz * gz >= cg.R2) continue;
                    if (half) {
                        if (q < I) continue;
                        if (q == I) {
                            // keep the zero shift and one of each +-shift pair
                            const int code = shift_code(sx, sy, sz);
                            if (code < 13) continue;
                        }
                    }
                    if (cnt < cap)
                        list[I * cap + cnt] = (int32_t)q | (shift_code(sx, sy, sz) << CODE_SHIFT);
                    ++cnt;
                }
            }
        }
    }
    len[I] = cnt;
    atomic_max_rare(maxlen, cnt);
}

// The same search with one wavefront per cluster I.  Phase 1: lane w takes
// search window w (column offset dy, dx and z shift sz, in the loop order of
// k_pair_search) and finds its range of candidate clusters by binary search
// on the slab keys; a scan over the wavefront gives each window its offset
// in one flattened candidate sequence (per wavefront in LDS: range start,
// offset and shift code of each of the nwin windows).  Phase 2: lane l
// tests candidates k0 + l of that sequence, and passing entries are
// compacted in order with a ballot, so the list is the one k_pair_search
// writes, entry for entry.
constexpr int PS_TB = 256;

__global__ __launch_bounds__(PS_TB) void k_pair_search_w(
    ClusterGeom cg, const double *__restrict__ bb, const int32_t *__restrict__ slabr,
    const int32_t *__restrict__ ccol, const int32_t *__restrict__ cbase, int half, int32_t cap,
    int32_t *__restrict__ list, int32_t *__restrict__ len, int32_t *__restrict__ maxlen, int nwin)
{
    extern __shared__ int32_t psh[];
    const int lane = threadIdx.x & (MDLJ_WAVE - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / MDLJ_WAVE);
    const int64_t I = (int64_t)blockIdx.x * (PS_TB / MDLJ_WAVE) + wv;
    if (I >= cg.nclu) return;  // whole wavefronts; no workgroup barrier below
    int32_t *wlo = psh + (size_t)wv * 3 * nwin;
    int32_t *woff = wlo + nwin;
    int32_t *wcode = woff + nwin;
    double ilo[3], ihi[3];
    for (int a = 0; a < 3; ++a) {
        ilo[a] = bb[6 * I + a];
        ihi[a] = bb[6 * I + 3 + a];
    }
    const int col = ccol[I];
    const int cx = col % cg.ncx, cy = col / cg.ncx;
    const double R = sqrt(cg.R2);
    const int nxw = 2 * cg.hx + 1;
    int32_t total = 0;
    for (int w0 = 0; w0 < nwin; w0 += MDLJ_WAVE) {
        const int w = w0 + lane;
        int32_t lo = 0, cnt = 0, code = 0;
        if (w < nwin) {
            const int sz = w % 3 - 1;
            const int dx = (w / 3) % nxw - cg.hx;
            const int dy = w / (3 * nxw) - cg.hy;
            int ny = cy + dy, sy = 0;
            while (ny < 0) { ny += cg.ncy; --sy; }
            while (ny >= cg.ncy) { ny -= cg.ncy; ++sy; }
            int nx = cx + dx, sx = 0;
            while (nx < 0) { nx += cg.ncx; --sx; }
            while (nx >= cg.ncx) { nx -= cg.ncx; ++sx; }
            const double shz = sz * cg.L[2];
            const double wl = ilo[2] - R - shz, wh = ihi[2] + R - shz;
            if (sy >= -1 && sy <= 1 && sx >= -1 && sx <= 1 && !(wh < 0.0 || wl > cg.L[2])) {
                const int ncol = nx + cg.ncx * ny;
                const int32_t q0 = cbase[ncol], q1 = cbase[ncol + 1];
                // first cluster whose last slab reaches the window, then the
                // first from there whose first slab lies beyond it (both keys
                // are monotone along a column)
                int32_t a = q0, b = q1;
                while (a < b) {
                    const int32_t mid = (a + b) >> 1;
                    if ((slabr[2 * (int64_t)mid + 1] + 1) * cg.slab < wl) a = mid + 1;
                    else b = mid;
                }
                lo = a;
                b = q1;
                while (a < b) {
                    const int32_t mid = (a + b) >> 1;
                    if (!(slabr[2 * (int64_t)mid] * cg.slab > wh)) a = mid + 1;
                    else b = mid;
                }
                cnt = a - lo;
                code = shift_code(sx, sy, sz);
            }
        }
        // exclusive offsets of the windows' ranges
        int32_t inc = cnt;
        for (int o = 1; o < MDLJ_WAVE; o <<= 1) {
            const int32_t t = __shfl_up(inc, o);
            if (lane >= o) inc += t;
        }
        if (w < nwin) {
            wlo[w] = lo;
            woff[w] = total + inc - cnt;
            wcode[w] = code;
        }
        total += __shfl(inc, MDLJ_WAVE - 1);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    int32_t cnt = 0;
    for (int32_t k0 = 0; k0 < total; k0 += MDLJ_WAVE) {
        const int32_t k = k0 + lane;
        bool keep = false;
        int32_t e = 0;
        if (k < total) {
            // the last window whose offset is <= k (empty windows share the
            // offset of the next one, so this is the window holding k)
            int a = 0, b = nwin - 1;
            while (a < b) {
                const int mid = (a + b + 1) >> 1;
                if (woff[mid] <= k) a = mid;
                else b = mid - 1;
            }
            const int32_t q = wlo[a] + (k - woff[a]);
            const int code = wcode[a];
            const int sx = code % 3 - 1, sy = (code / 3) % 3 - 1, sz = code / 9 - 1;
            const double shx = sx * cg.L[0], shy = sy * cg.L[1], shz = sz * cg.L[2];
            const double gx = gap(ilo[0], ihi[0], bb[6 * (int64_t)q] + shx, bb[6 * (int64_t)q + 3] + shx);
            const double gy = gap(ilo[1], ihi[1], bb[6 * (int64_t)q + 1] + shy, bb[6 * (int64_t)q + 4] + shy);
            const double gz = gap(ilo[2], ihi[2], bb[6 * (int64_t)q + 2] + shz, bb[6 * (int64_t)q + 5] + shz);
            keep = gx * gx + gy * gy + gz * gz < cg.R2;
            // Newton 3: I < J, or I == J with the zero shift or one of each
            // +- pair
            if (half) keep = keep && (q > I || (q == I && code >= 13));
            e = (int32_t)q | (code << CODE_SHIFT);
        }
        const uint64_t m = __builtin_amdgcn_ballot_w64(keep);
        const uint32_t pos = __builtin_amdgcn_mbcnt_hi(
            (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, (uint32_t)cnt));
        if (keep && pos < (uint32_t)cap) list[I * cap + pos] = e;
        cnt += (int32_t)__builtin_popcountll(m);
    }
    if (lane == 0) {
        len[I] = cnt;
        atomic_max_rare(maxlen, cnt);
    }
}

struct BoxL {
    double L[3];
};

// The 27 image shifts of the codes, one table per workgroup in LDS: the
// force kernels read a list entry's shift from it instead of decoding the
// code arithmetically (two integer divisions, three conversions and
// products per entry and lane).  Code 13 is the zero shift.
constexpr int CODE_NO_SHIFT = 13;

__device__ __forceinline__ void shift_table_load(double (*st)[4], const BoxL &bl, int tid)
{
    if (tid < 27) {
        st[tid][0] = (double)(tid % 3 - 1) * bl.L[0];
        st[tid][1] = (double)((tid / 3) % 3 - 1) * bl.L[1];
        st[tid][2] = (double)(tid / 9 - 1) * bl.L[2];
    }
}

// Cluster tile: M x AJ lanes per cluster pair, QI = 64 / (M AJ) cluster
// pairs per wavefront (M x 64/M: one cluster I per wavefront; M x 4: four
// for M = 4, two for M = 8), each in its own group of W = M AJ lanes with
// its own cluster I.  JMAJOR = false: within a group lanes run over j
// fastest (the 2/(VL/2) fill widened: lane l takes i = l / AJ and j-lane
// l % AJ); JMAJOR = true: over i fastest (the (VL/2)/2 fill widened: i =
// l % M, j-lane l / M).  The j-lanes walk I's list as j-slots, entry k and
// member m of its cluster being slot k M + m: step s gives j-lane b slot
// s AJ + b, so a step covers AJ / M entries when AJ >= M and a fraction
// AJ / M of one entry's cluster when AJ < M.
template <typename T, bool E, bool MS, bool N3, int M, bool JMAJOR, int AJ>
__global__ __launch_bounds__(256) void k_vcl_tile(const PosT *__restrict__ crec,
                                                  const int32_t *__restrict__ list,
                                                  const int32_t *__restrict__ len, int64_t nclu,
                                                  int32_t cap, BoxL bl, LJTable<T> tab,
                                                  ForceOut fo, int remap)
{
    constexpr int W = M * AJ;            // lanes per cluster pair
    constexpr int QI = MDLJ_WAVE / W;    // cluster pairs per wavefront
    static_assert(QI * W == MDLJ_WAVE && (AJ % M == 0 || M % AJ == 0), "tile shape");
    __shared__ LdsTable<T> lt;
    __shared__ double shifts[27][4];
    const double rc2 = tab.rc2d;
    if (MS) lds_table_load(lt, tab, threadIdx.x, blockDim.x);
    shift_table_load(shifts, bl, threadIdx.x);
    __syncthreads();
    const int64_t b = remap ? xcd_remap(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    const int lane = threadIdx.x & (MDLJ_WAVE - 1);
    const int64_t I = (b * (blockDim.x / MDLJ_WAVE) + threadIdx.x / MDLJ_WAVE) * QI + lane / W;
    constexpr int LAYOUT = JMAJOR ? LANE_J_MAJOR : LANE_I_MAJOR;
    const LanePair lp = lane_pair(LAYOUT, M, W, lane % W);
    const int a = lp.i;                  // i within the cluster
    const int bj = lp.j;                 // j lane
    Acc acc;
    acc_zero(acc);
    const bool live = I < nclu;
    const int64_t islot = live ? I * M + a : 0;
    const PosT pi = crec[islot];
    const int32_t Ln = live ? len[I] : 0;
    // A step covers JPS whole list entries (AJ >= M: the j-lane's entry of
    // the step is eo, its member m0 on every step) or 1/SPE of one entry
    // (AJ < M: the member also depends on the step).  The loop runs in
    // entries (AJ >= M) or steps (AJ < M), as far as the longest list of the
    // wavefront's groups on every lane: the shuffles need all of them.
    constexpr int JPS = AJ >= M ? AJ / M : 1;
    constexpr int SPE = AJ >= M ? 1 : M / AJ;
    constexpr int TRIP = (AJ >= M ? JPS : 1) * UNROLL;
    const int eo = AJ >= M ? bj / M : 0;
    const int m0 = AJ >= M ? bj % M : bj;
    int32_t Lw = Ln;
    if constexpr (QI > 1) {
#pragma unroll
        for (int o = W; o < MDLJ_WAVE; o <<= 1) Lw = max(Lw, __shfl_xor(Lw, o, MDLJ_WAVE));
    }
    const int32_t Tw = Lw * SPE;
    for (int32_t t00 = 0; t00 < Tw; t00 += TRIP) {
        // U steps per trip: their list and record loads are in flight together
        int32_t J[UNROLL], m[UNROLL], code[UNROLL];
        bool ok[UNROLL];
        PosT pj[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            int32_t k;                   // list entry
            if constexpr (AJ >= M) {
                k = t00 + u * JPS + eo;
                m[u] = m0;
            } else {
                const int32_t st = t00 + u;
                k = st / SPE;
                m[u] = (st % SPE) * AJ + m0;
            }
            ok[u] = k < Ln;
            // one load per step on every lane (a load in a branch is waited
            // for at the branch's end), always inside the list array: a lane
            // past its list reads the last entry of its own row; a lane
            // without a list (no cluster, or an empty list) reads the first
            // word of its row (or of row 0), which it ignores for cluster 0
            // and the zero shift.  The pairs of both are masked below.
            const int32_t e = list[(live ? I : 0) * cap + min(k, max(Ln - 1, 0))];
            J[u] = Ln > 0 ? (e & J_MASK) : 0;
            code[u] = ok[u] ? (int)((uint32_t)e >> CODE_SHIFT) : CODE_NO_SHIFT;
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) pj[u] = crec[(int64_t)J[u] * M + m[u]];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            // all lanes take part in the shuffles below; masked lanes add zero
            if (t00 + u * (TRIP / UNROLL) >= Tw) break;
            // the member as a loop invariant where it is one (reading the
            // array here would keep all its elements live)
            const int mu = AJ >= M ? m0 : m[u];
            const int64_t jslot = (int64_t)J[u] * M + mu;
            // self cluster without shift: skip the diagonal, and with Newton-3
            // the lower triangle
            const bool self0 = ok[u] && J[u] == I && code[u] == CODE_NO_SHIFT;
            const bool valid = ok[u] && !(self0 && (N3 ? mu <= a : mu == a));
            const PairP<T> p = pair_params<T, MS>(tab, lt, pi.t, pj[u].t);
            const double *sh = shifts[code[u]];
            double fxp, fyp, fzp;
            lj_pair<T, E>(pi.x, pi.y, pi.z, pj[u].x + sh[0], pj[u].y + sh[1], pj[u].z + sh[2], valid,
                          p, rc2, acc, fxp, fyp, fzp);
            if (N3) {
                // -F on j summed over the M i-lanes of its group that share
                // it (lanes AJ apart for j fastest, adjacent lanes for i
                // fastest)
                double gx = -fxp, gy = -fyp, gz = -fzp;
                const int o0 = JMAJOR ? 1 : AJ, o1 = JMAJOR ? M : W;
                for (int o = o0; o < o1; o <<= 1) {
                    gx += __shfl_xor(gx, o, MDLJ_WAVE);
                    gy += __shfl_xor(gy, o, MDLJ_WAVE);
                    gz += __shfl_xor(gz, o, MDLJ_WAVE);
                }
                // skip j's that no i-lane reaches inside the cutoff (and dummies)
                if (a == 0 && ok[u] && (gx != 0.0 || gy != 0.0 || gz != 0.0)) {
                    atomicAdd(&fo.fx[jslot], gx);
                    atomicAdd(&fo.fy[jslot], gy);
                    atomicAdd(&fo.fz[jslot], gz);
                }
            }
        }
    }
    // F on i summed over its AJ j-lanes: adjacent lanes for j fastest,
    // lanes M apart for i fastest (within the group)
    for (int o = JMAJOR ? M : 1; o < (JMAJOR ? W : AJ); o <<= 1) {
        acc.fx += __shfl_xor(acc.fx, o, MDLJ_WAVE);
        acc.fy += __shfl_xor(acc.fy, o, MDLJ_WAVE);
        acc.fz += __shfl_xor(acc.fz, o, MDLJ_WAVE);
    }
    if (live && bj == 0) {
        if (N3) {
            atomicAdd(&fo.fx[islot], acc.fx);
            atomicAdd(&fo.fy[islot], acc.fy);
            atomicAdd(&fo.fz[islot], acc.fz);
        } else {
            fo.fx[islot] = acc.fx;
            fo.fy[islot] = acc.fy;
            fo.fz[islot] = acc.fz;
        }
    }
    if (E)
        wave_partial(acc.u, acc.w, N3 ? 1.0 : 0.5, fo.partial,
                     (int64_t)blockIdx.x * (blockDim.x / MDLJ_WAVE) + threadIdx.x / MDLJ_WAVE);
}

// i-per-lane: 64/M clusters per wavefront, M lanes each.
template <typename T, bool E, bool MS, bool N3, int M>
__global__ __launch_bounds__(256) void k_vcl_ipl(const PosT *__restrict__ crec,
                                                 const int32_t *__restrict__ list,
                                                 const int32_t *__restrict__ len, int64_t nclu,
                                                 int32_t cap, BoxL bl, LJTable<T> tab,
                                                 ForceOut fo, int remap)
{
    __shared__ LdsTable<T> lt;
    __shared__ double shifts[27][4];
    const double rc2 = tab.rc2d;
    if (MS) lds_table_load(lt, tab, threadIdx.x, blockDim.x);
    shift_table_load(shifts, bl, threadIdx.x);
    __syncthreads();
    const int64_t b = remap ? xcd_remap(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    const int64_t g = b * blockDim.x + threadIdx.x;  // global lane
    const int64_t I = g / M;
    const int a = (int)(g % M);
    const bool live = I < nclu;
    const int64_t islot = live ? I * M + a : 0;
    const PosT pi = crec[islot];
    const int32_t Ln = live ? len[I] : 0;
    Acc acc;
    acc_zero(acc);
    for (int32_t k = 0; k < Ln; ++k) {
        const int32_t e = list[I * cap + k];
        const int32_t J = e & J_MASK;
        const int code = (int)((uint32_t)e >> CODE_SHIFT);
        const double sx = shifts[code][0], sy = shifts[code][1], sz = shifts[code][2];
        const bool self0 = J == I && code == CODE_NO_SHIFT;
        for (int mm = 0; mm < M; ++mm) {
            const int64_t jslot = (int64_t)J * M + mm;
            const PosT pj = crec[jslot];
            const bool valid = !(self0 && (N3 ? mm <= a : mm == a));
            const PairP<T> p = pair_params<T, MS>(tab, lt, pi.t, pj.t);
            double fxp, fyp, fzp;
            lj_pair<T, E>(pi.x, pi.y, pi.z, pj.x + sx, pj.y + sy, pj.z + sz, valid, p, rc2,
                          acc, fxp, fyp, fzp);
            if (N3) {
                double gx = -fxp, gy = -fyp, gz = -fzp;
                // sum over the M lanes of this cluster (they share j)
                for (int o = 1; o < M; o <<= 1) {
                    gx += __shfl_xor(gx, o, M);
                    gy += __shfl_xor(gy, o, M);
                    gz += __shfl_xor(gz, o, M);
                }
                if (a == 0 && (gx != 0.0 || gy != 0.0 || gz != 0.0)) {
                    atomicAdd(&fo.fx[jslot], gx);
                    atomicAdd(&fo.fy[jslot], gy);
                    atomicAdd(&fo.fz[jslot], gz);
                }
            }
        }
    }
    if (live) {
        if (N3) {
            atomicAdd(&fo.fx[islot], acc.fx);
            atomicAdd(&fo.fy[islot], acc.fy);
            atomicAdd(&fo.fz[islot], acc.fz);
        } else {
            fo.fx[islot] = acc.fx;
            fo.fy[islot] = acc.fy;
            fo.fz[islot] = acc.fz;
        }
    }
    if (E)
        wave_partial(acc.u, acc.w, N3 ? 1.0 : 0.5, fo.partial,
                     (int64_t)blockIdx.x * (blockDim.x / MDLJ_WAVE) + threadIdx.x / MDLJ_WAVE);
}

template <typename T, bool E, bool MS, bool N3, int M>
int64_t launch_vcl_m(mdlj_ctx *ctx, const mdlj_config &cfg, const LJTable<T> &tab, ForceOut &fo,
                     int remap)
{
    const int64_t nclu = ctx->n_ext / M;
    const PosT *crec = (const PosT *)ctx->b_sorted.p;
    const int32_t *list = (const int32_t *)ctx->b_nbr.p;
    const int32_t *len = (const int32_t *)ctx->b_nlen.p;
    const int32_t cap = (int32_t)ctx->nbr_cap;
    BoxL bl = {{ctx->box[0], ctx->box[1], ctx->box[2]}};
    hipStream_t s = ctx->stream;
    const int TB = 256;
    if (cfg.order == MDLJ_ORD_CLUSTER_TILE) {
        // tile_j = j-lanes per cluster pair: 64/M (one pair per wavefront)
        // or 4 (64/(4M) pairs per wavefront)
        if (cfg.tile_i != M || (cfg.tile_j != MDLJ_WAVE / M && cfg.tile_j != 4)) return -1;
        const int qi = MDLJ_WAVE / (M * cfg.tile_j);
        const int64_t nb = ceil_div(nclu, (int64_t)(TB / MDLJ_WAVE) * qi);
#define VCL_TILE(SW, AJ)                                                                         \
    k_vcl_tile<T, E, MS, N3, M, SW, AJ><<<nb, TB, 0, s>>>(crec, list, len, nclu, cap, bl, tab, fo, \
                                                          remap)
        if (cfg.tile_j == 4) {
            if (cfg.swap)
                VCL_TILE(true, 4);
            else
                VCL_TILE(false, 4);
        } else if (cfg.swap) {
            VCL_TILE(true, MDLJ_WAVE / M);
        } else {
            VCL_TILE(false, MDLJ_WAVE / M);
        }
#undef VCL_TILE
        return nb * (TB / MDLJ_WAVE);
    }
    const int64_t nb = ceil_div(nclu * M, TB);
    k_vcl_ipl<T, E, MS, N3, M><<<nb, TB, 0, s>>>(crec, list, len, nclu, cap, bl, tab, fo, remap);
    return nb * (TB / MDLJ_WAVE);
}

template <typename T, bool E, bool MS>
int64_t launch_vcl(mdlj_ctx *ctx, const mdlj_config &cfg, const LJTable<T> &tab, ForceOut &fo,
                   int remap)
{
    const bool n3 = cfg.newton3 != 0;
    if (cfg.cluster_size == 4)
        return n3 ? launch_vcl_m<T, E, MS, true, 4>(ctx, cfg, tab, fo, remap)
                  : launch_vcl_m<T, E, MS, false, 4>(ctx, cfg, tab, fo, remap);
    if (cfg.cluster_size == 8)
        return n3 ? launch_vcl_m<T, E, MS, true, 8>(ctx, cfg, tab, fo, remap)
                  : launch_vcl_m<T, E, MS, false, 8>(ctx, cfg, tab, fo, remap);
    return -1;
}

template <typename T>
mdlj_status vcl_forces_t(mdlj_ctx *ctx, const mdlj_config &cfg, bool energy, ForceOut &fo,
                         int64_t *nblocks)
{
    LJTable<T> tab;
    fill_table<T>(ctx, &tab);
    const bool ms = ctx->nspec > 1;
    const int remap = 1;
    if (cfg.newton3) STCHK(zero_forces(ctx, fo, ctx->n_ext + 1));
    int64_t nw;
    if (energy) {
        const int64_t maxw = ctx->n_ext + 64;
        STCHK(partial_buffer(ctx, 2 * maxw, &fo.partial));
        nw = ms ? launch_vcl<T, true, true>(ctx, cfg, tab, fo, remap)
                : launch_vcl<T, true, false>(ctx, cfg, tab, fo, remap);
    } else {
        nw = ms ? launch_vcl<T, false, true>(ctx, cfg, tab, fo, remap)
                : launch_vcl<T, false, false>(ctx, cfg, tab, fo, remap);
    }
    if (nw < 0) return set_err(ctx, MDLJ_ERR_ARG, "unsupported cluster size");
    HIPCHK(ctx, hipGetLastError());
    *nblocks = nw;
    return MDLJ_OK;
}

// Particle pairs of the stored cluster pairs, for checking the lists: for
// entry q of cluster I's row, the M x M pairs (i in I, j in J) at
// off[I] + (q M + a) M + b as caller indices; a dummy member, or a particle
// with itself under the zero shift, gives (-1, -1), and an entry naming no
// cluster gives j = -2.
__global__ __launch_bounds__(256) void k_vcl_pairs(const PosT *__restrict__ crec, int M,
                                                   int64_t nclu, const int32_t *__restrict__ list,
                                                   const int32_t *__restrict__ len, int32_t cap,
                                                   const int64_t *__restrict__ off,
                                                   int32_t *__restrict__ pi,
                                                   int32_t *__restrict__ pj)
{
    const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nclu) return;
    const int32_t L = len[I];
    for (int32_t q = 0; q < L; ++q) {
        const int32_t e = list[I * cap + q];
        const int64_t J = e & J_MASK;
        const int code = (int)((uint32_t)e >> CODE_SHIFT);
        for (int a = 0; a < M; ++a) {
            const int32_t i = crec[I * M + a].orig;
            for (int b = 0; b < M; ++b) {
                const int64_t k = off[I] + ((int64_t)q * M + a) * M + b;
                if (J >= nclu) {
                    pi[k] = i;
                    pj[k] = -2;
                    continue;
                }
                const int32_t j = crec[J * M + b].orig;
                const bool ok = i >= 0 && j >= 0 && !(i == j && code == 13);
                pi[k] = ok ? i : -1;
                pj[k] = ok ? j : -1;
            }
        }
    }
}

}  // namespace

mdlj_status vcl_build(mdlj_ctx *ctx, const mdlj_config &cfg)
{
    const int M = cfg.cluster_size;
    if (M != 4 && M != 8) return set_err(ctx, MDLJ_ERR_ARG, "cluster size must be 4 or 8");
    const double R = ctx->rc + ctx->skin;
    const double vol = ctx->box[0] * ctx->box[1] * ctx->box[2];
    const double rho = (double)ctx->n / vol;
    // columns of roughly cubic clusters; slabs thin enough that a slab-sorted
    // column is nearly z-sorted
    double edge = cbrt((double)M / rho);
    const double slab = fmin(0.5, 0.25 * edge);
    double rmin[3] = {edge, edge, slab};
    int h[3] = {0, 0, 0};
    Grid g;
    if (!make_grid(ctx->box, rmin, h, true, &g)) return set_err(ctx, MDLJ_ERR_GEOMETRY, "grid");
    for (int a = 0; a < 3; ++a)
        if (ctx->box[a] < 2.0 * R)
            return set_err(ctx, MDLJ_ERR_GEOMETRY, "box edge shorter than twice rc + skin");
    STCHK(bin_particles(ctx, g));
    const int64_t ncol = (int64_t)g.n[0] * g.n[1];
    STCHK(ensure(ctx, ctx->b_icnt, sizeof(int32_t) * (ncol + 1) * 2));
    int32_t *ccount = (int32_t *)ctx->b_icnt.p;
    int32_t *cbase = ccount + ncol + 1;
    hipStream_t s = ctx->stream;
    k_col_counts<<<ceil_div(ncol, 256), 256, 0, s>>>(g, (const int32_t *)ctx->b_start.p, M, ccount);
    HIPCHK(ctx, hipGetLastError());
    STCHK(exclusive_scan(ctx, ccount, cbase, ncol));
    int32_t hnclu = 0;
    HIPCHK(ctx, hipMemcpyAsync(&hnclu, cbase + ncol, sizeof hnclu, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    const int64_t nclu = hnclu;
    const int64_t nslot = nclu * M;
    if (nslot >= ((int64_t)1 << CODE_SHIFT)) return set_err(ctx, MDLJ_ERR_OVERFLOW, "too many clusters");
    // cluster records replace the binned records
    STCHK(ensure(ctx, ctx->b_clu, sizeof(PosT) * (nslot > 0 ? nslot : 1)));
    STCHK(ensure(ctx, ctx->b_cstart, sizeof(double) * 6 * (nclu > 0 ? nclu : 1)));
    STCHK(ensure(ctx, ctx->b_cpair, sizeof(int32_t) * 3 * (nclu > 0 ? nclu : 1)));
    int32_t *slabr = (int32_t *)ctx->b_cpair.p;
    int32_t *ccol = slabr + 2 * nclu;
    k_make_clusters<<<ncol, 64, 0, s>>>(g, (const int32_t *)ctx->b_start.p, cbase, M,
                                        (const PosT *)ctx->b_sorted.p, (PosT *)ctx->b_clu.p,
                                        (int32_t *)ctx->b_slot_of.p, (double *)ctx->b_cstart.p,
                                        slabr, ccol);
    HIPCHK(ctx, hipGetLastError());
    // swap: the force path reads b_sorted as the record array
    std::swap(ctx->b_sorted, ctx->b_clu);
    ctx->fx_valid = false;
    ctx->n_ext = nslot;
    STCHK(ensure(ctx, ctx->b_img, sizeof(char4) * (nslot > 0 ? nslot : 1)));
    HIPCHK(ctx, hipMemsetAsync(ctx->b_img.p, 0, sizeof(char4) * (nslot > 0 ? nslot : 1), s));

    ClusterGeom cg;
    cg.M = M;
    cg.ncx = g.n[0];
    cg.ncy = g.n[1];
    cg.nz = g.n[2];
    for (int a = 0; a < 3; ++a) cg.L[a] = ctx->box[a];
    cg.slab = g.edge[2];
    cg.nclu = nclu;
    cg.hx = (int)ceil(R / g.edge[0]);
    cg.hy = (int)ceil(R / g.edge[1]);
    // never visit a column twice with the same shift
    cg.hx = std::min(cg.hx, (g.n[0] - 1) / 2 + 1);
    cg.hy = std::min(cg.hy, (g.n[1] - 1) / 2 + 1);
    cg.R2 = R * R;
    const double est_pairs = rho * 4.18879020478639 * pow(R + edge, 3) / M;
    int64_t cap = (int64_t)((cfg.newton3 ? 0.6 : 1.2) * est_pairs) + 16;
    if (ctx->vcl_cap > cap && ctx->built_cfg.newton3 == cfg.newton3 &&
        ctx->built_cfg.cluster_size == M)
        cap = ctx->vcl_cap;
    STCHK(ensure(ctx, ctx->b_nlen, sizeof(int32_t) * (nclu > 0 ? nclu : 1)));
    int32_t *maxlen = (int32_t *)ctx->b_flags.p + 12;
    for (int attempt = 0; attempt < 3; ++attempt) {
        STCHK(ensure(ctx, ctx->b_nbr, sizeof(int32_t) * (nclu > 0 ? nclu : 1) * cap));
        HIPCHK(ctx, hipMemsetAsync(maxlen, 0, sizeof(int32_t), s));
        // one wavefront per cluster while its search windows fit the LDS
        const int nwin = (2 * cg.hy + 1) * (2 * cg.hx + 1) * 3;
        const size_t plds = sizeof(int32_t) * 3 * (size_t)nwin * (PS_TB / MDLJ_WAVE);
        if (nclu > 0 && plds <= 32768)
            k_pair_search_w<<<ceil_div(nclu, PS_TB / MDLJ_WAVE), PS_TB, plds, s>>>(
                cg, (const double *)ctx->b_cstart.p, slabr, ccol, cbase, cfg.newton3 ? 1 : 0,
                (int32_t)cap, (int32_t *)ctx->b_nbr.p, (int32_t *)ctx->b_nlen.p, maxlen, nwin);
        else if (nclu > 0)
            k_pair_search<<<ceil_div(nclu, 128), 128, 0, s>>>(
                cg, (const double *)ctx->b_cstart.p, slabr, ccol, cbase, cfg.newton3 ? 1 : 0,
                (int32_t)cap, (int32_t *)ctx->b_nbr.p, (int32_t *)ctx->b_nlen.p, maxlen);
        HIPCHK(ctx, hipGetLastError());
        int32_t hmax = 0;
        HIPCHK(ctx, hipMemcpyAsync(&hmax, maxlen, sizeof hmax, hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipStreamSynchronize(s));
        ctx->vl_max = hmax;
        if (hmax <= cap) {
            ctx->vcl_cap = cap;
            ctx->nbr_cap = cap;
            return MDLJ_OK;
        }
        cap = (int64_t)(hmax * 1.1) + 8;
    }
    return set_err(ctx, MDLJ_ERR_OVERFLOW, "cluster list capacity could not be grown");
}

mdlj_status vcl_pairs(mdlj_ctx *ctx, int64_t cap, int32_t *pi, int32_t *pj, int64_t *count)
{
    const int M = ctx->built_cfg.cluster_size;
    const int64_t nclu = ctx->n_ext / M;
    std::vector<int32_t> hl(nclu > 0 ? nclu : 1);
    if (nclu > 0) {
        HIPCHK(ctx, hipMemcpyAsync(hl.data(), ctx->b_nlen.p, sizeof(int32_t) * nclu,
                                   hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    }
    std::vector<int64_t> off(nclu > 0 ? nclu : 1);
    int64_t raw = 0;
    for (int64_t I = 0; I < nclu; ++I) {
        off[I] = raw;
        raw += (int64_t)hl[I] * M * M;
    }
    std::vector<int32_t> h(2 * (raw > 0 ? raw : 1));
    if (raw > 0) {
        int64_t *d_off = nullptr;
        int32_t *d_out = nullptr;
        hipError_t e = hipMalloc((void **)&d_off, sizeof(int64_t) * nclu);
        if (e == hipSuccess) e = hipMalloc((void **)&d_out, sizeof(int32_t) * 2 * raw);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_off, off.data(), sizeof(int64_t) * nclu, hipMemcpyHostToDevice,
                               ctx->stream);
        if (e == hipSuccess) {
            k_vcl_pairs<<<ceil_div(nclu, 256), 256, 0, ctx->stream>>>(
                (const PosT *)ctx->b_sorted.p, M, nclu, (const int32_t *)ctx->b_nbr.p,
                (const int32_t *)ctx->b_nlen.p, (int32_t)ctx->vcl_cap, d_off, d_out, d_out + raw);
            e = hipGetLastError();
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(h.data(), d_out, sizeof(int32_t) * 2 * raw, hipMemcpyDeviceToHost,
                               ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        (void)hipFree(d_off);
        (void)hipFree(d_out);
        if (e != hipSuccess) return hip_check(ctx, e, "cluster-list pair view");
    }
    // drop the (-1, -1) slots of dummies and of particles with themselves
    int64_t cnt = 0;
    for (int64_t k = 0; k < raw; ++k) {
        if (h[k] == -1 && h[raw + k] == -1) continue;
        if (pi && cnt < cap) {
            pi[cnt] = h[k];
            pj[cnt] = h[raw + k];
        }
        ++cnt;
    }
    *count = cnt;
    if (pi && cnt > cap) return set_err(ctx, MDLJ_ERR_OVERFLOW, "pair arrays too short");
    return MDLJ_OK;
}

mdlj_status vcl_forces(mdlj_ctx *ctx, const mdlj_config &cfg, bool energy, ForceOut &fo,
                       int64_t *nblocks)
{
    if (ctx->prec == MDLJ_PREC_F64) return vcl_forces_t<double>(ctx, cfg, energy, fo, nblocks);
    return vcl_forces_t<float>(ctx, cfg, energy, fo, nblocks);
}
