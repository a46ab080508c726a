// pair.h -- the Lennard-Jones 12-6 pair interaction used by every force
// kernel, in the pair arithmetic type T (float or double), accumulating
// into FP64 per-lane sums.
//
// The pair force is F_ij = 24 eps s6 (2 s6 - 1) / r^2 * d, s6 = (sig^2/r^2)^3,
// d = x_i - x_j, for r^2 < rc^2 (cutoff, section 2.1); pair energy
// 4 eps s6 (s6 - 1) - shift and pair virial r.F = 24 eps s6 (2 s6 - 1).
// The separation d and r^2 are formed in FP64.  The all-FP64 kernels and
// the FP32-pair kernels that read the FP64 records form them from FP64
// positions; the FP32-pair staged Verlet-list kernel forms them from
// fixed-point words (coordinates rounded to a grid of at most 1e-7 sigma,
// see fx_words in vl.hip), exactly for the rounded coordinates, so its
// separations carry that rounding and nothing more.  The pair law itself
// (reciprocal, powers, force factor, energy) runs in T.
#pragma once

#include "atomics.h"
#include "internal.h"
#include "lanemap.h"

template <typename T>
__device__ __forceinline__ T rcp_t(T x);
template <>
__device__ __forceinline__ float rcp_t<float>(float x)
{
    return __builtin_amdgcn_rcpf(x);
}
template <>
__device__ __forceinline__ double rcp_t<double>(double x)
{
    return 1.0 / x;
}

struct Acc {
    double fx, fy, fz, u, w;
};

__device__ __forceinline__ void acc_zero(Acc &a) { a.fx = a.fy = a.fz = a.u = a.w = 0.0; }

template <typename T>
struct PairP {
    T sig2, eps24, eps4, shift;
};

// Species table staged in LDS for multi-species kernels.
template <typename T>
struct LdsTable {
    T sig2[MDLJ_MAX_SPECIES * MDLJ_MAX_SPECIES];
    T eps24[MDLJ_MAX_SPECIES * MDLJ_MAX_SPECIES];
    T eps4[MDLJ_MAX_SPECIES * MDLJ_MAX_SPECIES];
    T shift[MDLJ_MAX_SPECIES * MDLJ_MAX_SPECIES];
};

template <typename T>
__device__ __forceinline__ void lds_table_load(LdsTable<T> &s, const LJTable<T> &t, int tid,
                                               int nthreads)
{
    for (int k = tid; k < t.ns * t.ns; k += nthreads) {
        s.sig2[k] = t.sig2[k];
        s.eps24[k] = t.eps24[k];
        s.eps4[k] = t.eps4[k];
        s.shift[k] = t.shift[k];
    }
}

// Parameters of the (ti, tj) pair: from kernel arguments for one species,
// from the LDS table otherwise.
template <typename T, bool MS>
__device__ __forceinline__ PairP<T> pair_params(const LJTable<T> &t, const LdsTable<T> &s, int ti,
                                                int tj)
{
    PairP<T> p;
    if (MS) {
        int k = ti * t.ns + tj;
        p.sig2 = s.sig2[k];
        p.eps24 = s.eps24[k];
        p.eps4 = s.eps4[k];
        p.shift = s.shift[k];
    } else {
        p.sig2 = t.sig2[0];
        p.eps24 = t.eps24[0];
        p.eps4 = t.eps4[0];
        p.shift = t.shift[0];
    }
    return p;
}

// One pair.  The separation d and r^2 are formed in FP64 (exact inputs, so
// |d| carries no more than binary64 rounding); the cutoff decision is taken
// on the FP64 r^2.  The pair law (reciprocal, s6, force factor, energy) runs
// in T.  The force factor is widened once and the force accumulated as
// F += fs * d with FP64 fused multiply-adds, which on this hardware issue
// at the FP32 rate.  Returns the force on i in (fxp, fyp, fzp) (zero, up to
// its sign, when masked or outside the cutoff) and whether the pair is
// inside the cutoff.
template <typename T, bool E>
__device__ __forceinline__ bool lj_pair(double pxi, double pyi, double pzi, double pxj,
                                        double pyj, double pzj, bool valid, const PairP<T> &p,
                                        double rc2, Acc &a, double &fxp, double &fyp, double &fzp)
{
    const double dx = pxi - pxj;
    const double dy = pyi - pyj;
    const double dz = pzi - pzj;
    const double r2d = dx * dx + dy * dy + dz * dz;
    const bool in = valid && (r2d < rc2);
    const T r2 = (T)r2d;
    // outside the cutoff 1/r^2 is taken as 0, which makes s6, the force
    // factor and the force exactly zero (one select instead of one per
    // result, and no inf or NaN for masked self pairs)
    const T ir2 = in ? rcp_t<T>(r2) : T(0);
    const T sr2 = p.sig2 * ir2;
    const T s6 = sr2 * sr2 * sr2;
    // 24 eps s6 (2 s6 - 1) as s6 (48 eps s6 - 24 eps): one fused multiply-add
    // and one product (48 eps = eps24 + eps24 is exact, and loop-invariant
    // for one species)
    const T rf = s6 * (((p.eps24 + p.eps24) * s6) - p.eps24);
    const double fs = (double)(rf * ir2);
    fxp = fs * dx;
    fyp = fs * dy;
    fzp = fs * dz;
    a.fx += fxp;
    a.fy += fyp;
    a.fz += fzp;
    if (E) {
        const T u = p.eps4 * s6 * (s6 - T(1)) - p.shift;
        a.u += in ? (double)u : 0.0;
        a.w += in ? (double)rf : 0.0;
    }
    return in;
}

// Sum of v over the `width` consecutive lanes of a segment (width a power
// of two <= 64), result in every lane of the segment.
__device__ __forceinline__ double seg_sum(double v, int width)
{
    for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, MDLJ_WAVE);
    return v;
}

// Workgroups are handed to the 8 XCDs round-robin; remap the block index so
// each XCD works on one contiguous run of tiles (neighbouring tiles share
// j-data, which then stays in one XCD's L2).
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb)
{
    const int64_t per = nb >> 3, rem = nb & 7;
    const int64_t x = b & 7, k = b >> 3;
    return x * per + (x < rem ? x : rem) + k;
}

// Energy/virial of the workgroup (one wavefront) into partial[2 * blk].
__device__ __forceinline__ void wave_partial(double u, double w, double scale, double *partial,
                                             int64_t blk)
{
    u = seg_sum(u, MDLJ_WAVE);
    w = seg_sum(w, MDLJ_WAVE);
    if ((threadIdx.x & (MDLJ_WAVE - 1)) == 0) {
        partial[2 * blk] = scale * u;
        partial[2 * blk + 1] = scale * w;
    }
}

// Raw buffer access to the sorted records: 32-bit byte offsets from one
// descriptor (and hardware range checks, reads past the end return zero).
// The descriptor's third dword is the gfx9-family default for raw buffers.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t records_rsrc(const PosT *rec, int64_t count)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)rec, (short)0, (int)(count * sizeof(PosT)),
                                             0x00020000);
}

// x, y, z of record j (one 16-byte and one 8-byte buffer load).
__device__ __forceinline__ void load_xyz(__amdgpu_buffer_rsrc_t r, int32_t j, double &x, double &y,
                                         double &z)
{
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(r, j * (int)sizeof(PosT), 0, 0);
    const u32x2 b = __builtin_amdgcn_raw_buffer_load_b64(r, j * (int)sizeof(PosT) + 16, 0, 0);
    x = __builtin_bit_cast(double, (unsigned long long)a.x | ((unsigned long long)a.y << 32));
    y = __builtin_bit_cast(double, (unsigned long long)a.z | ((unsigned long long)a.w << 32));
    z = __builtin_bit_cast(double, (unsigned long long)b.x | ((unsigned long long)b.y << 32));
}

// Position of the padding record that list rows are filled up with: far
// outside any box, so a pair with it never falls inside the cutoff.
constexpr double PAD_COORD = 1.0e7;

// LDS staging of a cell's 27-cell neighbourhood: the nine contiguous runs of
// sorted records (rows of three cells) are copied into LDS as separate x, y,
// z (FP64) and species arrays, candidate k at index k.  At most this many
// bytes of LDS per workgroup are used for it.
constexpr int STAGE_LDS_BYTES = 64 * 1024;

// One record per lane and trip (the form the per-wavefront staging of the
// linked-cell kernels runs fastest with).
__device__ __forceinline__ void stage_rows_simple(const PosT *__restrict__ rec, const int *seg_b,
                                                  const int *seg_c, int C, double *sx, double *sy,
                                                  double *sz, int *st, bool types, int lane,
                                                  int nthr)
{
    int r = 0;
    for (int k = lane; k < C; k += nthr) {
        while (k >= seg_c[r + 1]) ++r;
        const PosT p = rec[seg_b[r] + (k - seg_c[r])];
        sx[k] = p.x;
        sy[k] = p.y;
        sz[k] = p.z;
        if (types) st[k] = p.t;
    }
}

// Record k goes to sx[SD * k], sy[SD * k], sz[SD * k]: SD = 1 for separate
// arrays, SD = 3 with sy = sx + 1 and sz = sx + 2 for interleaved x, y, z.
template <int SD = 1>
__device__ __forceinline__ void stage_rows(const PosT *__restrict__ rec, const int *seg_b,
                                           const int *seg_c, int C, double *sx, double *sy,
                                           double *sz, int *st, bool types, int lane, int nthr)
{
    // four records per thread in flight: the row of staged index k is found
    // without branches (the number of row starts <= k), so the loads of all
    // four issue back to back before the stores
    constexpr int U = 4;
    int c[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) c[q] = seg_c[q + 1];
    for (int k0 = lane; k0 < C; k0 += U * nthr) {
        double x[U], y[U], z[U];
        int t[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            // past the end, load record C - 1 again (not stored): no branch
            const int k = min(k0 + u * nthr, C - 1);
            int r = 0;
#pragma unroll
            for (int q = 0; q < 8; ++q) r += k >= c[q];
            const PosT *p = rec + seg_b[r] + (k - seg_c[r]);
            x[u] = p->x;
            y[u] = p->y;
            z[u] = p->z;
            t[u] = types ? p->t : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u * nthr;
            if (k < C) {
                sx[SD * k] = x[u];
                sy[SD * k] = y[u];
                sz[SD * k] = z[u];
                if (types) st[k] = t[u];
            }
        }
    }
}
