// lanemap.h -- which pair each lane of a vector computes in one step of an
// interaction order (section 4.1.1, "Filling Registers", and the register
// fills of Fig. "vec_patterns").
//
// A vector of `width` lanes holds `ai` distinct i-particles and width / ai
// distinct j-particles.  Two layouts:
//   i-major  lanes run over j fastest: lane l computes (i + l / (width/ai),
//            j + l % (width/ai)).  ai = 1 is the 1/VectorLength fill (one i
//            broadcast, j across the vector); ai = 2 the
//            2/VectorLengthDiv2 fill (lower half i, upper half i + 1, each
//            with j .. j + width/2 - 1).
//   j-major  lanes run over i fastest: lane l computes (i + l % ai,
//            j + l / ai).  ai = width is the VectorLength/1 fill (i across
//            the vector, one j broadcast); ai = width / 2 the
//            VectorLengthDiv2/2 fill (both halves i .. i + width/2 - 1,
//            lower with j, upper with j + 1).
// The 64-lane wavefront uses the same maps with width 64.  The kernels take
// their lane -> (i, j) offsets from these functions; the library exports
// them (mdlj_lane_map) so the maps can be checked against the figures.
#pragma once

struct LanePair {
    int i, j;
};

enum { LANE_I_MAJOR = 0, LANE_J_MAJOR = 1 };

__host__ __device__ constexpr LanePair lane_pair(int layout, int ai, int width, int lane)
{
    return layout == LANE_I_MAJOR ? LanePair{lane / (width / ai), lane % (width / ai)}
                                  : LanePair{lane % ai, lane / ai};
}
