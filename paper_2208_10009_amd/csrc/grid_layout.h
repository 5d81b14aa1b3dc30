// grid_layout.h -- where the equiangular launch grid's setup (launch.hip)
// keeps its results, which ring a ray of the grid lies on, and what progress
// of the setup the ray's direction needs; host and device.
#pragma once
#include <math.h>
#include <stdint.h>

#include "geom.h"

namespace sbr {

// Icosahedron: the 12 cyclic permutations of (0, +-1, +-phi), normalized, in a
// fixed order; edges are the 30 pairs i < j of adjacent vertices (positive
// dot product), listed lexicographically; faces are the 20 mutually adjacent
// triples i < j < k, lexicographically, wound counter-clockwise seen from
// outside (clockwise seen from the launch point, the paper's ordering).
struct GridHdr {
    d3 V[12];
    int32_t e[30][2];
    int32_t f[20][3];
    int32_t nv, ne, nf;
};

static_assert(sizeof(GridHdr) % 8 == 0, "the header is stored as 64-bit words");

__host__ __device__ static inline int64_t ring_cap(int32_t n) { return n / 3 + 2; }
__host__ __device__ static inline double* side_angles(char* scratch, int32_t n)
{
    return (double*)(scratch + sizeof(GridHdr) + sizeof(d3) * 3 * 20 * (size_t)ring_cap(n));
}
// Angle each icosahedron edge subtends, [30], after the ring side angles.
__host__ __device__ static inline int64_t edge_angle_index(int32_t n)
{
    return 3 * 20 * ring_cap(n);
}

// Ring a (0: the first inside the face boundary) holding the in-face index q
// of a face with division n: ring a starts at S(a) = 3a(n-3) - 9a(a-1)/2
// (the rings before it have sides n-3, n-6, ... > 0); the last ring, of side
// 0, is the face centre.  Estimated from the quadratic, then settled.
__host__ __device__ static inline int64_t ring_of(int32_t n, int64_t q)
{
    const int64_t c1 = 3 * (int64_t)(n - 3);
    const double hb = (double)c1 + 4.5;
    const double disc = hb * hb - 18.0 * (double)q;
    int64_t a = (int64_t)((hb - sqrt(disc > 0.0 ? disc : 0.0)) / 9.0);
    if (a < 0) a = 0;
    while (a > 0 && a * c1 - 9 * a * (a - 1) / 2 > q) --a;
    while (n - 3 - 3 * (a + 1) >= 0 && (a + 1) * c1 - 9 * (a + 1) * a / 2 <= q) ++a;
    return a;
}

// The setup's progress a ray needs before its direction can be formed.  The
// setup publishes 1 once the header and the edge angles are stored, then
// 2 + a after its layer loop's iteration a has stored the corners of inside
// ring a (and the side angles of ring a - 1).  A vertex or edge ray needs 1;
// a ray of inside ring a needs its corners and, unless the ring is the face
// centre, its side angle: 3 + a, or 2 + a for the centre.
__host__ __device__ static inline uint32_t grid_need(int32_t n, int64_t i)
{
    if (i < 12 + 30 * (int64_t)(n - 1)) return 1u;
    const int64_t per_face = (int64_t)(n - 1) * (n - 2) / 2;
    const int64_t q = (i - 12 - 30 * (int64_t)(n - 1)) % per_face;
    const int64_t a = ring_of(n, q);
    return (uint32_t)(n - 3 - 3 * a == 0 ? 2 + a : 3 + a);
}

}  // namespace sbr
