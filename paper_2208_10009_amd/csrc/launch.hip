// launch.hip -- equiangular icosahedral launch directions (Sec. II.B) for
// gfx950: ring corners of the 20 faces layer by layer, then one thread per
// ray.  Every value is bit-identical to the correctly rounded FP64 grid (see
// geom.h for the double-double trigonometry).  The equidistant icosahedral
// and octahedral grids of Sec. II.A, which the paper compares against, are
// launch methods too.
#include <math.h>

#include "geom.h"
#include "internal.h"

namespace sbr {

// ===========================================================================
// Launch grid (Sec. II.B)
// ===========================================================================
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

__host__ __device__ static inline int64_t ring_cap(int32_t n) { return n / 3 + 2; }

// Scratch layout: the header; ring corners [20][cap][3] (d3); the angle each
// ring side subtends, [20][cap][3] (double); the angle of each icosahedron
// edge, [30] (double).
size_t grid_scratch_bytes(int32_t n)
{
    return sizeof(GridHdr) + (sizeof(d3) + sizeof(double)) * 3 * 20 * (size_t)ring_cap(n) +
           sizeof(double) * 30;
}

__host__ __device__ static inline double* side_angles(char* scratch, int32_t n)
{
    return (double*)(scratch + sizeof(GridHdr) + sizeof(d3) * 3 * 20 * (size_t)ring_cap(n));
}

__device__ static void ico_build(GridHdr* H)
{
    const double phi = (1.0 + sqrt(5.0)) / 2.0;
    const double raw[12][3] = {{0, 1, phi},  {0, -1, phi},  {0, 1, -phi},  {0, -1, -phi},
                               {1, phi, 0},  {-1, phi, 0},  {1, -phi, 0},  {-1, -phi, 0},
                               {phi, 0, 1},  {phi, 0, -1},  {-phi, 0, 1},  {-phi, 0, -1}};
    for (int i = 0; i < 12; ++i) H->V[i] = normalize(ld3(raw[i]));
    H->nv = 12;
    H->ne = 30;
    H->nf = 20;
    int ne = 0, nf = 0;
    for (int i = 0; i < 12; ++i)
        for (int j = i + 1; j < 12; ++j)
            if (dot(H->V[i], H->V[j]) > 0.0) {
                H->e[ne][0] = i;
                H->e[ne][1] = j;
                ++ne;
            }
    for (int i = 0; i < 12; ++i)
        for (int j = i + 1; j < 12; ++j)
            for (int k = j + 1; k < 12; ++k) {
                bool a = dot(H->V[i], H->V[j]) > 0.0, b = dot(H->V[j], H->V[k]) > 0.0,
                     c = dot(H->V[i], H->V[k]) > 0.0;
                if (a && b && c) {
                    double s = dot(H->V[i], cross(H->V[j], H->V[k]));
                    H->f[nf][0] = i;
                    H->f[nf][1] = s > 0.0 ? j : k;
                    H->f[nf][2] = s > 0.0 ? k : j;
                    ++nf;
                }
            }
}

// Central projection onto the plane x.g = 1 parallel to the face.
__device__ static d3 proj_face(d3 p, d3 g)
{
    double w = dot(p, g);
    return mk(p.x / w, p.y / w, p.z / w);
}

// Ring corners of every face, layer by layer.  Layer 0 is the face boundary
// (corners = face vertices, n equal-angle steps per side).  The corners of
// the next layer follow eq. (2): each corner moves by the sum of the vectors
// to its two neighbours on the ring, evaluated on the flat face (the
// construction of Fig. 3b), and the new side has three steps fewer.  Side 0
// is the single face-centre ray; negative sides end the face (the three
// innermost cases).  The layers depend on each other, so one block walks
// them in order.
//
// Each layer needs, per ring side (20 faces x 3), the side's angle
// th = acos(P.Q) and the sines of a = th/m and b = (m-1) th/m, all correctly
// rounded (the first step from one corner and the last step into the next
// corner use the same two sines, swapped).  To keep the chain short, three
// lanes per side start from the library's y0 = acos(P.Q) at once:
//   lane 0: cos y0 in double-double and sin y0 from the library; one Newton
//           step th = y0 + (cos y0 - P.Q) / sin y0 is accurate to ~1e-31
//           (the correction is ~1e-16, so a 1e-16 relative sine suffices);
//   lanes 1, 2: sin b0, sin a0 in double-double for b0, a0 formed from y0,
//           and cos b0, cos a0 from the library.
// Then sin a = sin a0 + cos a0 (a - a0) - sin a0 (a - a0)^2 / 2 with
// a - a0 ~ 1e-16 (exact in binary64), likewise for b; the neglected terms are
// below 1e-31 relative, so each value rounds as the exact one does (the
// results are checked bit for bit against the correctly rounded grid).
// The role is the wave index (lane = side, 60 of 64 lanes busy), so no wave
// runs the cosine and the sine series one after the other.
// The side angles are kept for k_grid_dirs.
__global__ __launch_bounds__(192) void k_grid_setup(int32_t n, char* scratch)
{
    GridHdr* H = (GridHdr*)scratch;
    d3* rings = (d3*)(scratch + sizeof(GridHdr));
    double* ths = side_angles(scratch, n);
    __shared__ GridHdr sh;
    __shared__ d3 W[20][3];
    __shared__ d3 P[20][3][2];
    __shared__ dd SV[60][3];    // lane 0: cos y0; lane 1: sin b0; lane 2: sin a0
    __shared__ double CV[60][3];  // lane 0: sin y0; lane 1: cos b0; lane 2: cos a0
    __shared__ double SN[60][2];  // sin a, sin b
    const int t = threadIdx.x;
    if (t == 0) {
        ico_build(&sh);
        *H = sh;
    }
    __syncthreads();
    if (t < 30) ths[3 * 20 * ring_cap(n) + t] = acos_cr(dot(sh.V[sh.e[t][0]], sh.V[sh.e[t][1]]));
    const int f60 = t / 3, s60 = t % 3;
    if (t < 60) W[f60][s60] = sh.V[sh.f[f60][s60]];
    __syncthreads();
    d3 g = mk(0.0, 0.0, 0.0);
    if (t < 60) {
        d3 A = sh.V[sh.f[f60][0]], B = sh.V[sh.f[f60][1]], C = sh.V[sh.f[f60][2]];
        g = add(add(A, B), C);
    }
    const int side = t & 63, role = t >> 6;
    const bool act = side < 60;
    const int fs = side / 3, ss = side % 3;
    const size_t cap3 = 3 * (size_t)ring_cap(n);
    int64_t m = n;
    for (int a = 0;; ++a) {
        // m >= 1 is the side of ring a (ring 0 is the face boundary); its
        // corners are W.
        d3 Pa = mk(0.0, 0.0, 0.0), Pb = Pa;
        double x = 0.0, y0 = 0.0, a0 = 0.0, b0 = 0.0;
        if (act) {
            Pa = W[fs][ss];
            Pb = W[fs][(ss + 1) % 3];
            x = dot(Pa, Pb);
            y0 = acos(x);
            a0 = ((double)1 * y0) / (double)m;
            b0 = ((double)(m - 1) * y0) / (double)m;
            const double arg = role == 0 ? y0 : role == 1 ? b0 : a0;
            const dd aa = dd{arg, 0.0};
            const dd tt = dd_mul(aa, aa);
            SV[side][role] = role == 0 ? dd_poly_alt(0, tt) : dd_mul(aa, dd_poly_alt(1, tt));
            CV[side][role] = role == 0 ? sin(arg) : cos(arg);
        }
        __syncthreads();
        double th = 0.0;
        if (act) {
            const dd r = dd_sub(SV[side][0], dd{x, 0.0});
            const dd y = dd_add(dd{y0, 0.0}, dd{r.hi / CV[side][0], 0.0});
            th = y.hi + y.lo;
            if (role == 0 && a > 0) ths[(size_t)fs * cap3 + 3 * (a - 1) + ss] = th;
        }
        const int64_t mp = m - 3;
        if (mp < 0) break;
        if (mp == 0) {
            if (t < 20) {
                d3 A = sh.V[sh.f[t][0]], B = sh.V[sh.f[t][1]], C = sh.V[sh.f[t][2]];
                d3 c = normalize(add(add(A, B), C));
                d3* out = rings + (size_t)t * cap3 + 3 * a;
                out[0] = c;
                out[1] = c;
                out[2] = c;
            }
            break;
        }
        if (act && role > 0) {
            // role 1: sin b with b = (m-1) th / m; role 2: sin a with a = th / m
            const double v = role == 1 ? ((double)(m - 1) * th) / (double)m
                                       : ((double)1 * th) / (double)m;
            const double dv = v - (role == 1 ? b0 : a0);
            const dd s0 = SV[side][role];
            dd r = dd_add(s0, two_prod(CV[side][role], dv));
            r = dd_add(r, dd{-(s0.hi * dv * dv * 0.5), 0.0});
            SN[side][role == 2 ? 0 : 1] = r.hi + r.lo;
        }
        __syncthreads();
        if (act && role < 2) {
            const double sa = SN[side][0], sb = SN[side][1];
            // role 0: step 1 from corner ss toward ss+1; role 1: step m-1 of
            // the same side, the last step into corner ss+1
            if (role == 0)
                P[fs][ss][0] = normalize(add(scl(sb, Pa), scl(sa, Pb)));
            else
                P[fs][(ss + 1) % 3][1] = normalize(add(scl(sa, Pa), scl(sb, Pb)));
        }
        __syncthreads();
        d3 Wn = mk(0.0, 0.0, 0.0);
        if (t < 60) {
            d3 X = sub(add(proj_face(P[f60][s60][0], g), proj_face(P[f60][s60][1], g)),
                       proj_face(W[f60][s60], g));
            Wn = normalize(X);
            rings[(size_t)f60 * cap3 + 3 * a + s60] = Wn;
        }
        __syncthreads();
        if (t < 60) W[f60][s60] = Wn;
        __syncthreads();
        m = mp;
    }
}

// Point k of m equal-angle steps from P to Q along their great circle, th
// being the angle P and Q subtend (acos_cr(P.Q)): the angles subtended at
// the centre by consecutive points are equal (eq. (1)).  Direction
// sin((m-k) th/m) P + sin(k th/m) Q, normalized.
__device__ static d3 arc_point_th(d3 P, d3 Q, double th, int64_t k, int64_t m)
{
    double a = ((double)k * th) / (double)m;
    double b = ((double)(m - k) * th) / (double)m;
    double sa = sin_cr(a), sb = sin_cr(b);
    return normalize(add(scl(sb, P), scl(sa, Q)));
}

// Ray order: the 12 vertex rays; then edge interiors, edge by edge, steps
// 1..n-1 from the lower to the higher vertex index; then face interiors, face
// by face, layer by layer, each ring starting at the corner that descends
// from the face's first vertex and following the winding.
__global__ void k_grid_dirs(int32_t n, int64_t N, const char* __restrict__ scratch,
                            double* __restrict__ dir)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const GridHdr* H = (const GridHdr*)scratch;
    const d3* rings = (const d3*)(scratch + sizeof(GridHdr));
    const double* ths = side_angles((char*)scratch, n);
    d3 r;
    int64_t idx = i;
    if (idx < 12) {
        r = H->V[idx];
    } else {
        idx -= 12;
        if (idx < 30 * (int64_t)(n - 1)) {
            int64_t e = idx / (n - 1), k = idx % (n - 1) + 1;
            r = arc_point_th(H->V[H->e[e][0]], H->V[H->e[e][1]], ths[3 * 20 * ring_cap(n) + e], k,
                             n);
        } else {
            idx -= 30 * (int64_t)(n - 1);
            int64_t per_face = (int64_t)(n - 1) * (n - 2) / 2;
            int64_t f = idx / per_face, q = idx % per_face;
            int a = 0;
            int64_t m = n - 3;
            for (;;) {
                int64_t sz = m > 0 ? 3 * m : 1;
                if (q < sz) break;
                q -= sz;
                ++a;
                m -= 3;
            }
            const d3* W = rings + (size_t)f * 3 * ring_cap(n) + 3 * a;
            if (m == 0) {
                r = W[0];
            } else {
                int64_t s = q / m, k = q % m;
                r = k == 0 ? W[s]
                           : arc_point_th(W[s], W[(s + 1) % 3],
                                          ths[(size_t)f * 3 * ring_cap(n) + 3 * a + s], k, m);
            }
        }
    }
    dir[i] = r.x;
    dir[N + i] = r.y;
    dir[2 * N + i] = r.z;
}

// ===========================================================================
// Equidistant division (Sec. II.A), the comparison grids: points at equal
// spacing on the flat faces of a regular polyhedron, projected onto the
// sphere.
// ===========================================================================
// Octahedron: vertices +x, -x, +y, -y, +z, -z in this order; edges are the
// 12 non-antipodal pairs i < j, lexicographically; faces are the 8 mutually
// adjacent triples i < j < k, lexicographically, wound counter-clockwise
// seen from outside (the same rules as the icosahedron's).
__device__ static void octa_build(GridHdr* H)
{
    const double raw[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
    for (int i = 0; i < 6; ++i) H->V[i] = ld3(raw[i]);
    H->nv = 6;
    int ne = 0, nf = 0;
    for (int i = 0; i < 6; ++i)
        for (int j = i + 1; j < 6; ++j)
            if (dot(H->V[i], H->V[j]) > -0.5) {
                H->e[ne][0] = i;
                H->e[ne][1] = j;
                ++ne;
            }
    for (int i = 0; i < 6; ++i)
        for (int j = i + 1; j < 6; ++j)
            for (int k = j + 1; k < 6; ++k) {
                bool a = dot(H->V[i], H->V[j]) > -0.5, b = dot(H->V[j], H->V[k]) > -0.5,
                     c = dot(H->V[i], H->V[k]) > -0.5;
                if (a && b && c) {
                    double sg = dot(H->V[i], cross(H->V[j], H->V[k]));
                    H->f[nf][0] = i;
                    H->f[nf][1] = sg > 0.0 ? j : k;
                    H->f[nf][2] = sg > 0.0 ? k : j;
                    ++nf;
                }
            }
    H->ne = ne;
    H->nf = nf;
}

__global__ void k_poly_setup(int32_t launch, char* scratch)
{
    if (threadIdx.x != 0) return;
    GridHdr* H = (GridHdr*)scratch;
    GridHdr h;
    if (launch == SBR_LAUNCH_EQUIDISTANT_OCTA)
        octa_build(&h);
    else
        ico_build(&h);
    *H = h;
}

// Ray order: the vertex rays; edge interiors edge by edge, k = 1..n-1 from
// the lower vertex, at (n-k) V_i + k V_j; face interiors face by face, rows
// i = 1..n-2 and j = 1..n-1-i, at (n-i-j) A + i B + j C for the face's
// corners A, B, C in winding order; each normalized.
__global__ void k_grid_equidistant(int32_t n, int64_t N, const char* __restrict__ scratch,
                                   double* __restrict__ dir)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N) return;
    const GridHdr* H = (const GridHdr*)scratch;
    const int64_t i0 = idx;
    d3 r;
    if (idx < H->nv) {
        r = H->V[idx];
    } else {
        idx -= H->nv;
        if (idx < (int64_t)H->ne * (n - 1)) {
            int64_t e = idx / (n - 1), k = idx % (n - 1) + 1;
            r = normalize(add(scl((double)(n - k), H->V[H->e[e][0]]),
                              scl((double)k, H->V[H->e[e][1]])));
        } else {
            idx -= (int64_t)H->ne * (n - 1);
            const int64_t per_face = (int64_t)(n - 1) * (n - 2) / 2;
            const int64_t f = idx / per_face, q = idx % per_face;
            // row i holds n-1-i points; rows before i hold (i-1)(2n-2-i)/2.
            // Estimate i from the quadratic, then settle it exactly.
            const double nn = (double)(2 * n - 3);
            int64_t i = (int64_t)((nn - sqrt(nn * nn - 8.0 * (double)q)) * 0.5) + 1;
            if (i < 1) i = 1;
            if (i > n - 2) i = n - 2;
            while (i > 1 && (i - 1) * (2 * (int64_t)n - 2 - i) / 2 > q) --i;
            while (i < n - 2 && i * (2 * (int64_t)n - 3 - i) / 2 <= q) ++i;
            const int64_t j = q - (i - 1) * (2 * (int64_t)n - 2 - i) / 2 + 1;
            const int64_t a = n - i - j;
            const d3 A = H->V[H->f[f][0]], B = H->V[H->f[f][1]], C = H->V[H->f[f][2]];
            r = normalize(add(add(scl((double)a, A), scl((double)i, B)), scl((double)j, C)));
        }
    }
    dir[i0] = r.x;
    dir[N + i0] = r.y;
    dir[2 * N + i0] = r.z;
}

hipError_t launch_grid(GridDev g, hipStream_t s, void* scratch)
{
    if (g.launch != SBR_LAUNCH_EQUIANGULAR) {
        hipLaunchKernelGGL(k_poly_setup, dim3(1), dim3(64), 0, s, g.launch, (char*)scratch);
        int64_t blocks = (g.N + 255) / 256;
        hipLaunchKernelGGL(k_grid_equidistant, dim3((unsigned)blocks), dim3(256), 0, s, g.n, g.N,
                           (const char*)scratch, g.dir);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_grid_setup, dim3(1), dim3(192), 0, s, g.n, (char*)scratch);
    int64_t blocks = (g.N + 255) / 256;
    hipLaunchKernelGGL(k_grid_dirs, dim3((unsigned)blocks), dim3(256), 0, s, g.n, g.N,
                       (const char*)scratch, g.dir);
    return hipGetLastError();
}

}  // namespace sbr
