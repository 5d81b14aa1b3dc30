// launch.hip -- equiangular icosahedral launch directions (Sec. II.B) for
// gfx950: ring corners of the 20 faces layer by layer, then one thread per
// ray.  Every value is bit-identical to the correctly rounded FP64 grid (see
// geom.h for the double-double trigonometry).  The equidistant icosahedral
// and octahedral grids of Sec. II.A, which the paper compares against, are
// launch methods too.
#include <math.h>

#include "geom.h"
#include "grid.h"
#include "internal.h"

namespace sbr {

// ===========================================================================
// Launch grid (Sec. II.B)
// ===========================================================================
// Scratch layout: the header; ring corners [20][cap][3] (d3); the angle each
// ring side subtends, [20][cap][3] (double); the angle of each icosahedron
// edge, [30] (double).
size_t grid_scratch_bytes(int32_t n)
{
    return sizeof(GridHdr) + (sizeof(d3) + sizeof(double)) * 3 * 20 * (size_t)ring_cap(n) +
           sizeof(double) * 30;
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
//   lane 0: cos y0 in double-double and sin y0 in double; one Newton step
//           th = y0 + (cos y0 - P.Q) / sin y0 (the correction is ~1e-16, so
//           a 1e-16 relative sine suffices);
//   lanes 1, 2: sin b0, sin a0 in double-double for b0, a0 formed from y0,
//           and cos b0, cos a0 in double.
// Then sin a = sin a0 + cos a0 (a - a0) - sin a0 (a - a0)^2 / 2 with
// a - a0 ~ 1e-16 (exact in binary64), likewise for b.
//
// Two passes per layer.  The first evaluates the series with only their
// leading terms in double-double (series_fast) and carries a rigorous
// bound on the error of every value; a value is accepted when rounding both
// ends of its error interval gives the same double (rounding is monotone, so
// the exact value rounds to it too).  When any value of the layer fails that
// test (about one layer in a hundred), the layer is recomputed with the full
// 18-term double-double series, whose error (~1e-31 relative) leaves each
// value rounding as the exact one does; the results are checked bit for bit
// against the correctly rounded grid either way.  2^check_log2 scales every
// bound (a larger value only sends more layers through the second pass).
//
// The role is the wave index (lane = side, 60 of 64 lanes busy), so no wave
// runs the cosine and the sine series one after the other.  The lanes that
// form the two step points next to a corner also project them onto the face
// plane, and the third wave projects the corners, so the new corners need one
// more step only.  The side angles are kept for k_grid_dirs.

// Stores of the setup's results: plain, or, when the setup publishes its
// progress to kernels running beside it, device-scope relaxed atomic stores.
// Those are written through to the device's coherence point (the consumers'
// device-scope atomic loads read them there), so publishing them needs only
// their completion: wave 0, which makes all of them, waits for its stores
// before it stores the progress word (no L2 write-back, which a release
// fence would add and which the trace's own stores would make slow).
__device__ static inline void grid_st(double* p, double v, bool atomic)
{
    if (atomic)
        __hip_atomic_store((unsigned long long*)p, (unsigned long long)__double_as_longlong(v),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        *p = v;
}

__device__ static inline void grid_st3(d3* p, d3 v, bool atomic)
{
    double* q = (double*)p;
    grid_st(q, v.x, atomic);
    grid_st(q + 1, v.y, atomic);
    grid_st(q + 2, v.z, atomic);
}

// With prog: *prog = epoch << 32 | k publishes the setup's progress k (see
// grid_need): 0 on entry, 1 once the header and the edge angles are stored,
// 2 + a after iteration a of the layer loop.
__global__ __launch_bounds__(192) void k_grid_setup(int32_t n, char* scratch, int32_t check_log2,
                                                    unsigned long long* prog, uint32_t epoch)
{
    GridHdr* H = (GridHdr*)scratch;
    d3* rings = (d3*)(scratch + sizeof(GridHdr));
    double* ths = side_angles(scratch, n);
    const bool pub = prog != nullptr;
    const unsigned long long tag = (unsigned long long)epoch << 32;
    auto publish = [&](uint32_t k) {
        // wave 0 made every store being published
        if (pub && threadIdx.x < 64) {
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            __builtin_amdgcn_s_waitcnt(0);  // every counter, stores included
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            if (threadIdx.x == 0)
                __hip_atomic_store(prog, tag | k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    };
    if (pub) {
        // the setup shares its CU's SIMDs with trace waves, and its serial
        // chain would otherwise get a fifth of their issue slots: its waves
        // issue first whenever they have an instruction ready
        __builtin_amdgcn_s_setprio(3);
        if (threadIdx.x == 0)
            __hip_atomic_store(prog, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __shared__ GridHdr sh;
    __shared__ d3 W[20][3];
    __shared__ d3 PP[20][3][2];   // the two step points next to each corner, projected
    __shared__ d3 PW[20][3];      // the corners, projected
    __shared__ dd SV[60][3];      // lane 0: cos y0; lane 1: sin b0; lane 2: sin a0
    __shared__ double CV[60][3];  // lane 0: 1 / sin y0; lane 1: cos b0; lane 2: cos a0
    __shared__ double SN[60][2];  // sin a, sin b
    __shared__ int wave_bad[3];   // a value of the wave failed its rounding test
    const int t = threadIdx.x;
    if (t == 0) ico_build(&sh);
    __syncthreads();
    if (t < 64) {
        // the header as 64-bit words (GridHdr is a multiple of 8 bytes)
        const unsigned long long* src = (const unsigned long long*)&sh;
        unsigned long long* dst = (unsigned long long*)H;
        for (int w = t; w < (int)(sizeof(GridHdr) / 8); w += 64) {
            if (pub)
                __hip_atomic_store(dst + w, src[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else
                dst[w] = src[w];
        }
    }
    if (t < 30)
        grid_st(ths + edge_angle_index(n) + t, acos_cr(dot(sh.V[sh.e[t][0]], sh.V[sh.e[t][1]])),
                pub);
    publish(1);
    if (t < 60) W[t / 3][t % 3] = sh.V[sh.f[t / 3][t % 3]];
    __syncthreads();
    const int side = t & 63, role = t >> 6;
    const bool act = side < 60;
    const int fs = act ? side / 3 : 0, ss = side % 3;
    d3 g = mk(0.0, 0.0, 0.0);  // face normal direction (sum of the face's vertices)
    if (act) {
        d3 A = sh.V[sh.f[fs][0]], B = sh.V[sh.f[fs][1]], C = sh.V[sh.f[fs][2]];
        g = add(add(A, B), C);
    }
    const double scale = ldexp(1.0, check_log2);
    const LaneSeries L = lane_series(role == 0);
    const size_t cap3 = 3 * (size_t)ring_cap(n);
    int64_t m = n;
    for (int a = 0;; ++a) {
        // m >= 1 is the side of ring a (ring 0 is the face boundary); its
        // corners are W.
        const int64_t mp = m - 3;
        const double rm = 1.0 / (double)m;
        d3 Pa = mk(0.0, 0.0, 0.0), Pb = Pa;
        double x = 0.0, y0 = 0.0, a0 = 0.0, b0 = 0.0, th = 0.0;
        if (act) {
            Pa = W[fs][ss];
            Pb = W[fs][(ss + 1) % 3];
            x = dot(Pa, Pb);
            y0 = acos(x);
            a0 = y0 * rm;  // any value within a few ulp of a serves
            b0 = ((double)(m - 1) * y0) * rm;
        }
        const double arg = role == 0 ? y0 : role == 1 ? b0 : a0;
        for (int full = 0; full < 2; ++full) {
            double err = 0.0;
            if (act) {
                if (full) {
                    const dd aa = dd{arg, 0.0};
                    const dd tt = dd_mul(aa, aa);
                    SV[side][role] = role == 0 ? dd_poly_alt(0, tt) : dd_mul(aa, dd_poly_alt(1, tt));
                } else {
                    double other;  // sin y0 (role 0), cos b0, cos a0
                    SV[side][role] = series_fast(L, arg, &err, &other);
                    CV[side][role] = role == 0 ? 1.0 / other : other;
                }
            }
            __syncthreads();
            bool bad = false;
            if (act) {
                // Newton step: th - y0 = (cos y0 - x) / sin y0 up to a term
                // (th - y0)^2 cot(y0) / 2.
                const dd r = dd_sub(SV[side][0], dd{x, 0.0});
                const double rs = CV[side][0];
                const double q = r.hi * rs;
                const dd y = two_sum(y0, q);
                th = y.hi + y.lo;
                if (!full && role == 0) {
                    const double e_th = err * rs + 2.0 * q * q * rs + 0x1p-38 * fabs(q) +
                                        0x1p-100 * y0;
                    bad = !(y0 <= 1.2) || !(fabs(q) <= 0x1p-30 * y0) ||
                          !rounds_safely(y, e_th * scale);
                }
                if (mp > 0 && role > 0) {
                    // role 1: sin b with b = (m-1) th / m; role 2: sin a with a = th / m
                    const double v = role == 1 ? ((double)(m - 1) * th) / (double)m
                                               : ((double)1 * th) / (double)m;
                    const double dv = v - arg;
                    const dd s0 = SV[side][role];
                    dd rr = dd_add(s0, two_prod(CV[side][role], dv));
                    rr = dd_add(rr, dd{-(s0.hi * dv * dv * 0.5), 0.0});
                    SN[side][role == 2 ? 0 : 1] = rr.hi + rr.lo;
                    if (!full) {
                        const double e_s = err + 0x1p-40 * fabs(dv) + 0x1p-98 * fabs(rr.hi);
                        bad = bad || !(arg <= 1.2) || !rounds_safely(rr, e_s * scale);
                    }
                }
            }
            const bool wb = __any(bad);
            if (side == 0) wave_bad[role] = wb;
            __syncthreads();
            if (!(wave_bad[0] | wave_bad[1] | wave_bad[2])) break;
        }
        if (act && role == 0 && a > 0) grid_st(ths + (size_t)fs * cap3 + 3 * (a - 1) + ss, th, pub);
        if (mp < 0) {
            publish(2 + a);
            break;
        }
        if (mp == 0) {
            if (t < 20) {
                d3 A = sh.V[sh.f[t][0]], B = sh.V[sh.f[t][1]], C = sh.V[sh.f[t][2]];
                d3 c = normalize(add(add(A, B), C));
                d3* out = rings + (size_t)t * cap3 + 3 * a;
                grid_st3(out, c, pub);
                grid_st3(out + 1, c, pub);
                grid_st3(out + 2, c, pub);
            }
            publish(2 + a);
            break;
        }
        if (act) {
            const double sa = SN[side][0], sb = SN[side][1];
            // role 0: step 1 from corner ss toward ss+1; role 1: step m-1 of
            // the same side, the last step into corner ss+1; role 2: corner ss
            if (role == 0)
                PP[fs][ss][0] = proj_face(normalize(add(scl(sb, Pa), scl(sa, Pb))), g);
            else if (role == 1)
                PP[fs][(ss + 1) % 3][1] = proj_face(normalize(add(scl(sa, Pa), scl(sb, Pb))), g);
            else
                PW[fs][ss] = proj_face(Pa, g);
        }
        __syncthreads();
        if (t < 60) {
            const d3 Wn = normalize(sub(add(PP[fs][ss][0], PP[fs][ss][1]), PW[fs][ss]));
            grid_st3(rings + (size_t)fs * cap3 + 3 * a + ss, Wn, pub);
            W[fs][ss] = Wn;
        }
        publish(2 + a);
        __syncthreads();
        m = mp;
    }
}

__global__ void k_grid_dirs(int32_t n, int64_t N, const char* __restrict__ scratch,
                            double* __restrict__ dir, int32_t check_log2)
{
    const double scale = ldexp(1.0, check_log2);
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const d3 r = grid_dir_of<GridPlainLoads>(n, scratch, (uint32_t)i, scale);
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

// ===========================================================================
// Hand-out order of a grid's rays
// ===========================================================================
// The cell of each ray on a cube map over the sphere: the face of the largest
// coordinate (2 axis + sign), then the Z-order index of the other two
// coordinates over that one, quantized to R x R (R a power of two).  Sorted
// by cell, rays next to each other in the order are close in direction.
__global__ void k_ray_cells(const double* __restrict__ dir, int64_t N, int32_t R,
                            uint32_t* __restrict__ cell)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double v[3] = {dir[i], dir[N + i], dir[2 * N + i]};
    int ax = 0;
    if (fabs(v[1]) > fabs(v[ax])) ax = 1;
    if (fabs(v[2]) > fabs(v[ax])) ax = 2;
    const double m = fabs(v[ax]);
    const double u = v[(ax + 1) % 3] / m, w = v[(ax + 2) % 3] / m;
    const int iu = min(R - 1, max(0, (int)((u + 1.0) * 0.5 * (double)R)));
    const int iw = min(R - 1, max(0, (int)((w + 1.0) * 0.5 * (double)R)));
    uint32_t z = 0;
    for (int b = 0; (1 << b) < R; ++b)
        z |= (uint32_t)((iu >> b) & 1) << (2 * b) | (uint32_t)((iw >> b) & 1) << (2 * b + 1);
    const uint32_t face = (uint32_t)(2 * ax + (v[ax] < 0.0 ? 1 : 0));
    cell[i] = face * (uint32_t)R * (uint32_t)R + z;
}

hipError_t launch_ray_cells(const double* dir, int64_t N, int32_t R, uint32_t* cell,
                            hipStream_t s)
{
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ray_cells, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, dir, N, R,
                       cell);
    return hipGetLastError();
}

hipError_t launch_grid(GridDev g, hipStream_t s, void* scratch, int32_t check_log2)
{
    if (g.launch != SBR_LAUNCH_EQUIANGULAR) {
        hipLaunchKernelGGL(k_poly_setup, dim3(1), dim3(64), 0, s, g.launch, (char*)scratch);
        int64_t blocks = (g.N + 255) / 256;
        hipLaunchKernelGGL(k_grid_equidistant, dim3((unsigned)blocks), dim3(256), 0, s, g.n, g.N,
                           (const char*)scratch, g.dir);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_grid_setup, dim3(1), dim3(192), 0, s, g.n, (char*)scratch, check_log2,
                       (unsigned long long*)nullptr, 0u);
    int64_t blocks = (g.N + 255) / 256;
    hipLaunchKernelGGL(k_grid_dirs, dim3((unsigned)blocks), dim3(256), 0, s, g.n, g.N,
                       (const char*)scratch, g.dir, check_log2);
    return hipGetLastError();
}

// The ring setup alone, publishing its progress at prog for a trace that
// forms its rays' directions itself (equiangular grids only).
hipError_t launch_grid_setup_streamed(int32_t n, void* scratch, int32_t check_log2,
                                      unsigned long long* prog, uint32_t epoch, hipStream_t s)
{
    hipLaunchKernelGGL(k_grid_setup, dim3(1), dim3(192), 0, s, n, (char*)scratch, check_log2,
                       prog, epoch);
    return hipGetLastError();
}

// Wait (one lane, bounded) until the setup of this epoch has started, so that
// the trace launched after it cannot take the slot the setup needs.
__global__ void k_grid_wait_started(const unsigned long long* prog, uint32_t epoch,
                                    int32_t* err, uint32_t max_spin)
{
    if (threadIdx.x != 0) return;
    for (uint32_t spin = 0;; ++spin) {
        const unsigned long long v =
            __hip_atomic_load(prog, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((uint32_t)(v >> 32) == epoch) return;
        if (spin > max_spin) {
            atomicOr(err, 8);
            return;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

hipError_t launch_grid_wait_started(const unsigned long long* prog, uint32_t epoch, int32_t* err,
                                    uint32_t max_spin, hipStream_t s)
{
    hipLaunchKernelGGL(k_grid_wait_started, dim3(1), dim3(64), 0, s, prog, epoch, err, max_spin);
    return hipGetLastError();
}

}  // namespace sbr
