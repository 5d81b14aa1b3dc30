// kernels.hip -- HIP kernels of the SBR hot path for gfx950 (CDNA4, wave64).
//
// Stages (paper section in brackets):
//   grid    equiangular icosahedral launch directions          [Sec. II.B]
//   trace   BVH traversal, specular bounces, cone reception      [Sec. III.A]
//   sort    canonical order of reception events; path test 1    [Sec. III.A]
//   refine  the iterative precise algorithm (sub-ray cones)     [Sec. III.B]
//   solve   path quantities, image solve, path test 2, power    [Sec. III.A, IV]
//
// Nothing here is a dense contraction, so no MFMA is used.  Traversal reads
// FP32 node boxes (64 B per node) and decides every ray-triangle hit in FP64
// with a fixed operation order; see geom.h for why that makes results
// deterministic.
#include <float.h>
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
};

__host__ __device__ static inline int64_t ring_cap(int32_t n) { return n / 3 + 2; }

size_t grid_scratch_bytes(int32_t n)
{
    return sizeof(GridHdr) + sizeof(d3) * 3 * 20 * (size_t)ring_cap(n);
}

__device__ static void ico_build(GridHdr* H)
{
    const double phi = (1.0 + sqrt(5.0)) / 2.0;
    const double raw[12][3] = {{0, 1, phi},  {0, -1, phi},  {0, 1, -phi},  {0, -1, -phi},
                               {1, phi, 0},  {-1, phi, 0},  {1, -phi, 0},  {-1, -phi, 0},
                               {phi, 0, 1},  {phi, 0, -1},  {-phi, 0, 1},  {-phi, 0, -1}};
    for (int i = 0; i < 12; ++i) H->V[i] = normalize(ld3(raw[i]));
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

// Point k of m equal-angle steps from P to Q along their great circle: the
// angles subtended at the centre by consecutive points are equal (eq. (1)).
// Direction sin((m-k) th/m) P + sin(k th/m) Q, normalized.
__device__ static d3 arc_point(d3 P, d3 Q, int64_t k, int64_t m, const dd* fact)
{
    double th = acos_cr(dot(P, Q), fact);
    double a = ((double)k * th) / (double)m;
    double b = ((double)(m - k) * th) / (double)m;
    double sa = sin_cr(a, fact), sb = sin_cr(b, fact);
    return normalize(add(scl(sb, P), scl(sa, Q)));
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
// them in order: 120 threads compute the 20 x 3 x 2 neighbour points of a
// layer, then 60 threads form the next corners.
__global__ __launch_bounds__(128) void k_grid_setup(int32_t n, char* scratch,
                                                    const dd* __restrict__ fact)
{
    GridHdr* H = (GridHdr*)scratch;
    d3* rings = (d3*)(scratch + sizeof(GridHdr));
    __shared__ GridHdr sh;
    __shared__ d3 W[20][3];
    __shared__ d3 P[20][3][2];
    const int t = threadIdx.x;
    if (t == 0) {
        ico_build(&sh);
        *H = sh;
    }
    __syncthreads();
    const int f60 = t / 3, s60 = t % 3;
    if (t < 60) W[f60][s60] = sh.V[sh.f[f60][s60]];
    __syncthreads();
    d3 g = mk(0.0, 0.0, 0.0);
    if (t < 60) {
        d3 A = sh.V[sh.f[f60][0]], B = sh.V[sh.f[f60][1]], C = sh.V[sh.f[f60][2]];
        g = add(add(A, B), C);
    }
    const size_t cap3 = 3 * (size_t)ring_cap(n);
    int64_t m = n;
    for (int a = 0;; ++a) {
        int64_t mp = m - 3;
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
        if (t < 120) {
            int f = t / 6, s = (t % 6) >> 1, w = t & 1;
            P[f][s][w] = w == 0 ? arc_point(W[f][s], W[f][(s + 1) % 3], 1, m, fact)
                                : arc_point(W[f][(s + 2) % 3], W[f][s], m - 1, m, fact);
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

// Ray order: the 12 vertex rays; then edge interiors, edge by edge, steps
// 1..n-1 from the lower to the higher vertex index; then face interiors, face
// by face, layer by layer, each ring starting at the corner that descends
// from the face's first vertex and following the winding.
__global__ void k_grid_dirs(int32_t n, int64_t N, const char* __restrict__ scratch,
                            const dd* __restrict__ fact, double* __restrict__ dir)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const GridHdr* H = (const GridHdr*)scratch;
    const d3* rings = (const d3*)(scratch + sizeof(GridHdr));
    d3 r;
    int64_t idx = i;
    if (idx < 12) {
        r = H->V[idx];
    } else {
        idx -= 12;
        if (idx < 30 * (int64_t)(n - 1)) {
            int64_t e = idx / (n - 1), k = idx % (n - 1) + 1;
            r = arc_point(H->V[H->e[e][0]], H->V[H->e[e][1]], k, n, fact);
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
                r = k == 0 ? W[s] : arc_point(W[s], W[(s + 1) % 3], k, m, fact);
            }
        }
    }
    dir[i] = r.x;
    dir[N + i] = r.y;
    dir[2 * N + i] = r.z;
}

hipError_t launch_grid(GridDev g, hipStream_t s, void* scratch, const dd* fact)
{
    hipLaunchKernelGGL(k_grid_setup, dim3(1), dim3(128), 0, s, g.n, (char*)scratch, fact);
    int64_t blocks = (g.N + 255) / 256;
    hipLaunchKernelGGL(k_grid_dirs, dim3((unsigned)blocks), dim3(256), 0, s, g.n, g.N,
                       (const char*)scratch, fact, g.dir);
    return hipGetLastError();
}

// ===========================================================================
// BVH traversal with FP64 ray-triangle decisions
// ===========================================================================
// Conservativeness.  The FP32 ray (o32, d32) differs from the FP64 ray by at
// most 2^-24 (|o| + t|d|) per component at parameter t; for any point of the
// scene this is below 3 * 2^-24 R, R = max(|Tx|, scene extent).  Each FP32
// box already contains its triangles (outward rounding) and is widened by
// delta = 2^-20 R > 3 * 2^-24 R plus the rounding of the widening itself, so
// the FP32 ray passes through the widened box wherever the FP64 ray passes
// through the true box.  The slab arithmetic then errs by a few ulp in t,
// covered by the factor 1 + 2^-20 on the exit and pruning bounds.  Culling
// therefore never removes a triangle that the FP64 test below would accept.

// Moller-Trumbore in exactly this order:
//   p = d x e2, det = e1.p (0: miss), s = o - v0, u = (s.p)/det,
//   q = s x e1, v = (d.q)/det, t = (e2.q)/det,
//   hit iff u >= 0, v >= 0, u + v <= 1 and t_lo < t < t_hi.
__device__ static inline bool mt_hit(const TriD& T, d3 o, d3 d, double t_lo, double t_hi,
                                     double* t_out)
{
    d3 e1 = mk(T.e1x, T.e1y, T.e1z), e2 = mk(T.e2x, T.e2y, T.e2z);
    d3 p = cross(d, e2);
    double det = dot(e1, p);
    if (det == 0.0) return false;
    d3 s = sub(o, mk(T.v0x, T.v0y, T.v0z));
    double u = dot(s, p) / det;
    if (!(u >= 0.0)) return false;
    d3 q = cross(s, e1);
    double v = dot(d, q) / det;
    if (!(v >= 0.0) || !(u + v <= 1.0)) return false;
    double t = dot(e2, q) / det;
    if (t > t_lo && t < t_hi) {
        *t_out = t;
        return true;
    }
    return false;
}

__device__ static inline TriD load_tri(const TriD* __restrict__ p)
{
    const double2* q = (const double2*)p;
    double2 a = q[0], b = q[1], c = q[2], d = q[3], e = q[4];
    TriD T;
    T.v0x = a.x; T.v0y = a.y; T.v0z = b.x; T.e1x = b.y; T.e1y = c.x;
    T.e1z = c.y; T.e2x = d.x; T.e2y = d.y; T.e2z = e.x;
    int2 fi = *(const int2*)&e.y;
    T.face = fi.x;
    T.orig = fi.y;
    return T;
}

struct HitRec {
    double t;
    int32_t pos, face, orig;
};

// Closest hit (ANY = false: smallest t; equal t -> lower face id -> lower
// input index) or any hit (ANY = true) of the ray o + t d, t_lo < t < t_hi,
// ignoring triangles of faces xa and xb.  Returns the leaf-order position of
// the hit or -1.
struct Tally {
    uint32_t nodes, tris;
};

template <bool ANY, bool COUNT = false>
__device__ static int32_t traverse(const SceneDev& S, d3 o, d3 d, int32_t xa, int32_t xb,
                                   double t_lo, double t_hi, float delta, HitRec* h,
                                   int32_t* err, Tally* tally = nullptr)
{
    const float slack = 1.0f + 9.5367431640625e-07f;  // 1 + 2^-20
    float ox = (float)o.x, oy = (float)o.y, oz = (float)o.z;
    float dx = (float)d.x, dy = (float)d.y, dz = (float)d.z;
    dx = dx >= 0.0f ? fmaxf(dx, 1e-20f) : fminf(dx, -1e-20f);
    dy = dy >= 0.0f ? fmaxf(dy, 1e-20f) : fminf(dy, -1e-20f);
    dz = dz >= 0.0f ? fmaxf(dz, 1e-20f) : fminf(dz, -1e-20f);
    const float ix = 1.0f / dx, iy = 1.0f / dy, iz = 1.0f / dz;
    // lo - delta - o = lo - (o + delta);  hi + delta - o = hi - (o - delta)
    const float lx = ox + delta, ly = oy + delta, lz = oz + delta;
    const float hx = ox - delta, hy = oy - delta, hz = oz - delta;

    h->pos = -1;
    h->t = INFINITY;
    h->face = 0x7fffffff;
    h->orig = 0x7fffffff;
    float tb = isinf(t_hi) ? INFINITY : (float)t_hi * slack;

    int32_t stack[kTraceStack];
    int sp = 0;
    int32_t node = 0;
    for (;;) {
        const float4* np = (const float4*)(S.nodes + node);
        if (COUNT) tally->nodes += 1;
        float4 a = np[0], b = np[1], c = np[2];
        int4 m = *(const int4*)(np + 3);
        // child 0: lo (a.x a.y a.z) hi (a.w b.x b.y); child 1: lo (b.z b.w c.x) hi (c.y c.z c.w)
        float t0x = (a.x - lx) * ix, t1x = (a.w - hx) * ix;
        float t0y = (a.y - ly) * iy, t1y = (b.x - hy) * iy;
        float t0z = (a.z - lz) * iz, t1z = (b.y - hz) * iz;
        float tn0 = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fminf(t0z, t1z));
        float tf0 = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fmaxf(t0z, t1z)) * slack;
        float u0x = (b.z - lx) * ix, u1x = (c.y - hx) * ix;
        float u0y = (b.w - ly) * iy, u1y = (c.z - hy) * iy;
        float u0z = (c.x - lz) * iz, u1z = (c.w - hz) * iz;
        float tn1 = fmaxf(fmaxf(fminf(u0x, u1x), fminf(u0y, u1y)), fminf(u0z, u1z));
        float tf1 = fminf(fminf(fmaxf(u0x, u1x), fmaxf(u0y, u1y)), fmaxf(u0z, u1z)) * slack;
        bool hit0 = m.z >= 0 && tn0 <= tf0 && tf0 >= 0.0f && tn0 <= tb;
        bool hit1 = m.w >= 0 && tn1 <= tf1 && tf1 >= 0.0f && tn1 <= tb;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            bool hl = side == 0 ? (hit0 && m.z > 0) : (hit1 && m.w > 0);
            if (!hl) continue;
            int32_t first = side == 0 ? m.x : m.y;
            int32_t cnt = side == 0 ? m.z : m.w;
            for (int32_t i = first; i < first + cnt; ++i) {
                TriD T = load_tri(S.tris + i);
                if (COUNT) tally->tris += 1;
                if (T.face == xa || T.face == xb) continue;
                double t;
                if (!mt_hit(T, o, d, t_lo, t_hi, &t)) continue;
                if (ANY) {
                    h->pos = i;
                    h->t = t;
                    h->face = T.face;
                    h->orig = T.orig;
                    return i;
                }
                bool better = h->pos < 0 || t < h->t ||
                              (t == h->t && (T.face < h->face ||
                                             (T.face == h->face && T.orig < h->orig)));
                if (better) {
                    h->pos = i;
                    h->t = t;
                    h->face = T.face;
                    h->orig = T.orig;
                    tb = (float)t * slack;
                    if ((double)tb < t) tb = nextafterf(tb, INFINITY);
                }
            }
        }
        bool go0 = hit0 && m.z == 0 && tn0 <= tb;
        bool go1 = hit1 && m.w == 0 && tn1 <= tb;
        if (go0 && go1) {
            bool first0 = tn0 <= tn1;
            int32_t nearc = first0 ? m.x : m.y, farc = first0 ? m.y : m.x;
            if (sp >= kTraceStack) {
                atomicOr(err, 1);
                return h->pos;
            }
            stack[sp++] = farc;
            node = nearc;
        } else if (go0) {
            node = m.x;
        } else if (go1) {
            node = m.y;
        } else {
            if (sp == 0) break;
            node = stack[--sp];
        }
    }
    return h->pos;
}

__device__ static inline d3 face_normal(const SceneDev& S, int32_t f)
{
    const double* p = S.fplane + 4 * (size_t)f;
    return mk(p[0], p[1], p[2]);
}

// Reception test and error angle (eq. (3)) of one segment (origin o,
// direction d, unfolded length D at o, next hit at t) for one Rx.  The foot
// of the perpendicular is at t* = (Rx - o).d; accepted iff 0 < t* <= t and,
// with thl >= 0, Rx lies inside the ray cone d_perp <= thl (D + t*).  The
// error angle's tangent is d_perp / (D + t*): the distance to Rx over the
// propagation distance of the ray.
__device__ static inline bool capture(d3 o, d3 d, double D, double t, d3 rx, double thl,
                                      double* tan_out)
{
    d3 w = sub(rx, o);
    double ts = dot(w, d);
    if (!(ts > 0.0)) return false;
    if (!(ts <= t)) return false;
    d3 f = sub(w, scl(ts, d));
    double dp = norm(f);
    double L = D + ts;
    if (thl >= 0.0 && !(dp <= thl * L)) return false;
    *tan_out = dp / L;
    return true;
}

// ===========================================================================
// Trace + reception (Sec. III.A), one thread per launch ray
// ===========================================================================
// With COUNT, per-ray totals of traversal work are added to tallies[0..3]:
// segments traced, BVH nodes visited, triangles tested, reception events.
template <bool COUNT>
__global__ __launch_bounds__(256) void k_trace(SceneDev S, GridDev g, TraceArgs A, int64_t first,
                                               int64_t count, sbr_candidate* __restrict__ cand,
                                               int64_t cap,
                                               unsigned long long* __restrict__ ccount,
                                               int32_t* __restrict__ out_tri,
                                               double* __restrict__ out_t,
                                               int32_t* __restrict__ err,
                                               unsigned long long* __restrict__ tallies)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    Tally tl{0u, 0u};
    uint32_t segs = 0, events = 0;
    const int64_t r = first + i;
    const int K = A.K;
    d3 o = mk(A.tx[0], A.tx[1], A.tx[2]);
    d3 d = mk(g.dir[r], g.dir[g.N + r], g.dir[2 * g.N + r]);
    double D = 0.0;
    int32_t prev = -1;
    int32_t faces[SBR_MAX_ORDER];
#pragma unroll
    for (int q = 0; q < SBR_MAX_ORDER; ++q) faces[q] = -1;
    for (int j = 0; j <= K; ++j) {
        HitRec h;
        int32_t hit = traverse<false, COUNT>(S, o, d, prev, prev, S.t_eps, INFINITY, A.delta, &h,
                                             err, &tl);
        if (COUNT) segs += 1;
        double t = hit < 0 ? INFINITY : h.t;
        if (out_tri) out_tri[i * (K + 1) + j] = hit < 0 ? -1 : h.orig;
        if (out_t) out_t[i * (K + 1) + j] = t;
        for (int x = 0; x < A.n_rx; ++x) {
            double tn;
            d3 rx = mk(A.rx[3 * x], A.rx[3 * x + 1], A.rx[3 * x + 2]);
            if (!capture(o, d, D, t, rx, A.thl, &tn)) continue;
            if (COUNT) events += 1;
            unsigned long long pos = atomicAdd(ccount, 1ull);
            if ((int64_t)pos < cap) {
                sbr_candidate c;
                c.rx = x;
                c.order = j;
#pragma unroll
                for (int q = 0; q < SBR_MAX_ORDER; ++q) c.face[q] = q < j ? faces[q] : -1;
                c.ray = r;
                c.tan_err = tn;
                cand[pos] = c;
            }
        }
        if (hit < 0 || j == K) {
            if (out_tri || out_t)
                for (int q = j + 1; q <= K; ++q) {
                    if (out_tri) out_tri[i * (K + 1) + q] = -1;
                    if (out_t) out_t[i * (K + 1) + q] = INFINITY;
                }
            break;
        }
        // specular reflection on the face plane: o' = o + t d,
        // d' = d - (2 d.n) n (no renormalization), D' = D + t
        int32_t f = h.face;
        d3 nf = face_normal(S, f);
        d3 on = add(o, scl(t, d));
        double k2 = 2.0 * dot(d, nf);
        d = sub(d, scl(k2, nf));
        D = D + t;
        o = on;
        prev = f;
        faces[j] = f;
    }
    if (COUNT) {
        atomicAdd(&tallies[0], (unsigned long long)segs);
        atomicAdd(&tallies[1], (unsigned long long)tl.nodes);
        atomicAdd(&tallies[2], (unsigned long long)tl.tris);
        atomicAdd(&tallies[3], (unsigned long long)events);
    }
}

hipError_t launch_trace(const SceneDev& S, const GridDev& g, const TraceArgs& A, int64_t first,
                        int64_t count, sbr_candidate* cand, int64_t cap,
                        unsigned long long* cand_count, int32_t* out_tri, double* out_t,
                        int32_t* err_flag, hipStream_t s, unsigned long long* tallies)
{
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (tallies)
        hipLaunchKernelGGL(k_trace<true>, dim3((unsigned)blocks), dim3(256), 0, s, S, g, A, first,
                           count, cand, cap, cand_count, out_tri, out_t, err_flag, tallies);
    else
        hipLaunchKernelGGL(k_trace<false>, dim3((unsigned)blocks), dim3(256), 0, s, S, g, A,
                           first, count, cand, cap, cand_count, out_tri, out_t, err_flag,
                           tallies);
    return hipGetLastError();
}

// ===========================================================================
// Canonical order of reception events and path test 1
// ===========================================================================
// Key (rx, order, face sequence); ties by smaller error angle, then lower
// launch ray (the double-counting test keeps the smaller error angle).
__device__ static inline int key_cmp(const sbr_candidate& a, const sbr_candidate& b)
{
    if (a.rx != b.rx) return a.rx < b.rx ? -1 : 1;
    if (a.order != b.order) return a.order < b.order ? -1 : 1;
#pragma unroll
    for (int j = 0; j < SBR_MAX_ORDER; ++j)
        if (a.face[j] != b.face[j]) return a.face[j] < b.face[j] ? -1 : 1;
    return 0;
}

__device__ static inline bool cand_less(const sbr_candidate* __restrict__ C, uint32_t ia,
                                        uint32_t ib)
{
    if (ia == 0xffffffffu) return false;
    if (ib == 0xffffffffu) return true;
    const sbr_candidate a = C[ia], b = C[ib];
    int c = key_cmp(a, b);
    if (c) return c < 0;
    if (a.tan_err != b.tan_err) return a.tan_err < b.tan_err;
    return a.ray < b.ray;
}

__global__ void k_iota(uint32_t* idx, int64_t n, int64_t P)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P) idx[i] = i < n ? (uint32_t)i : 0xffffffffu;
}

// One global compare-exchange pass of the bitonic network (stride j, stage k).
__global__ void k_bitonic_global(const sbr_candidate* __restrict__ C, uint32_t* idx, int64_t P,
                                 int64_t j, int64_t k)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    int64_t l = i ^ j;
    if (l <= i) return;
    bool asc = (i & k) == 0;
    uint32_t a = idx[i], b = idx[l];
    bool swap = asc ? cand_less(C, b, a) : cand_less(C, a, b);
    if (swap) {
        idx[i] = b;
        idx[l] = a;
    }
}

// All passes of stage k with stride j <= 512 inside one 1024-element tile in
// LDS.  With first_stage set, it runs every stage k = 2..1024 of the tile.
__global__ __launch_bounds__(512) void k_bitonic_local(const sbr_candidate* __restrict__ C,
                                                       uint32_t* idx, int64_t P, int64_t k,
                                                       int first_stage)
{
    __shared__ uint32_t s[1024];
    int64_t base = (int64_t)blockIdx.x * 1024;
    int t = threadIdx.x;
    s[t] = idx[base + t];
    s[t + 512] = idx[base + t + 512];
    __syncthreads();
    int64_t k_lo = first_stage ? 2 : k, k_hi = first_stage ? 1024 : k;
    for (int64_t kk = k_lo; kk <= k_hi; kk <<= 1) {
        for (int64_t j = (first_stage ? kk : 1024) >> 1; j > 0; j >>= 1) {
            if (!first_stage && j > 512) continue;
            int i = 2 * t - (t & (int)(j - 1));  // lower element of the pair
            int l = i + (int)j;
            bool asc = ((base + i) & kk) == 0;
            uint32_t a = s[i], b = s[l];
            bool swap = asc ? cand_less(C, b, a) : cand_less(C, a, b);
            if (swap) {
                s[i] = b;
                s[l] = a;
            }
            __syncthreads();
        }
    }
    idx[base + t] = s[t];
    idx[base + t + 512] = s[t + 512];
}

int64_t pow2_at_least(int64_t n)
{
    int64_t p = 1024;
    while (p < n) p <<= 1;
    return p;
}

hipError_t launch_sort_candidates(const sbr_candidate* C, int64_t n, uint32_t* idx,
                                  hipStream_t s)
{
    int64_t P = pow2_at_least(n);
    hipLaunchKernelGGL(k_iota, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, idx, n, P);
    if (n <= 1) return hipGetLastError();
    unsigned tiles = (unsigned)(P / 1024);
    hipLaunchKernelGGL(k_bitonic_local, dim3(tiles), dim3(512), 0, s, C, idx, P, (int64_t)0, 1);
    for (int64_t k = 2048; k <= P; k <<= 1) {
        for (int64_t j = k >> 1; j > 512; j >>= 1)
            hipLaunchKernelGGL(k_bitonic_global, dim3((unsigned)((P + 255) / 256)), dim3(256), 0,
                               s, C, idx, P, j, k);
        hipLaunchKernelGGL(k_bitonic_local, dim3(tiles), dim3(512), 0, s, C, idx, P, k, 0);
    }
    return hipGetLastError();
}

__global__ void k_heads(const sbr_candidate* __restrict__ C, const uint32_t* __restrict__ idx,
                        int64_t n, int32_t* __restrict__ flags)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    flags[i] = (i == 0 || key_cmp(C[idx[i]], C[idx[i - 1]]) != 0) ? 1 : 0;
}

hipError_t launch_heads(const sbr_candidate* C, const uint32_t* idx, int64_t n, int32_t* flags,
                        hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_heads, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, C, idx, n,
                       flags);
    return hipGetLastError();
}

// ---- exclusive scan (tiles of 1024 = 256 threads x 4) ---------------------
__global__ __launch_bounds__(256) void k_scan_tile(const int32_t* __restrict__ in,
                                                   int32_t* __restrict__ out, int64_t n,
                                                   int32_t* __restrict__ tile_sum)
{
    __shared__ int32_t s[256];
    int64_t base = (int64_t)blockIdx.x * 1024 + 4 * threadIdx.x;
    int32_t v[4];
    int32_t acc = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        v[q] = base + q < n ? in[base + q] : 0;
        acc += v[q];
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        int32_t add_v = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += add_v;
        __syncthreads();
    }
    int32_t run = s[threadIdx.x] - acc;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (base + q < n) out[base + q] = run;
        run += v[q];
    }
    if (threadIdx.x == 255) tile_sum[blockIdx.x] = s[255];
}

__global__ void k_scan_add(int32_t* __restrict__ out, int64_t n, const int32_t* __restrict__ add_v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += add_v[i / 1024];
}

__global__ void k_scan_total(const int32_t* in, const int32_t* out, int64_t n, int32_t* total)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *total = n > 0 ? out[n - 1] + in[n - 1] : 0;
}

size_t scan_scratch_bytes(int64_t n)
{
    size_t b = 0;
    int64_t m = n;
    do {
        m = (m + 1023) / 1024;
        b += 2 * sizeof(int32_t) * (size_t)(m + 1);
    } while (m > 1);
    return b + 256;
}

static hipError_t scan_rec(const int32_t* in, int32_t* out, int64_t n, int32_t* scratch,
                           hipStream_t s)
{
    int64_t tiles = (n + 1023) / 1024;
    int32_t* sums = scratch;
    int32_t* sums_scan = scratch + tiles + 1;
    hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)tiles), dim3(256), 0, s, in, out, n, sums);
    if (tiles > 1) {
        (void)scan_rec(sums, sums_scan, tiles, scratch + 2 * (tiles + 1), s);
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n,
                           sums_scan);
    }
    return hipGetLastError();
}

hipError_t launch_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* total, void* scratch,
                       hipStream_t s)
{
    if (n > 0) (void)scan_rec(in, out, n, (int32_t*)scratch, s);
    hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(64), 0, s, in, out, n, total);
    return hipGetLastError();
}

__global__ void k_gather_unique(const sbr_candidate* __restrict__ C,
                                const uint32_t* __restrict__ idx,
                                const int32_t* __restrict__ flags,
                                const int32_t* __restrict__ offs, int64_t n,
                                sbr_candidate* __restrict__ U)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flags[i]) return;
    U[offs[i]] = C[idx[i]];
}

hipError_t launch_gather_unique(const sbr_candidate* C, const uint32_t* idx, const int32_t* flags,
                                const int32_t* offs, int64_t n, sbr_candidate* U, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_unique, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, C,
                       idx, flags, offs, n, U);
    return hipGetLastError();
}

__global__ void k_gather_sorted(const sbr_candidate* __restrict__ C,
                                const uint32_t* __restrict__ idx, int64_t n,
                                sbr_candidate* __restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = C[idx[i]];
}

hipError_t launch_gather_sorted(const sbr_candidate* C, const uint32_t* idx, int64_t n,
                                sbr_candidate* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_sorted, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, C,
                       idx, n, out);
    return hipGetLastError();
}

// ===========================================================================
// Iterative precise algorithm (Sec. III.B)
// ===========================================================================
struct Follow {
    double tan_err, D, Llast;
};

// Trace direction d0 from Tx through exactly the faces of a path of order k
// and report the error angle of Rx on the last segment (no cone condition).
// A sub-ray is a usable path only if it meets the same faces in the same
// order and Rx lies ahead on its last segment before the next obstacle.
// With pts/din non-NULL the reflection points and incoming directions are
// stored.
__device__ static bool follow(const SceneDev& S, d3 tx, d3 d0, d3 rx, int k,
                              const int32_t* faces, float delta, Follow* F, d3* pts, d3* din,
                              int32_t* err)
{
    d3 o = tx, d = d0;
    double D = 0.0;
    int32_t prev = -1;
    for (int j = 0;; ++j) {
        HitRec h;
        int32_t hit = traverse<false>(S, o, d, prev, prev, S.t_eps, INFINITY, delta, &h, err);
        if (j == k) {
            double t = hit < 0 ? INFINITY : h.t;
            double tn;
            if (!capture(o, d, D, t, rx, -1.0, &tn)) return false;
            F->tan_err = tn;
            F->D = D;
            F->Llast = norm(sub(rx, o));
            return true;
        }
        if (hit < 0 || h.face != faces[j]) return false;
        d3 nf = face_normal(S, h.face);
        d3 on = add(o, scl(h.t, d));
        if (din) din[j] = d;
        double k2 = 2.0 * dot(d, nf);
        d = sub(d, scl(k2, nf));
        D = D + h.t;
        o = on;
        if (pts) pts[j] = on;
        prev = h.face;
    }
}

// Orthonormal basis (u, v) of the plane normal to the unit axis a: e is the
// coordinate axis with the smallest |a_i| (ties: lowest i),
// u = normalize(e - a_i a), v = a x u.
__device__ static inline void basis(d3 a, d3* u, d3* v)
{
    double c0 = fabs(a.x), c1 = fabs(a.y), c2 = fabs(a.z);
    int i = 0;
    double ci = c0;
    if (c1 < ci) { i = 1; ci = c1; }
    if (c2 < ci) { i = 2; }
    d3 e = mk(i == 0 ? 1.0 : 0.0, i == 1 ? 1.0 : 0.0, i == 2 ? 1.0 : 0.0);
    double ai = i == 0 ? a.x : (i == 1 ? a.y : a.z);
    *u = normalize(sub(e, scl(ai, a)));
    *v = cross(a, *u);
}

// Sub-ray s of a cone with axis a: the cone's disc (radius rho_prev in the
// plane tangent to the unit sphere at a) is covered by six discs of radius
// rho = rho_prev / sqrt(3) whose centres sit at distance rho from the axis at
// phases 0, 60, ..., 300 degrees; sub-ray 6 is the axis itself.
__device__ static inline d3 subray(d3 a, d3 u, d3 v, double rho, int s)
{
    if (s == 6) return a;
    const double h = sqrt(3.0) * 0.5;
    double cs, ss;
    switch (s) {
        case 0: cs = 1.0; ss = 0.0; break;
        case 1: cs = 0.5; ss = h; break;
        case 2: cs = -0.5; ss = h; break;
        case 3: cs = -1.0; ss = 0.0; break;
        case 4: cs = -0.5; ss = -h; break;
        default: cs = 0.5; ss = -h; break;
    }
    d3 w = add(scl(cs, u), scl(ss, v));
    return normalize(add(a, scl(rho, w)));
}

// Stop rule: with a target error angle, stop once
// tan(err) <= tan(target) * L_last / L_total (the AOA error grows from the AOD
// error by about L_total / L_last, so both meet the target).
__device__ static inline bool target_met(double tan_err, double tan_tgt, double D, double Llast)
{
    double Ltot = D + Llast;
    double thr = (tan_tgt * Llast) / Ltot;
    return tan_err <= thr;
}

// Eight lanes per path: lane s traces sub-ray s (s < subrays); the group
// keeps the smallest error angle (ties: lower s) as the next axis.
__global__ __launch_bounds__(256) void k_refine(SceneDev S, GridDev g, RefineArgs A, float delta,
                                                const sbr_candidate* __restrict__ uniq, int64_t U,
                                                RefineOut* __restrict__ out,
                                                int32_t* __restrict__ err)
{
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t p = gid >> 3;
    int s = (int)(gid & 7);
    if (p >= U) return;
    const sbr_candidate c = uniq[p];
    const d3 tx = mk(A.tx[0], A.tx[1], A.tx[2]);
    const d3 rx = mk(A.rx[3 * c.rx], A.rx[3 * c.rx + 1], A.rx[3 * c.rx + 2]);
    d3 axis = mk(g.dir[c.ray], g.dir[g.N + c.ray], g.dir[2 * g.N + c.ray]);
    Follow F0;
    if (!follow(S, tx, axis, rx, c.order, c.face, delta, &F0, nullptr, nullptr, err)) {
        if (s == 0) {
            RefineOut o;
            st3(o.axis, axis);
            o.tan_err = NAN;
            o.iters = 0;
            o.flags = SBR_PATH_STALLED;
            out[p] = o;
        }
        return;
    }
    double tan = F0.tan_err;
    uint32_t flags = 0;
    int32_t iters = 0;
    double rho = A.thl;
    bool met = A.tan_tgt > 0.0 && target_met(tan, A.tan_tgt, F0.D, F0.Llast);
    if (met) flags |= SBR_PATH_TARGET_MET;
    for (int i = 1; i <= A.iterations && !met; ++i) {
        rho = rho / sqrt(3.0);
        d3 u, v;
        basis(axis, &u, &v);
        Follow F;
        bool ok = false;
        if (s < A.subrays) ok = follow(S, tx, subray(axis, u, v, rho, s), rx, c.order, c.face,
                                       delta, &F, nullptr, nullptr, err);
        double bt = ok ? F.tan_err : INFINITY;
        int bs = ok ? s : 8;
        double myD = ok ? F.D : 0.0, myL = ok ? F.Llast : 0.0;
#pragma unroll
        for (int off = 1; off < 8; off <<= 1) {
            double ot = __shfl_xor(bt, off, 8);
            int os = __shfl_xor(bs, off, 8);
            if (ot < bt || (ot == bt && os < bs)) {
                bt = ot;
                bs = os;
            }
        }
        if (bs >= 8) {
            flags |= SBR_PATH_STALLED;
            break;
        }
        double wD = __shfl(myD, bs, 8), wL = __shfl(myL, bs, 8);
        axis = subray(axis, u, v, rho, bs);
        tan = bt;
        iters = i;
        if (A.tan_tgt > 0.0 && target_met(bt, A.tan_tgt, wD, wL)) {
            flags |= SBR_PATH_TARGET_MET;
            met = true;
        }
    }
    if (s == 0) {
        RefineOut o;
        st3(o.axis, axis);
        o.tan_err = tan;
        o.iters = iters;
        o.flags = flags;
        out[p] = o;
    }
}

hipError_t launch_refine(const SceneDev& S, const GridDev& g, const RefineArgs& A,
                         const sbr_candidate* uniq, int64_t U, RefineOut* out, float delta,
                         int32_t* err, hipStream_t s)
{
    if (U <= 0) return hipSuccess;
    int64_t threads = U * 8;
    hipLaunchKernelGGL(k_refine, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, S, g, A,
                       delta, uniq, U, out, err);
    return hipGetLastError();
}

// ===========================================================================
// Path quantities, path test 2 and power (Sec. III.A, Sec. IV)
// ===========================================================================
struct cx {
    double re, im;
};
__device__ static inline cx cadd(cx a, cx b) { return cx{a.re + b.re, a.im + b.im}; }
__device__ static inline cx csub(cx a, cx b) { return cx{a.re - b.re, a.im - b.im}; }
__device__ static inline cx cmulr(cx a, double r) { return cx{a.re * r, a.im * r}; }
__device__ static inline cx cdiv(cx a, cx b)
{
    double den = b.re * b.re + b.im * b.im;
    return cx{(a.re * b.re + a.im * b.im) / den, (a.im * b.re - a.re * b.im) / den};
}
__device__ static inline double cabs2(cx a) { return a.re * a.re + a.im * a.im; }
// principal square root
__device__ static inline cx csqrt_p(cx z)
{
    double r = hypot(z.re, z.im);
    if (r == 0.0) return cx{0.0, 0.0};
    if (z.re >= 0.0) {
        double t = sqrt(0.5 * (r + z.re));
        return cx{t, z.im / (2.0 * t)};
    }
    double t = sqrt(0.5 * (r - z.re));
    return cx{fabs(z.im) / (2.0 * t), copysign(t, z.im)};
}

// Fresnel reflection for relative permittivity er at incidence cosine c:
//   G_perp = (c - sqrt(er - s^2)) / (c + sqrt(er - s^2)),
//   G_par  = (er c - sqrt(er - s^2)) / (er c + sqrt(er - s^2)),
// and the unpolarized power reflectance 0.5 (|G_perp|^2 + |G_par|^2).
__device__ static inline double fresnel_avg(double c, cx er)
{
    double s2 = 1.0 - c * c;
    cx root = csqrt_p(csub(er, cx{s2, 0.0}));
    cx cc = cx{c, 0.0};
    cx gs = cdiv(csub(cc, root), cadd(cc, root));
    cx erc = cmulr(er, c);
    cx gp = cdiv(csub(erc, root), cadd(erc, root));
    return 0.5 * (cabs2(gs) + cabs2(gp));
}

__device__ static inline double refl_at(const SceneDev& S, int32_t f, d3 din)
{
    d3 n = face_normal(S, f);
    double c = fabs(dot(din, n)) / norm(din);
    int32_t m = S.fmat[f];
    return fresnel_avg(c, cx{S.eps[2 * m], S.eps[2 * m + 1]});
}

// P_r = P_t + 20 log10(lambda / (4 pi L)) + sum_j 10 log10(R_j)   [dBm]
__device__ static inline double path_power(double ptx, double freq, double L, const double* refl,
                                           int k)
{
    double lambda = kC0 / freq;
    double p = ptx + 20.0 * log10(lambda / (4.0 * kPi * L));
    for (int j = 0; j < k; ++j) p += 10.0 * log10(refl[j]);
    return p;
}

// Point p inside face f: inside any of its triangles, barycentric tolerance 1e-9.
__device__ static bool inside_face(const SceneDev& S, int32_t f, d3 p)
{
    const double tol = 1e-9;
    for (int32_t q = S.fstart[f]; q < S.fstart[f + 1]; ++q) {
        TriD T = load_tri(S.tris + S.ftris[q]);
        d3 v0 = mk(T.v0x, T.v0y, T.v0z), e1 = mk(T.e1x, T.e1y, T.e1z), e2 = mk(T.e2x, T.e2y, T.e2z);
        d3 w = sub(p, v0);
        double d00 = dot(e1, e1);
        double d01 = dot(e1, e2);
        double d11 = dot(e2, e2);
        double d20 = dot(w, e1);
        double d21 = dot(w, e2);
        double den = d00 * d11 - d01 * d01;
        if (den == 0.0) continue;
        double b = (d11 * d20 - d01 * d21) / den;
        double gg = (d00 * d21 - d01 * d20) / den;
        if (b >= -tol && gg >= -tol && b + gg <= 1.0 + tol) return true;
    }
    return false;
}

// Segment A -> B blocked by a triangle not of faces fa / fb, hit strictly
// inside (1e-9, 1 - 1e-9) of the segment parameter.
__device__ static bool blocked(const SceneDev& S, d3 A, d3 B, int32_t fa, int32_t fb,
                               float delta, int32_t* err)
{
    HitRec h;
    return traverse<true>(S, A, sub(B, A), fa, fb, 1e-9, 1.0 - 1e-9, delta, &h, err) >= 0;
}

// Image-method solve of a face sequence: images of Tx mirrored across the
// face planes in order, then back-projection from Rx.  Path test 2
// (validity): every back-projection parameter in (0, 1), every reflection
// point inside its face, no segment blocked.
__device__ static bool exact_solve(const SceneDev& S, d3 tx, d3 rx, int k, const int32_t* faces,
                                   d3* pts, float delta, int32_t* err)
{
    d3 img[SBR_MAX_ORDER + 1];
    img[0] = tx;
    for (int j = 0; j < k; ++j) {
        int32_t f = faces[j];
        d3 n = face_normal(S, f);
        double c = S.fplane[4 * (size_t)f + 3];
        double dd = dot(n, img[j]) - c;
        img[j + 1] = sub(img[j], scl(2.0 * dd, n));
    }
    bool ok = true;
    d3 X = rx;
    for (int j = k - 1; j >= 0; --j) {
        int32_t f = faces[j];
        d3 n = face_normal(S, f);
        double c = S.fplane[4 * (size_t)f + 3];
        d3 dir = sub(img[j + 1], X);
        double den = dot(n, dir);
        double s = (c - dot(n, X)) / den;
        if (!(s > 0.0 && s < 1.0)) ok = false;
        pts[j] = add(X, scl(s, dir));
        X = pts[j];
    }
    if (!ok) return false;
    for (int j = 0; j < k; ++j)
        if (!inside_face(S, faces[j], pts[j])) return false;
    d3 A = tx;
    int32_t fa = -1;
    for (int j = 0; j < k; ++j) {
        if (blocked(S, A, pts[j], fa, faces[j], delta, err)) return false;
        A = pts[j];
        fa = faces[j];
    }
    if (blocked(S, A, rx, fa, -1, delta, err)) return false;
    return true;
}

__device__ static inline double poly_length(d3 tx, const d3* p, int k, d3 rx)
{
    double L = 0.0;
    d3 prev = tx;
    for (int j = 0; j < k; ++j) {
        L = L + norm(sub(p[j], prev));
        prev = p[j];
    }
    L = L + norm(sub(rx, prev));
    return L;
}

__global__ __launch_bounds__(256) void k_solve(SceneDev S, SolveArgs A, float delta,
                                               const sbr_candidate* __restrict__ uniq,
                                               const RefineOut* __restrict__ rf, int64_t U,
                                               sbr_path* __restrict__ paths,
                                               int32_t* __restrict__ keep,
                                               int32_t* __restrict__ err)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= U) return;
    const sbr_candidate c = uniq[p];
    const RefineOut R = rf[p];
    const int k = c.order;
    const d3 tx = mk(A.tx[0], A.tx[1], A.tx[2]);
    const d3 rx = mk(A.rx[3 * c.rx], A.rx[3 * c.rx + 1], A.rx[3 * c.rx + 2]);
    d3 axis = ld3(R.axis);
    d3 pts[SBR_MAX_ORDER], din[SBR_MAX_ORDER];
    for (int j = 0; j < SBR_MAX_ORDER; ++j) {
        pts[j] = mk(0.0, 0.0, 0.0);
        din[j] = mk(0.0, 0.0, 0.0);
    }
    Follow F;
    follow(S, tx, axis, rx, k, c.face, delta, &F, pts, din, err);

    sbr_path o;
    o.rx = c.rx;
    o.order = k;
    for (int q = 0; q < SBR_MAX_ORDER; ++q) o.face[q] = c.face[q];
    o.launch_ray = c.ray;
    o.iters_used = R.iters;
    o.flags = R.flags;
    o.init_tan_err = c.tan_err;
    o.tan_err = R.tan_err;
    st3(o.axis, axis);
    // refined path: Tx -> reflection points of the final ray -> Rx
    double L = poly_length(tx, pts, k, rx);
    o.length_m = L;
    o.delay_s = L / kC0;
    st3(o.aod, axis);
    d3 last = k > 0 ? pts[k - 1] : tx;
    st3(o.aoa, normalize(sub(last, rx)));
    double refl[SBR_MAX_ORDER];
    for (int j = 0; j < k; ++j) refl[j] = refl_at(S, c.face[j], din[j]);
    o.power_dbm = path_power(A.tx_power_dbm, A.freq_hz, L, refl, k);
    o.err_angle_deg = atan(R.tan_err) * (180.0 / kPi);
    // exact path of the same faces
    d3 ep[SBR_MAX_ORDER];
    bool ok = exact_solve(S, tx, rx, k, c.face, ep, delta, err);
    double EL = poly_length(tx, ep, k, rx);
    o.exact_length_m = EL;
    o.exact_delay_s = EL / kC0;
    d3 firstp = k > 0 ? ep[0] : rx;
    st3(o.exact_aod, normalize(sub(firstp, tx)));
    d3 elast = k > 0 ? ep[k - 1] : tx;
    st3(o.exact_aoa, normalize(sub(elast, rx)));
    d3 prev = tx;
    for (int j = 0; j < k; ++j) {
        refl[j] = refl_at(S, c.face[j], sub(ep[j], prev));
        prev = ep[j];
    }
    o.exact_power_dbm = path_power(A.tx_power_dbm, A.freq_hz, EL, refl, k);
    if (!ok) o.flags |= SBR_PATH_INVALID;
    paths[p] = o;
    keep[p] = (ok || A.keep_invalid) ? 1 : 0;
}

hipError_t launch_solve(const SceneDev& S, const SolveArgs& A, const sbr_candidate* uniq,
                        const RefineOut* rf, int64_t U, sbr_path* paths, int32_t* keep,
                        float delta, int32_t* err, hipStream_t s)
{
    if (U <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_solve, dim3((unsigned)((U + 255) / 256)), dim3(256), 0, s, S, A, delta,
                       uniq, rf, U, paths, keep, err);
    return hipGetLastError();
}

__global__ void k_compact_paths(const sbr_path* __restrict__ paths,
                                const int32_t* __restrict__ keep,
                                const int32_t* __restrict__ offs, int64_t U,
                                sbr_path* __restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < U && keep[i]) out[offs[i]] = paths[i];
}

hipError_t launch_compact_paths(const sbr_path* paths, const int32_t* keep, const int32_t* offs,
                                int64_t U, sbr_path* out, hipStream_t s)
{
    if (U <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_compact_paths, dim3((unsigned)((U + 255) / 256)), dim3(256), 0, s, paths,
                       keep, offs, U, out);
    return hipGetLastError();
}

}  // namespace sbr
