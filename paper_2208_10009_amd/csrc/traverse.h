// traverse.h -- BVH traversal with FP64 ray-triangle decisions, shared by the
// trace, refinement and solve kernels.
//
// The scene is a BVH4 (128-byte nodes with four FP32 child boxes).  Memory
// plan per workgroup (dynamic LDS, see LdsPlan): the first n_nodes BVH
// nodes (the top levels: nodes are numbered breadth-first), all triangles
// when they fit, and a per-lane traversal stack of `depth` entries.  Deeper
// nodes are read from global memory, and stack entries beyond `depth` spill
// to a private array.
//
// Conservativeness.  The FP32 ray (o32, d32) differs from the FP64 ray by at
// most 2^-24 (|o| + t|d|) per component at parameter t; for any point of the
// scene this is below 3 * 2^-24 R, R = max(|Tx|, scene extent).  Each FP32
// box already contains its triangles (outward rounding) and is widened by
// delta = 2^-20 R > 3 * 2^-24 R plus the rounding of the widening itself, so
// the FP32 ray passes through the widened box wherever the FP64 ray passes
// through the true box.  The slab arithmetic then errs by a few ulp in t,
// covered by the factor 1 + 2^-20 on the exit and pruning bounds.  Culling
// therefore never removes a triangle that the FP64 test would accept.
#pragma once
#include <math.h>

#include "geom.h"
#include "layout.h"

namespace sbr {

extern __shared__ float4 g_smem4[];

// Copy the staged part of the scene into LDS (every thread of the block must
// call this before any traversal).
__device__ static inline void stage_scene(const SceneDev& S, const LdsPlan& L)
{
    const float4* sn = (const float4*)S.nodes;
    for (int i = threadIdx.x; i < 8 * L.n_nodes; i += blockDim.x) g_smem4[i] = sn[i];
    const float4* st = (const float4*)S.tris;
    float4* dt = g_smem4 + 8 * L.n_nodes;
    for (int i = threadIdx.x; i < 5 * L.n_tris; i += blockDim.x) dt[i] = st[i];
    __syncthreads();
}

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
    // the first test needs every part of the record (u is discarded when
    // det = 0), so the compiler issues the record's loads together rather
    // than loading v0 only after the det test
    d3 s = sub(o, mk(T.v0x, T.v0y, T.v0z));
    double u = dot(s, p) / det;
    if ((det == 0.0) | !(u >= 0.0)) return false;
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

// Loads through the global address space: the scene arrays are global
// memory, and telling the compiler so turns generic (flat) loads, which also
// count against the LDS wait counter, into global loads.
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float4 gld(const float4* p)
{
    const f4v v = *(const __attribute__((address_space(1))) f4v*)p;
    return make_float4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ double2 gld(const double2* p)
{
    const d2v v = *(const __attribute__((address_space(1))) d2v*)p;
    return make_double2(v.x, v.y);
}

__device__ __forceinline__ double gld(const double* p)
{
    return *(const __attribute__((address_space(1))) double*)p;
}

__device__ __forceinline__ int32_t gld(const int32_t* p)
{
    return *(const __attribute__((address_space(1))) int32_t*)p;
}

// Loads through the constant address space, for arrays that no kernel
// writes while it reads them (the receivers): at a wave-uniform address the
// compiler then issues scalar loads.
__device__ __forceinline__ double cld(const double* p)
{
    return *(const __attribute__((address_space(4))) double*)p;
}

__device__ __forceinline__ float4 cld4(const float4* p)
{
    const f4v v = *(const __attribute__((address_space(4))) f4v*)p;
    return make_float4(v.x, v.y, v.z, v.w);
}

// A triangle record from five 16-byte pieces (v0, e1, e2 as doubles; the
// last 8 bytes hold the face id and the input index).
__device__ static inline TriD make_tri(double2 a, double2 b, double2 c, double2 d, double2 e)
{
    TriD T;
    T.v0x = a.x; T.v0y = a.y; T.v0z = b.x; T.e1x = b.y; T.e1y = c.x;
    T.e1z = c.y; T.e2x = d.x; T.e2y = d.y; T.e2z = e.x;
    const long long w = __double_as_longlong(e.y);
    T.face = (int32_t)(w & 0xffffffffll);
    T.orig = (int32_t)(w >> 32);
    return T;
}

// Triangle i (leaf order), from LDS when staged (LDS instances only).
template <bool LDS>
__device__ static inline TriD tri_at(const SceneDev& S, const LdsPlan& L, int32_t i)
{
    if (LDS && i < L.n_tris) {
        const double2* q = (const double2*)(g_smem4 + 8 * L.n_nodes + 5 * i);
        return make_tri(q[0], q[1], q[2], q[3], q[4]);
    }
    const double2* q = (const double2*)(S.tris + i);
    return make_tri(gld(q), gld(q + 1), gld(q + 2), gld(q + 3), gld(q + 4));
}

struct HitRec {
    double t;
    int32_t pos, face, orig;
};

// Work counts of the instrumented trace kernel: node visits and triangle
// tests per lane, the tests not skipped as the face just left, and the steps
// of the wave (loop passes in which at least one lane visits a node, tests a
// triangle, traces a segment or tests receivers; 64 lanes per wave, so nodes
// / (64 wave_nodes) is the share of lanes busy in the node loop).
struct Tally {
    uint32_t nodes, tris, fp64_tris, wave_nodes, wave_tris, wave_segs, wave_rx;
    uint32_t rx_nodes, rx_tests;  // receiver-tree nodes tested, receivers tested (per lane)
};

// Whether this lane is the lowest active lane of its wave (counts once per
// wave and pass).
__device__ static inline bool first_active_lane()
{
    return (int)__lane_id() == __builtin_ctzll(__ballot(1));
}

constexpr int kShortStack = 16;  // LDS stack entries per lane without an LDS plan

// Closest hit (ANY = false: smallest t; equal t -> lower face id -> lower
// input index) or any hit (ANY = true) of the ray o + t d, t_lo < t < t_hi,
// ignoring triangles of faces xa and xb.  Returns the leaf-order position of
// the hit or -1.  LDS = false reads everything from global memory (no LDS
// plan needed) and keeps the top of the stack in a static LDS array.
template <bool ANY, bool COUNT, bool LDS, int BLK = 256>
__device__ static int32_t traverse(const SceneDev& S, const LdsPlan& L, d3 o, d3 d, int32_t xa,
                                   int32_t xb, double t_lo, double t_hi, float delta, HitRec* h,
                                   int32_t* err, Tally* tally = nullptr, bool seeded = false)
{
    const float slack = 1.0f + 9.5367431640625e-07f;  // 1 + 2^-20
    float ox = (float)o.x, oy = (float)o.y, oz = (float)o.z;
    float dx = (float)d.x, dy = (float)d.y, dz = (float)d.z;
    dx = dx >= 0.0f ? fmaxf(dx, 1e-20f) : fminf(dx, -1e-20f);
    dy = dy >= 0.0f ? fmaxf(dy, 1e-20f) : fminf(dy, -1e-20f);
    dz = dz >= 0.0f ? fmaxf(dz, 1e-20f) : fminf(dz, -1e-20f);
    const float ix = 1.0f / dx, iy = 1.0f / dy, iz = 1.0f / dz;
    // lo - delta - o = lo - (o + delta);  hi + delta - o = hi - (o - delta).
    // A slab parameter (lo - l) i is formed as fma(lo, i, -(l i)): the one
    // rounding of l i moves the plane by at most 2^-24 |l|, less than the
    // rounding of the subtraction it replaces, inside the widening delta.
    const float lx = ox + delta, ly = oy + delta, lz = oz + delta;
    const float hx = ox - delta, hy = oy - delta, hz = oz - delta;
    const float nlx = -(lx * ix), nly = -(ly * iy), nlz = -(lz * iz);
    const float nhx = -(hx * ix), nhy = -(hy * iy), nhz = -(hz * iz);
    // Near and far planes per axis by the sign of the direction: for i > 0,
    // lo < hi and nl <= nh give fma(lo, i, nl) <= fma(hi, i, nh) (products,
    // sums and roundings are monotonic), and the reverse for i < 0, so the
    // near plane's parameter is exactly the minimum of the two and the far
    // one's the maximum.  The lane loads the rows it needs instead of taking
    // minima and maxima: the near row of an axis at node + s (s = 0 for lo,
    // 64 for hi, plus the axis's row offset) and the far row at (node + s) ^ 64.
    const uint32_t sx = ix > 0.0f ? 0u : 64u, sy = iy > 0.0f ? 0u : 64u;
    const uint32_t sz = iz > 0.0f ? 0u : 64u;
    const float cnx = ix > 0.0f ? nlx : nhx, cfx = ix > 0.0f ? nhx : nlx;
    const float cny = iy > 0.0f ? nly : nhy, cfy = iy > 0.0f ? nhy : nly;
    const float cnz = iz > 0.0f ? nlz : nhz, cfz = iz > 0.0f ? nhz : nlz;

    float tb = isinf(t_hi) ? INFINITY : (float)t_hi * slack;
    if (seeded && h->pos >= 0) {
        // closest-hit search seeded with a hit the caller found (one of the
        // triangles this search would test, with the same arithmetic): the
        // pruning bound starts at it, and the result is the same
        float ts = (float)h->t * slack;
        if ((double)ts < h->t) ts = nextafterf(ts, INFINITY);
        tb = fminf(tb, ts);
    } else {
        h->pos = -1;
        h->t = INFINITY;
        h->face = 0x7fffffff;
        h->orig = 0x7fffffff;
    }

    // The first stack entries live in LDS: the plan's stack (LDS instances)
    // or a fixed short stack of kShortStack entries per lane (workgroups of
    // at most BLK lanes); deeper entries go to the private array.
    int32_t* lst;
    int bd, ldepth;
    if constexpr (LDS) {
        lst = (int32_t*)(g_smem4) + (L.stack_off >> 2) + threadIdx.x;
        bd = blockDim.x;
        ldepth = L.depth;
    } else {
        __shared__ int32_t s_stack[kShortStack * BLK];
        lst = s_stack + threadIdx.x;
        bd = BLK;
        // a lane beyond BLK (a caller instantiated for a smaller workgroup)
        // keeps its whole stack in private memory instead of past the array
        ldepth = threadIdx.x < BLK ? kShortStack : 0;
    }
    int32_t ost[kTraceStack];
    int sp = 0;
    int32_t node = 0;
    for (;;) {
        // near and far plane rows (x, y, z) and the child index and count rows
        float4 nx4, ny4, nz4, fx4, fy4, fz4, q6, q7;
        const uint32_t nb = (uint32_t)node << 7;
        const uint32_t ax = nb + sx, ay = nb + sy, az = nb + sz;
        if (LDS && node < L.n_nodes) {
            const char* np = (const char*)g_smem4;
            nx4 = *(const float4*)(np + ax);
            fx4 = *(const float4*)(np + (ax ^ 64u));
            ny4 = *(const float4*)(np + ay + 16);
            fy4 = *(const float4*)(np + (ay ^ 64u) + 16);
            nz4 = *(const float4*)(np + az + 32);
            fz4 = *(const float4*)(np + (az ^ 64u) + 32);
            q6 = *(const float4*)(np + nb + 48);
            q7 = *(const float4*)(np + nb + 112);
        } else {
            const char* np = (const char*)S.nodes;
            nx4 = gld((const float4*)(np + ax));
            fx4 = gld((const float4*)(np + (ax ^ 64u)));
            ny4 = gld((const float4*)(np + ay + 16));
            fy4 = gld((const float4*)(np + (ay ^ 64u) + 16));
            nz4 = gld((const float4*)(np + az + 32));
            fz4 = gld((const float4*)(np + (az ^ 64u) + 32));
            q6 = gld((const float4*)(np + nb + 48));
            q7 = gld((const float4*)(np + nb + 112));
        }
        const int4 cidx = __builtin_bit_cast(int4, q6), ccnt = __builtin_bit_cast(int4, q7);
        if (COUNT) {
            tally->nodes += 1;
            if (first_active_lane()) tally->wave_nodes += 1;
        }
        float tn[4];
        bool hit[4];
        int32_t first[4], cnt[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float nx = k == 0 ? nx4.x : k == 1 ? nx4.y : k == 2 ? nx4.z : nx4.w;
            const float ny = k == 0 ? ny4.x : k == 1 ? ny4.y : k == 2 ? ny4.z : ny4.w;
            const float nz = k == 0 ? nz4.x : k == 1 ? nz4.y : k == 2 ? nz4.z : nz4.w;
            const float fx = k == 0 ? fx4.x : k == 1 ? fx4.y : k == 2 ? fx4.z : fx4.w;
            const float fy = k == 0 ? fy4.x : k == 1 ? fy4.y : k == 2 ? fy4.z : fy4.w;
            const float fz = k == 0 ? fz4.x : k == 1 ? fz4.y : k == 2 ? fz4.z : fz4.w;
            first[k] = k == 0 ? cidx.x : k == 1 ? cidx.y : k == 2 ? cidx.z : cidx.w;
            cnt[k] = k == 0 ? ccnt.x : k == 1 ? ccnt.y : k == 2 ? ccnt.z : ccnt.w;
            tn[k] = fmaxf(fmaxf(fmaf(nx, ix, cnx), fmaf(ny, iy, cny)), fmaf(nz, iz, cnz));
            const float tf =
                fminf(fminf(fmaf(fx, ix, cfx), fmaf(fy, iy, cfy)), fmaf(fz, iz, cfz)) * slack;
            // an empty slot (cnt < 0) has the inverted box: tn = +inf, tf = -inf
            hit[k] = tn[k] <= tf && tf >= 0.0f && tn[k] <= tb;
        }
        // leaf children first: their hits can only shrink the pruning bound
        uint32_t leaves = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) leaves |= (hit[k] && cnt[k] > 0) ? (1u << k) : 0u;
        while (leaves) {
            const int k = __builtin_ctz(leaves);
            leaves &= leaves - 1;
            const int32_t lf = k == 0 ? first[0] : k == 1 ? first[1] : k == 2 ? first[2] : first[3];
            const int32_t lc = k == 0 ? cnt[0] : k == 1 ? cnt[1] : k == 2 ? cnt[2] : cnt[3];
            for (int32_t i = lf; i < lf + lc; ++i) {
                TriD T = tri_at<LDS>(S, L, i);
                if (COUNT) {
                    tally->tris += 1;
                    if (first_active_lane()) tally->wave_tris += 1;
                }
                // the face test joins the result rather than guarding the
                // test, which would load the face word before the rest
                const bool skip = (T.face == xa) | (T.face == xb);
                if (COUNT && !skip) tally->fp64_tris += 1;
                double t;
                if (!mt_hit(T, o, d, t_lo, t_hi, &t) | skip) continue;
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
        // inner children still within the bound, nearest first: a sorting
        // network on (entry distance, node); empty entries sort last
        float k0 = (hit[0] && cnt[0] == 0 && tn[0] <= tb) ? tn[0] : INFINITY;
        float k1 = (hit[1] && cnt[1] == 0 && tn[1] <= tb) ? tn[1] : INFINITY;
        float k2 = (hit[2] && cnt[2] == 0 && tn[2] <= tb) ? tn[2] : INFINITY;
        float k3 = (hit[3] && cnt[3] == 0 && tn[3] <= tb) ? tn[3] : INFINITY;
        int32_t n0 = first[0], n1 = first[1], n2 = first[2], n3 = first[3];
        auto cswap = [](float& ka, int32_t& na, float& kb, int32_t& nb) {
            if (kb < ka) {
                const float tk = ka;
                ka = kb;
                kb = tk;
                const int32_t tnn = na;
                na = nb;
                nb = tnn;
            }
        };
        cswap(k0, n0, k1, n1);
        cswap(k2, n2, k3, n3);
        cswap(k0, n0, k2, n2);
        cswap(k1, n1, k3, n3);
        cswap(k1, n1, k2, n2);
        if (k0 == INFINITY) {
            if (sp == 0) break;
            --sp;
            if (sp < ldepth)
                node = lst[sp * bd];
            else
                node = ost[sp - ldepth];
            continue;
        }
        // push the farther ones, farthest first, and descend into the nearest
        const int c1 = k1 < INFINITY, c2 = k2 < INFINITY, c3 = k3 < INFINITY;
        const int npush = c1 + c2 + c3;
        if (sp + 3 <= ldepth) {
            // all in the LDS part: three unconditional writes at the slots
            // the finite keys take (the finite ones form a prefix, so a slot
            // an infinite key writes is either overwritten or above the top)
            lst[sp * bd] = n3;
            lst[(sp + c3) * bd] = n2;
            lst[(sp + c3 + c2) * bd] = n1;
            sp += npush;
            node = n0;
            continue;
        }
        if (sp + npush > kTraceStack) {
            atomicOr(err, 1);
            return h->pos;
        }
        if (k3 < INFINITY) {
            if (sp < ldepth) lst[sp * bd] = n3;
            else ost[sp - ldepth] = n3;
            ++sp;
        }
        if (k2 < INFINITY) {
            if (sp < ldepth) lst[sp * bd] = n2;
            else ost[sp - ldepth] = n2;
            ++sp;
        }
        if (k1 < INFINITY) {
            if (sp < ldepth) lst[sp * bd] = n1;
            else ost[sp - ldepth] = n1;
            ++sp;
        }
        node = n0;
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
    double L = D + ts;
    double ff = dot(f, f);
    if (thl >= 0.0) {
        // Cheap exact reject: when ff exceeds (thl L)^2 by more than 1e-9
        // relative, the rounded sqrt(ff) exceeds the rounded thl L whatever
        // the rounding of the three products, so the test below would fail.
        double lim = thl * L;
        if (ff > (lim * lim) * (1.0 + 1e-9)) return false;
    }
    double dp = sqrt(ff);
    if (thl >= 0.0 && !(dp <= thl * L)) return false;
    *tan_out = dp / L;
    return true;
}

// Can any receiver inside the box c +- h of a receiver-tree node pass the
// reception test of the segment (o, d, D, t)?  A receiver x that passes has
// foot parameter t*(x) = (x - o).d in (0, t] and lies within
// thl (D + t*(x)) of o + t*(x) d.  Over the box t*(x) <= T = (c - o).d +
// sum_i h_i |d_i|, so o + t*(x) d, with t*(x) in (0, min(t, T)], lies inside
// the box widened by rho = thl (D + min(t, T)) on every side: the segment's
// parameter range [0, min(t, T)] meets every axis's slab of the widened box
// (parameters by the inverse direction inv; an axis with d_i = 0 needs o_i in
// its slab).  rho is widened by 1e-6 relative and by m = 1e-9 of the lengths
// involved, and the range by m, far above the rounding of this test or of
// capture(), so the cull never drops a receiver that capture() accepts.  For
// receivers spread over a plane a box stays flat where a ball around the same
// receivers would reach far above and below it.
__device__ static inline bool rx_box_may_capture(d3 o, d3 d, d3 inv, double D, double t, d3 c,
                                                 d3 h, double thl)
{
    const d3 v = sub(c, o);
    const double T = dot(v, d) + (h.x * fabs(d.x) + h.y * fabs(d.y) + h.z * fabs(d.z));
    const double m = 1e-9 * (D + fabs(o.x) + fabs(o.y) + fabs(o.z) + fabs(c.x) + fabs(c.y) +
                             fabs(c.z) + h.x + h.y + h.z);
    if (T + m <= 0.0) return false;
    const double s1 = fmin(t, T) + m;
    const double rho = thl * (D + s1) * (1.0 + 1e-6) + m;
    double slo = -m, shi = s1;
    const double vv[3] = {v.x, v.y, v.z}, hh[3] = {h.x, h.y, h.z}, dd[3] = {d.x, d.y, d.z},
                 ii[3] = {inv.x, inv.y, inv.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        // o_a + s d_a in [c_a - h_a - rho, c_a + h_a + rho]
        const double e = hh[a] + rho, lo = vv[a] - e, hi = vv[a] + e;
        if (dd[a] > 0.0) {
            slo = fmax(slo, lo * ii[a]);
            shi = fmin(shi, hi * ii[a]);
        } else if (dd[a] < 0.0) {
            slo = fmax(slo, hi * ii[a]);
            shi = fmin(shi, lo * ii[a]);
        } else if (lo > 0.0 || hi < 0.0) {
            return false;
        }
    }
    return slo <= shi;
}

}  // namespace sbr
