// traverse.h -- BVH traversal with FP64 ray-triangle decisions, shared by the
// trace, refinement and solve kernels.
//
// Memory plan per workgroup (dynamic LDS, see LdsPlan): the first n_nodes BVH
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
#include "internal.h"

namespace sbr {

extern __shared__ float4 g_smem4[];

// Copy the staged part of the scene into LDS (every thread of the block must
// call this before any traversal).
__device__ static inline void stage_scene(const SceneDev& S, const LdsPlan& L)
{
    const float4* sn = (const float4*)S.nodes;
    for (int i = threadIdx.x; i < 4 * L.n_nodes; i += blockDim.x) g_smem4[i] = sn[i];
    const float4* st = (const float4*)S.tris;
    float4* dt = g_smem4 + 4 * L.n_nodes;
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
        const double2* q = (const double2*)(g_smem4 + 4 * L.n_nodes + 5 * i);
        return make_tri(q[0], q[1], q[2], q[3], q[4]);
    }
    const double2* q = (const double2*)(S.tris + i);
    return make_tri(gld(q), gld(q + 1), gld(q + 2), gld(q + 3), gld(q + 4));
}

struct HitRec {
    double t;
    int32_t pos, face, orig;
};

struct Tally {
    uint32_t nodes, tris;
};

constexpr int kShortStack = 16;  // LDS stack entries per lane without an LDS plan

// Closest hit (ANY = false: smallest t; equal t -> lower face id -> lower
// input index) or any hit (ANY = true) of the ray o + t d, t_lo < t < t_hi,
// ignoring triangles of faces xa and xb.  Returns the leaf-order position of
// the hit or -1.  LDS = false reads everything from global memory (no LDS
// plan needed) and keeps the top of the stack in a static LDS array.
template <bool ANY, bool COUNT, bool LDS, int BLK = 256>
__device__ static int32_t traverse(const SceneDev& S, const LdsPlan& L, d3 o, d3 d, int32_t xa,
                                   int32_t xb, double t_lo, double t_hi, float delta, HitRec* h,
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
        float4 a, b, c, mf;
        if (LDS && node < L.n_nodes) {
            const float4* np = g_smem4 + 4 * node;
            a = np[0]; b = np[1]; c = np[2]; mf = np[3];
        } else {
            const float4* np = (const float4*)(S.nodes + node);
            a = gld(np); b = gld(np + 1); c = gld(np + 2); mf = gld(np + 3);
        }
        const int4 m = __builtin_bit_cast(int4, mf);
        if (COUNT) tally->nodes += 1;
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
                TriD T = tri_at<LDS>(S, L, i);
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
            if (sp < ldepth) lst[sp * bd] = farc;
            else ost[sp - ldepth] = farc;
            ++sp;
            node = nearc;
        } else if (go0) {
            node = m.x;
        } else if (go1) {
            node = m.y;
        } else {
            if (sp == 0) break;
            --sp;
            node = sp < ldepth ? lst[sp * bd] : ost[sp - ldepth];
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

// Can any receiver inside the ball (c, rho) of a receiver-tree node pass the
// reception test of the segment (o, d, D, t)?  For x in the ball, t*(x)
// differs from t*(c) by at most rho |d|, and the distance from x to the ray
// line from that of c by at most rho (x -> (x - o) - ((x - o).d) d has norm 1
// for |d| = 1 + O(eps)).  So a capture needs 0 < t*(c) + rho |d|,
// t*(c) - rho |d| <= t and d_perp(c) <= thl (D + t*(c) + rho |d|) + rho.  The
// radius r used here widens rho by 1e-6 relative and by 1e-9 of the lengths
// involved, far above the rounding of this test or of capture(), so the cull
// never drops a receiver that capture() accepts.
__device__ static inline bool rx_ball_may_capture(d3 o, d3 d, double D, double t, d3 c,
                                                  double rho, double thl)
{
    d3 v = sub(c, o);
    double tc = dot(v, d);
    double r = rho * (1.0 + 1e-6) + 1e-9 * (D + (fabs(v.x) + fabs(v.y) + fabs(v.z)));
    if (tc + r <= 0.0) return false;
    if (tc - r > t) return false;
    d3 w = sub(v, scl(tc, d));
    double A = thl * (D + tc + r) + r;
    return dot(w, w) <= A * A;
}

struct Follow {
    double tan_err, D, Llast;
};

// Trace direction d0 from Tx through exactly the faces of a path of order k
// and report the error angle of Rx on the last segment (no cone condition).
// A sub-ray is a usable path only if it meets the same faces in the same
// order and Rx lies ahead on its last segment before the next obstacle.
// With pts/din non-NULL the reflection points and incoming directions are
// stored.
template <bool LDS, int BLK = 256>
__device__ static bool follow(const SceneDev& S, const LdsPlan& L, d3 tx, d3 d0, d3 rx, int k,
                              const int32_t* faces, float delta, Follow* F, d3* pts, d3* din,
                              int32_t* err)
{
    d3 o = tx, d = d0;
    double D = 0.0;
    int32_t prev = -1;
    for (int j = 0;; ++j) {
        HitRec h;
        int32_t hit =
            traverse<false, false, LDS, BLK>(S, L, o, d, prev, prev, S.t_eps, INFINITY, delta, &h,
                                             err);
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

}  // namespace sbr
