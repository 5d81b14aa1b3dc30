// follow.h -- following a path's face sequence with a sub-ray, for the
// precise algorithm (Sec. III.B) and the solve: sequentially (follow) or with
// the segments spread over lanes (seg_lane).
#pragma once
#include "traverse.h"

namespace sbr {

struct Follow {
    double tan_err, D, Llast;
};

// faces[j] of a face sequence without a dynamic index, which would place the
// caller's list in private memory.
__device__ static inline int32_t face_at(const int32_t* faces, int j)
{
    // every load has a constant index; selecting values (not addresses)
    // lets the list stay in registers
    int32_t f = 0;
#pragma unroll
    for (int q = 0; q < SBR_MAX_ORDER; ++q) f |= q == j ? faces[q] : 0;
    return f;
}

// The last segment of a sub-ray (origin o after the path's reflections):
// Rx is captured when its foot t* = (Rx - o).d satisfies 0 < t* <= t for the
// segment's closest hit t.  That holds exactly when no triangle is hit in
// (t_eps, t*): the closest hit is then at t* or beyond (a hit exactly at t*
// lies outside the open range and passes, as t* <= t does), and a hit inside
// the range makes the closest one fall short.  So the last segment's search
// is bounded by t* instead of running along the whole ray, and the capture
// test then takes t = infinity.  last_bound gives t* (false: Rx is behind).
__device__ static inline bool last_bound(d3 o, d3 d, d3 rx, double* ts)
{
    *ts = dot(sub(rx, o), d);
    return *ts > 0.0;
}

__device__ static inline bool last_capture(d3 o, d3 d, double D, d3 rx, Follow* F)
{
    double tn;
    if (!capture(o, d, D, INFINITY, rx, -1.0, &tn)) return false;
    F->tan_err = tn;
    F->D = D;
    F->Llast = norm(sub(rx, o));
    return true;
}

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
        h.pos = -1;
        h.t = INFINITY;
        h.face = 0x7fffffff;
        h.orig = 0x7fffffff;
        if (j < k) {
            // seed with the closest hit on the face the path expects next:
            // it bounds the search from the start
            const int32_t fe = face_at(faces, j);
            if (fe != prev)
                for (int32_t q = S.fstart[fe]; q < S.fstart[fe + 1]; ++q) {
                    const int32_t i = S.ftris[q];
                    const TriD T = tri_at<LDS>(S, L, i);
                    double t;
                    if (!mt_hit(T, o, d, S.t_eps, INFINITY, &t)) continue;
                    if (h.pos < 0 || t < h.t ||
                        (t == h.t && (T.face < h.face || (T.face == h.face && T.orig < h.orig)))) {
                        h.pos = i;
                        h.t = t;
                        h.face = T.face;
                        h.orig = T.orig;
                    }
                }
        }
        double thi = INFINITY;
        if (j == k && !last_bound(o, d, rx, &thi)) return false;
        int32_t hit = traverse<false, false, LDS, BLK>(S, L, o, d, prev, prev, S.t_eps, thi,
                                                       delta, &h, err, nullptr, j < k);
        if (j == k) return hit < 0 && last_capture(o, d, D, rx, F);
        if (hit < 0 || h.face != face_at(faces, j)) return false;
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

// Triangle i read at a wave-uniform index: from LDS when staged, else
// through the constant address space, so that the compiler issues scalar
// loads (the scene is never written while a kernel reads it).
template <bool LDS>
__device__ static inline TriD tri_uniform(const SceneDev& S, const LdsPlan& L, int32_t i)
{
    if (LDS && i < L.n_tris) return tri_at<LDS>(S, L, i);
    typedef const __attribute__((address_space(4))) d2v* cp;
    const cp q = (cp)(S.tris + i);
    auto g = [](d2v v) { return make_double2(v.x, v.y); };
    return make_tri(g(q[0]), g(q[1]), g(q[2]), g(q[3]), g(q[4]));
}

__device__ static inline int32_t ild_uniform(const int32_t* p)
{
    return *(const __attribute__((address_space(4))) int32_t*)p;
}

// One lane's share of follow() with the segments of a sub-ray spread over
// lanes: lane j (0 <= j <= k) checks segment j only.  The segments before it
// are stepped through with the closest hit on each expected face, which is
// the hit follow() seeds its search with and, whenever that segment passes,
// the hit it then reflects at; so lane j starts segment j exactly where
// follow() would and runs the same search.  Segment j < k passes when its
// search ends on the expected face (the reflection point and incoming
// direction go to pt and din), segment k when Rx is captured before the next
// obstacle (F as follow()).  follow() succeeds exactly when every lane of the
// sub-ray does, with the same F and geometry.  faces and k must be uniform
// over the wave (the face data are then read with scalar loads).
template <bool LDS, int BLK = 256>
__device__ static bool seg_lane(const SceneDev& S, const LdsPlan& L, d3 tx, d3 d0, d3 rx, int k,
                                int j, const int32_t* faces, float delta, Follow* F, d3* pt,
                                d3* din, int32_t* err)
{
    d3 o = tx, d = d0;
    double D = 0.0;
    int32_t prev = -1;
    HitRec h;
    h.pos = -1;
    h.t = INFINITY;
    h.face = 0x7fffffff;
    h.orig = 0x7fffffff;
    for (int jj = 0; jj < k; ++jj) {
        // closest hit on the face expected at segment jj
        const int32_t fe = face_at(faces, jj);
        if (fe == prev) return false;  // follow() cannot meet fe there
        h.pos = -1;
        h.t = INFINITY;
        h.face = 0x7fffffff;
        h.orig = 0x7fffffff;
        const int32_t q1 = ild_uniform(S.fstart + fe + 1);
        for (int32_t q = ild_uniform(S.fstart + fe); q < q1; ++q) {
            const int32_t i = ild_uniform(S.ftris + q);
            const TriD T = tri_uniform<LDS>(S, L, i);
            double t;
            if (!mt_hit(T, o, d, S.t_eps, INFINITY, &t)) continue;
            if (h.pos < 0 || t < h.t ||
                (t == h.t && (T.face < h.face || (T.face == h.face && T.orig < h.orig)))) {
                h.pos = i;
                h.t = t;
                h.face = T.face;
                h.orig = T.orig;
            }
        }
        if (h.pos < 0) return false;  // no triangle of fe ahead: follow() fails
        if (jj == j) break;
        d3 nf = face_normal(S, fe);
        d3 on = add(o, scl(h.t, d));
        double k2 = 2.0 * dot(d, nf);
        d = sub(d, scl(k2, nf));
        D = D + h.t;
        o = on;
        prev = fe;
    }
    double thi = INFINITY;
    if (j == k) {
        if (!last_bound(o, d, rx, &thi)) return false;
        h.pos = -1;
        h.t = INFINITY;
        h.face = 0x7fffffff;
        h.orig = 0x7fffffff;
    }
    const int32_t hit = traverse<false, false, LDS, BLK>(S, L, o, d, prev, prev, S.t_eps, thi,
                                                         delta, &h, err, nullptr, j < k);
    if (j == k) return hit < 0 && last_capture(o, d, D, rx, F);
    if (hit < 0 || h.face != face_at(faces, j)) return false;
    *pt = add(o, scl(h.t, d));
    *din = d;
    return true;
}

}  // namespace sbr
