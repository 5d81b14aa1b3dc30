// diffract.hip -- order-1 diffraction (Sec. III.A: paths through faces or
// wedges; Sec. III.B: sub-rays diffracted in the recorded direction; Sec. IV:
// order-1 diffraction paths).
//
// A path Tx -> Q -> Rx with Q on a wedge's edge makes equal angles with the
// edge on both sides (Keller's law).  Rotating Rx about the edge line into the
// half-plane opposite Tx unfolds it into the straight line Tx -> Rx'; the
// angle between a ray and Rx' - Tx is that ray's departure-angle error, the
// diffraction form of eq. (3).  SBR: a launch ray diffracts at a wedge when
// its closest approach to the edge lies on the segment, in front of Tx, inside
// the ray cone and before the ray's first hit (or on one of the wedge's own
// faces, which a ray clipping the edge meets there); it reaches the receivers
// outside the wedge whose unfolded images lie inside the cone.  The precise
// algorithm runs the sub-ray cones of the reflection paths, each sub-ray
// diffracted at the same wedge toward the same receiver.
#include <math.h>

#include <algorithm>
#include <vector>

#include "cone.h"
#include "diffract.h"
#include "traverse.h"

namespace sbr {

// ===========================================================================
// Host: wedge extraction
// ===========================================================================
namespace {

// cos(10 deg), nearest binary64: faces meeting at a smaller angle form no wedge
constexpr double kCosWedge = 0.984807753012208;

struct EdgeRec {
    double lo[3], hi[3], c[3];  // endpoints (lo < hi lexicographically), third vertex
    int32_t face;
    int64_t tri;
};

int lex3(const double* p, const double* q)
{
    for (int i = 0; i < 3; ++i)
        if (p[i] != q[i]) return p[i] < q[i] ? -1 : 1;
    return 0;
}

bool edge_less(const EdgeRec& a, const EdgeRec& b)
{
    int c = lex3(a.lo, b.lo);
    if (c) return c < 0;
    c = lex3(a.hi, b.hi);
    if (c) return c < 0;
    if (a.face != b.face) return a.face < b.face;
    return a.tri < b.tri;
}

// unit vector in a face's plane, normal to the edge (a, e), toward vertex c
d3 in_face_dir(d3 a, d3 e, d3 c)
{
    d3 w = sub(c, a);
    return normalize(sub(w, scl(dot(w, e), e)));
}

float round_up(double x)
{
    float f = (float)x;
    if ((double)f < x) f = nextafterf(f, INFINITY);
    return f;
}

}  // namespace

void build_wedges(const double* tri_v, const int32_t* face, int64_t T, const double* fplane,
                  std::vector<WedgeDev>& out, std::vector<double>& b_out)
{
    out.clear();
    b_out.clear();
    std::vector<EdgeRec> E;
    E.reserve((size_t)(3 * T));
    for (int64_t i = 0; i < T; ++i)
        for (int k = 0; k < 3; ++k) {
            const double* p = tri_v + 9 * i + 3 * k;
            const double* q = tri_v + 9 * i + 3 * ((k + 1) % 3);
            const double* c = tri_v + 9 * i + 3 * ((k + 2) % 3);
            const int o = lex3(p, q);
            if (o == 0) continue;
            EdgeRec r;
            for (int j = 0; j < 3; ++j) {
                r.lo[j] = o < 0 ? p[j] : q[j];
                r.hi[j] = o < 0 ? q[j] : p[j];
                r.c[j] = c[j];
            }
            r.face = face[i];
            r.tri = i;
            E.push_back(r);
        }
    std::sort(E.begin(), E.end(), edge_less);
    for (size_t i = 0; i < E.size();) {
        size_t j = i;
        while (j < E.size() && lex3(E[j].lo, E[i].lo) == 0 && lex3(E[j].hi, E[i].hi) == 0) ++j;
        // records i..j-1 share the edge, by face then triangle: the first
        // record of each face is its lowest-index triangle on the edge
        size_t first[2] = {0, 0};
        int nf = 0;
        for (size_t q = i; q < j; ++q)
            if (q == i || E[q].face != E[q - 1].face) {
                if (nf < 2) first[nf] = q;
                ++nf;
            }
        if (nf == 2) {
            const EdgeRec &r0 = E[first[0]], &r1 = E[first[1]];
            const d3 n0 = ld3(fplane + 4 * (size_t)r0.face), n1 = ld3(fplane + 4 * (size_t)r1.face);
            if (fabs(dot(n0, n1)) <= kCosWedge) {
                WedgeDev w;
                const d3 a = ld3(r0.lo), b = ld3(r0.hi);
                const d3 d = sub(b, a);
                const double len = norm(d);
                const d3 e = mk(d.x / len, d.y / len, d.z / len);
                st3(w.a, a);
                st3(w.e, e);
                st3(w.u0, in_face_dir(a, e, ld3(r0.c)));
                st3(w.u1, in_face_dir(a, e, ld3(r1.c)));
                w.len = len;
                w.f0 = r0.face;
                w.f1 = r1.face;
                // bounding sphere of the segment in FP32: the centre rounded
                // to nearest moves it by at most 2^-24 of its coordinates,
                // which the radius absorbs with the relative slack
                const d3 m = add(a, scl(0.5, d));
                double cm = std::max(fabs(m.x), std::max(fabs(m.y), fabs(m.z)));
                w.c[0] = (float)m.x;
                w.c[1] = (float)m.y;
                w.c[2] = (float)m.z;
                w.r = round_up((0.5 * len) * (1.0 + 1e-6) + 1e-6 * cm);
                out.push_back(w);
                for (int q = 0; q < 3; ++q) b_out.push_back(r0.hi[q]);
            }
        }
        i = j;
    }
}

// ===========================================================================
// Device
// ===========================================================================
struct WedgeGeo {
    d3 a, e, u0, u1;
    double len;
    int32_t f0, f1;
};

__device__ static inline WedgeGeo wedge_at(const WedgeDev* __restrict__ w, int32_t k)
{
    const WedgeDev& W = w[k];
    WedgeGeo g;
    g.a = mk(W.a[0], W.a[1], W.a[2]);
    g.e = mk(W.e[0], W.e[1], W.e[2]);
    g.u0 = mk(W.u0[0], W.u0[1], W.u0[2]);
    g.u1 = mk(W.u1[0], W.u1[1], W.u1[2]);
    g.len = W.len;
    g.f0 = W.f0;
    g.f1 = W.f1;
    return g;
}

// Inside the wedge: strictly between its faces, where both faces lie (the
// part of P - a normal to the edge is b u0 + c u1 with b > 0 and c > 0).
__device__ static inline bool wedge_interior(const WedgeGeo& W, d3 P)
{
    d3 v = sub(P, W.a);
    d3 r = sub(v, scl(dot(v, W.e), W.e));
    double g = dot(W.u0, W.u1);
    double r0 = dot(r, W.u0), r1 = dot(r, W.u1);
    return (r0 - g * r1 > 0.0) && (r1 - g * r0 > 0.0);
}

// Closest approach of the ray o + t d and the edge line a + s e; false when
// the lines are (nearly) parallel.
__device__ static inline bool ray_edge(const WedgeGeo& W, d3 o, d3 d, double* t, double* s)
{
    d3 w0 = sub(o, W.a);
    double b = dot(d, W.e), dd = dot(d, d), ee = dot(W.e, W.e);
    double dw = dot(d, w0), ew = dot(W.e, w0);
    double den = dd * ee - b * b;
    if (!(den > 1e-12)) return false;
    *t = (b * ew - ee * dw) / den;
    *s = (dd * ew - b * dw) / den;
    return true;
}

// The ray passes the segment (closest approach at t > 0, 0 <= s <= len) and
// reaches it: its first hit (th on face fh; fh = -1: none) is beyond t or on
// one of the wedge's faces.
__device__ static inline bool reaches_edge(const WedgeGeo& W, d3 o, d3 d, double th, int32_t fh,
                                           double* t, double* s)
{
    if (!ray_edge(W, o, d, t, s)) return false;
    if (!(*t > 0.0) || !(*s >= 0.0) || !(*s <= W.len)) return false;
    if (fh >= 0 && !(th >= *t) && fh != W.f0 && fh != W.f1) return false;
    return true;
}

// The unfolded receiver rxp seen from the ray from tx along d (eq. (3) with
// D = 0): foot parameter ts, perpendicular distance dp, tan(error angle)
// dp / ts; false when rxp is not ahead.
__device__ static inline bool unfolded_tan(d3 tx, d3 d, d3 rxp, double* tan_out, double* ts_out,
                                           double* dp_out)
{
    d3 w = sub(rxp, tx);
    double ts = dot(w, d);
    if (!(ts > 0.0)) return false;
    d3 f = sub(w, scl(ts, d));
    double dp = norm(f);
    *tan_out = dp / ts;
    *ts_out = ts;
    *dp_out = dp;
    return true;
}

__global__ void k_diff_unfold(DiffArgs A)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)A.n_w * A.n_rx) return;
    const int32_t k = (int32_t)(i / A.n_rx), x = (int32_t)(i % A.n_rx);
    const WedgeGeo W = wedge_at(A.w, k);
    const d3 rx = mk(A.rx[3 * x], A.rx[3 * x + 1], A.rx[3 * x + 2]);
    const d3 tx = mk(A.tx[0], A.tx[1], A.tx[2]);
    double4 out = make_double4(0.0, 0.0, 0.0, 0.0);
    if (!wedge_interior(W, rx)) {
        d3 vx = sub(rx, W.a), vt = sub(tx, W.a);
        double ax = dot(vx, W.e), at = dot(vt, W.e);
        d3 rxv = sub(vx, scl(ax, W.e)), rtv = sub(vt, scl(at, W.e));
        double rho_x = norm(rxv), rho_t = norm(rtv);
        if (rho_t > 0.0 && rho_x > 0.0) {
            double kk = rho_x / rho_t;
            d3 p = sub(add(W.a, scl(ax, W.e)), scl(kk, rtv));
            out = make_double4(p.x, p.y, p.z, 1.0);
        }
    }
    A.rxp[i] = out;
}

hipError_t launch_diff_unfold(const DiffArgs& A, hipStream_t s)
{
    const int64_t n = (int64_t)A.n_w * A.n_rx;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_diff_unfold, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A);
    return hipGetLastError();
}

// Conservative FP32 cull of a wedge for one ray: false only when no point of
// the segment's bounding sphere (centre c, radius r) can have its closest
// approach inside the ray's cone in front of Tx.  A diffraction event needs
// an edge point Q with |Q - c| <= r at distance at most thl t from the ray
// line, t = (Q - o).d <= t_c + r, so the centre is within thl (t_c + r) + r
// of the line and t_c > -r.  The FP32 foot parameter and perpendicular of
// the centre err by less than dl = 2^-18 (max |o| + max |c|) (as in the
// receiver pre-test), covered below with the factors 1 + 2^-20 on thl and
// 1 + 2^-18 on the squared bound; NaN never rejects.
__device__ static inline bool wedge_may32(float ox, float oy, float oz, float dx, float dy,
                                          float dz, float thl, float dlo, float4 c)
{
    const float vx = c.x - ox, vy = c.y - oy, vz = c.z - oz;
    const float cm = fmaxf(fmaxf(fabsf(c.x), fabsf(c.y)), fabsf(c.z));
    const float dl = fmaf(0x1p-18f, cm, dlo);
    const float tc = fmaf(vz, dz, fmaf(vy, dy, vx * dx));
    if (tc + dl + c.w <= 0.0f) return false;
    const float wx = fmaf(-tc, dx, vx), wy = fmaf(-tc, dy, vy), wz = fmaf(-tc, dz, vz);
    const float ww = fmaf(wz, wz, fmaf(wy, wy, wx * wx));
    const float A = fmaf(thl, (tc + c.w) + dl, dl + c.w);
    return !(ww > (A * A) * (1.0f + 0x1p-18f));
}

__global__ __launch_bounds__(256) void k_diff_trace(SceneDev S, DiffArgs A,
                                                    sbr_candidate* __restrict__ cand, int64_t cap,
                                                    unsigned long long* __restrict__ count,
                                                    int32_t* __restrict__ err)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= A.N) return;
    const d3 tx = mk(A.tx[0], A.tx[1], A.tx[2]);
    const d3 d = mk(A.dir[r], A.dir[A.N + r], A.dir[2 * A.N + r]);
    LdsPlan L0{};
    L0.block = 256;
    HitRec h;
    const int32_t hit = traverse<false, false, false>(S, L0, tx, d, -1, -1, S.t_eps, INFINITY,
                                                      A.delta, &h, err);
    const double th = hit < 0 ? INFINITY : h.t;
    const int32_t fh = hit < 0 ? -1 : h.face;
    const float ox = (float)tx.x, oy = (float)tx.y, oz = (float)tx.z;
    const float dx = (float)d.x, dy = (float)d.y, dz = (float)d.z;
    const float thl32 = (float)A.thl * (1.0f + 0x1p-20f);
    const float dlo = 0x1p-18f * fmaxf(fmaxf(fabsf(ox), fabsf(oy)), fabsf(oz));
    for (int32_t k = 0; k < A.n_w; ++k) {
        // the sphere through the scalar cache (the same for every lane)
        const float4 c = cld4((const float4*)A.w[k].c);
        if (!wedge_may32(ox, oy, oz, dx, dy, dz, thl32, dlo, c)) continue;
        const WedgeGeo W = wedge_at(A.w, k);
        double t, s;
        if (!reaches_edge(W, tx, d, th, fh, &t, &s)) continue;
        const d3 p = add(tx, scl(t, d));
        const d3 q = add(W.a, scl(s, W.e));
        if (!(norm(sub(p, q)) <= A.thl * t)) continue;
        for (int32_t x = 0; x < A.n_rx; ++x) {
            const double4 rp = A.rxp[(int64_t)k * A.n_rx + x];
            if (rp.w == 0.0) continue;
            double tn, ts, dp;
            if (!unfolded_tan(tx, d, mk(rp.x, rp.y, rp.z), &tn, &ts, &dp)) continue;
            if (!(dp <= A.thl * ts)) continue;  // inside the cone: d_perp <= thl t*
            const unsigned long long pos = atomicAdd(count, 1ull);
            if ((int64_t)pos < cap) {
                sbr_candidate c2;
                c2.rx = x;
                c2.order = 1;
                c2.face[0] = k;
#pragma unroll
                for (int j = 1; j < SBR_MAX_ORDER; ++j) c2.face[j] = -1;
                c2.ray = r;
                c2.tan_err = tn;
                cand[pos] = c2;
            }
        }
    }
}

hipError_t launch_diff_trace(const SceneDev& S, const DiffArgs& A, sbr_candidate* cand,
                             int64_t cap, unsigned long long* count, int32_t* err,
                             hipStream_t s)
{
    if (A.N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_diff_trace, dim3((unsigned)((A.N + 255) / 256)), dim3(256), 0, s, S, A,
                       cand, cap, count, err);
    return hipGetLastError();
}

// One sub-ray of a diffraction path: whether direction d passes and reaches
// the wedge (closest hit traced from Tx), and its error angle and legs.
__device__ static bool follow_diff(const SceneDev& S, const WedgeGeo& W, d3 tx, d3 d, d3 rx,
                                   d3 rxp, float delta, int32_t* err, double* tan, double* L1,
                                   double* L2)
{
    LdsPlan L0{};
    L0.block = 256;
    HitRec h;
    const int32_t hit = traverse<false, false, false>(S, L0, tx, d, -1, -1, S.t_eps, INFINITY,
                                                      delta, &h, err);
    double t, s, ts, dp;
    if (!reaches_edge(W, tx, d, hit < 0 ? INFINITY : h.t, hit < 0 ? -1 : h.face, &t, &s))
        return false;
    if (!unfolded_tan(tx, d, rxp, tan, &ts, &dp)) return false;
    const d3 q = add(W.a, scl(s, W.e));
    *L1 = norm(sub(q, tx));
    *L2 = norm(sub(rx, q));
    return true;
}

// Eight lanes per path: lane s traces sub-ray s (s < subrays); the group
// keeps the smallest error angle (ties: lower s) as the next axis.
__global__ __launch_bounds__(256) void k_diff_refine(SceneDev S, DiffArgs A,
                                                     const sbr_candidate* __restrict__ uniq,
                                                     int64_t U, RefineOut* __restrict__ out,
                                                     int32_t* __restrict__ err)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = gid >> 3;
    const int s = (int)(gid & 7);
    if (p >= U) return;
    const sbr_candidate c = uniq[p];
    const int32_t k = c.face[0];
    const WedgeGeo W = wedge_at(A.w, k);
    const d3 tx = mk(A.tx[0], A.tx[1], A.tx[2]);
    const d3 rx = mk(A.rx[3 * c.rx], A.rx[3 * c.rx + 1], A.rx[3 * c.rx + 2]);
    const double4 rp = A.rxp[(int64_t)k * A.n_rx + c.rx];
    const d3 rxp = mk(rp.x, rp.y, rp.z);
    d3 axis = mk(A.dir[c.ray], A.dir[A.N + c.ray], A.dir[2 * A.N + c.ray]);
    double tan, L1, L2;
    if (rp.w == 0.0 || !follow_diff(S, W, tx, axis, rx, rxp, A.delta, err, &tan, &L1, &L2)) {
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
    bool met = A.tan_tgt > 0.0 && target_met(tan, A.tan_tgt, L1, L2);
    uint32_t flags = met ? SBR_PATH_TARGET_MET : 0u;
    int32_t iters = 0;
    double rho = A.thl;
    for (int i = 1; i <= A.iterations && !met; ++i) {
        rho = rho / sqrt(3.0);
        d3 u, v;
        basis(axis, &u, &v);
        double mt = INFINITY, m1 = 0.0, m2 = 0.0;
        bool ok = false;
        if (s < A.subrays)
            ok = follow_diff(S, W, tx, subray(axis, u, v, rho, s), rx, rxp, A.delta, err, &mt,
                             &m1, &m2);
        double bt = ok ? mt : INFINITY;
        int bs = ok ? s : 8;
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
        const double w1 = __shfl(m1, bs, 8), w2 = __shfl(m2, bs, 8);
        axis = subray(axis, u, v, rho, bs);
        tan = bt;
        iters = i;
        if (A.tan_tgt > 0.0 && target_met(bt, A.tan_tgt, w1, w2)) {
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

hipError_t launch_diff_refine(const SceneDev& S, const DiffArgs& A, const sbr_candidate* uniq,
                              int64_t U, RefineOut* out, int32_t* err, hipStream_t s)
{
    if (U <= 0) return hipSuccess;
    const int64_t threads = 8 * U;
    hipLaunchKernelGGL(k_diff_refine, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, S,
                       A, uniq, U, out, err);
    return hipGetLastError();
}

// Segment P0 -> P1 blocked by a triangle not of faces fa / fb, hit strictly
// inside (1e-9, 1 - 1e-9) of the segment parameter.
__device__ static bool seg_blocked(const SceneDev& S, d3 P0, d3 P1, int32_t fa, int32_t fb,
                                   float delta, int32_t* err)
{
    LdsPlan L0{};
    L0.block = 256;
    HitRec h;
    return traverse<true, false, false>(S, L0, P0, sub(P1, P0), fa, fb, 1e-9, 1.0 - 1e-9, delta,
                                        &h, err) >= 0;
}

// One lane per path: the refined path Tx -> (edge point nearest the final
// ray) -> Rx, the exact path by Keller's law, path test 2.
__global__ __launch_bounds__(256) void k_diff_solve(SceneDev S, DiffArgs A,
                                                    const sbr_candidate* __restrict__ uniq,
                                                    const RefineOut* __restrict__ rf, int64_t U,
                                                    sbr_diff_path* __restrict__ paths,
                                                    int32_t* __restrict__ keep,
                                                    int32_t* __restrict__ err)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= U) return;
    const sbr_candidate c = uniq[p];
    const int32_t k = c.face[0];
    const WedgeGeo W = wedge_at(A.w, k);
    const d3 tx = mk(A.tx[0], A.tx[1], A.tx[2]);
    const d3 rx = mk(A.rx[3 * c.rx], A.rx[3 * c.rx + 1], A.rx[3 * c.rx + 2]);
    const RefineOut R = rf[p];
    const d3 axis = ld3(R.axis);
    sbr_diff_path o;
    o.rx = c.rx;
    o.wedge = k;
    o.launch_ray = c.ray;
    o.iters_used = R.iters;
    o.flags = R.flags;
    o.init_tan_err = c.tan_err;
    o.tan_err = R.tan_err;
    st3(o.axis, axis);
    // refined: the edge point nearest the reported ray
    double t = 0.0, s = 0.0;
    (void)ray_edge(W, tx, axis, &t, &s);
    const d3 q = add(W.a, scl(s, W.e));
    const double L = norm(sub(q, tx)) + norm(sub(rx, q));
    st3(o.point, q);
    o.length_m = L;
    o.delay_s = L / kC0;
    st3(o.aod, axis);
    st3(o.aoa, normalize(sub(q, rx)));
    o.err_angle_deg = atan(R.tan_err) * (180.0 / kPi);
    // exact: s* = at + (ax - at) rho_t / (rho_t + rho_x)
    d3 vx = sub(rx, W.a), vt = sub(tx, W.a);
    double ax = dot(vx, W.e), at = dot(vt, W.e);
    double rho_x = norm(sub(vx, scl(ax, W.e))), rho_t = norm(sub(vt, scl(at, W.e)));
    bool ok = rho_t > 0.0 && rho_x > 0.0;
    d3 qe = W.a;
    if (ok) {
        double se = at + (ax - at) * (rho_t / (rho_t + rho_x));
        qe = add(W.a, scl(se, W.e));
        const double tol = 1e-9 * W.len;
        ok = se >= -tol && se <= W.len + tol && !wedge_interior(W, tx) &&
             !wedge_interior(W, rx) && !seg_blocked(S, tx, qe, W.f0, W.f1, A.delta, err) &&
             !seg_blocked(S, qe, rx, W.f0, W.f1, A.delta, err);
    }
    st3(o.exact_point, qe);
    const double EL = norm(sub(qe, tx)) + norm(sub(rx, qe));
    o.exact_length_m = EL;
    o.exact_delay_s = EL / kC0;
    st3(o.exact_aod, normalize(sub(qe, tx)));
    st3(o.exact_aoa, normalize(sub(qe, rx)));
    if (!ok) o.flags |= SBR_PATH_INVALID;
    paths[p] = o;
    keep[p] = (ok || A.keep_invalid) ? 1 : 0;
}

hipError_t launch_diff_solve(const SceneDev& S, const DiffArgs& A, const sbr_candidate* uniq,
                             const RefineOut* rf, int64_t U, sbr_diff_path* paths,
                             int32_t* keep, int32_t* err, hipStream_t s)
{
    if (U <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_diff_solve, dim3((unsigned)((U + 255) / 256)), dim3(256), 0, s, S, A,
                       uniq, rf, U, paths, keep, err);
    return hipGetLastError();
}

__global__ void k_compact_dpaths(const sbr_diff_path* __restrict__ paths,
                                 const int32_t* __restrict__ keep,
                                 const int32_t* __restrict__ offs, int64_t U,
                                 sbr_diff_path* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < U && keep[i]) out[offs[i]] = paths[i];
}

hipError_t launch_compact_dpaths(const sbr_diff_path* paths, const int32_t* keep,
                                 const int32_t* offs, int64_t U, sbr_diff_path* out,
                                 hipStream_t s)
{
    if (U <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_compact_dpaths, dim3((unsigned)((U + 255) / 256)), dim3(256), 0, s,
                       paths, keep, offs, U, out);
    return hipGetLastError();
}

}  // namespace sbr
