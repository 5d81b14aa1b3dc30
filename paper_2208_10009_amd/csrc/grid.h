// grid.h -- the equiangular launch grid's data in the setup scratch and the
// direction of one ray from it (Sec. II.B, eqs. (1)-(2)), shared by the grid
// kernels (launch.hip) and by the trace, which forms the directions of its
// rays itself while the ring setup runs beside it.  Every value is
// bit-identical to the correctly rounded FP64 grid (geom.h holds the
// double-double trigonometry).
#pragma once
#include <math.h>
#include <stdint.h>

#include "geom.h"
#include "grid_layout.h"

namespace sbr {

// Accept v (a normalized double-double, |v - exact| <= e) when both ends of
// [v - 2e, v + 2e] round to v.hi + v.lo.  The factor 2 covers the rounding of
// v.lo +- 2e, given e >= 2^-100 |v|.
__device__ static inline bool rounds_safely(dd v, double e)
{
    const double r = v.hi + v.lo, e2 = 2.0 * e;
    return v.hi + (v.lo + e2) == r && v.hi + (v.lo - e2) == r;
}

// Coefficients of one lane's series, chosen once per lane: the double-double
// series of cos (role 0) or sin (roles 1, 2), and the double series of the
// other function.
struct LaneSeries {
    dd head[5];       // 1/k! for the first five terms of the double-double series
    double tail[9];   // 1/k! for the next nine terms
    double e_tail, e_trunc;  // 1/k! of the first tail term and of the first omitted term
    double other[11]; // 1/k! of the double series
    bool cosine;
};

// The series coefficients 1/k! (kInvFact).  A caller whose loop must not
// keep them in registers (the trace) passes a pointer it has made opaque to
// the compiler, so that they are loaded where used rather than hoisted.
typedef const __attribute__((address_space(4))) dd* CoefPtr;

__device__ static inline CoefPtr coef_table() { return (CoefPtr)kInvFact; }

__device__ static inline dd coef(CoefPtr F, int k) { return dd{F[k].hi, F[k].lo}; }

__device__ static LaneSeries lane_series(bool cosine, CoefPtr F = coef_table())
{
    const int o = cosine ? 0 : 1;
    LaneSeries L;
    L.cosine = cosine;
#pragma unroll
    for (int k = 0; k < 5; ++k) L.head[k] = cosine ? coef(F, 2 * k) : coef(F, 2 * k + 1);
#pragma unroll
    for (int j = 0; j < 9; ++j) L.tail[j] = cosine ? F[2 * j + 10].hi : F[2 * j + 11].hi;
    L.e_tail = F[10 + o].hi;
    L.e_trunc = F[28 + o].hi;
#pragma unroll
    for (int k = 0; k < 11; ++k) L.other[k] = cosine ? F[2 * k + 1].hi : F[2 * k].hi;
    return L;
}

// Short series for 0 <= y <= 1.2: cos y (cosine lanes) or sin y with the terms up to y^8/8! (y^9/9!) in double-double (Horner's
// rule in t = y^2, exact as two_prod(y, y)) and the next nine terms in
// double, folded into the innermost coefficient.  *err bounds the error: the
// double-double steps (< 2^-100 relative to values below 1), the double tail
// (relative error below 5 ulp; 2^-47 t^5/10! (/11!) is 16 times that), and
// the omitted terms (alternating and decreasing: below t^14/28! (y t^14/29!)).
// *other is the other function in double (Taylor series to y^20/20!
// (y^21/21!), about 1e-16 relative).
__device__ static dd series_fast(const LaneSeries& L, double y, double* err, double* other)
{
    const double ym = L.cosine ? 1.0 : y;
    const dd t = two_prod(y, y);
    const double td = t.hi;
    double q = L.tail[8];
#pragma unroll
    for (int j = 7; j >= 0; --j) q = fma(-td, q, L.tail[j]);
    dd h = dd_sub(L.head[4], dd{td * q, 0.0});
#pragma unroll
    for (int k = 3; k >= 0; --k) h = dd_sub(L.head[k], dd_mul(t, h));
    const double t2 = td * td, t4 = t2 * t2, t5 = t4 * td, t14 = t4 * t4 * t4 * t2;
    *err = ym * (0x1p-96 + 0x1p-47 * t5 * L.e_tail + t14 * L.e_trunc);
    double p = L.other[10];
#pragma unroll
    for (int k = 9; k >= 0; --k) p = fma(-td, p, L.other[k]);
    *other = L.cosine ? y * p : p;
    return dd_mul(dd{ym, 0.0}, h);
}

// Correctly rounded sin y for 0 <= y <= 1.2: the short series of the grid
// setup when its error bound (times scale >= 1) proves the rounding (all but
// about two values in a million), else the full double-double series.
__device__ static double sin_rounded(double y, double scale, CoefPtr F = coef_table())
{
    const LaneSeries L = lane_series(false, F);
    double err, c;
    const dd s = series_fast(L, y, &err, &c);
    if (y <= 1.2 && rounds_safely(s, err * scale)) return s.hi + s.lo;
    // sin_cr (geom.h) with the coefficients read through F: the same
    // operations in the same order
    const dd f = dd{y, 0.0}, t = dd_mul(f, f);
    dd b[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) b[j] = dd_sub(coef(F, 4 * j + 1), dd_mul(coef(F, 4 * j + 3), t));
    const dd t2 = dd_mul(t, t);
    const dd c0 = dd_add(b[0], dd_mul(b[1], t2)), c1 = dd_add(b[2], dd_mul(b[3], t2));
    const dd c2 = dd_add(b[4], dd_mul(b[5], t2)), c3 = dd_add(b[6], dd_mul(b[7], t2));
    const dd t4 = dd_mul(t2, t2);
    const dd d0 = dd_add(c0, dd_mul(c1, t4)), d1 = dd_add(c2, dd_mul(c3, t4));
    const dd t8 = dd_mul(t4, t4);
    const dd e0 = dd_add(d0, dd_mul(d1, t8));
    const dd t16 = dd_mul(t8, t8);
    const dd r = dd_mul(f, dd_add(e0, dd_mul(b[8], t16)));
    return r.hi + r.lo;
}

// Point k of m equal-angle steps from P to Q along their great circle, th
// being the angle P and Q subtend (acos_cr(P.Q)): the angles subtended at
// the centre by consecutive points are equal (eq. (1)).  Direction
// sin((m-k) th/m) P + sin(k th/m) Q, normalized.
__device__ static d3 arc_point_th(d3 P, d3 Q, double th, int64_t k, int64_t m, double scale,
                                 CoefPtr F = coef_table())
{
    double a = ((double)k * th) / (double)m;
    double b = ((double)(m - k) * th) / (double)m;
    double sa = sin_rounded(a, scale, F), sb = sin_rounded(b, scale, F);
    return normalize(add(scl(sb, P), scl(sa, Q)));
}

// How the direction of a ray reads the setup's data: plain loads when the
// setup kernel has completed before (k_grid_dirs), device-scope relaxed
// atomic loads while it may still run on another stream (the trace, after
// the setup has published the layers the ray needs; its stores are atomic
// too and precede the publication by a release fence).
struct GridPlainLoads {
    __device__ static double f64(const double* p) { return *p; }
    __device__ static int32_t i32(const int32_t* p) { return *p; }
};

struct GridAtomicLoads {
    __device__ static double f64(const double* p)
    {
        return __longlong_as_double((long long)__hip_atomic_load(
            (const unsigned long long*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
    __device__ static int32_t i32(const int32_t* p)
    {
        return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
};

template <class LD>
__device__ static inline d3 grid_ld3(const d3* p)
{
    const double* q = (const double*)p;
    return mk(LD::f64(q), LD::f64(q + 1), LD::f64(q + 2));
}

// Ray order: the 12 vertex rays; then edge interiors, edge by edge, steps
// 1..n-1 from the lower to the higher vertex index; then face interiors, face
// by face, layer by layer, each ring starting at the corner that descends
// from the face's first vertex and following the winding.  n <= 10000, so
// every index fits in 32 bits.
template <class LD>
__device__ static inline d3 grid_dir_of(int32_t n, const char* scratch, uint32_t i, double scale,
                                       CoefPtr F = coef_table())
{
    const GridHdr* H = (const GridHdr*)scratch;
    const d3* rings = (const d3*)(scratch + sizeof(GridHdr));
    const double* ths = side_angles((char*)scratch, n);
    const uint32_t un = (uint32_t)n;
    uint32_t idx = i;
    if (idx < 12) return grid_ld3<LD>(&H->V[idx]);
    idx -= 12;
    if (idx < 30 * (un - 1)) {
        const uint32_t e = idx / (un - 1), k = idx % (un - 1) + 1;
        const d3 P = grid_ld3<LD>(&H->V[LD::i32(&H->e[e][0])]);
        const d3 Q = grid_ld3<LD>(&H->V[LD::i32(&H->e[e][1])]);
        return arc_point_th(P, Q, LD::f64(ths + edge_angle_index(n) + e), k, n, scale, F);
    }
    idx -= 30 * (un - 1);
    const uint32_t per_face = (un - 1) * (un - 2) / 2;
    const uint32_t f = idx / per_face;
    const int64_t q = idx % per_face;
    const int64_t c1 = 3 * (int64_t)(n - 3);
    const int64_t a = ring_of(n, q);
    const int64_t m = n - 3 - 3 * a;
    const uint32_t qq = (uint32_t)(q - (a * c1 - 9 * a * (a - 1) / 2));
    const d3* W = rings + (size_t)f * 3 * ring_cap(n) + 3 * a;
    if (m == 0) return grid_ld3<LD>(&W[0]);
    const uint32_t s = qq / (uint32_t)m, k = qq % (uint32_t)m;
    if (k == 0) return grid_ld3<LD>(&W[s]);
    return arc_point_th(grid_ld3<LD>(&W[s]), grid_ld3<LD>(&W[(s + 1) % 3]),
                        LD::f64(ths + (size_t)f * 3 * ring_cap(n) + 3 * a + s), k, m, scale, F);
}

}  // namespace sbr
