// geom.h -- FP64 vector arithmetic and correctly rounded trigonometry used by
// the launch, trace, capture, refinement and solve kernels.
//
// Every operation is written in a fixed evaluation order and the library is
// compiled with -ffp-contract=off, so each +, -, *, / and sqrt below is one
// IEEE-754 binary64 operation, correctly rounded (gfx950 FP64 division and
// square root are IEEE-exact).  The path set a trace returns is therefore a
// deterministic function of the inputs, independent of thread layout.
//
// The launch grid needs sin and acos.  Hardware libraries return them to
// about one ulp; here they are evaluated in double-double arithmetic (about
// 106 bits) and rounded once, which gives the correctly rounded binary64
// value except when the exact result lies within ~1e-30 (relative) of a
// rounding midpoint.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#define SBR_HD __host__ __device__ __forceinline__

namespace sbr {

struct d3 {
    double x, y, z;
};

SBR_HD d3 mk(double x, double y, double z) { return d3{x, y, z}; }
SBR_HD d3 add(d3 a, d3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
SBR_HD d3 sub(d3 a, d3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
SBR_HD d3 scl(double s, d3 a) { return mk(s * a.x, s * a.y, s * a.z); }
SBR_HD double dot(d3 a, d3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
SBR_HD d3 cross(d3 a, d3 b)
{
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
SBR_HD double norm(d3 a) { return sqrt(dot(a, a)); }
SBR_HD d3 normalize(d3 a)
{
    double r = norm(a);
    return mk(a.x / r, a.y / r, a.z / r);
}
SBR_HD d3 ld3(const double* p) { return mk(p[0], p[1], p[2]); }
SBR_HD void st3(double* p, d3 a)
{
    p[0] = a.x;
    p[1] = a.y;
    p[2] = a.z;
}

// Speed of light (m/s) and the binary64 value nearest to pi.
constexpr double kC0 = 299792458.0;
constexpr double kPi = 3.14159265358979323846;
// atan(2) rounded to the nearest binary64: the angle one icosahedron edge
// subtends at the centre (63.4349 degrees, Sec. III.B).
constexpr double kTheta0 = 1.1071487177940904;

// ---------------------------------------------------------------------------
// double-double arithmetic (Dekker / Knuth error-free transformations)
// ---------------------------------------------------------------------------
struct dd {
    double hi, lo;
};

SBR_HD dd two_sum(double a, double b)
{
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return dd{s, e};
}
SBR_HD dd fast_two_sum(double a, double b)
{
    double s = a + b;
    double e = b - (s - a);
    return dd{s, e};
}
SBR_HD dd two_prod(double a, double b)
{
    double p = a * b;
    double e = fma(a, b, -p);
    return dd{p, e};
}
SBR_HD dd dd_add(dd a, dd b)
{
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo = s.lo + t.hi;
    s = fast_two_sum(s.hi, s.lo);
    s.lo = s.lo + t.lo;
    return fast_two_sum(s.hi, s.lo);
}
SBR_HD dd dd_neg(dd a) { return dd{-a.hi, -a.lo}; }
SBR_HD dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }
SBR_HD dd dd_mul(dd a, dd b)
{
    dd p = two_prod(a.hi, b.hi);
    p.lo = p.lo + (a.hi * b.lo + a.lo * b.hi);
    return fast_two_sum(p.hi, p.lo);
}
SBR_HD dd dd_div(dd a, dd b)
{
    double q1 = a.hi / b.hi;
    dd r = dd_sub(a, dd_mul(dd{q1, 0.0}, b));
    double q2 = r.hi / b.hi;
    r = dd_sub(r, dd_mul(dd{q2, 0.0}, b));
    double q3 = r.hi / b.hi;
    dd q = fast_two_sum(q1, q2);
    return dd_add(q, dd{q3, 0.0});
}

// sin and cos of a double-double argument |x| <= 1.6 by their Taylor series;
// the remainder after 20 terms is below 1.6^41/41! < 1e-41.
SBR_HD void dd_sincos(dd x, dd* s, dd* c)
{
    dd x2 = dd_mul(x, x);
    dd ts = x, tc = dd{1.0, 0.0};
    dd ss = x, cc = dd{1.0, 0.0};
    for (int k = 1; k <= 20; ++k) {
        double a = (double)(2 * k), b = (double)(2 * k + 1), c0 = (double)(2 * k - 1);
        // ts_k = -ts_{k-1} x^2 / ((2k)(2k+1)),  tc_k = -tc_{k-1} x^2 / ((2k-1)(2k))
        ts = dd_neg(dd_div(dd_mul(ts, x2), dd{a * b, 0.0}));
        tc = dd_neg(dd_div(dd_mul(tc, x2), dd{c0 * a, 0.0}));
        ss = dd_add(ss, ts);
        cc = dd_add(cc, tc);
    }
    *s = ss;
    *c = cc;
}

// Correctly rounded sin(x) for 0 <= x <= 1.6.
SBR_HD double sin_cr(double x)
{
    dd s, c;
    dd_sincos(dd{x, 0.0}, &s, &c);
    return s.hi + s.lo;
}

// Correctly rounded acos(x) for cos(1.6) <= x < 1: two Newton steps on
// cos(y) = x in double-double from the library's acos.
SBR_HD double acos_cr(double x)
{
    dd y = dd{acos(x), 0.0};
    for (int it = 0; it < 2; ++it) {
        dd s, c;
        dd_sincos(y, &s, &c);
        // y <- y + (cos y - x) / sin y
        y = dd_add(y, dd_div(dd_sub(c, dd{x, 0.0}), s));
    }
    return y.hi + y.lo;
}

// Correctly rounded tan(x) for 0 <= x <= 1.5 (sin/cos in double-double).
SBR_HD double tan_cr(double x)
{
    dd s, c;
    dd_sincos(dd{x, 0.0}, &s, &c);
    dd t = dd_div(s, c);
    return t.hi + t.lo;
}

}  // namespace sbr
