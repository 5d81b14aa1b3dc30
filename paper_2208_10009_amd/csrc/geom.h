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

// 1/k! for k = 0 .. kFactN-1 in double-double (relative error ~1e-31),
// built by repeated double-double division; the device copy lives in the
// context and is passed to the kernels that need it.
constexpr int kFactN = 36;
SBR_HD void make_inv_fact(dd* f)
{
    f[0] = dd{1.0, 0.0};
    for (int k = 1; k < kFactN; ++k) f[k] = dd_div(f[k - 1], dd{(double)k, 0.0});
}

// sin and cos of a double-double argument |x| <= 1.6 by their Taylor series
// in Horner form over t = x^2 with 18 terms each: the first omitted terms are
// below 1.6^35/35! < 1e-33 and 1.6^36/36! < 1e-34.
SBR_HD void dd_sincos(dd x, const dd* f, dd* s, dd* c)
{
    dd t = dd_mul(x, x);
    dd as = f[35], ac = f[34];
    for (int k = 16; k >= 0; --k) {
        as = dd_sub(f[2 * k + 1], dd_mul(t, as));
        ac = dd_sub(f[2 * k], dd_mul(t, ac));
    }
    *s = dd_mul(x, as);
    *c = ac;
}

// Correctly rounded sin(x) for 0 <= x <= 1.6 (the sine series alone).
SBR_HD double sin_cr(double x, const dd* f)
{
    dd xx = dd{x, 0.0};
    dd t = dd_mul(xx, xx);
    dd as = f[35];
    for (int k = 16; k >= 0; --k) as = dd_sub(f[2 * k + 1], dd_mul(t, as));
    dd s = dd_mul(xx, as);
    return s.hi + s.lo;
}

// Correctly rounded acos(x) for cos(1.6) <= x < 1: one Newton step on
// cos(y) = x in double-double from the library's acos (error ~1 ulp, so the
// step leaves an error of order ulp^2).
SBR_HD double acos_cr(double x, const dd* f)
{
    dd y = dd{acos(x), 0.0};
    dd s, c;
    dd_sincos(y, f, &s, &c);
    // y <- y + (cos y - x) / sin y
    y = dd_add(y, dd_div(dd_sub(c, dd{x, 0.0}), s));
    return y.hi + y.lo;
}

// Correctly rounded tan(x) for 0 <= x <= 1.5 (sin/cos in double-double).
SBR_HD double tan_cr(double x, const dd* f)
{
    dd s, c;
    dd_sincos(dd{x, 0.0}, f, &s, &c);
    dd t = dd_div(s, c);
    return t.hi + t.lo;
}

}  // namespace sbr
