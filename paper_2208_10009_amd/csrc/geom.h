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

// 1/k! for k = 0..35 as double-double (hi = 1/k! rounded to nearest, lo = the
// remainder rounded to nearest), written out as exact literals.
constexpr int kFactN = 36;
constexpr dd kInvFact[kFactN] = {
    {0x1.0000000000000p+0, 0.0},  // 1/0!
    {0x1.0000000000000p+0, 0.0},  // 1/1!
    {0x1.0000000000000p-1, 0.0},  // 1/2!
    {0x1.5555555555555p-3, 0x1.5555555555555p-57},  // 1/3!
    {0x1.5555555555555p-5, 0x1.5555555555555p-59},  // 1/4!
    {0x1.1111111111111p-7, 0x1.1111111111111p-63},  // 1/5!
    {0x1.6c16c16c16c17p-10, -0x1.f49f49f49f49fp-65},  // 1/6!
    {0x1.a01a01a01a01ap-13, 0x1.a01a01a01a01ap-73},  // 1/7!
    {0x1.a01a01a01a01ap-16, 0x1.a01a01a01a01ap-76},  // 1/8!
    {0x1.71de3a556c734p-19, -0x1.c154f8ddc6c00p-73},  // 1/9!
    {0x1.27e4fb7789f5cp-22, 0x1.cbbc05b4fa99ap-76},  // 1/10!
    {0x1.ae64567f544e4p-26, -0x1.c062e06d1f209p-80},  // 1/11!
    {0x1.1eed8eff8d898p-29, -0x1.2aec959e14c06p-83},  // 1/12!
    {0x1.6124613a86d09p-33, 0x1.f28e0cc748ebep-87},  // 1/13!
    {0x1.93974a8c07c9dp-37, 0x1.05d6f8a2efd1fp-92},  // 1/14!
    {0x1.ae7f3e733b81fp-41, 0x1.1d8656b0ee8cbp-97},  // 1/15!
    {0x1.ae7f3e733b81fp-45, 0x1.1d8656b0ee8cbp-101},  // 1/16!
    {0x1.952c77030ad4ap-49, 0x1.ac981465ddc6cp-103},  // 1/17!
    {0x1.6827863b97d97p-53, 0x1.eec01221a8b0bp-107},  // 1/18!
    {0x1.2f49b46814157p-57, 0x1.2650f61dbdcb4p-112},  // 1/19!
    {0x1.e542ba4020225p-62, 0x1.ea72b4afe3c2fp-120},  // 1/20!
    {0x1.71b8ef6dcf572p-66, -0x1.d043ae40c4647p-120},  // 1/21!
    {0x1.0ce396db7f853p-70, -0x1.aebcdbd20331cp-124},  // 1/22!
    {0x1.761b41316381ap-75, -0x1.3423c7d91404fp-130},  // 1/23!
    {0x1.f2cf01972f578p-80, -0x1.9ada5fcc1ab14p-135},  // 1/24!
    {0x1.3f3ccdd165fa9p-84, -0x1.58ddadf344487p-139},  // 1/25!
    {0x1.88e85fc6a4e5ap-89, -0x1.71c37ebd16540p-143},  // 1/26!
    {0x1.d1ab1c2dccea3p-94, 0x1.054d0c78aea14p-149},  // 1/27!
    {0x1.0a18a2635085dp-98, 0x1.b9e2e28e1aa54p-153},  // 1/28!
    {0x1.259f98b4358adp-103, 0x1.eaf8c39dd9bc5p-157},  // 1/29!
    {0x1.3932c5047d60ep-108, 0x1.832b7b530a627p-162},  // 1/30!
    {0x1.434d2e783f5bcp-113, 0x1.0b87b91be9affp-167},  // 1/31!
    {0x1.434d2e783f5bcp-118, 0x1.0b87b91be9affp-172},  // 1/32!
    {0x1.3981254dd0d52p-123, -0x1.2b1f4c8015a2fp-177},  // 1/33!
    {0x1.2710231c0fd7ap-128, 0x1.3f8a2b4af9d6bp-184},  // 1/34!
    {0x1.0dc59c716d91fp-133, 0x1.419e3fad3f031p-188},  // 1/35!
};

// sum_{k=0}^{17} (-1)^k / (2k+off)! t^k in Estrin form (pairs, then powers
// t^2, t^4, t^8, t^16), so that the chain of dependent double-double
// operations is 6 deep instead of 17 for Horner's rule.
SBR_HD dd dd_poly_alt(int off, dd t)
{
    const dd* f = kInvFact;
    dd b[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) b[j] = dd_sub(f[4 * j + off], dd_mul(f[4 * j + 2 + off], t));
    dd t2 = dd_mul(t, t);
    dd c0 = dd_add(b[0], dd_mul(b[1], t2)), c1 = dd_add(b[2], dd_mul(b[3], t2));
    dd c2 = dd_add(b[4], dd_mul(b[5], t2)), c3 = dd_add(b[6], dd_mul(b[7], t2));
    dd t4 = dd_mul(t2, t2);
    dd d0 = dd_add(c0, dd_mul(c1, t4)), d1 = dd_add(c2, dd_mul(c3, t4));
    dd t8 = dd_mul(t4, t4);
    dd e0 = dd_add(d0, dd_mul(d1, t8));
    dd t16 = dd_mul(t8, t8);
    return dd_add(e0, dd_mul(b[8], t16));
}

// sin and cos of a double-double argument |x| <= 1.6 by their Taylor series
// over t = x^2 with 18 terms each: the first omitted terms are below
// 1.6^37/37! < 1e-35 and 1.6^36/36! < 1e-34.
SBR_HD void dd_sincos(dd x, dd* s, dd* c)
{
    dd t = dd_mul(x, x);
    *s = dd_mul(x, dd_poly_alt(1, t));
    *c = dd_poly_alt(0, t);
}

// Correctly rounded sin(x) for 0 <= x <= 1.6 (the sine series alone).
SBR_HD double sin_cr(double x)
{
    dd xx = dd{x, 0.0};
    dd s = dd_mul(xx, dd_poly_alt(1, dd_mul(xx, xx)));
    return s.hi + s.lo;
}

// Correctly rounded acos(x) for cos(1.6) <= x < 1: one Newton step on
// cos(y) = x in double-double from the library's acos (error ~1 ulp, so the
// step leaves an error of order ulp^2).
SBR_HD double acos_cr(double x)
{
    dd y = dd{acos(x), 0.0};
    dd s, c;
    dd_sincos(y, &s, &c);
    // y <- y + (cos y - x) / sin y
    y = dd_add(y, dd_div(dd_sub(c, dd{x, 0.0}), s));
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
