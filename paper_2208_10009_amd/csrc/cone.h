// cone.h -- the sub-ray cones of the precise algorithm (Sec. III.B), shared by
// the refinement of reflection paths and of diffraction paths.
#pragma once
#include "geom.h"

namespace sbr {

// Orthonormal basis (u, v) of the plane normal to the unit axis a: e is the
// coordinate axis with the smallest |a_i| (ties: lowest i),
// u = normalize(e - a_i a), v = a x u.
__device__ static inline void basis(d3 a, d3* u, d3* v)
{
    double c0 = fabs(a.x), c1 = fabs(a.y), c2 = fabs(a.z);
    int i = 0;
    double ci = c0;
    if (c1 < ci) {
        i = 1;
        ci = c1;
    }
    if (c2 < ci) i = 2;
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

}  // namespace sbr
