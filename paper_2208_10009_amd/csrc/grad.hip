// grad.hip -- differentiable path quantities at a fixed interaction sequence.
//
// For a face sequence f_1..f_k the path is the image-method path (Sec. III.A's
// path test 2 solves it; the precise algorithm of Sec. III.B converges to
// it): images I_j of Tx mirrored across the face planes, reflection points
// P_j by back-projection from Rx.  Its delay, departure and arrival
// directions and power (Friis spreading plus the unpolarized Fresnel
// reflectance of every bounce, Sec. IV's PDP quantities) are smooth
// functions of Tx, Rx and each material's complex permittivity.  The kernel
// evaluates them and, given upstream gradients, the exact gradients by a
// hand-written reverse pass (no tape: the forward intermediates are
// recomputed in registers).
#include <math.h>

#include "internal.h"

namespace sbr {

struct cz {
    double re, im;
};
__device__ static inline cz zadd(cz a, cz b) { return cz{a.re + b.re, a.im + b.im}; }
__device__ static inline cz zsub(cz a, cz b) { return cz{a.re - b.re, a.im - b.im}; }
__device__ static inline cz zmul(cz a, cz b)
{
    return cz{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ static inline cz zscl(double s, cz a) { return cz{s * a.re, s * a.im}; }
__device__ static inline cz zdiv(cz a, cz b)
{
    double den = b.re * b.re + b.im * b.im;
    return cz{(a.re * b.re + a.im * b.im) / den, (a.im * b.re - a.re * b.im) / den};
}
__device__ static inline cz zconj(cz a) { return cz{a.re, -a.im}; }
__device__ static inline cz zsqrt(cz z)
{
    double r = hypot(z.re, z.im);
    if (r == 0.0) return cz{0.0, 0.0};
    if (z.re >= 0.0) {
        double t = sqrt(0.5 * (r + z.re));
        return cz{t, z.im / (2.0 * t)};
    }
    double t = sqrt(0.5 * (r - z.re));
    return cz{fabs(z.im) / (2.0 * t), copysign(t, z.im)};
}

// Unpolarized Fresnel power reflectance R = (|G_perp|^2 + |G_par|^2) / 2 at
// incidence cosine c for er = a + j b, with r = sqrt(er - 1 + c^2):
//   G_perp = (c - r) / (c + r),  G_par = (er c - r) / (er c + r),
// and its partial derivatives dR/dc, dR/da, dR/db.  Both coefficients are
// holomorphic in (c, er); for a real variable x, d|G|^2/dx = 2 Re(conj(G) dG/dx),
// and d/db = j d/der.  With dr/dc = c / r and dr/der = 1 / (2 r):
//   dG_perp/dc  = 2 (r - c^2/r) / (c + r)^2,     dG_perp/der = -c / (r (c + r)^2),
//   dG_par/dc   = 2 er (r - c^2/r) / (er c + r)^2,
//   dG_par/der  = c (2 r^2 - er) / (r (er c + r)^2).
__device__ static inline double fresnel_grad(double c, cz er, double* dRdc, double* dRda,
                                             double* dRdb)
{
    cz cc = cz{c, 0.0};
    cz r = zsqrt(zsub(er, cz{1.0 - c * c, 0.0}));
    cz cpr = zadd(cc, r);
    cz gs = zdiv(zsub(cc, r), cpr);
    cz u = zscl(c, er);
    cz upr = zadd(u, r);
    cz gp = zdiv(zsub(u, r), upr);
    cz rmc = zsub(r, zdiv(cz{c * c, 0.0}, r));  // r - c^2 / r
    cz gs_c = zdiv(zscl(2.0, rmc), zmul(cpr, cpr));
    cz gs_e = zdiv(cz{-c, 0.0}, zmul(r, zmul(cpr, cpr)));
    cz gp_c = zdiv(zscl(2.0, zmul(er, rmc)), zmul(upr, upr));
    cz gp_e = zdiv(zscl(c, zsub(zscl(2.0, zmul(r, r)), er)), zmul(r, zmul(upr, upr)));
    cz ts_c = zmul(zconj(gs), gs_c), tp_c = zmul(zconj(gp), gp_c);
    cz ts_e = zmul(zconj(gs), gs_e), tp_e = zmul(zconj(gp), gp_e);
    *dRdc = ts_c.re + tp_c.re;
    *dRda = ts_e.re + tp_e.re;
    *dRdb = -(ts_e.im + tp_e.im);
    return 0.5 * ((gs.re * gs.re + gs.im * gs.im) + (gp.re * gp.re + gp.im * gp.im));
}



__device__ static inline d3 face_n(const SceneDev& S, int32_t f)
{
    const double* p = S.fplane + 4 * (size_t)f;
    return mk(p[0], p[1], p[2]);
}

// values per path: delay (s), AOD (unit, from Tx), AOA (unit, from Rx toward
// the last interaction), power (dBm)
__global__ __launch_bounds__(256) void k_path_grad(SceneDev S, GradArgs A)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= A.P) return;
    const int k = A.order[p];
    // rows with an order or face id outside the scene get NaN values and zero gradients
    bool bad = k < 0 || k > SBR_MAX_ORDER;
    for (int j = 0; j < k && !bad; ++j) {
        int32_t fj = A.faces[SBR_MAX_ORDER * p + j];
        bad = fj < 0 || fj >= S.n_face;
    }
    if (bad) {
        if (A.val)
            for (int q = 0; q < 8; ++q) A.val[8 * p + q] = NAN;
        if (A.up) {
            st3(A.gtx + 3 * p, mk(0.0, 0.0, 0.0));
            st3(A.grx + 3 * p, mk(0.0, 0.0, 0.0));
        }
        return;
    }
    int32_t f[SBR_MAX_ORDER];
    d3 n[SBR_MAX_ORDER];
    double c[SBR_MAX_ORDER];
    for (int j = 0; j < k; ++j) {
        f[j] = A.faces[SBR_MAX_ORDER * p + j];
        n[j] = face_n(S, f[j]);
        c[j] = S.fplane[4 * (size_t)f[j] + 3];
    }
    const d3 tx = ld3(A.tx + 3 * p), rx = ld3(A.rx + 3 * p);
    // ---- forward: images I[0..k], points Q[0..k+1] (Q[0] = Tx, Q[k+1] = Rx)
    d3 I[SBR_MAX_ORDER + 1];
    I[0] = tx;
    for (int j = 1; j <= k; ++j) {
        double a = dot(n[j - 1], I[j - 1]) - c[j - 1];
        I[j] = sub(I[j - 1], scl(2.0 * a, n[j - 1]));
    }
    d3 Q[SBR_MAX_ORDER + 2], dirv[SBR_MAX_ORDER + 1];
    double sv[SBR_MAX_ORDER + 1], denv[SBR_MAX_ORDER + 1];
    Q[0] = tx;
    Q[k + 1] = rx;
    for (int j = k; j >= 1; --j) {
        d3 X = Q[j + 1];
        d3 dir = sub(I[j], X);
        double num = c[j - 1] - dot(n[j - 1], X);
        double den = dot(n[j - 1], dir);
        double s = num / den;
        Q[j] = add(X, scl(s, dir));
        dirv[j] = dir;
        sv[j] = s;
        denv[j] = den;
    }
    d3 seg[SBR_MAX_ORDER + 2];
    double len[SBR_MAX_ORDER + 2];
    double L = 0.0;
    for (int j = 1; j <= k + 1; ++j) {
        seg[j] = sub(Q[j], Q[j - 1]);
        len[j] = norm(seg[j]);
        L = L + len[j];
    }
    const d3 aod = scl(1.0 / len[1], seg[1]);
    const d3 aoa = scl(-1.0 / len[k + 1], seg[k + 1]);
    const double ln10 = 2.302585092994046;
    double R[SBR_MAX_ORDER], dRc[SBR_MAX_ORDER], sig[SBR_MAX_ORDER], cs[SBR_MAX_ORDER];
    double power = A.tx_power_dbm + 20.0 * log10((kC0 / A.freq_hz) / (4.0 * kPi * L));
    for (int j = 1; j <= k; ++j) {
        double q = dot(seg[j], n[j - 1]);
        sig[j - 1] = q >= 0.0 ? 1.0 : -1.0;
        cs[j - 1] = fabs(q) / len[j];
        int32_t m = S.fmat[f[j - 1]];
        double da, db;
        R[j - 1] = fresnel_grad(cs[j - 1], cz{A.eps[2 * m], A.eps[2 * m + 1]}, &dRc[j - 1], &da,
                                &db);
        power += 10.0 * log10(R[j - 1]);
    }
    if (A.val) {
        double* v = A.val + 8 * p;
        v[0] = L / kC0;
        v[1] = aod.x; v[2] = aod.y; v[3] = aod.z;
        v[4] = aoa.x; v[5] = aoa.y; v[6] = aoa.z;
        v[7] = power;
    }
    if (!A.up) return;
    // ---- reverse
    const double* g = A.up + 8 * p;
    const d3 gaod = mk(g[1], g[2], g[3]), gaoa = mk(g[4], g[5], g[6]);
    const double gP = g[7];
    const double bL = g[0] / kC0 + gP * (-20.0 / (L * ln10));
    d3 bseg[SBR_MAX_ORDER + 2];
    for (int j = 1; j <= k + 1; ++j) bseg[j] = scl(bL / len[j], seg[j]);
    // aod = seg_1 / |seg_1|,  aoa = -seg_{k+1} / |seg_{k+1}|
    bseg[1] = add(bseg[1], scl(1.0 / len[1], sub(gaod, scl(dot(gaod, aod), aod))));
    bseg[k + 1] = sub(bseg[k + 1], scl(1.0 / len[k + 1], sub(gaoa, scl(dot(gaoa, aoa), aoa))));
    // Fresnel terms: cos_j = |seg_j . n_j| / |seg_j|
    for (int j = 1; j <= k; ++j) {
        const double bR = gP * 10.0 / (R[j - 1] * ln10);
        int32_t m = S.fmat[f[j - 1]];
        double dc, da, db;
        fresnel_grad(cs[j - 1], cz{A.eps[2 * m], A.eps[2 * m + 1]}, &dc, &da, &db);
        atomicAdd(&A.geps[2 * m], bR * da);
        atomicAdd(&A.geps[2 * m + 1], bR * db);
        const double bc = bR * dc;
        d3 dcos = scl(1.0 / len[j], sub(scl(sig[j - 1], n[j - 1]), scl(cs[j - 1] / len[j], seg[j])));
        bseg[j] = add(bseg[j], scl(bc, dcos));
    }
    // segments -> points
    d3 bQ[SBR_MAX_ORDER + 2];
    for (int j = 0; j <= k + 1; ++j) bQ[j] = mk(0.0, 0.0, 0.0);
    for (int j = 1; j <= k + 1; ++j) {
        bQ[j] = add(bQ[j], bseg[j]);
        bQ[j - 1] = sub(bQ[j - 1], bseg[j]);
    }
    // back-projection, reverse order: Q_j = X + s dir, X = Q_{j+1},
    // dir = I_j - X, s = (c_j - n.X) / (n.dir)
    d3 bI[SBR_MAX_ORDER + 1];
    for (int j = 0; j <= k; ++j) bI[j] = mk(0.0, 0.0, 0.0);
    for (int j = 1; j <= k; ++j) {
        const d3 nj = n[j - 1];
        const d3 bq = bQ[j];
        d3 bX = bq;
        const double bs = dot(bq, dirv[j]);
        d3 bdir = scl(sv[j], bq);
        const double bnum = bs / denv[j];
        const double bden = -bs * sv[j] / denv[j];
        bX = sub(bX, scl(bnum, nj));
        bdir = add(bdir, scl(bden, nj));
        bI[j] = add(bI[j], bdir);
        bX = sub(bX, bdir);
        bQ[j + 1] = add(bQ[j + 1], bX);
    }
    // images: I_j = I_{j-1} - 2 (n.I_{j-1} - c) n  (a reflection: symmetric Jacobian)
    for (int j = k; j >= 1; --j) {
        const d3 nj = n[j - 1];
        bI[j - 1] = add(bI[j - 1], sub(bI[j], scl(2.0 * dot(nj, bI[j]), nj)));
    }
    st3(A.gtx + 3 * p, add(bQ[0], bI[0]));
    st3(A.grx + 3 * p, bQ[k + 1]);
}

hipError_t launch_path_grad(const SceneDev& S, const GradArgs& A, hipStream_t s)
{
    if (A.P <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_path_grad, dim3((unsigned)((A.P + 255) / 256)), dim3(256), 0, s, S, A);
    return hipGetLastError();
}

}  // namespace sbr
