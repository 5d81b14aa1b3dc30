/*
 * sbr_oracle.c -- plain, slow FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Follows Zhou et al., "An Improved Equiangular Division Algorithm for SBR
 * based Ray Tracing Channel Modeling", step by step, brute force over every
 * triangle.  Readings of places where the paper is silent or garbled are
 * stated next to the code that takes them.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fopenmp -fPIC
 *        -shared sbr_oracle.c -lquadmath -lm
 */
#include "sbr_oracle.h"

#include <complex.h>
#include <math.h>
#include <quadmath.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#if defined(__FP_FAST_FMA) && !defined(ORC_ALLOW_FMA)
/* Not an error: -ffp-contract=off is what matters; this only documents it. */
#endif

/* ------------------------------------------------------------------------ */
/* small FP64 vector helpers; every operation is written in evaluation order */
/* ------------------------------------------------------------------------ */
typedef struct { double x, y, z; } v3;

static v3 mk(double x, double y, double z) { v3 r = {x, y, z}; return r; }
static v3 add(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 sub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3 scl(double s, v3 a) { return mk(s * a.x, s * a.y, s * a.z); }
static double dot(v3 a, v3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
static v3 cross(v3 a, v3 b)
{
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static double norm(v3 a) { return sqrt(dot(a, a)); }
static v3 normalize(v3 a)
{
    double r = norm(a);
    return mk(a.x / r, a.y / r, a.z / r);
}
static v3 ld3(const double* p) { return mk(p[0], p[1], p[2]); }
static void st3(double* p, v3 a) { p[0] = a.x; p[1] = a.y; p[2] = a.z; }

static const double C0 = 299792458.0;            /* speed of light, m/s   */
static const double PI_D = 3.14159265358979323846; /* nearest double to pi */

/* Correctly rounded transcendental values: binary128 then one rounding. */
double orc_sin_cr(double x) { return (double)sinq((__float128)x); }
double orc_acos_cr(double x) { return (double)acosq((__float128)x); }
static double tan_cr(double x) { return (double)tanq((__float128)x); }
static double atan_cr(double x) { return (double)atanq((__float128)x); }

/* theta_0 = angle subtended by one icosahedron edge = atan(2) (eq. (4)). */
static double theta0(void) { return atan_cr(2.0); }
/* Cone half-angle theta_launch = theta_0 / (sqrt(3) n), eq. (4), theta_0 the
 * angle subtended by a polyhedron edge.  Reading: the equidistant grids of
 * Sec. II.A keep the same rule with their own edge angle (atan 2 for the
 * icosahedron, pi/2 for the octahedron). */
static double theta_launch_m(int32_t method, int32_t n)
{
    double th = method == ORC_LAUNCH_EQUIDISTANT_OCTA ? PI_D / 2.0 : theta0();
    return th / (sqrt(3.0) * (double)n);
}
static double theta_launch(int32_t n) { return theta_launch_m(ORC_LAUNCH_EQUIANGULAR, n); }

/* ======================================================================== */
/* Launch grid -- Sec. II.B                                                  */
/* ======================================================================== */
/* Icosahedron: the 12 cyclic permutations of (0, +-1, +-phi), normalized, in
 * this fixed order.  Edges are the 30 vertex pairs with positive dot product
 * (adjacent vertices subtend theta_0; non-adjacent ones have dot <= -1/sqrt5),
 * listed lexicographically (i < j).  Faces are the 20 mutually adjacent
 * triples i < j < k, listed lexicographically, each wound so that it is
 * counter-clockwise seen from outside -- which is clockwise seen from the
 * launch point O, the paper's "arranged clockwise". */
typedef struct {
    v3 V[12];
    int e[30][2];
    int f[20][3];
} ico_t;

static void ico_build(ico_t* ic)
{
    double phi = (1.0 + sqrt(5.0)) / 2.0;
    const double raw[12][3] = {
        {0, 1, phi}, {0, -1, phi}, {0, 1, -phi}, {0, -1, -phi},
        {1, phi, 0}, {-1, phi, 0}, {1, -phi, 0}, {-1, -phi, 0},
        {phi, 0, 1}, {phi, 0, -1}, {-phi, 0, 1}, {-phi, 0, -1}};
    for (int i = 0; i < 12; ++i) ic->V[i] = normalize(ld3(raw[i]));
    int ne = 0, nf = 0;
    int adj[12][12];
    for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j) adj[i][j] = (i != j) && dot(ic->V[i], ic->V[j]) > 0.0;
    for (int i = 0; i < 12; ++i)
        for (int j = i + 1; j < 12; ++j)
            if (adj[i][j]) { ic->e[ne][0] = i; ic->e[ne][1] = j; ++ne; }
    for (int i = 0; i < 12; ++i)
        for (int j = i + 1; j < 12; ++j)
            for (int k = j + 1; k < 12; ++k)
                if (adj[i][j] && adj[j][k] && adj[i][k]) {
                    double s = dot(ic->V[i], cross(ic->V[j], ic->V[k]));
                    ic->f[nf][0] = i;
                    ic->f[nf][1] = s > 0.0 ? j : k;
                    ic->f[nf][2] = s > 0.0 ? k : j;
                    ++nf;
                }
}

/* Point k of m equal-angle steps from P to Q on the great circle (eq. (1):
 * consecutive points subtend the same angle at O).  The direction is
 * sin((m-k)th/m) P + sin(k th/m) Q, normalized (the 1/sin(th) factor of the
 * usual slerp only rescales and is dropped). */
static v3 arc_point(v3 P, v3 Q, int64_t k, int64_t m)
{
    double th = orc_acos_cr(dot(P, Q));
    double a = ((double)k * th) / (double)m;
    double b = ((double)(m - k) * th) / (double)m;
    double sa = orc_sin_cr(a), sb = orc_sin_cr(b);
    return normalize(add(scl(sb, P), scl(sa, Q)));
}

/* Rings of one icosahedron face.  Layer 0 is the face boundary: vertices
 * W0,W1,W2 = the face's corners and m = n equal-angle steps per side.  Layer
 * a+1 has side m-3; its corners come from eq. (2): X' = P^1 + P^{-1} - P^0,
 * i.e. the parallelogram completion at each corner using the two ring points
 * adjacent to it.  Reading: eq. (2) is evaluated on the flat icosahedron face
 * (Fig. 3b draws B, C, D on the edge AE), so every point is first centrally
 * projected onto a plane parallel to the face, X' is formed there and then
 * turned back into a direction.  The plane x.g = 1 with g = A+B+C is used
 * (any parallel plane gives the same direction, the construction is affine).
 * Side m' = 0 is the single centre ray normalize(A+B+C); m' < 0 ends. */
typedef struct {
    int32_t nl;        /* number of inner layers (a = 1..nl)            */
    v3* W;             /* [nl][3] corners of layer a (index a-1)         */
    int64_t* m;        /* [nl] side of layer a (0 = centre point)        */
    int64_t* start;    /* [nl] first interior index of layer a           */
} face_rings;

static v3 proj_face(v3 p, v3 g)
{
    double w = dot(p, g);
    return mk(p.x / w, p.y / w, p.z / w);
}

static void rings_build(face_rings* R, const ico_t* ic, int fi, int32_t n)
{
    v3 A = ic->V[ic->f[fi][0]], B = ic->V[ic->f[fi][1]], C = ic->V[ic->f[fi][2]];
    v3 g = add(add(A, B), C);
    int32_t cap = n / 3 + 2;
    R->W = (v3*)malloc(sizeof(v3) * 3 * (size_t)cap);
    R->m = (int64_t*)malloc(sizeof(int64_t) * (size_t)cap);
    R->start = (int64_t*)malloc(sizeof(int64_t) * (size_t)cap);
    v3 W[3] = {A, B, C};
    int64_t m = n;
    int32_t nl = 0;
    int64_t pos = 0;
    for (;;) {
        int64_t mp = m - 3;
        if (mp < 0) break;
        R->start[nl] = pos;
        if (mp == 0) {
            R->W[3 * nl + 0] = R->W[3 * nl + 1] = R->W[3 * nl + 2] = normalize(add(add(A, B), C));
            R->m[nl] = 0;
            ++nl;
            pos += 1;
            break;
        }
        v3 Wn[3];
        for (int s = 0; s < 3; ++s) {
            v3 P0 = W[s];
            v3 P1 = arc_point(W[s], W[(s + 1) % 3], 1, m);      /* next on side s   */
            v3 Pm = arc_point(W[(s + 2) % 3], W[s], m - 1, m);  /* last on side s-1 */
            v3 X = sub(add(proj_face(P1, g), proj_face(Pm, g)), proj_face(P0, g));
            Wn[s] = normalize(X);
        }
        for (int s = 0; s < 3; ++s) { W[s] = Wn[s]; R->W[3 * nl + s] = Wn[s]; }
        R->m[nl] = mp;
        ++nl;
        pos += 3 * mp;
        m = mp;
    }
    R->nl = nl;
}

static void rings_free(face_rings* R)
{
    free(R->W); free(R->m); free(R->start);
}

int64_t orc_num_rays(int32_t n)
{
    if (n < 1) return 0;
    return 10 * (int64_t)n * n + 2;
}

int64_t orc_num_rays_m(int32_t method, int32_t n)
{
    if (n < 1 || method < 0 || method > ORC_LAUNCH_EQUIDISTANT_OCTA) return 0;
    return (method == ORC_LAUNCH_EQUIDISTANT_OCTA ? 4 : 10) * (int64_t)n * n + 2;
}

/* A regular polyhedron with triangular faces for the equidistant grids of
 * Sec. II.A: vertices, edges (adjacent pairs i < j, lexicographic) and faces
 * (mutually adjacent triples i < j < k, lexicographic, wound counter-clockwise
 * seen from outside).  The icosahedron is the one above; the octahedron has
 * the vertices +x, -x, +y, -y, +z, -z in this order (adjacent: not
 * antipodal). */
typedef struct {
    int nv, ne, nf;
    v3 V[12];
    int e[30][2];
    int f[20][3];
} poly_t;

static void poly_build(poly_t* P, int32_t method)
{
    if (method == ORC_LAUNCH_EQUIDISTANT_OCTA) {
        const double raw[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
        P->nv = 6;
        for (int i = 0; i < 6; ++i) P->V[i] = ld3(raw[i]);
        P->ne = P->nf = 0;
        for (int i = 0; i < 6; ++i)
            for (int j = i + 1; j < 6; ++j)
                if (dot(P->V[i], P->V[j]) > -0.5) { P->e[P->ne][0] = i; P->e[P->ne][1] = j; ++P->ne; }
        for (int i = 0; i < 6; ++i)
            for (int j = i + 1; j < 6; ++j)
                for (int k = j + 1; k < 6; ++k)
                    if (dot(P->V[i], P->V[j]) > -0.5 && dot(P->V[j], P->V[k]) > -0.5 &&
                        dot(P->V[i], P->V[k]) > -0.5) {
                        double sg = dot(P->V[i], cross(P->V[j], P->V[k]));
                        P->f[P->nf][0] = i;
                        P->f[P->nf][1] = sg > 0.0 ? j : k;
                        P->f[P->nf][2] = sg > 0.0 ? k : j;
                        ++P->nf;
                    }
        return;
    }
    ico_t ic;
    ico_build(&ic);
    P->nv = 12; P->ne = 30; P->nf = 20;
    memcpy(P->V, ic.V, sizeof(ic.V));
    memcpy(P->e, ic.e, sizeof(ic.e));
    memcpy(P->f, ic.f, sizeof(ic.f));
}

/* Equidistant division (Sec. II.A): points at equal spacing on the flat
 * faces, projected onto the sphere.  Order: vertices; edge interiors edge by
 * edge, k = 1..n-1 from the lower vertex, at (n-k) V_i + k V_j; face
 * interiors face by face, rows i = 1..n-2 and j = 1..n-1-i, at
 * (n-i-j) A + i B + j C for the face's corners A, B, C; each normalized. */
static v3 equidistant_dir(const poly_t* P, int32_t n, int64_t idx)
{
    if (idx < P->nv) return P->V[idx];
    idx -= P->nv;
    if (idx < (int64_t)P->ne * (n - 1)) {
        int64_t e = idx / (n - 1), k = idx % (n - 1) + 1;
        return normalize(add(scl((double)(n - k), P->V[P->e[e][0]]), scl((double)k, P->V[P->e[e][1]])));
    }
    idx -= (int64_t)P->ne * (n - 1);
    int64_t per_face = (int64_t)(n - 1) * (n - 2) / 2;
    int64_t f = idx / per_face, q = idx % per_face;
    int64_t i = 1;
    while (q >= n - 1 - i) { q -= n - 1 - i; ++i; }
    int64_t j = q + 1, a = n - i - j;
    v3 A = P->V[P->f[f][0]], B = P->V[P->f[f][1]], C = P->V[P->f[f][2]];
    return normalize(add(add(scl((double)a, A), scl((double)i, B)), scl((double)j, C)));
}

typedef struct {
    int32_t n, method;
    ico_t ic;
    face_rings fr[20];
    poly_t poly;
} grid_t;

static void grid_init_m(grid_t* G, int32_t method, int32_t n)
{
    G->n = n;
    G->method = method;
    if (method != ORC_LAUNCH_EQUIANGULAR) {
        poly_build(&G->poly, method);
        return;
    }
    ico_build(&G->ic);
    for (int f = 0; f < 20; ++f) rings_build(&G->fr[f], &G->ic, f, n);
}
static void grid_init(grid_t* G, int32_t n) { grid_init_m(G, ORC_LAUNCH_EQUIANGULAR, n); }
static void grid_free(grid_t* G)
{
    if (G->method != ORC_LAUNCH_EQUIANGULAR) return;
    for (int f = 0; f < 20; ++f) rings_free(&G->fr[f]);
}

/* Ray order: 12 vertex rays; then edge interiors, edge by edge, k = 1..n-1
 * from the lower to the higher vertex index; then face interiors, face by
 * face, layer by layer, each ring P^0..P^{3m-1} starting at the corner that
 * descends from the face's first vertex. */
static v3 grid_dir(const grid_t* G, int64_t idx)
{
    const int64_t n = G->n;
    if (G->method != ORC_LAUNCH_EQUIANGULAR) return equidistant_dir(&G->poly, G->n, idx);
    if (idx < 12) return G->ic.V[idx];
    idx -= 12;
    if (idx < 30 * (n - 1)) {
        int64_t e = idx / (n - 1), k = idx % (n - 1) + 1;
        return arc_point(G->ic.V[G->ic.e[e][0]], G->ic.V[G->ic.e[e][1]], k, n);
    }
    idx -= 30 * (n - 1);
    int64_t per_face = (n - 1) * (n - 2) / 2;
    int64_t f = idx / per_face, r = idx % per_face;
    const face_rings* R = &G->fr[f];
    int32_t a = 0;
    while (a + 1 < R->nl && R->start[a + 1] <= r) ++a;
    r -= R->start[a];
    int64_t m = R->m[a];
    const v3* W = &R->W[3 * a];
    if (m == 0) return W[0];
    int64_t s = r / m, k = r % m;
    if (k == 0) return W[s];
    return arc_point(W[s], W[(s + 1) % 3], k, m);
}

int orc_launch_dirs(int32_t n, const int64_t* ids, int64_t m, double* out)
{
    return orc_launch_dirs_m(ORC_LAUNCH_EQUIANGULAR, n, ids, m, out);
}

int orc_launch_dirs_m(int32_t method, int32_t n, const int64_t* ids, int64_t m, double* out)
{
    if (n < 1 || !out || method < 0 || method > ORC_LAUNCH_EQUIDISTANT_OCTA) return -1;
    int64_t N = orc_num_rays_m(method, n);
    if (!ids) m = N;
    grid_t G;
    grid_init_m(&G, method, n);
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t i = 0; i < m; ++i) {
        int64_t id = ids ? ids[i] : i;
        if (id < 0 || id >= N) { bad = 1; continue; }
        st3(out + 3 * i, grid_dir(&G, id));
    }
    grid_free(&G);
    return bad ? -1 : 0;
}

/* ======================================================================== */
/* Scene and closest hit -- Sec. III.A                                       */
/* ======================================================================== */
typedef struct {
    int64_t T;
    int32_t F;
    v3 *v0, *e1, *e2;
    const int32_t *face, *mat;
    v3* fn;          /* [F] face plane unit normal                        */
    double* fc;      /* [F] plane offset fn . v0                          */
    int32_t* fmat;   /* [F] material of the face                          */
    double t_eps;    /* 1e-9 * diagonal of the scene bounding box         */
} scene_t;

/* Reading: a face is a planar polygon (face_id); its plane is taken from its
 * lowest-index triangle, n = normalize(e1 x e2), and so is its material. */
static int scene_init(scene_t* S, const double* tri_v, const int32_t* face_id,
                      const int32_t* mat_id, int64_t T)
{
    memset(S, 0, sizeof(*S));
    S->T = T;
    S->face = face_id;
    S->mat = mat_id;
    S->v0 = (v3*)malloc(sizeof(v3) * (size_t)(T > 0 ? T : 1));
    S->e1 = (v3*)malloc(sizeof(v3) * (size_t)(T > 0 ? T : 1));
    S->e2 = (v3*)malloc(sizeof(v3) * (size_t)(T > 0 ? T : 1));
    int32_t F = 0;
    v3 lo = mk(INFINITY, INFINITY, INFINITY), hi = mk(-INFINITY, -INFINITY, -INFINITY);
    for (int64_t i = 0; i < T; ++i) {
        v3 a = ld3(tri_v + 9 * i), b = ld3(tri_v + 9 * i + 3), c = ld3(tri_v + 9 * i + 6);
        S->v0[i] = a;
        S->e1[i] = sub(b, a);
        S->e2[i] = sub(c, a);
        if (face_id[i] < 0) return -1;
        if (face_id[i] + 1 > F) F = face_id[i] + 1;
        v3 p[3] = {a, b, c};
        for (int q = 0; q < 3; ++q) {
            lo.x = fmin(lo.x, p[q].x); lo.y = fmin(lo.y, p[q].y); lo.z = fmin(lo.z, p[q].z);
            hi.x = fmax(hi.x, p[q].x); hi.y = fmax(hi.y, p[q].y); hi.z = fmax(hi.z, p[q].z);
        }
    }
    S->F = F;
    S->fn = (v3*)calloc((size_t)(F > 0 ? F : 1), sizeof(v3));
    S->fc = (double*)calloc((size_t)(F > 0 ? F : 1), sizeof(double));
    S->fmat = (int32_t*)calloc((size_t)(F > 0 ? F : 1), sizeof(int32_t));
    int32_t* seen = (int32_t*)calloc((size_t)(F > 0 ? F : 1), sizeof(int32_t));
    for (int64_t i = 0; i < T; ++i) {
        int32_t f = face_id[i];
        if (seen[f]) continue;
        seen[f] = 1;
        S->fn[f] = normalize(cross(S->e1[i], S->e2[i]));
        S->fc[f] = dot(S->fn[f], S->v0[i]);
        S->fmat[f] = mat_id ? mat_id[i] : 0;
    }
    free(seen);
    if (T > 0) {
        v3 d = sub(hi, lo);
        S->t_eps = 1e-9 * norm(d);
    }
    return 0;
}

static void scene_free(scene_t* S)
{
    free(S->v0); free(S->e1); free(S->e2); free(S->fn); free(S->fc); free(S->fmat);
}

/* Moller-Trumbore, in exactly this order:
 *   p = d x e2, det = e1.p (det == 0: miss), s = o - v0,
 *   u = (s.p)/det, q = s x e1, v = (d.q)/det, t = (e2.q)/det,
 *   hit iff u >= 0, v >= 0, u + v <= 1 and t_lo < t < t_hi. */
static int mt_hit(const scene_t* S, int64_t i, v3 o, v3 d, double t_lo, double t_hi, double* t_out)
{
    v3 p = cross(d, S->e2[i]);
    double det = dot(S->e1[i], p);
    if (det == 0.0) return 0;
    v3 s = sub(o, S->v0[i]);
    double u = dot(s, p) / det;
    v3 q = cross(s, S->e1[i]);
    double v = dot(d, q) / det;
    double t = dot(S->e2[i], q) / det;
    if (u >= 0.0 && v >= 0.0 && u + v <= 1.0 && t > t_lo && t < t_hi) {
        *t_out = t;
        return 1;
    }
    return 0;
}

/* Closest hit over every triangle except those of the face just left (a
 * planar face cannot be hit again right after reflecting on it).  Ties of t
 * go to the lower face id, then the lower triangle index. */
static int64_t closest_hit(const scene_t* S, v3 o, v3 d, int32_t prev_face, double* t_out)
{
    int64_t best = -1;
    double bt = INFINITY;
    for (int64_t i = 0; i < S->T; ++i) {
        if (S->face[i] == prev_face) continue;
        double t;
        if (!mt_hit(S, i, o, d, S->t_eps, INFINITY, &t)) continue;
        if (best < 0 || t < bt || (t == bt && S->face[i] < S->face[best])) {
            best = i;
            bt = t;
        }
    }
    *t_out = best < 0 ? INFINITY : bt;
    return best;
}

/* Specular reflection off the face plane: d' = d - 2 (d.n) n (no
 * renormalization).  Next origin o' = o + t d. */
static v3 reflect_dir(v3 d, v3 n)
{
    double k = 2.0 * dot(d, n);
    return sub(d, scl(k, n));
}

/* One traced segment of a ray. */
typedef struct {
    v3 o, d;
    double D;          /* unfolded length from Tx to o                   */
    double t;          /* parameter of the next hit (+inf: none)         */
    int64_t tri;       /* next hit triangle (-1: none)                   */
} seg_t;

/* Trace up to K reflections: fills segs[0..ns-1], returns ns (<= K+1).
 * Segment j starts after j reflections. */
static int trace_ray(const scene_t* S, v3 tx, v3 d0, int32_t K, seg_t* segs)
{
    v3 o = tx, d = d0;
    double D = 0.0;
    int32_t prev = -1;
    int ns = 0;
    for (int32_t j = 0; j <= K; ++j) {
        double t;
        int64_t tri = closest_hit(S, o, d, prev, &t);
        segs[ns].o = o; segs[ns].d = d; segs[ns].D = D; segs[ns].t = t; segs[ns].tri = tri;
        ++ns;
        if (tri < 0 || j == K) break;
        int32_t f = S->face[tri];
        v3 on = add(o, scl(t, d));
        d = reflect_dir(d, S->fn[f]);
        D = D + t;
        o = on;
        prev = f;
    }
    return ns;
}

/* Reception test and error angle (eq. (3)) for one segment and one Rx.
 * t* = (Rx - o).d is the foot of the perpendicular; accept iff 0 < t* <= t
 * (Rx in front of the segment start and before its next hit) and Rx lies
 * inside the ray cone, d_perp <= theta_launch (D + t*).  Reading: the
 * propagation distance d_ray of eq. (3) is the unfolded length to the foot
 * D + t*, so tan(theta_error) = d_perp / (D + t*) is the angle between the
 * ray and the exact departure direction toward the image of Rx.  With
 * thl < 0 the cone condition is skipped (used by the precise algorithm). */
static int capture_seg(const seg_t* sg, v3 rx, double thl, double* tan_out)
{
    v3 w = sub(rx, sg->o);
    double ts = dot(w, sg->d);
    if (!(ts > 0.0)) return 0;
    if (!(ts <= sg->t)) return 0;
    v3 f = sub(w, scl(ts, sg->d));
    double dp = norm(f);
    double L = sg->D + ts;
    if (thl >= 0.0 && !(dp <= thl * L)) return 0;
    *tan_out = dp / L;
    return 1;
}

int orc_trace_rays(const double* tri_v, const int32_t* face_id, int64_t n_tri,
                   const double tx[3], int32_t n, int32_t launch, int32_t K,
                   const int64_t* ids, int64_t m, int32_t n_threads,
                   int32_t* out_tri, int32_t* out_face, double* out_t)
{
    if (n < 1 || K < 0 || K > ORC_MAX_ORDER || n_tri < 0 || launch < 0 ||
        launch > ORC_LAUNCH_EQUIDISTANT_OCTA)
        return -1;
    int64_t N = orc_num_rays_m(launch, n);
    if (!ids) m = N;
    scene_t S;
    if (scene_init(&S, tri_v, face_id, NULL, n_tri)) { scene_free(&S); return -1; }
    grid_t G;
    grid_init_m(&G, launch, n);
    v3 T = ld3(tx);
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : bad)
    for (int64_t i = 0; i < m; ++i) {
        int64_t id = ids ? ids[i] : i;
        if (id < 0 || id >= N) { bad = 1; continue; }
        seg_t segs[ORC_MAX_ORDER + 1];
        int ns = trace_ray(&S, T, grid_dir(&G, id), K, segs);
        for (int j = 0; j <= K; ++j) {
            int64_t o = i * (K + 1) + j;
            int64_t tri = j < ns ? segs[j].tri : -1;
            if (out_tri) out_tri[o] = (int32_t)tri;
            if (out_face) out_face[o] = tri < 0 ? -1 : face_id[tri];
            if (out_t) out_t[o] = j < ns ? segs[j].t : INFINITY;
        }
    }
    grid_free(&G);
    scene_free(&S);
    return bad ? -1 : 0;
}

int orc_trace_dirs(const double* tri_v, const int32_t* face_id, int64_t n_tri,
                   const double tx[3], const double* dirs, int64_t m, int32_t K,
                   int32_t* out_tri, int32_t* out_face, double* out_t, double* out_D)
{
    if (K < 0 || K > ORC_MAX_ORDER || n_tri < 0 || m < 0) return -1;
    scene_t S;
    if (scene_init(&S, tri_v, face_id, NULL, n_tri)) { scene_free(&S); return -1; }
    v3 T = ld3(tx);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < m; ++i) {
        seg_t segs[ORC_MAX_ORDER + 1];
        int ns = trace_ray(&S, T, ld3(dirs + 3 * i), K, segs);
        for (int j = 0; j <= K; ++j) {
            int64_t o = i * (K + 1) + j;
            int64_t tri = j < ns ? segs[j].tri : -1;
            if (out_tri) out_tri[o] = (int32_t)tri;
            if (out_face) out_face[o] = tri < 0 ? -1 : face_id[tri];
            if (out_t) out_t[o] = j < ns ? segs[j].t : INFINITY;
            if (out_D) out_D[o] = j < ns ? segs[j].D : NAN;
        }
    }
    scene_free(&S);
    return 0;
}

/* ======================================================================== */
/* Path test 1 (double counting) -- Sec. III.A                               */
/* ======================================================================== */
static int key_cmp(const orc_candidate* a, const orc_candidate* b)
{
    if (a->rx != b->rx) return a->rx < b->rx ? -1 : 1;
    if (a->order != b->order) return a->order < b->order ? -1 : 1;
    for (int j = 0; j < a->order; ++j)
        if (a->face[j] != b->face[j]) return a->face[j] < b->face[j] ? -1 : 1;
    return 0;
}

/* Same faces: keep the smaller error angle; reading: equal angles keep the
 * lower launch-ray index. */
static int cand_cmp(const void* pa, const void* pb)
{
    const orc_candidate *a = (const orc_candidate*)pa, *b = (const orc_candidate*)pb;
    int c = key_cmp(a, b);
    if (c) return c;
    if (a->tan_err != b->tan_err) return a->tan_err < b->tan_err ? -1 : 1;
    if (a->ray != b->ray) return a->ray < b->ray ? -1 : 1;
    return 0;
}

/* ======================================================================== */
/* Precise algorithm -- Sec. III.B                                           */
/* ======================================================================== */
/* Trace direction d from Tx through exactly the faces of the path and report
 * the error angle of Rx on the last segment (no cone condition): the
 * sub-ray is a usable path only if it meets the same faces in the same order
 * and Rx lies ahead on its last segment before the next obstacle. */
typedef struct {
    double tan_err;
    double D, Llast;    /* unfolded length to the last reflection, |Rx - p_k| */
    v3 p[ORC_MAX_ORDER];
    v3 din[ORC_MAX_ORDER];
} follow_t;

static int follow_path(const scene_t* S, v3 tx, v3 d0, v3 rx, int32_t k, const int32_t* faces,
                       follow_t* out)
{
    seg_t segs[ORC_MAX_ORDER + 1];
    int ns = trace_ray(S, tx, d0, k, segs);
    if (ns != k + 1) return 0;
    for (int j = 0; j < k; ++j)
        if (segs[j].tri < 0 || S->face[segs[j].tri] != faces[j]) return 0;
    double tn;
    if (!capture_seg(&segs[k], rx, -1.0, &tn)) return 0;
    if (out) {
        out->tan_err = tn;
        out->D = segs[k].D;
        out->Llast = norm(sub(rx, segs[k].o));
        for (int j = 0; j < k; ++j) { out->p[j] = segs[j + 1].o; out->din[j] = segs[j].d; }
    }
    return 1;
}

/* Orthonormal basis (u, v) of the plane normal to axis a: e is the
 * coordinate axis with the smallest |a_i| (ties: lowest i),
 * u = normalize(e - a_i a), v = a x u. */
static void basis(v3 a, v3* u, v3* v)
{
    double c[3] = {fabs(a.x), fabs(a.y), fabs(a.z)};
    int i = 0;
    if (c[1] < c[i]) i = 1;
    if (c[2] < c[i]) i = 2;
    v3 e = mk(i == 0 ? 1.0 : 0.0, i == 1 ? 1.0 : 0.0, i == 2 ? 1.0 : 0.0);
    double ai = i == 0 ? a.x : (i == 1 ? a.y : a.z);
    *u = normalize(sub(e, scl(ai, a)));
    *v = cross(a, *u);
}

/* Sub-ray s of a cone with axis a: the cone's disc (radius rho_prev in the
 * plane tangent to the unit sphere at a) is covered by six discs of radius
 * rho = rho_prev / sqrt(3) centred at distance rho from the axis, at phases
 * 0, 60, ..., 300 degrees (six circles of radius r/sqrt3 at distance r/sqrt3
 * exactly cover the disc of radius r).  The seventh sub-ray (s = 6) is the
 * axis itself. */
static v3 subray(v3 a, v3 u, v3 v, double rho, int s)
{
    if (s == 6) return a;
    const double h = sqrt(3.0) * 0.5;
    const double cs[6] = {1.0, 0.5, -0.5, -1.0, -0.5, 0.5};
    const double ss[6] = {0.0, h, h, 0.0, -h, -h};
    v3 w = add(scl(cs[s], u), scl(ss[s], v));
    return normalize(add(a, scl(rho, w)));
}

/* Stop rule "error satisfies the requirement" (reading): with a target error
 * angle, stop once tan(err) <= tan(target) * Llast / Ltot.  The AOA error of
 * a path grows from its AOD error roughly by D_k / Llast, so this scale makes
 * both AOD and AOA meet the target. */
static int target_met(double tan_err, double tan_tgt, double D, double Llast)
{
    double Ltot = D + Llast;
    double thr = (tan_tgt * Llast) / Ltot;
    return tan_err <= thr;
}

/* The precise algorithm's loop, shared by reflection and diffraction paths.
 * follow(ctx, d, ...) decides whether direction d still forms the path (for a
 * reflection path: meets its faces in order with Rx ahead; for a diffraction
 * path: passes and reaches its wedge) and gives tan(error angle), the
 * unfolded length D to the last interaction and the last leg Llast, and the
 * path's geometry in *g. */
typedef struct dfollow_s dfollow_t;
typedef int (*follow_fn)(const void* ctx, v3 d, double* tan_err, double* D, double* Llast,
                         void* g);

typedef struct {
    v3 axis;
    double tan_err;
    int32_t iters;
    uint32_t flags;
} refine_state;

/* Start from the winner of path test 1 (axis a0) and iterate: per iteration
 * shrink the cone by 1/sqrt3 and launch the sub-rays; the smallest error
 * angle among those that still form the path becomes the new axis (ties:
 * lower sub-ray); none: STALLED, stop.  Stop after n_it iterations or once
 * the target is met.  cur, tmp, win: three geometry buffers of `gsz` bytes;
 * cur ends with the reported ray's. */
static void refine_loop(follow_fn follow, const void* ctx, void* cur, void* tmp, void* win,
                        size_t gsz, v3 a0, int32_t n_it, int32_t Sn, double tan_tgt, double thl,
                        refine_state* R, double* hist)
{
    double tn, D, Ll;
    R->axis = a0;
    R->iters = 0;
    R->flags = 0;
    if (!follow(ctx, a0, &tn, &D, &Ll, cur)) {
        /* cannot happen for a captured ray; guarded for external rows */
        R->tan_err = NAN;
        R->flags |= 1u;
        if (hist) hist[0] = NAN;
        return;
    }
    R->tan_err = tn;
    if (hist) hist[0] = R->tan_err;
    double rho = thl;
    int met = tan_tgt > 0.0 && target_met(R->tan_err, tan_tgt, D, Ll);
    if (met) R->flags |= 4u;
    for (int32_t i = 1; i <= n_it && !met; ++i) {
        rho = rho / sqrt(3.0);
        v3 u, v;
        basis(R->axis, &u, &v);
        int bs = -1;
        double bt = INFINITY, bD = 0.0, bL = 0.0;
        v3 bd = R->axis;
        for (int s = 0; s < Sn; ++s) {
            v3 ds = subray(R->axis, u, v, rho, s);
            if (!follow(ctx, ds, &tn, &D, &Ll, tmp)) continue;
            if (tn < bt) {
                bt = tn;
                bs = s;
                bd = ds;
                bD = D;
                bL = Ll;
                memcpy(win, tmp, gsz);
            }
        }
        if (bs < 0) {
            R->flags |= 1u;   /* STALLED: no sub-ray still forms the path */
            if (hist) for (int32_t q = i; q <= n_it; ++q) hist[q] = R->tan_err;
            break;
        }
        R->axis = bd;
        R->tan_err = bt;
        memcpy(cur, win, gsz);
        R->iters = i;
        if (hist) hist[i] = bt;
        if (tan_tgt > 0.0 && target_met(bt, tan_tgt, bD, bL)) {
            R->flags |= 4u;
            met = 1;
        }
    }
}

typedef struct {
    v3 axis;
    double tan_err;
    int32_t iters;
    uint32_t flags;
    follow_t fw;
} refine_t;

typedef struct {
    const scene_t* S;
    v3 tx, rx;
    int32_t k;
    const int32_t* faces;
} refl_ctx;

static int follow_refl_cb(const void* c, v3 d, double* tn, double* D, double* Ll, void* g)
{
    const refl_ctx* x = (const refl_ctx*)c;
    follow_t* fw = (follow_t*)g;
    if (!follow_path(x->S, x->tx, d, x->rx, x->k, x->faces, fw)) return 0;
    *tn = fw->tan_err;
    *D = fw->D;
    *Ll = fw->Llast;
    return 1;
}

/* One reflection path: the precise algorithm from its path-test-1 winner. */
static void refine_path(const scene_t* S, v3 tx, v3 rx, int32_t k, const int32_t* faces,
                        v3 a0, int32_t n_it, int32_t Sn, double tan_tgt, double thl,
                        refine_t* R, double* hist)
{
    refl_ctx x = {S, tx, rx, k, faces};
    follow_t tmp, win;
    refine_state st;
    refine_loop(follow_refl_cb, &x, &R->fw, &tmp, &win, sizeof(follow_t), a0, n_it, Sn, tan_tgt,
                thl, &st, hist);
    R->axis = st.axis;
    R->tan_err = st.tan_err;
    R->iters = st.iters;
    R->flags = st.flags;
}

/* ======================================================================== */
/* Path quantities, validity (path test 2) and power                         */
/* ======================================================================== */
/* Fresnel reflection coefficients for relative permittivity er (e^{jwt}
 * convention, er = e' - j e''), principal complex square root:
 *   G_perp = (c - sqrt(er - s^2)) / (c + sqrt(er - s^2))
 *   G_par  = (er c - sqrt(er - s^2)) / (er c + sqrt(er - s^2)).
 * Reading (the paper gives no power formula): unpolarized average
 * 0.5 (|G_perp|^2 + |G_par|^2). */
double orc_fresnel_avg(double c, double er_re, double er_im)
{
    double complex er = CMPLX(er_re, er_im);
    double s2 = 1.0 - c * c;
    double complex root = csqrt(er - s2);
    double complex gs = (c - root) / (c + root);
    double complex gp = (er * c - root) / (er * c + root);
    double as = cabs(gs), ap = cabs(gp);
    return 0.5 * (as * as + ap * ap);
}

/* P_r = P_t + 20 log10(lambda / (4 pi L)) + sum_j 10 log10(R_j)  [dBm] */
static double path_power(double ptx, double freq, double L, const double* refl, int k)
{
    double lambda = C0 / freq;
    double p = ptx + 20.0 * log10(lambda / (4.0 * PI_D * L));
    for (int j = 0; j < k; ++j) p += 10.0 * log10(refl[j]);
    return p;
}

static double refl_at(const scene_t* S, const double* er, const double* ei, int32_t f, v3 din)
{
    double c = fabs(dot(din, S->fn[f])) / norm(din);
    int32_t mt = S->fmat[f];
    return orc_fresnel_avg(c, er[mt], ei[mt]);
}

/* Point inside a face: inside any triangle of the face, barycentric
 * coordinates with tolerance 1e-9. */
static int inside_face(const scene_t* S, int32_t f, v3 p)
{
    const double tol = 1e-9;
    for (int64_t i = 0; i < S->T; ++i) {
        if (S->face[i] != f) continue;
        v3 w = sub(p, S->v0[i]);
        double d00 = dot(S->e1[i], S->e1[i]);
        double d01 = dot(S->e1[i], S->e2[i]);
        double d11 = dot(S->e2[i], S->e2[i]);
        double d20 = dot(w, S->e1[i]);
        double d21 = dot(w, S->e2[i]);
        double den = d00 * d11 - d01 * d01;
        if (den == 0.0) continue;
        double b = (d11 * d20 - d01 * d21) / den;
        double g = (d00 * d21 - d01 * d20) / den;
        if (b >= -tol && g >= -tol && b + g <= 1.0 + tol) return 1;
    }
    return 0;
}

/* Segment A -> B blocked by any triangle not of faces fa / fb, hit strictly
 * inside (1e-9, 1 - 1e-9) of the segment parameter. */
static int blocked(const scene_t* S, v3 A, v3 B, int32_t fa, int32_t fb)
{
    v3 d = sub(B, A);
    for (int64_t i = 0; i < S->T; ++i) {
        int32_t f = S->face[i];
        if (f == fa || f == fb) continue;
        double t;
        if (mt_hit(S, i, A, d, 1e-9, 1.0 - 1e-9, &t)) return 1;
    }
    return 0;
}

/* Exact path for a face sequence by the image method: images of Tx mirrored
 * across the face planes in order, then back-projection from Rx.  Path test
 * 2 (validity): every back-projection parameter in (0,1), every reflection
 * point inside its face, no segment blocked. */
static int exact_solve(const scene_t* S, v3 tx, v3 rx, int32_t k, const int32_t* faces, v3* pts)
{
    v3 img[ORC_MAX_ORDER + 1];
    img[0] = tx;
    for (int j = 0; j < k; ++j) {
        int32_t f = faces[j];
        if (f < 0 || f >= S->F) return 0;
        v3 n = S->fn[f];
        double dd = dot(n, img[j]) - S->fc[f];
        img[j + 1] = sub(img[j], scl(2.0 * dd, n));
    }
    int ok = 1;
    v3 X = rx;
    for (int j = k - 1; j >= 0; --j) {
        int32_t f = faces[j];
        v3 n = S->fn[f];
        v3 dir = sub(img[j + 1], X);
        double den = dot(n, dir);
        double s = (S->fc[f] - dot(n, X)) / den;
        if (!(s > 0.0 && s < 1.0)) ok = 0;
        pts[j] = add(X, scl(s, dir));
        X = pts[j];
    }
    if (!ok) return 0;
    for (int j = 0; j < k; ++j)
        if (!inside_face(S, faces[j], pts[j])) return 0;
    v3 A = tx;
    int32_t fa = -1;
    for (int j = 0; j < k; ++j) {
        if (blocked(S, A, pts[j], fa, faces[j])) return 0;
        A = pts[j];
        fa = faces[j];
    }
    if (blocked(S, A, rx, fa, -1)) return 0;
    return 1;
}

static double poly_length(v3 tx, const v3* p, int k, v3 rx)
{
    double L = 0.0;
    v3 prev = tx;
    for (int j = 0; j < k; ++j) { L = L + norm(sub(p[j], prev)); prev = p[j]; }
    L = L + norm(sub(rx, prev));
    return L;
}

int orc_exact_path(const double* tri_v, const int32_t* face_id, const int32_t* mat_id,
                   int64_t n_tri, const double* eps_re, const double* eps_im,
                   const double tx[3], const double rx[3], int32_t order,
                   const int32_t* faces, double freq_hz, double ptx,
                   double* points, double* length_m, double* power_dbm, int32_t* valid)
{
    if (order < 0 || order > ORC_MAX_ORDER) return -1;
    scene_t S;
    if (scene_init(&S, tri_v, face_id, mat_id, n_tri)) { scene_free(&S); return -1; }
    v3 T = ld3(tx), R = ld3(rx), p[ORC_MAX_ORDER];
    int ok = exact_solve(&S, T, R, order, faces, p);
    if (valid) *valid = ok;
    double L = poly_length(T, p, order, R);
    if (length_m) *length_m = L;
    double refl[ORC_MAX_ORDER];
    v3 prev = T;
    for (int j = 0; j < order; ++j) {
        refl[j] = refl_at(&S, eps_re, eps_im, faces[j], sub(p[j], prev));
        prev = p[j];
        if (points) st3(points + 3 * j, p[j]);
    }
    if (power_dbm) *power_dbm = path_power(ptx, freq_hz, L, refl, order);
    scene_free(&S);
    return 0;
}

/* ======================================================================== */
/* Analytic Jacobian of the image-method path quantities                     */
/* ======================================================================== */
/* For a face sequence f_0..f_{k-1} with unit normals n_j and offsets c_j
 * (n_j . x = c_j), the mirror across plane j is x -> H_j x + 2 c_j n_j with
 * the Householder matrix H_j = I - 2 n_j n_j^T.  Unfolding:
 *   - the image of Tx, I = M Tx + b with M = H_{k-1} ... H_0, lies on the
 *     straight line through Rx and the last reflection point, so the length
 *     is L = |I - Rx| and the arrival direction AOA = u = (I - Rx) / L;
 *   - the image of Rx across the planes in reverse order, J = M^T Rx + b',
 *     lies on the line of the first segment, so AOD = w = (J - Tx) / D
 *     (D = |J - Tx| = L);
 *   - the segment arriving at reflection j has direction
 *     d_j = H_{j-1} ... H_0 w, incidence cosine cos_j = |d_j . n_j|.
 * Values (as orc_exact_path): delay L / c0, AOD, AOA and
 * P = P_t + 20 log10(lambda / (4 pi L)) + sum_j 10 log10 R_j(cos_j, er_j).
 * Derivatives (x = Tx or Rx), with P_v = I - v v^T:
 *   dL/dTx = M^T u,  dL/dRx = -u,
 *   dAOA/dTx = P_u M / L,  dAOA/dRx = -P_u / L,
 *   dAOD/dTx = -P_w / D,  dAOD/dRx = P_w M^T / D,
 *   dcos_j/dx = sign(d_j . n_j) n_j^T (H_{j-1} ... H_0) dw/dx,
 *   dP/dx = -20 / (ln 10 L) dL/dx + 10 / ln 10 sum_j (dR_j/dcos_j) / R_j dcos_j/dx,
 *   dP/d(re, im) of material m = 10 / ln 10 sum_{j of m} (dR_j/d(re, im)) / R_j.
 * R = (|G_s|^2 + |G_p|^2) / 2 with r = sqrt(er - 1 + c^2),
 * G_s = (c - r) / (c + r), G_p = (er c - r) / (er c + r); by the quotient rule
 *   dG_s = 2 (r dc - c dr) / (c + r)^2,
 *   dG_p = 2 (r d(er c) - er c dr) / (er c + r)^2,
 * with dr = (2 c dc + d er) / (2 r), d(er c) = er dc + c d er, d|G|^2 =
 * 2 Re(conj(G) dG), and d er = 1 for the real part, j for the imaginary. */
static void fresnel_derivs(double c, double complex er, double* R, double* dRdc,
                           double* dRdre, double* dRdim)
{
    double complex r = csqrt(er - (1.0 - c * c));
    double complex gs = (c - r) / (c + r), gp = (er * c - r) / (er * c + r);
    *R = 0.5 * (cabs(gs) * cabs(gs) + cabs(gp) * cabs(gp));
    /* three directions of (dc, d er): (1, 0), (0, 1), (0, j) */
    const double complex dcs[3] = {1.0, 0.0, 0.0};
    const double complex des[3] = {0.0, 1.0, I};
    double out[3];
    for (int q = 0; q < 3; ++q) {
        double complex dc = dcs[q], de = des[q];
        double complex dr = (2.0 * c * dc + de) / (2.0 * r);
        double complex dgs = 2.0 * (r * dc - c * dr) / ((c + r) * (c + r));
        double complex dec = er * dc + c * de;
        double complex dgp = 2.0 * (r * dec - er * c * dr) / ((er * c + r) * (er * c + r));
        out[q] = 0.5 * (2.0 * creal(conj(gs) * dgs) + 2.0 * creal(conj(gp) * dgp));
    }
    *dRdc = out[0];
    *dRdre = out[1];
    *dRdim = out[2];
}

typedef struct { double a[3][3]; } m3;

static m3 m3_id(void)
{
    m3 A;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) A.a[i][j] = i == j ? 1.0 : 0.0;
    return A;
}

static m3 m3_mul(m3 A, m3 B)
{
    m3 C;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int l = 0; l < 3; ++l) s += A.a[i][l] * B.a[l][j];
            C.a[i][j] = s;
        }
    return C;
}

static m3 m3_t(m3 A)
{
    m3 C;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C.a[i][j] = A.a[j][i];
    return C;
}

static m3 householder(v3 n)
{
    const double v[3] = {n.x, n.y, n.z};
    m3 H;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) H.a[i][j] = (i == j ? 1.0 : 0.0) - 2.0 * v[i] * v[j];
    return H;
}

static m3 proj_perp(v3 u)  /* I - u u^T */
{
    return householder(scl(sqrt(0.5), u));
}

static v3 m3_apply(m3 A, v3 x)
{
    return mk(A.a[0][0] * x.x + A.a[0][1] * x.y + A.a[0][2] * x.z,
              A.a[1][0] * x.x + A.a[1][1] * x.y + A.a[1][2] * x.z,
              A.a[2][0] * x.x + A.a[2][1] * x.y + A.a[2][2] * x.z);
}

int orc_path_jacobian(const double* tri_v, const int32_t* face_id, const int32_t* mat_id,
                      int64_t n_tri, const double* eps_re, const double* eps_im, int32_t n_mat,
                      const double tx[3], const double rx[3], int32_t order,
                      const int32_t* faces, double freq_hz, double ptx, double* val,
                      double* jac)
{
    if (order < 0 || order > ORC_MAX_ORDER || n_mat < 0) return -1;
    scene_t S;
    if (scene_init(&S, tri_v, face_id, mat_id, n_tri)) { scene_free(&S); return -1; }
    for (int j = 0; j < order; ++j)
        if (faces[j] < 0 || faces[j] >= S.F || S.fmat[faces[j]] < 0 ||
            S.fmat[faces[j]] >= n_mat) {
            scene_free(&S);
            return -1;
        }
    const int ncol = 6 + 2 * n_mat;
    v3 T = ld3(tx), Rx = ld3(rx);
    /* images and the product of the mirrors */
    m3 H[ORC_MAX_ORDER], M = m3_id();
    v3 img = T;
    for (int j = 0; j < order; ++j) {
        v3 n = S.fn[faces[j]];
        H[j] = householder(n);
        M = m3_mul(H[j], M);
        img = sub(img, scl(2.0 * (dot(n, img) - S.fc[faces[j]]), n));
    }
    v3 jr = Rx;
    for (int j = order - 1; j >= 0; --j) {
        v3 n = S.fn[faces[j]];
        jr = sub(jr, scl(2.0 * (dot(n, jr) - S.fc[faces[j]]), n));
    }
    const m3 Mt = m3_t(M);
    v3 du = sub(img, Rx), dw = sub(jr, T);
    const double L = norm(du), D = norm(dw);
    const v3 u = scl(1.0 / L, du), w = scl(1.0 / D, dw);
    const m3 Pu = proj_perp(u), Pw = proj_perp(w);
    /* dw/dTx = -Pw / D, dw/dRx = Pw M^T / D; dL/dTx = M^T u, dL/dRx = -u */
    m3 dw_t, dw_r = m3_mul(Pw, Mt);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            dw_t.a[i][j] = -Pw.a[i][j] / D;
            dw_r.a[i][j] /= D;
        }
    const v3 dL_t = m3_apply(Mt, u), dL_r = scl(-1.0, u);
    const m3 dA_t = m3_mul(Pu, M);
    for (int c = 0; c < 8 * ncol; ++c) jac[c] = 0.0;
    /* values */
    val[0] = L / C0;
    val[1] = w.x; val[2] = w.y; val[3] = w.z;
    val[4] = u.x; val[5] = u.y; val[6] = u.z;
    const double lambda = C0 / freq_hz, k10 = 10.0 / log(10.0);
    double P = ptx + 20.0 * log10(lambda / (4.0 * PI_D * L));
    /* delay, AOD, AOA rows */
    const double dLv_t[3] = {dL_t.x, dL_t.y, dL_t.z}, dLv_r[3] = {dL_r.x, dL_r.y, dL_r.z};
    for (int a = 0; a < 3; ++a) {
        jac[0 * ncol + a] = dLv_t[a] / C0;
        jac[0 * ncol + 3 + a] = dLv_r[a] / C0;
        for (int i = 0; i < 3; ++i) {
            jac[(1 + i) * ncol + a] = dw_t.a[i][a];
            jac[(1 + i) * ncol + 3 + a] = dw_r.a[i][a];
            jac[(4 + i) * ncol + a] = dA_t.a[i][a] / L;
            jac[(4 + i) * ncol + 3 + a] = -Pu.a[i][a] / L;
        }
        /* Friis */
        jac[7 * ncol + a] = -2.0 * k10 / L * dLv_t[a];
        jac[7 * ncol + 3 + a] = -2.0 * k10 / L * dLv_r[a];
    }
    /* reflections */
    m3 A = m3_id();  /* H_{j-1} ... H_0 */
    for (int j = 0; j < order; ++j) {
        const v3 n = S.fn[faces[j]];
        const v3 d = m3_apply(A, w);
        const double dn = dot(d, n), cj = fabs(dn), sg = dn >= 0.0 ? 1.0 : -1.0;
        const int32_t m = S.fmat[faces[j]];
        double Rj, dRdc, dRdre, dRdim;
        fresnel_derivs(cj, CMPLX(eps_re[m], eps_im[m]), &Rj, &dRdc, &dRdre, &dRdim);
        P += 10.0 * log10(Rj);
        /* n^T A, then times dw/dx */
        const v3 g = m3_apply(m3_t(A), n);
        for (int a = 0; a < 3; ++a) {
            const double dct = sg * (g.x * dw_t.a[0][a] + g.y * dw_t.a[1][a] + g.z * dw_t.a[2][a]);
            const double dcr = sg * (g.x * dw_r.a[0][a] + g.y * dw_r.a[1][a] + g.z * dw_r.a[2][a]);
            jac[7 * ncol + a] += k10 * dRdc / Rj * dct;
            jac[7 * ncol + 3 + a] += k10 * dRdc / Rj * dcr;
        }
        jac[7 * ncol + 6 + 2 * m] += k10 * dRdre / Rj;
        jac[7 * ncol + 6 + 2 * m + 1] += k10 * dRdim / Rj;
        A = m3_mul(H[j], A);
    }
    val[7] = P;
    scene_free(&S);
    return 0;
}

/* ======================================================================== */
/* Whole method                                                              */
/* ======================================================================== */
typedef struct { orc_candidate* a; int64_t n, cap; } cvec;
static int cpush(cvec* v, const orc_candidate* c)
{
    if (v->n == v->cap) {
        int64_t nc = v->cap ? 2 * v->cap : 256;
        orc_candidate* p = (orc_candidate*)realloc(v->a, sizeof(orc_candidate) * (size_t)nc);
        if (!p) return -2;
        v->a = p;
        v->cap = nc;
    }
    v->a[v->n++] = *c;
    return 0;
}

static int ray_order_cmp(const void* pa, const void* pb)
{
    const orc_candidate *a = (const orc_candidate*)pa, *b = (const orc_candidate*)pb;
    if (a->ray != b->ray) return a->ray < b->ray ? -1 : 1;
    if (a->order != b->order) return a->order < b->order ? -1 : 1;
    if (a->rx != b->rx) return a->rx < b->rx ? -1 : 1;
    return 0;
}

/* Step 1 for one launch ray r: trace it (Sec. III.A) and append a reception
 * event for every (segment, Rx) pair that passes the cone test, eq. (3). */
static void ray_events(const scene_t* S, v3 TX, const grid_t* G, int64_t r, int32_t K,
                       const double* rx, int32_t n_rx, double thl, cvec* out)
{
    seg_t segs[ORC_MAX_ORDER + 1];
    int ns = trace_ray(S, TX, grid_dir(G, r), K, segs);
    orc_candidate c;
    memset(&c, 0, sizeof(c));
    c.ray = r;
    for (int j = 0; j < ns; ++j) {
        c.order = j;
        for (int q = 0; q < ORC_MAX_ORDER; ++q)
            c.face[q] = q < j ? S->face[segs[q].tri] : -1;
        for (int32_t x = 0; x < n_rx; ++x) {
            double tn;
            if (!capture_seg(&segs[j], ld3(rx + 3 * x), thl, &tn)) continue;
            c.rx = x;
            c.tan_err = tn;
            cpush(out, &c);
        }
    }
}

/* Steps 3-4 for one path-test-1 winner c: the precise algorithm (Sec. III.B)
 * from c's launch ray, the refined path's quantities (Sec. IV), the exact
 * image-method solve and path test 2.  Fills *o; returns the validity. */
static int path_record(const scene_t* S, v3 TX, const grid_t* G, const double* rx,
                       const orc_candidate* c, const orc_params* P, const double* eps_re,
                       const double* eps_im, double tan_tgt, double thl, orc_path* o)
{
    v3 R = ld3(rx + 3 * c->rx);
    refine_t rf;
    refine_path(S, TX, R, c->order, c->face, grid_dir(G, c->ray), P->iterations, P->subrays,
                tan_tgt, thl, &rf, NULL);
    o->rx = c->rx;
    o->order = c->order;
    for (int q = 0; q < ORC_MAX_ORDER; ++q) o->face[q] = c->face[q];
    o->launch_ray = c->ray;
    o->iters_used = rf.iters;
    o->flags = rf.flags;
    o->init_tan_err = c->tan_err;
    o->tan_err = rf.tan_err;
    st3(o->axis, rf.axis);
    const int k = c->order;
    /* refined path: Tx -> hit points of the final axis ray -> Rx */
    double L = poly_length(TX, rf.fw.p, k, R);
    o->length_m = L;
    o->delay_s = L / C0;
    st3(o->aod, rf.axis);
    v3 last = k > 0 ? rf.fw.p[k - 1] : TX;
    st3(o->aoa, normalize(sub(last, R)));
    double refl[ORC_MAX_ORDER];
    for (int j = 0; j < k; ++j) refl[j] = refl_at(S, eps_re, eps_im, c->face[j], rf.fw.din[j]);
    o->power_dbm = path_power(P->tx_power_dbm, P->freq_hz, L, refl, k);
    o->err_angle_deg = atan_cr(rf.tan_err) * (180.0 / PI_D);
    /* exact path for the same faces */
    v3 ep[ORC_MAX_ORDER];
    int ok = exact_solve(S, TX, R, k, c->face, ep);
    double EL = poly_length(TX, ep, k, R);
    o->exact_length_m = EL;
    o->exact_delay_s = EL / C0;
    v3 first = k > 0 ? ep[0] : R;
    st3(o->exact_aod, normalize(sub(first, TX)));
    v3 elast = k > 0 ? ep[k - 1] : TX;
    st3(o->exact_aoa, normalize(sub(elast, R)));
    v3 prev = TX;
    for (int j = 0; j < k; ++j) {
        refl[j] = refl_at(S, eps_re, eps_im, c->face[j], sub(ep[j], prev));
        prev = ep[j];
    }
    o->exact_power_dbm = path_power(P->tx_power_dbm, P->freq_hz, EL, refl, k);
    if (!ok) o->flags |= 2u;
    return ok;
}

int orc_run(const double* tri_v, const int32_t* face_id, const int32_t* mat_id,
            int64_t T, const double* eps_re, const double* eps_im, int32_t n_mat,
            const double tx[3], const double* rx, int32_t n_rx, const orc_params* P,
            orc_candidate** cand_out, int64_t* n_cand_out,
            orc_candidate** uniq_out, int64_t* n_uniq_out,
            orc_path** paths_out, int64_t* n_paths_out)
{
    if (!P || P->division_n < 1 || P->max_order < 0 || P->max_order > ORC_MAX_ORDER ||
        P->iterations < 0 || (P->subrays != 6 && P->subrays != 7) || n_rx < 0 || T < 0 ||
        !(P->freq_hz > 0.0) || P->launch < 0 || P->launch > ORC_LAUNCH_EQUIDISTANT_OCTA)
        return -1;
    for (int64_t i = 0; i < T; ++i)
        if (mat_id && (mat_id[i] < 0 || mat_id[i] >= n_mat)) return -1;
    scene_t S;
    if (scene_init(&S, tri_v, face_id, mat_id, T)) { scene_free(&S); return -1; }
    const int32_t n = P->division_n, K = P->max_order;
    const int64_t N = orc_num_rays_m(P->launch, n);
    const double thl = theta_launch_m(P->launch, n);
    const v3 TX = ld3(tx);
    grid_t G;
    grid_init_m(&G, P->launch, n);
#ifdef _OPENMP
    if (P->n_threads > 0) omp_set_num_threads(P->n_threads);
    int nth = omp_get_max_threads();
#else
    int nth = 1;
#endif
    /* 1. launch, trace and capture every ray */
    cvec* tv = (cvec*)calloc((size_t)nth, sizeof(cvec));
#pragma omp parallel
    {
#ifdef _OPENMP
        int me = omp_get_thread_num();
#else
        int me = 0;
#endif
#pragma omp for schedule(dynamic, 256)
        for (int64_t r = 0; r < N; ++r) ray_events(&S, TX, &G, r, K, rx, n_rx, thl, &tv[me]);
    }
    int64_t nc = 0;
    for (int t = 0; t < nth; ++t) nc += tv[t].n;
    orc_candidate* cand = (orc_candidate*)malloc(sizeof(orc_candidate) * (size_t)(nc > 0 ? nc : 1));
    nc = 0;
    for (int t = 0; t < nth; ++t) {
        if (tv[t].n) memcpy(cand + nc, tv[t].a, sizeof(orc_candidate) * (size_t)tv[t].n);
        nc += tv[t].n;
        free(tv[t].a);
    }
    free(tv);
    qsort(cand, (size_t)nc, sizeof(orc_candidate), ray_order_cmp);

    /* 2. path test 1 */
    orc_candidate* srt = (orc_candidate*)malloc(sizeof(orc_candidate) * (size_t)(nc > 0 ? nc : 1));
    if (nc) memcpy(srt, cand, sizeof(orc_candidate) * (size_t)nc);
    qsort(srt, (size_t)nc, sizeof(orc_candidate), cand_cmp);
    int64_t nu = 0;
    for (int64_t i = 0; i < nc; ++i)
        if (i == 0 || key_cmp(&srt[i], &srt[nu - 1]) != 0) srt[nu++] = srt[i];

    /* 3. precise algorithm, 4. path quantities and path test 2 */
    double tan_tgt = 0.0;
    if (P->target_err_deg > 0.0) tan_tgt = tan_cr((P->target_err_deg * PI_D) / 180.0);
    orc_path* out = (orc_path*)calloc((size_t)(nu > 0 ? nu : 1), sizeof(orc_path));
    int32_t* keep = (int32_t*)calloc((size_t)(nu > 0 ? nu : 1), sizeof(int32_t));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nu; ++i) {
        keep[i] = path_record(&S, TX, &G, rx, &srt[i], P, eps_re, eps_im, tan_tgt, thl, &out[i]) ||
                  P->keep_invalid;
    }
    int64_t np = 0;
    for (int64_t i = 0; i < nu; ++i)
        if (keep[i]) out[np++] = out[i];
    free(keep);
    grid_free(&G);
    scene_free(&S);

    if (cand_out) *cand_out = cand; else free(cand);
    if (n_cand_out) *n_cand_out = nc;
    if (uniq_out) *uniq_out = srt; else free(srt);
    if (n_uniq_out) *n_uniq_out = nu;
    if (paths_out) *paths_out = out; else free(out);
    if (n_paths_out) *n_paths_out = np;
    return 0;
}

void orc_free(void* p) { free(p); }

int orc_ray_events(const double* tri_v, const int32_t* face_id, int64_t T, const double tx[3],
                   int32_t n, int32_t launch, int32_t K, const double* rx, int32_t n_rx,
                   const int64_t* ids, int64_t m, int32_t n_threads, orc_candidate** out,
                   int64_t* n_out)
{
    if (n < 1 || K < 0 || K > ORC_MAX_ORDER || T < 0 || n_rx < 0 || m < 0 || !ids || !out ||
        !n_out || launch < 0 || launch > ORC_LAUNCH_EQUIDISTANT_OCTA)
        return -1;
    const int64_t N = orc_num_rays_m(launch, n);
    for (int64_t i = 0; i < m; ++i)
        if (ids[i] < 0 || ids[i] >= N) return -1;
    scene_t S;
    if (scene_init(&S, tri_v, face_id, NULL, T)) { scene_free(&S); return -1; }
    grid_t G;
    grid_init_m(&G, launch, n);
    const double thl = theta_launch_m(launch, n);
    const v3 TX = ld3(tx);
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
    cvec* per = (cvec*)calloc((size_t)(m > 0 ? m : 1), sizeof(cvec));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < m; ++i) ray_events(&S, TX, &G, ids[i], K, rx, n_rx, thl, &per[i]);
    int64_t nc = 0;
    for (int64_t i = 0; i < m; ++i) nc += per[i].n;
    orc_candidate* all = (orc_candidate*)malloc(sizeof(orc_candidate) * (size_t)(nc > 0 ? nc : 1));
    nc = 0;
    for (int64_t i = 0; i < m; ++i) {
        if (per[i].n) memcpy(all + nc, per[i].a, sizeof(orc_candidate) * (size_t)per[i].n);
        nc += per[i].n;
        free(per[i].a);
    }
    free(per);
    grid_free(&G);
    scene_free(&S);
    *out = all;
    *n_out = nc;
    return 0;
}

int orc_path_test1(const orc_candidate* in, int64_t n, orc_candidate** out, int64_t* n_out)
{
    if (n < 0 || (n > 0 && !in) || !out || !n_out) return -1;
    orc_candidate* srt = (orc_candidate*)malloc(sizeof(orc_candidate) * (size_t)(n > 0 ? n : 1));
    if (!srt) return -2;
    if (n) memcpy(srt, in, sizeof(orc_candidate) * (size_t)n);
    qsort(srt, (size_t)n, sizeof(orc_candidate), cand_cmp);
    int64_t nu = 0;
    for (int64_t i = 0; i < n; ++i)
        if (i == 0 || key_cmp(&srt[i], &srt[nu - 1]) != 0) srt[nu++] = srt[i];
    *out = srt;
    *n_out = nu;
    return 0;
}

int orc_path_records(const double* tri_v, const int32_t* face_id, const int32_t* mat_id,
                     int64_t T, const double* eps_re, const double* eps_im, int32_t n_mat,
                     const double tx[3], const double* rx, int32_t n_rx, const orc_params* P,
                     const orc_candidate* win, int64_t m, orc_path* out)
{
    if (!P || P->division_n < 1 || P->max_order < 0 || P->max_order > ORC_MAX_ORDER ||
        P->iterations < 0 || (P->subrays != 6 && P->subrays != 7) || n_rx < 0 || T < 0 ||
        m < 0 || !(P->freq_hz > 0.0) || P->launch < 0 || P->launch > ORC_LAUNCH_EQUIDISTANT_OCTA)
        return -1;
    const int64_t N = orc_num_rays_m(P->launch, P->division_n);
    for (int64_t i = 0; i < T; ++i)
        if (mat_id && (mat_id[i] < 0 || mat_id[i] >= n_mat)) return -1;
    for (int64_t i = 0; i < m; ++i)
        if (win[i].rx < 0 || win[i].rx >= n_rx || win[i].order < 0 ||
            win[i].order > P->max_order || win[i].ray < 0 || win[i].ray >= N)
            return -1;
    scene_t S;
    if (scene_init(&S, tri_v, face_id, mat_id, T)) { scene_free(&S); return -1; }
    grid_t G;
    grid_init_m(&G, P->launch, P->division_n);
    const double thl = theta_launch_m(P->launch, P->division_n);
    double tan_tgt = 0.0;
    if (P->target_err_deg > 0.0) tan_tgt = tan_cr((P->target_err_deg * PI_D) / 180.0);
#ifdef _OPENMP
    if (P->n_threads > 0) omp_set_num_threads(P->n_threads);
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < m; ++i)
        (void)path_record(&S, ld3(tx), &G, rx, &win[i], P, eps_re, eps_im, tan_tgt, thl, &out[i]);
    grid_free(&G);
    scene_free(&S);
    return 0;
}

int orc_refine_history(const double* tri_v, const int32_t* face_id, int64_t T,
                       const double tx[3], const orc_params* P,
                       const double* rx, const int32_t* order, const int32_t* faces,
                       const double* axis0, int64_t m, double* hist)
{
    if (!P || P->division_n < 1 || (P->subrays != 6 && P->subrays != 7) || P->iterations < 0)
        return -1;
    scene_t S;
    if (scene_init(&S, tri_v, face_id, NULL, T)) { scene_free(&S); return -1; }
    const double thl = theta_launch_m(P->launch, P->division_n);
    const int32_t n_it = P->iterations;
#ifdef _OPENMP
    if (P->n_threads > 0) omp_set_num_threads(P->n_threads);
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < m; ++i) {
        refine_t rf;
        double* h = hist + i * (n_it + 1);
        for (int32_t q = 0; q <= n_it; ++q) h[q] = NAN;
        refine_path(&S, ld3(tx), ld3(rx + 3 * i), order[i], faces + ORC_MAX_ORDER * i,
                    ld3(axis0 + 3 * i), n_it, P->subrays, 0.0, thl, &rf, h);
    }
    scene_free(&S);
    return 0;
}

/* ======================================================================== */
/* Order-1 diffraction -- Sec. III.A ("faces or wedges"), Sec. III.B         */
/* (recorded diffraction directions), Sec. IV (order-1 diffraction paths)    */
/* ======================================================================== */
/* Reading: a wedge is a mesh edge (two endpoints with exactly equal
 * coordinates) shared by triangles of exactly two faces whose planes meet at
 * an angle of at least 10 degrees (|n0 . n1| <= cos 10 deg).  Its endpoints
 * are ordered lexicographically (x, then y, then z), a < b; wedges are listed
 * in that order of (a, b).  e = (b - a) / |b - a|.  For each of its faces
 * (f0 < f1) u_k is the unit vector in the face's plane, normal to the edge,
 * pointing into the face (toward the third vertex of the face's
 * lowest-index triangle on the edge). */
static const double COS_WEDGE = 0.984807753012208; /* cos(10 deg), nearest double */

typedef struct {
    v3 a, b, e, u0, u1;
    double len;
    int32_t f0, f1;
} wedge_t;

typedef struct {
    double lo[3], hi[3];
    int32_t face;
    int64_t tri;
    double c[3];      /* third vertex */
} edge_rec;

static int lex3(const double* p, const double* q)
{
    for (int i = 0; i < 3; ++i)
        if (p[i] != q[i]) return p[i] < q[i] ? -1 : 1;
    return 0;
}

static int edge_cmp(const void* pa, const void* pb)
{
    const edge_rec *a = (const edge_rec*)pa, *b = (const edge_rec*)pb;
    int c = lex3(a->lo, b->lo);
    if (c) return c;
    c = lex3(a->hi, b->hi);
    if (c) return c;
    if (a->face != b->face) return a->face < b->face ? -1 : 1;
    if (a->tri != b->tri) return a->tri < b->tri ? -1 : 1;
    return 0;
}

static v3 in_face_dir(v3 a, v3 e, v3 c)
{
    v3 w = sub(c, a);
    return normalize(sub(w, scl(dot(w, e), e)));
}

/* Wedges of the scene; returns their number (malloc'd array in *out). */
static int64_t wedges_build(const scene_t* S, const double* tri_v, wedge_t** out)
{
    int64_t T = S->T, ne = 3 * T;
    edge_rec* E = (edge_rec*)malloc(sizeof(edge_rec) * (size_t)(ne > 0 ? ne : 1));
    int64_t m = 0;
    for (int64_t i = 0; i < T; ++i)
        for (int k = 0; k < 3; ++k) {
            const double* p = tri_v + 9 * i + 3 * k;
            const double* q = tri_v + 9 * i + 3 * ((k + 1) % 3);
            const double* c = tri_v + 9 * i + 3 * ((k + 2) % 3);
            int o = lex3(p, q);
            if (o == 0) continue;
            edge_rec r;
            memcpy(r.lo, o < 0 ? p : q, sizeof r.lo);
            memcpy(r.hi, o < 0 ? q : p, sizeof r.hi);
            memcpy(r.c, c, sizeof r.c);
            r.face = S->face[i];
            r.tri = i;
            E[m++] = r;
        }
    qsort(E, (size_t)m, sizeof(edge_rec), edge_cmp);
    wedge_t* W = (wedge_t*)malloc(sizeof(wedge_t) * (size_t)(m > 0 ? m : 1));
    int64_t nw = 0;
    for (int64_t i = 0; i < m;) {
        int64_t j = i;
        while (j < m && lex3(E[j].lo, E[i].lo) == 0 && lex3(E[j].hi, E[i].hi) == 0) ++j;
        /* records i..j-1 share the edge, sorted by face then triangle */
        int nf = 0;
        int64_t first[2] = {-1, -1};
        for (int64_t q = i; q < j; ++q)
            if (q == i || E[q].face != E[q - 1].face) {
                if (nf < 2) first[nf] = q;
                ++nf;
            }
        if (nf == 2) {
            const edge_rec *r0 = &E[first[0]], *r1 = &E[first[1]];
            double cs = fabs(dot(S->fn[r0->face], S->fn[r1->face]));
            if (cs <= COS_WEDGE) {
                wedge_t w;
                w.a = ld3(r0->lo);
                w.b = ld3(r0->hi);
                v3 d = sub(w.b, w.a);
                w.len = norm(d);
                w.e = mk(d.x / w.len, d.y / w.len, d.z / w.len);
                w.f0 = r0->face;
                w.f1 = r1->face;
                w.u0 = in_face_dir(w.a, w.e, ld3(r0->c));
                w.u1 = in_face_dir(w.a, w.e, ld3(r1->c));
                W[nw++] = w;
            }
        }
        i = j;
    }
    free(E);
    *out = W;
    return nw;
}

int64_t orc_wedges(const double* tri_v, const int32_t* face_id, int64_t T, double* out,
                   int64_t cap)
{
    if (T < 0 || (T > 0 && (!tri_v || !face_id))) return -1;
    scene_t S;
    if (scene_init(&S, tri_v, face_id, NULL, T)) { scene_free(&S); return -1; }
    wedge_t* W;
    int64_t nw = wedges_build(&S, tri_v, &W);
    for (int64_t i = 0; i < nw && i < cap && out; ++i) {
        double* o = out + 17 * i;
        st3(o, W[i].a); st3(o + 3, W[i].b); st3(o + 6, W[i].e);
        st3(o + 9, W[i].u0); st3(o + 12, W[i].u1);
        o[15] = (double)W[i].f0;
        o[16] = (double)W[i].f1;
    }
    free(W);
    scene_free(&S);
    return nw;
}

/* Inside the wedge: strictly between its two faces, in the sector where both
 * faces lie (the solid side of a convex edge): the part of P - a normal to the
 * edge is b u0 + c u1 with b > 0 and c > 0. */
static int wedge_interior(const wedge_t* W, v3 P)
{
    v3 v = sub(P, W->a);
    v3 r = sub(v, scl(dot(v, W->e), W->e));
    double g = dot(W->u0, W->u1);
    double r0 = dot(r, W->u0), r1 = dot(r, W->u1);
    return (r0 - g * r1 > 0.0) && (r1 - g * r0 > 0.0);
}

/* Closest approach of the ray o + t d and the edge line a + s e:
 * t (along the ray) and s (along the edge); 0 when the lines are (nearly)
 * parallel. */
static int ray_edge(const wedge_t* W, v3 o, v3 d, double* t_out, double* s_out)
{
    v3 w0 = sub(o, W->a);
    double b = dot(d, W->e), dd = dot(d, d), ee = dot(W->e, W->e);
    double dw = dot(d, w0), ew = dot(W->e, w0);
    double den = dd * ee - b * b;
    if (!(den > 1e-12)) return 0;
    *t_out = (b * ew - ee * dw) / den;
    *s_out = (dd * ew - b * dw) / den;
    return 1;
}

/* The receiver unfolded about the edge: Rx rotated about the edge line into
 * the half-plane through the edge opposite Tx.  The exact order-1 diffraction
 * path Tx -> Q -> Rx (equal angles with the edge on both sides, Keller's law)
 * unfolds into the straight line Tx -> Rx', so the angle between a ray and
 * Rx' - Tx is that ray's departure-angle error -- the diffraction reading of
 * eq. (3), as for reflections.  Returns 0 when Tx or Rx lies on the edge
 * line.  *rho_t, *rho_x, *at, *ax: distances from and positions along the
 * edge line. */
static int unfold_rx(const wedge_t* W, v3 tx, v3 rx, v3* rxp, double* at, double* ax,
                     double* rho_t, double* rho_x)
{
    v3 vx = sub(rx, W->a), vt = sub(tx, W->a);
    *ax = dot(vx, W->e);
    *at = dot(vt, W->e);
    v3 rxv = sub(vx, scl(*ax, W->e)), rtv = sub(vt, scl(*at, W->e));
    *rho_x = norm(rxv);
    *rho_t = norm(rtv);
    if (!(*rho_t > 0.0) || !(*rho_x > 0.0)) return 0;
    double k = *rho_x / *rho_t;
    *rxp = sub(add(W->a, scl(*ax, W->e)), scl(k, rtv));
    return 1;
}

/* One ray from Tx in direction d, taken as diffracted at the wedge W toward
 * Rx (its unfolded image rxp): the ray must pass the edge segment
 * (closest approach at t > 0, 0 <= s <= len) and reach it (its first hit is
 * beyond t, or on one of the wedge's own faces, which it clips at the edge);
 * then tan(error angle) is that of rxp on the ray, as in eq. (3) with D = 0.
 * Q is the diffraction point, the edge point nearest the ray. */
struct dfollow_s {
    double tan_err, t, s, delta, L1, L2;
    v3 q;
};

/* The ray from Tx in direction d passes the edge segment (closest approach
 * at t > 0, 0 <= s <= len) and reaches it: its first hit (th, on face fh;
 * fh = -1: none) lies beyond t or on one of the wedge's own faces, which a ray
 * clipping the edge meets there. */
static int ray_reaches_edge(const wedge_t* W, v3 tx, v3 d, double th, int32_t fh, double* t,
                            double* s)
{
    if (!ray_edge(W, tx, d, t, s)) return 0;
    if (!(*t > 0.0) || !(*s >= 0.0) || !(*s <= W->len)) return 0;
    if (fh >= 0 && !(th >= *t) && fh != W->f0 && fh != W->f1) return 0;
    return 1;
}

static int follow_diff(const scene_t* S, const wedge_t* W, v3 tx, v3 d, v3 rx, v3 rxp,
                       dfollow_t* F)
{
    double th, t, s;
    int64_t hit = closest_hit(S, tx, d, -1, &th);
    if (!ray_reaches_edge(W, tx, d, th, hit < 0 ? -1 : S->face[hit], &t, &s)) return 0;
    v3 w = sub(rxp, tx);
    double ts = dot(w, d);
    if (!(ts > 0.0)) return 0;
    v3 f = sub(w, scl(ts, d));
    double dp = norm(f);
    v3 p = add(tx, scl(t, d));
    F->q = add(W->a, scl(s, W->e));
    F->delta = norm(sub(p, F->q));
    F->tan_err = dp / ts;
    F->t = t;
    F->s = s;
    F->L1 = norm(sub(F->q, tx));
    F->L2 = norm(sub(rx, F->q));
    return 1;
}

/* Reception of a diffracted ray (the SBR step), for a ray that passes and
 * reaches the edge (closest approach t, edge point q): the edge crosses the
 * ray cone there (|p - q| <= theta_launch t), and the receiver's unfolded
 * image lies inside the ray cone (tan error <= theta_launch: eq. (3) with
 * D = 0 and the unfolded receiver).  Receivers inside the wedge are skipped
 * before (they are not unfolded). */
static int capture_diff(v3 tx, v3 d, v3 rxp, double thl, double* tan_out)
{
    v3 w = sub(rxp, tx);
    double ts = dot(w, d);
    if (!(ts > 0.0)) return 0;
    v3 f = sub(w, scl(ts, d));
    double dp = norm(f);
    if (!(dp <= thl * ts)) return 0;
    *tan_out = dp / ts;
    return 1;
}

/* Precise algorithm for a diffraction path (Sec. III.B): the sub-ray cones
 * of the reflection paths, each sub-ray diffracted in the recorded direction
 * -- at the same wedge, toward the same receiver -- so only rays that pass
 * that edge and reach it count; the smallest error angle wins. */
typedef struct {
    v3 axis;
    double tan_err;
    int32_t iters;
    uint32_t flags;
    dfollow_t fw;
} drefine_t;

typedef struct {
    const scene_t* S;
    const wedge_t* W;
    v3 tx, rx, rxp;
} diff_ctx;

static int follow_diff_cb(const void* c, v3 d, double* tn, double* D, double* Ll, void* g)
{
    const diff_ctx* x = (const diff_ctx*)c;
    dfollow_t* fw = (dfollow_t*)g;
    if (!follow_diff(x->S, x->W, x->tx, d, x->rx, x->rxp, fw)) return 0;
    *tn = fw->tan_err;
    *D = fw->L1;
    *Ll = fw->L2;
    return 1;
}

static void refine_diff(const scene_t* S, const wedge_t* W, v3 tx, v3 rx, v3 a0, int32_t n_it,
                        int32_t Sn, double tan_tgt, double thl, drefine_t* R, double* hist)
{
    diff_ctx x = {S, W, tx, rx, rx};
    double at, ax, rt, rr;
    refine_state st;
    memset(&R->fw, 0, sizeof(R->fw));
    if (!unfold_rx(W, tx, rx, &x.rxp, &at, &ax, &rt, &rr)) {
        R->axis = a0;
        R->tan_err = NAN;
        R->iters = 0;
        R->flags = 1u;
        if (hist) hist[0] = NAN;
        return;
    }
    dfollow_t tmp, win;
    refine_loop(follow_diff_cb, &x, &R->fw, &tmp, &win, sizeof(dfollow_t), a0, n_it, Sn, tan_tgt,
                thl, &st, hist);
    R->axis = st.axis;
    R->tan_err = st.tan_err;
    R->iters = st.iters;
    R->flags = st.flags;
}

/* Exact order-1 diffraction path (Keller's law: the path makes equal angles
 * with the edge on both sides): Q = a + s e with
 * s = at + (ax - at) rho_t / (rho_t + rho_x).  Path test 2: Q on the edge
 * segment (tolerance 1e-9 of its length), Tx and Rx outside the wedge, both
 * segments unobstructed by any face but the wedge's two. */
static int exact_diff(const scene_t* S, const wedge_t* W, v3 tx, v3 rx, v3* q)
{
    v3 rxp;
    double at, ax, rt, rr;
    if (!unfold_rx(W, tx, rx, &rxp, &at, &ax, &rt, &rr)) {
        *q = W->a;
        return 0;
    }
    double s = at + (ax - at) * (rt / (rt + rr));
    *q = add(W->a, scl(s, W->e));
    const double tol = 1e-9 * W->len;
    if (!(s >= -tol) || !(s <= W->len + tol)) return 0;
    if (wedge_interior(W, tx) || wedge_interior(W, rx)) return 0;
    if (blocked(S, tx, *q, W->f0, W->f1)) return 0;
    if (blocked(S, *q, rx, W->f0, W->f1)) return 0;
    return 1;
}

static void diff_record(const scene_t* S, const wedge_t* W, v3 TX, const grid_t* G,
                        const double* rx, const orc_candidate* c, const orc_params* P,
                        double tan_tgt, double thl, orc_dpath* o)
{
    v3 R = ld3(rx + 3 * c->rx);
    drefine_t rf;
    refine_diff(S, W, TX, R, grid_dir(G, c->ray), P->iterations, P->subrays, tan_tgt, thl, &rf,
                NULL);
    memset(o, 0, sizeof(*o));
    o->rx = c->rx;
    o->wedge = c->face[0];
    o->launch_ray = c->ray;
    o->iters_used = rf.iters;
    o->flags = rf.flags;
    o->init_tan_err = c->tan_err;
    o->tan_err = rf.tan_err;
    st3(o->axis, rf.axis);
    /* refined path: Tx -> the edge point nearest the final ray -> Rx */
    st3(o->point, rf.fw.q);
    double L = rf.fw.L1 + rf.fw.L2;
    o->length_m = L;
    o->delay_s = L / C0;
    st3(o->aod, rf.axis);
    st3(o->aoa, normalize(sub(rf.fw.q, R)));
    o->err_angle_deg = atan_cr(rf.tan_err) * (180.0 / PI_D);
    v3 q;
    int ok = exact_diff(S, W, TX, R, &q);
    st3(o->exact_point, q);
    double EL = norm(sub(q, TX)) + norm(sub(R, q));
    o->exact_length_m = EL;
    o->exact_delay_s = EL / C0;
    st3(o->exact_aod, normalize(sub(q, TX)));
    st3(o->exact_aoa, normalize(sub(q, R)));
    if (!ok) o->flags |= 2u;
}

int orc_diffract(const double* tri_v, const int32_t* face_id, int64_t T, const double tx[3],
                 const double* rx, int32_t n_rx, const orc_params* P, orc_candidate** cand_out,
                 int64_t* n_cand_out, orc_candidate** uniq_out, int64_t* n_uniq_out,
                 orc_dpath** paths_out, int64_t* n_paths_out)
{
    if (!P || P->division_n < 1 || P->iterations < 0 || (P->subrays != 6 && P->subrays != 7) ||
        n_rx < 0 || T < 0 || P->launch < 0 || P->launch > ORC_LAUNCH_EQUIDISTANT_OCTA)
        return -1;
    scene_t S;
    if (scene_init(&S, tri_v, face_id, NULL, T)) { scene_free(&S); return -1; }
    wedge_t* W;
    int64_t nw = wedges_build(&S, tri_v, &W);
    const int32_t n = P->division_n;
    const int64_t N = orc_num_rays_m(P->launch, n);
    const double thl = theta_launch_m(P->launch, n);
    const v3 TX = ld3(tx);
    grid_t G;
    grid_init_m(&G, P->launch, n);
#ifdef _OPENMP
    if (P->n_threads > 0) omp_set_num_threads(P->n_threads);
    int nth = omp_get_max_threads();
#else
    int nth = 1;
#endif
    /* the receivers' images unfolded about each wedge (receivers inside a
     * wedge, or on its edge line, receive nothing from it) */
    v3* rxp = (v3*)malloc(sizeof(v3) * (size_t)(nw * n_rx > 0 ? nw * n_rx : 1));
    char* rxok = (char*)calloc((size_t)(nw * n_rx > 0 ? nw * n_rx : 1), 1);
    for (int64_t w = 0; w < nw; ++w)
        for (int32_t x = 0; x < n_rx; ++x) {
            double at, ax, rt, rr;
            v3 R = ld3(rx + 3 * x);
            rxok[w * n_rx + x] = !wedge_interior(&W[w], R) &&
                                 unfold_rx(&W[w], TX, R, &rxp[w * n_rx + x], &at, &ax, &rt, &rr);
        }
    /* 1. launch; every ray that passes a wedge, reaches it and whose cone
     * the edge crosses diffracts there toward every receiver its cone
     * captures */
    cvec* tv = (cvec*)calloc((size_t)nth, sizeof(cvec));
#pragma omp parallel
    {
#ifdef _OPENMP
        int me = omp_get_thread_num();
#else
        int me = 0;
#endif
#pragma omp for schedule(dynamic, 256)
        for (int64_t r = 0; r < N; ++r) {
            v3 d = grid_dir(&G, r);
            double th;
            int64_t hit = closest_hit(&S, TX, d, -1, &th);
            int32_t fh = hit < 0 ? -1 : S.face[hit];
            orc_candidate c;
            memset(&c, 0, sizeof(c));
            c.ray = r;
            c.order = 1;
            for (int q = 1; q < ORC_MAX_ORDER; ++q) c.face[q] = -1;
            for (int64_t w = 0; w < nw; ++w) {
                double t, s;
                if (!ray_reaches_edge(&W[w], TX, d, th, fh, &t, &s)) continue;
                v3 p = add(TX, scl(t, d));
                v3 q = add(W[w].a, scl(s, W[w].e));
                if (!(norm(sub(p, q)) <= thl * t)) continue;
                for (int32_t x = 0; x < n_rx; ++x) {
                    double tn;
                    if (!rxok[w * n_rx + x]) continue;
                    if (!capture_diff(TX, d, rxp[w * n_rx + x], thl, &tn)) continue;
                    c.rx = x;
                    c.face[0] = (int32_t)w;
                    c.tan_err = tn;
                    cpush(&tv[me], &c);
                }
            }
        }
    }
    int64_t nc = 0;
    for (int t = 0; t < nth; ++t) nc += tv[t].n;
    orc_candidate* cand = (orc_candidate*)malloc(sizeof(orc_candidate) * (size_t)(nc > 0 ? nc : 1));
    nc = 0;
    for (int t = 0; t < nth; ++t) {
        if (tv[t].n) memcpy(cand + nc, tv[t].a, sizeof(orc_candidate) * (size_t)tv[t].n);
        nc += tv[t].n;
        free(tv[t].a);
    }
    free(tv);
    qsort(cand, (size_t)nc, sizeof(orc_candidate), ray_order_cmp);
    /* 2. path test 1: one path per (rx, wedge), the smallest error angle */
    orc_candidate* srt;
    int64_t nu;
    orc_path_test1(cand, nc, &srt, &nu);
    /* 3. precise algorithm, 4. path quantities and path test 2 */
    double tan_tgt = 0.0;
    if (P->target_err_deg > 0.0) tan_tgt = tan_cr((P->target_err_deg * PI_D) / 180.0);
    orc_dpath* out = (orc_dpath*)calloc((size_t)(nu > 0 ? nu : 1), sizeof(orc_dpath));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nu; ++i)
        diff_record(&S, &W[srt[i].face[0]], TX, &G, rx, &srt[i], P, tan_tgt, thl, &out[i]);
    int64_t np = 0;
    for (int64_t i = 0; i < nu; ++i)
        if (!(out[i].flags & 2u) || P->keep_invalid) out[np++] = out[i];
    free(rxp);
    free(rxok);
    free(W);
    grid_free(&G);
    scene_free(&S);
    if (cand_out) *cand_out = cand; else free(cand);
    if (n_cand_out) *n_cand_out = nc;
    if (uniq_out) *uniq_out = srt; else free(srt);
    if (n_uniq_out) *n_uniq_out = nu;
    if (paths_out) *paths_out = out; else free(out);
    if (n_paths_out) *n_paths_out = np;
    return 0;
}

int orc_diffract_history(const double* tri_v, const int32_t* face_id, int64_t T,
                         const double tx[3], const orc_params* P, const double* rx,
                         const int32_t* wedge, const double* axis0, int64_t m, double* hist)
{
    if (!P || P->division_n < 1 || (P->subrays != 6 && P->subrays != 7) || P->iterations < 0)
        return -1;
    scene_t S;
    if (scene_init(&S, tri_v, face_id, NULL, T)) { scene_free(&S); return -1; }
    wedge_t* W;
    int64_t nw = wedges_build(&S, tri_v, &W);
    const double thl = theta_launch_m(P->launch, P->division_n);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int64_t i = 0; i < m; ++i) {
        double* h = hist + i * (P->iterations + 1);
        for (int32_t q = 0; q <= P->iterations; ++q) h[q] = NAN;
        if (wedge[i] < 0 || wedge[i] >= nw) { bad = 1; continue; }
        drefine_t rf;
        refine_diff(&S, &W[wedge[i]], ld3(tx), ld3(rx + 3 * i), ld3(axis0 + 3 * i),
                    P->iterations, P->subrays, 0.0, thl, &rf, h);
    }
    free(W);
    scene_free(&S);
    return bad ? -1 : 0;
}
