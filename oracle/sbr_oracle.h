/*
 * sbr_oracle.h -- plain FP64 CPU oracle for the equiangular-launch SBR method
 * with the iterative precise algorithm (Zhou et al., "An Improved Equiangular
 * Division Algorithm for SBR based Ray Tracing Channel Modeling").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this code: only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no source with the HIP implementation.
 *
 * Everything is brute force in FP64 (no BVH, every triangle tested), compiled
 * with -ffp-contract=off so that every +,-,*,/ and sqrt is one IEEE-754
 * correctly rounded operation in the order written.  The few transcendental
 * values that decide geometry (sin/acos of the launch grid) are evaluated in
 * binary128 and rounded once to binary64, i.e. correctly rounded.
 *
 * Conventions (all geometry in metres, FP64):
 *   tri_v   [T][3][3]  triangle vertices v0,v1,v2
 *   face_id [T]        planar polygon id ("face" of the paper, Sec. III.A),
 *                      0 <= face_id < n_faces
 *   mat_id  [T]        material index into eps_re/eps_im
 *   Return codes: 0 ok, -1 invalid argument, -2 out of memory.
 */
#ifndef SBR_ORACLE_H
#define SBR_ORACLE_H
#include <stdint.h>

#define ORC_MAX_ORDER 8

/* Launch methods: the equiangular icosahedral division of Sec. II.B and the
 * equidistant divisions of Sec. II.A on the icosahedron and octahedron. */
#define ORC_LAUNCH_EQUIANGULAR 0
#define ORC_LAUNCH_EQUIDISTANT_ICOSA 1
#define ORC_LAUNCH_EQUIDISTANT_OCTA 2

/* Launch grid: Sec. II.B, eqs. (1)-(2) and the innermost-layer cases;
 * ray count 10 n^2 + 2 stated with eq. (4). */
int64_t orc_num_rays(int32_t n);
/* Directions for ray indices ids[0..m-1] (ids == NULL: all rays in order). */
int orc_launch_dirs(int32_t n, const int64_t* ids, int64_t m, double* out_xyz);
/* The same for any launch method (4 n^2 + 2 rays for the octahedron). */
int64_t orc_num_rays_m(int32_t method, int32_t n);
int orc_launch_dirs_m(int32_t method, int32_t n, const int64_t* ids, int64_t m, double* out_xyz);
/* Correctly rounded helpers exposed for pin tests. */
double orc_sin_cr(double x);
double orc_acos_cr(double x);

typedef struct {
    int32_t max_order;      /* K: reflections per ray, 0..8                   */
    int32_t division_n;     /* n: 10 n^2 + 2 launch rays                      */
    int32_t iterations;     /* I: precise-algorithm iterations (cap if target) */
    int32_t subrays;        /* 6 (paper) or 7 (axis kept)                      */
    double  target_err_deg; /* <= 0: run exactly I iterations                  */
    double  freq_hz;
    double  tx_power_dbm;
    int32_t keep_invalid;   /* keep paths that fail the validity test          */
    int32_t n_threads;      /* OpenMP threads, <= 0: runtime default           */
    int32_t launch;         /* ORC_LAUNCH_*                                    */
} orc_params;

typedef struct {
    int32_t rx, order, face[ORC_MAX_ORDER];
    int64_t launch_ray;
    int32_t iters_used;
    uint32_t flags;            /* 1 STALLED, 2 INVALID, 4 TARGET_MET          */
    double tan_err;            /* tan(theta_error) of the reported axis       */
    double axis[3];            /* reported departure direction (AOD)          */
    double delay_s, aod[3], aoa[3], power_dbm, err_angle_deg, length_m;
    double exact_delay_s, exact_aod[3], exact_aoa[3], exact_power_dbm, exact_length_m;
    double init_tan_err;       /* tan(theta_error) of the dedup winner        */
} orc_path;

typedef struct {
    int32_t rx, order, face[ORC_MAX_ORDER];
    int64_t ray;
    double tan_err;
} orc_candidate;

/* Per-ray closest hits of segments 0..K (ray "ids", or all if ids == NULL):
 * out_tri/out_face [m][K+1] (-1 = no hit), out_t [m][K+1] (+inf = no hit). */
int orc_trace_rays(const double* tri_v, const int32_t* face_id, int64_t n_tri,
                   const double tx[3], int32_t n, int32_t launch, int32_t max_order,
                   const int64_t* ids, int64_t m, int32_t n_threads,
                   int32_t* out_tri, int32_t* out_face, double* out_t);

/* Same for explicit directions dirs[m][3]; out_D = unfolded length at the
 * start of each segment. */
int orc_trace_dirs(const double* tri_v, const int32_t* face_id, int64_t n_tri,
                   const double tx[3], const double* dirs, int64_t m, int32_t max_order,
                   int32_t* out_tri, int32_t* out_face, double* out_t, double* out_D);

/* Full method.  Candidates and paths are returned in malloc'd arrays that the
 * caller releases with orc_free.  Any output pointer may be NULL. */
int orc_run(const double* tri_v, const int32_t* face_id, const int32_t* mat_id,
            int64_t n_tri, const double* eps_re, const double* eps_im, int32_t n_mat,
            const double tx[3], const double* rx, int32_t n_rx, const orc_params* prm,
            orc_candidate** cand, int64_t* n_cand,
            orc_candidate** uniq, int64_t* n_uniq,
            orc_path** paths, int64_t* n_paths);
void orc_free(void* p);

/* Step 1 alone for the launch rays ids[0..m-1]: their reception events, in
 * the order (ids order, segment, rx), returned in a malloc'd array. */
int orc_ray_events(const double* tri_v, const int32_t* face_id, int64_t n_tri,
                   const double tx[3], int32_t n, int32_t launch, int32_t max_order,
                   const double* rx,
                   int32_t n_rx, const int64_t* ids, int64_t m, int32_t n_threads,
                   orc_candidate** out, int64_t* n_out);

/* Path test 1 alone: of the events in[0..n-1], one per (rx, order, face
 * sequence), the smallest tan_err (ties: lowest ray), sorted by that key;
 * returned in a malloc'd array. */
int orc_path_test1(const orc_candidate* in, int64_t n, orc_candidate** out, int64_t* n_out);

/* Steps 3-4 alone for given path-test-1 winners win[0..m-1] (rx, order,
 * faces, launch ray, tan_err): out[i] is the record orc_run produces for
 * that winner, with the INVALID flag set but nothing dropped. */
int orc_path_records(const double* tri_v, const int32_t* face_id, const int32_t* mat_id,
                     int64_t n_tri, const double* eps_re, const double* eps_im, int32_t n_mat,
                     const double tx[3], const double* rx, int32_t n_rx, const orc_params* prm,
                     const orc_candidate* win, int64_t m, orc_path* out);

/* Precise algorithm on given (rx, face sequence, start axis, start tan) rows;
 * records tan(theta_error) after every iteration in err_hist[row][0..iters]. */
int orc_refine_history(const double* tri_v, const int32_t* face_id, int64_t n_tri,
                       const double tx[3], const orc_params* prm,
                       const double* rx /* [m][3] */, const int32_t* order,
                       const int32_t* faces /* [m][8] */,
                       const double* axis0 /* [m][3] */, int64_t m,
                       double* err_hist /* [m][iterations+1], NaN = no candidate */);

/* Exact image-method solve for one face sequence (validity test + geometry). */
int orc_exact_path(const double* tri_v, const int32_t* face_id, const int32_t* mat_id,
                   int64_t n_tri, const double* eps_re, const double* eps_im,
                   const double tx[3], const double rx[3], int32_t order,
                   const int32_t* faces, double freq_hz, double tx_power_dbm,
                   double* points /* [order][3] */, double* length_m,
                   double* power_dbm, int32_t* valid);

/* Values and analytic Jacobian of the image-method path quantities for one
 * face sequence: val[8] = delay (s), AOD (3), AOA (3), power (dBm) as
 * orc_exact_path computes them; jac[8][6 + 2 n_mat] = d val / d(Tx (3), Rx
 * (3), (re, im) of each material's permittivity).  Returns -1 on bad
 * arguments (order, face ids, materials). */
int orc_path_jacobian(const double* tri_v, const int32_t* face_id, const int32_t* mat_id,
                      int64_t n_tri, const double* eps_re, const double* eps_im, int32_t n_mat,
                      const double tx[3], const double rx[3], int32_t order,
                      const int32_t* faces, double freq_hz, double ptx, double* val,
                      double* jac);

/* ---- Order-1 diffraction (Sec. III.A wedges, Sec. III.B, Sec. IV) ---- */
/* Wedges: out [cap][17] = a[3], b[3], e[3], u0[3], u1[3], f0, f1 (as doubles);
 * returns the number of wedges (all of them even when cap is smaller). */
int64_t orc_wedges(const double* tri_v, const int32_t* face_id, int64_t n_tri, double* out,
                   int64_t cap);

/* One order-1 diffraction path: Tx -> point on the edge of `wedge` -> Rx. */
typedef struct {
    int32_t rx, wedge;
    int64_t launch_ray;
    int32_t iters_used;
    uint32_t flags;            /* 1 STALLED, 2 INVALID, 4 TARGET_MET          */
    double tan_err, axis[3], point[3], delay_s, aod[3], aoa[3], err_angle_deg, length_m;
    double exact_point[3], exact_delay_s, exact_aod[3], exact_aoa[3], exact_length_m;
    double init_tan_err;
} orc_dpath;

/* The whole method for order-1 diffraction paths.  Events and winners use
 * orc_candidate with order 1 and face[0] = wedge index. */
int orc_diffract(const double* tri_v, const int32_t* face_id, int64_t n_tri, const double tx[3],
                 const double* rx, int32_t n_rx, const orc_params* prm,
                 orc_candidate** cand, int64_t* n_cand, orc_candidate** uniq, int64_t* n_uniq,
                 orc_dpath** paths, int64_t* n_paths);

/* Precise algorithm of diffraction rows (rx[m][3], wedge[m], start axis);
 * tan(theta_error) after every iteration in hist[m][iterations + 1]. */
int orc_diffract_history(const double* tri_v, const int32_t* face_id, int64_t n_tri,
                         const double tx[3], const orc_params* prm, const double* rx,
                         const int32_t* wedge, const double* axis0, int64_t m, double* hist);

/* Fresnel average power reflectance 0.5(|G_perp|^2+|G_par|^2) for cos(theta_i). */
double orc_fresnel_avg(double cos_i, double eps_re, double eps_im);

#endif
