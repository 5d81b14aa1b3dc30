/*
 * sbr.h -- C ABI of the MI355X (gfx950) shooting-and-bouncing-ray tracer with
 * equiangular launch and the iterative precise algorithm of Zhou et al.,
 * "An Improved Equiangular Division Algorithm for SBR based Ray Tracing
 * Channel Modeling" (arXiv 2208.10009).
 *
 * The problem (Sec. I and Sec. IV): given a scene of planar faces with
 * materials, one transmitter (Tx) and a set of receivers (Rx), return the
 * propagation paths with their delay, angle of departure (AOD), angle of
 * arrival (AOA) and power.  Every stage of the computation runs in HIP
 * kernels on one GPU; the host only validates arguments, builds the BVH and
 * moves inputs and results.
 *
 * Conventions shared by every entry point:
 *  - All geometry is FP64, metres, right-handed; inputs are caller-owned host
 *    arrays, read during the call and never retained.
 *  - Outputs are caller-allocated host arrays.  Calls that return a list take
 *    a capacity; when it is too small they return SBR_E_CAPACITY, write the
 *    required count to *n_out and nothing else.
 *  - Every call is synchronous: results are complete on return (except
 *    sbr_path_gradients, which works on device arrays in stream order).
 *  - On error nothing is left half-built; sbr_last_error() gives a message.
 *  - A context is bound to one device and one HIP stream and must be used by
 *    one thread at a time.  Scenes belong to the context that created them.
 */
#ifndef SBR_H
#define SBR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SBR_MAX_ORDER 8 /* highest reflection order a path may have */

typedef int32_t sbr_status;
#define SBR_OK 0
#define SBR_E_INVALID_ARG (-1) /* a pointer, size or parameter is out of range   */
#define SBR_E_NO_SCENE (-2)    /* scene handle is NULL or destroyed              */
#define SBR_E_NO_BVH (-3)      /* sbr_bvh_build was not called on the scene      */
#define SBR_E_CAPACITY (-4)    /* output too small; *n_out = required count      */
#define SBR_E_OOM (-5)         /* device or host allocation failed               */
#define SBR_E_DEVICE (-6)      /* a HIP call failed (message has the HIP error)  */
#define SBR_E_INTERNAL (-7)    /* internal consistency check failed              */
#define SBR_E_SCRATCH (-8)     /* sbr_trace_device_noalloc: the call needs more
                                  than its fixed scratch holds                    */

typedef struct sbr_context sbr_context;
typedef struct sbr_scene sbr_scene;

/* Relative permittivity er = re + j im of a material (e^{jwt} convention, so
 * lossy materials have im < 0, e.g. 15 - 1j). */
typedef struct {
    double re, im;
} sbr_complex;

/* Trace parameters (Sec. II.B and Sec. III). */
typedef struct {
    int32_t max_order;     /* K: specular reflections per ray, 0..SBR_MAX_ORDER        */
    int32_t division_n;    /* n >= 1: polyhedron edges split into n parts; with the
                              equiangular icosahedron 10 n^2 + 2 launch rays
                              (Sec. III.B, with eq. (4))                              */
    int32_t iterations;    /* I >= 0: precise-algorithm iterations (Sec. III.B);
                              0 gives the plain SBR result ("traditional SBR")        */
    int32_t subrays;       /* 6 (the paper's six sub-cones) or 7 (six plus the axis)  */
    double target_err_deg; /* > 0: a path stops iterating once its error angle is
                              below target * L_last / L_total; <= 0: exactly I
                              iterations                                             */
    double freq_hz;        /* carrier frequency, > 0                                 */
    double tx_power_dbm;   /* transmit power                                          */
    uint32_t flags;        /* SBR_FLAG_*                                              */
    int32_t launch;        /* SBR_LAUNCH_*: launch grid (0: the paper's equiangular)  */
} sbr_trace_params;

/* Launch grids.  EQUIANGULAR is the paper's method (Sec. II.B: equal angles
 * along icosahedron edges and rings, eqs. (1)-(2)), 10 n^2 + 2 rays.  The
 * equidistant divisions it is compared with (Sec. II.A, Fig. 2) space points
 * equally on the flat faces of the icosahedron (10 n^2 + 2 rays) or the
 * octahedron (4 n^2 + 2 rays) and project them onto the sphere.  The cone
 * half-angle is theta_edge / (sqrt(3) n), eq. (4), with the polyhedron's edge
 * angle theta_edge (atan 2 for the icosahedron, pi / 2 for the octahedron). */
#define SBR_LAUNCH_EQUIANGULAR 0
#define SBR_LAUNCH_EQUIDISTANT_ICOSA 1
#define SBR_LAUNCH_EQUIDISTANT_OCTA 2

#define SBR_FLAG_KEEP_INVALID 1u /* keep paths that fail path test 2 (flag INVALID) */
#define SBR_FLAG_FRESH_GRID 2u   /* recompute the launch directions even when cached.
                                    sbr_trace and sbr_trace_device may then run the
                                    equiangular ring setup on a second stream of the
                                    context beside the trace, which forms the directions
                                    itself (the same values; a call whose setup cannot
                                    run concurrently is redone with the grid formed
                                    first).  Environment at context creation:
                                    SBR_GRID_STREAM=1 (default) when a previous fresh
                                    call of that grid traced at least three times as long
                                    as it formed the grid, 2 always, 0 never */
#define SBR_FLAG_GRAPH 4u        /* sbr_trace_device, sbr_trace_batch: capture the call as
                                    a HIP graph and replay it on later calls of the same
                                    shape */

/* Path flags (sbr_path.flags). */
#define SBR_PATH_STALLED 1u    /* an iteration found no sub-ray with the same faces  */
#define SBR_PATH_INVALID 2u    /* failed path test 2 (validity, Sec. III.A)          */
#define SBR_PATH_TARGET_MET 4u /* stopped early on target_err_deg                   */

/* One path (Sec. III and Sec. IV).  "Refined" fields come from the precise
 * algorithm's final ray; "exact_" fields from the image-method solve of the
 * same face sequence, which also decides path test 2.  Angles are unit
 * vectors: aod points from Tx along the departing ray, aoa points from Rx
 * back toward the last interaction (or Tx). */
typedef struct {
    int32_t rx;                  /* receiver index                                   */
    int32_t order;               /* number of reflections k                          */
    int32_t face[SBR_MAX_ORDER]; /* face ids hit in order; -1 beyond order           */
    int64_t launch_ray;          /* launch ray that won path test 1                  */
    int32_t iters_used;          /* precise-algorithm iterations whose winning sub-ray
                                    became the path's axis (upturns included): the
                                    index of the last such iteration, 0 if none      */
    uint32_t flags;              /* SBR_PATH_*                                       */
    double tan_err;              /* tan of the error angle of the reported ray       */
    double axis[3];              /* reported departure direction                     */
    double delay_s, aod[3], aoa[3], power_dbm, err_angle_deg, length_m;
    double exact_delay_s, exact_aod[3], exact_aoa[3], exact_power_dbm, exact_length_m;
    double init_tan_err;         /* tan error angle of the path-test-1 winner        */
} sbr_path;

/* A reception event before path test 1 (Sec. III.A, eq. (3)). */
typedef struct {
    int32_t rx, order, face[SBR_MAX_ORDER];
    int64_t ray;
    double tan_err;
} sbr_candidate;

/* Per-call timings (ms, measured with HIP events on the context stream),
 * counts, and the LDS staging of the trace kernel (bytes per workgroup, BVH
 * nodes and triangles held in LDS, device limit per workgroup). */
typedef struct {
    int64_t n_rays, n_candidates, n_unique, n_paths;
    double ms_launch, ms_trace, ms_dedup, ms_refine, ms_solve, ms_emit, ms_total;
    int64_t lds_bytes, lds_nodes, lds_tris, lds_max;
} sbr_trace_stats;

/* BVH build options; NULL means defaults (leaf size 4, 64 SAH bins, no
 * split references).  With split_pct > 0 a triangle whose box is large next
 * to the scene's median triangle box may enter the hierarchy as several
 * references, each bounding the part of the triangle in one cell of a
 * midpoint subdivision of its box, up to split_pct percent extra references
 * in all (largest boxes first).  The hierarchy only decides which nodes a ray
 * visits: paths do not depend on these options. */
typedef struct {
    int32_t max_leaf_size; /* 1..16 */
    int32_t sah_bins;      /* 4..64 */
    int32_t split_pct;     /* 0..400; 0: one reference per triangle */
} sbr_bvh_params;

/* Launch tuning of a context (the results never depend on it).  The trace
 * kernel is persistent: waves take packets of 64 * trace_chunk rays from a
 * device queue; persist_blocks workgroups are launched.  lds_budget > 0
 * stages the BVH's top nodes (and all triangles when they fit) plus a
 * stack_depth-entry traversal stack per lane in LDS, with trace_block lanes
 * per workgroup (a budget of just 4 * stack_depth * trace_block bytes keeps
 * only the stack there); 0 traverses from global memory with a private stack
 * (256 lanes per workgroup).
 * With at most lookahead_max_paths paths the refinement resolves
 * lookahead_depth iterations per traversal step (3: a 512-lane workgroup per
 * path, with its own LDS plan, for at most lookahead3_max_paths paths,
 * since it traces 399 sub-rays per path and step; 2: one wave per path);
 * otherwise, or with depth 1, one iteration per step with eight lanes per
 * path.  Depth 0 (single calls and batches) refines in one persistent
 * launch whose lanes take sub-rays from a device work queue: the lane that
 * completes an iteration's last sub-ray picks the winner and queues the next
 * iteration's sub-rays, so every path runs its own number of iterations
 * without a relaunch (calls whose queue would exceed 256 MiB use depth 1).
 * A job with at least rx_tree_min receivers tests reception through
 * a box tree over its receivers (a conservative cull before the exact test
 * of eq. (3)) instead of testing every receiver on every segment.  The
 * equiangular grid's setup takes a value from short series when its error
 * bound, scaled by 2^grid_check_log2, proves the rounding, and otherwise
 * recomputes that layer with the full series (same grid; larger values only
 * send more layers through the full series).  With ray_order = 1 a job that
 * traces every ray of its grid hands its rays to the waves sorted by
 * direction (cube-map cells in Z order, the order made once per grid of at
 * most 2^27 rays), so the 64 rays of a wave leave in nearby directions and
 * traverse the same BVH nodes; 0 hands them out by index (same results).
 * With refine_segments = 1 (and a depth other than 0), up to
 * lookahead_max_paths paths are refined with the k + 1 segments of every
 * sub-ray traced at once by separate lanes: a lane starts its segment where
 * the chain of closest hits on the expected faces puts it, so a step waits
 * for the slowest segment instead of the k + 1 segments in a row (same
 * results).  Up to lookahead3_max_paths paths get a 512-lane workgroup each
 * and two iterations per step; more get one wave each and one iteration per
 * step, and those still running after ten iterations continue two per step
 * on 512-lane workgroups. */
typedef struct {
    int32_t trace_chunk;         /* 1..64                                   */
    int32_t persist_blocks;      /* >= 1                                    */
    int32_t trace_block;         /* 64..256, multiple of 64 (LDS staging)   */
    int32_t stack_depth;         /* 0..96                                   */
    int32_t lds_budget;          /* bytes, 0..device limit per workgroup    */
    int32_t rx_tree_min;         /* >= 1                                    */
    int64_t lookahead_max_paths; /* >= 0                                    */
    int32_t lookahead_depth;     /* 0..3                                    */
    int32_t lookahead3_max_paths; /* >= 0                                   */
    int32_t grid_check_log2;     /* 0..200                                  */
    int32_t ray_order;           /* 0 or 1                                  */
    int32_t refine_segments;     /* 0 or 1                                  */
} sbr_tuning;

sbr_status sbr_context_get_tuning(const sbr_context* ctx, sbr_tuning* out);
/* Errors: SBR_E_INVALID_ARG when a field is out of range. */
sbr_status sbr_context_set_tuning(sbr_context* ctx, const sbr_tuning* tuning);

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t the
 * caller owns (for example torch's current stream) or NULL for the default
 * stream.  Errors: SBR_E_INVALID_ARG (bad device / out == NULL), SBR_E_DEVICE. */
sbr_status sbr_context_create(int32_t device, void* hip_stream, sbr_context** out);
/* Release the context and every device buffer it holds.  Scenes created on it
 * must be destroyed first (SBR_E_INVALID_ARG otherwise). */
sbr_status sbr_context_destroy(sbr_context* ctx);

/* Scene (Sec. IV: faces with material information).  xyz [n_vertices][3];
 * tri [n_triangles][3] vertex indices; face_id [n_triangles] >= 0 names the
 * planar polygon ("face") a triangle belongs to -- a face's plane and
 * material are those of its lowest-index triangle and every triangle of a face
 * must lie in that plane (within 1e-9 of the scene's bounding-box diagonal);
 * mat_id [n_triangles] indexes eps_r [n_materials].  Degenerate triangles are
 * accepted and never hit, except as a face's lowest-index triangle, which
 * must define the plane.  Errors: SBR_E_INVALID_ARG (index out of range,
 * non-finite vertex or permittivity, a face's first triangle degenerate, a
 * triangle off its face's plane), SBR_E_OOM, SBR_E_DEVICE. */
sbr_status sbr_scene_upload(sbr_context* ctx, const double* xyz, int64_t n_vertices,
                            const int32_t* tri, const int32_t* face_id, const int32_t* mat_id,
                            int64_t n_triangles, const sbr_complex* eps_r, int32_t n_materials,
                            sbr_scene** out);
/* Build the acceleration structure (binned SAH BVH with conservative FP32
 * boxes; not part of the paper's method, which leaves acceleration open).
 * Errors: SBR_E_INVALID_ARG (a parameter out of range, or a hierarchy of more
 * than 2^25 nodes, 4 GiB: about 100 M triangles), SBR_E_INTERNAL (hierarchy
 * deeper than the traversal stack), SBR_E_OOM, SBR_E_DEVICE. */
sbr_status sbr_bvh_build(sbr_scene* scene, const sbr_bvh_params* params);
sbr_status sbr_scene_destroy(sbr_scene* scene);

/* The whole method (Sec. II-III): equiangular launch from tx, SBR tracing with
 * specular reflection up to max_order, cone reception at every rx (eq. (3)),
 * path test 1 (one path per receiver and face sequence, the smaller error
 * angle wins), the precise algorithm, path test 2 and the path quantities.
 * rx [n_rx][3] (n_rx may be 0).  Paths are written to out[0..*n_out) sorted by
 * (rx, order, face sequence).  stats may be NULL. */
sbr_status sbr_trace(sbr_scene* scene, const double tx[3], const double* rx, int32_t n_rx,
                     const sbr_trace_params* params, sbr_path* out, int64_t capacity,
                     int64_t* n_out, sbr_trace_stats* stats);

/* sbr_trace with the receivers and the output in device memory (for example
 * torch tensors on the context's device): rx [n_rx][3] and out [capacity]
 * are device pointers, tx and params stay on the host.  The work is queued on
 * the context's stream after everything already queued there, and the call
 * returns when out and *n_out (host) are complete.  When n_rx reaches the
 * context's rx_tree_min the receivers are read back once to build the
 * receiver tree on the host.  Receivers are not validated: non-finite ones
 * are never captured.
 * With SBR_FLAG_GRAPH (and fewer than rx_tree_min receivers) a call that
 * ends with at most 4096 reception events captures its launch sequence as a
 * HIP graph; a later call with the same scene, rx and out pointers, n_rx,
 * capacity, params (flags included) and tuning replays it, reading the
 * transmitter from this call and the receivers from rx.  A replay whose
 * counts exceed what was captured (more than 4096 events, or more than twice
 * the capturing call's unique paths) is redone as a normal call.  Results
 * are identical either way; with a replay only the count and ms_total fields
 * of stats are set.  Errors as sbr_trace. */
sbr_status sbr_trace_device(sbr_scene* scene, const double tx[3], const double* rx, int32_t n_rx,
                            const sbr_trace_params* params, sbr_path* out, int64_t capacity,
                            int64_t* n_out, sbr_trace_stats* stats);

/* sbr_trace_device for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, results and stream semantics as sbr_trace_device, but the
 * call allocates nothing (no hipMalloc, hipFree or pinned host memory): all of
 * its working memory -- the launch grid, the FP32 receivers, reception events,
 * path-test-1 winners, refinement state and path records -- lives in one
 * fixed 24 MiB array of device memory per GPU, set up when the library's
 * context is created and held until the process ends.  Limits, checked before
 * any work is queued unless noted: n_rx <= 4096; the launch grid (24 bytes per
 * ray) must fit beside the other buffers, which allows up to about 900,000
 * rays (division n <= 300 on the icosahedron); at most 4096 reception events
 * (known only after the trace: the call then returns SBR_E_SCRATCH and leaves
 * out unwritten).  Any limit exceeded gives SBR_E_SCRATCH and a message;
 * sbr_trace_device has none of these limits.  SBR_FLAG_GRAPH is rejected
 * (SBR_E_INVALID_ARG).  Rays are handed out by index and every receiver is
 * tested on every segment (no receiver tree), which gives the same paths.
 * Every call on one GPU, from any context, shares that GPU's array: calls
 * that overlap in time on one GPU race and give undefined results.  The array
 * keeps the last call's launch grid, which a later call with the same launch
 * method and n reuses (SBR_FLAG_FRESH_GRID recomputes it).  Errors as
 * sbr_trace_device, plus SBR_E_SCRATCH, and SBR_E_DEVICE when the array's
 * device address could not be obtained. */
sbr_status sbr_trace_device_noalloc(sbr_scene* scene, const double tx[3], const double* rx,
                                    int32_t n_rx, const sbr_trace_params* params, sbr_path* out,
                                    int64_t capacity, int64_t* n_out, sbr_trace_stats* stats);

/* One job of a batched trace: transmitter tx on scenes[scene], its receivers
 * rx[rx_first .. rx_first + n_rx) of the batch's receiver array (a receiver
 * belongs to at most one job), and its own trace parameters. */
typedef struct {
    int32_t scene;
    int32_t rx_first;
    int32_t n_rx;
    int32_t reserved; /* must be 0 */
    double tx[3];
    sbr_trace_params params;
} sbr_job;

/* Many transmitter/receiver jobs over several scenes in one pass of the path:
 * one persistent trace launch whose device queue hands out ray packets of all
 * jobs, one path test 1 over all reception events, one refinement launch over
 * all paths (the context's lookahead tuning; with depth 0 a persistent launch
 * whose device work queue holds every path's sub-rays, each path iterating as
 * far as its own job's iteration count and target take it), and one solve
 * launch over all paths.  Each job's paths are exactly those sbr_trace
 * returns for it alone, with sbr_path.rx numbering the batch's receiver
 * array; the list is sorted by (rx, order, face sequence).  rx [n_rx_total][3]
 * host FP64.  All scenes must belong to ctx and have a BVH.
 * When every job has SBR_FLAG_GRAPH (none SBR_FLAG_FRESH_GRID, none with
 * rx_tree_min or more receivers) and the call ends with at most 4096
 * reception events, its launch sequence is captured as a HIP graph; a later
 * call with the same scenes, the same jobs apart from their transmitters
 * and the same receiver count replays it with this call's transmitters and
 * receivers (the job table and the receivers go through pinned staging, the
 * paths through a device buffer sized by the capture).  A replay whose counts
 * exceed the captured sizes (more than 4096 events, or more than twice the
 * capturing call's unique paths) is redone as a normal call.  Results are
 * identical either way; with a replay only the count and ms_total fields of
 * stats are set.  Errors as for sbr_trace, plus SBR_E_INVALID_ARG for a job
 * whose scene index, receiver slice or parameters are out of range. */
sbr_status sbr_trace_batch(sbr_context* ctx, sbr_scene* const* scenes, int32_t n_scenes,
                           const sbr_job* jobs, int32_t n_jobs, const double* rx,
                           int32_t n_rx_total, sbr_path* out, int64_t capacity, int64_t* n_out,
                           sbr_trace_stats* stats);

/* The reception events before path test 1 (same launch, trace and reception
 * as sbr_trace), sorted by (rx, order, face sequence, tan_err, ray). */
sbr_status sbr_candidates(sbr_scene* scene, const double tx[3], const double* rx, int32_t n_rx,
                          const sbr_trace_params* params, sbr_candidate* out, int64_t capacity,
                          int64_t* n_out);

/* Launch directions of method `launch` (SBR_LAUNCH_*) for division n
 * (unit vectors, FP64), copied to out [count][3] for ray indices
 * first..first+count-1. */
sbr_status sbr_launch_grid(sbr_context* ctx, int32_t launch, int32_t n, int64_t first,
                           int64_t count, double* out);

/* Per-ray trace of launch rays first..first+count-1 of a launch grid
 * (Sec. III.A):
 * out_tri [count][max_order+1] is the triangle (input index) closing each
 * segment, -1 when the segment leaves the scene or was not reached;
 * out_t [count][max_order+1] the segment's ray parameter (+inf: none).
 * Either output may be NULL. */
sbr_status sbr_trace_rays(sbr_scene* scene, const double tx[3], int32_t launch, int32_t n,
                          int32_t max_order, int64_t first, int64_t count, int32_t* out_tri,
                          double* out_t);

/* Differentiable path quantities at fixed interaction sequences (the
 * gradients of the paths sbr_trace returns with respect to transmitter and
 * receiver positions and the materials' permittivities).  For path i with
 * order[i] reflections on faces[i][0..order[i]) -- a face sequence sbr_trace
 * returned -- the path is the image-method path between tx[i] and rx[i] that
 * the precise algorithm converges to.  values[i][0..8) = delay (s), AOD unit
 * vector (3), AOA unit vector (3), power (dBm), computed as in sbr_path's
 * exact_* fields but with the permittivities eps [n_materials][2] (re, im)
 * given here instead of the scene's.  With upstream [n_paths][8] (dLoss /
 * dvalue), grad_tx[i], grad_rx[i] ([n_paths][3]) receive dLoss / dposition and
 * grad_eps ([n_materials][2], caller-zeroed) accumulates dLoss / d(re, im) over
 * all paths.  Any of values / upstream may be NULL.
 * ALL ARRAYS ARE DEVICE MEMORY; the work is queued on the context's stream and
 * the call returns without waiting (stream order makes the results visible to
 * later work on that stream).  Rows whose order or face ids lie outside the
 * scene get NaN values and zero position gradients.  Errors: SBR_E_INVALID_ARG
 * (NULL arrays, n_paths < 0, freq_hz <= 0). */
sbr_status sbr_path_gradients(sbr_scene* scene, int64_t n_paths, const double* tx,
                              const double* rx, const int32_t* order, const int32_t* faces,
                              const double* eps, double freq_hz, double tx_power_dbm,
                              const double* upstream, double* values, double* grad_tx,
                              double* grad_rx, double* grad_eps);

/* ---- Order-1 diffraction (Sec. III.A: paths through faces or wedges;
 * Sec. III.B: sub-rays diffracted in the recorded direction; Sec. IV:
 * order-1 diffraction paths) ---- */

/* A wedge: a mesh edge (endpoints with exactly equal coordinates) shared by
 * triangles of exactly two faces whose planes meet at an angle of at least
 * 10 degrees.  a < b lexicographically (x, then y, then z); face[0] < face[1].
 * Wedges are numbered in the order of (a, b). */
typedef struct {
    double a[3], b[3];
    int32_t face[2];
} sbr_wedge;

/* The wedges of a scene (made from its triangles on first use).  out may be
 * NULL with capacity 0 to query the count.  Errors: SBR_E_CAPACITY. */
sbr_status sbr_scene_wedges(sbr_scene* scene, sbr_wedge* out, int64_t capacity, int64_t* n_out);

/* One order-1 diffraction path Tx -> point on a wedge's edge -> Rx.  The
 * refined fields come from the precise algorithm's final ray (point = the edge
 * point nearest that ray), the exact_ fields from the path that makes equal
 * angles with the edge on both sides (Keller's law), which also decides path
 * test 2 (the point on the edge segment, Tx and Rx outside the wedge, both
 * legs unobstructed).  Angles as in sbr_path.  No power: the paper gives no
 * diffraction coefficient. */
typedef struct {
    int32_t rx, wedge;
    int64_t launch_ray;
    int32_t iters_used;          /* as sbr_path.iters_used                          */
    uint32_t flags;              /* SBR_PATH_*                                      */
    double tan_err, axis[3], point[3], delay_s, aod[3], aoa[3], err_angle_deg, length_m;
    double exact_point[3], exact_delay_s, exact_aod[3], exact_aoa[3], exact_length_m;
    double init_tan_err;
} sbr_diff_path;

/* Order-1 diffraction paths from tx to rx [n_rx][3] (host FP64): every
 * launch ray whose closest approach to a wedge's edge lies on the segment, in
 * front of Tx, inside the ray cone and before the ray's first hit (or on one
 * of the wedge's faces) diffracts there; it reaches each receiver outside the
 * wedge whose image, the receiver rotated about the edge into the half-plane
 * opposite Tx, lies inside the ray cone; the error angle is the angle to that
 * image (the departure-angle error, eq. (3) unfolded).  Path test 1 keeps one
 * path per (receiver, wedge); the precise algorithm (params->iterations,
 * subrays, target_err_deg) refines each; path test 2 drops invalid ones
 * (unless SBR_FLAG_KEEP_INVALID).  max_order, freq_hz and tx_power_dbm are
 * checked but not used.  Output sorted by (rx, wedge).  Errors as sbr_trace. */
sbr_status sbr_diffract(sbr_scene* scene, const double tx[3], const double* rx, int32_t n_rx,
                        const sbr_trace_params* params, sbr_diff_path* out, int64_t capacity,
                        int64_t* n_out, sbr_trace_stats* stats);

/* The diffraction events before path test 1 (order 1, face[0] = wedge),
 * sorted by (rx, wedge, tan_err, ray). */
sbr_status sbr_diff_candidates(sbr_scene* scene, const double tx[3], const double* rx,
                               int32_t n_rx, const sbr_trace_params* params, sbr_candidate* out,
                               int64_t capacity, int64_t* n_out);

/* Work counts of the trace stage of sbr_trace with the same arguments, from
 * an instrumented copy of the trace kernel: counts[0] segments traced
 * (ray-bounces), counts[1] BVH4 nodes visited (128 B each), counts[2]
 * ray-triangle tests, counts[3] reception events, counts[4] triangle tests
 * run (not skipped as lying on the face the segment leaves), counts[5],
 * counts[6], counts[7] and counts[8] the passes of the wave-wide node loop,
 * triangle loop, segment loop and receiver loops (one per wave and pass in
 * which any lane visits a node, tests a triangle, traces a segment, tests a
 * receiver or receiver-tree node), so that counts[1] / (64 counts[5]) is the
 * share of lanes busy in the node loop; counts[9] receiver-tree nodes (boxes)
 * tested against a segment's reception cone, counts[10] receivers tested on
 * a segment (eq. (3): every receiver of a segment that can reach the
 * receivers' box, or of a tree leaf whose box passed); counts[11] is 0.
 * counts[0..2], [9] and [10] define the algorithmic work of the trace
 * kernel for its roofline. */
sbr_status sbr_trace_counters(sbr_scene* scene, const double tx[3], const double* rx,
                              int32_t n_rx, const sbr_trace_params* params, int64_t counts[12]);

const char* sbr_status_string(sbr_status status);
/* Message of the last failing call on ctx (empty if none); valid until the
 * next call on ctx.  ctx may be NULL for failures of sbr_context_create. */
const char* sbr_last_error(const sbr_context* ctx);

#ifdef __cplusplus
}
#endif
#endif /* SBR_H */
