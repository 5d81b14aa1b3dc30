// internal.h -- declarations shared by the library's host and device sources
// (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/sbr.h"
#include "geom.h"

namespace sbr {

// One triangle for the FP64 ray-triangle test, in BVH leaf order: v0 and the
// edges e1 = v1 - v0, e2 = v2 - v0, its face and its index in the input.
struct TriD {
    double v0x, v0y, v0z, e1x, e1y, e1z, e2x, e2y, e2z;
    int32_t face, orig;
};
static_assert(sizeof(TriD) == 80, "TriD layout");

// BVH2 node, 64 bytes: the FP32 boxes of both children (rounded outward)
// and, per child, (index, count): count > 0 is a leaf of `count` triangles
// starting at `index` in leaf order, count == 0 an inner node, count < 0 an
// empty child.  Packed as 4 x 16 B:
//   a = lo0.xyz hi0.x | b = hi0.yz lo1.xy | c = lo1.z hi1.xyz | m = c0 c1 n0 n1
// The builder's intermediate form; the device traverses the BVH4 below.
struct BvhNode {
    float a[4], b[4], c[4];
    int32_t m[4];
};
static_assert(sizeof(BvhNode) == 64, "BvhNode layout");

// BVH4 node, 128 bytes (8 x 16 B): the FP32 boxes of four children in SoA
// rows of four (lo x, lo y, lo z at bytes 0, 16, 32; hi x, hi y, hi z at 64,
// 80, 96: each axis's lo and hi rows 64 bytes apart, so a traversal lane
// finds the far row of an axis by flipping bit 6 of the near row's offset),
// and per child (index, count) at 48 and 112 with the BvhNode meaning; an
// empty child has the inverted box lo = +inf, hi = -inf, which no ray enters.
// Collapsed from the BVH2, whose outward-rounded child boxes it keeps.
struct Bvh4Node {
    float lox[4], loy[4], loz[4];
    int32_t idx[4];
    float hix[4], hiy[4], hiz[4];
    int32_t cnt[4];
};
static_assert(sizeof(Bvh4Node) == 128, "Bvh4Node layout");

constexpr int kMaxBvhDepth = 48;  // builder cap on the BVH2 depth
constexpr int64_t kMaxBvhNodes = int64_t(1) << 25;  // node byte offsets fit 32 bits
constexpr int kTraceStack = 96;   // traversal stack; a BVH4 level pushes at most 3

// Host-side BVH build (binned SAH BVH2, collapsed to BVH4) over triangle
// references: large triangles may be split into up to T split_pct / 100
// extra references with clipped boxes.  tri_v is [T][9] FP64 vertices.
// Nodes are numbered depth-first, or breadth-first with bfs (so that the top
// levels form a prefix for LDS staging).  perm receives the leaf order (the
// input index of each reference's triangle; a split triangle appears once
// per reference); returns the BVH4 depth.
int build_bvh(const double* tri_v, int64_t T, int max_leaf, int bins, int split_pct, bool bfs,
              std::vector<Bvh4Node>& nodes, std::vector<int32_t>& perm);

// Device view of a scene.
struct SceneDev {
    const Bvh4Node* nodes;
    const TriD* tris;       // leaf order
    const double* fplane;   // [F][4]: unit normal, offset n.v0
    const int32_t* fmat;    // [F]
    const int32_t* fstart;  // [F+1] CSR of triangles per face
    const int32_t* ftris;   // positions in `tris`
    const double* eps;      // [M][2] relative permittivity re, im
    int32_t n_tri, n_face, n_node;
    double t_eps;           // 1e-9 x scene bounding-box diagonal
};

// Per-launch LDS plan of a traversal kernel: the first n_nodes BVH nodes and
// the first n_tris triangles of the (single) scene are copied into LDS,
// followed by a per-lane stack of `depth` entries (stride `block`) at byte
// offset stack_off.  bytes == 0: traverse from global memory with a private
// stack.
struct LdsPlan {
    int32_t n_nodes, n_tris, depth, stack_off, block;
    int32_t bytes;  // dynamic LDS per block
};

// Largest LDS plan for a block of `block` lanes with `depth` stack entries
// in `budget` bytes: everything when the scene fits, else a node prefix.
LdsPlan make_lds_plan(int64_t n_nodes, int64_t n_tris, int block, int depth, int budget);

// Launch-grid tables for one launch method and division n (device, FP64 SoA).
struct GridDev {
    double* dir;       // [3][N]: x, y, z
    int64_t N;
    int32_t n;
    int32_t launch;    // SBR_LAUNCH_*
};

// Rays of a launch method at division n: 10 n^2 + 2 on the icosahedron,
// 4 n^2 + 2 on the octahedron.
inline int64_t num_rays(int32_t launch, int32_t n)
{
    return (launch == SBR_LAUNCH_EQUIDISTANT_OCTA ? 4 : 10) * (int64_t)n * n + 2;
}

// Ball-tree node over receivers (48 B), in depth-first preorder: the ball
// (centre c, radius rho) holds every receiver below.  count > 0: a leaf of
// the receivers perm[first .. first + count) (global receiver indices);
// count == 0: an inner node whose left child is the next node.  skip is the
// node after this subtree, where a walk goes when the ball is rejected.
struct RxNode {
    double c[3];
    double rho;
    int32_t first, count, skip, pad;
};
static_assert(sizeof(RxNode) == 48, "RxNode layout");
constexpr int kRxLeaf = 4;

// One job of a trace call: a transmitter, its receivers (a slice of the
// call's receiver array) and its parameters, on one scene.  A plain trace is
// a call with one job.
struct JobDev {
    double tx[3];
    double thl;            // theta_launch (rad), eq. (4)
    double tan_tgt;        // tan(target error angle); <= 0: fixed iterations
    double freq_hz, tx_power_dbm;
    const double* dir;     // launch directions [3][N] for this job's division n
    int64_t N;             // rays of the division
    int64_t ray_begin;     // launch rays traced: [ray_begin, ray_begin + ray_count)
    int64_t ray_count;
    int64_t packet_first;  // index of the job's first ray packet in the call
    int32_t scene, rx_first, n_rx, K;
    int32_t iterations, subrays, keep_invalid;
    float delta;           // box inflation (m) making FP32 traversal conservative
    int32_t rx_root;       // root of the job's receiver tree; -1: test every receiver
    const uint32_t* order; // whole-grid jobs: the order rays are handed out in (NULL: by index)
};

// Everything the kernels of one call see.
struct CallDev {
    const JobDev* jobs;
    const SceneDev* scenes;
    const double* rx;       // [n_rx_total][3]: receivers of all jobs
    const int32_t* rx_job;  // job of each receiver
    const RxNode* rx_nodes; // receiver trees of the jobs that have one
    const int32_t* rx_perm; // receiver indices in tree-leaf order
    const float4* rx32;     // [n_rx_total]: receivers in FP32 and max |coordinate|
    int32_t n_jobs;
    int32_t chunk;          // 64-ray groups per packet
    int64_t n_packets;
};

// ---- launchers -----------------------------------------------------------
// FP32 copies of n receivers for the reception pre-test: (x, y, z, m) with m
// at least max(|x|, |y|, |z|) of the FP64 receiver; the same launch zeroes
// zero_bytes (a multiple of 4) at zero.
hipError_t launch_rx32(const double* rx, int64_t n, float4* out, hipStream_t s,
                       void* zero = nullptr, size_t zero_bytes = 0);
// check_log2 scales the error bounds of the equiangular grid's fast pass.
hipError_t launch_grid(GridDev g, hipStream_t s, void* scratch, int32_t check_log2 = 0);
size_t grid_scratch_bytes(int32_t n);
// cell[i] = the cube-map cell (R x R per cube face, Z order) of ray i's
// direction, R a power of two <= 8192.
hipError_t launch_ray_cells(const double* dir, int64_t N, int32_t R, uint32_t* cell,
                            hipStream_t s);

// Persistent trace + reception over all packets of the call.  Reception
// events are appended to cand (up to cap; *cand_count counts all); queue is a
// zeroed packet counter.  With out_tri/out_t (single-job calls) the per-ray
// hits are written at (ray - ray_begin) * (K + 1) + segment.  With tallies
// the counting variant adds (segments, nodes visited, triangles tested,
// events) to tallies[0..3].  s0 is the scene staged in LDS when L.bytes > 0.
hipError_t launch_trace(const CallDev& call, const LdsPlan& L, const SceneDev& s0, int blocks,
                        uint32_t* queue, sbr_candidate* cand, int64_t cap,
                        unsigned long long* cand_count, int32_t* out_tri, double* out_t,
                        int32_t* err_flag, hipStream_t s, unsigned long long* tallies = nullptr);
hipError_t trace_set_lds_limit(int bytes);
hipError_t refine_set_lds_limit(int bytes);
hipError_t refine_la3_set_lds_limit(int bytes);

// Sort candidates (sbr_candidate records) by (rx, order, faces, tan, ray);
// idx (pow2_at_least(n) entries) receives the permutation.
hipError_t launch_sort_candidates(const sbr_candidate* cand, int64_t n, uint32_t* idx,
                                  hipStream_t s);
int64_t pow2_at_least(int64_t n);

// head flags of the sorted candidates: 1 where the key differs from the
// previous entry.
hipError_t launch_heads(const sbr_candidate* cand, const uint32_t* idx, int64_t n,
                        int32_t* flags, hipStream_t s);

// Exclusive scan of int32 flags -> int32 offsets, total written to *total.
size_t scan_scratch_bytes(int64_t n);
hipError_t launch_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* total, void* scratch,
                       hipStream_t s);

// Gather the unique candidates (heads) into uniq in sorted order.
hipError_t launch_gather_unique(const sbr_candidate* cand, const uint32_t* idx,
                                const int32_t* flags, const int32_t* offs, int64_t n,
                                sbr_candidate* uniq, hipStream_t s);

// Reflection points and incoming directions of a path's reported ray, stored
// by the refinement for the winning sub-ray (valid when iterations > 0).
struct PathGeom {
    d3 pts[SBR_MAX_ORDER];
    d3 din[SBR_MAX_ORDER];
};

// Per-path state after the precise algorithm.
struct RefineOut {
    double axis[3];
    double tan_err;
    int32_t iters;
    uint32_t flags;
};

// U_max paths (the first min(U_max, *n_dev) when n_dev is non-NULL).  Depth
// 3 (without an LDS plan): one 512-lane workgroup per path resolves three
// iterations per step; depth 2: one wave per path, two iterations per step;
// depth 1: eight lanes per path, one iteration per step; depth
// kRefineSegments: one wave per path, one iteration per step, the segments
// of every sub-ray traced in parallel lanes.
// L3 is the plan of the three-level kernel (512 lanes; bytes == 0: global
// memory), used when depth is 3 whatever L is.
constexpr int kRefineSegments = 4;
hipError_t launch_refine(const CallDev& call, const LdsPlan& L, const LdsPlan& L3,
                         const SceneDev& s0, const sbr_candidate* uniq, int64_t U_max,
                         const int32_t* n_dev, int depth, RefineOut* out, PathGeom* geom,
                         int32_t* err, hipStream_t s);

// Path test 2, path quantities and power (Sec. III.A, Sec. IV) in two
// launches: the exact (image-method) path and its validity, which need no
// refinement result and may run beside the refinement, then the refined
// path's quantities and the refinement's flags.  geom0 (optional): the
// launch rays' geometry, traced by the first launch for the paths the
// refinement ends without an iteration.  replay: the refinement stored no
// geometry (the work queue), so the final axis is traced.
hipError_t launch_solve_exact(const CallDev& call, const sbr_candidate* uniq, int64_t U_max,
                              const int32_t* n_dev, sbr_path* paths, int32_t* keep,
                              PathGeom* geom0, int32_t* err, hipStream_t s);
hipError_t launch_solve_refined(const CallDev& call, const sbr_candidate* uniq,
                                const RefineOut* rf, PathGeom* geom, const PathGeom* geom0,
                                int64_t U_max, const int32_t* n_dev, sbr_path* paths,
                                int32_t* err, hipStream_t s, bool replay = false);
// Both, in order on one stream.
hipError_t launch_solve(const CallDev& call, const sbr_candidate* uniq, const RefineOut* rf,
                        PathGeom* geom, int64_t U_max, const int32_t* n_dev, sbr_path* paths,
                        int32_t* keep, int32_t* err, hipStream_t s, bool replay = false);

hipError_t launch_compact_paths(const sbr_path* paths, const int32_t* keep, const int32_t* offs,
                                int64_t U, sbr_path* out, hipStream_t s);

hipError_t launch_gather_sorted(const sbr_candidate* cand, const uint32_t* idx, int64_t n,
                                sbr_candidate* out, hipStream_t s);

// Up to kSmallEvents reception events, path test 1 and the final compaction
// run in one workgroup each and leave their counts on the device.
constexpr int kSmallEvents = 4096;
// With n_dev the event count is min(n, *n_dev), read on the device.
hipError_t launch_dedup_small(const sbr_candidate* C, int64_t n, sbr_candidate* U,
                              int32_t* n_unique, hipStream_t s,
                              const unsigned long long* n_dev = nullptr);
hipError_t launch_emit_small(const sbr_path* paths, const int32_t* keep, int64_t U_max,
                             const int32_t* n_dev, sbr_path* out, int64_t capacity,
                             int32_t* n_paths, hipStream_t s);
// Zero `bytes` (a multiple of 4) with a kernel.
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);

// Differentiable path quantities (grad.hip); all pointers are device memory.
struct GradArgs {
    const double* tx;      // [P][3]
    const double* rx;      // [P][3]
    const int32_t* order;  // [P]
    const int32_t* faces;  // [P][8]
    const double* eps;     // [M][2]
    const double* up;      // [P][8] upstream gradients or NULL
    double* val;           // [P][8] values or NULL
    double* gtx;           // [P][3]
    double* grx;           // [P][3]
    double* geps;          // [M][2], accumulated
    int64_t P;
    double freq_hz, tx_power_dbm;
};
hipError_t launch_path_grad(const SceneDev& S, const GradArgs& A, hipStream_t s);

}  // namespace sbr
