// layout.h -- data layouts and constants shared by the library's host and
// device sources (not part of the public ABI): scene, BVH, receivers, jobs
// and calls as the kernels see them.
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

// Receiver-tree node (64 B), in depth-first preorder: the box c +- h holds
// every receiver below.  count > 0: a leaf of the receivers perm[first ..
// first + count) (global receiver indices); count == 0: an inner node whose
// left child is the next node.  skip is the node after this subtree, where a
// walk goes when the box is rejected.
struct RxNode {
    double c[3];
    double h[3];
    int32_t first, count, skip, pad;
};
static_assert(sizeof(RxNode) == 64, "RxNode layout");
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
    // Streamed launch grid (single-job calls over a whole equiangular grid):
    // the ring setup runs beside the trace, publishing its progress at gprog
    // (epoch << 32 | progress), and the trace forms each packet's directions
    // from the setup's scratch gscr into the job's dir once the progress its
    // rays need is out.  gscr NULL: the directions are there beforehand.
    const char* gscr;
    const unsigned long long* gprog;
    uint32_t gepoch;
    int32_t gn;           // the grid's division n
    int32_t gcheck;       // the grid's check_log2
    uint32_t gspin;       // polls before a wave gives up waiting for the setup (sets err 4)
};

}  // namespace sbr
