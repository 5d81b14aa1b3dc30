// internal.h -- the launchers of the library's kernels and the other
// host-side declarations shared by its sources (not part of the public ABI);
// declarations only, the data layouts are in layout.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "layout.h"

namespace sbr {

// ---- launchers -----------------------------------------------------------
// FP32 copies of n receivers for the reception pre-test: (x, y, z, m) with m
// at least max(|x|, |y|, |z|) of the FP64 receiver; the same launch zeroes
// zero_bytes (a multiple of 4) at zero.
hipError_t launch_rx32(const double* rx, int64_t n, float4* out, hipStream_t s,
                       void* zero = nullptr, size_t zero_bytes = 0);
// check_log2 scales the error bounds of the equiangular grid's fast pass.
hipError_t launch_grid(GridDev g, hipStream_t s, void* scratch, int32_t check_log2 = 0);
size_t grid_scratch_bytes(int32_t n);
// The equiangular ring setup alone, publishing its progress at prog (see
// grid_need in grid.h) for a trace that forms its rays' directions itself;
// and a one-lane wait (at most max_spin polls; err |= 8 on time-out) until the
// setup of this epoch has started.
hipError_t launch_grid_setup_streamed(int32_t n, void* scratch, int32_t check_log2,
                                      unsigned long long* prog, uint32_t epoch, hipStream_t s);
hipError_t launch_grid_wait_started(const unsigned long long* prog, uint32_t epoch, int32_t* err,
                                    uint32_t max_spin, hipStream_t s);
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
// depth 1: eight lanes per path, one iteration per step.  The segments of
// every sub-ray traced in parallel lanes: depth kRefineSegments2, a 512-lane
// workgroup per path and two iterations per step; depth kRefineSegments,
// one wave per path and one iteration per step, the paths still running
// after tail_after iterations (when max_iters, the largest iteration count
// of the call's jobs, is larger; tail_after 0: never) continuing two
// iterations per step on 512-lane workgroups.
// L3 is the 512-lane plan (three-level kernel and the two-level segment
// kernel; bytes == 0: global memory), used whatever L is.
constexpr int kRefineSegments = 4;
constexpr int kRefineSegments2 = 5;
hipError_t launch_refine(const CallDev& call, const LdsPlan& L, const LdsPlan& L3,
                         const SceneDev& s0, const sbr_candidate* uniq, int64_t U_max,
                         const int32_t* n_dev, int depth, RefineOut* out, PathGeom* geom,
                         int32_t* err, hipStream_t s, int32_t max_iters, int32_t tail_after);

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
