// diffract.h -- declarations of the order-1 diffraction stages (diffract.hip),
// shared with the host orchestration (api.hip); not part of the public ABI.
#pragma once
#include "internal.h"

namespace sbr {

// ---- order-1 diffraction (diffract.hip) ---------------------------------
// One wedge (an edge where two faces meet at >= 10 degrees): endpoint a, unit
// direction e, length, the in-face unit vectors u0, u1 of faces f0 < f1 (for
// the inside test), and an FP32 bounding sphere (centre c, radius r, rounded
// up) of the segment for the conservative cull.  128 bytes.
struct WedgeDev {
    double a[3], e[3], u0[3], u1[3];
    double len;
    int32_t f0, f1;
    float c[3], r;
};
static_assert(sizeof(WedgeDev) == 128, "WedgeDev layout");

// Host-side wedge extraction: the wedges of a scene given its triangles'
// vertices tri_v [T][9], face ids and the faces' unit normals fplane [F][4],
// sorted by their endpoints.
void build_wedges(const double* tri_v, const int32_t* face, int64_t T, const double* fplane,
                  std::vector<WedgeDev>& out, std::vector<double>& b_out);

struct DiffArgs {
    const double* dir;    // launch directions [3][N]
    int64_t N;
    double tx[3];
    double thl, tan_tgt;
    float delta;          // box inflation of the FP32 traversal
    int32_t iterations, subrays, keep_invalid;
    const WedgeDev* w;
    int32_t n_w;
    const double* rx;     // [n_rx][3]
    int32_t n_rx;
    double4* rxp;         // [n_w][n_rx]: receiver unfolded about the wedge (w = 1: usable)
};

// Receivers unfolded about every wedge (inside a wedge or on its edge line:
// not usable).
hipError_t launch_diff_unfold(const DiffArgs& A, hipStream_t s);
// SBR diffraction of every launch ray: events (order 1, face[0] = wedge) are
// appended to cand (up to cap; *count counts all).
hipError_t launch_diff_trace(const SceneDev& S, const DiffArgs& A, sbr_candidate* cand,
                             int64_t cap, unsigned long long* count, int32_t* err,
                             hipStream_t s);
// Precise algorithm of the path-test-1 winners uniq[0..U).
hipError_t launch_diff_refine(const SceneDev& S, const DiffArgs& A, const sbr_candidate* uniq,
                              int64_t U, RefineOut* out, int32_t* err, hipStream_t s);
// Path quantities and path test 2; keep[i] = 1 for the paths to emit.
hipError_t launch_diff_solve(const SceneDev& S, const DiffArgs& A, const sbr_candidate* uniq,
                             const RefineOut* rf, int64_t U, sbr_diff_path* paths,
                             int32_t* keep, int32_t* err, hipStream_t s);
hipError_t launch_compact_dpaths(const sbr_diff_path* paths, const int32_t* keep,
                                 const int32_t* offs, int64_t U, sbr_diff_path* out,
                                 hipStream_t s);

}  // namespace sbr
