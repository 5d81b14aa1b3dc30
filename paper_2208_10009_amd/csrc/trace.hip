// trace.hip -- SBR tracing and reception (Sec. III.A), one lane per launch
// ray: closest hit per segment, specular reflection up to K bounces, and the
// cone reception test of every receiver on every segment (eq. (3)), fused.
#include <math.h>

#include "traverse.h"

namespace sbr {

// With COUNT, per-ray totals of traversal work are added to tallies[0..3]:
// segments traced, BVH nodes visited, triangles tested, reception events.
template <bool COUNT, bool LDS>
__global__ __launch_bounds__(LDS ? 1024 : 256) void k_trace(SceneDev S, LdsPlan L, GridDev g, TraceArgs A,
                                                int64_t first, int64_t count,
                                                sbr_candidate* __restrict__ cand, int64_t cap,
                                                unsigned long long* __restrict__ ccount,
                                                int32_t* __restrict__ out_tri,
                                                double* __restrict__ out_t,
                                                int32_t* __restrict__ err,
                                                unsigned long long* __restrict__ tallies)
{
    if (LDS) stage_scene(S, L);
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    Tally tl{0u, 0u};
    uint32_t segs = 0, events = 0;
    const int64_t r = first + i;
    const int K = A.K;
    d3 o = mk(A.tx[0], A.tx[1], A.tx[2]);
    d3 d = mk(g.dir[r], g.dir[g.N + r], g.dir[2 * g.N + r]);
    double D = 0.0;
    int32_t prev = -1;
    int32_t faces[SBR_MAX_ORDER];
#pragma unroll
    for (int q = 0; q < SBR_MAX_ORDER; ++q) faces[q] = -1;
    for (int j = 0; j <= K; ++j) {
        HitRec h;
        int32_t hit = traverse<false, COUNT, LDS>(S, L, o, d, prev, prev, S.t_eps, INFINITY,
                                                  A.delta, &h, err, &tl);
        if (COUNT) segs += 1;
        double t = hit < 0 ? INFINITY : h.t;
        if (out_tri) out_tri[i * (K + 1) + j] = hit < 0 ? -1 : h.orig;
        if (out_t) out_t[i * (K + 1) + j] = t;
        for (int x = 0; x < A.n_rx; ++x) {
            double tn;
            d3 rx = mk(A.rx[3 * x], A.rx[3 * x + 1], A.rx[3 * x + 2]);
            if (!capture(o, d, D, t, rx, A.thl, &tn)) continue;
            if (COUNT) events += 1;
            unsigned long long pos = atomicAdd(ccount, 1ull);
            if ((int64_t)pos < cap) {
                sbr_candidate c;
                c.rx = x;
                c.order = j;
#pragma unroll
                for (int q = 0; q < SBR_MAX_ORDER; ++q) c.face[q] = q < j ? faces[q] : -1;
                c.ray = r;
                c.tan_err = tn;
                cand[pos] = c;
            }
        }
        if (hit < 0 || j == K) {
            if (out_tri || out_t)
                for (int q = j + 1; q <= K; ++q) {
                    if (out_tri) out_tri[i * (K + 1) + q] = -1;
                    if (out_t) out_t[i * (K + 1) + q] = INFINITY;
                }
            break;
        }
        // specular reflection on the face plane: o' = o + t d,
        // d' = d - (2 d.n) n (no renormalization), D' = D + t
        int32_t f = h.face;
        d3 nf = face_normal(S, f);
        d3 on = add(o, scl(t, d));
        double k2 = 2.0 * dot(d, nf);
        d = sub(d, scl(k2, nf));
        D = D + t;
        o = on;
        prev = f;
        faces[j] = f;
    }
    if (COUNT) {
        atomicAdd(&tallies[0], (unsigned long long)segs);
        atomicAdd(&tallies[1], (unsigned long long)tl.nodes);
        atomicAdd(&tallies[2], (unsigned long long)tl.tris);
        atomicAdd(&tallies[3], (unsigned long long)events);
    }
}

template <bool COUNT, bool LDS>
static void launch_trace_t(const SceneDev& S, const LdsPlan& L, const GridDev& g,
                           const TraceArgs& A, int64_t first, int64_t count, sbr_candidate* cand,
                           int64_t cap, unsigned long long* cand_count, int32_t* out_tri,
                           double* out_t, int32_t* err_flag, hipStream_t s,
                           unsigned long long* tallies)
{
    int64_t blocks = (count + L.block - 1) / L.block;
    hipLaunchKernelGGL((k_trace<COUNT, LDS>), dim3((unsigned)blocks), dim3(L.block),
                       LDS ? L.bytes : 0, s, S, L, g, A, first, count, cand, cap, cand_count,
                       out_tri, out_t, err_flag, tallies);
}

hipError_t launch_trace(const SceneDev& S, const LdsPlan& L, const GridDev& g, const TraceArgs& A,
                        int64_t first, int64_t count, sbr_candidate* cand, int64_t cap,
                        unsigned long long* cand_count, int32_t* out_tri, double* out_t,
                        int32_t* err_flag, hipStream_t s, unsigned long long* tallies)
{
    if (count <= 0) return hipSuccess;
    const bool lds = L.bytes > 0;
    if (tallies && lds)
        launch_trace_t<true, true>(S, L, g, A, first, count, cand, cap, cand_count, out_tri, out_t,
                                   err_flag, s, tallies);
    else if (tallies)
        launch_trace_t<true, false>(S, L, g, A, first, count, cand, cap, cand_count, out_tri,
                                    out_t, err_flag, s, tallies);
    else if (lds)
        launch_trace_t<false, true>(S, L, g, A, first, count, cand, cap, cand_count, out_tri,
                                    out_t, err_flag, s, tallies);
    else
        launch_trace_t<false, false>(S, L, g, A, first, count, cand, cap, cand_count, out_tri,
                                     out_t, err_flag, s, tallies);
    return hipGetLastError();
}

hipError_t trace_set_lds_limit(int bytes)
{
    hipError_t e = hipFuncSetAttribute((const void*)k_trace<true, true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_trace<false, true>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

}  // namespace sbr
