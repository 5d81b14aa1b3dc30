// trace.hip -- SBR tracing and reception (Sec. III.A): closest hit per
// segment, specular reflection up to K bounces, and the cone reception test
// of every receiver on every segment (eq. (3)), fused, one lane per launch
// ray.  Jobs with many receivers walk a ball tree over them and run the
// exact test only where a conservative cull lets a receiver through.  The kernel is persistent: waves take packets of 64 x chunk rays from
// a device queue until it is empty, so jobs of uneven size and rays of uneven
// length are balanced over the machine.  A packet never spans two jobs, so
// the job and its scene are uniform across a wave.
#include <math.h>

#include "traverse.h"

namespace sbr {

// Launch ray r of job J: trace, receive, record.
template <bool COUNT, bool LDS>
__device__ static inline void trace_ray(const SceneDev& S, const LdsPlan& L, const JobDev& J,
                                        const double* __restrict__ rx_all,
                                        const RxNode* __restrict__ rx_nodes,
                                        const int32_t* __restrict__ rx_perm, int64_t r,
                                        sbr_candidate* __restrict__ cand, int64_t cap,
                                        unsigned long long* __restrict__ ccount,
                                        int32_t* __restrict__ out_tri, double* __restrict__ out_t,
                                        int32_t* __restrict__ err, Tally* tl, uint32_t* segs,
                                        uint32_t* events)
{
    const int K = J.K;
    const int64_t ro = (r - J.ray_begin) * (K + 1);
    d3 o = mk(J.tx[0], J.tx[1], J.tx[2]);
    d3 d = mk(J.dir[r], J.dir[J.N + r], J.dir[2 * J.N + r]);
    double D = 0.0;
    int32_t prev = -1;
    int32_t faces[SBR_MAX_ORDER];
#pragma unroll
    for (int q = 0; q < SBR_MAX_ORDER; ++q) faces[q] = -1;
    for (int j = 0; j <= K; ++j) {
        HitRec h;
        int32_t hit = traverse<false, COUNT, LDS>(S, L, o, d, prev, prev, S.t_eps, INFINITY,
                                                  J.delta, &h, err, tl);
        if (COUNT) *segs += 1;
        double t = hit < 0 ? INFINITY : h.t;
        if (out_tri) out_tri[ro + j] = hit < 0 ? -1 : h.orig;
        if (out_t) out_t[ro + j] = t;
        // reception test of receiver gx on this segment; events are appended
        auto receive = [&](int32_t gx) {
            double tn;
            d3 rx = mk(rx_all[3 * gx], rx_all[3 * gx + 1], rx_all[3 * gx + 2]);
            if (!capture(o, d, D, t, rx, J.thl, &tn)) return;
            if (COUNT) *events += 1;
            unsigned long long pos = atomicAdd(ccount, 1ull);
            if ((int64_t)pos < cap) {
                sbr_candidate c;
                c.rx = gx;
                c.order = j;
#pragma unroll
                for (int q = 0; q < SBR_MAX_ORDER; ++q) c.face[q] = q < j ? faces[q] : -1;
                c.ray = r;
                c.tan_err = tn;
                cand[pos] = c;
            }
        };
        if (J.rx_root < 0) {
            for (int x = 0; x < J.n_rx; ++x) receive(J.rx_first + x);
        } else {
            // stackless preorder walk of the job's receiver tree
            int32_t nd = J.rx_root;
            const int32_t end = rx_nodes[nd].skip;
            while (nd != end) {
                const RxNode N = rx_nodes[nd];
                if (!rx_ball_may_capture(o, d, D, t, mk(N.c[0], N.c[1], N.c[2]), N.rho, J.thl)) {
                    nd = N.skip;
                } else if (N.count == 0) {
                    nd = nd + 1;
                } else {
                    for (int q = 0; q < N.count; ++q) receive(rx_perm[N.first + q]);
                    nd = N.skip;
                }
            }
        }
        if (hit < 0 || j == K) {
            if (out_tri || out_t)
                for (int q = j + 1; q <= K; ++q) {
                    if (out_tri) out_tri[ro + q] = -1;
                    if (out_t) out_t[ro + q] = INFINITY;
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
}

template <bool COUNT, bool LDS>
__global__ __launch_bounds__(LDS ? 1024 : 256) void k_trace(CallDev call, LdsPlan L, SceneDev s0,
                                               uint32_t* __restrict__ queue,
                                               sbr_candidate* __restrict__ cand, int64_t cap,
                                               unsigned long long* __restrict__ ccount,
                                               int32_t* __restrict__ out_tri,
                                               double* __restrict__ out_t,
                                               int32_t* __restrict__ err,
                                               unsigned long long* __restrict__ tallies)
{
    if (LDS) stage_scene(s0, L);
    const int lane = threadIdx.x & 63;
    Tally tl{0u, 0u};
    uint32_t segs = 0, events = 0;
    for (;;) {
        uint32_t pk = 0;
        if (lane == 0) pk = atomicAdd(queue, 1u);
        pk = __builtin_amdgcn_readfirstlane(__shfl(pk, 0));
        if ((int64_t)pk >= call.n_packets) break;
        // the job of packet pk: the last job whose first packet is <= pk
        int lo = 0, hi = call.n_jobs - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (call.jobs[mid].packet_first <= (int64_t)pk)
                lo = mid;
            else
                hi = mid - 1;
        }
        const JobDev J = call.jobs[lo];
        const SceneDev S = LDS ? s0 : call.scenes[J.scene];
        const int64_t base = J.ray_begin + ((int64_t)pk - J.packet_first) * 64 * call.chunk;
        const int64_t end = J.ray_begin + J.ray_count;
        for (int c = 0; c < call.chunk; ++c) {
            const int64_t r = base + 64 * c + lane;
            if (r < end)
                trace_ray<COUNT, LDS>(S, L, J, call.rx, call.rx_nodes, call.rx_perm, r, cand, cap,
                                      ccount, out_tri, out_t, err, &tl, &segs, &events);
        }
    }
    if (COUNT) {
        atomicAdd(&tallies[0], (unsigned long long)segs);
        atomicAdd(&tallies[1], (unsigned long long)tl.nodes);
        atomicAdd(&tallies[2], (unsigned long long)tl.tris);
        atomicAdd(&tallies[3], (unsigned long long)events);
    }
}

template <bool COUNT, bool LDS>
static void launch_trace_t(const CallDev& call, const LdsPlan& L, const SceneDev& s0, int blocks,
                           uint32_t* queue, sbr_candidate* cand, int64_t cap,
                           unsigned long long* cand_count, int32_t* out_tri, double* out_t,
                           int32_t* err_flag, hipStream_t s, unsigned long long* tallies)
{
    hipLaunchKernelGGL((k_trace<COUNT, LDS>), dim3((unsigned)blocks), dim3(L.block),
                       LDS ? L.bytes : 0, s, call, L, s0, queue, cand, cap, cand_count, out_tri,
                       out_t, err_flag, tallies);
}

hipError_t launch_trace(const CallDev& call, const LdsPlan& L, const SceneDev& s0, int blocks,
                        uint32_t* queue, sbr_candidate* cand, int64_t cap,
                        unsigned long long* cand_count, int32_t* out_tri, double* out_t,
                        int32_t* err_flag, hipStream_t s, unsigned long long* tallies)
{
    if (call.n_packets <= 0 || blocks <= 0) return hipSuccess;
    const bool lds = L.bytes > 0;
    if (tallies && lds)
        launch_trace_t<true, true>(call, L, s0, blocks, queue, cand, cap, cand_count, out_tri,
                                   out_t, err_flag, s, tallies);
    else if (tallies)
        launch_trace_t<true, false>(call, L, s0, blocks, queue, cand, cap, cand_count, out_tri,
                                    out_t, err_flag, s, tallies);
    else if (lds)
        launch_trace_t<false, true>(call, L, s0, blocks, queue, cand, cap, cand_count, out_tri,
                                    out_t, err_flag, s, tallies);
    else
        launch_trace_t<false, false>(call, L, s0, blocks, queue, cand, cap, cand_count, out_tri,
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
