// refine.hip -- the iterative precise algorithm (Sec. III.B) and the path
// quantities, path test 2 and power (Sec. III.A, Sec. IV).
#include <math.h>

#include <algorithm>

#include "cone.h"
#include "follow.h"
#include "refine_queue.h"

namespace sbr {

// ===========================================================================
// Iterative precise algorithm (Sec. III.B)
// ===========================================================================
// Reflection points and incoming directions of the winning sub-ray.
__device__ static inline void store_geom(PathGeom* g, int k, const d3* pts, const d3* din)
{
    for (int j = 0; j < k; ++j) {
        g->pts[j] = pts[j];
        g->din[j] = din[j];
    }
}

// Start of the precise algorithm for one path: the launch ray that won path
// test 1 is the first axis.  Its error angle is the reception event's (the
// event was produced by the same FP64 arithmetic as a replay), so without a
// target no replay is needed; with a target the replay gives the unfolded
// lengths of the stop rule.  Returns false if the replay does not reproduce
// the path.
template <bool LDS, int BLK = 256>
__device__ static inline bool start_path(const SceneDev& S, const LdsPlan& L, double tan_tgt,
                                         const sbr_candidate& c, d3 tx, d3 rx, d3 axis,
                                         float delta, int32_t* err, double* tan, bool* met)
{
    *met = false;
    if (!(tan_tgt > 0.0)) {
        *tan = c.tan_err;
        return true;
    }
    Follow F0;
    if (!follow<LDS, BLK>(S, L, tx, axis, rx, c.order, c.face, delta, &F0, nullptr, nullptr, err))
        return false;
    *tan = F0.tan_err;
    *met = target_met(F0.tan_err, tan_tgt, F0.D, F0.Llast);
    return true;
}

__device__ static inline RefineOut stalled_at_start(d3 axis)
{
    RefineOut o;
    st3(o.axis, axis);
    o.tan_err = NAN;
    o.iters = 0;
    o.flags = SBR_PATH_STALLED;
    return o;
}

// Eight lanes per path: lane s traces sub-ray s (s < subrays); the group
// keeps the smallest error angle (ties: lower s) as the next axis.
template <bool LDS>
__global__ __launch_bounds__(256) void k_refine(CallDev call, LdsPlan L, SceneDev s0,
                                                const sbr_candidate* __restrict__ uniq,
                                                int64_t U_max, const int32_t* __restrict__ n_dev,
                                                RefineOut* __restrict__ out,
                                                PathGeom* __restrict__ geom,
                                                int32_t* __restrict__ err)
{
    if (LDS) stage_scene(s0, L);
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t p = gid >> 3;
    int s = (int)(gid & 7);
    const int64_t U = n_dev ? min(U_max, (int64_t)*n_dev) : U_max;
    if (p >= U) return;
    const sbr_candidate c = uniq[p];
    int jb = call.rx_job[c.rx];
    const JobDev J = call.jobs[jb];
    const SceneDev S = LDS ? s0 : call.scenes[J.scene];
    const d3 tx = mk(J.tx[0], J.tx[1], J.tx[2]);
    const d3 rx = mk(call.rx[3 * c.rx], call.rx[3 * c.rx + 1], call.rx[3 * c.rx + 2]);
    d3 axis = mk(J.dir[c.ray], J.dir[J.N + c.ray], J.dir[2 * J.N + c.ray]);
    double tan;
    bool met;
    if (!start_path<LDS>(S, L, J.tan_tgt, c, tx, rx, axis, J.delta, err, &tan, &met)) {
        if (s == 0) out[p] = stalled_at_start(axis);
        return;
    }
    uint32_t flags = met ? SBR_PATH_TARGET_MET : 0u;
    int32_t iters = 0;
    double rho = J.thl;
    for (int i = 1; i <= J.iterations && !met; ++i) {
        rho = rho / sqrt(3.0);
        d3 u, v;
        basis(axis, &u, &v);
        Follow F;
        bool ok = false;
        d3 gp[SBR_MAX_ORDER], gd[SBR_MAX_ORDER];
        if (s < J.subrays)
            ok = follow<LDS>(S, L, tx, subray(axis, u, v, rho, s), rx, c.order, c.face, J.delta, &F,
                             gp, gd, err);
        double bt = ok ? F.tan_err : INFINITY;
        int bs = ok ? s : 8;
        double myD = ok ? F.D : 0.0, myL = ok ? F.Llast : 0.0;
#pragma unroll
        for (int off = 1; off < 8; off <<= 1) {
            double ot = __shfl_xor(bt, off, 8);
            int os = __shfl_xor(bs, off, 8);
            if (ot < bt || (ot == bt && os < bs)) {
                bt = ot;
                bs = os;
            }
        }
        if (bs >= 8) {
            flags |= SBR_PATH_STALLED;
            break;
        }
        double wD = __shfl(myD, bs, 8), wL = __shfl(myL, bs, 8);
        if (s == bs) store_geom(geom + p, c.order, gp, gd);
        __threadfence_block();
        axis = subray(axis, u, v, rho, bs);
        tan = bt;
        iters = i;
        if (J.tan_tgt > 0.0 && target_met(bt, J.tan_tgt, wD, wL)) {
            flags |= SBR_PATH_TARGET_MET;
            met = true;
        }
    }
    if (s == 0) {
        RefineOut o;
        st3(o.axis, axis);
        o.tan_err = tan;
        o.iters = iters;
        o.flags = flags;
        out[p] = o;
    }
}

// One wave per path, two iterations per step.  Lane (s1, 7) traces first-level
// sub-ray s1; lane (s1, s2), s2 < subrays, traces sub-ray s2 of the cone that
// first-level sub-ray s1 would open in the next iteration.  Once the
// first-level winner b1 is known, the second-level winner among lanes
// (b1, *) is the next iteration's.  Every sub-ray is computed with exactly the
// arithmetic of the one-iteration-at-a-time order, so the result is the same
// bit for bit; the latency of two iterations becomes that of one.
template <bool LDS>
__global__ __launch_bounds__(256) void k_refine_la(CallDev call, LdsPlan L, SceneDev s0,
                                                   const sbr_candidate* __restrict__ uniq,
                                                   int64_t U_max,
                                                   const int32_t* __restrict__ n_dev,
                                                   RefineOut* __restrict__ out,
                                                   PathGeom* __restrict__ geom,
                                                   int32_t* __restrict__ err)
{
    if (LDS) stage_scene(s0, L);
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t p = gid >> 6;
    const int lane = (int)(gid & 63);
    const int s1 = lane >> 3, s2 = lane & 7;
    const int64_t U = n_dev ? min(U_max, (int64_t)*n_dev) : U_max;
    if (p >= U) return;
    const sbr_candidate c = uniq[p];
    int jb = call.rx_job[c.rx];
    jb = __builtin_amdgcn_readfirstlane(jb);  // one path per wave
    const JobDev J = call.jobs[jb];
    const SceneDev S = LDS ? s0 : call.scenes[J.scene];
    const d3 tx = mk(J.tx[0], J.tx[1], J.tx[2]);
    const d3 rx = mk(call.rx[3 * c.rx], call.rx[3 * c.rx + 1], call.rx[3 * c.rx + 2]);
    d3 axis = mk(J.dir[c.ray], J.dir[J.N + c.ray], J.dir[2 * J.N + c.ray]);
    double tan;
    bool met;
    if (!start_path<LDS>(S, L, J.tan_tgt, c, tx, rx, axis, J.delta, err, &tan, &met)) {
        if (lane == 0) out[p] = stalled_at_start(axis);
        return;
    }
    uint32_t flags = met ? SBR_PATH_TARGET_MET : 0u;
    int32_t iters = 0;
    double rho = J.thl;
    for (int i = 1; i <= J.iterations && !met; i += 2) {
        const double rho1 = rho / sqrt(3.0);
        const double rho2 = rho1 / sqrt(3.0);
        d3 u, v;
        basis(axis, &u, &v);
        const bool two = i + 1 <= J.iterations;
        const bool lvl1 = s2 == 7 && s1 < J.subrays;
        const bool lvl2 = two && s2 < J.subrays && s1 < J.subrays;
        Follow F;
        bool ok = false;
        d3 gp[SBR_MAX_ORDER], gd[SBR_MAX_ORDER];
        if (lvl1 || lvl2) {
            d3 dt = subray(axis, u, v, rho1, s1);
            if (lvl2) {
                d3 u2, v2;
                basis(dt, &u2, &v2);
                dt = subray(dt, u2, v2, rho2, s2);
            }
            ok = follow<LDS>(S, L, tx, dt, rx, c.order, c.face, J.delta, &F, gp, gd, err);
        }
        const double myD = ok ? F.D : 0.0, myL = ok ? F.Llast : 0.0;
        // first level: argmin over lanes (s1, 7)
        double k1 = (lvl1 && ok) ? F.tan_err : INFINITY;
        int b1 = (lvl1 && ok) ? s1 : 8;
#pragma unroll
        for (int off = 8; off < 64; off <<= 1) {
            double ot = __shfl_xor(k1, off);
            int ob = __shfl_xor(b1, off);
            if (ot < k1 || (ot == k1 && ob < b1)) {
                k1 = ot;
                b1 = ob;
            }
        }
        k1 = __shfl(k1, 7);
        b1 = __shfl(b1, 7);
        if (b1 >= 8) {
            flags |= SBR_PATH_STALLED;
            break;
        }
        double wD = __shfl(myD, b1 * 8 + 7), wL = __shfl(myL, b1 * 8 + 7);
        if (lane == b1 * 8 + 7) store_geom(geom + p, c.order, gp, gd);
        __threadfence_block();
        axis = subray(axis, u, v, rho1, b1);
        tan = k1;
        iters = i;
        rho = rho1;
        if (J.tan_tgt > 0.0 && target_met(k1, J.tan_tgt, wD, wL)) {
            flags |= SBR_PATH_TARGET_MET;
            break;
        }
        if (!two) break;
        // second level: argmin over lanes (b1, s2)
        double k2 = (lvl2 && ok && s1 == b1) ? F.tan_err : INFINITY;
        int b2 = (lvl2 && ok && s1 == b1) ? s2 : 8;
#pragma unroll
        for (int off = 1; off < 8; off <<= 1) {
            double ot = __shfl_xor(k2, off);
            int ob = __shfl_xor(b2, off);
            if (ot < k2 || (ot == k2 && ob < b2)) {
                k2 = ot;
                b2 = ob;
            }
        }
        k2 = __shfl(k2, b1 * 8);
        b2 = __shfl(b2, b1 * 8);
        if (b2 >= 8) {
            flags |= SBR_PATH_STALLED;
            break;
        }
        wD = __shfl(myD, b1 * 8 + b2);
        wL = __shfl(myL, b1 * 8 + b2);
        if (lane == b1 * 8 + b2) store_geom(geom + p, c.order, gp, gd);
        __threadfence_block();
        basis(axis, &u, &v);
        axis = subray(axis, u, v, rho2, b2);
        tan = k2;
        iters = i + 1;
        rho = rho2;
        if (J.tan_tgt > 0.0 && target_met(k2, J.tan_tgt, wD, wL)) {
            flags |= SBR_PATH_TARGET_MET;
            break;
        }
    }
    if (lane == 0) {
        RefineOut o;
        st3(o.axis, axis);
        o.tan_err = tan;
        o.iters = iters;
        o.flags = flags;
        out[p] = o;
    }
}

// One workgroup of 512 lanes per path, two iterations per step, every
// sub-ray's segments traced at once: lane t = sub (k + 1) + j checks segment j
// of sub-ray sub = 8 s1 + s2, where s2 = 7 marks first-level sub-ray s1 and
// s2 < subrays the second-level sub-ray s2 of the cone that s1 would open
// (as k_refine_la); at most 56 sub-rays of 9 segments fill 504 lanes.  A
// sub-ray's lanes may lie in different waves, so failures and error angles
// meet in LDS; the winners are picked level by level with the ties, stop
// rules and geometry of k_refine, so the result is the same bit for bit.
// resume = 0 starts every path (step 0 replays the launch ray with a
// target); resume = 1 continues the paths k_refine_seg left unfinished at
// its iteration limit (neither stalled nor at the target, iterations left),
// from their recorded axis, error, flags and iteration count (the cone
// radius rebuilt by the same successive divisions), and leaves the others.
template <bool LDS>
__global__ __launch_bounds__(512) void k_refine_seg2(CallDev call, LdsPlan L, SceneDev s0,
                                                     const sbr_candidate* __restrict__ uniq,
                                                     int64_t U_max,
                                                     const int32_t* __restrict__ n_dev,
                                                     RefineOut* __restrict__ out,
                                                     PathGeom* __restrict__ geom,
                                                     int32_t* __restrict__ err, int32_t resume)
{
    if (LDS) stage_scene(s0, L);
    __shared__ double sk[64], sD[64], sL[64];
    __shared__ int32_t sbad[64];
    const int64_t p = blockIdx.x;
    const int t = threadIdx.x;
    const int64_t U = n_dev ? min(U_max, (int64_t)*n_dev) : U_max;
    if (p >= U) return;  // uniform over the workgroup
    const sbr_candidate c = uniq[p];
    const JobDev J = call.jobs[call.rx_job[c.rx]];
    const SceneDev S = LDS ? s0 : call.scenes[J.scene];
    const d3 tx = mk(J.tx[0], J.tx[1], J.tx[2]);
    const d3 rx = mk(call.rx[3 * c.rx], call.rx[3 * c.rx + 1], call.rx[3 * c.rx + 2]);
    d3 axis = mk(J.dir[c.ray], J.dir[J.N + c.ray], J.dir[2 * J.N + c.ray]);
    const int k = __builtin_amdgcn_readfirstlane(c.order);
    int32_t faces[SBR_MAX_ORDER];
#pragma unroll
    for (int q = 0; q < SBR_MAX_ORDER; ++q) faces[q] = __builtin_amdgcn_readfirstlane(c.face[q]);
    const int K1 = k + 1;
    const int sub = t / K1, j = t - sub * K1;
    const int s1 = sub >> 3, s2 = sub & 7;
    const int S_ = J.subrays;
    double tan = c.tan_err;
    uint32_t flags = 0u;
    int32_t iters = 0;
    double rho = J.thl;
    int first = J.tan_tgt > 0.0 ? 0 : 1;
    if (resume) {
        const RefineOut o = out[p];
        if ((o.flags & (SBR_PATH_STALLED | SBR_PATH_TARGET_MET)) || o.iters >= J.iterations)
            return;  // uniform over the workgroup
        axis = mk(o.axis[0], o.axis[1], o.axis[2]);
        tan = o.tan_err;
        flags = o.flags;
        iters = o.iters;
        for (int q = 0; q < iters; ++q) rho = rho / sqrt(3.0);
        first = iters + 1;
    }
    Follow F{0.0, 0.0, 0.0};
    d3 pt = mk(0.0, 0.0, 0.0), din = pt;
    // the smallest error among slots base + q step, q < S_ (ties: lower q;
    // a slot whose sub-ray failed counts as infinite); 8 when none is finite
    auto argmin = [&](int base, int step, double* kb) {
        int b = 8;
        *kb = INFINITY;
        for (int q = 0; q < S_; ++q) {
            const int x = base + q * step;
            const double v = sbad[x] ? INFINITY : sk[x];
            if (v < *kb) {
                *kb = v;
                b = q;
            }
        }
        return b;
    };
    for (int i = first; i <= J.iterations; i += 2) {
        // step 0: lanes of sub-ray 0 replay the launch ray (start_path)
        const bool replay = i == 0;
        const double rho1 = rho / sqrt(3.0), rho2 = rho1 / sqrt(3.0);
        d3 u, v;
        basis(axis, &u, &v);
        const bool two = !replay && i + 1 <= J.iterations;
        const bool lvl1 = !replay && s2 == 7 && s1 < S_;
        const bool lvl2 = two && s1 < S_ && s2 < S_;
        const bool on = replay ? sub == 0 : (lvl1 || lvl2);
        if (t < 64) sbad[t] = 0;
        __syncthreads();
        bool ok = false;
        if (on) {
            d3 dt = axis;
            if (!replay) {
                dt = subray(axis, u, v, rho1, s1);
                if (lvl2) {
                    d3 u2, v2;
                    basis(dt, &u2, &v2);
                    dt = subray(dt, u2, v2, rho2, s2);
                }
            }
            ok = seg_lane<LDS, 512>(S, L, tx, dt, rx, k, j, faces, J.delta, &F, &pt, &din, err);
            if (!ok) sbad[sub] = 1;
            if (j == k) {
                sk[sub] = ok ? F.tan_err : INFINITY;
                sD[sub] = ok ? F.D : 0.0;
                sL[sub] = ok ? F.Llast : 0.0;
            }
        }
        if (!on && j == k && sub < 64) sk[sub] = INFINITY;
        __syncthreads();
        if (replay) {
            if (sbad[0]) {
                if (t == 0) out[p] = stalled_at_start(axis);
                return;
            }
            tan = sk[0];
            const bool met = target_met(tan, J.tan_tgt, sD[0], sL[0]);
            __syncthreads();
            if (met) {
                flags = SBR_PATH_TARGET_MET;
                break;
            }
            i = -1;  // the iterations start at 1
            continue;
        }
        // first level: slots (s1, 7)
        double k1;
        const int b1 = argmin(7, 8, &k1);
        if (b1 >= 8) {
            flags |= SBR_PATH_STALLED;
            break;
        }
        const double w1D = sD[b1 * 8 + 7], w1L = sL[b1 * 8 + 7];
        if (on && sub == b1 * 8 + 7 && j < k) {
            geom[p].pts[j] = pt;
            geom[p].din[j] = din;
        }
        axis = subray(axis, u, v, rho1, b1);
        tan = k1;
        iters = i;
        rho = rho1;
        if (J.tan_tgt > 0.0 && target_met(k1, J.tan_tgt, w1D, w1L)) {
            flags |= SBR_PATH_TARGET_MET;
            break;
        }
        if (!two) break;
        // second level: slots (b1, s2)
        double k2;
        const int b2 = argmin(b1 * 8, 1, &k2);
        if (b2 >= 8) {
            flags |= SBR_PATH_STALLED;
            break;
        }
        const double w2D = sD[b1 * 8 + b2], w2L = sL[b1 * 8 + b2];
        __threadfence_block();
        __syncthreads();  // the first level's geometry is written
        if (on && sub == b1 * 8 + b2 && j < k) {
            geom[p].pts[j] = pt;
            geom[p].din[j] = din;
        }
        basis(axis, &u, &v);
        axis = subray(axis, u, v, rho2, b2);
        tan = k2;
        iters = i + 1;
        rho = rho2;
        if (J.tan_tgt > 0.0 && target_met(k2, J.tan_tgt, w2D, w2L)) {
            flags |= SBR_PATH_TARGET_MET;
            break;
        }
        __syncthreads();  // every lane has read the slots of this step
    }
    if (t == 0) {
        RefineOut o;
        st3(o.axis, axis);
        o.tan_err = tan;
        o.iters = iters;
        o.flags = flags;
        out[p] = o;
    }
}

// One workgroup of 512 lanes per path, three iterations per step.  Lane
// (s1, s2, s3) = (t >> 6, (t >> 3) & 7, t & 7) traces the sub-ray that the
// sub-ray choices s1, then s2, then s3 would give; index 7 marks a level the
// lane does not reach, so lanes (s1, 7, 7) are the first level, (s1, s2, 7)
// the second and (s1, s2, s3) the third.  The winners are picked level by
// level through LDS; as in k_refine_la every sub-ray is computed with the
// arithmetic of the one-iteration-at-a-time order, so the result is the same
// bit for bit and three iterations take the latency of one.
template <bool LDS>
__global__ __launch_bounds__(512) void k_refine_la3(CallDev call, LdsPlan L, SceneDev s0,
                                                    const sbr_candidate* __restrict__ uniq,
                                                    int64_t U_max,
                                                    const int32_t* __restrict__ n_dev,
                                                    RefineOut* __restrict__ out,
                                                    PathGeom* __restrict__ geom,
                                                    int32_t* __restrict__ err)
{
    if (LDS) stage_scene(s0, L);
    __shared__ double sk[8], sD[8], sL[8];
    const int64_t p = blockIdx.x;
    const int t = threadIdx.x;
    const int s1 = t >> 6, s2 = (t >> 3) & 7, s3 = t & 7;
    const int64_t U = n_dev ? min(U_max, (int64_t)*n_dev) : U_max;
    if (p >= U) return;  // uniform over the workgroup
    const sbr_candidate c = uniq[p];
    const int jb = call.rx_job[c.rx];
    const JobDev J = call.jobs[jb];
    const SceneDev S = LDS ? s0 : call.scenes[J.scene];
    const d3 tx = mk(J.tx[0], J.tx[1], J.tx[2]);
    const d3 rx = mk(call.rx[3 * c.rx], call.rx[3 * c.rx + 1], call.rx[3 * c.rx + 2]);
    d3 axis = mk(J.dir[c.ray], J.dir[J.N + c.ray], J.dir[2 * J.N + c.ray]);
    double tan;
    bool met;
    if (!start_path<LDS, 512>(S, L, J.tan_tgt, c, tx, rx, axis, J.delta, err, &tan, &met)) {
        if (t == 0) out[p] = stalled_at_start(axis);
        return;
    }
    const int S_ = J.subrays;
    uint32_t flags = met ? SBR_PATH_TARGET_MET : 0u;
    int32_t iters = 0;
    double rho = J.thl;
    // the smallest of the 8 slots (ties: lower index); 8 when all are empty
    auto argmin8 = [&](double* k) {
        int b = 8;
        double kb = INFINITY;
        for (int q = 0; q < 8; ++q)
            if (k[q] < kb) {
                kb = k[q];
                b = q;
            }
        return b;
    };
    for (int i = 1; i <= J.iterations && !met; i += 3) {
        const double rho1 = rho / sqrt(3.0);
        const double rho2 = rho1 / sqrt(3.0);
        const double rho3 = rho2 / sqrt(3.0);
        const int levels = min(3, J.iterations - i + 1);
        d3 u, v;
        basis(axis, &u, &v);
        // A step of one or two levels (the last one, when I is not a
        // multiple of 3) packs its 7 + 49 sub-rays into the first wave,
        // lanes (a1, a2) = (t / 8, t % 8), so that this wave has its SIMD to
        // itself; the sub-rays are the same as with the full layout.
        const bool packed = levels < 3;
        const bool on = !packed || t < 64;
        const int a1 = packed ? (t >> 3) & 7 : s1, a2 = packed ? t & 7 : s2, a3 = packed ? 7 : s3;
        const bool lvl1 = on && a2 == 7 && a3 == 7 && a1 < S_;
        const bool lvl2 = on && levels >= 2 && a3 == 7 && a1 < S_ && a2 < S_;
        const bool lvl3 = on && levels >= 3 && a1 < S_ && a2 < S_ && a3 < S_;
        Follow F;
        bool ok = false;
        d3 gp[SBR_MAX_ORDER], gd[SBR_MAX_ORDER];
        if (lvl1 || lvl2 || lvl3) {
            d3 dt = subray(axis, u, v, rho1, a1);
            if (lvl2 || lvl3) {
                d3 u2, v2;
                basis(dt, &u2, &v2);
                dt = subray(dt, u2, v2, rho2, a2);
            }
            if (lvl3) {
                d3 u3, v3;
                basis(dt, &u3, &v3);
                dt = subray(dt, u3, v3, rho3, a3);
            }
            ok = follow<LDS, 512>(S, L, tx, dt, rx, c.order, c.face, J.delta, &F, gp, gd, err);
        }
        // first level: lanes (a1, 7, 7)
        if (on && a2 == 7 && a3 == 7) {
            sk[a1] = (lvl1 && ok) ? F.tan_err : INFINITY;
            sD[a1] = (lvl1 && ok) ? F.D : 0.0;
            sL[a1] = (lvl1 && ok) ? F.Llast : 0.0;
        }
        __syncthreads();
        const int b1 = argmin8(sk);
        const double k1 = b1 < 8 ? sk[b1] : INFINITY, w1D = b1 < 8 ? sD[b1] : 0.0,
                     w1L = b1 < 8 ? sL[b1] : 0.0;
        __syncthreads();
        if (b1 >= 8) {
            flags |= SBR_PATH_STALLED;
            break;
        }
        if (on && a1 == b1 && a2 == 7 && a3 == 7) store_geom(geom + p, c.order, gp, gd);
        axis = subray(axis, u, v, rho1, b1);
        tan = k1;
        iters = i;
        rho = rho1;
        if (J.tan_tgt > 0.0 && target_met(k1, J.tan_tgt, w1D, w1L)) {
            flags |= SBR_PATH_TARGET_MET;
            break;
        }
        if (levels < 2) break;
        // second level: lanes (b1, a2, 7)
        if (on && a1 == b1 && a3 == 7) {
            sk[a2] = (lvl2 && ok) ? F.tan_err : INFINITY;
            sD[a2] = (lvl2 && ok) ? F.D : 0.0;
            sL[a2] = (lvl2 && ok) ? F.Llast : 0.0;
        }
        __threadfence_block();
        __syncthreads();
        const int b2 = argmin8(sk);
        const double k2 = b2 < 8 ? sk[b2] : INFINITY, w2D = b2 < 8 ? sD[b2] : 0.0,
                     w2L = b2 < 8 ? sL[b2] : 0.0;
        __syncthreads();
        if (b2 >= 8) {
            flags |= SBR_PATH_STALLED;
            break;
        }
        if (on && a1 == b1 && a2 == b2 && a3 == 7) store_geom(geom + p, c.order, gp, gd);
        basis(axis, &u, &v);
        axis = subray(axis, u, v, rho2, b2);
        tan = k2;
        iters = i + 1;
        rho = rho2;
        if (J.tan_tgt > 0.0 && target_met(k2, J.tan_tgt, w2D, w2L)) {
            flags |= SBR_PATH_TARGET_MET;
            break;
        }
        if (levels < 3) break;
        // third level (full layout): lanes (b1, b2, a3)
        if (a1 == b1 && a2 == b2) {
            sk[a3] = (lvl3 && ok) ? F.tan_err : INFINITY;
            sD[a3] = (lvl3 && ok) ? F.D : 0.0;
            sL[a3] = (lvl3 && ok) ? F.Llast : 0.0;
        }
        __threadfence_block();
        __syncthreads();
        const int b3 = argmin8(sk);
        const double k3 = b3 < 8 ? sk[b3] : INFINITY, w3D = b3 < 8 ? sD[b3] : 0.0,
                     w3L = b3 < 8 ? sL[b3] : 0.0;
        __syncthreads();
        if (b3 >= 8) {
            flags |= SBR_PATH_STALLED;
            break;
        }
        if (a1 == b1 && a2 == b2 && a3 == b3) store_geom(geom + p, c.order, gp, gd);
        basis(axis, &u, &v);
        axis = subray(axis, u, v, rho3, b3);
        tan = k3;
        iters = i + 2;
        rho = rho3;
        if (J.tan_tgt > 0.0 && target_met(k3, J.tan_tgt, w3D, w3L)) {
            flags |= SBR_PATH_TARGET_MET;
            break;
        }
    }
    if (t == 0) {
        RefineOut o;
        st3(o.axis, axis);
        o.tan_err = tan;
        o.iters = iters;
        o.flags = flags;
        out[p] = o;
    }
}

// One wave per path, one iteration per step, every sub-ray's segments traced
// at once: lane (s, j) = (lane / (k + 1), lane % (k + 1)), s < subrays,
// checks segment j of sub-ray s (seg_lane), so a step waits for the slowest
// single segment (plus the short chain of expected-face hits that places
// it) instead of k + 1 traversals in a row.  A sub-ray is kept when none of
// its lanes failed; its error angle is on lane (s, k).  Winner, ties, stop
// rules and stored geometry are those of k_refine, so the result is the same
// bit for bit.  6 or 7 sub-rays of at most 9 segments fill at most 63 lanes.
template <bool LDS>
__global__ __launch_bounds__(256) void k_refine_seg(CallDev call, LdsPlan L, SceneDev s0,
                                                    const sbr_candidate* __restrict__ uniq,
                                                    int64_t U_max,
                                                    const int32_t* __restrict__ n_dev,
                                                    RefineOut* __restrict__ out,
                                                    PathGeom* __restrict__ geom,
                                                    int32_t* __restrict__ err, int32_t it_limit)
{
    if (LDS) stage_scene(s0, L);
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = gid >> 6;
    const int lane = (int)(gid & 63);
    const int64_t U = n_dev ? min(U_max, (int64_t)*n_dev) : U_max;
    if (p >= U) return;  // uniform over the wave
    const sbr_candidate c = uniq[p];
    const int jb = __builtin_amdgcn_readfirstlane(call.rx_job[c.rx]);  // one path per wave
    const JobDev J = call.jobs[jb];
    const SceneDev S = LDS ? s0 : call.scenes[J.scene];
    const d3 tx = mk(J.tx[0], J.tx[1], J.tx[2]);
    const d3 rx = mk(call.rx[3 * c.rx], call.rx[3 * c.rx + 1], call.rx[3 * c.rx + 2]);
    d3 axis = mk(J.dir[c.ray], J.dir[J.N + c.ray], J.dir[2 * J.N + c.ray]);
    const int k = __builtin_amdgcn_readfirstlane(c.order);
    int32_t faces[SBR_MAX_ORDER];
#pragma unroll
    for (int q = 0; q < SBR_MAX_ORDER; ++q) faces[q] = __builtin_amdgcn_readfirstlane(c.face[q]);
    const int K1 = k + 1;
    int s = 0, j = lane;
    while (j >= K1) {
        j -= K1;
        ++s;
    }
    Follow F{0.0, 0.0, 0.0};
    d3 pt = mk(0.0, 0.0, 0.0), din = pt;
    const bool act = s < J.subrays;
    const unsigned long long segs = ((1ull << K1) - 1) << (act ? s * K1 : 0);
    double tan = c.tan_err;
    bool met = false;
    uint32_t flags = 0u;
    int32_t iters = 0;
    double rho = J.thl;
    // Step 0 (with a target only) replays the launch ray on lanes (0, j), as
    // start_path does; steps 1.. are the iterations.  One loop, so that the
    // kernel holds a single copy of the segment search.  With it_limit > 0
    // the kernel stops after that many iterations; k_refine_seg2 resumes.
    const int32_t last = it_limit > 0 ? min(J.iterations, it_limit) : J.iterations;
    for (int i = J.tan_tgt > 0.0 ? 0 : 1; i <= last && !met; ++i) {
        d3 u, v, dt = axis;
        if (i > 0) {
            rho = rho / sqrt(3.0);
            basis(axis, &u, &v);
            dt = subray(axis, u, v, rho, s);
        }
        const bool on = i > 0 ? act : s == 0;
        bool ok = false;
        if (on) ok = seg_lane<LDS>(S, L, tx, dt, rx, k, j, faces, J.delta, &F, &pt, &din, err);
        const unsigned long long bad = __ballot(on && !ok);
        if (i == 0) {
            if (bad) {
                if (lane == 0) out[p] = stalled_at_start(axis);
                return;
            }
            tan = __shfl(F.tan_err, k);
            met = target_met(tan, J.tan_tgt, __shfl(F.D, k), __shfl(F.Llast, k));
            if (met) flags = SBR_PATH_TARGET_MET;
            continue;
        }
        const bool keep = act && j == k && (bad & segs) == 0;
        double bt = keep ? F.tan_err : INFINITY;
        int bs = keep ? s : 8;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            double ot = __shfl_xor(bt, off);
            int os = __shfl_xor(bs, off);
            if (ot < bt || (ot == bt && os < bs)) {
                bt = ot;
                bs = os;
            }
        }
        if (bs >= 8) {
            flags |= SBR_PATH_STALLED;
            break;
        }
        const int wl = bs * K1 + k;
        const double wD = __shfl(F.D, wl), wL = __shfl(F.Llast, wl);
        if (act && s == bs && j < k) {
            geom[p].pts[j] = pt;
            geom[p].din[j] = din;
        }
        __threadfence_block();
        axis = subray(axis, u, v, rho, bs);
        tan = bt;
        iters = i;
        if (J.tan_tgt > 0.0 && target_met(bt, J.tan_tgt, wD, wL)) {
            flags |= SBR_PATH_TARGET_MET;
            met = true;
        }
    }
    if (lane == 0) {
        RefineOut o;
        st3(o.axis, axis);
        o.tan_err = tan;
        o.iters = iters;
        o.flags = flags;
        out[p] = o;
    }
}

// ---------------------------------------------------------------------------
// The precise algorithm fed by a device work queue of sub-rays: one
// persistent launch refines every path of a call (of every job of a batch),
// whatever its order and iteration count.  A work item is one sub-ray of one
// path's current iteration.  Lanes take items in the order they were pushed;
// the lane that finishes the last sub-ray of an iteration (the path's pending
// count reaching zero) picks the winner (smallest error, ties: lower sub-ray)
// and either ends the path or pushes the next iteration's sub-rays.  Every
// sub-ray is traced with the arithmetic of k_refine, so the results are the
// same; the winner's geometry is not kept (the solve traces the final axis).
//
// Memory order.  Data one lane hands to another (the path state, the
// sub-ray slots, the items) is written and read only with device-scope
// atomic loads and stores, which are coherent across the chip's L2 caches
// on their own; every handoff is published by a release operation (items
// after the state, the pending count after the slot) and read through a
// value the reader has already loaded (the item names the path; the pending
// count tells the last lane to read the slots).  No acquire is used: on this
// chip an acquire at device scope invalidates the L2 cache, which would
// evict the scene that every lane is traversing.
// A lane leaves when every path is done, when its item index lies beyond the
// last item any path can push, or -- never in a correct run -- after a
// bounded wait (error flag 2).
// ---------------------------------------------------------------------------
constexpr int kQueueBlock = 256;

__device__ static inline unsigned long long q_item(int64_t p, int s)
{
    return ((unsigned long long)p << 3 | (unsigned long long)s) + 1ull;
}

template <int W>
__device__ static inline void q_store_words(void* dst, const void* src)
{
    unsigned long long* d = (unsigned long long*)dst;
    const unsigned long long* v = (const unsigned long long*)src;
#pragma unroll
    for (int k = 0; k < W; ++k)
        __hip_atomic_store(d + k, v[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int W>
__device__ static inline void q_load_words(void* dst, const void* src)
{
    unsigned long long* d = (unsigned long long*)dst;
    const unsigned long long* v = (const unsigned long long*)src;
#pragma unroll
    for (int k = 0; k < W; ++k)
        d[k] = __hip_atomic_load(v + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The state of path p, then (after a release fence) its sub-rays 0..S-1 of
// the state's iteration.
__device__ static inline void q_push(const RefineQueue& Q, int64_t p, const QState& q, int S)
{
    q_store_words<sizeof(QState) / 8>(Q.state + p, &q);
    const unsigned int base = atomicAdd(&Q.ctr[1], (unsigned int)S);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    for (int s = 0; s < S; ++s)
        if ((int64_t)base + s < Q.cap)
            __hip_atomic_store(&Q.items[base + s], q_item(p, s), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
}

__device__ static inline void q_finish(const RefineQueue& Q, RefineOut* out, int64_t p, d3 axis,
                                       double tan, int32_t iters, uint32_t flags)
{
    RefineOut o;
    st3(o.axis, axis);
    o.tan_err = tan;
    o.iters = iters;
    o.flags = flags;
    out[p] = o;
    __hip_atomic_fetch_add(&Q.ctr[2], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(256) void k_queue_init(CallDev call,
                                                    const sbr_candidate* __restrict__ uniq,
                                                    int64_t U_max, const int32_t* __restrict__ n_dev,
                                                    RefineQueue Q, RefineOut* __restrict__ out,
                                                    int32_t* __restrict__ err)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t U = n_dev ? min(U_max, (int64_t)*n_dev) : U_max;
    if (p >= U) return;
    const sbr_candidate c = uniq[p];
    const JobDev J = call.jobs[call.rx_job[c.rx]];
    const SceneDev S = call.scenes[J.scene];
    const d3 tx = mk(J.tx[0], J.tx[1], J.tx[2]);
    const d3 rx = mk(call.rx[3 * c.rx], call.rx[3 * c.rx + 1], call.rx[3 * c.rx + 2]);
    const d3 axis = mk(J.dir[c.ray], J.dir[J.N + c.ray], J.dir[2 * J.N + c.ray]);
    LdsPlan L0{};
    L0.block = 256;
    double tan;
    bool met;
    if (!start_path<false>(S, L0, J.tan_tgt, c, tx, rx, axis, J.delta, err, &tan, &met)) {
        q_finish(Q, out, p, axis, NAN, 0, SBR_PATH_STALLED);
        return;
    }
    if (met || J.iterations == 0) {
        q_finish(Q, out, p, axis, tan, 0, met ? SBR_PATH_TARGET_MET : 0u);
        return;
    }
    QState q;
    st3(q.axis, axis);
    q.rho = J.thl / sqrt(3.0);
    q.tan = tan;
    q.i = 1;
    q.iters = 0;
    q.flags = 0u;
    q.pending = J.subrays;
    q_push(Q, p, q, J.subrays);
}

// One work item v: trace its sub-ray, record it, and if it was the
// iteration's last, pick the winner and end the path or queue the next
// iteration's sub-rays.
__device__ static inline void q_process(const CallDev& call, const sbr_candidate* uniq,
                                        const RefineQueue& Q, unsigned long long v,
                                        RefineOut* out, int32_t* err)
{
    LdsPlan L0{};
    L0.block = kQueueBlock;
    const int64_t p = (int64_t)((v - 1ull) >> 3);
    const int s = (int)((v - 1ull) & 7ull);
    const sbr_candidate c = uniq[p];
    const JobDev J = call.jobs[call.rx_job[c.rx]];
    const SceneDev S = call.scenes[J.scene];
    const d3 tx = mk(J.tx[0], J.tx[1], J.tx[2]);
    const d3 rx = mk(call.rx[3 * c.rx], call.rx[3 * c.rx + 1], call.rx[3 * c.rx + 2]);
    QState q;
    q_load_words<sizeof(QState) / 8>(&q, Q.state + p);
    const d3 axis = ld3(q.axis);
    d3 u, w;
    basis(axis, &u, &w);
    Follow F;
    const bool ok = follow<false, kQueueBlock>(S, L0, tx, subray(axis, u, w, q.rho, s), rx,
                                               c.order, c.face, J.delta, &F, nullptr, nullptr,
                                               err);
    QSlot sl;
    sl.tan = ok ? F.tan_err : INFINITY;
    sl.D = ok ? F.D : 0.0;
    sl.Llast = ok ? F.Llast : 0.0;
    sl.ok = ok ? 1 : 0;
    sl.pad = 0;
    q_store_words<sizeof(QSlot) / 8>(Q.slot + 8 * p + s, &sl);
    const int32_t left = __hip_atomic_fetch_add(&Q.state[p].pending, -1, __ATOMIC_RELEASE,
                                                __HIP_MEMORY_SCOPE_AGENT);
    if (left != 1) return;
    // the iteration's last sub-ray: its winner, then the next iteration
    double bt = INFINITY;
    int bs = 8;
    QSlot win;
    for (int k = 0; k < J.subrays; ++k) {
        QSlot o;
        if (k == s)
            o = sl;
        else
            q_load_words<sizeof(QSlot) / 8>(&o, Q.slot + 8 * p + k);
        if (o.ok && o.tan < bt) {
            bt = o.tan;
            bs = k;
            win = o;
        }
    }
    if (bs >= 8) {
        q_finish(Q, out, p, axis, q.tan, q.iters, q.flags | SBR_PATH_STALLED);
        return;
    }
    const d3 naxis = subray(axis, u, w, q.rho, bs);
    uint32_t flags = q.flags;
    const bool met = J.tan_tgt > 0.0 && target_met(bt, J.tan_tgt, win.D, win.Llast);
    if (met) flags |= SBR_PATH_TARGET_MET;
    if (met || q.i >= J.iterations) {
        q_finish(Q, out, p, naxis, bt, q.i, flags);
        return;
    }
    QState nq;
    st3(nq.axis, naxis);
    nq.rho = q.rho / sqrt(3.0);
    nq.tan = bt;
    nq.i = q.i + 1;
    nq.iters = q.i;
    nq.flags = flags;
    nq.pending = J.subrays;
    q_push(Q, p, nq, J.subrays);
}

// The lanes of a wave wait for their items independently, and a lane whose
// item is there traces it in the same pass of the loop, so a lane never waits
// for a lane of its own wave.  The loop therefore has a single back edge: the
// empty asm hides the item index's value from the optimiser, which would
// otherwise thread the waiting path straight back to the item load and so
// make the wait an inner loop that the whole wave must leave together.
__global__ __launch_bounds__(kQueueBlock) void k_refine_queue(
    CallDev call, const sbr_candidate* __restrict__ uniq, int64_t U_max,
    const int32_t* __restrict__ n_dev, RefineQueue Q, RefineOut* __restrict__ out,
    int32_t* __restrict__ err)
{
    const uint32_t U = (uint32_t)(n_dev ? min(U_max, (int64_t)*n_dev) : U_max);
    int32_t idx = -1;
    uint32_t spins = 0;
    for (;;) {
        asm volatile("" : "+v"(idx));
        if (idx < 0) {
            idx = (int32_t)atomicAdd(&Q.ctr[0], 1u);
            spins = 0;
        }
        bool leave = (int64_t)(uint32_t)idx >= Q.cap;
        unsigned long long v = 0ull;
        if (!leave)
            v = __hip_atomic_load(&Q.items[(uint32_t)idx], __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
        if (v != 0ull) {
            q_process(call, uniq, Q, v, out, err);
            idx = -1;
        } else if (!leave) {
            if (__hip_atomic_load(&Q.ctr[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= U) {
                leave = true;
            } else if (++spins > (1u << 22)) {
                atomicOr(err, 2);
                leave = true;
            } else {
                __builtin_amdgcn_s_sleep(2);
            }
        }
        if (leave) break;
    }
}

hipError_t launch_refine_queue(const CallDev& call, const sbr_candidate* uniq, int64_t U_max,
                               const int32_t* n_dev, const RefineQueue& Q, int blocks,
                               RefineOut* out, int32_t* err, hipStream_t s)
{
    if (U_max <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_queue_init, dim3((unsigned)((U_max + 255) / 256)), dim3(256), 0, s, call,
                       uniq, U_max, n_dev, Q, out, err);
    hipLaunchKernelGGL(k_refine_queue, dim3((unsigned)std::max(blocks, 1)), dim3(kQueueBlock), 0, s,
                       call, uniq, U_max, n_dev, Q, out, err);
    return hipGetLastError();
}

hipError_t launch_refine(const CallDev& call, const LdsPlan& L, const LdsPlan& L3,
                         const SceneDev& s0, const sbr_candidate* uniq, int64_t U,
                         const int32_t* n_dev, int depth, RefineOut* out, PathGeom* geom,
                         int32_t* err, hipStream_t s, int32_t max_iters, int32_t tail_after)
{
    if (U <= 0) return hipSuccess;
    if (depth == kRefineSegments || depth == kRefineSegments2) {
        int32_t resume = 0;
        if (depth == kRefineSegments) {
            // one wave per path; with a tail, it stops after tail_after
            // iterations and the paths still running continue below
            const int32_t lim = tail_after > 0 && max_iters > tail_after ? tail_after : 0;
            dim3 grid((unsigned)((U * 64 + L.block - 1) / L.block));
            if (L.bytes > 0)
                hipLaunchKernelGGL(k_refine_seg<true>, grid, dim3(L.block), L.bytes, s, call, L,
                                   s0, uniq, U, n_dev, out, geom, err, lim);
            else
                hipLaunchKernelGGL(k_refine_seg<false>, grid, dim3(L.block), 0, s, call, L, s0,
                                   uniq, U, n_dev, out, geom, err, lim);
            if (lim == 0) return hipGetLastError();
            resume = 1;
        }
        // 512 lanes per path, two iterations per step (its own LDS plan, L3)
        if (L3.bytes > 0)
            hipLaunchKernelGGL(k_refine_seg2<true>, dim3((unsigned)U), dim3(512), L3.bytes, s,
                               call, L3, s0, uniq, U, n_dev, out, geom, err, resume);
        else
            hipLaunchKernelGGL(k_refine_seg2<false>, dim3((unsigned)U), dim3(512), 0, s, call,
                               LdsPlan{}, s0, uniq, U, n_dev, out, geom, err, resume);
        return hipGetLastError();
    }
    // the three-level kernel has its own LDS plan (L3), whatever the trace's
    if (depth >= 3) {
        if (L3.bytes > 0)
            hipLaunchKernelGGL(k_refine_la3<true>, dim3((unsigned)U), dim3(512), L3.bytes, s, call,
                               L3, s0, uniq, U, n_dev, out, geom, err);
        else
            hipLaunchKernelGGL(k_refine_la3<false>, dim3((unsigned)U), dim3(512), 0, s, call,
                               LdsPlan{}, s0, uniq, U, n_dev, out, geom, err);
        return hipGetLastError();
    }
    const bool lookahead = depth >= 2;
    int64_t threads = U * (lookahead ? 64 : 8);
    dim3 grid((unsigned)((threads + L.block - 1) / L.block));
    if (lookahead && L.bytes > 0)
        hipLaunchKernelGGL(k_refine_la<true>, grid, dim3(L.block), L.bytes, s, call, L, s0, uniq,
                           U, n_dev, out, geom, err);
    else if (lookahead)
        hipLaunchKernelGGL(k_refine_la<false>, grid, dim3(L.block), 0, s, call, L, s0, uniq, U,
                           n_dev, out, geom, err);
    else if (L.bytes > 0)
        hipLaunchKernelGGL(k_refine<true>, grid, dim3(L.block), L.bytes, s, call, L, s0, uniq, U,
                           n_dev, out, geom, err);
    else
        hipLaunchKernelGGL(k_refine<false>, grid, dim3(L.block), 0, s, call, L, s0, uniq, U, n_dev,
                           out, geom, err);
    return hipGetLastError();
}

// ===========================================================================
// Path quantities, path test 2 and power (Sec. III.A, Sec. IV)
// ===========================================================================
struct cx {
    double re, im;
};
__device__ static inline cx cadd(cx a, cx b) { return cx{a.re + b.re, a.im + b.im}; }
__device__ static inline cx csub(cx a, cx b) { return cx{a.re - b.re, a.im - b.im}; }
__device__ static inline cx cmulr(cx a, double r) { return cx{a.re * r, a.im * r}; }
__device__ static inline cx cdiv(cx a, cx b)
{
    double den = b.re * b.re + b.im * b.im;
    return cx{(a.re * b.re + a.im * b.im) / den, (a.im * b.re - a.re * b.im) / den};
}
__device__ static inline double cabs2(cx a) { return a.re * a.re + a.im * a.im; }
// principal square root
__device__ static inline cx csqrt_p(cx z)
{
    double r = hypot(z.re, z.im);
    if (r == 0.0) return cx{0.0, 0.0};
    if (z.re >= 0.0) {
        double t = sqrt(0.5 * (r + z.re));
        return cx{t, z.im / (2.0 * t)};
    }
    double t = sqrt(0.5 * (r - z.re));
    return cx{fabs(z.im) / (2.0 * t), copysign(t, z.im)};
}

// Fresnel reflection for relative permittivity er at incidence cosine c:
//   G_perp = (c - sqrt(er - s^2)) / (c + sqrt(er - s^2)),
//   G_par  = (er c - sqrt(er - s^2)) / (er c + sqrt(er - s^2)),
// and the unpolarized power reflectance 0.5 (|G_perp|^2 + |G_par|^2).
__device__ static inline double fresnel_avg(double c, cx er)
{
    double s2 = 1.0 - c * c;
    cx root = csqrt_p(csub(er, cx{s2, 0.0}));
    cx cc = cx{c, 0.0};
    cx gs = cdiv(csub(cc, root), cadd(cc, root));
    cx erc = cmulr(er, c);
    cx gp = cdiv(csub(erc, root), cadd(erc, root));
    return 0.5 * (cabs2(gs) + cabs2(gp));
}

__device__ static inline double refl_at(const SceneDev& S, int32_t f, d3 din)
{
    d3 n = face_normal(S, f);
    double c = fabs(dot(din, n)) / norm(din);
    int32_t m = S.fmat[f];
    return fresnel_avg(c, cx{S.eps[2 * m], S.eps[2 * m + 1]});
}

// P_r = P_t + 20 log10(lambda / (4 pi L)) + sum_j 10 log10(R_j)   [dBm]
__device__ static inline double path_power(double ptx, double freq, double L, const double* refl,
                                           int k)
{
    double lambda = kC0 / freq;
    double p = ptx + 20.0 * log10(lambda / (4.0 * kPi * L));
    // unrolled with a guard, so that a register array stays in registers
#pragma unroll
    for (int j = 0; j < SBR_MAX_ORDER; ++j)
        if (j < k) p += 10.0 * log10(refl[j]);
    return p;
}

// Point p inside face f: inside any of its triangles, barycentric tolerance 1e-9.
template <bool LDS>
__device__ static bool inside_face(const SceneDev& S, const LdsPlan& L, int32_t f, d3 p)
{
    const double tol = 1e-9;
    for (int32_t q = S.fstart[f]; q < S.fstart[f + 1]; ++q) {
        TriD T = tri_at<LDS>(S, L, S.ftris[q]);
        d3 v0 = mk(T.v0x, T.v0y, T.v0z), e1 = mk(T.e1x, T.e1y, T.e1z), e2 = mk(T.e2x, T.e2y, T.e2z);
        d3 w = sub(p, v0);
        double d00 = dot(e1, e1);
        double d01 = dot(e1, e2);
        double d11 = dot(e2, e2);
        double d20 = dot(w, e1);
        double d21 = dot(w, e2);
        double den = d00 * d11 - d01 * d01;
        if (den == 0.0) continue;
        double b = (d11 * d20 - d01 * d21) / den;
        double gg = (d00 * d21 - d01 * d20) / den;
        if (b >= -tol && gg >= -tol && b + gg <= 1.0 + tol) return true;
    }
    return false;
}

// Segment A -> B blocked by a triangle not of faces fa / fb, hit strictly
// inside (1e-9, 1 - 1e-9) of the segment parameter.
template <bool LDS>
__device__ static bool blocked(const SceneDev& S, const LdsPlan& L, d3 A, d3 B, int32_t fa,
                               int32_t fb, float delta, int32_t* err)
{
    HitRec h;
    return traverse<true, false, LDS>(S, L, A, sub(B, A), fa, fb, 1e-9, 1.0 - 1e-9, delta, &h,
                                      err) >= 0;
}

// Image-method points of a face sequence: images of Tx mirrored across the
// face planes in order, then back-projection from Rx.  Returns false when a
// back-projection parameter falls outside (0, 1) (first part of path test 2);
// the points are computed either way.
__device__ static bool image_points(const SceneDev& S, d3 tx, d3 rx, int k, const int32_t* faces,
                                    d3* pts)
{
    // loops unrolled with guards: every index is a constant, so the arrays
    // stay in registers
    d3 img[SBR_MAX_ORDER + 1];
    img[0] = tx;
#pragma unroll
    for (int j = 0; j < SBR_MAX_ORDER; ++j) {
        img[j + 1] = img[j];
        if (j < k) {
            int32_t f = faces[j];
            d3 n = face_normal(S, f);
            double c = S.fplane[4 * (size_t)f + 3];
            double dd = dot(n, img[j]) - c;
            img[j + 1] = sub(img[j], scl(2.0 * dd, n));
        }
    }
    bool ok = true;
    d3 X = rx;
#pragma unroll
    for (int j = SBR_MAX_ORDER - 1; j >= 0; --j) {
        pts[j] = mk(0.0, 0.0, 0.0);
        if (j < k) {
            int32_t f = faces[j];
            d3 n = face_normal(S, f);
            double c = S.fplane[4 * (size_t)f + 3];
            d3 dir = sub(img[j + 1], X);
            double den = dot(n, dir);
            double s = (c - dot(n, X)) / den;
            if (!(s > 0.0 && s < 1.0)) ok = false;
            pts[j] = add(X, scl(s, dir));
            X = pts[j];
        }
    }
    return ok;
}

// a[j] of an 8-entry point list by value (no dynamic index)
__device__ static inline d3 pick8(const d3* a, int j)
{
    d3 r = a[0];
#pragma unroll
    for (int q = 1; q < SBR_MAX_ORDER; ++q)
        if (q == j) r = a[q];
    return r;
}

__device__ static inline double poly_length(d3 tx, const d3* p, int k, d3 rx)
{
    double L = 0.0;
    d3 prev = tx;
#pragma unroll
    for (int j = 0; j < SBR_MAX_ORDER; ++j)
        if (j < k) {
            L = L + norm(sub(p[j], prev));
            prev = p[j];
        }
    L = L + norm(sub(rx, prev));
    return L;
}

// Path quantities of one path from its reflection points P[0..k) and the
// incoming directions Din (the refined path: the final ray's; the exact
// path: the image points), the departure direction aod given.
struct PathQ {
    double L, delay, pw;
    d3 aod, aoa;
};

__device__ static inline PathQ path_quantities(const SceneDev& S, const JobDev& J,
                                               const sbr_candidate& c, d3 tx, d3 rx, d3 aod,
                                               const d3* P, const d3* Din)
{
    const int k = c.order;
    PathQ q;
    // Tx -> reflection points -> Rx
    q.L = poly_length(tx, P, k, rx);
    q.delay = q.L / kC0;
    q.aod = aod;
    const d3 lastq = k > 0 ? pick8(P, k - 1) : tx;
    q.aoa = normalize(sub(lastq, rx));
    double refl[SBR_MAX_ORDER];
#pragma unroll
    for (int j = 0; j < SBR_MAX_ORDER; ++j) refl[j] = j < k ? refl_at(S, c.face[j], Din[j]) : 1.0;
    q.pw = path_power(J.tx_power_dbm, J.freq_hz, q.L, refl, k);
    return q;
}

// Path test 2 and the exact path, one wave per path.  Lane 1 + j checks
// segment j of the image-method path (reflection point j inside its face,
// segment j unobstructed), so the test costs one traversal of latency
// instead of k + 1; lane 1 then forms the exact path's quantities.  With
// geom0, lanes 32 + j trace segment j of the path's launch ray (seg_lane)
// into geom0[p], the geometry of a path that the refinement ends without an
// iteration: as follow() writes it, a segment's reflection point and
// incoming direction when it and every segment before it meet the expected
// faces, zeros from the first that does not.  None of this needs a
// refinement result, so it runs beside the refinement.  Writes the record's
// identity, the exact_* fields, the INVALID flag (as the whole flags field)
// and keep.
__global__ __launch_bounds__(256) void k_solve_exact(CallDev call,
                                                     const sbr_candidate* __restrict__ uniq,
                                                     int64_t U_max,
                                                     const int32_t* __restrict__ n_dev,
                                                     sbr_path* __restrict__ paths,
                                                     int32_t* __restrict__ keep,
                                                     PathGeom* __restrict__ geom0,
                                                     int32_t* __restrict__ err)
{
    LdsPlan L{};
    L.block = 256;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = gid >> 6;
    const int lane = (int)(gid & 63);
    const int64_t U = n_dev ? min(U_max, (int64_t)*n_dev) : U_max;
    if (p >= U) return;  // uniform over the wave
    const sbr_candidate c = uniq[p];
    const JobDev J = call.jobs[__builtin_amdgcn_readfirstlane(call.rx_job[c.rx])];
    const SceneDev S = call.scenes[J.scene];
    const float delta = J.delta;
    const int k = __builtin_amdgcn_readfirstlane(c.order);
    int32_t faces[SBR_MAX_ORDER];
#pragma unroll
    for (int q = 0; q < SBR_MAX_ORDER; ++q) faces[q] = __builtin_amdgcn_readfirstlane(c.face[q]);
    const d3 tx = mk(J.tx[0], J.tx[1], J.tx[2]);
    const d3 rx = mk(call.rx[3 * c.rx], call.rx[3 * c.rx + 1], call.rx[3 * c.rx + 2]);
    // the launch ray's segments (geom0)
    const int jg = lane - 32;
    bool gok = false;
    d3 gpt = mk(0.0, 0.0, 0.0), gdin = gpt;
    if (geom0 && jg >= 0 && jg < k) {
        const d3 axis0 = mk(J.dir[c.ray], J.dir[J.N + c.ray], J.dir[2 * J.N + c.ray]);
        Follow F;
        gok = seg_lane<false>(S, L, tx, axis0, rx, k, jg, faces, delta, &F, &gpt, &gdin, err);
    }
    const unsigned long long gfail = __ballot(geom0 && jg >= 0 && jg < k && !gok);
    if (geom0 && jg >= 0 && jg < SBR_MAX_ORDER) {
        // written when segments 0 .. jg all meet their faces
        const bool w = jg < k && (gfail & (((2ull << jg) - 1) << 32)) == 0;
        PathGeom* gm = geom0 + p;
        gm->pts[jg] = w ? gpt : mk(0.0, 0.0, 0.0);
        gm->din[jg] = w ? gdin : mk(0.0, 0.0, 0.0);
    }
    d3 ep[SBR_MAX_ORDER];
    const bool geo_ok = image_points(S, tx, rx, k, faces, ep);
    bool bad = false;
    if (geo_ok && lane >= 1 && lane <= k + 1) {
        // by value from the register lists (a dynamic index would move
        // them to private memory)
        const int j = lane - 1;
        const d3 ej = pick8(ep, j), ejm = pick8(ep, j - 1);
        const int32_t fj = face_at(faces, j), fjm = face_at(faces, j - 1);
        if (j < k && !inside_face<false>(S, L, fj, ej)) {
            bad = true;
        } else {
            d3 Pa = j == 0 ? tx : ejm;
            d3 Pb = j < k ? ej : rx;
            int32_t fa = j == 0 ? -1 : fjm;
            int32_t fb = j < k ? fj : -1;
            bad = blocked<false>(S, L, Pa, Pb, fa, fb, delta, err);
        }
    }
    const bool any_bad = __ballot(bad) != 0;
    if (lane != 1) return;
    // the exact path: the image points; incoming direction = point minus
    // the previous point
    d3 Din[SBR_MAX_ORDER];
    d3 prev = tx;
#pragma unroll
    for (int j = 0; j < SBR_MAX_ORDER; ++j) {
        Din[j] = sub(ep[j], prev);
        prev = ep[j];
    }
    const d3 firstq = k > 0 ? ep[0] : rx;
    const PathQ E = path_quantities(S, J, c, tx, rx, normalize(sub(firstq, tx)), ep, Din);
    sbr_path* o = paths + p;
    o->rx = c.rx;
    o->order = k;
    for (int q = 0; q < SBR_MAX_ORDER; ++q) o->face[q] = c.face[q];
    o->launch_ray = c.ray;
    o->init_tan_err = c.tan_err;
    o->exact_length_m = E.L;
    o->exact_delay_s = E.delay;
    st3(o->exact_aod, E.aod);
    st3(o->exact_aoa, E.aoa);
    o->exact_power_dbm = E.pw;
    const bool ok = geo_ok && !any_bad;
    o->flags = ok ? 0u : SBR_PATH_INVALID;
    keep[p] = (ok || J.keep_invalid) ? 1 : 0;
}

// The refined path, one lane per path, after the refinement and
// k_solve_exact: its quantities from the final ray's reflection points and
// incoming directions, and the refinement's flags.  The refinement stored
// the final ray's geometry in geom[p]; a path without iterations has the
// launch ray's, traced by k_solve_exact into geom0[p]; without geom0, or
// when the refinement stored none (replay), the final axis is traced here.
// Every trace of an axis uses the arithmetic of the winning sub-ray's, so
// the geometry is the same whichever kernel forms it.
__global__ __launch_bounds__(64) void k_solve_refined(CallDev call,
                                                      const sbr_candidate* __restrict__ uniq,
                                                      const RefineOut* __restrict__ rf,
                                                      PathGeom* __restrict__ geom,
                                                      const PathGeom* __restrict__ geom0,
                                                      int64_t U_max,
                                                      const int32_t* __restrict__ n_dev,
                                                      sbr_path* __restrict__ paths,
                                                      int32_t* __restrict__ err, int replay)
{
    LdsPlan L{};
    L.block = 64;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t U = n_dev ? min(U_max, (int64_t)*n_dev) : U_max;
    if (p >= U) return;
    const sbr_candidate c = uniq[p];
    const JobDev J = call.jobs[call.rx_job[c.rx]];
    const SceneDev S = call.scenes[J.scene];
    const int k = c.order;
    const d3 tx = mk(J.tx[0], J.tx[1], J.tx[2]);
    const d3 rx = mk(call.rx[3 * c.rx], call.rx[3 * c.rx + 1], call.rx[3 * c.rx + 2]);
    const RefineOut R = rf[p];
    const d3 axis = ld3(R.axis);
    const bool from0 = R.iters == 0 && geom0;
    PathGeom* gm = geom + p;
    if (!from0 && (R.iters == 0 || replay)) {
        for (int j = 0; j < SBR_MAX_ORDER; ++j) {
            gm->pts[j] = mk(0.0, 0.0, 0.0);
            gm->din[j] = mk(0.0, 0.0, 0.0);
        }
        Follow F;
        follow<false, 64>(S, L, tx, axis, rx, k, c.face, J.delta, &F, gm->pts, gm->din, err);
    }
    const PathGeom* g = from0 ? geom0 + p : gm;
    d3 P[SBR_MAX_ORDER], Din[SBR_MAX_ORDER];
#pragma unroll
    for (int j = 0; j < SBR_MAX_ORDER; ++j) {
        P[j] = g->pts[j];
        Din[j] = g->din[j];
    }
    const PathQ Q = path_quantities(S, J, c, tx, rx, axis, P, Din);
    sbr_path* o = paths + p;
    o->iters_used = R.iters;
    o->flags |= R.flags;
    o->tan_err = R.tan_err;
    st3(o->axis, axis);
    o->length_m = Q.L;
    o->delay_s = Q.delay;
    st3(o->aod, Q.aod);
    st3(o->aoa, Q.aoa);
    o->power_dbm = Q.pw;
    o->err_angle_deg = atan(R.tan_err) * (180.0 / kPi);
}

hipError_t launch_solve_exact(const CallDev& call, const sbr_candidate* uniq, int64_t U,
                              const int32_t* n_dev, sbr_path* paths, int32_t* keep,
                              PathGeom* geom0, int32_t* err, hipStream_t s)
{
    if (U <= 0) return hipSuccess;
    const int64_t threads = U * 64;
    hipLaunchKernelGGL(k_solve_exact, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s,
                       call, uniq, U, n_dev, paths, keep, geom0, err);
    return hipGetLastError();
}

hipError_t launch_solve_refined(const CallDev& call, const sbr_candidate* uniq,
                                const RefineOut* rf, PathGeom* geom, const PathGeom* geom0,
                                int64_t U, const int32_t* n_dev, sbr_path* paths, int32_t* err,
                                hipStream_t s, bool replay)
{
    if (U <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_solve_refined, dim3((unsigned)((U + 63) / 64)), dim3(64), 0, s, call,
                       uniq, rf, geom, geom0, U, n_dev, paths, err, replay ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_solve(const CallDev& call, const sbr_candidate* uniq, const RefineOut* rf,
                        PathGeom* geom, int64_t U, const int32_t* n_dev, sbr_path* paths,
                        int32_t* keep, int32_t* err, hipStream_t s, bool replay)
{
    hipError_t e = launch_solve_exact(call, uniq, U, n_dev, paths, keep, nullptr, err, s);
    if (e != hipSuccess) return e;
    return launch_solve_refined(call, uniq, rf, geom, nullptr, U, n_dev, paths, err, s, replay);
}

// The three-level kernel also has 192 bytes of static LDS: its dynamic
// limit is set separately, to what the caller's plans for it may use.
hipError_t refine_la3_set_lds_limit(int bytes)
{
    hipError_t e = hipFuncSetAttribute((const void*)k_refine_la3<true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_refine_seg2<true>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t refine_set_lds_limit(int bytes)
{
    hipError_t e = hipFuncSetAttribute((const void*)k_refine<true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)k_refine_la<true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_refine_seg<true>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

}  // namespace sbr
