// trace.hip -- SBR tracing and reception (Sec. III.A): closest hit per
// segment, specular reflection up to K bounces, and the cone reception test
// of every receiver on every segment (eq. (3)), fused, one lane per launch
// ray.  Jobs with many receivers walk a box tree over them and run the
// exact test only where a conservative cull lets a receiver through.  The
// kernel is persistent: waves take packets of 64 x chunk rays from a device
// queue until it is empty, so jobs of uneven size are balanced over the
// machine, and lanes whose ray has ended take the packet's next ray, so rays
// of uneven length keep the lanes busy.
#include <math.h>

#include <algorithm>

#include "grid.h"
#include "internal.h"
#include "traverse.h"

namespace sbr {

// Per-lane state of the ray a lane is tracing: its current segment starts at
// o with direction d after j reflections on faces[0..j), unfolded length D.
// The faces are only ever indexed by unrolled constant indices, so the whole
// state stays in registers.
struct RayState {
    d3 o, d;
    double D;
    int64_t r;  // launch ray index; -1: the lane is idle
    int32_t prev, j;
    int32_t faces[SBR_MAX_ORDER];
};

__device__ static inline void start_ray(const JobDev& J, int64_t i, RayState& R)
{
    const int64_t r = J.order ? (int64_t)gld((const int32_t*)J.order + i) : i;
    R.r = r;
    R.o = mk(J.tx[0], J.tx[1], J.tx[2]);
    R.d = mk(gld(J.dir + r), gld(J.dir + J.N + r), gld(J.dir + 2 * J.N + r));
    R.D = 0.0;
    R.prev = -1;
    R.j = 0;
#pragma unroll
    for (int q = 0; q < SBR_MAX_ORDER; ++q) R.faces[q] = -1;
}

// faces[j] = f without a dynamic index.
__device__ static inline void set_face(RayState& R, int32_t j, int32_t f)
{
#pragma unroll
    for (int q = 0; q < SBR_MAX_ORDER; ++q) R.faces[q] = q == j ? f : R.faces[q];
}

// ---------------------------------------------------------------------------
// FP32 pre-test of reception.  capture() decides in FP64; this cheaper test
// only rejects receivers that capture() would reject too.  With u = 2^-24,
// M = max(|o|inf, |rx|inf) and v = rx - o, the FP32 foot parameter tc is
// within 24 u M of the exact one and the FP32 perpendicular within 38 u M of
// the exact distance, so a capture needs
//   tc > -dl,   tc - dl <= t,   |w|^2 <= (thl (D + tc + dl) + dl)^2 (1 + small)
// with dl = 2^-18 (M + D) = 64 u (M + D); the thresholds below carry factors
// 1 + 2^-20 (t, thl) and 1 + 2^-18 (the squared bound) for their own
// roundings, and every comparison is written so that NaN never rejects.
struct Seg32 {
    float ox, oy, oz, dx, dy, dz, D, t, thl, dl;
};

__device__ static inline Seg32 seg32(const RayState& R, double t, double thl)
{
    Seg32 g;
    g.ox = (float)R.o.x;
    g.oy = (float)R.o.y;
    g.oz = (float)R.o.z;
    g.dx = (float)R.d.x;
    g.dy = (float)R.d.y;
    g.dz = (float)R.d.z;
    g.D = (float)R.D;
    const float up = 1.0f + 0x1p-20f;
    g.t = (float)t * up;
    g.thl = (float)thl * up;
    g.dl = 0x1p-18f * (fmaxf(fmaxf(fabsf(g.ox), fabsf(g.oy)), fabsf(g.oz)) + g.D);
    return g;
}

__device__ static inline bool rx_may_capture32(const Seg32& g, float4 r)
{
    const float vx = r.x - g.ox, vy = r.y - g.oy, vz = r.z - g.oz;
    const float tc = fmaf(vz, g.dz, fmaf(vy, g.dy, vx * g.dx));
    const float dl = fmaf(0x1p-18f, r.w, g.dl);
    if (tc + dl <= 0.0f) return false;
    if (tc - dl > g.t) return false;
    const float wx = fmaf(-tc, g.dx, vx), wy = fmaf(-tc, g.dy, vy), wz = fmaf(-tc, g.dz, vz);
    const float ww = fmaf(wz, wz, fmaf(wy, wy, wx * wx));
    const float A = fmaf(g.thl, (g.D + tc) + dl, dl);
    return !(ww > (A * A) * (1.0f + 0x1p-18f));
}

// Bounding box of a job's FP32 receivers and the largest of their max
// |coordinate|, reduced over the wave (all 64 lanes take part).
struct RxBox {
    float lo[3], hi[3], w;
};

__device__ static RxBox rx_box(const float4* __restrict__ rx32, int32_t first, int32_t n)
{
    RxBox b;
    for (int a = 0; a < 3; ++a) {
        b.lo[a] = INFINITY;
        b.hi[a] = -INFINITY;
    }
    b.w = 0.0f;
    for (int32_t x = (int32_t)(threadIdx.x & 63); x < n; x += 64) {
        const float4 r = gld(rx32 + first + x);
        b.lo[0] = fminf(b.lo[0], r.x);
        b.lo[1] = fminf(b.lo[1], r.y);
        b.lo[2] = fminf(b.lo[2], r.z);
        b.hi[0] = fmaxf(b.hi[0], r.x);
        b.hi[1] = fmaxf(b.hi[1], r.y);
        b.hi[2] = fmaxf(b.hi[2], r.z);
        b.w = fmaxf(b.w, r.w);
    }
    for (int off = 32; off >= 1; off >>= 1)
        for (int a = 0; a < 3; ++a) {
            b.lo[a] = fminf(b.lo[a], __shfl_xor(b.lo[a], off));
            b.hi[a] = fmaxf(b.hi[a], __shfl_xor(b.hi[a], off));
        }
    for (int off = 32; off >= 1; off >>= 1) b.w = fmaxf(b.w, __shfl_xor(b.w, off));
    // wave-uniform: held in scalar registers
    auto uni = [](float v) {
        return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
    };
    for (int a = 0; a < 3; ++a) {
        b.lo[a] = uni(b.lo[a]);
        b.hi[a] = uni(b.hi[a]);
    }
    b.w = uni(b.w);
    return b;
}

// Whether any receiver in box b can pass rx_may_capture32 on segment g.  A
// receiver that passes is r = o + tc d + w with -dl < tc <= t + dl and
// |w| <= A(tc) = c0 + thl tc up to factors 1 + 2^-19 (c0 = thl (D + dl) + dl),
// so along each axis r lies between the linear functions
// o + tc (d -+ thl) -+ c0 of tc, whose extremes over that range are at its
// ends (infinite for an escaping segment on the side it heads to).  A margin
// of 0.1% of the coordinates, the unfolded length and the segment covers the
// roundings of this bound and of the pre-test.
__device__ static inline bool rx_box_may(const Seg32& g, const RxBox& b)
{
    const float dl = fmaf(0x1p-18f, b.w, g.dl);
    const float c0 = fmaf(g.thl, g.D + dl, dl);
    const float T = g.t + dl;
    const float M = fmaxf(fmaxf(fabsf(g.ox), fabsf(g.oy)), fabsf(g.oz)) + g.D;
    const float m = 1e-3f * (1.0f + M + (T < INFINITY ? T : 0.0f));
    const float o[3] = {g.ox, g.oy, g.oz}, d[3] = {g.dx, g.dy, g.dz};
    bool may = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float dm = d[a] - g.thl, dp = d[a] + g.thl;
        const float lo = o[a] + (dm >= 0.0f ? -dl * dm : T * dm) - c0 - m;
        const float hi = o[a] + (dp <= 0.0f ? -dl * dp : T * dp) + c0 + m;
        may = may && !(lo > b.hi[a]) && !(hi < b.lo[a]);
    }
    return may;
}

// Per-call preparation in one launch: the FP32 receivers, and zeroing of
// n_zero 32-bit words (the call's counters).
__global__ void k_prep(const double* __restrict__ rx, int64_t n, float4* __restrict__ out,
                       uint32_t* __restrict__ zero, int32_t n_zero)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_zero) zero[i] = 0u;
    if (i >= n) return;
    const float x = (float)rx[3 * i], y = (float)rx[3 * i + 1], z = (float)rx[3 * i + 2];
    // rounding to FP32 may lower a magnitude by 2^-24 relative; the bound
    // dl keeps a factor 1.6 of slack for that
    out[i] = make_float4(x, y, z, fmaxf(fmaxf(fabsf(x), fabsf(y)), fabsf(z)));
}

hipError_t launch_rx32(const double* rx, int64_t n, float4* out, hipStream_t s, void* zero,
                       size_t zero_bytes)
{
    const int32_t nz = (int32_t)(zero_bytes / 4);
    const int64_t m = std::max<int64_t>(n, nz);
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_prep, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, rx, n, out,
                       (uint32_t*)zero, nz);
    return hipGetLastError();
}

// Append the reception event of receiver gx at rx on the lane's current
// segment (closed by the hit at t) when it passes the cone test of eq. (3).
__device__ static inline void receive_at(const JobDev& J, const RayState& R, double t, int32_t gx,
                                         d3 rx, sbr_candidate* __restrict__ cand, int64_t cap,
                                         unsigned long long* __restrict__ ccount,
                                         uint32_t* events, bool count)
{
    double tn;
    if (!capture(R.o, R.d, R.D, t, rx, J.thl, &tn)) return;
    if (count) *events += 1;
    unsigned long long pos = atomicAdd(ccount, 1ull);
    if ((int64_t)pos < cap) {
        sbr_candidate c;
        c.rx = gx;
        c.order = R.j;
#pragma unroll
        for (int q = 0; q < SBR_MAX_ORDER; ++q) c.face[q] = q < R.j ? R.faces[q] : -1;
        c.ray = R.r;
        c.tan_err = tn;
        cand[pos] = c;
    }
}

__device__ static inline void receive(const JobDev& J, const double* __restrict__ rx_all,
                                      const RayState& R, double t, int32_t gx,
                                      sbr_candidate* __restrict__ cand, int64_t cap,
                                      unsigned long long* __restrict__ ccount, uint32_t* events,
                                      bool count)
{
    d3 rx = mk(gld(rx_all + 3 * gx), gld(rx_all + 3 * gx + 1), gld(rx_all + 3 * gx + 2));
    receive_at(J, R, t, gx, rx, cand, cap, ccount, events, count);
}

// The directions of the rays next..pend-1 of a streamed grid (see CallDev):
// the wave waits (lane 0, bounded) until the ring setup has published the
// progress the packet's rays need, then forms their directions with the
// setup's arithmetic (bit-identical to k_grid_dirs) and stores them in the
// job's direction array, from which the lanes then start their rays.
// The streamed grid's arguments, kept in LDS for the whole launch so that
// they take no scalar registers in the trace loop.
struct StreamArgs {
    const char* scr;
    const unsigned long long* prog;
    uint32_t epoch;
    int32_t n, check;
    uint32_t spin;
};

__device__ static void stream_dirs(const StreamArgs& sa, uint32_t* seen, const JobDev& J,
                                   int64_t next, int64_t pend, int lane, int32_t* err)
{
    uint32_t need = 0;
    for (int64_t b = next; b < pend; b += 64) {
        const int64_t i = b + lane;
        if (i < pend) {
            const int64_t r = J.order ? (int64_t)gld((const int32_t*)J.order + i) : i;
            need = max(need, grid_need(sa.n, r));
        }
    }
    for (int off = 32; off >= 1; off >>= 1) need = max(need, (uint32_t)__shfl_xor((int)need, off));
    // The progress word is read only when the packet needs more than the
    // workgroup has already seen (*seen, in LDS): every wave of the machine
    // reading one word for every packet would queue them all at the memory
    // channel that holds it.
    if (need > *seen && lane == 0) {
        // once one wave has timed out, the others no longer wait (the call
        // reports the error)
        const bool late =
            (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 4) != 0;
        for (uint32_t spin = 0; !late; ++spin) {
            const unsigned long long v =
                __hip_atomic_load(sa.prog, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((uint32_t)(v >> 32) == sa.epoch && (uint32_t)v >= need) {
                atomicMax(seen, (uint32_t)v);
                break;
            }
            if (spin > sa.spin) {
                atomicOr(err, 4);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    const double scale = ldexp(1.0, sa.check);
    CoefPtr F = coef_table();
    asm volatile("" : "+s"(F));  // keeps the coefficient loads in this branch
    double* dir = (double*)J.dir;
    for (int64_t b = next; b < pend; b += 64) {
        const int64_t i = b + lane;
        if (i < pend) {
            const int64_t r = J.order ? (int64_t)gld((const int32_t*)J.order + i) : i;
            const d3 d = grid_dir_of<GridAtomicLoads>(sa.n, sa.scr, (uint32_t)r, scale, F);
            dir[r] = d.x;
            dir[J.N + r] = d.y;
            dir[2 * J.N + r] = d.z;
        }
    }
    // lanes start rays whose directions other lanes of the wave stored
    __threadfence_block();
}

// Persistent trace.  A wave takes a packet of 64 x chunk consecutive launch
// rays of one job and hands them out to its lanes; each round, every busy
// lane traces one segment (closest hit), runs the reception test of its
// job's receivers on it and reflects, and a lane whose ray has ended takes
// the packet's next ray.  Lanes thus stay busy while rays of different
// lengths (escaping at once or bouncing K times) share a wave.  The wave
// takes a new packet only when all its lanes are idle, so the job and its
// scene stay uniform across the wave.
template <bool COUNT, bool LDS, bool STREAM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
void k_trace(CallDev call, LdsPlan L, SceneDev s0,
                                               uint32_t* __restrict__ queue,
                                               sbr_candidate* __restrict__ cand, int64_t cap,
                                               unsigned long long* __restrict__ ccount,
                                               int32_t* __restrict__ out_tri,
                                               double* __restrict__ out_t,
                                               int32_t* __restrict__ err,
                                               unsigned long long* __restrict__ tallies)
{
    __shared__ StreamArgs s_stream;
    __shared__ uint32_t s_seen;  // the setup progress this workgroup has seen
    if (STREAM) {
        if (threadIdx.x == 0) {
            s_stream = StreamArgs{call.gscr, call.gprog, call.gepoch, call.gn, call.gcheck,
                                  call.gspin};
            s_seen = 0;
        }
        if (!LDS) __syncthreads();
    }
    if (LDS) stage_scene(s0, L);
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1ull;
    Tally tl{0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
    uint32_t segs = 0, events = 0;
    JobDev J{};
    SceneDev S = s0;
    RxBox box{};  // box of the current job's receivers
    int64_t next = 0, pend = 0;  // rays of the current packet not yet handed out
    RayState R;
    R.r = -1;
    for (;;) {
        const uint64_t idle = __ballot(R.r < 0);
        if (idle != 0 && next < pend) {
            const int64_t mine = next + __popcll(idle & below);
            if (R.r < 0 && mine < pend) start_ray(J, mine, R);
            next = min(pend, next + (int64_t)__popcll(idle));
        }
        if (__ballot(R.r >= 0) == 0) {
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
            J = call.jobs[lo];
            if (!LDS) S = call.scenes[J.scene];
            box = rx_box(call.rx32, J.rx_first, J.n_rx);
            next = J.ray_begin + ((int64_t)pk - J.packet_first) * 64 * call.chunk;
            pend = min(next + 64 * (int64_t)call.chunk, J.ray_begin + J.ray_count);
            if (STREAM) {
                // every lane is idle: its ray state is dead here, which frees its
                // registers for forming the directions
                R = RayState{};
                R.r = -1;
                StreamArgs sa = s_stream;
                stream_dirs(sa, &s_seen, J, next, pend, lane, err);
            }
            continue;
        }
        if (R.r < 0) continue;
        if (COUNT && first_active_lane()) tl.wave_segs += 1;
        // one segment: closest hit, excluding the face just reflected on
        const int K = J.K;
        HitRec h;
        const int32_t hit = traverse<false, COUNT, LDS>(S, L, R.o, R.d, R.prev, R.prev, S.t_eps,
                                                        INFINITY, J.delta, &h, err, &tl);
        if (COUNT) segs += 1;
        const double t = hit < 0 ? INFINITY : h.t;
        const int64_t ro = (R.r - J.ray_begin) * (K + 1);
        if (out_tri) out_tri[ro + R.j] = hit < 0 ? -1 : h.orig;
        if (out_t) out_t[ro + R.j] = t;
        // reception on the segment
        const Seg32 g32 = seg32(R, t, J.thl);
        if (J.rx_root < 0) {
            // FP32 pre-test of every receiver (wave-uniform, scalar loads),
            // the FP64 test for the few it lets through; skipped when no
            // busy lane's segment can reach the receivers' box
            const bool mine = rx_box_may(g32, box);
            if (__ballot(mine) != 0) {
                if (COUNT && first_active_lane()) tl.wave_rx += (uint32_t)J.n_rx;
                if (COUNT && mine) tl.rx_tests += (uint32_t)J.n_rx;
                for (int x = 0; x < J.n_rx; ++x) {
                    const int32_t gx = J.rx_first + x;
                    if (rx_may_capture32(g32, cld4(call.rx32 + gx)))
                        receive(J, call.rx, R, t, gx, cand, cap, ccount, &events, COUNT);
                }
            }
        } else if (rx_box_may(g32, box)) {
            // stackless preorder walk of the job's receiver tree (lanes whose
            // segment cannot reach the receivers' box skip it)
            int32_t nd = J.rx_root;
            const int32_t end = call.rx_nodes[nd].skip;
            const d3 inv = mk(1.0 / R.d.x, 1.0 / R.d.y, 1.0 / R.d.z);
            while (nd != end) {
                if (COUNT && first_active_lane()) tl.wave_rx += 1;
                if (COUNT) tl.rx_nodes += 1;
                const double2* q = (const double2*)(call.rx_nodes + nd);
                const double2 c01 = gld(q), c2h0 = gld(q + 1), h12 = gld(q + 2), m = gld(q + 3);
                RxNode N;
                N.first = (int32_t)(__double_as_longlong(m.x) & 0xffffffffll);
                N.count = (int32_t)(__double_as_longlong(m.x) >> 32);
                N.skip = (int32_t)(__double_as_longlong(m.y) & 0xffffffffll);
                if (!rx_box_may_capture(R.o, R.d, inv, R.D, t, mk(c01.x, c01.y, c2h0.x),
                                        mk(c2h0.y, h12.x, h12.y), J.thl)) {
                    nd = N.skip;
                } else if (N.count == 0) {
                    nd = nd + 1;
                } else {
                    for (int q = 0; q < N.count; ++q) {
                        if (COUNT && first_active_lane()) tl.wave_rx += 1;
                        if (COUNT) tl.rx_tests += 1;
                        const int32_t gx = gld(call.rx_perm + N.first + q);
                        if (rx_may_capture32(g32, gld(call.rx32 + gx)))
                            receive(J, call.rx, R, t, gx, cand, cap, ccount, &events, COUNT);
                    }
                    nd = N.skip;
                }
            }
        }
        if (hit < 0 || R.j == K) {
            if (out_tri || out_t)
                for (int q = R.j + 1; q <= K; ++q) {
                    if (out_tri) out_tri[ro + q] = -1;
                    if (out_t) out_t[ro + q] = INFINITY;
                }
            R.r = -1;
            continue;
        }
        // specular reflection on the face plane: o' = o + t d,
        // d' = d - (2 d.n) n (no renormalization), D' = D + t
        const int32_t f = h.face;
        const d3 nf = face_normal(S, f);
        const d3 on = add(R.o, scl(t, R.d));
        const double k2 = 2.0 * dot(R.d, nf);
        R.d = sub(R.d, scl(k2, nf));
        R.D = R.D + t;
        R.o = on;
        R.prev = f;
        set_face(R, R.j, f);
        R.j += 1;
    }
    if (COUNT) {
        atomicAdd(&tallies[0], (unsigned long long)segs);
        atomicAdd(&tallies[1], (unsigned long long)tl.nodes);
        atomicAdd(&tallies[2], (unsigned long long)tl.tris);
        atomicAdd(&tallies[3], (unsigned long long)events);
        atomicAdd(&tallies[4], (unsigned long long)tl.fp64_tris);
        atomicAdd(&tallies[5], (unsigned long long)tl.wave_nodes);
        atomicAdd(&tallies[6], (unsigned long long)tl.wave_tris);
        atomicAdd(&tallies[7], (unsigned long long)tl.wave_segs);
        atomicAdd(&tallies[8], (unsigned long long)tl.wave_rx);
        atomicAdd(&tallies[9], (unsigned long long)tl.rx_nodes);
        atomicAdd(&tallies[10], (unsigned long long)tl.rx_tests);
    }
}

template <bool COUNT, bool LDS, bool STREAM>
static void launch_trace_t(const CallDev& call, const LdsPlan& L, const SceneDev& s0, int blocks,
                           uint32_t* queue, sbr_candidate* cand, int64_t cap,
                           unsigned long long* cand_count, int32_t* out_tri, double* out_t,
                           int32_t* err_flag, hipStream_t s, unsigned long long* tallies)
{
    hipLaunchKernelGGL((k_trace<COUNT, LDS, STREAM>), dim3((unsigned)blocks), dim3(L.block),
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
    // a streamed grid is never combined with the counting instance (the
    // library makes counting calls with their directions in place)
    if (call.gscr && tallies) return hipErrorInvalidValue;
    if (call.gscr && lds)
        launch_trace_t<false, true, true>(call, L, s0, blocks, queue, cand, cap, cand_count,
                                          out_tri, out_t, err_flag, s, tallies);
    else if (call.gscr)
        launch_trace_t<false, false, true>(call, L, s0, blocks, queue, cand, cap, cand_count,
                                           out_tri, out_t, err_flag, s, tallies);
    else if (tallies && lds)
        launch_trace_t<true, true, false>(call, L, s0, blocks, queue, cand, cap, cand_count,
                                          out_tri, out_t, err_flag, s, tallies);
    else if (tallies)
        launch_trace_t<true, false, false>(call, L, s0, blocks, queue, cand, cap, cand_count,
                                           out_tri, out_t, err_flag, s, tallies);
    else if (lds)
        launch_trace_t<false, true, false>(call, L, s0, blocks, queue, cand, cap, cand_count,
                                           out_tri, out_t, err_flag, s, tallies);
    else
        launch_trace_t<false, false, false>(call, L, s0, blocks, queue, cand, cap, cand_count,
                                            out_tri, out_t, err_flag, s, tallies);
    return hipGetLastError();
}

hipError_t trace_set_lds_limit(int bytes)
{
    hipError_t e = hipFuncSetAttribute((const void*)k_trace<true, true, false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)k_trace<false, true, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_trace<false, true, false>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

}  // namespace sbr
