// api.hip -- C ABI (include/sbr.h): contexts, scenes, BVH upload and the
// orchestration of the trace stages on one HIP stream.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "diffract.h"
#include "geom.h"
#include "grid_layout.h"
#include "internal.h"
#include "refine_queue.h"

using namespace sbr;

namespace {

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    template <class T>
    T* as() const { return (T*)p; }
};

// Bumped whenever a device buffer is (re)allocated or released: a captured
// graph is only replayed while the buffers it was captured with still exist.
// Atomic because contexts may run on different threads; a bump by another
// context only costs this one a recapture.
std::atomic<uint64_t> g_alloc_epoch{1};

hipError_t ensure(DevBuf& b, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    if (b.cap >= bytes) return hipSuccess;
    ++g_alloc_epoch;
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e == hipSuccess) b.cap = bytes;
    return e;
}

void release(DevBuf& b)
{
    ++g_alloc_epoch;
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

// Device-side counters read back between stages.
struct Counters {
    unsigned long long cand;
    int32_t err;
    int32_t n_unique;
    int32_t n_paths;
    uint32_t queue;  // packets handed out by the persistent trace kernel
};

}  // namespace

// BVH defaults when sbr_bvh_build gets no parameters.
constexpr int kDefaultSahBins = 64;
constexpr int kDefaultSplitPct = 0;

// Device memory of sbr_trace_device_noalloc: everything that entry point needs
// beyond its inputs and outputs lives in this array (one copy per device,
// held until the process ends).  Host code never passes `scratch` itself to a
// kernel or copy: the device address comes from hipGetSymbolAddress, taken
// once per device (noalloc_scratch_ptr).
constexpr size_t kNoAllocBytes = size_t(24) << 20;
constexpr int32_t kNoAllocMaxRx = 4096;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

// The device address of `scratch` on `device` (which must be current), looked
// up on the first call for that device and kept.
hipError_t noalloc_scratch_ptr(int device, void** out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_done[device]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
        g_scratch_err[device] = e;
        g_scratch_ptr[device] = e == hipSuccess ? ptr : nullptr;
        g_scratch_done[device] = true;
        if (e != hipSuccess) (void)hipGetLastError();
    }
    *out = g_scratch_ptr[device];
    return g_scratch_err[device];
}

// Which launch grid (launch * 100000 + n, -1: none) the scratch of each device
// holds at the grid offset for that n, as left by the last completed call.
int32_t g_scratch_grid[kMaxDevices] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1,
                                       -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1,
                                       -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1,
                                       -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1,
                                       -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1};

}  // namespace

struct sbr_context {
    int32_t device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int32_t n_scenes = 0;
    std::map<int32_t, DevBuf> grids;  // division n -> [3][N] FP64 directions
    // whole-grid jobs hand their rays out by direction cell (get_order), the
    // order cached per grid
    std::map<int32_t, DevBuf> orders;
    int32_t ray_order = 1;
    void* scratch = nullptr;  // device address of the no-allocation scratch (NULL: unavailable)
    hipError_t scratch_err = hipSuccess;
    int64_t noalloc_unique = -1;  // path count of the last no-allocation call
    DevBuf grid_scratch, rx, rx32, cand, idx, flags, offs, scan, uniq, refine, paths, keep, outp,
        counters, rays_tri, rays_t, tally, geom, d_jobs, d_scenes, d_rxjob, d_rxnodes, d_rxperm,
        d_rxp, dpaths, dout, q_state, q_slot, q_items, q_ctr, geom0;
    Counters* host_ctr = nullptr;  // pinned
    sbr_path* host_paths = nullptr;  // pinned staging of the path list
    int64_t host_paths_cap = 0;
    hipEvent_t ev[8] = {};
    // streamed launch grids: a fresh equiangular grid whose ray orders exist
    // can have its ring setup run on grid_stream (default priority) beside
    // the trace, which forms the directions itself; gprog holds the setup's
    // published progress, grid_epoch numbers the setups
    // the ray order of a streamed grid (stream_order; SBR_GRID_ORDER,
    // SBR_GRID_PREFIX; 0: the cell order, no separate order)
    int32_t grid_order = 2, grid_prefix = 35;
    std::map<int32_t, DevBuf> orders_stream;
    // the launch-grid and trace times (ms) of the last fresh call of each
    // grid that formed its grid first and made no order: with
    // grid_stream_mode 1 a grid is streamed when its trace took at least
    // three times as long as the grid (the setup then finishes well inside
    // the trace, and the directions the trace forms cost less than the grid
    // saved); 2 streams whenever possible, 0 never (SBR_GRID_STREAM)
    std::map<int32_t, std::pair<float, float>> grid_times;
    int32_t grid_stream_mode = 1;
    hipStream_t grid_stream = nullptr;
    hipEvent_t ev_grid_fork = nullptr, ev_grid_join = nullptr;
    DevBuf gprog;
    uint32_t grid_epoch = 0;
    // failure injection for tests (SBR_GRID_STREAM_MISS=1): the trace and the
    // start wait expect an epoch the setup never writes and give up after a
    // few polls, so the call takes the fallback path
    bool grid_stream_miss = false;
    // second stream (default priority) for the exact solve beside the
    // refinement, and the events that fork to it and join back
    hipStream_t stream2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // LDS staging of the traversal kernels: budget per block (0 = traverse
    // from global memory with a private stack), lanes per block of the trace
    // kernel, LDS stack entries per lane.  Defaults can be overridden with
    // SBR_LDS_BUDGET, SBR_TRACE_BLOCK, SBR_STACK_DEPTH.
    int32_t lds_max = 65536, lds_budget = 65536, trace_block = 256, stack_depth = 24;
    // path counts up to which the refinement uses the two-iteration lookahead
    // (64 lanes per path); SBR_LOOKAHEAD_PATHS overrides
    int64_t lookahead_max_paths = 4096;
    // persistent trace: 64-ray groups per queue packet, resident workgroups
    // (SBR_TRACE_CHUNK, SBR_TRACE_BLOCKS)
    int32_t trace_chunk = 1, persist_blocks = 2048;
    int32_t rx_tree_min = 64;
    int32_t lookahead_depth = 3;
    int32_t lookahead3_max_paths = 256;
    int32_t refine_segments = 1;
    // segment-parallel refinement of many paths: iterations on one wave per
    // path before the paths still running move to 512-lane workgroups
    // (SBR_SEG_TAIL; 0: never)
    int32_t seg_tail = 10;
    // The receiver tree of the last single-job call, kept for the next call
    // over the same receivers (compared bytewise); rxt_on_device: d_rxnodes
    // and d_rxperm hold it.
    std::vector<double> rxt_rx;
    std::vector<RxNode> rxt_nodes;
    std::vector<int32_t> rxt_perm;
    bool rxt_on_device = false;
    int32_t grid_check_log2 = 0;
    bool la3_lds = true;  // stage the scene in LDS for the three-level refinement
    // event and path counts of the last device-memory call, which predict
    // the next one's (-1: no prediction)
    int64_t spec_events = -1, spec_unique = 0;
    // bytes of the job, scene and receiver-job tables last copied to the
    // device, valid while no buffer was (re)allocated since and no graph
    // wrote those buffers
    std::vector<char> up_last;
    uint64_t up_epoch = 0;
    // one captured graph of a sbr_trace_device call (SBR_FLAG_GRAPH)
    struct Graph {
        bool valid = false;
        uint64_t epoch = 0, scene_id = 0;
        const double* rx = nullptr;
        int32_t n_rx = 0;
        sbr_path* out = nullptr;
        int64_t capacity = 0, u_cap = 0, n_rays = 0;
        sbr_trace_params params{};
        sbr_tuning tuning{};
        hipGraphExec_t exec = nullptr;
        hipStream_t cap_stream = nullptr;
        JobDev* h_job = nullptr;      // pinned staging read by the graph
        SceneDev* h_scene = nullptr;  // pinned
        int32_t* h_rxjob = nullptr;   // pinned [n_rx]
        int32_t h_rxjob_cap = 0;
    } graph;
    // one captured graph of a sbr_trace_batch call (every job SBR_FLAG_GRAPH)
    struct BatchGraph {
        bool valid = false;
        uint64_t epoch = 0;
        std::vector<uint64_t> scene_ids;
        std::vector<sbr_job> jobs;  // the key (tx not compared)
        int32_t n_rx = 0;
        int64_t u_cap = 0, n_rays = 0;
        sbr_tuning tuning{};
        hipGraphExec_t exec = nullptr;
        hipStream_t cap_stream = nullptr;
        // pinned staging read by the graph
        JobDev* h_jobs = nullptr;
        SceneDev* h_scenes = nullptr;
        int32_t* h_rxjob = nullptr;
        double* h_rx = nullptr;
        int64_t jobs_cap = 0, scenes_cap = 0, rxjob_cap = 0, rx_cap = 0;
    } bgraph;
};

struct sbr_scene {
    sbr_context* ctx = nullptr;
    uint64_t id = 0;  // unique per upload (keys captured graphs)
    int64_t T = 0;
    int64_t R = 0;  // triangle records in leaf order (references; >= T)
    int32_t F = 0, M = 0;
    std::vector<double> tri_v;  // [T][9]
    std::vector<int32_t> face, mat;
    std::vector<double> eps;     // [M][2]
    std::vector<double> fplane;  // [F][4]
    std::vector<int32_t> fmat;   // [F]
    double t_eps = 0.0, R_s = 0.0;
    bool has_bvh = false;
    int32_t bvh_depth = 0;
    int64_t n_nodes = 0;
    DevBuf nodes, tris, d_fplane, d_fmat, fstart, ftris, d_eps;
    // wedges for order-1 diffraction, made on first use
    bool has_wedges = false;
    std::vector<WedgeDev> wedges;
    std::vector<double> wedge_b;  // [n][3] second endpoints
    DevBuf d_wedges;
};

namespace {

void drop_graph(sbr_context* c)
{
    if (c->graph.exec) (void)hipGraphExecDestroy(c->graph.exec);
    c->graph.exec = nullptr;
    c->graph.valid = false;
}

void drop_bgraph(sbr_context* c)
{
    if (c->bgraph.exec) (void)hipGraphExecDestroy(c->bgraph.exec);
    c->bgraph.exec = nullptr;
    c->bgraph.valid = false;
}

sbr_status fail(sbr_context* c, sbr_status st, const char* fmt, ...)
    __attribute__((format(printf, 3, 4)));
sbr_status fail(sbr_context* c, sbr_status st, const char* fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return st;
}

thread_local std::string g_create_err;

#define HIPCHK(ctx, expr)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((ctx), e_ == hipErrorOutOfMemory ? SBR_E_OOM : SBR_E_DEVICE,        \
                        "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
    } while (0)

bool finite3(const double* p) { return isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]); }

sbr_status get_grid(sbr_context* c, int32_t launch, int32_t n, GridDev* g, bool* built,
                    bool fresh = false)
{
    const int64_t N = num_rays(launch, n);
    const int32_t key = launch * 100000 + n;
    auto it = c->grids.find(key);
    *built = false;
    if (it != c->grids.end() && fresh) {
        HIPCHK(c, ensure(c->grid_scratch, grid_scratch_bytes(n)));
        GridDev gd{it->second.as<double>(), N, n, launch};
        HIPCHK(c, launch_grid(gd, c->stream, c->grid_scratch.p, c->grid_check_log2));
        *built = true;
    }
    if (it == c->grids.end()) {
        DevBuf b;
        HIPCHK(c, ensure(b, sizeof(double) * 3 * (size_t)N));
        HIPCHK(c, ensure(c->grid_scratch, grid_scratch_bytes(n)));
        GridDev gd{b.as<double>(), N, n, launch};
        hipError_t e = launch_grid(gd, c->stream, c->grid_scratch.p, c->grid_check_log2);
        if (e != hipSuccess) {
            release(b);
            return fail(c, SBR_E_DEVICE, "launch grid: %s", hipGetErrorString(e));
        }
        it = c->grids.emplace(key, b).first;
        *built = true;
    }
    *g = GridDev{it->second.as<double>(), N, n, launch};
    return SBR_OK;
}

// Grids up to this many rays (n = 3663 on the icosahedron) get a hand-out
// order; larger ones, whose order would take seconds and gigabytes of host
// memory to make, are traced by index.
constexpr int64_t kOrderMaxRays = int64_t(1) << 27;

// The order of a streamed grid's rays (see sbr_context::grid_order): groups
// of 64 consecutive rays of the cell order, the groups first whose rays need
// the least of the grid setup's progress (grid_need), by the power-of-two
// bucket of that need, then the others in cell order.  Bucket b holds about
// 2^b layers' rays, whose tracing takes far longer than the setup needs for
// the layers of bucket b + 1, so the packets taken while the setup runs find
// their layers published; the buckets first hold grid_prefix percent of the
// rays, which the trace takes longer to work through than the setup needs to
// finish (mode 2), or every bucket is (mode 1).  The packets keep their
// rays, so each still traces nearby directions.
std::vector<uint32_t> stream_order(const sbr_context* c, int32_t n, const std::vector<uint32_t>& ord)
{
    const int64_t N = (int64_t)ord.size();
    const int64_t G = (N + 63) / 64;
    std::vector<uint32_t> gb((size_t)G, 0);
    for (int64_t i = 0; i < N; ++i) {
        uint32_t& x = gb[(size_t)(i / 64)];
        x = std::max(x, grid_need(n, ord[(size_t)i]));
    }
    uint32_t top = 0;
    for (auto& x : gb) {
        uint32_t b = 0;
        while ((2u << b) <= x) ++b;  // floor(log2(need)), need >= 1
        x = b;
        top = std::max(top, b);
    }
    uint32_t cut = top;
    if (c->grid_order == 2) {
        std::vector<int64_t> rays((size_t)top + 1, 0);
        for (int64_t g = 0; g < G; ++g) rays[gb[(size_t)g]] += std::min<int64_t>(64, N - 64 * g);
        int64_t acc = 0;
        for (cut = 0; cut < top; ++cut) {
            acc += rays[cut];
            if (100 * acc >= (int64_t)c->grid_prefix * N) break;
        }
    }
    auto key = [&](int64_t g) { return gb[(size_t)g] <= cut ? gb[(size_t)g] : cut + 1; };
    std::vector<int64_t> start((size_t)top + 3, 0);
    for (int64_t g = 0; g < G; ++g) ++start[key(g) + 1];
    for (size_t k = 1; k < start.size(); ++k) start[k] += start[k - 1];
    std::vector<int64_t> gorder((size_t)G);
    for (int64_t g = 0; g < G; ++g) gorder[(size_t)start[key(g)]++] = g;
    std::vector<uint32_t> out((size_t)N);
    int64_t o = 0;
    for (int64_t g : gorder)
        for (int64_t i = 64 * g; i < std::min<int64_t>(N, 64 * g + 64); ++i)
            out[(size_t)o++] = ord[(size_t)i];
    return out;
}

// A hand-out order of a grid's rays that keeps each wave's rays close in
// direction: rays sorted by their cube-map cell (about one ray per cell, cells
// in Z order per cube face; launch_ray_cells), by index within a cell
// (stable two-pass radix sort of the 32-bit cells on the host).  Made once per
// grid, with the order of a streamed grid beside it (equiangular grids,
// stream_order); it changes the order rays are traced in, not the results.
// *built: this call made them.
sbr_status get_order(sbr_context* c, int32_t launch, int32_t n, const GridDev& g,
                     const uint32_t** out, bool streamed, bool* built)
{
    const int32_t key = launch * 100000 + n;
    *built = false;
    auto it = c->orders.find(key);
    if (it == c->orders.end()) {
        *built = true;
        const int64_t N = g.N;
        int32_t R = 1;
        while (R < 8192 && (int64_t)R * R * 6 < N) R *= 2;
        DevBuf b, bs;
        HIPCHK(c, ensure(b, sizeof(uint32_t) * (size_t)N));
        std::vector<uint32_t> cell((size_t)N), ord((size_t)N), tmp((size_t)N);
        hipError_t e = launch_ray_cells(g.dir, N, R, b.as<uint32_t>(), c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(cell.data(), b.p, sizeof(uint32_t) * (size_t)N,
                               hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            release(b);
            return fail(c, SBR_E_DEVICE, "ray order: %s", hipGetErrorString(e));
        }
        for (int64_t i = 0; i < N; ++i) ord[(size_t)i] = (uint32_t)i;
        std::vector<int64_t> cnt(1 << 16);
        for (int pass = 0; pass < 2; ++pass) {
            const int sh = 16 * pass;
            std::fill(cnt.begin(), cnt.end(), 0);
            for (int64_t i = 0; i < N; ++i) ++cnt[(cell[ord[(size_t)i]] >> sh) & 0xffff];
            int64_t run = 0;
            for (auto& x : cnt) {
                const int64_t k = x;
                x = run;
                run += k;
            }
            for (int64_t i = 0; i < N; ++i) {
                const uint32_t r = ord[(size_t)i];
                tmp[(size_t)cnt[(cell[r] >> sh) & 0xffff]++] = r;
            }
            ord.swap(tmp);
        }
        e = hipMemcpyAsync(b.p, ord.data(), sizeof(uint32_t) * (size_t)N, hipMemcpyHostToDevice,
                           c->stream);
        std::vector<uint32_t> so;
        if (e == hipSuccess && launch == SBR_LAUNCH_EQUIANGULAR && c->grid_order > 0) {
            so = stream_order(c, n, ord);
            e = ensure(bs, sizeof(uint32_t) * (size_t)N);
            if (e == hipSuccess)
                e = hipMemcpyAsync(bs.p, so.data(), sizeof(uint32_t) * (size_t)N,
                                   hipMemcpyHostToDevice, c->stream);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            release(b);
            release(bs);
            return fail(c, SBR_E_DEVICE, "ray order: %s", hipGetErrorString(e));
        }
        it = c->orders.emplace(key, b).first;
        if (bs.p) c->orders_stream.emplace(key, bs);
    }
    if (streamed) {
        auto is = c->orders_stream.find(key);
        *out = is != c->orders_stream.end() ? is->second.as<const uint32_t>()
                                            : it->second.as<const uint32_t>();
    } else {
        *out = it->second.as<const uint32_t>();
    }
    return SBR_OK;
}

SceneDev scene_dev(const sbr_scene* s)
{
    SceneDev S;
    S.nodes = s->nodes.as<const Bvh4Node>();
    S.tris = s->tris.as<const TriD>();
    S.fplane = s->d_fplane.as<const double>();
    S.fmat = s->d_fmat.as<const int32_t>();
    S.fstart = s->fstart.as<const int32_t>();
    S.ftris = s->ftris.as<const int32_t>();
    S.eps = s->d_eps.as<const double>();
    S.n_tri = (int32_t)s->R;
    S.n_face = s->F;
    S.n_node = (int32_t)s->n_nodes;
    S.t_eps = s->t_eps;
    return S;
}

// Box widening that makes FP32 traversal conservative for rays starting at
// tx or inside the scene: 2^-20 max(|tx|_inf, scene max |coordinate|).
float traversal_delta(const sbr_scene* s, const double* tx)
{
    double R = s->R_s;
    for (int i = 0; i < 3; ++i) R = std::max(R, fabs(tx[i]));
    double d = ldexp(R, -20);
    float f = (float)d;
    if ((double)f < d) f = nextafterf(f, INFINITY);
    return std::max(f, 1e-30f);
}

int env_int(const char* name, int dflt, int lo, int hi)
{
    const char* v = getenv(name);
    if (!v || !*v) return dflt;
    long x = strtol(v, nullptr, 10);
    return (int)std::min<long>(hi, std::max<long>(lo, x));
}

// Plan of the three-level refinement (512 lanes, a 16-entry LDS stack per
// lane): the whole scene in LDS when it fits next to the stacks and the
// kernel's static LDS, else none (global memory).
LdsPlan plan_la3(const sbr_scene* s)
{
    const sbr_context* c = s->ctx;
    // 2 KB left for the kernels' static LDS
    LdsPlan L = make_lds_plan(s->n_nodes, s->R, 512, 16, c->lds_max - 2048);
    if (!c->la3_lds || L.n_tris != s->R || L.depth != 16) {
        L = LdsPlan{};
        L.block = 512;
    }
    return L;
}

LdsPlan plan_for(const sbr_scene* s, int block)
{
    const sbr_context* c = s->ctx;
    if (c->lds_budget <= 0) {  // global-memory traversal, private stack
        LdsPlan L{};
        L.block = 256;
        return L;
    }
    return make_lds_plan(s->n_nodes, s->R, block, c->stack_depth, c->lds_budget);
}

// theta_launch = theta_0 / (sqrt(3) n), eq. (4); the equidistant grids use
// their polyhedron's edge angle (pi / 2 for the octahedron).
double theta_launch(int32_t launch, int32_t n)
{
    const double th = launch == SBR_LAUNCH_EQUIDISTANT_OCTA ? kPi / 2.0 : kTheta0;
    return th / (sqrt(3.0) * (double)n);
}

// Make `device` current, calling hipSetDevice only when another device is.
hipError_t use_device(int device)
{
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur == device) return hipSuccess;
    return hipSetDevice(device);
}

sbr_status check_params(sbr_context* c, const sbr_trace_params* p)
{
    if (!p) return fail(c, SBR_E_INVALID_ARG, "params is NULL");
    if (p->max_order < 0 || p->max_order > SBR_MAX_ORDER)
        return fail(c, SBR_E_INVALID_ARG, "max_order %d outside 0..%d", p->max_order, SBR_MAX_ORDER);
    if (p->division_n < 1 || p->division_n > 10000)
        return fail(c, SBR_E_INVALID_ARG, "division_n %d outside 1..10000", p->division_n);
    if (p->iterations < 0 || p->iterations > 200)
        return fail(c, SBR_E_INVALID_ARG, "iterations %d outside 0..200", p->iterations);
    if (p->subrays != 6 && p->subrays != 7)
        return fail(c, SBR_E_INVALID_ARG, "subrays must be 6 or 7 (got %d)", p->subrays);
    if (!(p->freq_hz > 0.0) || !isfinite(p->freq_hz))
        return fail(c, SBR_E_INVALID_ARG, "freq_hz must be finite and > 0");
    if (!isfinite(p->tx_power_dbm) || !isfinite(p->target_err_deg) || p->target_err_deg >= 45.0)
        return fail(c, SBR_E_INVALID_ARG, "tx_power_dbm / target_err_deg out of range");
    if (p->flags & ~(SBR_FLAG_KEEP_INVALID | SBR_FLAG_FRESH_GRID | SBR_FLAG_GRAPH))
        return fail(c, SBR_E_INVALID_ARG, "unknown flags");
    if (p->launch < SBR_LAUNCH_EQUIANGULAR || p->launch > SBR_LAUNCH_EQUIDISTANT_OCTA)
        return fail(c, SBR_E_INVALID_ARG, "unknown launch method %d", p->launch);
    return SBR_OK;
}

sbr_status check_scene(sbr_scene* s)
{
    if (!s || !s->ctx) return SBR_E_NO_SCENE;
    if (!s->has_bvh) return fail(s->ctx, SBR_E_NO_BVH, "sbr_bvh_build has not been called");
    return SBR_OK;
}

// One call of the trace pipeline: jobs over scenes, the receivers of all
// jobs, and what the front half (launch, trace, path test 1) produced.
struct Call {
    std::vector<JobDev> jobs;
    std::vector<const sbr_scene*> scenes;
    std::vector<int32_t> rx_job;
    std::vector<RxNode> rx_nodes;  // receiver trees of the jobs that have one
    std::vector<int32_t> rx_perm;  // receiver indices in tree-leaf order
    bool rx_tree_cached = false;   // rx_nodes / rx_perm are the context's kept tree
    const double* rx = nullptr;      // host [n_rx][3] (NULL with only device receivers)
    const double* rx_dev = nullptr;  // device [n_rx][3] when the caller passed device memory
    int32_t n_rx = 0;
    int64_t n_rays = 0, n_packets = 0;
    int32_t chunk = 1;
    CallDev dev{};
    LdsPlan lp{};
    SceneDev s0{};
    int64_t n_cand = 0, n_uniq = 0;
    bool small = false;  // path test 1 ran in one workgroup; n_uniq is on the device
    bool grids_built = false;
    // the job's launch grid is streamed (see sbr_context::grid_stream_mode):
    // its ring setup is launched beside the trace of the first pass
    bool stream_grid = false;
    int32_t stream_n = 0;
    bool order_built = false;  // a ray order was made for this call
    bool streamed = false;     // the trace formed the directions (stream_grid was set)
    // speculative call: the event count was not read back after the trace;
    // n_cand holds the bound the one-workgroup stages were launched for, and
    // u_pred the path count that picks the refinement kernel
    bool spec = false;
    int64_t u_pred = 0;
    int64_t cap = 0;
    float ms_launch = 0, ms_trace = 0;
};

// Returned by run_paths when a speculative call found more events than its
// bound: the caller runs the call again without speculation.
constexpr sbr_status kSpecMiss = (sbr_status)1000;

// Returned when a streamed launch grid's setup did not publish in time (for
// instance when a tool serializes the streams' kernels, so that the setup
// cannot run beside the trace): streaming is then switched off for the
// context and the caller runs the call again, its grid formed before its
// trace.
constexpr sbr_status kGridStreamMiss = (sbr_status)1001;

sbr_status grid_stream_missed(sbr_context* c)
{
    c->grid_stream_mode = 0;
    return kGridStreamMiss;
}

// Box tree over the receivers perm[lo, hi) (global indices into rx), built
// in preorder by median splits on the widest axis; returns the node index.
// Each node's box c +- h holds its receivers (h widened by 1e-12 relative
// and 1e-300 over the largest offset from c).
int32_t build_rx_tree(const double* rx, std::vector<int32_t>& perm, int32_t lo, int32_t hi,
                      std::vector<RxNode>& nodes)
{
    const int32_t me = (int32_t)nodes.size();
    nodes.push_back(RxNode{});
    double bl[3] = {INFINITY, INFINITY, INFINITY}, bh[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int32_t i = lo; i < hi; ++i)
        for (int a = 0; a < 3; ++a) {
            bl[a] = std::min(bl[a], rx[3 * perm[i] + a]);
            bh[a] = std::max(bh[a], rx[3 * perm[i] + a]);
        }
    RxNode nd{};
    for (int a = 0; a < 3; ++a) {
        nd.c[a] = 0.5 * (bl[a] + bh[a]);
        double e = 0.0;
        for (int32_t i = lo; i < hi; ++i) e = std::max(e, fabs(rx[3 * perm[i] + a] - nd.c[a]));
        nd.h[a] = e * (1.0 + 1e-12) + 1e-300;
    }
    if (hi - lo <= kRxLeaf) {
        nd.first = lo;
        nd.count = hi - lo;
    } else {
        int ax = 0;
        for (int a = 1; a < 3; ++a)
            if (bh[a] - bl[a] > bh[ax] - bl[ax]) ax = a;
        const int32_t mid = lo + (hi - lo) / 2;
        std::nth_element(perm.begin() + lo, perm.begin() + mid, perm.begin() + hi,
                         [&](int32_t a, int32_t b) {
                             double xa = rx[3 * a + ax], xb = rx[3 * b + ax];
                             return xa < xb || (xa == xb && a < b);
                         });
        (void)build_rx_tree(rx, perm, lo, mid, nodes);
        (void)build_rx_tree(rx, perm, mid, hi, nodes);
        nd.first = -1;
        nd.count = 0;
    }
    nd.skip = (int32_t)nodes.size();
    nodes[me] = nd;
    return me;
}

// The job of transmitter tx with parameters p over launch directions dir
// [3][N], rays [ray_begin, ray_begin + ray_count) handed out by index, as the
// only job of a call (first packet 0, scene 0, its receivers the call's
// first n_rx, no receiver tree).
JobDev make_job(const sbr_scene* s, const double* tx, const sbr_trace_params* p,
                const double* dir, int64_t N, int64_t ray_begin, int64_t ray_count)
{
    JobDev J{};
    for (int i = 0; i < 3; ++i) J.tx[i] = tx[i];
    J.thl = theta_launch(p->launch, p->division_n);
    J.tan_tgt = p->target_err_deg > 0.0 ? tan_cr((p->target_err_deg * kPi) / 180.0) : 0.0;
    J.freq_hz = p->freq_hz;
    J.tx_power_dbm = p->tx_power_dbm;
    J.dir = dir;
    J.N = N;
    J.order = nullptr;
    J.ray_begin = ray_begin;
    J.ray_count = ray_count;
    J.packet_first = 0;
    J.scene = 0;
    J.rx_first = 0;
    J.n_rx = 0;
    J.K = p->max_order;
    J.iterations = p->iterations;
    J.subrays = p->subrays;
    J.keep_invalid = (p->flags & SBR_FLAG_KEEP_INVALID) ? 1 : 0;
    J.delta = traversal_delta(s, tx);
    J.rx_root = -1;
    return J;
}

// Add a job: its launch directions (cached per division n), parameters and
// packets of 64 x chunk rays.
sbr_status add_job(sbr_context* c, Call& call, int32_t scene_idx, const double* tx,
                   int32_t rx_first, int32_t n_rx, const sbr_trace_params* p, int64_t ray_begin,
                   int64_t ray_count)
{
    GridDev g;
    bool built = false;
    const int32_t key = p->launch * 100000 + p->division_n;
    const int64_t N = num_rays(p->launch, p->division_n);
    // a fresh grid of a single whole-grid job whose grid and ray order exist
    // is streamed: nothing is launched for it here
    bool stream = (p->flags & SBR_FLAG_FRESH_GRID) != 0 && c->grid_stream_mode > 0 &&
                  c->ray_order && p->launch == SBR_LAUNCH_EQUIANGULAR && call.jobs.empty() &&
                  ray_begin == 0 && ray_count == N && N <= kOrderMaxRays &&
                  c->grids.count(key) && c->orders_stream.count(key);
    if (stream && c->grid_stream_mode == 1) {
        auto t = c->grid_times.find(key);
        stream = t != c->grid_times.end() && t->second.second >= 3.0f * t->second.first;
    }
    sbr_status r = get_grid(c, p->launch, p->division_n, &g, &built,
                            (p->flags & SBR_FLAG_FRESH_GRID) != 0 && !stream);
    if (r) return r;
    call.grids_built = call.grids_built || built;
    if (stream) {
        HIPCHK(c, ensure(c->grid_scratch, grid_scratch_bytes(p->division_n)));
        call.stream_grid = true;
        call.stream_n = p->division_n;
    }
    const sbr_scene* s = call.scenes[scene_idx];
    JobDev J = make_job(s, tx, p, g.dir, g.N, ray_begin, ray_count);
    if (c->ray_order && ray_begin == 0 && ray_count == g.N && g.N <= kOrderMaxRays) {
        bool made = false;
        r = get_order(c, p->launch, p->division_n, g, &J.order, stream, &made);
        if (r) return r;
        call.order_built = call.order_built || made;
    }
    J.packet_first = call.n_packets;
    J.scene = scene_idx;
    J.rx_first = rx_first;
    J.n_rx = n_rx;
    if (n_rx > 0 && n_rx >= c->rx_tree_min) {
        // a call whose only receivers are this job's may reuse (or keep) the
        // tree: it depends on the receivers alone
        const bool single = rx_first == 0 && n_rx == call.n_rx && call.rx_nodes.empty();
        const size_t nb = sizeof(double) * 3 * (size_t)n_rx;
        if (single && c->rxt_rx.size() == 3 * (size_t)n_rx &&
            memcmp(c->rxt_rx.data(), call.rx, nb) == 0) {
            call.rx_perm = c->rxt_perm;
            call.rx_nodes = c->rxt_nodes;
            call.rx_tree_cached = true;
            J.rx_root = 0;
        } else {
            if (call.rx_perm.size() != (size_t)call.n_rx) {
                call.rx_perm.resize((size_t)call.n_rx);
                for (int32_t x = 0; x < call.n_rx; ++x) call.rx_perm[x] = x;
            }
            J.rx_root =
                build_rx_tree(call.rx, call.rx_perm, rx_first, rx_first + n_rx, call.rx_nodes);
            if (single) {
                c->rxt_rx.assign(call.rx, call.rx + 3 * (size_t)n_rx);
                c->rxt_nodes = call.rx_nodes;
                c->rxt_perm = call.rx_perm;
                c->rxt_on_device = false;
                call.rx_tree_cached = true;
            }
        }
    }
    const int64_t per = 64 * (int64_t)call.chunk;
    call.n_packets += (ray_count + per - 1) / per;
    call.n_rays += ray_count;
    for (int32_t x = 0; x < n_rx; ++x) call.rx_job[rx_first + x] = (int32_t)call.jobs.size();
    call.jobs.push_back(J);
    return SBR_OK;
}

// Copy the job, scene and receiver tables to the device (skipped when they
// equal the last copy), point the kernels at the receivers (device-memory
// receivers are read in place), and in one launch form the FP32 receivers
// and zero the call's counters.
sbr_status upload_call(sbr_context* c, Call& call)
{
    hipStream_t st = c->stream;
    std::vector<SceneDev> sd;
    for (const sbr_scene* s : call.scenes) sd.push_back(scene_dev(s));
    HIPCHK(c, ensure(c->d_jobs, sizeof(JobDev) * std::max<size_t>(call.jobs.size(), 1)));
    HIPCHK(c, ensure(c->d_scenes, sizeof(SceneDev) * std::max<size_t>(sd.size(), 1)));
    HIPCHK(c, ensure(c->rx32, sizeof(float4) * (size_t)std::max(call.n_rx, 1)));
    HIPCHK(c, ensure(c->d_rxjob, sizeof(int32_t) * (size_t)std::max(call.n_rx, 1)));
    HIPCHK(c, ensure(c->counters, sizeof(Counters)));
    if (!call.rx_dev) HIPCHK(c, ensure(c->rx, sizeof(double) * 3 * (size_t)std::max(call.n_rx, 1)));
    const size_t bj = sizeof(JobDev) * call.jobs.size(), bs = sizeof(SceneDev) * sd.size(),
                 br = sizeof(int32_t) * call.rx_job.size();
    std::vector<char> now(bj + bs + br);
    if (bj) memcpy(now.data(), call.jobs.data(), bj);
    if (bs) memcpy(now.data() + bj, sd.data(), bs);
    if (br) memcpy(now.data() + bj + bs, call.rx_job.data(), br);
    if (c->up_epoch != g_alloc_epoch || now != c->up_last) {
        if (bj)
            HIPCHK(c, hipMemcpyAsync(c->d_jobs.p, call.jobs.data(), bj, hipMemcpyHostToDevice, st));
        if (bs)
            HIPCHK(c, hipMemcpyAsync(c->d_scenes.p, sd.data(), bs, hipMemcpyHostToDevice, st));
        if (br)
            HIPCHK(c, hipMemcpyAsync(c->d_rxjob.p, call.rx_job.data(), br, hipMemcpyHostToDevice, st));
        c->up_last.swap(now);
        c->up_epoch = g_alloc_epoch;
    }
    const double* rx_src = call.rx_dev;
    if (!rx_src) {
        if (call.n_rx > 0)
            HIPCHK(c, hipMemcpyAsync(c->rx.p, call.rx, sizeof(double) * 3 * (size_t)call.n_rx,
                                     hipMemcpyHostToDevice, st));
        rx_src = c->rx.as<const double>();
    }
    HIPCHK(c, launch_rx32(rx_src, call.n_rx, c->rx32.as<float4>(), st, c->counters.p,
                          sizeof(Counters)));
    call.dev.jobs = c->d_jobs.as<const JobDev>();
    call.dev.scenes = c->d_scenes.as<const SceneDev>();
    call.dev.rx = rx_src;
    call.dev.rx32 = c->rx32.as<const float4>();
    call.dev.rx_job = c->d_rxjob.as<const int32_t>();
    call.dev.rx_nodes = nullptr;
    call.dev.rx_perm = nullptr;
    if (!call.rx_nodes.empty()) {
        // the kept tree is uploaded once; any other tree replaces it there
        if (!(call.rx_tree_cached && c->rxt_on_device)) {
            c->rxt_on_device = false;
            HIPCHK(c, ensure(c->d_rxnodes, sizeof(RxNode) * call.rx_nodes.size()));
            HIPCHK(c, ensure(c->d_rxperm, sizeof(int32_t) * call.rx_perm.size()));
            HIPCHK(c, hipMemcpyAsync(c->d_rxnodes.p, call.rx_nodes.data(),
                                     sizeof(RxNode) * call.rx_nodes.size(), hipMemcpyHostToDevice,
                                     st));
            HIPCHK(c, hipMemcpyAsync(c->d_rxperm.p, call.rx_perm.data(),
                                     sizeof(int32_t) * call.rx_perm.size(), hipMemcpyHostToDevice,
                                     st));
            c->rxt_on_device = call.rx_tree_cached;
        }
        call.dev.rx_nodes = c->d_rxnodes.as<const RxNode>();
        call.dev.rx_perm = c->d_rxperm.as<const int32_t>();
    }
    call.dev.n_jobs = (int32_t)call.jobs.size();
    call.dev.chunk = call.chunk;
    call.dev.n_packets = call.n_packets;
    // LDS staging only when every job traces the same scene
    bool one_scene = call.scenes.size() == 1;
    call.s0 = sd.empty() ? SceneDev{} : sd[0];
    if (one_scene) {
        call.lp = plan_for(call.scenes[0], c->trace_block);
    } else {
        call.lp = LdsPlan{};
        call.lp.block = 256;
    }
    return SBR_OK;
}

int trace_blocks(const sbr_context* c, const Call& call)
{
    int64_t per_block = std::max<int64_t>(1, call.lp.block / 64);
    int64_t want = (call.n_packets + per_block - 1) / per_block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, c->persist_blocks));
}

// Iterations per refinement step for U paths: three only for few paths
// (latency-bound), two up to lookahead_max_paths, else one; 0 selects the
// persistent work-queue refinement.
int32_t max_iterations(const Call& call)
{
    int32_t m = 0;
    for (const JobDev& J : call.jobs) m = std::max(m, J.iterations);
    return m;
}

int refine_depth(const sbr_context* c, int64_t U)
{
    if (c->lookahead_depth == 0) return 0;
    if (U > c->lookahead_max_paths) return 1;
    if (c->refine_segments) return U > c->lookahead3_max_paths ? kRefineSegments : kRefineSegments2;
    if (c->lookahead_depth >= 3 && U > c->lookahead3_max_paths) return 2;
    return c->lookahead_depth;
}

// The call's trace.  With a streamed grid (first pass only), the ring setup
// goes to the grid stream once the main stream has reached this point (so
// the previous call's trace has finished reading the setup's scratch); a
// one-lane kernel then waits until the setup has started, so that the
// persistent trace cannot take the slot it needs, and the main stream joins
// the setup after the trace.  A streamed counting call forms its grid first.
sbr_status trace_launch(sbr_context* c, Call& call, int64_t cap, int32_t* out_tri,
                        double* out_t, unsigned long long* tallies)
{
    hipStream_t st = c->stream;
    Counters* dc = c->counters.as<Counters>();
    call.dev.gscr = nullptr;
    call.dev.gprog = nullptr;
    if (call.stream_grid && tallies) {
        const JobDev& J = call.jobs[0];
        HIPCHK(c, launch_grid(GridDev{(double*)J.dir, J.N, call.stream_n, SBR_LAUNCH_EQUIANGULAR},
                              st, c->grid_scratch.p, c->grid_check_log2));
        call.stream_grid = false;
    }
    if (call.stream_grid) {
        call.streamed = true;
        if (!c->grid_stream)
            HIPCHK(c, hipStreamCreateWithFlags(&c->grid_stream, hipStreamNonBlocking));
        if (!c->ev_grid_fork)
            HIPCHK(c, hipEventCreateWithFlags(&c->ev_grid_fork, hipEventDisableTiming));
        if (!c->ev_grid_join)
            HIPCHK(c, hipEventCreateWithFlags(&c->ev_grid_join, hipEventDisableTiming));
        HIPCHK(c, ensure(c->gprog, sizeof(unsigned long long)));
        if (++c->grid_epoch == 0) c->grid_epoch = 1;
        unsigned long long* prog = c->gprog.as<unsigned long long>();
        HIPCHK(c, hipEventRecord(c->ev_grid_fork, st));
        HIPCHK(c, hipStreamWaitEvent(c->grid_stream, c->ev_grid_fork, 0));
        HIPCHK(c, launch_grid_setup_streamed(call.stream_n, c->grid_scratch.p, c->grid_check_log2,
                                             prog, c->grid_epoch, c->grid_stream));
        HIPCHK(c, hipEventRecord(c->ev_grid_join, c->grid_stream));
        // the setup starts within microseconds when it can; a wave waits at
        // most about a second for a layer
        const uint32_t want = c->grid_epoch + (c->grid_stream_miss ? 1u : 0u);
        HIPCHK(c, launch_grid_wait_started(prog, want, &dc->err,
                                           c->grid_stream_miss ? 16u : (1u << 16), st));
        call.dev.gscr = (const char*)c->grid_scratch.p;
        call.dev.gprog = prog;
        call.dev.gepoch = want;
        call.dev.gn = call.stream_n;
        call.dev.gcheck = c->grid_check_log2;
        call.dev.gspin = c->grid_stream_miss ? 16u : (1u << 20);
    }
    HIPCHK(c, hipEventRecord(c->ev[7], st));
    HIPCHK(c, launch_trace(call.dev, call.lp, call.s0, trace_blocks(c, call), &dc->queue,
                           c->cand.as<sbr_candidate>(), cap, &dc->cand, out_tri, out_t, &dc->err,
                           st, tallies));
    HIPCHK(c, hipEventRecord(c->ev[2], st));
    if (call.stream_grid) {
        HIPCHK(c, hipStreamWaitEvent(st, c->ev_grid_join, 0));
        // a later pass finds the directions in place
        call.stream_grid = false;
        call.dev.gscr = nullptr;
        call.dev.gprog = nullptr;
    }
    return SBR_OK;
}

// What a nonzero error word of the device counters means.
const char* device_error(int32_t err)
{
    if (err & 1) return "traversal stack overflow";
    if (err & 2) return "refinement work queue did not drain";
    if (err & 12) return "streamed launch grid: the ring setup did not publish in time";
    return "device error";
}

// Launch, trace and reception, then path test 1.  On return the context
// holds cand (n_cand events) and, with need_unique, uniq (the path-test-1
// winners, n_uniq or -- small -- a count on the device).  Without
// need_unique, idx holds the sorted permutation of the events.
sbr_status run_front(sbr_context* c, Call& call, bool need_unique, int32_t* out_tri,
                     double* out_t, unsigned long long* tallies, bool speculate = false)
{
    hipStream_t st = c->stream;
    sbr_status r = upload_call(c, call);
    if (r) return r;
    HIPCHK(c, hipEventRecord(c->ev[1], st));
    HIPCHK(c, ensure(c->counters, sizeof(Counters)));
    int64_t cap = std::max<int64_t>(65536, (int64_t)(c->cand.cap / sizeof(sbr_candidate)));
    Counters* hc = c->host_ctr;
    Counters* dc = c->counters.as<Counters>();
    if (speculate && need_unique && !tallies && c->spec_events >= 0 &&
        c->spec_events <= kSmallEvents / 2) {
        // The last call had few events: trace and run path test 1 in one
        // workgroup for up to twice as many, reading the count on the device;
        // run_paths checks it after its one read-back.
        const int64_t bound = std::min<int64_t>(kSmallEvents, std::max<int64_t>(256, 2 * c->spec_events));
        HIPCHK(c, ensure(c->cand, sizeof(sbr_candidate) * (size_t)cap));
        sbr_status r2 = trace_launch(c, call, cap, out_tri, out_t, nullptr);
        if (r2) return r2;
        HIPCHK(c, ensure(c->uniq, sizeof(sbr_candidate) * (size_t)bound));
        HIPCHK(c, launch_dedup_small(c->cand.as<sbr_candidate>(), bound, c->uniq.as<sbr_candidate>(),
                                     &dc->n_unique, st, &dc->cand));
        HIPCHK(c, hipEventRecord(c->ev[3], st));
        call.small = true;
        call.spec = true;
        call.cap = cap;
        call.n_cand = bound;
        call.n_uniq = -1;
        call.u_pred = c->spec_unique;
        return SBR_OK;
    }
    for (int pass = 0;; ++pass) {
        HIPCHK(c, ensure(c->cand, sizeof(sbr_candidate) * (size_t)cap));
        if (pass > 0)  // upload_call zeroed them for the first pass
            HIPCHK(c, hipMemsetAsync(c->counters.p, 0, sizeof(Counters), st));
        if (tallies) HIPCHK(c, hipMemsetAsync(tallies, 0, 12 * sizeof(unsigned long long), st));
        const bool streamed = call.stream_grid;
        sbr_status r2 = trace_launch(c, call, cap, out_tri, out_t, tallies);
        if (r2) return r2;
        HIPCHK(c, hipMemcpyAsync(hc, c->counters.p, sizeof(Counters), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        if (streamed && (hc->err & 12)) return grid_stream_missed(c);
        if (hc->err) return fail(c, SBR_E_INTERNAL, "%s", device_error(hc->err));
        if ((int64_t)hc->cand <= cap) break;
        if (hc->cand >= (1ull << 31))
            return fail(c, SBR_E_CAPACITY, "%llu reception events exceed 2^31", hc->cand);
        cap = (int64_t)(hc->cand + hc->cand / 4 + 1024);
    }
    call.n_cand = (int64_t)hc->cand;
    HIPCHK(c, hipEventElapsedTime(&call.ms_launch, c->ev[0], c->ev[1]));
    if (!call.grids_built) call.ms_launch = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&call.ms_trace, c->ev[7], c->ev[2]));

    // sort + path test 1
    const int64_t C = call.n_cand;
    if (need_unique && C <= kSmallEvents) {
        HIPCHK(c, ensure(c->uniq, sizeof(sbr_candidate) * (size_t)std::max<int64_t>(C, 1)));
        HIPCHK(c, launch_dedup_small(c->cand.as<sbr_candidate>(), C, c->uniq.as<sbr_candidate>(),
                                     &dc->n_unique, st));
        call.small = true;
        call.n_uniq = -1;
        HIPCHK(c, hipEventRecord(c->ev[3], st));
        return SBR_OK;
    }
    int64_t P2 = pow2_at_least(C);
    HIPCHK(c, ensure(c->idx, sizeof(uint32_t) * (size_t)P2));
    HIPCHK(c, launch_sort_candidates(c->cand.as<sbr_candidate>(), C, c->idx.as<uint32_t>(), st));
    if (need_unique) {
        HIPCHK(c, ensure(c->flags, sizeof(int32_t) * (size_t)std::max<int64_t>(C, 1)));
        HIPCHK(c, ensure(c->offs, sizeof(int32_t) * (size_t)std::max<int64_t>(C, 1)));
        HIPCHK(c, ensure(c->scan, scan_scratch_bytes(C)));
        HIPCHK(c, launch_heads(c->cand.as<sbr_candidate>(), c->idx.as<uint32_t>(), C,
                               c->flags.as<int32_t>(), st));
        HIPCHK(c, launch_scan(c->flags.as<int32_t>(), c->offs.as<int32_t>(), C, &dc->n_unique,
                              c->scan.p, st));
        HIPCHK(c, hipMemcpyAsync(hc, c->counters.p, sizeof(Counters), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        call.n_uniq = hc->n_unique;
        HIPCHK(c, ensure(c->uniq, sizeof(sbr_candidate) * (size_t)std::max<int64_t>(call.n_uniq, 1)));
        HIPCHK(c, launch_gather_unique(c->cand.as<sbr_candidate>(), c->idx.as<uint32_t>(),
                                       c->flags.as<int32_t>(), c->offs.as<int32_t>(), C,
                                       c->uniq.as<sbr_candidate>(), st));
    }
    HIPCHK(c, hipEventRecord(c->ev[3], st));
    return SBR_OK;
}

sbr_status ensure_host_paths(sbr_context* c, int64_t n)
{
    if (n <= c->host_paths_cap) return SBR_OK;
    if (c->host_paths) (void)hipHostFree(c->host_paths);
    c->host_paths = nullptr;
    c->host_paths_cap = 0;
    HIPCHK(c, hipHostMalloc((void**)&c->host_paths, sizeof(sbr_path) * (size_t)n, 0));
    c->host_paths_cap = n;
    return SBR_OK;
}

// Items beyond this many bytes send the refinement to the lookahead kernels.
constexpr int64_t kQueueMaxBytes = int64_t(256) << 20;

// The precise algorithm through the persistent work queue (refine_queue.h):
// buffers for Umax paths of the call's jobs, zeroed items and counters.
sbr_status refine_by_queue(sbr_context* c, Call& call, int64_t Umax, const int32_t* ndev,
                           int32_t* err)
{
    hipStream_t st = c->stream;
    int32_t max_it = 1;
    for (const JobDev& J : call.jobs) max_it = std::max(max_it, J.iterations);
    RefineQueue Q;
    Q.cap = refine_queue_cap(std::max<int64_t>(Umax, 1), max_it);
    const size_t U1 = (size_t)std::max<int64_t>(Umax, 1);
    HIPCHK(c, ensure(c->q_state, sizeof(QState) * U1));
    HIPCHK(c, ensure(c->q_slot, sizeof(QSlot) * 8 * U1));
    HIPCHK(c, ensure(c->q_items, sizeof(unsigned long long) * (size_t)Q.cap));
    HIPCHK(c, ensure(c->q_ctr, 16));
    HIPCHK(c, launch_zero(c->q_items.p, sizeof(unsigned long long) * (size_t)Q.cap, st));
    HIPCHK(c, launch_zero(c->q_ctr.p, 16, st));
    Q.state = c->q_state.as<QState>();
    Q.slot = c->q_slot.as<QSlot>();
    Q.items = c->q_items.as<unsigned long long>();
    Q.ctr = c->q_ctr.as<uint32_t>();
    const int blocks = (int)std::max<int64_t>(
        1, std::min<int64_t>((Umax * 7 + 255) / 256, c->persist_blocks));
    HIPCHK(c, launch_refine_queue(call.dev, c->uniq.as<sbr_candidate>(), Umax, ndev, Q, blocks,
                                  c->refine.as<RefineOut>(), err, st));
    return SBR_OK;
}

bool queue_fits(const Call& call, int64_t Umax)
{
    int32_t max_it = 1;
    for (const JobDev& J : call.jobs) max_it = std::max(max_it, J.iterations);
    return refine_queue_cap(std::max<int64_t>(Umax, 1), max_it) * 8 <= kQueueMaxBytes;
}

// The back half: precise algorithm, path quantities / path test 2 / power,
// and the canonical emit into out.
sbr_status run_paths(sbr_context* c, Call& call, sbr_path* out, int64_t capacity, int64_t* n_out,
                     sbr_trace_stats* stats, bool out_on_device = false)
{
    hipStream_t st = c->stream;
    Counters* hc = c->host_ctr;
    Counters* dc = c->counters.as<Counters>();
    sbr_status r;
    // U_max bounds the number of unique paths; with the one-workgroup path
    // test 1 the exact count stays on the device and the kernels read it.
    const int64_t Umax = call.small ? call.n_cand : call.n_uniq;
    const int32_t* ndev = call.small ? &dc->n_unique : nullptr;
    const size_t U1 = (size_t)std::max<int64_t>(Umax, 1);
    HIPCHK(c, ensure(c->refine, sizeof(RefineOut) * U1));
    HIPCHK(c, ensure(c->geom, sizeof(PathGeom) * U1));
    HIPCHK(c, ensure(c->geom0, sizeof(PathGeom) * U1));
    HIPCHK(c, ensure(c->paths, sizeof(sbr_path) * U1));
    HIPCHK(c, ensure(c->keep, sizeof(int32_t) * U1));
    HIPCHK(c, ensure(c->offs, sizeof(int32_t) * U1));
    HIPCHK(c, ensure(c->scan, scan_scratch_bytes(Umax)));
    LdsPlan lp256 = call.scenes.size() == 1 ? plan_for(call.scenes[0], 256) : LdsPlan{};
    lp256.block = 256;
    int depth = refine_depth(c, call.spec ? call.u_pred : Umax);
    if (depth == 0 && !queue_fits(call, Umax)) depth = 1;
    LdsPlan lp3 = call.scenes.size() == 1 ? plan_la3(call.scenes[0]) : LdsPlan{};
    if (depth == 0) {
        // the work queue allocates as it goes: its launches stay on one stream
        HIPCHK(c, launch_solve_exact(call.dev, c->uniq.as<sbr_candidate>(), Umax, ndev,
                                     c->paths.as<sbr_path>(), c->keep.as<int32_t>(),
                                     c->geom0.as<PathGeom>(), &dc->err, st));
        r = refine_by_queue(c, call, Umax, ndev, &dc->err);
        if (r) return r;
        HIPCHK(c, hipEventRecord(c->ev[4], st));
    } else {
        // path test 2 and the exact path need no refinement result: they run
        // on the second stream beside the refinement, which leaves most of the
        // machine idle
        HIPCHK(c, hipEventRecord(c->ev_fork, st));
        HIPCHK(c, hipStreamWaitEvent(c->stream2, c->ev_fork, 0));
        HIPCHK(c, launch_solve_exact(call.dev, c->uniq.as<sbr_candidate>(), Umax, ndev,
                                     c->paths.as<sbr_path>(), c->keep.as<int32_t>(),
                                     c->geom0.as<PathGeom>(), &dc->err, c->stream2));
        HIPCHK(c, hipEventRecord(c->ev_join, c->stream2));
        HIPCHK(c, launch_refine(call.dev, lp256, lp3, call.s0, c->uniq.as<sbr_candidate>(), Umax,
                                ndev, depth, c->refine.as<RefineOut>(), c->geom.as<PathGeom>(),
                                &dc->err, st, max_iterations(call), c->seg_tail));
        HIPCHK(c, hipEventRecord(c->ev[4], st));
        HIPCHK(c, hipStreamWaitEvent(st, c->ev_join, 0));
    }
    HIPCHK(c, launch_solve_refined(call.dev, c->uniq.as<sbr_candidate>(),
                                   c->refine.as<RefineOut>(), c->geom.as<PathGeom>(),
                                   c->geom0.as<PathGeom>(), Umax, ndev, c->paths.as<sbr_path>(),
                                   &dc->err, st, depth == 0));
    HIPCHK(c, hipEventRecord(c->ev[5], st));

    // emit: stable compaction of kept paths (already in canonical order)
    int64_t P = 0, U = call.n_uniq;
    if (call.small) {
        // one workgroup compacts; the list (at most Umax records) and the
        // counts come back in one round trip.  Device output is written in
        // place (only when it fits the capacity).
        if (out_on_device) {
            HIPCHK(c, launch_emit_small(c->paths.as<sbr_path>(), c->keep.as<int32_t>(), Umax, ndev,
                                        out, capacity, &dc->n_paths, st));
        } else {
            HIPCHK(c, ensure(c->outp, sizeof(sbr_path) * U1));
            HIPCHK(c, launch_emit_small(c->paths.as<sbr_path>(), c->keep.as<int32_t>(), Umax, ndev,
                                        c->outp.as<sbr_path>(), (int64_t)U1, &dc->n_paths, st));
            r = ensure_host_paths(c, (int64_t)U1);
            if (r) return r;
            if (Umax > 0)
                HIPCHK(c, hipMemcpyAsync(c->host_paths, c->outp.p, sizeof(sbr_path) * (size_t)Umax,
                                         hipMemcpyDeviceToHost, st));
        }
        HIPCHK(c, hipMemcpyAsync(hc, c->counters.p, sizeof(Counters), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipEventRecord(c->ev[6], st));
        HIPCHK(c, hipEventSynchronize(c->ev[6]));
        if (call.spec) {
            if ((hc->err & 2) != 0)
                return fail(c, SBR_E_INTERNAL, "refinement work queue did not drain");
            if (call.streamed && (hc->err & 12)) return grid_stream_missed(c);
            if (hc->err || (int64_t)hc->cand > call.n_cand) return kSpecMiss;
            call.n_cand = (int64_t)hc->cand;
            HIPCHK(c, hipEventElapsedTime(&call.ms_launch, c->ev[0], c->ev[1]));
            if (!call.grids_built) call.ms_launch = 0.0f;
            HIPCHK(c, hipEventElapsedTime(&call.ms_trace, c->ev[7], c->ev[2]));
        }
        if (call.streamed && (hc->err & 12)) return grid_stream_missed(c);
        if (hc->err) return fail(c, SBR_E_INTERNAL, "%s", device_error(hc->err));
        P = hc->n_paths;
        U = hc->n_unique;
        *n_out = P;
        if (P > capacity)
            return fail(c, SBR_E_CAPACITY, "%lld paths, capacity %lld", (long long)P,
                        (long long)capacity);
        if (P > 0 && !out_on_device) memcpy(out, c->host_paths, sizeof(sbr_path) * (size_t)P);
    } else {
        HIPCHK(c, launch_scan(c->keep.as<int32_t>(), c->offs.as<int32_t>(), U, &dc->n_paths,
                              c->scan.p, st));
        HIPCHK(c, hipMemcpyAsync(hc, c->counters.p, sizeof(Counters), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        if (hc->err) return fail(c, SBR_E_INTERNAL, "%s", device_error(hc->err));
        P = hc->n_paths;
        *n_out = P;
        if (P > capacity)
            return fail(c, SBR_E_CAPACITY, "%lld paths, capacity %lld", (long long)P,
                        (long long)capacity);
        HIPCHK(c, ensure(c->outp, sizeof(sbr_path) * (size_t)std::max<int64_t>(P, 1)));
        HIPCHK(c, launch_compact_paths(c->paths.as<sbr_path>(), c->keep.as<int32_t>(),
                                       c->offs.as<int32_t>(), U, c->outp.as<sbr_path>(), st));
        if (P > 0)
            HIPCHK(c, hipMemcpyAsync(out, c->outp.p, sizeof(sbr_path) * (size_t)P,
                                     out_on_device ? hipMemcpyDeviceToDevice
                                                   : hipMemcpyDeviceToHost,
                                     st));
        HIPCHK(c, hipEventRecord(c->ev[6], st));
        HIPCHK(c, hipEventSynchronize(c->ev[6]));
    }
    if (stats) {
        memset(stats, 0, sizeof(*stats));
        stats->n_rays = call.n_rays;
        stats->n_candidates = call.n_cand;
        stats->n_unique = U;
        stats->n_paths = P;
        float a = 0, b = 0, e = 0, tot = 0, dd = 0;
        (void)hipEventElapsedTime(&dd, c->ev[2], c->ev[3]);
        (void)hipEventElapsedTime(&a, c->ev[3], c->ev[4]);
        (void)hipEventElapsedTime(&b, c->ev[4], c->ev[5]);
        (void)hipEventElapsedTime(&e, c->ev[5], c->ev[6]);
        (void)hipEventElapsedTime(&tot, c->ev[0], c->ev[6]);
        stats->ms_launch = call.ms_launch;
        stats->ms_trace = call.ms_trace;
        stats->ms_dedup = dd;
        stats->ms_refine = a;
        stats->ms_solve = b;
        stats->ms_emit = e;
        stats->ms_total = tot;
        stats->lds_bytes = call.lp.bytes;
        stats->lds_nodes = call.lp.n_nodes;
        stats->lds_tris = call.lp.n_tris;
        stats->lds_max = c->lds_max;
    }
    return SBR_OK;
}

// A call with one job on one scene.
// After a completed single-job call with a fresh equiangular grid formed
// before its trace (and no ray order made): its grid and trace times, which
// decide whether later calls stream the grid (sbr_context::grid_times).
void note_grid_times(sbr_context* c, const Call& call, const sbr_trace_params* p)
{
    if (!(p->flags & SBR_FLAG_FRESH_GRID) || p->launch != SBR_LAUNCH_EQUIANGULAR ||
        call.jobs.size() != 1 || call.streamed || !call.grids_built || call.order_built)
        return;
    c->grid_times[p->launch * 100000 + p->division_n] = {call.ms_launch, call.ms_trace};
}

sbr_status single_call(sbr_scene* s, Call& call, const double* tx, const double* rx,
                       int32_t n_rx, const sbr_trace_params* p, int64_t ray_begin,
                       int64_t ray_count)
{
    sbr_context* c = s->ctx;
    call.scenes.push_back(s);
    call.rx = rx;
    call.n_rx = n_rx;
    call.rx_job.assign((size_t)n_rx, 0);
    call.chunk = c->trace_chunk;
    HIPCHK(c, hipEventRecord(c->ev[0], c->stream));
    int64_t N = num_rays(p->launch, p->division_n);
    return add_job(c, call, 0, tx, 0, n_rx, p, ray_begin, ray_count < 0 ? N : ray_count);
}

}  // namespace

namespace sbr {
LdsPlan make_lds_plan(int64_t NN, int64_t T, int block, int depth, int budget)
{
    LdsPlan L;
    L.block = block;
    int64_t per_entry = 4 * (int64_t)block;
    depth = (int)std::min<int64_t>(depth, std::max<int64_t>(0, budget / per_entry));
    L.depth = depth;
    int64_t avail = (int64_t)budget - per_entry * depth;
    if (NN * (int64_t)sizeof(Bvh4Node) + T * (int64_t)sizeof(TriD) <= avail) {
        L.n_nodes = (int32_t)NN;
        L.n_tris = (int32_t)T;
    } else {
        L.n_nodes = (int32_t)std::min<int64_t>(NN, avail / (int64_t)sizeof(Bvh4Node));
        L.n_tris = 0;
    }
    L.stack_off = (int32_t)(L.n_nodes * (int64_t)sizeof(Bvh4Node) + L.n_tris * (int64_t)sizeof(TriD));
    L.bytes = (int32_t)(L.stack_off + per_entry * depth);
    return L;
}
}  // namespace sbr

extern "C" {

const char* sbr_status_string(sbr_status s)
{
    switch (s) {
        case SBR_OK: return "ok";
        case SBR_E_INVALID_ARG: return "invalid argument";
        case SBR_E_NO_SCENE: return "no scene";
        case SBR_E_NO_BVH: return "no BVH";
        case SBR_E_CAPACITY: return "output capacity too small";
        case SBR_E_OOM: return "out of memory";
        case SBR_E_DEVICE: return "HIP device error";
        case SBR_E_INTERNAL: return "internal error";
        case SBR_E_SCRATCH: return "exceeds the fixed scratch of the no-allocation entry point";
        default: return "unknown status";
    }
}

const char* sbr_last_error(const sbr_context* ctx)
{
    return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

sbr_status sbr_context_create(int32_t device, void* hip_stream, sbr_context** out)
{
    g_create_err.clear();
    if (!out) {
        g_create_err = "out is NULL";
        return SBR_E_INVALID_ARG;
    }
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) {
        g_create_err = std::string("no HIP device: ") + hipGetErrorString(e);
        return SBR_E_DEVICE;
    }
    if (device < 0 || device >= count) {
        g_create_err = "device index out of range";
        return SBR_E_INVALID_ARG;
    }
    e = hipSetDevice(device);
    if (e != hipSuccess) {
        g_create_err = std::string("hipSetDevice: ") + hipGetErrorString(e);
        return SBR_E_DEVICE;
    }
    sbr_context* c = new sbr_context();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    for (auto& ev : c->ev) {
        e = hipEventCreate(&ev);
        if (e != hipSuccess) break;
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->host_ctr, sizeof(Counters), 0);
    if (e == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) ==
                hipSuccess && v > 0)
            c->lds_max = v;
        if (trace_set_lds_limit(c->lds_max) != hipSuccess ||
            refine_set_lds_limit(c->lds_max) != hipSuccess) {
            (void)hipGetLastError();
            c->lds_max = 65536;
        }
        c->lds_budget = env_int("SBR_LDS_BUDGET", 0, 0, c->lds_max);
        c->trace_block = env_int("SBR_TRACE_BLOCK", 256, 64, 256) / 64 * 64;
        c->stack_depth = env_int("SBR_STACK_DEPTH", 24, 0, kTraceStack);
        c->lookahead_max_paths = env_int("SBR_LOOKAHEAD_PATHS", 4096, 0, 1 << 30);
        c->trace_chunk = env_int("SBR_TRACE_CHUNK", 1, 1, 64);
        c->persist_blocks = env_int("SBR_TRACE_BLOCKS", 2048, 1, 1 << 20);
        c->rx_tree_min = env_int("SBR_RX_TREE_MIN", 64, 1, 0x7fffffff);
        c->lookahead_depth = env_int("SBR_LOOKAHEAD_DEPTH", 3, 0, 3);
        c->lookahead3_max_paths = env_int("SBR_LOOKAHEAD3_PATHS", 256, 0, 1 << 30);
        c->refine_segments = env_int("SBR_REFINE_SEGMENTS", 1, 0, 1);
        c->seg_tail = env_int("SBR_SEG_TAIL", 10, 0, 200);
        c->la3_lds = env_int("SBR_LA3_LDS", 1, 0, 1) != 0;
        c->ray_order = env_int("SBR_RAY_ORDER", 1, 0, 1);
        c->grid_stream_mode = env_int("SBR_GRID_STREAM", 1, 0, 2);
        c->grid_stream_miss = env_int("SBR_GRID_STREAM_MISS", 0, 0, 1) != 0;
        c->grid_order = env_int("SBR_GRID_ORDER", 2, 0, 2);
        c->grid_prefix = env_int("SBR_GRID_PREFIX", 35, 0, 100);
        if (refine_la3_set_lds_limit(c->lds_max - 2048) != hipSuccess) {
            (void)hipGetLastError();
            c->la3_lds = false;
        }
        // the no-allocation entry point's scratch (a failure only disables it)
        c->scratch_err = noalloc_scratch_ptr(device, &c->scratch);
    }
    if (e != hipSuccess) {
        g_create_err = std::string("context setup: ") + hipGetErrorString(e);
        for (auto& ev : c->ev)
            if (ev) (void)hipEventDestroy(ev);
        if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
        if (c->ev_join) (void)hipEventDestroy(c->ev_join);
        if (c->stream2) (void)hipStreamDestroy(c->stream2);
        delete c;
        return SBR_E_DEVICE;
    }
    *out = c;
    return SBR_OK;
}

sbr_status sbr_context_get_tuning(const sbr_context* c, sbr_tuning* t)
{
    if (!c || !t) return SBR_E_INVALID_ARG;
    t->trace_chunk = c->trace_chunk;
    t->persist_blocks = c->persist_blocks;
    t->trace_block = c->trace_block;
    t->stack_depth = c->stack_depth;
    t->lds_budget = c->lds_budget;
    t->rx_tree_min = c->rx_tree_min;
    t->lookahead_max_paths = c->lookahead_max_paths;
    t->lookahead_depth = c->lookahead_depth;
    t->lookahead3_max_paths = c->lookahead3_max_paths;
    t->grid_check_log2 = c->grid_check_log2;
    t->ray_order = c->ray_order;
    t->refine_segments = c->refine_segments;
    return SBR_OK;
}

sbr_status sbr_context_set_tuning(sbr_context* c, const sbr_tuning* t)
{
    if (!c) return SBR_E_INVALID_ARG;
    c->err.clear();
    if (!t) return fail(c, SBR_E_INVALID_ARG, "tuning is NULL");
    if (t->trace_chunk < 1 || t->trace_chunk > 64 || t->persist_blocks < 1 ||
        t->trace_block < 64 || t->trace_block > 256 || t->trace_block % 64 != 0 ||
        t->stack_depth < 0 || t->stack_depth > kTraceStack || t->lds_budget < 0 ||
        t->lds_budget > c->lds_max || t->rx_tree_min < 1 || t->lookahead_max_paths < 0 ||
        t->lookahead_depth < 0 || t->lookahead_depth > 3 || t->lookahead3_max_paths < 0 ||
        t->grid_check_log2 < 0 || t->grid_check_log2 > 200 || t->ray_order < 0 ||
        t->ray_order > 1 || t->refine_segments < 0 || t->refine_segments > 1)
        return fail(c, SBR_E_INVALID_ARG, "tuning field out of range");
    if (t->grid_check_log2 != c->grid_check_log2) {
        // cached grids were made under the old setting (they are the same
        // values; dropping them lets the next call exercise the new one)
        for (auto& kv : c->grids) release(kv.second);
        c->grids.clear();
    }
    c->trace_chunk = t->trace_chunk;
    c->persist_blocks = t->persist_blocks;
    c->trace_block = t->trace_block;
    c->stack_depth = t->stack_depth;
    c->lds_budget = t->lds_budget;
    c->rx_tree_min = t->rx_tree_min;
    c->lookahead_max_paths = t->lookahead_max_paths;
    c->lookahead_depth = t->lookahead_depth;
    c->lookahead3_max_paths = t->lookahead3_max_paths;
    c->grid_check_log2 = t->grid_check_log2;
    c->ray_order = t->ray_order;
    c->refine_segments = t->refine_segments;
    return SBR_OK;
}

sbr_status sbr_context_destroy(sbr_context* c)
{
    if (!c) return SBR_E_INVALID_ARG;
    if (c->n_scenes > 0) return fail(c, SBR_E_INVALID_ARG, "%d scene(s) still alive", c->n_scenes);
    (void)use_device(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->grid_stream) (void)hipStreamSynchronize(c->grid_stream);
    for (auto& kv : c->grids) release(kv.second);
    for (auto& kv : c->orders) release(kv.second);
    for (auto& kv : c->orders_stream) release(kv.second);
    release(c->gprog);
    if (c->ev_grid_fork) (void)hipEventDestroy(c->ev_grid_fork);
    if (c->ev_grid_join) (void)hipEventDestroy(c->ev_grid_join);
    if (c->grid_stream) (void)hipStreamDestroy(c->grid_stream);
    DevBuf* bufs[] = {&c->grid_scratch, &c->rx,    &c->rx32,  &c->cand,  &c->idx,  &c->flags,
                      &c->offs,         &c->scan,  &c->uniq,  &c->refine, &c->paths,
                      &c->keep,         &c->outp,  &c->counters, &c->rays_tri, &c->rays_t, &c->tally,
                      &c->geom,         &c->d_jobs, &c->d_scenes, &c->d_rxjob,
                      &c->d_rxnodes,    &c->d_rxperm, &c->d_rxp, &c->dpaths, &c->dout,
                      &c->q_state,      &c->q_slot,  &c->q_items, &c->q_ctr, &c->geom0};
    for (DevBuf* b : bufs) release(*b);
    for (auto& ev : c->ev)
        if (ev) (void)hipEventDestroy(ev);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->stream2) (void)hipStreamDestroy(c->stream2);
    if (c->host_ctr) (void)hipHostFree(c->host_ctr);
    if (c->host_paths) (void)hipHostFree(c->host_paths);
    drop_graph(c);
    if (c->graph.cap_stream) (void)hipStreamDestroy(c->graph.cap_stream);
    if (c->graph.h_job) (void)hipHostFree(c->graph.h_job);
    if (c->graph.h_scene) (void)hipHostFree(c->graph.h_scene);
    if (c->graph.h_rxjob) (void)hipHostFree(c->graph.h_rxjob);
    drop_bgraph(c);
    auto& B = c->bgraph;
    if (B.cap_stream) (void)hipStreamDestroy(B.cap_stream);
    void* pinned[] = {B.h_jobs, B.h_scenes, B.h_rxjob, B.h_rx};
    for (void* q : pinned)
        if (q) (void)hipHostFree(q);
    delete c;
    return SBR_OK;
}

sbr_status sbr_scene_upload(sbr_context* c, const double* xyz, int64_t nv, const int32_t* tri,
                            const int32_t* face_id, const int32_t* mat_id, int64_t T,
                            const sbr_complex* eps_r, int32_t M, sbr_scene** out)
{
    if (!c) return SBR_E_INVALID_ARG;
    c->err.clear();
    if (!out) return fail(c, SBR_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (nv < 0 || T < 0 || T >= (1ll << 31) || M < 0)
        return fail(c, SBR_E_INVALID_ARG, "negative or too large sizes");
    if (T > 0 && (!xyz || !tri || !face_id || !mat_id || !eps_r || M < 1))
        return fail(c, SBR_E_INVALID_ARG, "NULL scene array");
    for (int64_t i = 0; i < nv; ++i)
        if (!finite3(xyz + 3 * i)) return fail(c, SBR_E_INVALID_ARG, "vertex %lld not finite", (long long)i);
    for (int32_t m = 0; m < M; ++m)
        if (!isfinite(eps_r[m].re) || !isfinite(eps_r[m].im))
            return fail(c, SBR_E_INVALID_ARG, "eps_r[%d] not finite", m);
    static uint64_t next_scene_id = 0;
    sbr_scene* s = new sbr_scene();
    s->ctx = c;
    s->id = ++next_scene_id;
    s->T = T;
    s->M = M;
    s->tri_v.resize((size_t)T * 9);
    s->face.assign(face_id, face_id + T);
    s->mat.assign(mat_id, mat_id + T);
    s->eps.resize((size_t)std::max(M, 1) * 2);
    for (int32_t m = 0; m < M; ++m) {
        s->eps[2 * m] = eps_r[m].re;
        s->eps[2 * m + 1] = eps_r[m].im;
    }
    int32_t F = 0;
    d3 lo = mk(INFINITY, INFINITY, INFINITY), hi = mk(-INFINITY, -INFINITY, -INFINITY);
    double R = 0.0;
    for (int64_t t = 0; t < T; ++t) {
        for (int v = 0; v < 3; ++v) {
            int32_t vi = tri[3 * t + v];
            if (vi < 0 || vi >= nv) {
                delete s;
                return fail(c, SBR_E_INVALID_ARG, "triangle %lld: vertex index out of range", (long long)t);
            }
            const double* P = xyz + 3 * (size_t)vi;
            for (int q = 0; q < 3; ++q) s->tri_v[9 * t + 3 * v + q] = P[q];
            lo.x = fmin(lo.x, P[0]); lo.y = fmin(lo.y, P[1]); lo.z = fmin(lo.z, P[2]);
            hi.x = fmax(hi.x, P[0]); hi.y = fmax(hi.y, P[1]); hi.z = fmax(hi.z, P[2]);
            R = std::max(R, std::max(fabs(P[0]), std::max(fabs(P[1]), fabs(P[2]))));
        }
        if (face_id[t] < 0 || mat_id[t] < 0 || mat_id[t] >= M) {
            delete s;
            return fail(c, SBR_E_INVALID_ARG, "triangle %lld: face or material id out of range", (long long)t);
        }
        F = std::max(F, face_id[t] + 1);
    }
    s->F = F;
    s->R_s = R;
    if (T > 0) s->t_eps = 1e-9 * norm(sub(hi, lo));
    double diag = T > 0 ? norm(sub(hi, lo)) : 0.0;
    // Face planes: the lowest-index triangle of each face, n = normalize(e1 x e2).
    s->fplane.assign((size_t)std::max(F, 1) * 4, 0.0);
    s->fmat.assign((size_t)std::max(F, 1), 0);
    std::vector<char> seen((size_t)std::max(F, 1), 0);
    for (int64_t t = 0; t < T; ++t) {
        int32_t f = face_id[t];
        if (seen[f]) continue;
        seen[f] = 1;
        const double* V = &s->tri_v[9 * t];
        d3 v0 = ld3(V), e1 = sub(ld3(V + 3), v0), e2 = sub(ld3(V + 6), v0);
        d3 cr = cross(e1, e2);
        if (!(norm(cr) > 0.0)) {
            delete s;
            return fail(c, SBR_E_INVALID_ARG, "face %d: its first triangle is degenerate", f);
        }
        d3 n = normalize(cr);
        s->fplane[4 * f + 0] = n.x;
        s->fplane[4 * f + 1] = n.y;
        s->fplane[4 * f + 2] = n.z;
        s->fplane[4 * f + 3] = dot(n, v0);
        s->fmat[f] = mat_id[t];
    }
    for (int64_t t = 0; t < T; ++t) {
        int32_t f = face_id[t];
        d3 n = ld3(&s->fplane[4 * f]);
        for (int v = 0; v < 3; ++v) {
            double dist = fabs(dot(n, ld3(&s->tri_v[9 * t + 3 * v])) - s->fplane[4 * f + 3]);
            if (!(dist <= 1e-9 * diag + 1e-300)) {
                delete s;
                return fail(c, SBR_E_INVALID_ARG, "triangle %lld is not in the plane of face %d",
                            (long long)t, f);
            }
        }
    }
    c->n_scenes += 1;
    *out = s;
    return SBR_OK;
}

sbr_status sbr_bvh_build(sbr_scene* s, const sbr_bvh_params* bp)
{
    if (!s || !s->ctx) return SBR_E_NO_SCENE;
    sbr_context* c = s->ctx;
    c->err.clear();
    int leaf = bp ? bp->max_leaf_size : 4, bins = bp ? bp->sah_bins : kDefaultSahBins;
    int split = bp ? bp->split_pct : kDefaultSplitPct;
    if (leaf < 1 || leaf > 16 || bins < 4 || bins > 64 || split < 0 || split > 400)
        return fail(c, SBR_E_INVALID_ARG, "bvh params out of range");
    std::vector<Bvh4Node> nodes;
    std::vector<int32_t> perm;
    s->bvh_depth =
        build_bvh(s->tri_v.data(), s->T, leaf, bins, split, c->lds_budget > 0, nodes, perm);
    s->n_nodes = (int64_t)nodes.size();
    // the traversal addresses a node by a 32-bit byte offset
    if (s->n_nodes > kMaxBvhNodes)
        return fail(c, SBR_E_INVALID_ARG, "BVH of %lld nodes: at most %lld", (long long)s->n_nodes,
                    (long long)kMaxBvhNodes);
    if (3 * s->bvh_depth >= kTraceStack) return fail(c, SBR_E_INTERNAL, "BVH too deep");
    // triangle records in leaf order, one per reference
    s->R = (int64_t)perm.size();
    std::vector<TriD> tris((size_t)s->R);
    std::vector<int32_t> pos_of((size_t)s->T, -1);
    for (int64_t q = 0; q < s->R; ++q) {
        int32_t t = perm[q];
        const double* V = &s->tri_v[9 * (size_t)t];
        TriD& d = tris[q];
        d.v0x = V[0]; d.v0y = V[1]; d.v0z = V[2];
        d.e1x = V[3] - V[0]; d.e1y = V[4] - V[1]; d.e1z = V[5] - V[2];
        d.e2x = V[6] - V[0]; d.e2y = V[7] - V[1]; d.e2z = V[8] - V[2];
        d.face = s->face[t];
        d.orig = t;
        if (pos_of[t] < 0) pos_of[t] = (int32_t)q;
    }
    // CSR of triangles per face (positions in leaf order, input order within a face)
    std::vector<int32_t> fstart((size_t)s->F + 1, 0), ftris((size_t)s->T);
    for (int64_t t = 0; t < s->T; ++t) fstart[s->face[t] + 1] += 1;
    for (int32_t f = 0; f < s->F; ++f) fstart[f + 1] += fstart[f];
    std::vector<int32_t> fill(fstart.begin(), fstart.end() - 1);
    for (int64_t t = 0; t < s->T; ++t) ftris[fill[s->face[t]]++] = pos_of[t];

    HIPCHK(c, use_device(c->device));
    HIPCHK(c, ensure(s->nodes, sizeof(Bvh4Node) * nodes.size()));
    HIPCHK(c, ensure(s->tris, sizeof(TriD) * tris.size()));
    HIPCHK(c, ensure(s->d_fplane, sizeof(double) * s->fplane.size()));
    HIPCHK(c, ensure(s->d_fmat, sizeof(int32_t) * s->fmat.size()));
    HIPCHK(c, ensure(s->fstart, sizeof(int32_t) * fstart.size()));
    HIPCHK(c, ensure(s->ftris, sizeof(int32_t) * ftris.size()));
    HIPCHK(c, ensure(s->d_eps, sizeof(double) * s->eps.size()));
    HIPCHK(c, hipMemcpy(s->nodes.p, nodes.data(), sizeof(Bvh4Node) * nodes.size(), hipMemcpyHostToDevice));
    if (!tris.empty())
        HIPCHK(c, hipMemcpy(s->tris.p, tris.data(), sizeof(TriD) * tris.size(), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(s->d_fplane.p, s->fplane.data(), sizeof(double) * s->fplane.size(), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(s->d_fmat.p, s->fmat.data(), sizeof(int32_t) * s->fmat.size(), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(s->fstart.p, fstart.data(), sizeof(int32_t) * fstart.size(), hipMemcpyHostToDevice));
    if (!ftris.empty())
        HIPCHK(c, hipMemcpy(s->ftris.p, ftris.data(), sizeof(int32_t) * ftris.size(), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(s->d_eps.p, s->eps.data(), sizeof(double) * s->eps.size(), hipMemcpyHostToDevice));
    s->has_bvh = true;
    return SBR_OK;
}

sbr_status sbr_scene_destroy(sbr_scene* s)
{
    if (!s || !s->ctx) return SBR_E_NO_SCENE;
    (void)use_device(s->ctx->device);
    (void)hipStreamSynchronize(s->ctx->stream);
    DevBuf* bufs[] = {&s->nodes, &s->tris,  &s->d_fplane, &s->d_fmat,
                      &s->fstart, &s->ftris, &s->d_eps,    &s->d_wedges};
    for (DevBuf* b : bufs) release(*b);
    s->ctx->n_scenes -= 1;
    s->ctx = nullptr;
    delete s;
    return SBR_OK;
}

sbr_status sbr_launch_grid(sbr_context* c, int32_t launch, int32_t n, int64_t first,
                           int64_t count, double* out)
{
    if (!c) return SBR_E_INVALID_ARG;
    c->err.clear();
    if (n < 1 || n > 10000) return fail(c, SBR_E_INVALID_ARG, "n outside 1..10000");
    if (launch < SBR_LAUNCH_EQUIANGULAR || launch > SBR_LAUNCH_EQUIDISTANT_OCTA)
        return fail(c, SBR_E_INVALID_ARG, "unknown launch method %d", launch);
    int64_t N = num_rays(launch, n);
    if (first < 0 || count < 0 || first + count > N || (count > 0 && !out))
        return fail(c, SBR_E_INVALID_ARG, "ray range outside 0..%lld", (long long)N);
    HIPCHK(c, use_device(c->device));
    GridDev g;
    bool built;
    sbr_status r = get_grid(c, launch, n, &g, &built);
    if (r) return r;
    if (count == 0) return SBR_OK;
    std::vector<double> tmp((size_t)count * 3);
    for (int a = 0; a < 3; ++a)
        HIPCHK(c, hipMemcpyAsync(tmp.data() + a * count, g.dir + a * N + first,
                                 sizeof(double) * (size_t)count, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int64_t i = 0; i < count; ++i)
        for (int a = 0; a < 3; ++a) out[3 * i + a] = tmp[a * count + i];
    return SBR_OK;
}

sbr_status sbr_trace_rays(sbr_scene* s, const double tx[3], int32_t launch, int32_t n, int32_t K,
                          int64_t first, int64_t count, int32_t* out_tri, double* out_t)
{
    sbr_status r = check_scene(s);
    if (r) return r;
    sbr_context* c = s->ctx;
    c->err.clear();
    if (!tx || !finite3(tx)) return fail(c, SBR_E_INVALID_ARG, "tx missing or not finite");
    if (n < 1 || n > 10000 || K < 0 || K > SBR_MAX_ORDER || launch < SBR_LAUNCH_EQUIANGULAR ||
        launch > SBR_LAUNCH_EQUIDISTANT_OCTA)
        return fail(c, SBR_E_INVALID_ARG, "n, launch or max_order out of range");
    int64_t N = num_rays(launch, n);
    if (first < 0 || count < 0 || first + count > N)
        return fail(c, SBR_E_INVALID_ARG, "ray range outside 0..%lld", (long long)N);
    HIPCHK(c, use_device(c->device));
    if (count == 0) return SBR_OK;
    sbr_trace_params p{};
    p.max_order = K;
    p.division_n = n;
    p.launch = launch;
    p.iterations = 0;
    p.subrays = 6;
    p.freq_hz = 1.0;
    Call call;
    r = single_call(s, call, tx, nullptr, 0, &p, first, count);
    if (r) return r;
    size_t cells = (size_t)count * (K + 1);
    HIPCHK(c, ensure(c->rays_tri, sizeof(int32_t) * cells));
    HIPCHK(c, ensure(c->rays_t, sizeof(double) * cells));
    r = run_front(c, call, false, c->rays_tri.as<int32_t>(), c->rays_t.as<double>(), nullptr);
    if (r) return r;
    if (out_tri)
        HIPCHK(c, hipMemcpyAsync(out_tri, c->rays_tri.p, sizeof(int32_t) * cells,
                                 hipMemcpyDeviceToHost, c->stream));
    if (out_t)
        HIPCHK(c, hipMemcpyAsync(out_t, c->rays_t.p, sizeof(double) * cells, hipMemcpyDeviceToHost,
                                 c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SBR_OK;
}

static sbr_status check_trace_inputs(sbr_scene* s, const double* tx, const double* rx,
                                     int32_t n_rx, const sbr_trace_params* p, int64_t capacity,
                                     const void* out, int64_t* n_out)
{
    sbr_status r = check_scene(s);
    if (r) return r;
    sbr_context* c = s->ctx;
    c->err.clear();
    if (!n_out) return fail(c, SBR_E_INVALID_ARG, "n_out is NULL");
    *n_out = 0;
    if (!tx || !finite3(tx)) return fail(c, SBR_E_INVALID_ARG, "tx missing or not finite");
    if (n_rx < 0 || (n_rx > 0 && !rx)) return fail(c, SBR_E_INVALID_ARG, "bad rx array");
    for (int32_t x = 0; x < n_rx; ++x)
        if (!finite3(rx + 3 * x)) return fail(c, SBR_E_INVALID_ARG, "rx %d not finite", x);
    if (capacity < 0 || (capacity > 0 && !out)) return fail(c, SBR_E_INVALID_ARG, "bad output array");
    return check_params(c, p);
}

sbr_status sbr_candidates(sbr_scene* s, const double tx[3], const double* rx, int32_t n_rx,
                          const sbr_trace_params* p, sbr_candidate* out, int64_t capacity,
                          int64_t* n_out)
{
    sbr_status r = check_trace_inputs(s, tx, rx, n_rx, p, capacity, out, n_out);
    if (r) return r;
    sbr_context* c = s->ctx;
    HIPCHK(c, use_device(c->device));
    Call call;
    r = single_call(s, call, tx, rx, n_rx, p, 0, -1);
    if (r) return r;
    r = run_front(c, call, false, nullptr, nullptr, nullptr);
    if (r) return r;
    *n_out = call.n_cand;
    if (call.n_cand > capacity)
        return fail(c, SBR_E_CAPACITY, "%lld events, capacity %lld", (long long)call.n_cand,
                    (long long)capacity);
    if (call.n_cand == 0) return SBR_OK;
    HIPCHK(c, ensure(c->uniq, sizeof(sbr_candidate) * (size_t)call.n_cand));
    HIPCHK(c, launch_gather_sorted(c->cand.as<sbr_candidate>(), c->idx.as<uint32_t>(),
                                   call.n_cand, c->uniq.as<sbr_candidate>(), c->stream));
    HIPCHK(c, hipMemcpyAsync(out, c->uniq.p, sizeof(sbr_candidate) * (size_t)call.n_cand,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SBR_OK;
}

sbr_status sbr_trace_counters(sbr_scene* s, const double tx[3], const double* rx, int32_t n_rx,
                              const sbr_trace_params* p, int64_t counts[12])
{
    int64_t dummy;
    sbr_status r = check_trace_inputs(s, tx, rx, n_rx, p, 0, nullptr, &dummy);
    if (r) return r;
    sbr_context* c = s->ctx;
    if (!counts) return fail(c, SBR_E_INVALID_ARG, "counts is NULL");
    HIPCHK(c, use_device(c->device));
    HIPCHK(c, ensure(c->tally, 12 * sizeof(unsigned long long)));
    Call call;
    r = single_call(s, call, tx, rx, n_rx, p, 0, -1);
    if (r) return r;
    r = run_front(c, call, false, nullptr, nullptr, c->tally.as<unsigned long long>());
    if (r) return r;
    unsigned long long h[12];
    HIPCHK(c, hipMemcpy(h, c->tally.p, sizeof h, hipMemcpyDeviceToHost));
    for (int i = 0; i < 12; ++i) counts[i] = (int64_t)h[i];
    return SBR_OK;
}

sbr_status sbr_trace(sbr_scene* s, const double tx[3], const double* rx, int32_t n_rx,
                     const sbr_trace_params* p, sbr_path* out, int64_t capacity, int64_t* n_out,
                     sbr_trace_stats* stats)
{
    sbr_status r = check_trace_inputs(s, tx, rx, n_rx, p, capacity, out, n_out);
    if (r) return r;
    sbr_context* c = s->ctx;
    HIPCHK(c, use_device(c->device));
    for (int attempt = 0;; ++attempt) {
        Call call;
        r = single_call(s, call, tx, rx, n_rx, p, 0, -1);
        if (r) return r;
        r = run_front(c, call, true, nullptr, nullptr, nullptr);
        if (r == SBR_OK) r = run_paths(c, call, out, capacity, n_out, stats);
        if (r == kGridStreamMiss && attempt == 0) continue;  // again, grid formed first
        if (r == kGridStreamMiss) return fail(c, SBR_E_INTERNAL, "%s", device_error(12));
        if (!r) note_grid_times(c, call, p);
        return r;
    }
}

// ---------------------------------------------------------------------------
// Captured graphs of sbr_trace_device calls (SBR_FLAG_GRAPH).  A call whose
// scene, receiver and output buffers, parameters and tuning match the
// captured one replays the graph: the job table (the transmitter and what
// depends on it) is written to pinned staging that the graph copies to the
// device, everything else is fixed at capture.  The graph holds the one-
// workgroup path test 1 and emit, sized by the capturing call; a replay whose
// counts exceed those sizes is detected from the counters and redone as a
// normal call.  Memory is cleared by kernels, not memset nodes.
// ---------------------------------------------------------------------------
namespace {

// Field by field: the struct has tail padding, which memcmp would compare.
bool same_tuning(const sbr_context* c, const sbr_tuning& t)
{
    sbr_tuning now;
    (void)sbr_context_get_tuning(c, &now);
    return now.trace_chunk == t.trace_chunk && now.persist_blocks == t.persist_blocks &&
           now.trace_block == t.trace_block && now.stack_depth == t.stack_depth &&
           now.lds_budget == t.lds_budget && now.rx_tree_min == t.rx_tree_min &&
           now.lookahead_max_paths == t.lookahead_max_paths &&
           now.lookahead_depth == t.lookahead_depth &&
           now.lookahead3_max_paths == t.lookahead3_max_paths &&
           now.grid_check_log2 == t.grid_check_log2 && now.ray_order == t.ray_order &&
           now.refine_segments == t.refine_segments;
}

bool graph_matches(const sbr_context* c, const sbr_scene* s, const double* rx, int32_t n_rx,
                   const sbr_trace_params* p, const sbr_path* out, int64_t capacity)
{
    const auto& G = c->graph;
    return G.valid && G.epoch == g_alloc_epoch && G.scene_id == s->id && G.rx == rx &&
           G.n_rx == n_rx && G.out == out && G.capacity == capacity &&
           memcmp(&G.params, p, sizeof(*p)) == 0 && same_tuning(c, G.tuning);
}

// Build the job of a call without launching anything (the launch grid
// already exists: the capturing call created it).
sbr_status graph_job(sbr_context* c, sbr_scene* s, const double* tx, int32_t n_rx,
                     const sbr_trace_params* p, Call& call)
{
    sbr_trace_params q = *p;
    q.flags &= ~(SBR_FLAG_FRESH_GRID | SBR_FLAG_GRAPH);
    call.scenes.push_back(s);
    call.rx = nullptr;
    call.n_rx = n_rx;
    call.rx_job.assign((size_t)n_rx, 0);
    call.chunk = c->trace_chunk;
    return add_job(c, call, 0, tx, 0, n_rx, &q, 0, num_rays(p->launch, p->division_n));
}

// Capture the whole pipeline of the call described by `call` (one job, no
// receiver tree) into c->graph.  Buffers are sized first: nothing is
// allocated while capturing.  u_cap bounds the paths a replay may hold;
// u_pred (the capturing call's path count) picks the refinement kernel, as
// for an eager call (every choice gives the same bytes).
sbr_status capture_graph(sbr_context* c, sbr_scene* s, Call& call, const double* rx_dev,
                         const sbr_trace_params* p, sbr_path* out, int64_t capacity,
                         int64_t u_cap, int64_t u_pred)
{
    c->up_epoch = 0;  // the graph writes the job, scene and receiver-job buffers
    auto& G = c->graph;
    const int32_t n_rx = call.n_rx;
    if (!G.cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&G.cap_stream, hipStreamNonBlocking));
    if (!G.h_job) HIPCHK(c, hipHostMalloc((void**)&G.h_job, sizeof(JobDev), 0));
    if (!G.h_scene) HIPCHK(c, hipHostMalloc((void**)&G.h_scene, sizeof(SceneDev), 0));
    if (G.h_rxjob_cap < std::max(n_rx, 1)) {
        if (G.h_rxjob) (void)hipHostFree(G.h_rxjob);
        G.h_rxjob = nullptr;
        G.h_rxjob_cap = 0;
        HIPCHK(c, hipHostMalloc((void**)&G.h_rxjob, sizeof(int32_t) * (size_t)std::max(n_rx, 1), 0));
        G.h_rxjob_cap = std::max(n_rx, 1);
    }
    *G.h_job = call.jobs[0];
    *G.h_scene = scene_dev(s);
    for (int32_t x = 0; x < n_rx; ++x) G.h_rxjob[x] = 0;
    const size_t U1 = (size_t)u_cap;
    HIPCHK(c, ensure(c->d_jobs, sizeof(JobDev)));
    HIPCHK(c, ensure(c->d_scenes, sizeof(SceneDev)));
    HIPCHK(c, ensure(c->rx, sizeof(double) * 3 * (size_t)std::max(n_rx, 1)));
    HIPCHK(c, ensure(c->rx32, sizeof(float4) * (size_t)std::max(n_rx, 1)));
    HIPCHK(c, ensure(c->d_rxjob, sizeof(int32_t) * (size_t)std::max(n_rx, 1)));
    HIPCHK(c, ensure(c->counters, sizeof(Counters)));
    HIPCHK(c, ensure(c->cand, sizeof(sbr_candidate) * (size_t)kSmallEvents));
    HIPCHK(c, ensure(c->uniq, sizeof(sbr_candidate) * (size_t)kSmallEvents));
    HIPCHK(c, ensure(c->refine, sizeof(RefineOut) * U1));
    HIPCHK(c, ensure(c->geom, sizeof(PathGeom) * U1));
    HIPCHK(c, ensure(c->paths, sizeof(sbr_path) * U1));
    HIPCHK(c, ensure(c->keep, sizeof(int32_t) * U1));
    GridDev g;
    bool built = false;
    sbr_status r = get_grid(c, p->launch, p->division_n, &g, &built);
    if (r) return r;
    if (p->flags & SBR_FLAG_FRESH_GRID) HIPCHK(c, ensure(c->grid_scratch, grid_scratch_bytes(p->division_n)));
    HIPCHK(c, hipStreamSynchronize(c->stream));

    call.dev.jobs = c->d_jobs.as<const JobDev>();
    call.dev.scenes = c->d_scenes.as<const SceneDev>();
    call.dev.rx = rx_dev;
    call.dev.rx32 = c->rx32.as<const float4>();
    call.dev.rx_job = c->d_rxjob.as<const int32_t>();
    call.dev.rx_nodes = nullptr;
    call.dev.rx_perm = nullptr;
    call.dev.n_jobs = 1;
    call.dev.chunk = call.chunk;
    call.dev.n_packets = call.n_packets;
    call.s0 = *G.h_scene;
    call.lp = plan_for(s, c->trace_block);
    LdsPlan lp256 = plan_for(s, 256);
    lp256.block = 256;
    Counters* dc = c->counters.as<Counters>();
    const hipStream_t st = G.cap_stream;
    // the graph holds the lookahead kernels (the queue is for batches)
    const int depth = std::max(1, refine_depth(c, u_pred));

    HIPCHK(c, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    auto step = [&](hipError_t x) {
        if (e == hipSuccess) e = x;
    };
    step(hipMemcpyAsync(c->d_jobs.p, G.h_job, sizeof(JobDev), hipMemcpyHostToDevice, st));
    step(hipMemcpyAsync(c->d_scenes.p, G.h_scene, sizeof(SceneDev), hipMemcpyHostToDevice, st));
    if (n_rx > 0)
        step(hipMemcpyAsync(c->d_rxjob.p, G.h_rxjob, sizeof(int32_t) * (size_t)n_rx,
                            hipMemcpyHostToDevice, st));
    // the receivers are read in place (a replay requires the same pointer)
    step(launch_rx32(rx_dev, n_rx, c->rx32.as<float4>(), st, c->counters.p, sizeof(Counters)));
    if (p->flags & SBR_FLAG_FRESH_GRID)
        step(launch_grid(g, st, c->grid_scratch.p, c->grid_check_log2));
    step(launch_trace(call.dev, call.lp, call.s0, trace_blocks(c, call), &dc->queue,
                      c->cand.as<sbr_candidate>(), kSmallEvents, &dc->cand, nullptr, nullptr,
                      &dc->err, st));
    step(launch_dedup_small(c->cand.as<sbr_candidate>(), kSmallEvents, c->uniq.as<sbr_candidate>(),
                            &dc->n_unique, st, &dc->cand));
    step(launch_refine(call.dev, lp256, plan_la3(s), call.s0, c->uniq.as<sbr_candidate>(), u_cap,
                       &dc->n_unique, depth, c->refine.as<RefineOut>(), c->geom.as<PathGeom>(),
                       &dc->err, st, max_iterations(call), c->seg_tail));
    step(launch_solve(call.dev, c->uniq.as<sbr_candidate>(), c->refine.as<RefineOut>(),
                      c->geom.as<PathGeom>(), u_cap, &dc->n_unique, c->paths.as<sbr_path>(),
                      c->keep.as<int32_t>(), &dc->err, st));
    step(launch_emit_small(c->paths.as<sbr_path>(), c->keep.as<int32_t>(), u_cap, &dc->n_unique,
                           out, capacity, &dc->n_paths, st));
    step(hipMemcpyAsync(c->host_ctr, c->counters.p, sizeof(Counters), hipMemcpyDeviceToHost, st));
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(st, &graph);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        G.exec = nullptr;
        return fail(c, SBR_E_DEVICE, "graph capture: %s", hipGetErrorString(e));
    }
    G.valid = true;
    G.epoch = g_alloc_epoch;
    G.scene_id = s->id;
    G.rx = rx_dev;
    G.n_rx = n_rx;
    G.out = out;
    G.capacity = capacity;
    G.u_cap = u_cap;
    G.n_rays = call.n_rays;
    G.params = *p;
    (void)sbr_context_get_tuning(c, &G.tuning);
    return SBR_OK;
}

// Replay the captured graph for transmitter tx.  Returns SBR_OK with
// *replayed false when the counts overflowed the captured sizes (the caller
// then runs the call normally).
sbr_status replay_graph(sbr_context* c, sbr_scene* s, const double* tx, int32_t n_rx,
                        const sbr_trace_params* p, int64_t capacity, int64_t* n_out,
                        sbr_trace_stats* stats, bool* replayed)
{
    c->up_epoch = 0;  // the graph writes the job, scene and receiver-job buffers
    auto& G = c->graph;
    *replayed = false;
    Call call;
    sbr_status r = graph_job(c, s, tx, n_rx, p, call);
    if (r) return r;
    *G.h_job = call.jobs[0];
    HIPCHK(c, hipEventRecord(c->ev[0], c->stream));
    HIPCHK(c, hipGraphLaunch(G.exec, c->stream));
    HIPCHK(c, hipEventRecord(c->ev[6], c->stream));
    HIPCHK(c, hipEventSynchronize(c->ev[6]));
    const Counters* hc = c->host_ctr;
    if (hc->err) return fail(c, SBR_E_INTERNAL, "traversal stack overflow");
    if (hc->cand > (unsigned long long)kSmallEvents || hc->n_unique > G.u_cap) {
        drop_graph(c);
        return SBR_OK;
    }
    *replayed = true;
    *n_out = hc->n_paths;
    if (stats) {
        memset(stats, 0, sizeof(*stats));
        stats->n_rays = G.n_rays;
        stats->n_candidates = (int64_t)hc->cand;
        stats->n_unique = hc->n_unique;
        stats->n_paths = hc->n_paths;
        float tot = 0;
        (void)hipEventElapsedTime(&tot, c->ev[0], c->ev[6]);
        stats->ms_total = tot;
        stats->lds_max = c->lds_max;
    }
    if (hc->n_paths > capacity)
        return fail(c, SBR_E_CAPACITY, "%d paths, capacity %lld", hc->n_paths,
                    (long long)capacity);
    return SBR_OK;
}

// ---------------------------------------------------------------------------
// Captured sbr_trace_batch calls: every job carries SBR_FLAG_GRAPH (and not
// SBR_FLAG_FRESH_GRID), no job is large enough for a receiver tree, and the
// capturing call ended with at most kSmallEvents reception events.  A later
// call with the same scenes, the same jobs apart from their transmitters and
// the same number of receivers replays the graph: the job table and the
// receivers go to pinned staging that the graph copies to the device; the
// paths land in a device buffer sized by the capture, of which the host
// copies the ones produced.  Counts beyond the captured sizes are detected
// from the counters and the call is redone normally.
// ---------------------------------------------------------------------------
// Pinned host buffer *p of at least n elements of `elem` bytes.
sbr_status grow_pinned(sbr_context* c, void** p, int64_t* cap, int64_t n, size_t elem)
{
    n = std::max<int64_t>(n, 1);
    if (*cap >= n) return SBR_OK;
    if (*p) (void)hipHostFree(*p);
    *p = nullptr;
    *cap = 0;
    HIPCHK(c, hipHostMalloc(p, elem * (size_t)n, 0));
    *cap = n;
    return SBR_OK;
}

// The call of a batch (job table, receiver-job map), launching nothing:
// every launch grid and ray order it names already exists or is made here.
sbr_status batch_call(sbr_context* c, sbr_scene* const* scenes, int32_t n_scenes,
                      const sbr_job* jobs, int32_t n_jobs, const double* rx, int32_t n_rx,
                      Call& call)
{
    for (int32_t i = 0; i < n_scenes; ++i) call.scenes.push_back(scenes[i]);
    call.rx = rx;
    call.n_rx = n_rx;
    call.rx_job.assign((size_t)n_rx, 0);
    call.chunk = c->trace_chunk;
    for (int32_t j = 0; j < n_jobs; ++j) {
        const sbr_job& J = jobs[j];
        const int64_t N = num_rays(J.params.launch, J.params.division_n);
        sbr_status r = add_job(c, call, J.scene, J.tx, J.rx_first, J.n_rx, &J.params, 0, N);
        if (r) return r;
    }
    return SBR_OK;
}

bool batch_wants_graph(const sbr_context* c, const sbr_job* jobs, int32_t n_jobs)
{
    if (n_jobs < 1) return false;
    for (int32_t j = 0; j < n_jobs; ++j) {
        const sbr_job& J = jobs[j];
        if (!(J.params.flags & SBR_FLAG_GRAPH) || (J.params.flags & SBR_FLAG_FRESH_GRID) ||
            (J.n_rx > 0 && J.n_rx >= c->rx_tree_min))
            return false;
    }
    return true;
}

bool bgraph_matches(const sbr_context* c, sbr_scene* const* scenes, int32_t n_scenes,
                    const sbr_job* jobs, int32_t n_jobs, int32_t n_rx)
{
    const auto& B = c->bgraph;
    if (!B.valid || B.epoch != g_alloc_epoch || (int32_t)B.scene_ids.size() != n_scenes ||
        (int32_t)B.jobs.size() != n_jobs || B.n_rx != n_rx || !same_tuning(c, B.tuning))
        return false;
    for (int32_t i = 0; i < n_scenes; ++i)
        if (scenes[i]->id != B.scene_ids[i]) return false;
    for (int32_t j = 0; j < n_jobs; ++j) {
        const sbr_job &a = jobs[j], &b = B.jobs[j];
        if (a.scene != b.scene || a.rx_first != b.rx_first || a.n_rx != b.n_rx ||
            memcmp(&a.params, &b.params, sizeof(a.params)) != 0)
            return false;
    }
    return true;
}

sbr_status capture_bgraph(sbr_context* c, Call& call, const sbr_job* jobs, int32_t n_jobs,
                          int64_t u_cap, int64_t u_pred)
{
    c->up_epoch = 0;  // the graph writes the job, scene and receiver-job buffers
    auto& B = c->bgraph;
    const int32_t n_rx = call.n_rx, nj = (int32_t)call.jobs.size();
    const int32_t ns = (int32_t)call.scenes.size();
    if (!B.cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&B.cap_stream, hipStreamNonBlocking));
    sbr_status r;
    if ((r = grow_pinned(c, (void**)&B.h_jobs, &B.jobs_cap, nj, sizeof(JobDev)))) return r;
    if ((r = grow_pinned(c, (void**)&B.h_scenes, &B.scenes_cap, ns, sizeof(SceneDev)))) return r;
    if ((r = grow_pinned(c, (void**)&B.h_rxjob, &B.rxjob_cap, n_rx, sizeof(int32_t)))) return r;
    if ((r = grow_pinned(c, (void**)&B.h_rx, &B.rx_cap, n_rx, 3 * sizeof(double)))) return r;
    for (int32_t j = 0; j < nj; ++j) B.h_jobs[j] = call.jobs[j];
    for (int32_t i = 0; i < ns; ++i) B.h_scenes[i] = scene_dev(call.scenes[i]);
    for (int32_t x = 0; x < n_rx; ++x) B.h_rxjob[x] = call.rx_job[x];
    if (n_rx > 0) memcpy(B.h_rx, call.rx, sizeof(double) * 3 * (size_t)n_rx);
    const size_t U1 = (size_t)u_cap;
    HIPCHK(c, ensure(c->d_jobs, sizeof(JobDev) * (size_t)std::max(nj, 1)));
    HIPCHK(c, ensure(c->d_scenes, sizeof(SceneDev) * (size_t)std::max(ns, 1)));
    HIPCHK(c, ensure(c->rx, sizeof(double) * 3 * (size_t)std::max(n_rx, 1)));
    HIPCHK(c, ensure(c->rx32, sizeof(float4) * (size_t)std::max(n_rx, 1)));
    HIPCHK(c, ensure(c->d_rxjob, sizeof(int32_t) * (size_t)std::max(n_rx, 1)));
    HIPCHK(c, ensure(c->counters, sizeof(Counters)));
    HIPCHK(c, ensure(c->cand, sizeof(sbr_candidate) * (size_t)kSmallEvents));
    HIPCHK(c, ensure(c->uniq, sizeof(sbr_candidate) * (size_t)kSmallEvents));
    HIPCHK(c, ensure(c->refine, sizeof(RefineOut) * U1));
    HIPCHK(c, ensure(c->geom, sizeof(PathGeom) * U1));
    HIPCHK(c, ensure(c->paths, sizeof(sbr_path) * U1));
    HIPCHK(c, ensure(c->keep, sizeof(int32_t) * U1));
    HIPCHK(c, ensure(c->dout, sizeof(sbr_path) * U1));
    HIPCHK(c, hipStreamSynchronize(c->stream));

    call.dev.jobs = c->d_jobs.as<const JobDev>();
    call.dev.scenes = c->d_scenes.as<const SceneDev>();
    call.dev.rx = c->rx.as<const double>();
    call.dev.rx32 = c->rx32.as<const float4>();
    call.dev.rx_job = c->d_rxjob.as<const int32_t>();
    call.dev.rx_nodes = nullptr;
    call.dev.rx_perm = nullptr;
    call.dev.n_jobs = nj;
    call.dev.chunk = call.chunk;
    call.dev.n_packets = call.n_packets;
    const bool one = ns == 1;
    call.s0 = scene_dev(call.scenes[0]);
    if (one) {
        call.lp = plan_for(call.scenes[0], c->trace_block);
    } else {
        call.lp = LdsPlan{};
        call.lp.block = 256;
    }
    LdsPlan lp256 = one ? plan_for(call.scenes[0], 256) : LdsPlan{};
    lp256.block = 256;
    const LdsPlan lp3 = one ? plan_la3(call.scenes[0]) : LdsPlan{};
    Counters* dc = c->counters.as<Counters>();
    const hipStream_t st = B.cap_stream;
    // the graph holds the lookahead kernels (the work queue allocates)
    const int depth = std::max(1, refine_depth(c, u_pred));

    HIPCHK(c, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    auto step = [&](hipError_t x) {
        if (e == hipSuccess) e = x;
    };
    step(hipMemcpyAsync(c->d_jobs.p, B.h_jobs, sizeof(JobDev) * (size_t)nj,
                        hipMemcpyHostToDevice, st));
    step(hipMemcpyAsync(c->d_scenes.p, B.h_scenes, sizeof(SceneDev) * (size_t)ns,
                        hipMemcpyHostToDevice, st));
    if (n_rx > 0) {
        step(hipMemcpyAsync(c->d_rxjob.p, B.h_rxjob, sizeof(int32_t) * (size_t)n_rx,
                            hipMemcpyHostToDevice, st));
        step(hipMemcpyAsync(c->rx.p, B.h_rx, sizeof(double) * 3 * (size_t)n_rx,
                            hipMemcpyHostToDevice, st));
    }
    step(launch_rx32(c->rx.as<const double>(), n_rx, c->rx32.as<float4>(), st, c->counters.p,
                     sizeof(Counters)));
    step(launch_trace(call.dev, call.lp, call.s0, trace_blocks(c, call), &dc->queue,
                      c->cand.as<sbr_candidate>(), kSmallEvents, &dc->cand, nullptr, nullptr,
                      &dc->err, st));
    step(launch_dedup_small(c->cand.as<sbr_candidate>(), kSmallEvents, c->uniq.as<sbr_candidate>(),
                            &dc->n_unique, st, &dc->cand));
    step(launch_refine(call.dev, lp256, lp3, call.s0, c->uniq.as<sbr_candidate>(), u_cap,
                       &dc->n_unique, depth, c->refine.as<RefineOut>(), c->geom.as<PathGeom>(),
                       &dc->err, st, max_iterations(call), c->seg_tail));
    step(launch_solve(call.dev, c->uniq.as<sbr_candidate>(), c->refine.as<RefineOut>(),
                      c->geom.as<PathGeom>(), u_cap, &dc->n_unique, c->paths.as<sbr_path>(),
                      c->keep.as<int32_t>(), &dc->err, st));
    step(launch_emit_small(c->paths.as<sbr_path>(), c->keep.as<int32_t>(), u_cap, &dc->n_unique,
                           c->dout.as<sbr_path>(), u_cap, &dc->n_paths, st));
    step(hipMemcpyAsync(c->host_ctr, c->counters.p, sizeof(Counters), hipMemcpyDeviceToHost, st));
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(st, &graph);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&B.exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        B.exec = nullptr;
        return fail(c, SBR_E_DEVICE, "batch graph capture: %s", hipGetErrorString(e));
    }
    B.valid = true;
    B.epoch = g_alloc_epoch;
    B.scene_ids.clear();
    for (const sbr_scene* sc : call.scenes) B.scene_ids.push_back(sc->id);
    B.jobs.assign(jobs, jobs + n_jobs);
    B.n_rx = n_rx;
    B.u_cap = u_cap;
    B.n_rays = call.n_rays;
    (void)sbr_context_get_tuning(c, &B.tuning);
    return SBR_OK;
}

// Replay for the job table and receivers of `call`.  *replayed false: the
// counts overflowed the captured sizes (the caller runs the call normally).
sbr_status replay_bgraph(sbr_context* c, const Call& call, sbr_path* out, int64_t capacity,
                         int64_t* n_out, sbr_trace_stats* stats, bool* replayed)
{
    c->up_epoch = 0;
    auto& B = c->bgraph;
    *replayed = false;
    if (B.epoch != g_alloc_epoch) {  // making the job table reallocated a buffer
        drop_bgraph(c);
        return SBR_OK;
    }
    for (size_t j = 0; j < call.jobs.size(); ++j) B.h_jobs[j] = call.jobs[j];
    if (call.n_rx > 0) memcpy(B.h_rx, call.rx, sizeof(double) * 3 * (size_t)call.n_rx);
    HIPCHK(c, hipEventRecord(c->ev[0], c->stream));
    HIPCHK(c, hipGraphLaunch(B.exec, c->stream));
    HIPCHK(c, hipEventRecord(c->ev[6], c->stream));
    HIPCHK(c, hipEventSynchronize(c->ev[6]));
    const Counters* hc = c->host_ctr;
    if (hc->err) return fail(c, SBR_E_INTERNAL, "traversal stack overflow");
    if (hc->cand > (unsigned long long)kSmallEvents || hc->n_unique > B.u_cap) {
        drop_bgraph(c);
        return SBR_OK;
    }
    *replayed = true;
    *n_out = hc->n_paths;
    if (stats) {
        memset(stats, 0, sizeof(*stats));
        stats->n_rays = B.n_rays;
        stats->n_candidates = (int64_t)hc->cand;
        stats->n_unique = hc->n_unique;
        stats->n_paths = hc->n_paths;
        float tot = 0;
        (void)hipEventElapsedTime(&tot, c->ev[0], c->ev[6]);
        stats->ms_total = tot;
        stats->lds_max = c->lds_max;
    }
    if (hc->n_paths > capacity)
        return fail(c, SBR_E_CAPACITY, "%d paths, capacity %lld", hc->n_paths,
                    (long long)capacity);
    if (hc->n_paths > 0)
        HIPCHK(c, hipMemcpy(out, c->dout.p, sizeof(sbr_path) * (size_t)hc->n_paths,
                            hipMemcpyDeviceToHost));
    return SBR_OK;
}

}  // namespace

sbr_status sbr_trace_device(sbr_scene* s, const double tx[3], const double* rx, int32_t n_rx,
                            const sbr_trace_params* p, sbr_path* out, int64_t capacity,
                            int64_t* n_out, sbr_trace_stats* stats)
{
    sbr_status r = check_trace_inputs(s, tx, nullptr, 0, p, capacity, out, n_out);
    if (r) return r;
    sbr_context* c = s->ctx;
    if (n_rx < 0 || (n_rx > 0 && !rx)) return fail(c, SBR_E_INVALID_ARG, "bad rx array");
    HIPCHK(c, use_device(c->device));
    const bool want_graph = (p->flags & SBR_FLAG_GRAPH) != 0 && n_rx < c->rx_tree_min;
    if (want_graph && graph_matches(c, s, rx, n_rx, p, out, capacity)) {
        bool replayed = false;
        r = replay_graph(c, s, tx, n_rx, p, capacity, n_out, stats, &replayed);
        if (r || replayed) return r;
    }
    // The receiver tree is built on the host: read the receivers back once
    // when the job is large enough to use it.
    std::vector<double> rx_host;
    if (n_rx > 0 && n_rx >= c->rx_tree_min) {
        rx_host.resize(3 * (size_t)n_rx);
        HIPCHK(c, hipMemcpyAsync(rx_host.data(), rx, sizeof(double) * rx_host.size(),
                                 hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    Call call;
    for (int attempt = 0;; ++attempt) {
        call = Call{};
        call.rx_dev = rx;
        r = single_call(s, call, tx, rx_host.empty() ? nullptr : rx_host.data(), n_rx, p, 0, -1);
        if (r) return r;
        r = run_front(c, call, true, nullptr, nullptr, nullptr, attempt == 0);
        if (r == SBR_OK) r = run_paths(c, call, out, capacity, n_out, stats, true);
        if (r == kGridStreamMiss && attempt < 3) continue;  // again, grid formed first
        if (r == kGridStreamMiss) return fail(c, SBR_E_INTERNAL, "%s", device_error(12));
        if (r != kSpecMiss) break;
        c->spec_events = -1;  // more events than predicted: again, reading the count
    }
    if (!r && call.small) {
        c->spec_events = call.n_cand;
        c->spec_unique = c->host_ctr->n_unique;
    } else if (!r) {
        c->spec_events = call.n_cand;
    }
    if (!r) note_grid_times(c, call, p);
    if (r || !want_graph || !call.small) return r;
    // capture for the next calls of this shape, with room for twice this
    // call's paths
    drop_graph(c);
    const int64_t u_now = c->host_ctr->n_unique;
    const int64_t u_cap = std::min<int64_t>(kSmallEvents, std::max<int64_t>(64, 2 * u_now));
    Call cap;
    r = graph_job(c, s, tx, n_rx, p, cap);
    if (r) return r;
    return capture_graph(c, s, cap, rx, p, out, capacity, u_cap, u_now);
}

}  // extern "C"

namespace {

// Where sbr_trace_device_noalloc keeps its buffers in the scratch (byte
// offsets, 256-aligned).  The counters and the receivers' job indices come
// first, so that one kernel zeroes both; the launch grid comes last, at an
// offset that depends only on n, so that the grid of the last call can be
// reused in place.
struct NoAllocLayout {
    size_t counters, rxjob, job, scene, rx32, cand, uniq, refine, geom, paths, keep, gscr, grid,
        end;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

NoAllocLayout noalloc_layout(int32_t n, int64_t N)
{
    NoAllocLayout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    L.counters = take(sizeof(Counters));
    L.rxjob = take(sizeof(int32_t) * kNoAllocMaxRx);
    L.job = take(sizeof(JobDev));
    L.scene = take(sizeof(SceneDev));
    L.rx32 = take(sizeof(float4) * kNoAllocMaxRx);
    L.cand = take(sizeof(sbr_candidate) * kSmallEvents);
    L.uniq = take(sizeof(sbr_candidate) * kSmallEvents);
    L.refine = take(sizeof(RefineOut) * kSmallEvents);
    L.geom = take(sizeof(PathGeom) * kSmallEvents);
    L.paths = take(sizeof(sbr_path) * kSmallEvents);
    L.keep = take(sizeof(int32_t) * kSmallEvents);
    L.gscr = take(grid_scratch_bytes(n));
    L.grid = take(sizeof(double) * 3 * (size_t)N);
    L.end = o;
    return L;
}

}  // namespace

extern "C" {

sbr_status sbr_trace_device_noalloc(sbr_scene* s, const double tx[3], const double* rx,
                                    int32_t n_rx, const sbr_trace_params* p, sbr_path* out,
                                    int64_t capacity, int64_t* n_out, sbr_trace_stats* stats)
{
    sbr_status r = check_trace_inputs(s, tx, nullptr, 0, p, capacity, out, n_out);
    if (r) return r;
    sbr_context* c = s->ctx;
    if (n_rx < 0 || (n_rx > 0 && !rx)) return fail(c, SBR_E_INVALID_ARG, "bad rx array");
    if (p->flags & SBR_FLAG_GRAPH)
        return fail(c, SBR_E_INVALID_ARG, "SBR_FLAG_GRAPH needs allocation; capture the call instead");
    if (!c->scratch)
        return fail(c, SBR_E_DEVICE, "no-allocation scratch unavailable: %s",
                    hipGetErrorString(c->scratch_err));
    if (n_rx > kNoAllocMaxRx)
        return fail(c, SBR_E_SCRATCH, "%d receivers; the no-allocation scratch holds at most %d",
                    n_rx, kNoAllocMaxRx);
    const int64_t N = num_rays(p->launch, p->division_n);
    const NoAllocLayout L = noalloc_layout(p->division_n, N);
    if (L.end > kNoAllocBytes)
        return fail(c, SBR_E_SCRATCH,
                    "%lld launch rays need %zu bytes of scratch; the no-allocation scratch has %zu",
                    (long long)N, L.end, kNoAllocBytes);
    HIPCHK(c, use_device(c->device));
    const hipStream_t st = c->stream;
    char* base = (char*)c->scratch;
    double* dir = (double*)(base + L.grid);
    JobDev J = make_job(s, tx, p, dir, N, 0, N);
    J.n_rx = n_rx;
    const SceneDev S0 = scene_dev(s);
    Counters* dc = (Counters*)(base + L.counters);
    sbr_candidate* cand = (sbr_candidate*)(base + L.cand);
    sbr_candidate* uniq = (sbr_candidate*)(base + L.uniq);
    RefineOut* rf = (RefineOut*)(base + L.refine);
    PathGeom* geom = (PathGeom*)(base + L.geom);
    sbr_path* paths = (sbr_path*)(base + L.paths);
    int32_t* keep = (int32_t*)(base + L.keep);

    HIPCHK(c, hipEventRecord(c->ev[0], st));
    HIPCHK(c, hipMemcpyAsync(base + L.job, &J, sizeof J, hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(base + L.scene, &S0, sizeof S0, hipMemcpyHostToDevice, st));
    // FP32 receivers; the counters and the receivers' job (all 0) zeroed
    HIPCHK(c, launch_rx32(rx, n_rx, (float4*)(base + L.rx32), st, base,
                          L.rxjob + sizeof(int32_t) * (size_t)n_rx));
    const int32_t dev = c->device;
    const int32_t key = p->launch * 100000 + p->division_n;
    const bool grid_fresh = (p->flags & SBR_FLAG_FRESH_GRID) || g_scratch_grid[dev] != key;
    g_scratch_grid[dev] = -1;  // until this call has completed
    if (grid_fresh)
        HIPCHK(c, launch_grid(GridDev{dir, N, p->division_n, p->launch}, st, base + L.gscr,
                              c->grid_check_log2));
    HIPCHK(c, hipEventRecord(c->ev[1], st));

    CallDev D{};
    D.jobs = (const JobDev*)(base + L.job);
    D.scenes = (const SceneDev*)(base + L.scene);
    D.rx = rx;
    D.rx_job = (const int32_t*)(base + L.rxjob);
    D.rx_nodes = nullptr;
    D.rx_perm = nullptr;
    D.rx32 = (const float4*)(base + L.rx32);
    D.n_jobs = 1;
    D.chunk = c->trace_chunk;
    const int64_t per = 64 * (int64_t)D.chunk;
    D.n_packets = (N + per - 1) / per;
    const LdsPlan lp = plan_for(s, c->trace_block);
    const int64_t per_block = std::max<int64_t>(1, lp.block / 64);
    const int blocks = (int)std::max<int64_t>(
        1, std::min<int64_t>((D.n_packets + per_block - 1) / per_block, c->persist_blocks));
    HIPCHK(c, hipEventRecord(c->ev[7], st));
    HIPCHK(c, launch_trace(D, lp, S0, blocks, &dc->queue, cand, kSmallEvents, &dc->cand, nullptr,
                           nullptr, &dc->err, st));
    HIPCHK(c, hipEventRecord(c->ev[2], st));
    HIPCHK(c, launch_dedup_small(cand, kSmallEvents, uniq, &dc->n_unique, st, &dc->cand));
    HIPCHK(c, hipEventRecord(c->ev[3], st));
    LdsPlan lp256 = plan_for(s, 256);
    lp256.block = 256;
    const int depth = std::max(1, refine_depth(c, c->noalloc_unique >= 0 ? c->noalloc_unique : 256));
    HIPCHK(c, launch_refine(D, lp256, plan_la3(s), S0, uniq, kSmallEvents, &dc->n_unique, depth,
                            rf, geom, &dc->err, st, p->iterations, c->seg_tail));
    HIPCHK(c, hipEventRecord(c->ev[4], st));
    HIPCHK(c, launch_solve(D, uniq, rf, geom, kSmallEvents, &dc->n_unique, paths, keep,
                           &dc->err, st));
    HIPCHK(c, hipEventRecord(c->ev[5], st));
    HIPCHK(c, launch_emit_small(paths, keep, kSmallEvents, &dc->n_unique, out, capacity,
                                &dc->n_paths, st));
    HIPCHK(c, hipMemcpyAsync(c->host_ctr, dc, sizeof(Counters), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipEventRecord(c->ev[6], st));
    HIPCHK(c, hipEventSynchronize(c->ev[6]));
    const Counters* hc = c->host_ctr;
    if (hc->err) return fail(c, SBR_E_INTERNAL, "traversal stack overflow");
    g_scratch_grid[dev] = key;
    if (hc->cand > (unsigned long long)kSmallEvents)
        return fail(c, SBR_E_SCRATCH,
                    "%llu reception events; the no-allocation scratch holds at most %d",
                    hc->cand, kSmallEvents);
    c->noalloc_unique = hc->n_unique;
    *n_out = hc->n_paths;
    if (stats) {
        memset(stats, 0, sizeof(*stats));
        stats->n_rays = N;
        stats->n_candidates = (int64_t)hc->cand;
        stats->n_unique = hc->n_unique;
        stats->n_paths = hc->n_paths;
        float t[7] = {};
        (void)hipEventElapsedTime(&t[0], c->ev[0], c->ev[1]);
        (void)hipEventElapsedTime(&t[1], c->ev[7], c->ev[2]);
        (void)hipEventElapsedTime(&t[2], c->ev[2], c->ev[3]);
        (void)hipEventElapsedTime(&t[3], c->ev[3], c->ev[4]);
        (void)hipEventElapsedTime(&t[4], c->ev[4], c->ev[5]);
        (void)hipEventElapsedTime(&t[5], c->ev[5], c->ev[6]);
        (void)hipEventElapsedTime(&t[6], c->ev[0], c->ev[6]);
        stats->ms_launch = grid_fresh ? t[0] : 0.0;
        stats->ms_trace = t[1];
        stats->ms_dedup = t[2];
        stats->ms_refine = t[3];
        stats->ms_solve = t[4];
        stats->ms_emit = t[5];
        stats->ms_total = t[6];
        stats->lds_bytes = lp.bytes;
        stats->lds_nodes = lp.n_nodes;
        stats->lds_tris = lp.n_tris;
        stats->lds_max = c->lds_max;
    }
    if (hc->n_paths > capacity)
        return fail(c, SBR_E_CAPACITY, "%d paths, capacity %lld", hc->n_paths, (long long)capacity);
    return SBR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Order-1 diffraction
// ---------------------------------------------------------------------------
namespace {

sbr_status ensure_wedges(sbr_scene* s)
{
    sbr_context* c = s->ctx;
    if (s->has_wedges) return SBR_OK;
    build_wedges(s->tri_v.data(), s->face.data(), s->T, s->fplane.data(), s->wedges, s->wedge_b);
    if (!s->wedges.empty()) {
        HIPCHK(c, ensure(s->d_wedges, sizeof(WedgeDev) * s->wedges.size()));
        HIPCHK(c, hipMemcpy(s->d_wedges.p, s->wedges.data(), sizeof(WedgeDev) * s->wedges.size(),
                            hipMemcpyHostToDevice));
    }
    s->has_wedges = true;
    return SBR_OK;
}

// Launch grid, unfolded receivers and the SBR diffraction of every launch
// ray: the events are left in c->cand (count in *n_cand), A describes the
// call for the later stages.
sbr_status diff_front(sbr_scene* s, const double* tx, const double* rx, int32_t n_rx,
                      const sbr_trace_params* p, DiffArgs* A, int64_t* n_cand, float* ms_launch,
                      float* ms_trace)
{
    sbr_context* c = s->ctx;
    const hipStream_t st = c->stream;
    sbr_status r = ensure_wedges(s);
    if (r) return r;
    HIPCHK(c, hipEventRecord(c->ev[0], st));
    GridDev g;
    bool built = false;
    r = get_grid(c, p->launch, p->division_n, &g, &built, (p->flags & SBR_FLAG_FRESH_GRID) != 0);
    if (r) return r;
    HIPCHK(c, hipEventRecord(c->ev[1], st));
    const int32_t n_w = (int32_t)s->wedges.size();
    HIPCHK(c, ensure(c->rx, sizeof(double) * 3 * (size_t)std::max(n_rx, 1)));
    HIPCHK(c, ensure(c->d_rxp, sizeof(double4) * (size_t)std::max<int64_t>((int64_t)n_w * n_rx, 1)));
    HIPCHK(c, ensure(c->counters, sizeof(Counters)));
    if (n_rx > 0)
        HIPCHK(c, hipMemcpyAsync(c->rx.p, rx, sizeof(double) * 3 * (size_t)n_rx,
                                 hipMemcpyHostToDevice, st));
    *A = DiffArgs{};
    A->dir = g.dir;
    A->N = g.N;
    for (int i = 0; i < 3; ++i) A->tx[i] = tx[i];
    A->thl = theta_launch(p->launch, p->division_n);
    A->tan_tgt = p->target_err_deg > 0.0 ? tan_cr((p->target_err_deg * kPi) / 180.0) : 0.0;
    A->delta = traversal_delta(s, tx);
    A->iterations = p->iterations;
    A->subrays = p->subrays;
    A->keep_invalid = (p->flags & SBR_FLAG_KEEP_INVALID) ? 1 : 0;
    A->w = s->d_wedges.as<const WedgeDev>();
    A->n_w = n_w;
    A->rx = c->rx.as<const double>();
    A->n_rx = n_rx;
    A->rxp = c->d_rxp.as<double4>();
    HIPCHK(c, launch_diff_unfold(*A, st));
    Counters* hc = c->host_ctr;
    Counters* dc = c->counters.as<Counters>();
    int64_t cap = std::max<int64_t>(65536, (int64_t)(c->cand.cap / sizeof(sbr_candidate)));
    for (;;) {
        HIPCHK(c, ensure(c->cand, sizeof(sbr_candidate) * (size_t)cap));
        HIPCHK(c, launch_zero(c->counters.p, sizeof(Counters), st));
        HIPCHK(c, hipEventRecord(c->ev[7], st));
        if (n_w > 0 && n_rx > 0)
            HIPCHK(c, launch_diff_trace(scene_dev(s), *A, c->cand.as<sbr_candidate>(), cap,
                                        &dc->cand, &dc->err, st));
        HIPCHK(c, hipEventRecord(c->ev[2], st));
        HIPCHK(c, hipMemcpyAsync(hc, c->counters.p, sizeof(Counters), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        if (hc->err) return fail(c, SBR_E_INTERNAL, "traversal stack overflow");
        if ((int64_t)hc->cand <= cap) break;
        if (hc->cand >= (1ull << 31))
            return fail(c, SBR_E_CAPACITY, "%llu diffraction events exceed 2^31", hc->cand);
        cap = (int64_t)(hc->cand + hc->cand / 4 + 1024);
    }
    *n_cand = (int64_t)hc->cand;
    HIPCHK(c, hipEventElapsedTime(ms_launch, c->ev[0], c->ev[1]));
    if (!built) *ms_launch = 0.0f;
    HIPCHK(c, hipEventElapsedTime(ms_trace, c->ev[7], c->ev[2]));
    return SBR_OK;
}

}  // namespace

extern "C" {

sbr_status sbr_scene_wedges(sbr_scene* s, sbr_wedge* out, int64_t capacity, int64_t* n_out)
{
    if (!s || !s->ctx) return SBR_E_NO_SCENE;
    sbr_context* c = s->ctx;
    c->err.clear();
    if (!n_out) return fail(c, SBR_E_INVALID_ARG, "n_out is NULL");
    *n_out = 0;
    if (capacity < 0 || (capacity > 0 && !out)) return fail(c, SBR_E_INVALID_ARG, "bad output array");
    HIPCHK(c, use_device(c->device));
    sbr_status r = ensure_wedges(s);
    if (r) return r;
    const int64_t n = (int64_t)s->wedges.size();
    *n_out = n;
    if (n > capacity)
        return fail(c, SBR_E_CAPACITY, "%lld wedges, capacity %lld", (long long)n, (long long)capacity);
    for (int64_t i = 0; i < n; ++i) {
        for (int q = 0; q < 3; ++q) {
            out[i].a[q] = s->wedges[(size_t)i].a[q];
            out[i].b[q] = s->wedge_b[3 * (size_t)i + q];
        }
        out[i].face[0] = s->wedges[(size_t)i].f0;
        out[i].face[1] = s->wedges[(size_t)i].f1;
    }
    return SBR_OK;
}

sbr_status sbr_diff_candidates(sbr_scene* s, const double tx[3], const double* rx, int32_t n_rx,
                               const sbr_trace_params* p, sbr_candidate* out, int64_t capacity,
                               int64_t* n_out)
{
    sbr_status r = check_trace_inputs(s, tx, rx, n_rx, p, capacity, out, n_out);
    if (r) return r;
    sbr_context* c = s->ctx;
    HIPCHK(c, use_device(c->device));
    DiffArgs A;
    int64_t C = 0;
    float ml = 0, mt = 0;
    r = diff_front(s, tx, rx, n_rx, p, &A, &C, &ml, &mt);
    if (r) return r;
    *n_out = C;
    if (C > capacity)
        return fail(c, SBR_E_CAPACITY, "%lld events, capacity %lld", (long long)C, (long long)capacity);
    if (C == 0) return SBR_OK;
    HIPCHK(c, ensure(c->idx, sizeof(uint32_t) * (size_t)pow2_at_least(C)));
    HIPCHK(c, launch_sort_candidates(c->cand.as<sbr_candidate>(), C, c->idx.as<uint32_t>(),
                                     c->stream));
    HIPCHK(c, ensure(c->uniq, sizeof(sbr_candidate) * (size_t)C));
    HIPCHK(c, launch_gather_sorted(c->cand.as<sbr_candidate>(), c->idx.as<uint32_t>(), C,
                                   c->uniq.as<sbr_candidate>(), c->stream));
    HIPCHK(c, hipMemcpyAsync(out, c->uniq.p, sizeof(sbr_candidate) * (size_t)C,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SBR_OK;
}

sbr_status sbr_diffract(sbr_scene* s, const double tx[3], const double* rx, int32_t n_rx,
                        const sbr_trace_params* p, sbr_diff_path* out, int64_t capacity,
                        int64_t* n_out, sbr_trace_stats* stats)
{
    sbr_status r = check_trace_inputs(s, tx, rx, n_rx, p, capacity, out, n_out);
    if (r) return r;
    sbr_context* c = s->ctx;
    HIPCHK(c, use_device(c->device));
    const hipStream_t st = c->stream;
    DiffArgs A;
    int64_t C = 0;
    float ms_launch = 0, ms_trace = 0;
    r = diff_front(s, tx, rx, n_rx, p, &A, &C, &ms_launch, &ms_trace);
    if (r) return r;
    Counters* hc = c->host_ctr;
    Counters* dc = c->counters.as<Counters>();
    const SceneDev S = scene_dev(s);
    // path test 1: one path per (receiver, wedge)
    int64_t U = 0;
    if (C > 0) {
        if (C <= kSmallEvents) {
            HIPCHK(c, ensure(c->uniq, sizeof(sbr_candidate) * (size_t)C));
            HIPCHK(c, launch_dedup_small(c->cand.as<sbr_candidate>(), C,
                                         c->uniq.as<sbr_candidate>(), &dc->n_unique, st));
        } else {
            HIPCHK(c, ensure(c->idx, sizeof(uint32_t) * (size_t)pow2_at_least(C)));
            HIPCHK(c, launch_sort_candidates(c->cand.as<sbr_candidate>(), C,
                                             c->idx.as<uint32_t>(), st));
            HIPCHK(c, ensure(c->flags, sizeof(int32_t) * (size_t)C));
            HIPCHK(c, ensure(c->offs, sizeof(int32_t) * (size_t)C));
            HIPCHK(c, ensure(c->scan, scan_scratch_bytes(C)));
            HIPCHK(c, launch_heads(c->cand.as<sbr_candidate>(), c->idx.as<uint32_t>(), C,
                                   c->flags.as<int32_t>(), st));
            HIPCHK(c, launch_scan(c->flags.as<int32_t>(), c->offs.as<int32_t>(), C,
                                  &dc->n_unique, c->scan.p, st));
            HIPCHK(c, ensure(c->uniq, sizeof(sbr_candidate) * (size_t)C));
            HIPCHK(c, launch_gather_unique(c->cand.as<sbr_candidate>(), c->idx.as<uint32_t>(),
                                           c->flags.as<int32_t>(), c->offs.as<int32_t>(), C,
                                           c->uniq.as<sbr_candidate>(), st));
        }
        HIPCHK(c, hipMemcpyAsync(hc, c->counters.p, sizeof(Counters), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        U = hc->n_unique;
    }
    HIPCHK(c, hipEventRecord(c->ev[3], st));
    const size_t U1 = (size_t)std::max<int64_t>(U, 1);
    HIPCHK(c, ensure(c->refine, sizeof(RefineOut) * U1));
    HIPCHK(c, ensure(c->dpaths, sizeof(sbr_diff_path) * U1));
    HIPCHK(c, ensure(c->keep, sizeof(int32_t) * U1));
    HIPCHK(c, ensure(c->offs, sizeof(int32_t) * U1));
    HIPCHK(c, ensure(c->scan, scan_scratch_bytes(U)));
    HIPCHK(c, launch_diff_refine(S, A, c->uniq.as<sbr_candidate>(), U, c->refine.as<RefineOut>(),
                                 &dc->err, st));
    HIPCHK(c, hipEventRecord(c->ev[4], st));
    HIPCHK(c, launch_diff_solve(S, A, c->uniq.as<sbr_candidate>(), c->refine.as<RefineOut>(), U,
                                c->dpaths.as<sbr_diff_path>(), c->keep.as<int32_t>(), &dc->err,
                                st));
    HIPCHK(c, hipEventRecord(c->ev[5], st));
    int64_t P = 0;
    if (U > 0) {
        HIPCHK(c, launch_scan(c->keep.as<int32_t>(), c->offs.as<int32_t>(), U, &dc->n_paths,
                              c->scan.p, st));
        HIPCHK(c, hipMemcpyAsync(hc, c->counters.p, sizeof(Counters), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        if (hc->err) return fail(c, SBR_E_INTERNAL, "traversal stack overflow");
        P = hc->n_paths;
    }
    *n_out = P;
    if (P > capacity)
        return fail(c, SBR_E_CAPACITY, "%lld paths, capacity %lld", (long long)P, (long long)capacity);
    if (P > 0) {
        HIPCHK(c, ensure(c->dout, sizeof(sbr_diff_path) * (size_t)P));
        HIPCHK(c, launch_compact_dpaths(c->dpaths.as<sbr_diff_path>(), c->keep.as<int32_t>(),
                                        c->offs.as<int32_t>(), U, c->dout.as<sbr_diff_path>(), st));
        HIPCHK(c, hipMemcpyAsync(out, c->dout.p, sizeof(sbr_diff_path) * (size_t)P,
                                 hipMemcpyDeviceToHost, st));
    }
    HIPCHK(c, hipEventRecord(c->ev[6], st));
    HIPCHK(c, hipEventSynchronize(c->ev[6]));
    if (stats) {
        memset(stats, 0, sizeof(*stats));
        stats->n_rays = A.N;
        stats->n_candidates = C;
        stats->n_unique = U;
        stats->n_paths = P;
        float dd = 0, a = 0, b = 0, e = 0, tot = 0;
        (void)hipEventElapsedTime(&dd, c->ev[2], c->ev[3]);
        (void)hipEventElapsedTime(&a, c->ev[3], c->ev[4]);
        (void)hipEventElapsedTime(&b, c->ev[4], c->ev[5]);
        (void)hipEventElapsedTime(&e, c->ev[5], c->ev[6]);
        (void)hipEventElapsedTime(&tot, c->ev[0], c->ev[6]);
        stats->ms_launch = ms_launch;
        stats->ms_trace = ms_trace;
        stats->ms_dedup = dd;
        stats->ms_refine = a;
        stats->ms_solve = b;
        stats->ms_emit = e;
        stats->ms_total = tot;
        stats->lds_max = c->lds_max;
    }
    return SBR_OK;
}

sbr_status sbr_trace_batch(sbr_context* c, sbr_scene* const* scenes, int32_t n_scenes,
                           const sbr_job* jobs, int32_t n_jobs, const double* rx,
                           int32_t n_rx_total, sbr_path* out, int64_t capacity, int64_t* n_out,
                           sbr_trace_stats* stats)
{
    if (!c) return SBR_E_INVALID_ARG;
    c->err.clear();
    if (!n_out) return fail(c, SBR_E_INVALID_ARG, "n_out is NULL");
    *n_out = 0;
    if (n_scenes < 1 || !scenes || n_jobs < 0 || (n_jobs > 0 && !jobs) || n_rx_total < 0 ||
        (n_rx_total > 0 && !rx) || capacity < 0 || (capacity > 0 && !out))
        return fail(c, SBR_E_INVALID_ARG, "bad batch arrays or sizes");
    for (int32_t i = 0; i < n_scenes; ++i) {
        if (!scenes[i] || scenes[i]->ctx != c)
            return fail(c, SBR_E_NO_SCENE, "scene %d missing or from another context", i);
        if (!scenes[i]->has_bvh) return fail(c, SBR_E_NO_BVH, "scene %d has no BVH", i);
    }
    for (int32_t x = 0; x < n_rx_total; ++x)
        if (!finite3(rx + 3 * x)) return fail(c, SBR_E_INVALID_ARG, "rx %d not finite", x);
    std::vector<char> used((size_t)n_rx_total, 0);
    for (int32_t j = 0; j < n_jobs; ++j) {
        const sbr_job& J = jobs[j];
        if (J.scene < 0 || J.scene >= n_scenes || J.reserved != 0 || J.n_rx < 0 ||
            J.rx_first < 0 || (int64_t)J.rx_first + J.n_rx > n_rx_total || !finite3(J.tx))
            return fail(c, SBR_E_INVALID_ARG, "job %d: bad scene, receivers or tx", j);
        for (int32_t x = 0; x < J.n_rx; ++x) {
            if (used[J.rx_first + x])
                return fail(c, SBR_E_INVALID_ARG, "receiver %d belongs to two jobs", J.rx_first + x);
            used[J.rx_first + x] = 1;
        }
        sbr_status r = check_params(c, &J.params);
        if (r) return r;
    }
    HIPCHK(c, use_device(c->device));
    const bool want_graph = batch_wants_graph(c, jobs, n_jobs);
    if (want_graph && bgraph_matches(c, scenes, n_scenes, jobs, n_jobs, n_rx_total)) {
        Call rc;
        sbr_status r = batch_call(c, scenes, n_scenes, jobs, n_jobs, rx, n_rx_total, rc);
        if (r) return r;
        bool replayed = false;
        r = replay_bgraph(c, rc, out, capacity, n_out, stats, &replayed);
        if (r || replayed) return r;
    }
    Call call;
    HIPCHK(c, hipEventRecord(c->ev[0], c->stream));
    sbr_status r = batch_call(c, scenes, n_scenes, jobs, n_jobs, rx, n_rx_total, call);
    if (r) return r;
    r = run_front(c, call, true, nullptr, nullptr, nullptr);
    if (r) return r;
    r = run_paths(c, call, out, capacity, n_out, stats);
    if (r || !want_graph || !call.small) return r;
    // capture for the next calls of this shape, with room for twice this
    // call's paths
    drop_bgraph(c);
    const int64_t u_now = c->host_ctr->n_unique;
    const int64_t u_cap = std::min<int64_t>(kSmallEvents, std::max<int64_t>(64, 2 * u_now));
    Call cap;
    r = batch_call(c, scenes, n_scenes, jobs, n_jobs, rx, n_rx_total, cap);
    if (r) return r;
    return capture_bgraph(c, cap, jobs, n_jobs, u_cap, u_now);
}

sbr_status sbr_path_gradients(sbr_scene* s, int64_t n_paths, const double* tx, const double* rx,
                              const int32_t* order, const int32_t* faces, const double* eps,
                              double freq_hz, double tx_power_dbm, const double* upstream,
                              double* values, double* grad_tx, double* grad_rx, double* grad_eps)
{
    sbr_status r = check_scene(s);
    if (r) return r;
    sbr_context* c = s->ctx;
    c->err.clear();
    if (n_paths < 0) return fail(c, SBR_E_INVALID_ARG, "n_paths < 0");
    if (!(freq_hz > 0.0) || !isfinite(freq_hz) || !isfinite(tx_power_dbm))
        return fail(c, SBR_E_INVALID_ARG, "freq_hz / tx_power_dbm out of range");
    if (n_paths > 0 && (!tx || !rx || !order || !faces || !eps))
        return fail(c, SBR_E_INVALID_ARG, "NULL input array");
    if (upstream && (!grad_tx || !grad_rx || !grad_eps))
        return fail(c, SBR_E_INVALID_ARG, "upstream gradients given but no gradient outputs");
    if (n_paths == 0) return SBR_OK;
    HIPCHK(c, use_device(c->device));
    GradArgs A;
    A.tx = tx;
    A.rx = rx;
    A.order = order;
    A.faces = faces;
    A.eps = eps;
    A.up = upstream;
    A.val = values;
    A.gtx = grad_tx;
    A.grx = grad_rx;
    A.geps = grad_eps;
    A.P = n_paths;
    A.freq_hz = freq_hz;
    A.tx_power_dbm = tx_power_dbm;
    HIPCHK(c, launch_path_grad(scene_dev(s), A, c->stream));
    return SBR_OK;
}

}  // extern "C"
