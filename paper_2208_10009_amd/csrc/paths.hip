// paths.hip -- canonical order of reception events, path test 1 (Sec.
// III.A: one path per receiver and face sequence, the smaller error angle
// wins) and the stable compaction of the final path list.
#include <math.h>

#include "geom.h"
#include "internal.h"

namespace sbr {

// ===========================================================================
// Canonical order of reception events and path test 1
// ===========================================================================
// Key (rx, order, face sequence); ties by smaller error angle, then lower
// launch ray (the double-counting test keeps the smaller error angle).
__device__ static inline int key_cmp(const sbr_candidate& a, const sbr_candidate& b)
{
    if (a.rx != b.rx) return a.rx < b.rx ? -1 : 1;
    if (a.order != b.order) return a.order < b.order ? -1 : 1;
#pragma unroll
    for (int j = 0; j < SBR_MAX_ORDER; ++j)
        if (a.face[j] != b.face[j]) return a.face[j] < b.face[j] ? -1 : 1;
    return 0;
}

__device__ static inline bool cand_less(const sbr_candidate* __restrict__ C, uint32_t ia,
                                        uint32_t ib)
{
    if (ia == 0xffffffffu) return false;
    if (ib == 0xffffffffu) return true;
    const sbr_candidate a = C[ia], b = C[ib];
    int c = key_cmp(a, b);
    if (c) return c < 0;
    if (a.tan_err != b.tan_err) return a.tan_err < b.tan_err;
    return a.ray < b.ray;
}

__global__ void k_iota(uint32_t* idx, int64_t n, int64_t P)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P) idx[i] = i < n ? (uint32_t)i : 0xffffffffu;
}

// One global compare-exchange pass of the bitonic network (stride j, stage k).
__global__ void k_bitonic_global(const sbr_candidate* __restrict__ C, uint32_t* idx, int64_t P,
                                 int64_t j, int64_t k)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    int64_t l = i ^ j;
    if (l <= i) return;
    bool asc = (i & k) == 0;
    uint32_t a = idx[i], b = idx[l];
    bool swap = asc ? cand_less(C, b, a) : cand_less(C, a, b);
    if (swap) {
        idx[i] = b;
        idx[l] = a;
    }
}

// All passes of stage k with stride j <= 512 inside one 1024-element tile in
// LDS.  With first_stage set, it runs every stage k = 2..1024 of the tile.
__global__ __launch_bounds__(512) void k_bitonic_local(const sbr_candidate* __restrict__ C,
                                                       uint32_t* idx, int64_t P, int64_t k,
                                                       int first_stage)
{
    __shared__ uint32_t s[1024];
    int64_t base = (int64_t)blockIdx.x * 1024;
    int t = threadIdx.x;
    s[t] = idx[base + t];
    s[t + 512] = idx[base + t + 512];
    __syncthreads();
    int64_t k_lo = first_stage ? 2 : k, k_hi = first_stage ? 1024 : k;
    for (int64_t kk = k_lo; kk <= k_hi; kk <<= 1) {
        for (int64_t j = (first_stage ? kk : 1024) >> 1; j > 0; j >>= 1) {
            if (!first_stage && j > 512) continue;
            int i = 2 * t - (t & (int)(j - 1));  // lower element of the pair
            int l = i + (int)j;
            bool asc = ((base + i) & kk) == 0;
            uint32_t a = s[i], b = s[l];
            bool swap = asc ? cand_less(C, b, a) : cand_less(C, a, b);
            if (swap) {
                s[i] = b;
                s[l] = a;
            }
            __syncthreads();
        }
    }
    idx[base + t] = s[t];
    idx[base + t + 512] = s[t + 512];
}

int64_t pow2_at_least(int64_t n)
{
    int64_t p = 1024;
    while (p < n) p <<= 1;
    return p;
}

hipError_t launch_sort_candidates(const sbr_candidate* C, int64_t n, uint32_t* idx,
                                  hipStream_t s)
{
    int64_t P = pow2_at_least(n);
    hipLaunchKernelGGL(k_iota, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, idx, n, P);
    if (n <= 1) return hipGetLastError();
    unsigned tiles = (unsigned)(P / 1024);
    hipLaunchKernelGGL(k_bitonic_local, dim3(tiles), dim3(512), 0, s, C, idx, P, (int64_t)0, 1);
    for (int64_t k = 2048; k <= P; k <<= 1) {
        for (int64_t j = k >> 1; j > 512; j >>= 1)
            hipLaunchKernelGGL(k_bitonic_global, dim3((unsigned)((P + 255) / 256)), dim3(256), 0,
                               s, C, idx, P, j, k);
        hipLaunchKernelGGL(k_bitonic_local, dim3(tiles), dim3(512), 0, s, C, idx, P, k, 0);
    }
    return hipGetLastError();
}

__global__ void k_heads(const sbr_candidate* __restrict__ C, const uint32_t* __restrict__ idx,
                        int64_t n, int32_t* __restrict__ flags)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    flags[i] = (i == 0 || key_cmp(C[idx[i]], C[idx[i - 1]]) != 0) ? 1 : 0;
}

hipError_t launch_heads(const sbr_candidate* C, const uint32_t* idx, int64_t n, int32_t* flags,
                        hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_heads, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, C, idx, n,
                       flags);
    return hipGetLastError();
}

// ---- exclusive scan (tiles of 1024 = 256 threads x 4) ---------------------
__global__ __launch_bounds__(256) void k_scan_tile(const int32_t* __restrict__ in,
                                                   int32_t* __restrict__ out, int64_t n,
                                                   int32_t* __restrict__ tile_sum)
{
    __shared__ int32_t s[256];
    int64_t base = (int64_t)blockIdx.x * 1024 + 4 * threadIdx.x;
    int32_t v[4];
    int32_t acc = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        v[q] = base + q < n ? in[base + q] : 0;
        acc += v[q];
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        int32_t add_v = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += add_v;
        __syncthreads();
    }
    int32_t run = s[threadIdx.x] - acc;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (base + q < n) out[base + q] = run;
        run += v[q];
    }
    if (threadIdx.x == 255) tile_sum[blockIdx.x] = s[255];
}

__global__ void k_scan_add(int32_t* __restrict__ out, int64_t n, const int32_t* __restrict__ add_v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += add_v[i / 1024];
}

__global__ void k_scan_total(const int32_t* in, const int32_t* out, int64_t n, int32_t* total)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *total = n > 0 ? out[n - 1] + in[n - 1] : 0;
}

size_t scan_scratch_bytes(int64_t n)
{
    size_t b = 0;
    int64_t m = n;
    do {
        m = (m + 1023) / 1024;
        b += 2 * sizeof(int32_t) * (size_t)(m + 1);
    } while (m > 1);
    return b + 256;
}

static hipError_t scan_rec(const int32_t* in, int32_t* out, int64_t n, int32_t* scratch,
                           hipStream_t s)
{
    int64_t tiles = (n + 1023) / 1024;
    int32_t* sums = scratch;
    int32_t* sums_scan = scratch + tiles + 1;
    hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)tiles), dim3(256), 0, s, in, out, n, sums);
    if (tiles > 1) {
        (void)scan_rec(sums, sums_scan, tiles, scratch + 2 * (tiles + 1), s);
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n,
                           sums_scan);
    }
    return hipGetLastError();
}

hipError_t launch_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* total, void* scratch,
                       hipStream_t s)
{
    if (n > 0) (void)scan_rec(in, out, n, (int32_t*)scratch, s);
    hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(64), 0, s, in, out, n, total);
    return hipGetLastError();
}

__global__ void k_gather_unique(const sbr_candidate* __restrict__ C,
                                const uint32_t* __restrict__ idx,
                                const int32_t* __restrict__ flags,
                                const int32_t* __restrict__ offs, int64_t n,
                                sbr_candidate* __restrict__ U)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flags[i]) return;
    U[offs[i]] = C[idx[i]];
}

hipError_t launch_gather_unique(const sbr_candidate* C, const uint32_t* idx, const int32_t* flags,
                                const int32_t* offs, int64_t n, sbr_candidate* U, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_unique, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, C,
                       idx, flags, offs, n, U);
    return hipGetLastError();
}

__global__ void k_gather_sorted(const sbr_candidate* __restrict__ C,
                                const uint32_t* __restrict__ idx, int64_t n,
                                sbr_candidate* __restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = C[idx[i]];
}

hipError_t launch_gather_sorted(const sbr_candidate* C, const uint32_t* idx, int64_t n,
                                sbr_candidate* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_sorted, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, C,
                       idx, n, out);
    return hipGetLastError();
}

__global__ void k_compact_paths(const sbr_path* __restrict__ paths,
                                const int32_t* __restrict__ keep,
                                const int32_t* __restrict__ offs, int64_t U,
                                sbr_path* __restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < U && keep[i]) out[offs[i]] = paths[i];
}

hipError_t launch_compact_paths(const sbr_path* paths, const int32_t* keep, const int32_t* offs,
                                int64_t U, sbr_path* out, hipStream_t s)
{
    if (U <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_compact_paths, dim3((unsigned)((U + 255) / 256)), dim3(256), 0, s, paths,
                       keep, offs, U, out);
    return hipGetLastError();
}

}  // namespace sbr

namespace sbr {

// ===========================================================================
// Single-workgroup variants for up to kSmallEvents events: one launch each,
// no host round trip in between (the counts stay on the device).
// ===========================================================================
// Threads of the one-workgroup path test 1 and the events each handles in
// the scan (256 threads measured slower: the head tests then run 16 deep).
constexpr int kDedupThreads = 1024;
constexpr int kDedupPer = kSmallEvents / kDedupThreads;
static_assert(kDedupPer <= 32, "head bits of one thread must fit a 32-bit mask");

// Bitonic sort of the index list idx[0..P) of the n events in C (P = the
// power of two >= n; empty slots hold 0xffffffff and sort last).
__device__ static void bitonic_block(const sbr_candidate* C, uint32_t* idx, int P)
{
    const int t = threadIdx.x;
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int q = t; q < P / 2; q += kDedupThreads) {
                int i = 2 * q - (q & (j - 1));
                int l = i + j;
                bool asc = (i & k) == 0;
                uint32_t a = idx[i], b = idx[l];
                bool swap = asc ? cand_less(C, b, a) : cand_less(C, a, b);
                if (swap) {
                    idx[i] = b;
                    idx[l] = a;
                }
            }
            __syncthreads();
        }
    }
}

// The sort key of an event as 16 unsigned words whose lexicographic order is
// the canonical order (rx, order, face sequence, then the smaller error
// angle, then the lower ray): signed fields are offset by 2^31, tan_err >= 0
// and ray >= 0 compare as their bit patterns; the last two words are zero.
__device__ static inline void pack_key(const sbr_candidate& c, uint4* K)
{
    const uint32_t o = 0x80000000u;
    const unsigned long long tb = (unsigned long long)__double_as_longlong(c.tan_err);
    const unsigned long long rb = (unsigned long long)c.ray;
    K[0] = make_uint4((uint32_t)c.rx ^ o, (uint32_t)c.order ^ o, (uint32_t)c.face[0] ^ o,
                      (uint32_t)c.face[1] ^ o);
    K[1] = make_uint4((uint32_t)c.face[2] ^ o, (uint32_t)c.face[3] ^ o, (uint32_t)c.face[4] ^ o,
                      (uint32_t)c.face[5] ^ o);
    K[2] = make_uint4((uint32_t)c.face[6] ^ o, (uint32_t)c.face[7] ^ o, (uint32_t)(tb >> 32),
                      (uint32_t)tb);
    K[3] = make_uint4((uint32_t)(rb >> 32), (uint32_t)rb, 0u, 0u);
}

__device__ static inline void unpack16(const uint4* K, uint32_t* w)
{
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint4 v = K[q];
        w[4 * q] = v.x;
        w[4 * q + 1] = v.y;
        w[4 * q + 2] = v.z;
        w[4 * q + 3] = v.w;
    }
}

// Is the key of event ia before that of ib (empty slots last)?  Compares
// words 0..nw-1, branch-free from the last word up.
__device__ static inline bool key_less16(const uint4* K, uint32_t ia, uint32_t ib, int nw)
{
    if (ia == 0xffffffffu) return false;
    if (ib == 0xffffffffu) return true;
    uint32_t a[16], b[16];
    unpack16(K + 4 * (size_t)ia, a);
    unpack16(K + 4 * (size_t)ib, b);
    // (less, equal) per word, merged pairwise in a tree: the first word
    // decides unless equal, then the second
    bool lt[16], eq[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        lt[q] = q < nw && a[q] < b[q];
        eq[q] = q >= nw || a[q] == b[q];
    }
#pragma unroll
    for (int w = 1; w < 16; w <<= 1)
#pragma unroll
        for (int q = 0; q + w < 16; q += 2 * w) {
            lt[q] = lt[q] || (eq[q] && lt[q + w]);
            eq[q] = eq[q] && eq[q + w];
        }
    return lt[0];
}

// Events staged in LDS (as packed keys) for the sort when there are at most
// this many.
constexpr int kDedupLds = 2048;

// Sort (bitonic, in LDS), path test 1 (heads of equal keys) and compaction of
// the winners, in sorted order; writes the number of unique paths to
// *n_unique.  Up to kDedupLds events are first packed into LDS keys, so that
// each comparison is four LDS reads and a branch-free word compare.  With a
// device count n_dev above n_max (more events than the call was sized for,
// a result every caller discards) there are no winners: the later stages
// then do no work and write no paths.
__global__ __launch_bounds__(kDedupThreads) void k_dedup_small(const sbr_candidate* __restrict__ C,
                                                      int32_t n_max,
                                                      const unsigned long long* __restrict__ n_dev,
                                                      sbr_candidate* __restrict__ U,
                                                      int32_t* __restrict__ n_unique)
{
    __shared__ uint32_t idx[kSmallEvents];
    __shared__ int32_t part[kDedupThreads];
    __shared__ uint4 sK[4 * kDedupLds];
    const int t = threadIdx.x;
    const int n = n_dev ? (*n_dev > (unsigned long long)n_max ? 0 : (int)*n_dev) : n_max;
    int P = 1;
    while (P < n) P <<= 1;
    for (int i = t; i < P; i += kDedupThreads) idx[i] = i < n ? (uint32_t)i : 0xffffffffu;
    const bool staged = n <= kDedupLds;  // uniform over the workgroup
    if (staged)
        for (int i = t; i < n; i += kDedupThreads) pack_key(C[i], sK + 4 * i);
    __syncthreads();
    if (staged) {
        for (int k = 2; k <= P; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int q = t; q < P / 2; q += kDedupThreads) {
                    int i = 2 * q - (q & (j - 1));
                    int l = i + j;
                    bool asc = (i & k) == 0;
                    uint32_t a = idx[i], b = idx[l];
                    // keys are distinct (one event per ray, order and
                    // receiver), so b < a is !(a < b) but for two empty
                    // slots, whose swap changes nothing
                    const bool ab = key_less16(sK, a, b, 14);
                    bool swap = asc ? !ab : ab;
                    if (swap) {
                        idx[i] = b;
                        idx[l] = a;
                    }
                }
                __syncthreads();
            }
        }
    } else {
        bitonic_block(C, idx, P);
    }
    uint32_t hm = 0;  // bit q: event kDedupPer t + q heads its key
#pragma unroll
    for (int q = 0; q < kDedupPer; ++q) {
        int i = kDedupPer * t + q;
        bool head = false;
        if (i < n) {
            if (i == 0)
                head = true;
            else if (staged)  // keys differ in (rx, order, face sequence): words 0..9
                head = key_less16(sK, idx[i - 1], idx[i], 10);
            else
                head = key_cmp(C[idx[i]], C[idx[i - 1]]) != 0;
        }
        hm |= head ? 1u << q : 0u;
    }
    const int sum = __popc(hm);
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < kDedupThreads; off <<= 1) {
        int v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - sum;
    for (int q = 0; q < kDedupPer; ++q)
        if (hm >> q & 1u) U[run++] = C[idx[kDedupPer * t + q]];
    if (t == kDedupThreads - 1) *n_unique = part[kDedupThreads - 1];
}

hipError_t launch_dedup_small(const sbr_candidate* C, int64_t n, sbr_candidate* U,
                              int32_t* n_unique, hipStream_t s, const unsigned long long* n_dev)
{
    hipLaunchKernelGGL(k_dedup_small, dim3(1), dim3(kDedupThreads), 0, s, C, (int32_t)n, n_dev, U,
                       n_unique);
    return hipGetLastError();
}

// Stable compaction of the kept paths (path test 2) of the first
// min(U_max, *n_dev) records; writes the count to *n_paths, and the records
// to out only when they fit in its capacity.
__global__ __launch_bounds__(1024) void k_emit_small(const sbr_path* __restrict__ paths,
                                                     const int32_t* __restrict__ keep,
                                                     int32_t U_max, const int32_t* __restrict__ n_dev,
                                                     sbr_path* __restrict__ out, int64_t capacity,
                                                     int32_t* __restrict__ n_paths)
{
    __shared__ int32_t part[1024];
    const int t = threadIdx.x;
    const int U = min(U_max, *n_dev);
    int h[4], sum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int i = 4 * t + q;
        h[q] = (i < U && keep[i]) ? 1 : 0;
        sum += h[q];
    }
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - sum;
    if ((int64_t)part[1023] <= capacity) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (h[q]) out[run++] = paths[4 * t + q];
    }
    if (t == 1023) *n_paths = part[1023];
}

hipError_t launch_emit_small(const sbr_path* paths, const int32_t* keep, int64_t U_max,
                             const int32_t* n_dev, sbr_path* out, int64_t capacity,
                             int32_t* n_paths, hipStream_t s)
{
    hipLaunchKernelGGL(k_emit_small, dim3(1), dim3(1024), 0, s, paths, keep, (int32_t)U_max, n_dev,
                       out, capacity, n_paths);
    return hipGetLastError();
}

// Zero n 32-bit words (a kernel, so that it can sit in a captured graph).
__global__ void k_zero(uint32_t* __restrict__ p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s)
{
    const int64_t n = (int64_t)(bytes / 4);
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (uint32_t*)p, n);
    return hipGetLastError();
}

}  // namespace sbr
