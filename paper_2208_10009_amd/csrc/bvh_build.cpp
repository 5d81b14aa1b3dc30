// bvh_build.cpp -- host-side binned-SAH BVH2 builder, collapsed to a BVH4.
//
// The paper leaves the acceleration of SBR open (Sec. I mentions acceleration
// work only); this BVH is the build's own choice.  Boxes are computed in FP64
// and rounded outward to FP32, so each FP32 box contains its triangles
// exactly; the traversal adds a per-call margin on top (see the trace kernel)
// so that no triangle the FP64 test would hit is ever culled.
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "internal.h"

namespace sbr {
namespace {

struct Box {
    double lo[3], hi[3];
    void reset()
    {
        for (int i = 0; i < 3; ++i) {
            lo[i] = INFINITY;
            hi[i] = -INFINITY;
        }
    }
    void grow(const double* p)
    {
        for (int i = 0; i < 3; ++i) {
            lo[i] = std::min(lo[i], p[i]);
            hi[i] = std::max(hi[i], p[i]);
        }
    }
    void grow(const Box& b)
    {
        for (int i = 0; i < 3; ++i) {
            lo[i] = std::min(lo[i], b.lo[i]);
            hi[i] = std::max(hi[i], b.hi[i]);
        }
    }
    double area() const
    {
        if (!(hi[0] >= lo[0])) return 0.0;
        double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
        return 2.0 * (dx * dy + dy * dz + dz * dx);
    }
};

float round_down(double x)
{
    float f = (float)x;
    if ((double)f > x) f = nextafterf(f, -INFINITY);
    return f;
}
float round_up(double x)
{
    float f = (float)x;
    if ((double)f < x) f = nextafterf(f, INFINITY);
    return f;
}

struct Builder {
    const double* tv;
    std::vector<Box> tb;       // per-triangle box
    std::vector<double> cen;   // per-triangle centroid [3]
    std::vector<int32_t> idx;  // working permutation
    std::vector<BvhNode> nodes;
    int max_leaf, bins, depth_reached = 0;

    struct Ref {
        int32_t index, count;  // count > 0 leaf, 0 inner, < 0 empty
        Box box;
    };

    Box range_box(int32_t b, int32_t e) const
    {
        Box r;
        r.reset();
        for (int32_t i = b; i < e; ++i) r.grow(tb[idx[i]]);
        return r;
    }

    // Split [b, e): returns the split position, or -1 for "make a leaf".
    int32_t split(int32_t b, int32_t e, const Box& bx, int depth)
    {
        int32_t n = e - b;
        if (n <= 1) return -1;
        Box cb;
        cb.reset();
        for (int32_t i = b; i < e; ++i) cb.grow(&cen[3 * idx[i]]);
        double best_cost = INFINITY;
        int best_axis = -1, best_bin = -1;
        std::vector<Box> bb(bins);
        std::vector<int32_t> bc(bins);
        std::vector<double> right_area(bins);
        std::vector<int32_t> right_count(bins);
        for (int ax = 0; ax < 3; ++ax) {
            double ext = cb.hi[ax] - cb.lo[ax];
            if (!(ext > 0.0)) continue;
            for (int k = 0; k < bins; ++k) {
                bb[k].reset();
                bc[k] = 0;
            }
            for (int32_t i = b; i < e; ++i) {
                int t = idx[i];
                int k = (int)((cen[3 * t + ax] - cb.lo[ax]) / ext * bins);
                k = std::min(std::max(k, 0), bins - 1);
                bb[k].grow(tb[t]);
                bc[k] += 1;
            }
            Box acc;
            acc.reset();
            int32_t cnt = 0;
            for (int k = bins - 1; k >= 1; --k) {
                acc.grow(bb[k]);
                cnt += bc[k];
                right_area[k] = acc.area();
                right_count[k] = cnt;
            }
            acc.reset();
            cnt = 0;
            for (int k = 0; k < bins - 1; ++k) {
                acc.grow(bb[k]);
                cnt += bc[k];
                if (cnt == 0 || right_count[k + 1] == 0) continue;
                double c = acc.area() * cnt + right_area[k + 1] * right_count[k + 1];
                if (c < best_cost) {
                    best_cost = c;
                    best_axis = ax;
                    best_bin = k;
                }
            }
        }
        double pa = bx.area();
        double leaf_cost = (double)n;
        double split_cost = pa > 0.0 ? 1.0 + best_cost / pa : INFINITY;
        bool must_split = n > max_leaf;
        if (depth >= kMaxBvhDepth - 1) return -1;
        if (best_axis < 0) {
            // all centroids coincide: split by count if the leaf is too big
            if (!must_split) return -1;
            return b + n / 2;
        }
        if (!must_split && split_cost >= leaf_cost) return -1;
        double ext = cb.hi[best_axis] - cb.lo[best_axis];
        int32_t* first = idx.data() + b;
        int32_t* last = idx.data() + e;
        int32_t* mid = std::partition(first, last, [&](int32_t t) {
            int k = (int)((cen[3 * t + best_axis] - cb.lo[best_axis]) / ext * bins);
            k = std::min(std::max(k, 0), bins - 1);
            return k <= best_bin;
        });
        int32_t m = (int32_t)(mid - idx.data());
        if (m == b || m == e) m = b + n / 2;
        return m;
    }

    // Build the subtree of [b, e) and return its reference.
    Ref build(int32_t b, int32_t e, int depth)
    {
        depth_reached = std::max(depth_reached, depth);
        Ref r;
        r.box = range_box(b, e);
        int32_t m = split(b, e, r.box, depth);
        if (m < 0) {
            r.index = b;
            r.count = e - b;
            return r;
        }
        int32_t me = (int32_t)nodes.size();
        nodes.push_back(BvhNode{});
        Ref L = build(b, m, depth + 1);
        Ref R = build(m, e, depth + 1);
        emit(me, L, R);
        r.index = me;
        r.count = 0;
        return r;
    }

    void emit(int32_t at, const Ref& L, const Ref& R)
    {
        BvhNode& nd = nodes[at];
        const Ref* c[2] = {&L, &R};
        float lo[2][3], hi[2][3];
        for (int s = 0; s < 2; ++s)
            for (int i = 0; i < 3; ++i) {
                if (c[s]->count < 0) {
                    lo[s][i] = 0.0f;
                    hi[s][i] = 0.0f;
                } else {
                    lo[s][i] = round_down(c[s]->box.lo[i]);
                    hi[s][i] = round_up(c[s]->box.hi[i]);
                }
            }
        nd.a[0] = lo[0][0]; nd.a[1] = lo[0][1]; nd.a[2] = lo[0][2]; nd.a[3] = hi[0][0];
        nd.b[0] = hi[0][1]; nd.b[1] = hi[0][2]; nd.b[2] = lo[1][0]; nd.b[3] = lo[1][1];
        nd.c[0] = lo[1][2]; nd.c[1] = hi[1][0]; nd.c[2] = hi[1][1]; nd.c[3] = hi[1][2];
        nd.m[0] = L.index;
        nd.m[1] = R.index;
        nd.m[2] = L.count < 0 ? -1 : L.count;
        nd.m[3] = R.count < 0 ? -1 : R.count;
    }
};

}  // namespace

namespace {

// One child slot of a BVH4 node under construction.
struct Slot {
    float lo[3], hi[3];
    int32_t index, count;
    double area() const
    {
        double dx = (double)hi[0] - lo[0], dy = (double)hi[1] - lo[1], dz = (double)hi[2] - lo[2];
        return 2.0 * (dx * dy + dy * dz + dz * dx);
    }
};

void bvh2_children(const BvhNode& nd, Slot* s)
{
    s[0] = Slot{{nd.a[0], nd.a[1], nd.a[2]}, {nd.a[3], nd.b[0], nd.b[1]}, nd.m[0], nd.m[2]};
    s[1] = Slot{{nd.b[2], nd.b[3], nd.c[0]}, {nd.c[1], nd.c[2], nd.c[3]}, nd.m[1], nd.m[3]};
}

// Collapse the BVH2 subtree at n2 into a BVH4 node (depth-first preorder):
// start from n2's two children and open the inner child of largest surface
// area until there are four children or only leaves.  Returns the depth.
int collapse(const std::vector<BvhNode>& n2, int32_t r, std::vector<Bvh4Node>& n4, int32_t at)
{
    Slot s[4];
    int ns = 2;
    bvh2_children(n2[r], s);
    while (ns < 4) {
        int best = -1;
        for (int k = 0; k < ns; ++k)
            if (s[k].count == 0 && (best < 0 || s[k].area() > s[best].area())) best = k;
        if (best < 0) break;
        Slot two[2];
        bvh2_children(n2[s[best].index], two);
        s[best] = two[0];
        s[ns++] = two[1];
    }
    int depth = 1;
    for (int k = 0; k < ns; ++k)
        if (s[k].count == 0) {
            const int32_t child = (int32_t)n4.size();
            n4.push_back(Bvh4Node{});
            depth = std::max(depth, 1 + collapse(n2, s[k].index, n4, child));
            s[k].index = child;
        }
    Bvh4Node& nd = n4[at];
    for (int k = 0; k < 4; ++k) {
        const bool used = k < ns && s[k].count >= 0;
        nd.lox[k] = used ? s[k].lo[0] : 0.0f;
        nd.loy[k] = used ? s[k].lo[1] : 0.0f;
        nd.loz[k] = used ? s[k].lo[2] : 0.0f;
        nd.hix[k] = used ? s[k].hi[0] : 0.0f;
        nd.hiy[k] = used ? s[k].hi[1] : 0.0f;
        nd.hiz[k] = used ? s[k].hi[2] : 0.0f;
        nd.idx[k] = used ? s[k].index : 0;
        nd.cnt[k] = used ? s[k].count : -1;
    }
    return depth;
}

}  // namespace

int build_bvh(const double* tri_v, int64_t T, int max_leaf, int bins, bool bfs,
              std::vector<Bvh4Node>& nodes, std::vector<int32_t>& perm)
{
    Builder B;
    B.tv = tri_v;
    B.max_leaf = max_leaf;
    B.bins = bins;
    B.tb.resize((size_t)T);
    B.cen.resize((size_t)T * 3);
    B.idx.resize((size_t)T);
    for (int64_t t = 0; t < T; ++t) {
        B.tb[t].reset();
        for (int v = 0; v < 3; ++v) B.tb[t].grow(tri_v + 9 * t + 3 * v);
        for (int i = 0; i < 3; ++i)
            B.cen[3 * t + i] = (tri_v[9 * t + i] + tri_v[9 * t + 3 + i] + tri_v[9 * t + 6 + i]) / 3.0;
        B.idx[t] = (int32_t)t;
    }
    // The root is always an inner node so that traversal starts uniformly.
    B.nodes.push_back(BvhNode{});
    Builder::Ref L, R;
    if (T == 0) {
        L.index = 0; L.count = -1; L.box.reset();
        R = L;
    } else {
        Box all = B.range_box(0, (int32_t)T);
        int32_t m = B.split(0, (int32_t)T, all, 0);
        if (m < 0) {
            L.index = 0;
            L.count = (int32_t)T;
            L.box = all;
            R.index = 0;
            R.count = -1;
            R.box.reset();
        } else {
            L = B.build(0, m, 1);
            R = B.build(m, (int32_t)T, 1);
        }
    }
    B.emit(0, L, R);
    // BVH4 in depth-first preorder: the first child usually follows its
    // parent in memory
    std::vector<Bvh4Node> n4;
    n4.push_back(Bvh4Node{});
    const int depth = collapse(B.nodes, 0, n4, 0);
    perm.swap(B.idx);
    if (!bfs) {
        nodes.swap(n4);
        return depth;
    }
    // Renumber breadth-first, so that the top levels of the tree form a
    // prefix of the node array (the part staged in LDS).
    const size_t NN = n4.size();
    std::vector<int32_t> order;
    order.reserve(NN);
    std::vector<int32_t> new_id(NN, -1);
    order.push_back(0);
    new_id[0] = 0;
    for (size_t q = 0; q < order.size(); ++q) {
        const Bvh4Node& nd = n4[order[q]];
        for (int k = 0; k < 4; ++k) {
            if (nd.cnt[k] != 0) continue;  // leaf or empty child
            new_id[nd.idx[k]] = (int32_t)order.size();
            order.push_back(nd.idx[k]);
        }
    }
    nodes.resize(order.size());
    for (size_t q = 0; q < order.size(); ++q) {
        Bvh4Node nd = n4[order[q]];
        for (int k = 0; k < 4; ++k)
            if (nd.cnt[k] == 0) nd.idx[k] = new_id[nd.idx[k]];
        nodes[q] = nd;
    }
    return depth;
}

}  // namespace sbr
