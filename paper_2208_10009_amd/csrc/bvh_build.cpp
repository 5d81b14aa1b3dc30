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
#include <queue>
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

// ---------------------------------------------------------------------------
// Reference splitting.  A triangle whose box is large next to the scene's
// typical triangle enters the hierarchy as several references, each with the
// box of the part of the triangle inside one cell of a recursive midpoint
// subdivision of its box (largest boxes first, until the budget of extra
// references is spent or every box is below twice the median triangle box
// area).  Every reference names the same triangle record, so traversal
// results do not change; only which nodes a ray visits does.
// Conservativeness: a cell's part of the triangle is clipped (Sutherland-
// Hodgman) against the cell enlarged by pad = 1e-12 (max |vertex coordinate|
// + 1) on every side, and its box is widened by pad again.  Vertex
// classification against a plane is exact; a crossing point has the plane's
// coordinate exactly and the others within a few ulps (far below pad), so
// every point of the exact triangle inside the exact cell lies in the padded
// box.  The boxes are then rounded outward to FP32 like any other.
struct P3 {
    double x[3];
};

void clip_plane(const std::vector<P3>& in, int ax, double m, bool keep_le, std::vector<P3>& out)
{
    out.clear();
    const size_t n = in.size();
    for (size_t i = 0; i < n; ++i) {
        const P3& P = in[i];
        const P3& Q = in[(i + 1) % n];
        const bool inP = keep_le ? P.x[ax] <= m : P.x[ax] >= m;
        const bool inQ = keep_le ? Q.x[ax] <= m : Q.x[ax] >= m;
        if (inP) out.push_back(P);
        if (inP != inQ) {
            const double t = (m - P.x[ax]) / (Q.x[ax] - P.x[ax]);
            P3 X;
            for (int k = 0; k < 3; ++k) X.x[k] = P.x[k] + t * (Q.x[k] - P.x[k]);
            X.x[ax] = m;
            out.push_back(X);
        }
    }
}

// Box of triangle t's part inside cell (false: the triangle misses the cell).
bool clipped_box(const double* V, const Box& tbox, const Box& cell, Box* out)
{
    double mx = 0.0;
    for (int k = 0; k < 9; ++k) mx = std::max(mx, fabs(V[k]));
    const double pad = 1e-12 * (mx + 1.0);
    std::vector<P3> a(3), b;
    for (int v = 0; v < 3; ++v)
        for (int k = 0; k < 3; ++k) a[v].x[k] = V[3 * v + k];
    for (int ax = 0; ax < 3 && !a.empty(); ++ax) {
        clip_plane(a, ax, cell.lo[ax] - pad, false, b);
        clip_plane(b, ax, cell.hi[ax] + pad, true, a);
    }
    if (a.empty()) return false;
    Box r;
    r.reset();
    for (const P3& p : a) r.grow(p.x);
    for (int k = 0; k < 3; ++k) {
        r.lo[k] = std::max(r.lo[k] - pad, tbox.lo[k]);
        r.hi[k] = std::min(r.hi[k] + pad, tbox.hi[k]);
    }
    *out = r;
    return true;
}

struct SplitRef {
    int32_t tri;
    Box cell, box;
    int depth;
};

// References of all triangles: rtri[r] (the triangle), rbox[r] (its box),
// rsplit[r] (whether the box is a clipped part).  Unsplit triangles keep
// their own box.
void make_refs(const double* tri_v, int64_t T, const std::vector<Box>& tb, int split_pct,
               std::vector<int32_t>& rtri, std::vector<Box>& rbox, std::vector<char>& rsplit)
{
    std::vector<SplitRef> refs((size_t)T);
    std::vector<double> areas((size_t)T);
    for (int64_t t = 0; t < T; ++t) {
        refs[t] = SplitRef{(int32_t)t, tb[t], tb[t], 0};
        areas[t] = tb[t].area();
    }
    const int64_t budget = split_pct > 0 ? T * (int64_t)split_pct / 100 : 0;
    if (budget > 0 && T > 0) {
        std::vector<double> sorted = areas;
        std::nth_element(sorted.begin(), sorted.begin() + T / 2, sorted.end());
        const double thresh = 2.0 * sorted[T / 2];
        typedef std::pair<double, int32_t> Item;
        std::priority_queue<Item> heap;
        for (int64_t t = 0; t < T; ++t)
            if (areas[t] > thresh) heap.push(Item(areas[t], (int32_t)t));
        int64_t extra = 0;
        while (!heap.empty() && extra < budget) {
            const int32_t r = heap.top().second;
            heap.pop();
            SplitRef& R = refs[r];
            const Box bx = R.box;
            int ax = 0;
            for (int k = 1; k < 3; ++k)
                if (bx.hi[k] - bx.lo[k] > bx.hi[ax] - bx.lo[ax]) ax = k;
            const double m = 0.5 * (bx.lo[ax] + bx.hi[ax]);
            if (!(m > bx.lo[ax] && m < bx.hi[ax]) || R.depth >= 24) continue;
            Box cl = R.cell, cr = R.cell;
            cl.hi[ax] = m;
            cr.lo[ax] = m;
            const double* V = tri_v + 9 * (size_t)R.tri;
            Box bl, br;
            const bool hl = clipped_box(V, tb[R.tri], cl, &bl);
            const bool hr = clipped_box(V, tb[R.tri], cr, &br);
            if (hl && hr) {
                const SplitRef right{R.tri, cr, br, R.depth + 1};
                R.cell = cl;
                R.box = bl;
                R.depth += 1;
                refs.push_back(right);
                extra += 1;
                const int32_t nr = (int32_t)refs.size() - 1;
                if (refs[r].box.area() > thresh) heap.push(Item(refs[r].box.area(), r));
                if (refs[nr].box.area() > thresh) heap.push(Item(refs[nr].box.area(), nr));
            } else if (hl || hr) {
                // the triangle lies in one half: a tighter cell, same reference
                R.cell = hl ? cl : cr;
                const Box nb = hl ? bl : br;
                const bool shrank = nb.area() < R.box.area();
                R.box = nb;
                R.depth += 1;
                if (shrank && R.box.area() > thresh) heap.push(Item(R.box.area(), r));
            }
        }
    }
    rtri.resize(refs.size());
    rbox.resize(refs.size());
    rsplit.resize(refs.size());
    for (size_t r = 0; r < refs.size(); ++r) {
        rtri[r] = refs[r].tri;
        rbox[r] = refs[r].box;
        rsplit[r] = refs[r].depth > 0;
    }
}

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
        // an empty slot gets the inverted box (lo = +inf, hi = -inf): its
        // entry parameter is +inf and its exit -inf on every axis, whatever
        // the sign of the direction, so no ray enters it
        const bool used = k < ns && s[k].count >= 0;
        nd.lox[k] = used ? s[k].lo[0] : INFINITY;
        nd.loy[k] = used ? s[k].lo[1] : INFINITY;
        nd.loz[k] = used ? s[k].lo[2] : INFINITY;
        nd.hix[k] = used ? s[k].hi[0] : -INFINITY;
        nd.hiy[k] = used ? s[k].hi[1] : -INFINITY;
        nd.hiz[k] = used ? s[k].hi[2] : -INFINITY;
        nd.idx[k] = used ? s[k].index : 0;
        nd.cnt[k] = used ? s[k].count : -1;
    }
    return depth;
}

}  // namespace

int build_bvh(const double* tri_v, int64_t T0, int max_leaf, int bins, int split_pct, bool bfs,
              std::vector<Bvh4Node>& nodes, std::vector<int32_t>& perm)
{
    Builder B;
    B.tv = tri_v;
    B.max_leaf = max_leaf;
    B.bins = bins;
    std::vector<Box> tbox((size_t)T0);
    for (int64_t t = 0; t < T0; ++t) {
        tbox[t].reset();
        for (int v = 0; v < 3; ++v) tbox[t].grow(tri_v + 9 * t + 3 * v);
    }
    // the hierarchy is built over references (several per split triangle)
    std::vector<int32_t> rtri;
    std::vector<char> rsplit;
    make_refs(tri_v, T0, tbox, split_pct, rtri, B.tb, rsplit);
    const int64_t T = (int64_t)rtri.size();
    B.cen.resize((size_t)T * 3);
    B.idx.resize((size_t)T);
    for (int64_t r = 0; r < T; ++r) {
        const int64_t t = rtri[r];
        for (int i = 0; i < 3; ++i)
            B.cen[3 * r + i] =
                rsplit[r] ? 0.5 * (B.tb[r].lo[i] + B.tb[r].hi[i])
                          : (tri_v[9 * t + i] + tri_v[9 * t + 3 + i] + tri_v[9 * t + 6 + i]) / 3.0;
        B.idx[r] = (int32_t)r;
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
    perm.resize((size_t)T);
    for (int64_t q = 0; q < T; ++q) perm[q] = rtri[B.idx[q]];
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
