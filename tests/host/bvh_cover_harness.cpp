// Host harness for the BVH builder: every point of every triangle must be
// reachable from the root through FP32 child boxes that contain it (exact
// comparisons) down to a leaf holding a reference to that triangle.  Reads
// T and [T][9] FP64 vertices from a file; checks the vertices, the edge
// midpoints and random barycentric points of every triangle that was split
// into several references and of a sample of the others.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "internal.h"

using namespace sbr;

static std::vector<Bvh4Node> g_nodes;
static std::vector<int32_t> g_perm;

static bool in_box(const Bvh4Node& n, int k, const double* p)
{
    return (double)n.lox[k] <= p[0] && p[0] <= (double)n.hix[k] && (double)n.loy[k] <= p[1] &&
           p[1] <= (double)n.hiy[k] && (double)n.loz[k] <= p[2] && p[2] <= (double)n.hiz[k];
}

static bool reach(int32_t node, const double* p, int32_t t)
{
    const Bvh4Node& n = g_nodes[node];
    for (int k = 0; k < 4; ++k) {
        if (n.cnt[k] < 0 || !in_box(n, k, p)) continue;
        if (n.cnt[k] == 0) {
            if (reach(n.idx[k], p, t)) return true;
        } else {
            for (int32_t q = n.idx[k]; q < n.idx[k] + n.cnt[k]; ++q)
                if (g_perm[q] == t) return true;
        }
    }
    return false;
}

int main(int argc, char** argv)
{
    if (argc < 4) return 2;
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t T = 0;
    if (fread(&T, 8, 1, f) != 1) return 2;
    std::vector<double> v((size_t)T * 9);
    if (fread(v.data(), 8, v.size(), f) != v.size()) return 2;
    fclose(f);
    const int split = atoi(argv[2]);
    const int samples = atoi(argv[3]);
    build_bvh(v.data(), T, 4, 64, split, argc > 4, g_nodes, g_perm);
    std::vector<int32_t> nref((size_t)T, 0);
    for (int32_t t : g_perm) nref[t] += 1;
    int64_t split_tris = 0, checked = 0, bad = 0;
    for (int64_t t = 0; t < T; ++t) split_tris += nref[t] > 1;
    std::mt19937_64 g(7);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    for (int64_t t = 0; t < T; ++t) {
        if (nref[t] == 0) {
            ++bad;
            continue;
        }
        if (nref[t] == 1 && (t % 97) != 0) continue;
        const double* V = &v[9 * (size_t)t];
        const int n = nref[t] > 1 ? samples : 8;
        for (int s = 0; s < n + 6; ++s) {
            double a, b;
            if (s < 3) {
                a = s == 1;
                b = s == 2;
            } else if (s < 6) {
                a = s == 3 ? 0.5 : s == 4 ? 0.0 : 0.5;
                b = s == 3 ? 0.0 : 0.5;
            } else {
                a = U(g);
                b = U(g);
                if (a + b > 1.0) {
                    a = 1.0 - a;
                    b = 1.0 - b;
                }
            }
            double p[3];
            for (int k = 0; k < 3; ++k)
                p[k] = V[k] + a * (V[3 + k] - V[k]) + b * (V[6 + k] - V[k]);
            ++checked;
            if (!reach(0, p, (int32_t)t)) {
                if (bad < 5) printf("unreachable: tri %lld point %d\n", (long long)t, s);
                ++bad;
            }
        }
    }
    printf("T=%lld refs=%zu split_tris=%lld checked=%lld bad=%lld\n", (long long)T, g_perm.size(),
           (long long)split_tris, (long long)checked, (long long)bad);
    return bad != 0;
}
