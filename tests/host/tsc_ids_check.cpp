// Host check of the TSC stencil resolution (TscCache::gather in device.h,
// compiled here for the host): on random full octrees, periodic and not, in
// the library's id order (coarse cells by Morton index, then the 8 children
// of each refined cell as a block, level by level), the payloads it gathers
// for the 27 cells around a cell at any level, and whether it finds them
// all, must equal those of 27 direct lookups (lookup_cell).  Test
// infrastructure; prints one summary line and exits non-zero on a mismatch.
#include <hip/hip_runtime.h>

#include <array>
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "device.h"

using namespace mpath;

struct Tree {
    std::vector<int> child;
    std::vector<float4> payload;
    std::vector<std::array<int, 3>> pos;
    std::vector<int> level_start;
};

// Cells near a random centre are refined with high probability, others with
// low probability, so that refined regions of several cells exist at every level.
static Tree make_tree(int n0, int max_level, std::mt19937& rng)
{
    Tree t;
    const int nc = n0 * n0 * n0;
    t.child.assign(nc, -1);
    t.pos.resize(nc);
    for (int i = 0; i < n0; ++i)
        for (int j = 0; j < n0; ++j)
            for (int k = 0; k < n0; ++k) t.pos[morton3(i, j, k)] = {i, j, k};
    t.level_start.push_back(0);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    const double cx = U(rng) * n0, cy = U(rng) * n0, cz = U(rng) * n0;
    int lo = 0, hi = nc;
    for (int l = 0; l < max_level; ++l) {
        t.level_start.push_back(hi);
        int next = hi;
        for (int c = lo; c < hi; ++c) {
            const double h = 1.0 / (1 << l);
            const double x = (t.pos[c][0] + 0.5) * h - cx, y = (t.pos[c][1] + 0.5) * h - cy,
                         z = (t.pos[c][2] + 0.5) * h - cz;
            if (U(rng) < (std::sqrt(x * x + y * y + z * z) < 2.5 ? 0.85 : 0.15)) {
                t.child[c] = next;
                for (int o = 0; o < 8; ++o) {
                    t.pos.push_back({2 * t.pos[c][0] + (o & 1), 2 * t.pos[c][1] + ((o >> 1) & 1),
                                     2 * t.pos[c][2] + (o >> 2)});
                    t.child.push_back(-1);
                }
                next += 8;
            }
        }
        lo = hi;
        hi = next;
    }
    while ((int)t.level_start.size() < kMaxLevels + 1) t.level_start.push_back(hi);
    t.payload.resize(hi);
    for (int c = 0; c < hi; ++c) t.payload[c] = make_float4((float)c, c + 0.25f, c + 0.5f, -(float)c);
    return t;
}

template <bool AMR>
static bool same(const GridDev& g, const Tree& t, int l, const int cc[3], bool& all)
{
    int ids[27];
    all = true;
    for (int q = 0; q < 27; ++q) {
        ids[q] = lookup_cell(g, l, cc[0] + q % 3 - 1, cc[1] + (q / 3) % 3 - 1, cc[2] + q / 9 - 1);
        all = all && ids[q] >= 0;
    }
    TscCache<AMR> tc;
    const bool ok = tc.gather(g, l, cc);
    if (ok != all) return false;
    if (ok)
        for (int q = 0; q < 27; ++q)
            if (tc.p[q].x != t.payload[ids[q]].x || tc.p[q].w != t.payload[ids[q]].w) return false;
    return true;
}

int main()
{
    std::mt19937 rng(20261203);
    long checks = 0, complete = 0, complete_refined = 0, bad = 0;
    for (int trial = 0; trial < 48; ++trial) {
        const int periodic = trial & 1, n0 = trial % 3 == 0 ? 4 : 8, max_level = trial % 4;
        const Tree t = make_tree(n0, max_level, rng);
        GridDev g{};
        g.payload = t.payload.data();
        g.child = t.child.data();
        g.n0 = n0;
        g.max_level = max_level;
        g.periodic = periodic;
        for (int k = 0; k <= kMaxLevels; ++k) g.level_start[k] = t.level_start[k];
        for (int rep = 0; rep < 3000; ++rep) {
            const int l = std::uniform_int_distribution<int>(0, max_level)(rng);
            const int M = n0 << l;
            int cc[3];
            if ((rep & 1) && l > 0 && t.level_start[l + 1] > t.level_start[l]) {
                // around an existing cell of level l, unwrapped by a box length on periodic grids
                const int c = std::uniform_int_distribution<int>(t.level_start[l], t.level_start[l + 1] - 1)(rng);
                for (int d = 0; d < 3; ++d) cc[d] = t.pos[c][d];
                if (periodic) cc[rep % 3] += (rep & 2) ? M : -M;
            } else {
                for (int d = 0; d < 3; ++d) cc[d] = std::uniform_int_distribution<int>(-M - 2, 2 * M + 1)(rng);
            }
            bool all = false;
            const bool ok = max_level == 0 ? same<false>(g, t, l, cc, all) && same<true>(g, t, l, cc, all)
                                           : same<true>(g, t, l, cc, all);
            bad += !ok;
            ++checks;
            complete += all;
            complete_refined += all && l > 0;
        }
    }
    std::printf("tsc ids: %ld checks, %ld complete stencils (%ld refined), %ld mismatches\n", checks, complete,
                complete_refined, bad);
    return bad != 0 || complete_refined == 0;
}
