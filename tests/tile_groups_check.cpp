// CPU check of the grouping of tile pairs for the split-BF16 rank-k
// workgroups: every pair in exactly one group, at most four tile slots per
// group, and each wave's operand slots holding the tiles of its pair.  Exit
// status 0 on success; prints the group counts of the two layouts it covers.
#include <cstdio>
#include <vector>

#include "tile_groups.h"

static int check(const std::vector<int> &ta, const std::vector<int> &tb, bool same, int nrt,
                 int nct, int *ngroups, int *idle)
{
    const int ntp = (int)ta.size();
    const std::vector<int> sb = gke::group_tile_pairs(ta, tb, ntp, same);
    if (sb.size() % 12) return 1;
    std::vector<int> seen(ntp, 0);
    *ngroups = (int)sb.size() / 12;
    *idle = 0;
    for (size_t s = 0; s < sb.size(); s += 12) {
        for (int w = 0; w < 4; ++w) {
            const int c = sb[s + w];
            if (c < 0) continue;
            const int t = c & 0xffff, direct = c >> 16;
            if (direct > 1 || (direct ? t >= nct : t >= nrt) || (same && direct)) return 2;
        }
        for (int w = 0; w < 4; ++w) {
            const int tp = sb[s + 4 + w], ops = sb[s + 8 + w];
            if (tp < 0) {
                ++*idle;
                continue;
            }
            if (tp >= ntp) return 3;
            ++seen[tp];
            const int l = ops & 15, r = ops >> 4;
            if (l > 3 || r > 3 || sb[s + l] < 0 || sb[s + r] < 0) return 4;
            const int lc = sb[s + l], rc = sb[s + r];
            if ((lc >> 16) != 0 || (lc & 0xffff) != ta[tp]) return 5;
            if ((rc & 0xffff) != tb[tp] || (rc >> 16) != (same ? 0 : 1)) return 6;
        }
    }
    for (int t = 0; t < ntp; ++t)
        if (seen[t] != 1) return 7;
    return 0;
}

int main()
{
    int ng = 0, idle = 0;
    // the all-pairs mode: tile pairs a <= b
    for (int nt = 0; nt <= 17; ++nt) {
        std::vector<int> ta, tb;
        for (int a = 0; a < nt; ++a)
            for (int b = a; b < nt; ++b) {
                ta.push_back(a);
                tb.push_back(b);
            }
        if (int e = check(ta, tb, true, nt, nt, &ng, &idle)) {
            std::printf("triangle %d: error %d\n", nt, e);
            return 1;
        }
        std::printf("triangle %d %d %d\n", nt, ng, idle);
    }
    // slabs: every row tile against every column tile
    for (int nrt = 0; nrt <= 6; ++nrt)
        for (int nt = 0; nt <= 17; ++nt) {
            std::vector<int> ta, tb;
            for (int a = 0; a < nrt; ++a)
                for (int b = 0; b < nt; ++b) {
                    ta.push_back(a);
                    tb.push_back(b);
                }
            if (int e = check(ta, tb, false, nrt, nt, &ng, &idle)) {
                std::printf("rectangle %dx%d: error %d\n", nrt, nt, e);
                return 1;
            }
            std::printf("rectangle %d %d %d %d\n", nrt, nt, ng, idle);
        }
    return 0;
}
