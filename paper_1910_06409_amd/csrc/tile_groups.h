// tile_groups.h -- host-side grouping of the cross-spectral tile pairs for the
// split-BF16 rank-k workgroups (plain C++, no HIP: also built by a CPU test).
#pragma once
#include <algorithm>
#include <map>
#include <utility>
#include <vector>

namespace gke {

// The tile pairs grouped four at a time for the split-BF16 rank-k, whose
// workgroups hold at most four tiles in LDS: first the full 2 x 2 blocks
// (pairs with the same (a / 2, b / 2)), then the other pairs in (a, b) order,
// each joining the open group while it has fewer than four pairs and its
// tiles stay within four.  Per group twelve ints: the four tile slots
// (t: row tile t, planes through the row-plane table; t | 1 << 16: column
// tile t, planes 16 t .. 16 t + 15; -1: empty), the tile-pair index of each
// wave (-1: none), and each wave's left and right slot (l | r << 4).
// same_planes: row tile t is column tile t (the all-pairs mode), so that the
// two share a slot.
inline std::vector<int> group_tile_pairs(const std::vector<int> &ta, const std::vector<int> &tb,
                                         int ntp, bool same_planes)
{
    struct Group {
        std::vector<int> slots, tps, ops;
    };
    auto col = [&](int t) { return same_planes ? t : t | 1 << 16; };
    auto slot_of = [](Group &g, int code, bool add) {
        for (size_t i = 0; i < g.slots.size(); ++i)
            if (g.slots[i] == code) return (int)i;
        if (!add) return -1;
        g.slots.push_back(code);
        return (int)g.slots.size() - 1;
    };
    auto add_pair = [&](Group &g, int i) {
        const int l = slot_of(g, ta[i], true), r = slot_of(g, col(tb[i]), true);
        g.tps.push_back(i);
        g.ops.push_back(l | r << 4);
    };
    std::map<std::pair<int, int>, std::vector<int>> blk;
    for (int i = 0; i < ntp; ++i) blk[{ta[i] >> 1, tb[i] >> 1}].push_back(i);
    std::vector<Group> groups;
    std::vector<int> rest;
    for (const auto &kv : blk) {
        if (kv.second.size() == 4) {
            Group g;
            for (int i : kv.second) add_pair(g, i);
            groups.push_back(g);
        } else {
            rest.insert(rest.end(), kv.second.begin(), kv.second.end());
        }
    }
    std::sort(rest.begin(), rest.end(), [&](int x, int y) {
        return ta[x] != ta[y] ? ta[x] < ta[y] : tb[x] < tb[y];
    });
    Group open;
    for (int i : rest) {
        const int a = ta[i], b = col(tb[i]);
        const int extra = (slot_of(open, a, false) < 0) + (b != a && slot_of(open, b, false) < 0);
        if (open.tps.size() == 4 || open.slots.size() + extra > 4) {
            groups.push_back(open);
            open = Group();
        }
        add_pair(open, i);
    }
    if (!open.tps.empty()) groups.push_back(open);
    std::vector<int> out;
    for (const Group &g : groups) {
        for (int w = 0; w < 4; ++w) out.push_back(w < (int)g.slots.size() ? g.slots[w] : -1);
        for (int w = 0; w < 4; ++w) out.push_back(w < (int)g.tps.size() ? g.tps[w] : -1);
        for (int w = 0; w < 4; ++w) out.push_back(w < (int)g.ops.size() ? g.ops[w] : 0);
    }
    return out;
}

}  // namespace gke
