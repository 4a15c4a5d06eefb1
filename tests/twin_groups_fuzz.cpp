#include <algorithm>
#include <cassert>
#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <random>
#include <set>
#include <vector>
#include "twins.inc"
// Randomised check of the twin-group index of the BIRCH update labelling
// (member lists, groups of two or more, the open-addressing key table with
// backward-shift removal) against a plain model: random joins and leaves,
// keys shared by several groups, table growth.  The structure's source is
// cut out of birch.hip into twins.inc by tests/test_twin_groups.py.
int main() {
    std::mt19937_64 rng(1);
    for (int trial = 0; trial < 200; ++trial) {
        TwinGroups T;
        const int nid = 2000;
        T.resize(nid);
        std::map<int32_t, std::set<int32_t>> model;   // group -> members
        std::vector<int32_t> grp_of(nid, -1);
        std::map<uint64_t, std::multiset<int32_t>> bykey;
        const int nkeys = 1 + rng() % 300;
        for (int op = 0; op < 20000; ++op) {
            const int32_t id = rng() % nid;
            if (grp_of[id] >= 0) {
                const int32_t gi = grp_of[id];
                T.remove(gi, id);
                model[gi].erase(id);
                grp_of[id] = -1;
                if (model[gi].empty()) {
                    bykey[T.g[gi].key].erase(bykey[T.g[gi].key].find(gi));
                    T.drop(gi);
                    model.erase(gi);
                }
            } else {
                // keys collide on purpose: low bits few, and several groups share one key
                const uint64_t key = (rng() % nkeys) * 0x9E3779B97F4A7C15ull;
                const bool join = !bykey[key].empty() && (rng() % 3);
                int32_t gi;
                if (join) {
                    auto it = bykey[key].begin();
                    std::advance(it, rng() % bykey[key].size());
                    gi = *it;
                    // it must be findable through the table
                    const size_t mask = T.hgrp.size() - 1;
                    bool found = false;
                    for (size_t i = key & mask; T.hgrp[i] >= 0; i = (i + 1) & mask)
                        if (T.hkey[i] == key && T.hgrp[i] == gi) found = true;
                    assert(found);
                } else {
                    gi = T.make(key);
                    assert(!model.count(gi));
                    bykey[key].insert(gi);
                }
                T.add(gi, id);
                model[gi].insert(id);
                grp_of[id] = gi;
            }
            if (op % 997 == 0) {
                // full consistency
                size_t multi = 0, live = 0;
                for (auto &kv : model) {
                    const auto &G = T.g[kv.first];
                    std::set<int32_t> got;
                    for (int32_t x = G.head; x >= 0; x = T.next[x]) { got.insert(x); assert(T.of[x] == kv.first); }
                    assert(got == kv.second);
                    assert(G.size == (int)kv.second.size());
                    if (G.size >= 2) { ++multi; assert(G.mpos >= 0 && T.multi[G.mpos] == kv.first); }
                    else assert(G.mpos == -1);
                    ++live;
                }
                assert(T.multi.size() == multi);
                size_t used = 0;
                for (size_t i = 0; i < T.hgrp.size(); ++i) if (T.hgrp[i] >= 0) ++used;
                assert(used == live && T.used == live);
                // every live group reachable from its home slot
                const size_t mask = T.hgrp.size() - 1;
                for (auto &kv : model) {
                    const uint64_t key = T.g[kv.first].key;
                    bool found = false;
                    for (size_t i = key & mask; T.hgrp[i] >= 0; i = (i + 1) & mask)
                        if (T.hgrp[i] == kv.first) found = true;
                    assert(found);
                }
            }
        }
    }
    std::puts("twin groups: ok");
}
