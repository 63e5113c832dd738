// Periodic octree of the dynamic AMR (host side): leaves, 2:1 balance, the
// refine / coarsen pass, Morton order and the mesh tables of a leaf set.
//
// Sec. New Developments (elements split into 8; 2:1 non-conforming faces
// joined by mortars) and Sec. Results (AMR Taylor-Green case: three levels
// with two indicator thresholds).  The pass: every leaf whose target level
// exceeds its level is split once; leaves are then split until face
// neighbours differ by at most one level; then each family of 8 unsplit
// sibling leaves whose targets are all below their level is merged into its
// parent unless the parent would face a leaf two levels finer.
#pragma once

#include <algorithm>
#include <cstdint>
#include <map>
#include <unordered_map>
#include <string>
#include <unordered_set>
#include <vector>

#include "host_parallel.h"

namespace dgx {

struct OctLeaf {
    int L, i, j, k;
};
inline bool operator<(const OctLeaf &a, const OctLeaf &b) {
    if (a.L != b.L) return a.L < b.L;
    if (a.i != b.i) return a.i < b.i;
    if (a.j != b.j) return a.j < b.j;
    return a.k < b.k;
}
inline bool operator==(const OctLeaf &a, const OctLeaf &b) {
    return a.L == b.L && a.i == b.i && a.j == b.j && a.k == b.k;
}

constexpr int kOctMaxLevel = 12;  // finest level; base * 2^L stays below 2^20
constexpr int kOctMaxBase = 64;

inline uint64_t oct_key(int L, int i, int j, int k) {
    return ((uint64_t)L << 60) | ((uint64_t)(uint32_t)i << 40) | ((uint64_t)(uint32_t)j << 20) | (uint64_t)(uint32_t)k;
}
inline uint64_t oct_key(const OctLeaf &c) { return oct_key(c.L, c.i, c.j, c.k); }

struct OctTree {
    int base = 1;
    std::unordered_set<uint64_t> leaves;

    int cells(int L) const { return base << L; }
    bool has(const OctLeaf &c) const { return leaves.count(oct_key(c)) != 0; }
    OctLeaf wrap(int L, int i, int j, int k) const {
        const int n = cells(L);
        return {L, ((i % n) + n) % n, ((j % n) + n) % n, ((k % n) + n) % n};
    }
    // the leaf containing level-L cell (i, j, k); false when that cell is split
    bool leaf_at(int L, int i, int j, int k, OctLeaf &out) const {
        const OctLeaf w = wrap(L, i, j, k);
        for (int s = 0; s <= L; ++s) {
            const OctLeaf c{L - s, w.i >> s, w.j >> s, w.k >> s};
            if (has(c)) {
                out = c;
                return true;
            }
        }
        return false;
    }
    // the four level-(L+1) cells across face (d, sgn) of c, sub-face order
    // a + 2b over the two tangential directions in increasing order
    void face_cells(const OctLeaf &c, int d, int sgn, OctLeaf out[4]) const {
        int q[3] = {2 * c.i, 2 * c.j, 2 * c.k};
        const int cd = d == 0 ? c.i : d == 1 ? c.j : c.k;
        q[d] = sgn > 0 ? 2 * cd + 2 : 2 * cd - 1;
        const int t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                int r[3] = {q[0], q[1], q[2]};
                r[t0] += a;
                r[t1] += b;
                out[a + 2 * b] = wrap(c.L + 1, r[0], r[1], r[2]);
            }
    }
    int finest_neighbour(const OctLeaf &c) const {
        int best = -1;
        for (int d = 0; d < 3; ++d)
            for (int sgn = -1; sgn <= 1; sgn += 2) {
                int ii[3] = {c.i, c.j, c.k};
                ii[d] += sgn;
                OctLeaf nb;
                if (leaf_at(c.L, ii[0], ii[1], ii[2], nb)) {
                    best = std::max(best, nb.L);
                    continue;
                }
                OctLeaf fc[4];
                face_cells(c, d, sgn, fc);
                for (int s = 0; s < 4; ++s) {
                    OctLeaf lf;
                    best = std::max(best, leaf_at(fc[s].L, fc[s].i, fc[s].j, fc[s].k, lf) ? lf.L : c.L + 2);
                }
            }
        return best;
    }
    static void children(const OctLeaf &c, OctLeaf out[8]) {
        for (int z = 0; z < 2; ++z)
            for (int y = 0; y < 2; ++y)
                for (int x = 0; x < 2; ++x) out[x + 2 * y + 4 * z] = {c.L + 1, 2 * c.i + x, 2 * c.j + y, 2 * c.k + z};
    }
    void split(const OctLeaf &c) {
        leaves.erase(oct_key(c));
        OctLeaf ch[8];
        children(c, ch);
        for (auto &x : ch) leaves.insert(oct_key(x));
    }
    std::vector<OctLeaf> list() const {
        std::vector<OctLeaf> v;
        v.reserve(leaves.size());
        for (uint64_t key : leaves)
            v.push_back({(int)(key >> 60), (int)((key >> 40) & 0xFFFFF), (int)((key >> 20) & 0xFFFFF), (int)(key & 0xFFFFF)});
        std::sort(v.begin(), v.end());
        return v;
    }
};

// Z-order of the leaves' lower corners on the finest grid
inline void morton_sort(std::vector<OctLeaf> &v) {
    int lmax = 0;
    for (auto &c : v) lmax = std::max(lmax, c.L);
    auto spread = [](uint64_t x) {
        uint64_t r = 0;
        for (int b = 0; b < 21; ++b) r |= ((x >> b) & 1ull) << (3 * b);
        return r;
    };
    std::vector<std::pair<uint64_t, OctLeaf>> keyed;
    keyed.reserve(v.size());
    for (auto &c : v) {
        const int s = lmax - c.L;
        keyed.push_back({spread((uint64_t)c.i << s) | spread((uint64_t)c.j << s) << 1 | spread((uint64_t)c.k << s) << 2, c});
    }
    std::sort(keyed.begin(), keyed.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
    for (size_t e = 0; e < v.size(); ++e) v[e] = keyed[e].second;
}

// Checks a leaf set: levels and indices in range, no leaf inside another,
// the leaves fill the cube, 2:1 balanced.  Empty string when valid.
inline std::string oct_check(int base, const std::vector<OctLeaf> &v, OctTree &t) {
    if (base < 1 || base > kOctMaxBase) return "octree base out of range";
    t.base = base;
    t.leaves.clear();
    t.leaves.reserve(v.size() * 2);
    int lmax = 0;
    for (auto &c : v) {
        if (c.L < 0 || c.L > kOctMaxLevel) return "octree level out of range";
        const int n = base << c.L;
        if (c.i < 0 || c.j < 0 || c.k < 0 || c.i >= n || c.j >= n || c.k >= n) return "octree index out of range";
        if (!t.leaves.insert(oct_key(c)).second) return "duplicate octree leaf";
        lmax = std::max(lmax, c.L);
    }
    unsigned __int128 vol = 0;
    for (auto &c : v) {
        for (int s = 1; s <= c.L; ++s)
            if (t.has({c.L - s, c.i >> s, c.j >> s, c.k >> s})) return "octree leaf inside another leaf";
        vol += (unsigned __int128)1 << (3 * (lmax - c.L));
    }
    if (vol != ((unsigned __int128)base * base * base) << (3 * lmax)) return "octree leaves do not fill the cube";
    std::vector<unsigned char> unbalanced(16, 0);
    host_parallel((int)v.size(), [&](int b, int e, int th) {
        for (int i = b; i < e && !unbalanced[th]; ++i) unbalanced[th] = t.finest_neighbour(v[i]) > v[i].L + 1;
    });
    if (std::count(unbalanced.begin(), unbalanced.end(), (unsigned char)1)) return "octree is not 2:1 balanced";
    return "";
}

// Conforming face rows and mortar rows of the leaves in element order
inline void oct_tables(const OctTree &t, const std::vector<OctLeaf> &order, std::vector<int32_t> &faces,
                       std::vector<int32_t> &morts) {
    std::unordered_map<uint64_t, int> eid;
    eid.reserve(order.size() * 2);
    for (size_t e = 0; e < order.size(); ++e) eid[oct_key(order[e])] = (int)e;
    // rows per thread over contiguous element ranges, joined in element order
    std::vector<std::vector<int32_t>> fpart(16), mpart(16);
    host_parallel((int)order.size(), [&](int e0, int e1, int th) {
        std::vector<int32_t> &fo = fpart[th], &mo = mpart[th];
        for (int e = e0; e < e1; ++e) {
            const OctLeaf &c = order[e];
            for (int d = 0; d < 3; ++d)
                for (int sgn = 1; sgn >= -1; sgn -= 2) {
                    int ii[3] = {c.i, c.j, c.k};
                    ii[d] += sgn;
                    OctLeaf nb;
                    if (t.leaf_at(c.L, ii[0], ii[1], ii[2], nb)) {
                        if (nb.L == c.L && sgn == 1) {
                            fo.push_back((int32_t)e);
                            fo.push_back(2 * d + 1);
                            fo.push_back(eid.at(oct_key(nb)));
                            fo.push_back(2 * d);
                        }
                        continue;  // coarser neighbour: the large side records the mortar
                    }
                    OctLeaf fc[4];
                    t.face_cells(c, d, sgn, fc);
                    const int fl = 2 * d + (sgn == 1 ? 1 : 0);
                    mo.push_back((int32_t)e);
                    mo.push_back(fl);
                    for (int s = 0; s < 4; ++s) mo.push_back(eid.at(oct_key(fc[s])));
                    mo.push_back(fl ^ 1);
                }
        }
    });
    faces.clear();
    morts.clear();
    for (int th = 0; th < 16; ++th) {
        faces.insert(faces.end(), fpart[th].begin(), fpart[th].end());
        morts.insert(morts.end(), mpart[th].begin(), mpart[th].end());
    }
}

// Transfer table row of a new element (kOctTab ints): kind (0 keep, 1 split,
// 2 merge), depth of the split path, the path's child indices (3 bits each,
// first split first), then the source elements (keep / split: 1, merge: 8
// children in child order x + 2y + 4z).
constexpr int kOctTab = 12;

// One adaptation pass.  target: per old element (old order).  Writes the
// new leaves in Morton order and their transfer rows.
inline std::string oct_adapt(int base, const std::vector<OctLeaf> &old_order, const int *target,
                             std::vector<OctLeaf> &new_order, std::vector<int32_t> &tab) {
    OctTree t;
    t.base = base;
    std::unordered_map<uint64_t, int> oid;
    t.leaves.reserve(old_order.size() * 4);
    oid.reserve(old_order.size() * 2);
    for (size_t e = 0; e < old_order.size(); ++e) {
        t.leaves.insert(oct_key(old_order[e]));
        oid[oct_key(old_order[e])] = (int)e;
    }
    std::unordered_set<uint64_t> split;
    for (size_t e = 0; e < old_order.size(); ++e) {
        const OctLeaf &c = old_order[e];
        if (target[e] > c.L) {
            if (c.L + 1 > kOctMaxLevel) return "refinement beyond the finest octree level";
            split.insert(oct_key(c));
        }
    }
    for (uint64_t key : split) {
        const OctLeaf c{(int)(key >> 60), (int)((key >> 40) & 0xFFFFF), (int)((key >> 20) & 0xFFFFF), (int)(key & 0xFFFFF)};
        t.split(c);
    }
    // 2:1 balance.  A leaf that faces one two levels finer must be split in
    // every balanced refinement of the current tree, so each sweep finds all
    // such leaves (in parallel, the tree read-only) and splits them together;
    // the sweeps end at the unique smallest balanced refinement.
    for (;;) {
        const std::vector<OctLeaf> cur = t.list();
        std::vector<unsigned char> need(cur.size(), 0);
        host_parallel((int)cur.size(), [&](int b, int e, int) {
            for (int i = b; i < e; ++i) need[i] = t.finest_neighbour(cur[i]) > cur[i].L + 1;
        });
        bool any = false;
        for (size_t i = 0; i < cur.size(); ++i) {
            if (!need[i]) continue;
            const OctLeaf &c = cur[i];
            if (c.L + 1 > kOctMaxLevel) return "2:1 balance beyond the finest octree level";
            t.split(c);
            if (oid.count(oct_key(c))) split.insert(oct_key(c));
            any = true;
        }
        if (!any) break;
    }
    // merges of unsplit families whose targets all lie below their level
    std::map<OctLeaf, std::vector<int>> fam;
    for (size_t e = 0; e < old_order.size(); ++e) {
        const OctLeaf &c = old_order[e];
        if (c.L > 0 && !split.count(oct_key(c))) fam[{c.L - 1, c.i >> 1, c.j >> 1, c.k >> 1}].push_back((int)e);
    }
    std::unordered_map<uint64_t, std::vector<int>> merged;
    for (auto &kv : fam) {
        const OctLeaf &p = kv.first;
        const auto &kids = kv.second;
        if (kids.size() != 8) continue;
        bool ok = true;
        for (int e : kids) ok = ok && t.has(old_order[e]) && target[e] < old_order[e].L;
        if (!ok) continue;
        for (int e : kids) t.leaves.erase(oct_key(old_order[e]));
        t.leaves.insert(oct_key(p));
        if (t.finest_neighbour(p) > p.L + 1) {
            t.leaves.erase(oct_key(p));
            for (int e : kids) t.leaves.insert(oct_key(old_order[e]));
            continue;
        }
        std::vector<int> byc(8);
        for (int e : kids) {
            const OctLeaf &c = old_order[e];
            byc[(c.i & 1) + 2 * (c.j & 1) + 4 * (c.k & 1)] = e;
        }
        merged[oct_key(p)] = byc;
    }
    new_order = t.list();
    morton_sort(new_order);
    tab.assign(new_order.size() * kOctTab, 0);
    for (size_t e = 0; e < new_order.size(); ++e) {
        int32_t *row = tab.data() + e * kOctTab;
        const OctLeaf &c = new_order[e];
        auto it = oid.find(oct_key(c));
        if (it != oid.end()) {
            row[0] = 0;
            row[3] = it->second;
            continue;
        }
        auto mt = merged.find(oct_key(c));
        if (mt != merged.end()) {
            row[0] = 2;
            for (int s = 0; s < 8; ++s) row[3 + s] = mt->second[s];
            continue;
        }
        // a descendant of a split old leaf
        OctLeaf a = c;
        int path[kOctMaxLevel + 1], depth = 0;
        while (!oid.count(oct_key(a))) {
            if (a.L == 0 || depth >= 8) return "octree transfer: no source leaf";
            path[depth++] = (a.i & 1) + 2 * (a.j & 1) + 4 * (a.k & 1);
            a = {a.L - 1, a.i >> 1, a.j >> 1, a.k >> 1};
        }
        if (depth > 2) return "octree transfer: split deeper than two levels";
        row[0] = 1;
        row[1] = depth;
        int code = 0;
        for (int q = 0; q < depth; ++q) code |= path[depth - 1 - q] << (3 * q);
        row[2] = code;
        row[3] = oid.at(oct_key(a));
    }
    return "";
}

}  // namespace dgx
