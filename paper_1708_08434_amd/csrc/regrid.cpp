// One step of mesh adaptation on the host (paper section 2.5): which boxes a
// tree should have after the charge has moved, from per-box refinement
// scores computed on the GPU (k_refine_scores).
//
// Criterion (the space-charge criterion of section 2.5): a cell needs
// refinement when |b| h^2 > c3 (b = -rho/eps0, h the cell size), i.e. when h
// exceeds sqrt(c3 eps0 / |rho|).  A leaf box is refined (all 8 children are
// added) when one of its cells, or a cell of a same-level leaf neighbour
// within 3 cells of it (the refinement buffer), needs refinement and the box
// is below max_level.  The 8 children of a box are removed when all of them
// are leaves, none is refined in this step, and neither their cells nor the
// cells of same-level leaf neighbours within 3 cells exceed deref * c3
// (section 2.5 derefines with a smaller constant), unless a box two levels
// finer than the parent would then touch it.  Finally 2:1 proper nesting over
// all 26 neighbours is restored by refining coarse leaves.  A step changes a
// leaf by at most one level, apart from the refinement the nesting forces.
#include <algorithm>
#include <unordered_set>

#include "mg_internal.h"

namespace mg {

namespace {

// (tree, level, i, j, k): 16 + 4 + 3 x 14 bits (levels <= 15)
uint64_t key(int64_t tree, int l, int64_t i, int64_t j, int64_t k) {
    return ((uint64_t)tree << 48) | ((uint64_t)l << 42) | ((uint64_t)i << 28) | ((uint64_t)j << 14) |
           (uint64_t)k;
}

}  // namespace

int regrid_plan(const mg_tree *t, const double *sc, double c3, double deref, int max_level,
                std::vector<int32_t> &level, std::vector<int32_t> &ijk, std::vector<int32_t> &tree) {
    const int64_t n = t->n;
    std::vector<char> leaf(n), refine(n, 0), drop(n, 0);
    for (int64_t b = 0; b < n; b++) leaf[b] = t->child[8 * b] < 0;
    // a cell of box b, or of a same-level leaf neighbour within 3 cells of
    // b, above thr; scores[b][r] is the largest |b| h^2 over the cells of b
    // in region r = (sx+1) + 3 (sy+1) + 9 (sz+1) (s_a = -1: cells 0..2 along
    // a, +1: cells 5..7, 0: all), and the cells of neighbour b + o within 3
    // cells of b form its region -o, i.e. 26 - o
    auto hot = [&](int64_t b, double thr) {
        if (sc[27 * b + 13] > thr) return true;
        for (int o = 0; o < 27; o++) {
            if (o == 13) continue;
            int32_t N = t->n27[27 * b + o];
            if (N >= 0 && leaf[N] && sc[27 * (int64_t)N + (26 - o)] > thr) return true;
        }
        return false;
    };
    for (int64_t b = 0; b < n; b++)
        if (leaf[b] && t->lev[b] < max_level && hot(b, c3)) refine[b] = 1;
    for (int64_t p = 0; p < n; p++) {
        if (leaf[p]) continue;
        bool ok = true;
        for (int q = 0; q < 8 && ok; q++) {
            int64_t c = t->child[8 * p + q];
            ok = leaf[c] && !refine[c] && !hot(c, deref * c3);
        }
        // after the removal p is a leaf of level l: no box of level l+2 may
        // touch it, i.e. no same-level neighbour may have (or get) grandchildren
        for (int o = 0; o < 27 && ok; o++) {
            int32_t Q = t->n27[27 * p + o];
            if (o == 13 || Q < 0 || leaf[Q]) continue;
            for (int q = 0; q < 8 && ok; q++) {
                int64_t c = t->child[8 * (int64_t)Q + q];
                ok = leaf[c] && !refine[c];
            }
        }
        drop[p] = ok;
    }
    std::unordered_set<uint64_t> set;
    std::vector<uint64_t> work;
    set.reserve((size_t)(n * 1.3) + 64);
    auto add = [&](int64_t tr, int l, int64_t i, int64_t j, int64_t k) {
        if (set.insert(key(tr, l, i, j, k)).second) work.push_back(key(tr, l, i, j, k));
    };
    for (int64_t b = 0; b < n; b++) {
        if (t->lev[b] >= 2 && drop[t->parent[b]]) continue;
        int64_t tr = t->tid[b], i = t->ijk[3 * b], j = t->ijk[3 * b + 1], k = t->ijk[3 * b + 2];
        add(tr, t->lev[b], i, j, k);
        if (refine[b])
            for (int q = 0; q < 8; q++)
                add(tr, t->lev[b] + 1, 2 * i + (q & 1), 2 * j + ((q >> 1) & 1), 2 * k + (q >> 2));
    }
    // 2:1 nesting: every position next to a box of level l (26 directions,
    // inside the domain) must be covered down to level l-1; otherwise the
    // deepest box that covers it is refined (and its children checked in turn)
    while (!work.empty()) {
        std::vector<uint64_t> cur;
        cur.swap(work);
        for (uint64_t kb : cur) {
            int64_t tr = (int64_t)(kb >> 48);
            int l = (int)((kb >> 42) & 63);
            int64_t i = (int64_t)((kb >> 28) & 16383), j = (int64_t)((kb >> 14) & 16383),
                    k = (int64_t)(kb & 16383);
            if (l < 3) continue;
            int64_t lim = (int64_t)1 << (l - 1);
            for (int oz = -1; oz <= 1; oz++)
                for (int oy = -1; oy <= 1; oy++)
                    for (int ox = -1; ox <= 1; ox++) {
                        int64_t pi = i + ox, pj = j + oy, pk = k + oz;
                        if ((ox | oy | oz) == 0 || pi < 0 || pj < 0 || pk < 0 || pi >= lim ||
                            pj >= lim || pk >= lim)
                            continue;
                        if (set.count(key(tr, l - 1, pi >> 1, pj >> 1, pk >> 1))) continue;
                        for (int m = l - 2; m >= 1; m--) {
                            int sh = l - m;
                            if (set.count(key(tr, m, pi >> sh, pj >> sh, pk >> sh))) {
                                int64_t ai = pi >> sh, aj = pj >> sh, ak = pk >> sh;
                                for (int q = 0; q < 8; q++)
                                    add(tr, m + 1, 2 * ai + (q & 1), 2 * aj + ((q >> 1) & 1),
                                        2 * ak + (q >> 2));
                                break;
                            }
                        }
                    }
        }
    }
    std::vector<uint64_t> keys(set.begin(), set.end());
    std::sort(keys.begin(), keys.end());
    level.resize(keys.size());
    tree.resize(keys.size());
    ijk.resize(3 * keys.size());
    for (size_t q = 0; q < keys.size(); q++) {
        uint64_t kb = keys[q];
        tree[q] = (int32_t)(kb >> 48);
        level[q] = (int32_t)((kb >> 42) & 63);
        ijk[3 * q] = (int32_t)((kb >> 28) & 16383);
        ijk[3 * q + 1] = (int32_t)((kb >> 14) & 16383);
        ijk[3 * q + 2] = (int32_t)(kb & 16383);
    }
    return MG_OK;
}

}  // namespace mg
