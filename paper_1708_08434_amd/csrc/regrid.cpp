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
// (section 2.5 derefines with a smaller constant, 1/8 there) and their cell
// size is below h_deref (the paper's Delta x_deref, which keeps a floor on
// the resolution where the discharge has stopped growing), unless a box two
// levels finer than the parent would then touch it.  Finally 2:1 proper
// nesting over all 26 neighbours is restored by refining coarse leaves.  A
// step changes a leaf by at most one level, apart from the refinement the
// nesting forces.
#include <algorithm>
#include <unordered_set>

#include "mg_internal.h"

namespace mg {

namespace {

// Box keys sort like the canonical box order: level (bits 58..61), tree
// (42..57), Morton code of (i, j, k) (0..41; 14 bits per coordinate).
uint64_t key(int64_t tree, int l, int64_t i, int64_t j, int64_t k) {
    return ((uint64_t)l << 58) | ((uint64_t)tree << 42) | morton((int32_t)i, (int32_t)j, (int32_t)k);
}

// The coordinate bits of m from bit s (bits s, s+3, ..., s+39), packed: the
// inverse of morton()'s spread, with the level and tree bits masked off.
int32_t compact3(uint64_t m, int s) {
    uint64_t v = (m >> s) & 0x0000009249249249ULL;
    v = (v | (v >> 2)) & 0x10c30c30c30c30c3ULL;
    v = (v | (v >> 4)) & 0x100f00f00f00f00fULL;
    v = (v | (v >> 8)) & 0x001f0000ff0000ffULL;
    v = (v | (v >> 16)) & 0x001f00000000ffffULL;
    v = (v | (v >> 32)) & 0x00000000001fffffULL;
    return (int32_t)v;
}

}  // namespace

void regrid_near(const mg_tree *t, const double *sc, double *near) {
    const int64_t n = t->n;
    // near[b] (leaves): the largest score over the cells of b and the cells
    // of same-level leaf neighbours within 3 cells of b; scores[b][r] is the
    // largest |b| h^2 over the cells of b in region r = (sx+1) + 3 (sy+1) +
    // 9 (sz+1) (s_a = -1: cells 0..2 along a, +1: cells 5..7, 0: all), and
    // the cells of neighbour b + o within 3 cells of b form its region -o,
    // i.e. 26 - o.  Scores are >= 0, so a missing neighbour reads b's own.
    parallel_for(n, [&](int64_t lo, int64_t hi) {
        for (int64_t b = lo; b < hi; b++) {
            near[b] = 0.0;
            if (t->child[8 * b] >= 0) continue;
            const int32_t *nb = &t->n27[27 * b];
            double m = sc[27 * b + 13];
            for (int o = 0; o < 27; o++) {
                int64_t N = nb[o];
                bool use = N >= 0 && t->child[8 * (N >= 0 ? N : b)] < 0;
                m = std::max(m, sc[use ? 27 * N + (26 - o) : 27 * b + 13]);
            }
            near[b] = m;
        }
    });
}

int regrid_plan(const mg_tree *t, const double *sc, double c3, double deref, double h_deref, int max_level,
                std::vector<int32_t> &level, std::vector<int32_t> &ijk, std::vector<int32_t> &tree) {
    std::vector<double> near(t->n);
    regrid_near(t, sc, near.data());
    return regrid_plan_near(t, near.data(), c3, deref, h_deref, max_level, level, ijk, tree);
}

int regrid_plan_near(const mg_tree *t, const double *near, double c3, double deref, double h_deref,
                     int max_level, std::vector<int32_t> &level, std::vector<int32_t> &ijk,
                     std::vector<int32_t> &tree) {
    const int64_t n = t->n;
    std::vector<char> leaf(n), refine(n, 0), drop(n, 0);
    parallel_for(n, [&](int64_t lo, int64_t hi) {
        for (int64_t b = lo; b < hi; b++) leaf[b] = t->child[8 * b] < 0;
    });
    parallel_for(n, [&](int64_t lo, int64_t hi) {
        for (int64_t b = lo; b < hi; b++)
            if (leaf[b] && t->lev[b] < max_level && near[b] > c3) refine[b] = 1;
    });
    const double thr_d = deref * c3;
    parallel_for(n, [&](int64_t lo, int64_t hi) {
    for (int64_t p = lo; p < hi; p++) {
        if (leaf[p] || !(t->dom.len / (8.0 * (double)(1 << t->lev[p])) < h_deref)) continue;
        bool ok = true;
        for (int q = 0; q < 8 && ok; q++) {
            int64_t c = t->child[8 * p + q];
            ok = leaf[c] && !refine[c] && !(near[c] > thr_d);
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
    });
    // the kept boxes, in canonical order (so their keys are sorted); they
    // satisfy 2:1 nesting among themselves: the tree did, and a removal is
    // only allowed where no box two levels finer touches the new leaf, so
    // only added boxes (and what they force) need the nesting check
    std::vector<uint64_t> all(n);
    parallel_for(n, [&](int64_t lo, int64_t hi) {
        for (int64_t b = lo; b < hi; b++)
            all[b] = (t->lev[b] >= 2 && drop[t->parent[b]])
                         ? ~(uint64_t)0
                         : key(t->tid[b], t->lev[b], t->ijk[3 * b], t->ijk[3 * b + 1], t->ijk[3 * b + 2]);
    });
    std::vector<uint64_t> kept;
    kept.reserve(n);
    for (int64_t b = 0; b < n; b++)
        if (all[b] != ~(uint64_t)0) kept.push_back(all[b]);
    if (!std::is_sorted(kept.begin(), kept.end())) std::sort(kept.begin(), kept.end());
    std::unordered_set<uint64_t> added;
    std::vector<uint64_t> work;
    auto has = [&](uint64_t kb) { return std::binary_search(kept.begin(), kept.end(), kb) || added.count(kb); };
    auto add = [&](uint64_t kb) {
        if (!std::binary_search(kept.begin(), kept.end(), kb) && added.insert(kb).second) work.push_back(kb);
    };
    auto add_children = [&](int64_t tr, int l, int64_t i, int64_t j, int64_t k) {
        for (int q = 0; q < 8; q++) add(key(tr, l + 1, 2 * i + (q & 1), 2 * j + ((q >> 1) & 1), 2 * k + (q >> 2)));
    };
    for (int64_t b = 0; b < n; b++)
        if (refine[b]) add_children(t->tid[b], t->lev[b], t->ijk[3 * b], t->ijk[3 * b + 1], t->ijk[3 * b + 2]);
    // 2:1 nesting: every position next to a box of level l (26 directions,
    // inside the domain) must be covered down to level l-1; otherwise the
    // deepest box that covers it is refined (and its children checked in turn)
    while (!work.empty()) {
        std::vector<uint64_t> cur;
        cur.swap(work);
        for (uint64_t kb : cur) {
            int l = (int)(kb >> 58);
            int64_t tr = (int64_t)((kb >> 42) & 0xffff);
            int64_t i = compact3(kb, 0), j = compact3(kb, 1), k = compact3(kb, 2);
            if (l < 3) continue;
            int64_t lim = (int64_t)1 << (l - 1);
            for (int oz = -1; oz <= 1; oz++)
                for (int oy = -1; oy <= 1; oy++)
                    for (int ox = -1; ox <= 1; ox++) {
                        int64_t pi = i + ox, pj = j + oy, pk = k + oz;
                        if ((ox | oy | oz) == 0 || pi < 0 || pj < 0 || pk < 0 || pi >= lim ||
                            pj >= lim || pk >= lim)
                            continue;
                        if (has(key(tr, l - 1, pi >> 1, pj >> 1, pk >> 1))) continue;
                        for (int m = l - 2; m >= 1; m--) {
                            int sh = l - m;
                            if (has(key(tr, m, pi >> sh, pj >> sh, pk >> sh))) {
                                add_children(tr, m, pi >> sh, pj >> sh, pk >> sh);
                                break;
                            }
                        }
                    }
        }
    }
    std::vector<uint64_t> extra(added.begin(), added.end()), keys(kept.size() + added.size());
    std::sort(extra.begin(), extra.end());
    std::merge(kept.begin(), kept.end(), extra.begin(), extra.end(), keys.begin());
    level.resize(keys.size());
    tree.resize(keys.size());
    ijk.resize(3 * keys.size());
    parallel_for((int64_t)keys.size(), [&](int64_t lo, int64_t hi) {
        for (int64_t q = lo; q < hi; q++) {
            uint64_t kb = keys[q];
            level[q] = (int32_t)(kb >> 58);
            tree[q] = (int32_t)((kb >> 42) & 0xffff);
            ijk[3 * q] = compact3(kb, 0);
            ijk[3 * q + 1] = compact3(kb, 1);
            ijk[3 * q + 2] = compact3(kb, 2);
        }
    });
    return MG_OK;
}

}  // namespace mg
