// Host-side octree construction: validation, canonical ordering and the
// index tables the kernels use.
//
// Octree of N^3 boxes with N = 8 (paper section 2.1.1): a refined box is
// covered by all 2^3 children, and proper nesting limits neighbouring boxes
// (here: all 26 neighbours) to one level of difference.  Tables are built
// level by level from parent relations, so a mesh change costs one linear
// pass plus a sort (section 2.1.2 notes that geometric multigrid needs almost
// no extra work when the mesh changes).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <atomic>
#include <cstring>
#include <thread>
#include <tuple>

#include "kernels.h"
#include "mg_internal.h"

namespace mg {

// Spread the low 21 bits of x so that bit b lands on bit 3b.
static uint64_t spread_bits3(uint32_t x) {
    uint64_t v = x & 0x1fffffu;
    v = (v | (v << 32)) & 0x1f00000000ffffULL;
    v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
    v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
    v = (v | (v << 2)) & 0x1249249249249249ULL;
    return v;
}

uint64_t morton(int32_t i, int32_t j, int32_t k) {
    return spread_bits3((uint32_t)i) | (spread_bits3((uint32_t)j) << 1) |
           (spread_bits3((uint32_t)k) << 2);
}

namespace {

// Sorts keys in (level, tree, Morton) order: an LSD radix sort of the packed
// 62-bit key level << 58 | tree << 42 | Morton (four 16-bit digits).
template <typename K> void sort_keys(std::vector<K> &keys) {
    const size_t n = keys.size();
    std::vector<uint64_t> a(n), b(n);
    std::vector<int32_t> ia(n), ib(n);
    for (size_t q = 0; q < n; q++) {
        a[q] = ((uint64_t)keys[q].level << 58) | ((uint64_t)keys[q].tree << 42) | keys[q].m;
        ia[q] = (int32_t)q;
    }
    std::vector<uint32_t> cnt(65537);
    for (int pass = 0; pass < 4; pass++) {
        int sh = 16 * pass;
        std::fill(cnt.begin(), cnt.end(), 0u);
        for (size_t q = 0; q < n; q++) cnt[((a[q] >> sh) & 0xffff) + 1]++;
        if (cnt[1] == n) continue;  // every key has this digit 0
        for (int d = 0; d < 65536; d++) cnt[d + 1] += cnt[d];
        for (size_t q = 0; q < n; q++) {
            uint32_t at = cnt[(a[q] >> sh) & 0xffff]++;
            b[at] = a[q];
            ib[at] = ia[q];
        }
        a.swap(b);
        ia.swap(ib);
    }
    std::vector<K> out(n);
    for (size_t q = 0; q < n; q++) out[q] = keys[ia[q]];
    keys.swap(out);
}

// smallest box index reported by any thread (-1: none)
struct FirstBad {
    std::atomic<int64_t> v{-1};
    void add(int64_t b) {
        int64_t cur = v.load();
        while ((cur < 0 || b < cur) && !v.compare_exchange_weak(cur, b)) {
        }
    }
};

struct Key {
    int32_t level, tree;
    uint64_t m;
    int32_t src;
    bool operator<(const Key &o) const {
        return std::tie(level, tree, m) < std::tie(o.level, o.tree, o.m);
    }
    bool same(const Key &o) const { return level == o.level && tree == o.tree && m == o.m; }
};

thread_local char g_buf[256];  // error text, per thread like mg_last_error()

}  // namespace

int build_tree(mg_tree *t, const mg_domain *dom, int64_t n, const int32_t *level,
               const int32_t *ijk, const int32_t *tree) {
    if (n <= 0 || n > (int64_t)1 << 30 || !level || !ijk || !dom || !(dom->len > 0)) {
        set_error("mg_tree_create: invalid arguments");
        return MG_EINVAL;
    }
    int dirichlet = 0;
    for (int d = 0; d < 6; d++) {
        if (dom->bc_type[d] != MG_DIRICHLET && dom->bc_type[d] != MG_NEUMANN) {
            snprintf(g_buf, sizeof g_buf, "face %d: unknown boundary type %d", d, dom->bc_type[d]);
            set_error(g_buf);
            return MG_EINVAL;
        }
        dirichlet += dom->bc_type[d] == MG_DIRICHLET;
    }
    if (!dirichlet) {
        set_error("all faces Neumann: the problem is singular");
        return MG_EINVAL;
    }
    t->dom = *dom;

    std::vector<Key> keys((size_t)n);
    int ntree = 0;
    for (int64_t b = 0; b < n; b++) {
        int32_t l = level[b], tr = tree ? tree[b] : 0;
        int32_t i = ijk[3 * b], j = ijk[3 * b + 1], k = ijk[3 * b + 2];
        int32_t lim = (l >= 1 && l <= kMaxLevel) ? (1 << (l - 1)) : 0;
        if (l < 1 || l > kMaxLevel || tr < 0 || tr > 65535 || i < 0 || j < 0 || k < 0 ||
            i >= lim || j >= lim || k >= lim) {
            snprintf(g_buf, sizeof g_buf, "box %lld: level %d / coordinates (%d,%d,%d) / tree %d out of range",
                     (long long)b, l, i, j, k, tr);
            set_error(g_buf);
            return MG_EINVAL;
        }
        ntree = std::max(ntree, tr + 1);
        keys[b] = Key{l, tr, morton(i, j, k), (int32_t)b};
    }
    if (!std::is_sorted(keys.begin(), keys.end())) sort_keys(keys);
    for (int64_t b = 1; b < n; b++)
        if (keys[b].same(keys[b - 1])) {
            snprintf(g_buf, sizeof g_buf, "boxes %d and %d are duplicates", keys[b - 1].src, keys[b].src);
            set_error(g_buf);
            return MG_EINVAL;
        }

    t->n = n;
    t->ntree = ntree;
    t->order.resize(n);
    t->lev.resize(n);
    t->tid.resize(n);
    t->ijk.resize(3 * n);
    for (int64_t b = 0; b < n; b++) {
        int32_t s = keys[b].src;
        t->order[b] = s;
        t->lev[b] = level[s];
        t->tid[b] = tree ? tree[s] : 0;
        for (int a = 0; a < 3; a++) t->ijk[3 * b + a] = ijk[3 * s + a];
    }
    t->nlev = t->lev[n - 1];
    for (int l = 0; l <= kMaxLevel + 1; l++) t->lstart[l] = 0;
    {
        int64_t b = 0;
        for (int l = 1; l <= kMaxLevel + 1; l++) {
            t->lstart[l - 1] = b;  // level l starts at lstart[l-1]
            while (b < n && t->lev[b] == l) b++;
        }
        t->lstart[kMaxLevel + 1] = n;
    }
    // From here on, boxes of level l occupy [lstart[l-1], lstart[l]).
    auto lbegin = [&](int l) { return t->lstart[l - 1]; };
    auto lend = [&](int l) { return l <= kMaxLevel ? t->lstart[l] : n; };

    // roots: trees 0..T-1 each own a level-1 box
    if (lend(1) - lbegin(1) != ntree) {
        snprintf(g_buf, sizeof g_buf, "%d trees but %lld root boxes", ntree,
                 (long long)(lend(1) - lbegin(1)));
        set_error(g_buf);
        return MG_ETOPO;
    }
    for (int64_t b = lbegin(1); b < lend(1); b++)
        if (t->tid[b] != b - lbegin(1)) {
            snprintf(g_buf, sizeof g_buf, "tree %lld has no root box", (long long)(b - lbegin(1)));
            set_error(g_buf);
            return MG_ETOPO;
        }

    // parents by binary search in the previous level's sorted range
    t->parent.assign(n, -1);
    t->child.assign(8 * n, -1);
    // (the parents of a level's boxes, in order, are non-decreasing in the
    // previous level's order: one forward walk)
    for (int l = 2; l <= t->nlev; l++) {
        int64_t pq = lbegin(l - 1), pe = lend(l - 1);
        for (int64_t b = lbegin(l); b < lend(l); b++) {
            Key want{l - 1, t->tid[b], keys[b].m >> 3, 0};
            while (pq < pe && keys[pq] < want) pq++;
            if (pq == pe || !keys[pq].same(want)) {
                snprintf(g_buf, sizeof g_buf, "box %d (level %d) has no parent", t->order[b], l);
                set_error(g_buf);
                return MG_ETOPO;
            }
            int32_t p = (int32_t)pq;
            int oct = (int)(keys[b].m & 7);  // (i&1) + 2(j&1) + 4(k&1)
            t->parent[b] = p;
            t->child[8 * p + oct] = (int32_t)b;
        }
    }
    {
        FirstBad bad;
        parallel_for(n, [&](int64_t lo, int64_t hi) {
            for (int64_t b = lo; b < hi; b++) {
                int c = 0;
                for (int q = 0; q < 8; q++) c += t->child[8 * b + q] >= 0;
                if (c != 0 && c != 8) bad.add(b);
            }
        });
        if (bad.v >= 0) {
            int64_t b = bad.v;
            int c = 0;
            for (int q = 0; q < 8; q++) c += t->child[8 * b + q] >= 0;
            snprintf(g_buf, sizeof g_buf, "box %d has %d of its 8 children", t->order[b], c);
            set_error(g_buf);
            return MG_ETOPO;
        }
    }

    // 27-neighbourhood tables level by level: entry (ox,oy,oz) of box b is the
    // same-level box at ijk + o, -1 when that position is covered only by a
    // coarser leaf, -2 outside the domain.  A level-l box whose neighbour
    // position is not covered down to level l-1 violates proper nesting.
    RawArray<int32_t> n27;
    n27.reset((size_t)27 * n);
    for (int64_t b = lbegin(1); b < lend(1); b++)
        for (int o = 0; o < 27; o++) n27[27 * b + o] = o == 13 ? (int32_t)b : -2;
    // For a box whose coordinates have parities par (bit a: coordinate a
    // odd) and a direction oi, the containing level-(l-1) box's direction
    // from the parent and the octant of the neighbour position in it depend
    // on par and oi only: tabulated once.
    struct Up27 {
        uint8_t up, oct;
    };
    static const auto up_tab = [] {
        std::array<std::array<Up27, 27>, 8> tab{};
        for (int par = 0; par < 8; par++)
            for (int oi = 0; oi < 27; oi++) {
                int o[3] = {oi % 3 - 1, (oi / 3) % 3 - 1, oi / 9 - 1}, up = 0, oct = 0, mul = 1;
                for (int a = 0; a < 3; a++) {
                    int s = ((par >> a) & 1) + o[a];  // position relative to the parent's first child, -1..2
                    up += mul * ((s + 2) / 2);        // -1, 0, +1 parent directions -> 0, 1, 2
                    oct |= (s & 1) << a;
                    mul *= 3;
                }
                tab[par][oi] = Up27{(uint8_t)up, (uint8_t)oct};
            }
        return tab;
    }();
    for (int l = 2; l <= t->nlev; l++) {
        int32_t lim = 1 << (l - 1);
        // fills the 27 entries of box b; returns the first direction that
        // violates nesting, or -1
        auto fill27 = [&](int64_t b) {
            const int32_t *P27 = &n27[27 * (int64_t)t->parent[b]];
            const int32_t *B = &t->ijk[3 * b];
            const auto &tab = up_tab[(B[0] & 1) | ((B[1] & 1) << 1) | ((B[2] & 1) << 2)];
            // directions along each axis that leave the domain
            const bool lo[3] = {B[0] == 0, B[1] == 0, B[2] == 0};
            const bool hi[3] = {B[0] == lim - 1, B[1] == lim - 1, B[2] == lim - 1};
            int32_t *out = &n27[27 * b];
            for (int oi = 0; oi < 27; oi++) {
                int ox = oi % 3, oy = (oi / 3) % 3, oz = oi / 9;
                if ((ox == 0 && lo[0]) || (ox == 2 && hi[0]) || (oy == 0 && lo[1]) || (oy == 2 && hi[1]) ||
                    (oz == 0 && lo[2]) || (oz == 2 && hi[2])) {
                    out[oi] = -2;
                    continue;
                }
                int32_t cont = P27[tab[oi].up];
                if (cont < 0) return oi;
                out[oi] = t->child[8 * (int64_t)cont + tab[oi].oct];  // -1: coarser leaf
            }
            return -1;
        };
        // The 8 children of the k-th refined box P of level l-1 are the boxes
        // 8k .. 8k+7 of level l in octant order, and a child's parities are
        // its octant.  So the entries of fill27 for all eight follow from one
        // value per direction u of P's 27-neighbourhood: the first child of
        // the level-(l-1) box there (children are consecutive in octant
        // order, so child oct is first + oct), -1 for a leaf, -2 outside the
        // domain (a level-l position is outside exactly when its level-(l-1)
        // position is), -3 in the domain but not covered down to level l-1
        // (a nesting violation).
        auto fill_octet = [&](int64_t c0) {
            const int32_t *P27 = &n27[27 * (int64_t)t->parent[c0]];
            int32_t first[27];
            for (int u = 0; u < 27; u++) {
                int32_t cont = P27[u];
                first[u] = cont == -2 ? -2 : cont < 0 ? -3 : t->child[8 * (int64_t)cont];
            }
            for (int o = 0; o < 8; o++) {
                const auto &tab = up_tab[o];
                int32_t *outp = &n27[27 * (c0 + o)];
                bool bad_o = false;
                for (int oi = 0; oi < 27; oi++) {
                    int32_t f = first[tab[oi].up];
                    outp[oi] = f >= 0 ? f + tab[oi].oct : f;
                    bad_o = bad_o || f == -3;
                }
                if (bad_o) return c0 + o;
            }
            return (int64_t)-1;
        };
        FirstBad bad;
        int64_t l0 = lbegin(l);
        parallel_for(lend(l) - l0, [&](int64_t lo, int64_t hi) {
            // octets whose first box lies in [lo, hi)
            for (int64_t q = (lo + 7) / 8; q < (hi + 7) / 8; q++) {
                int64_t bb = fill_octet(l0 + 8 * q);
                if (bb >= 0) bad.add(bb);
            }
        });
        if (bad.v >= 0) {
            int64_t bb = bad.v;
            int oi = fill27(bb);
            snprintf(g_buf, sizeof g_buf, "box %d (level %d) violates 2:1 nesting towards (%d,%d,%d)",
                     t->order[bb], l, oi % 3 - 1, (oi / 3) % 3 - 1, oi / 9 - 1);
            set_error(g_buf);
            return MG_ENESTING;
        }
    }
    // face tables (the 27-neighbourhood is kept for the regrid planner)
    static const int face_oi[6] = {12, 14, 10, 16, 4, 22};
    t->nbr.assign(6 * n, -2);
    t->cfq.assign(6 * n, -1);
    parallel_for(n, [&](int64_t lo, int64_t hi) {
    for (int64_t b = lo; b < hi; b++) {
        for (int d = 0; d < 6; d++) {
            int32_t v = n27[27 * b + face_oi[d]];
            t->nbr[6 * b + d] = v;
            if (v == -1) {
                int a = d >> 1, s = d & 1;
                int32_t p = t->parent[b];
                const int32_t *B = &t->ijk[3 * b];
                int up[3] = {0, 0, 0};
                up[a] = ((B[a] & 1) + (s ? 1 : -1) + 2) / 2 - 1;
                t->cfq[6 * b + d] = n27[27 * (int64_t)p + (up[0] + 1) + 3 * (up[1] + 1) + 9 * (up[2] + 1)];
            }
        }
    }
    });
    // refinement-boundary face slots, grouped by level
    t->cfslot.assign(6 * n, -1);
    t->slots.clear();
    for (int l = 1; l <= kMaxLevel + 1; l++) {
        t->sstart[l] = (int64_t)t->slots.size() / 2;
        if (l > t->nlev) continue;
        for (int64_t b = lbegin(l); b < lend(l); b++)
            for (int d = 0; d < 6; d++)
                if (t->nbr[6 * b + d] == -1) {
                    t->cfslot[6 * b + d] = (int32_t)(t->slots.size() / 2);
                    t->slots.push_back((int32_t)b);
                    t->slots.push_back(d);
                }
    }
    t->sstart[0] = 0;
    t->nslot = (int64_t)t->slots.size() / 2;
    // per slot, the coarse-side indices of its c_hat: the coarser box Q, the
    // base coordinates of the face's quarter of Q along the two tangential
    // axes, and Q's face neighbours across them (-t1, +t1, -t2, +t2)
    t->slotx.assign((size_t)8 * t->nslot, 0);
    parallel_for(t->nslot, [&](int64_t lo, int64_t hi) {
    for (int64_t q = lo; q < hi; q++) {
        int64_t b = t->slots[2 * q];
        int d = t->slots[2 * q + 1], a = d >> 1, t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
        int32_t Q = t->cfq[6 * b + d];
        int32_t *x = &t->slotx[8 * q];
        x[0] = Q;
        x[1] = 4 * (t->ijk[3 * b + t1] & 1);
        x[2] = 4 * (t->ijk[3 * b + t2] & 1);
        x[3] = t->nbr[6 * (int64_t)Q + 2 * t1];
        x[4] = t->nbr[6 * (int64_t)Q + 2 * t1 + 1];
        x[5] = t->nbr[6 * (int64_t)Q + 2 * t2];
        x[6] = t->nbr[6 * (int64_t)Q + 2 * t2 + 1];
    }
    });
    // per-level lists of refined and leaf boxes
    t->refined.clear();
    t->leaf.clear();
    for (int l = 1; l <= kMaxLevel + 1; l++) {
        t->rstart[l] = (int64_t)t->refined.size();
        t->fstart[l] = (int64_t)t->leaf.size();
        if (l > t->nlev) continue;
        for (int64_t b = lbegin(l); b < lend(l); b++)
            (t->child[8 * b] >= 0 ? t->refined : t->leaf).push_back((int32_t)b);
    }
    t->nleaf = (int64_t)t->leaf.size();
    t->leafpos.assign(n, -1);  // position in the leaf list, -1 for boxes with children
    for (int64_t q = 0; q < t->nleaf; q++) t->leafpos[t->leaf[q]] = (int32_t)q;
    // per-level lists of the leaf boxes whose phi a down-leg copies into
    // phi_old.  The prolongation into level l+1 reads phi - phi_old of level l
    // only on the parents of level-(l+1) boxes and one cell layer around them,
    // which lies in those parents' face and edge neighbours; the parents' own
    // cells (all covered) get phi_old from the restriction.  So a leaf box
    // needs the copy only when a same-level face or edge neighbour has children.
    t->oldcp.clear();
    for (int l = 1; l <= kMaxLevel + 1; l++) {
        t->ostart[l] = (int64_t)t->oldcp.size();
        if (l > t->nlev) continue;
        // the 6 face and 12 edge directions of the 27-neighbourhood
        static const int fe[18] = {1, 3, 4, 5, 7, 9, 10, 11, 12, 14, 15, 16, 17, 19, 21, 22, 23, 25};
        for (int64_t q = t->fstart[l]; q < (int64_t)t->leaf.size() && t->lev[t->leaf[q]] == l; q++) {
            int64_t b = t->leaf[q];
            const int32_t *N27 = &n27[27 * b];
            for (int e = 0; e < 18; e++) {
                int32_t nb = N27[fe[e]];
                if (nb >= 0 && t->child[8 * (int64_t)nb] >= 0) {
                    t->oldcp.push_back((int32_t)b);
                    break;
                }
            }
        }
    }
    // leaf boxes whose parent cells a stopping test can read: a residual or a
    // c_hat reads a covered cell only next to a leaf cell of its own level,
    // so only across the parent's outer faces on the child's side, and only
    // where the parent's neighbour there is a leaf box (a refined box has
    // all 8 children and no refinement-boundary face)
    t->cleaf.clear();
    t->cmask.assign(n, 0);
    for (int64_t q = 0; q < t->nleaf; q++) {
        int64_t b = t->leaf[q];
        if (t->lev[b] < 2) continue;
        int64_t p = t->parent[b];
        for (int a = 0; a < 3; a++) {
            int32_t nb = t->nbr[6 * p + 2 * a + (t->ijk[3 * b + a] & 1)];
            if (nb >= 0 && t->child[8 * (int64_t)nb] < 0) {
                t->cleaf.push_back((int32_t)b);
                t->cmask[b] = 1;
                break;
            }
        }
    }
    // the list follows the leaf list's level order: level l's entries are
    // [cstart[l], cstart[l+1])
    for (int l = 0; l <= kMaxLevel + 1; l++) {
        int64_t c = 0;
        while (c < (int64_t)t->cleaf.size() && t->lev[t->cleaf[c]] < l) c++;
        t->cstart[l] = c;
    }
    // leaf-list positions grouped by tree, ascending inside each tree (the
    // order of the per-tree norm reduction)
    t->tree_off.assign(ntree + 1, 0);
    for (int64_t q = 0; q < t->nleaf; q++) t->tree_off[t->tid[t->leaf[q]] + 1]++;
    for (int tr = 0; tr < ntree; tr++) t->tree_off[tr + 1] += t->tree_off[tr];
    t->leaf_tree.assign(t->nleaf, 0);
    {
        std::vector<int32_t> fill(t->tree_off.begin(), t->tree_off.end() - 1);
        for (int64_t q = 0; q < t->nleaf; q++) t->leaf_tree[fill[t->tid[t->leaf[q]]]++] = (int32_t)q;
    }
    // chunks of at most kReduceChunk leaf positions inside one tree, for the
    // first stage of the per-tree norm reduction
    t->chunk.clear();
    t->choff.assign(ntree + 1, 0);
    for (int tr = 0; tr < ntree; tr++) {
        for (int32_t b = t->tree_off[tr]; b < t->tree_off[tr + 1]; b += kReduceChunk) {
            t->chunk.push_back(tr);
            t->chunk.push_back(b);
            t->chunk.push_back(std::min<int32_t>(b + kReduceChunk, t->tree_off[tr + 1]));
        }
        t->choff[tr + 1] = (int32_t)(t->chunk.size() / 3);
    }
    // first level-2 box of each tree (its 8 children of the root, in octant
    // order), or -1 for a tree that is a single root box; the one-launch
    // bottom of the V-cycle needs level 2 free of refinement boundaries,
    // which holds because a refined root has all 8 children
    t->root2.assign(ntree, -1);
    for (int tr = 0; tr < ntree; tr++) t->root2[tr] = t->child[8 * (lbegin(1) + tr)];
    t->bottom_ok = t->nlev >= 2 && t->sstart[3] == t->sstart[2];
    t->n27 = std::move(n27);
    t->beff_tree.assign(ntree, 0.0);
    t->rel_tree.assign(ntree, 0.0);
    root_eigen(dom->bc_type, t->eig);

    // workspace layout
    auto align = [](int64_t x) { return (x + 255) & ~(int64_t)255; };
    int64_t o = 0;
    auto take = [&](int64_t bytes) { int64_t r = o; o = align(o + std::max<int64_t>(bytes, 8)); return r; };
    t->off.nbr = take(24 * n);
    t->off.cfslot = take(24 * n);
    t->off.cfq = take(24 * n);
    t->off.n27 = take(108 * n);
    t->off.ijk = take(16 * n);
    t->off.parent = take(4 * n);
    t->off.refined = take(4 * (int64_t)t->refined.size());
    t->off.leaf = take(4 * t->nleaf);
    t->off.cleaf = take(4 * (int64_t)t->cleaf.size());
    t->off.oldcp = take(4 * (int64_t)t->oldcp.size());
    t->off.leafpos = take(4 * n);
    t->off.cmask = take(4 * n);
    t->off.slots = take(8 * t->nslot);
    t->off.slotx = take(32 * t->nslot);
    t->off.leaf_tree = take(4 * t->nleaf);
    t->off.tree_off = take(4 * (int64_t)(ntree + 1));
    t->off.chunk = take(4 * (int64_t)t->chunk.size());
    t->off.choff = take(4 * (int64_t)(ntree + 1));
    t->off.part2 = take(16 * (int64_t)(t->chunk.size() / 3));
    t->off.isleaf = take(4 * n);
    t->off.tid = take(4 * n);
    t->off.root2 = take(4 * (int64_t)ntree);
    t->off.eig = take(8 * (3 * 64 + 3 * 8));
    t->off.xt = take(192 * n);  // last of the tables: formed on the GPU, not uploaded
    t->off.phi = take(8 * kCells * n);
    t->off.rhs = take(8 * kCells * n);
    t->off.old = take(8 * kCells * n);
    t->off.chat = take(8 * 64 * t->nslot);
    t->off.bcval = dom->per_cell_bc ? take(8 * 6 * 64 * n) : -1;
    t->off.partial = take(16 * t->nleaf);
    t->off.result = take(8 * 4 * (int64_t)ntree);
    t->off.e32 = take(4 * kCells * n);
    t->off.r32 = take(4 * kCells * n);
    t->off.old32 = take(4 * kCells * n);
    t->off.chat32 = take(4 * 64 * t->nslot);
    t->off.swp = take(8 * kCells * n);
    t->off.fas = take(8 * kCells * n);
    {  // padded correction blocks of the refined boxes of one level
        int64_t mref = 0;
        for (int l = 1; l <= t->nlev; l++) mref = std::max(mref, t->rstart[l + 1] - t->rstart[l]);
        t->off.dpad = take(8 * 1000 * mref);
    }
    t->off.total = o;
    return MG_OK;
}

// Eigen-decomposition of the 1-D second-difference matrix of the root box
// along each axis (-2 on the diagonal, 1 off it; the end entries become -3
// for a Dirichlet face and -1 for a Neumann face), by cyclic Jacobi rotations.
// Used by the exact root solve (fast diagonalisation, Lynch, Rice & Thomas
// 1964): A = (T_x (+) T_y (+) T_z) / h^2 is diagonal in the product basis.
void root_eigen(const int32_t bc_type[6], double *eig) {
    for (int a = 0; a < 3; a++) {
        double A[8][8] = {{0}}, V[8][8] = {{0}};
        for (int i = 0; i < 8; i++) {
            A[i][i] = -2.0;
            if (i > 0) A[i][i - 1] = 1.0;
            if (i < 7) A[i][i + 1] = 1.0;
            V[i][i] = 1.0;
        }
        A[0][0] += bc_type[2 * a] == MG_DIRICHLET ? -1.0 : 1.0;
        A[7][7] += bc_type[2 * a + 1] == MG_DIRICHLET ? -1.0 : 1.0;
        for (int sweep = 0; sweep < 100; sweep++) {
            double off = 0.0;
            for (int p = 0; p < 8; p++)
                for (int q = p + 1; q < 8; q++) off += A[p][q] * A[p][q];
            if (off < 1e-40) break;
            for (int p = 0; p < 8; p++)
                for (int q = p + 1; q < 8; q++) {
                    if (std::fabs(A[p][q]) < 1e-300) continue;
                    double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                    double tt = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                    double c = 1.0 / std::sqrt(tt * tt + 1.0), s = tt * c;
                    for (int k = 0; k < 8; k++) {  // A <- A J
                        double akp = A[k][p], akq = A[k][q];
                        A[k][p] = c * akp - s * akq;
                        A[k][q] = s * akp + c * akq;
                    }
                    for (int k = 0; k < 8; k++) {  // A <- J^T A
                        double apk = A[p][k], aqk = A[q][k];
                        A[p][k] = c * apk - s * aqk;
                        A[q][k] = s * apk + c * aqk;
                    }
                    for (int k = 0; k < 8; k++) {  // V <- V J
                        double vkp = V[k][p], vkq = V[k][q];
                        V[k][p] = c * vkp - s * vkq;
                        V[k][q] = s * vkp + c * vkq;
                    }
                }
        }
        for (int i = 0; i < 8; i++)
            for (int m = 0; m < 8; m++) eig[a * 64 + i * 8 + m] = V[i][m];  // row i, eigenvector m
        for (int m = 0; m < 8; m++) eig[192 + a * 8 + m] = A[m][m];
    }
}

}  // namespace mg
