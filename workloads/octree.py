"""Box lists for synthetic octree workloads.

A box is (level, i, j, k, tree): level 1 is the single 8^3 root box of a tree,
a box at level l has integer coordinates 0 <= i, j, k < 2^(l-1), and its 8
children at level l+1 have coordinates 2*(i, j, k) + (0|1).  Refinement follows
the paper's octree description (section 2.1.1): a refined box is covered by all
2^3 children, and neighbouring boxes differ by at most one level (proper
nesting, taken over all 26 neighbours).

This module only *generates* box lists.  Validation, ordering and every table
the solvers use are built independently by each solver from these coordinates.
"""
import numpy as np

OFFSETS26 = np.array([(a, b, c) for c in (-1, 0, 1) for b in (-1, 0, 1)
                      for a in (-1, 0, 1) if (a, b, c) != (0, 0, 0)], dtype=np.int64)
CHILD_OFFSETS = np.array([(a, b, c) for c in (0, 1) for b in (0, 1) for a in (0, 1)],
                         dtype=np.int64)

_SH = 20  # bits per coordinate in a packed key


def pack(ijk):
    ijk = np.asarray(ijk, dtype=np.int64)
    return (ijk[..., 0] << (2 * _SH)) | (ijk[..., 1] << _SH) | ijk[..., 2]


def unpack(keys):
    keys = np.asarray(keys, dtype=np.int64)
    m = (1 << _SH) - 1
    return np.stack([(keys >> (2 * _SH)) & m, (keys >> _SH) & m, keys & m], axis=-1)


class BoxList:
    """Flat arrays describing a forest of octrees (in no particular order)."""

    def __init__(self, level, ijk, tree=None):
        self.level = np.ascontiguousarray(level, dtype=np.int32)
        self.ijk = np.ascontiguousarray(np.asarray(ijk).reshape(-1, 3), dtype=np.int32)
        n = self.level.shape[0]
        if tree is None:
            tree = np.zeros(n, dtype=np.int32)
        self.tree = np.ascontiguousarray(tree, dtype=np.int32)

    @property
    def n(self):
        return int(self.level.shape[0])

    def leaf_mask(self):
        """True for boxes that have no children in the list."""
        def key(tree, level, ijk):
            # 14 bits per coordinate (levels <= 15), 4 for the level, 17 for the tree
            ijk = np.asarray(ijk, dtype=np.int64)
            return (tree.astype(np.int64) << 46) | (level.astype(np.int64) << 42) \
                | (ijk[:, 0] << 28) | (ijk[:, 1] << 14) | ijk[:, 2]
        own = key(self.tree, self.level, self.ijk)
        has_parent = self.level > 1
        par = key(self.tree, self.level - 1, self.ijk.astype(np.int64) >> 1)
        return ~np.isin(own, par[has_parent])

    def n_leaf_cells(self, n_cell=8):
        return int(self.leaf_mask().sum()) * n_cell ** 3

    def shuffled(self, seed):
        """Same boxes in a seeded random order (exercises the solvers' sorting)."""
        p = np.random.default_rng(seed).permutation(self.n)
        return BoxList(self.level[p], self.ijk[p], self.tree[p])

    @staticmethod
    def concat(lists):
        return BoxList(np.concatenate([b.level for b in lists]),
                       np.concatenate([b.ijk for b in lists]),
                       np.concatenate([b.tree for b in lists]))


def uniform_boxes(top_level, tree=0):
    """Every box of levels 1..top_level (a uniform grid of 8*2^(top-1) cells)."""
    lv, ij = [], []
    for l in range(1, top_level + 1):
        n = 1 << (l - 1)
        g = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"),
                     axis=-1).reshape(-1, 3)[:, ::-1]  # x fastest
        lv.append(np.full(len(g), l, dtype=np.int32))
        ij.append(g.astype(np.int32))
    lv = np.concatenate(lv)
    return BoxList(lv, np.concatenate(ij), np.full(len(lv), tree, dtype=np.int32))


class _Forest:
    """Incremental 2:1-balanced refinement of one tree (26-neighbour nesting)."""

    def __init__(self, base_level, max_level):
        self.max_level = max_level
        self.boxes = {l: set() for l in range(1, max_level + 1)}
        self.refined = {l: set() for l in range(1, max_level + 1)}
        self.boxes[1].add(0)
        for l in range(1, base_level):
            for k in list(self.boxes[l]):
                self._add_children(l, k)

    def _add_children(self, l, key):
        self.refined[l].add(key)
        ch = pack((unpack(key)[None, :] * 2) + CHILD_OFFSETS)
        self.boxes[l + 1].update(ch.tolist())

    def ensure_refined(self, l, key):
        """Refine box (l, key), first refining coarser boxes so that all 26
        neighbours at level l exist (then its children are properly nested)."""
        if key in self.refined[l] or l >= self.max_level:
            return
        n = 1 << (l - 1)
        nb = unpack(key)[None, :] + OFFSETS26
        ok = np.all((nb >= 0) & (nb < n), axis=1)
        for p in pack(nb[ok]).tolist():
            if p not in self.boxes[l]:
                self.ensure_refined(l - 1, int(pack(unpack(p) >> 1)))
        self._add_children(l, key)

    def box_list(self, tree=0):
        lv, ij = [], []
        for l in range(1, self.max_level + 1):
            ks = np.array(sorted(self.boxes[l]), dtype=np.int64)
            if len(ks) == 0:
                continue
            lv.append(np.full(len(ks), l, dtype=np.int32))
            ij.append(unpack(ks).astype(np.int32))
        lv = np.concatenate(lv)
        return BoxList(lv, np.concatenate(ij), np.full(len(lv), tree, dtype=np.int32))


def refine_by_score(base_level, max_level, score_fn, threshold, tree=0):
    """Build a balanced tree: uniform up to ``base_level``, then a box at level
    l < max_level is refined when ``score_fn(l, ijk) > threshold``.

    ``score_fn`` may be memoised by the caller; it returns one float per box.
    """
    f = _Forest(base_level, max_level)
    for l in range(base_level, max_level):
        seen = set()
        while True:
            todo = np.array(sorted(f.boxes[l] - seen - f.refined[l]), dtype=np.int64)
            seen.update(todo.tolist())
            if len(todo) == 0:
                break
            s = score_fn(l, unpack(todo))
            for key in todo[s > threshold].tolist():
                f.ensure_refined(l, key)
    return f.box_list(tree)


def refine_boxes_explicit(base_level, refine, max_level=12, tree=0):
    """Balanced tree from an explicit list of (level, i, j, k) boxes to refine."""
    f = _Forest(base_level, max_level)

    def make_exist(l, key):
        if key in f.boxes[l]:
            return
        par = int(pack(unpack(key) >> 1))
        make_exist(l - 1, par)
        f.ensure_refined(l - 1, par)

    for l, i, j, k in sorted(refine):
        key = int(pack(np.array([i, j, k])))
        make_exist(l, key)
        f.ensure_refined(l, key)
    return f.box_list(tree)
