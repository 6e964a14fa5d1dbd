"""Mesh adaptation (paper section 2.5): refinement scores, the regrid plan
and the transfer of the potential to the new tree.

CPU (no GPU):
* the library's planner (mg_regrid_plan, host code) against a second,
  independent implementation of the same rules written here (refine a leaf
  when |b| h^2 > c3 in it or within 3 cells in a same-level leaf neighbour;
  drop quiet leaf octets unless a box two levels finer would touch the
  parent; restore 2:1 nesting over 26 neighbours), on random and on
  structured scores; its output is a valid tree for both the library and the
  oracle;
* the oracle's transfer: exact for linear potentials across refinement,
  derefinement and nesting refinement; the identity on an unchanged tree; and
  a new box checked cell by cell against the stencil evaluated by hand.
* the plan from the per-box values of the criterion (mg_regrid_plan_near)
  against the same rules and against the plan from the 27 scores.
GPU: the scores against numpy, the per-box values against the rule applied
to those scores, the transfer against the oracle, and a whole regrid step
(plan, transfer, warm V-cycles) against the oracle."""
import itertools

import numpy as np
import pytest

import oracle as O
from paper_1708_08434_amd import mg as M
from workloads import streamer_small, refine_boxes_explicit, uniform_boxes
from workloads.octree import BoxList
from tests import _geom as G

OFFS = [o for o in itertools.product((-1, 0, 1), repeat=3) if o != (0, 0, 0)]


def reg(o):
    return (o[0] + 1) + 3 * (o[1] + 1) + 9 * (o[2] + 1)


def numpy_scores(level, ijk, rhs):
    """[n][27] region maxima of |b| h^2 (b natural [box][k][j][i])."""
    h = 1.0 / (8.0 * 2.0 ** (np.asarray(level) - 1))
    v = np.abs(rhs) * (h * h)[:, None, None, None]
    sl = {-1: slice(0, 3), 0: slice(0, 8), 1: slice(5, 8)}
    out = np.zeros((len(level), 27))
    for sz, sy, sx in itertools.product((-1, 0, 1), repeat=3):
        out[:, reg((sx, sy, sz))] = v[:, sl[sz], sl[sy], sl[sx]].reshape(len(level), -1).max(axis=1)
    return out


def children(k):
    t, l, i, j, kk = k
    return [(t, l + 1, 2 * i + a, 2 * j + b, 2 * kk + c) for c in (0, 1) for b in (0, 1) for a in (0, 1)]


def ref_plan(level, ijk, tree, scores, c3, deref, max_level, h_deref=np.inf, length=1.0):
    keys = [(int(t), int(l), int(c[0]), int(c[1]), int(c[2])) for l, c, t in zip(level, ijk, tree)]
    idx = {k: q for q, k in enumerate(keys)}
    leaf = {k: children(k)[0] not in idx for k in keys}

    def nbrs(k):
        t, l, i, j, kk = k
        lim = 1 << (l - 1)
        for o in OFFS:
            p = (i + o[0], j + o[1], kk + o[2])
            if min(p) >= 0 and max(p) < lim and (t, l) + p in idx:
                yield o, (t, l) + p

    def hot(k, thr):
        if scores[idx[k]][13] > thr:
            return True
        return any(leaf[n] and scores[idx[n]][reg(tuple(-x for x in o))] > thr for o, n in nbrs(k))

    refine = {k for k in keys if leaf[k] and k[1] < max_level and hot(k, c3)}
    drop = set()
    for k in keys:
        if leaf[k] or not length / (8 * 2 ** k[1]) < h_deref:   # children's cell size
            continue
        ok = all(leaf[c] and c not in refine and not hot(c, deref * c3) for c in children(k))
        if ok:
            for _, n in nbrs(k):
                if not leaf[n] and any(not leaf[c] or c in refine for c in children(n)):
                    ok = False
                    break
        if ok:
            drop.add(k)
    out = set()
    for k in keys:
        t, l, i, j, kk = k
        if l >= 2 and (t, l - 1, i >> 1, j >> 1, kk >> 1) in drop:
            continue
        out.add(k)
        if k in refine:
            out.update(children(k))
    changed = True
    while changed:
        changed = False
        for k in list(out):
            t, l, i, j, kk = k
            if l < 3:
                continue
            lim = 1 << (l - 1)
            for o in OFFS:
                p = (i + o[0], j + o[1], kk + o[2])
                if min(p) < 0 or max(p) >= lim or (t, l - 1, p[0] >> 1, p[1] >> 1, p[2] >> 1) in out:
                    continue
                for m in range(l - 2, 0, -1):
                    sh = l - m
                    a = (t, m, p[0] >> sh, p[1] >> sh, p[2] >> sh)
                    if a in out:
                        out.update(children(a))
                        changed = True
                        break
    return out


def forest_boxes():
    a = refine_boxes_explicit(2, [(2, 0, 0, 0), (3, 1, 1, 1), (3, 0, 1, 0), (4, 2, 2, 2)], tree=0)
    b = refine_boxes_explicit(2, [(2, 1, 1, 1)], tree=1)
    return BoxList.concat([a, b])


@pytest.mark.parametrize("seed,h_deref", [(0, np.inf), (1, np.inf), (2, np.inf), (3, np.inf),
                                          (0, 1 / 40), (2, 1 / 40)])
def test_plan_matches_the_rules_on_random_scores(seed, h_deref):
    bl = forest_boxes()
    rng = np.random.default_rng(seed)
    # per-box magnitudes over four decades, so that quiet octets exist
    sc = rng.lognormal(0.0, 1.5, (bl.n, 27)) * 10.0 ** rng.uniform(-4, 0, (bl.n, 1))
    sc[:, 13] = np.maximum(sc[:, 13], sc.max(axis=1))  # the whole box bounds its regions
    c3 = float(np.quantile(sc[:, 13], 0.98))
    h = M.mg_tree_create(M.make_domain(), bl.level, bl.ijk, bl.tree)
    try:
        order = M.mg_tree_index(h, M.MG_IDX_ORDER, bl.n).reshape(-1)
        canon = sc[order]                       # scores of canonical box q = caller box order[q]
        lv, ij, tr = M.mg_regrid_plan(h, canon, c3, 0.3, 6, h_deref)
    finally:
        M.mg_tree_destroy(h)
    got = {(int(t), int(l), *map(int, c)) for l, c, t in zip(lv, ij, tr)}
    want = ref_plan(bl.level, bl.ijk, bl.tree, sc, c3, 0.3, 6, h_deref)
    old = {(int(t), int(l), *map(int, c)) for l, c, t in zip(bl.level, bl.ijk, bl.tree)}
    assert got == want, (len(got ^ want), sorted(got ^ want)[:5])
    assert got - old                             # refined somewhere
    if seed < 3 and h_deref == np.inf:
        assert old - got                         # and derefined somewhere
    # removed boxes are finer than h_deref (cell size 1 / (8 * 2^(level-1)))
    assert all(1.0 / (8 * 2 ** (k[1] - 1)) < h_deref for k in old - got)
    if h_deref < np.inf:
        assert got != ref_plan(bl.level, bl.ijk, bl.tree, sc, c3, 0.3, 6) or seed >= 3
    # valid trees for the library and the oracle
    h2 = M.mg_tree_create(M.make_domain(), lv, ij, tr)
    M.mg_tree_destroy(h2)
    O.OracleTree(lv, ij, tr)


def near_of(level, ijk, tree, scores):
    """Per box, the value the criterion tests (written from the rule): for a
    leaf, the largest score over its cells and the cells of its same-level
    leaf neighbours within 3 cells of it; 0 for a refined box."""
    keys = [(int(t), int(l), int(c[0]), int(c[1]), int(c[2])) for l, c, t in zip(level, ijk, tree)]
    idx = {k: q for q, k in enumerate(keys)}
    out = np.zeros(len(keys))
    for q, k in enumerate(keys):
        if children(k)[0] in idx:
            continue
        t, l, i, j, kk = k
        lim = 1 << (l - 1)
        v = [scores[q][13]]
        for o in OFFS:
            p = (i + o[0], j + o[1], kk + o[2])
            n = (t, l) + p
            if min(p) >= 0 and max(p) < lim and n in idx and children(n)[0] not in idx:
                v.append(scores[idx[n]][reg(tuple(-x for x in o))])
        out[q] = max(v)
    return out


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_plan_from_near_values_matches_the_rules(seed):
    """mg_regrid_plan_near on the per-box values of the criterion gives the
    reference rules' plan, and the same list as mg_regrid_plan on the 27
    scores."""
    bl = forest_boxes()
    rng = np.random.default_rng(seed)
    sc = rng.lognormal(0.0, 1.5, (bl.n, 27)) * 10.0 ** rng.uniform(-4, 0, (bl.n, 1))
    sc[:, 13] = np.maximum(sc[:, 13], sc.max(axis=1))
    c3 = float(np.quantile(sc[:, 13], 0.98))
    near = near_of(bl.level, bl.ijk, bl.tree, sc)
    h = M.mg_tree_create(M.make_domain(), bl.level, bl.ijk, bl.tree)
    try:
        order = M.mg_tree_index(h, M.MG_IDX_ORDER, bl.n).reshape(-1)
        a = M.mg_regrid_plan_near(h, near[order], c3, 0.3, 6)
        b = M.mg_regrid_plan(h, sc[order], c3, 0.3, 6)
    finally:
        M.mg_tree_destroy(h)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    got = {(int(t), int(l), *map(int, c)) for l, c, t in zip(a[0], a[1], a[2])}
    assert got == ref_plan(bl.level, bl.ijk, bl.tree, sc, c3, 0.3, 6)


@pytest.mark.parametrize("seed", [0, 1])
def test_plan_on_the_deepest_level_matches_the_rules(seed):
    """A tree refined at its far corner down to level 15, so that box
    coordinates reach 2^14 - 1 and every bit of the planner's packed keys is
    used; both planner entry points against the rules, with refinement
    capped at level 15."""
    corner = [(l, (1 << (l - 1)) - 1, (1 << (l - 1)) - 1, (1 << (l - 1)) - 1) for l in range(1, 15)]
    bl = refine_boxes_explicit(1, corner, max_level=15)
    assert int(bl.level.max()) == 15 and int(bl.ijk.max()) == (1 << 14) - 1
    rng = np.random.default_rng(seed)
    sc = rng.lognormal(0.0, 1.5, (bl.n, 27)) * 10.0 ** rng.uniform(-4, 0, (bl.n, 1))
    sc[:, 13] = np.maximum(sc[:, 13], sc.max(axis=1))
    c3 = float(np.quantile(sc[:, 13], 0.8))
    near = near_of(bl.level, bl.ijk, bl.tree, sc)
    h = M.mg_tree_create(M.make_domain(), bl.level, bl.ijk, bl.tree)
    try:
        order = M.mg_tree_index(h, M.MG_IDX_ORDER, bl.n).reshape(-1)
        a = M.mg_regrid_plan(h, sc[order], c3, 0.3, 15)
        b = M.mg_regrid_plan_near(h, near[order], c3, 0.3, 15)
    finally:
        M.mg_tree_destroy(h)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    got = {(int(t), int(l), *map(int, c)) for l, c, t in zip(a[0], a[1], a[2])}
    want = ref_plan(bl.level, bl.ijk, bl.tree, sc, c3, 0.3, 15)
    old = {(int(t), int(l), *map(int, c)) for l, c, t in zip(bl.level, bl.ijk, bl.tree)}
    assert got == want, (len(got ^ want), sorted(got ^ want)[:5])
    assert got != old
    assert max(k[1] for k in got) == 15 and max(max(k[2:]) for k in got) == (1 << 14) - 1
    h2 = M.mg_tree_create(M.make_domain(), *a)
    M.mg_tree_destroy(h2)


def test_plan_refines_around_a_charge_and_derefines_behind_it():
    """Structured case: a uniform level-3 tree whose finest boxes near x = 0.2
    are refined; the charge is now at x = 0.8.  Boxes near the charge get
    children, the quiet octets near 0.2 lose theirs, and the library agrees
    with the reference rules."""
    bl = refine_boxes_explicit(3, [(3, 1, 1, 1), (3, 1, 2, 1)])
    lv_c, ij_c = bl.level, bl.ijk
    x, y, z, h = G.cell_centres(lv_c, ij_c)
    rhs = 1e4 * np.exp(-((x - 0.8) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2) / (2 * 0.03 ** 2))
    sc = numpy_scores(lv_c, ij_c, rhs)
    h_ = M.mg_tree_create(M.make_domain(), bl.level, bl.ijk, bl.tree)
    try:
        order = M.mg_tree_index(h_, M.MG_IDX_ORDER, bl.n).reshape(-1)
        lv, ij, tr = M.mg_regrid_plan(h_, sc[order], 1.0, 0.125, 5)
    finally:
        M.mg_tree_destroy(h_)
    got = {(int(t), int(l), *map(int, c)) for l, c, t in zip(lv, ij, tr)}
    assert got == ref_plan(bl.level, bl.ijk, bl.tree, sc, 1.0, 0.125, 5)
    assert (0, 4, 2, 2, 2) not in got            # behind the charge: derefined
    near = [k for k in got if k[1] == 4 and k[2] >= 5]
    assert near                                  # at the charge: refined


def test_oracle_transfer_is_exact_for_linear_potentials():
    fn = lambda x, y, z: 0.3 + 1.7 * x - 0.9 * y + 2.2 * z
    old = refine_boxes_explicit(2, [(2, 0, 0, 0), (3, 1, 1, 1)])
    new = refine_boxes_explicit(2, [(2, 1, 1, 1), (3, 3, 3, 3), (3, 2, 3, 3)])
    bc = dict(bc_type=(0,) * 6)
    o_old = O.OracleTree(old.level, old.ijk, old.tree)
    o_new = O.OracleTree(new.level, new.ijk, new.tree)
    for o in (o_old, o_new):
        lv, ij = o.index(O.IDX_LEVEL), o.index(O.IDX_IJK)
        o.set_bcval(G.face_values(lv, ij, fn))
    lv, ij = o_old.index(O.IDX_LEVEL), o_old.index(O.IDX_IJK)
    x, y, z, _ = G.cell_centres(lv, ij)
    o_old.set_field(O.PHI, fn(x, y, z))
    o_new.transfer_from(o_old)
    lv, ij = o_new.index(O.IDX_LEVEL), o_new.index(O.IDX_IJK)
    x, y, z, _ = G.cell_centres(lv, ij)
    assert np.abs(o_new.get_field(O.PHI) - fn(x, y, z)).max() < 1e-13


def test_oracle_transfer_identity_and_a_hand_computed_box():
    bl = uniform_boxes(2)
    rng = np.random.default_rng(3)
    a = O.OracleTree(bl.level, bl.ijk, bl.tree)
    phi = rng.standard_normal((bl.n, 8, 8, 8))
    a.set_field(O.PHI, phi)
    b = O.OracleTree(bl.level, bl.ijk, bl.tree)
    b.transfer_from(a)
    np.testing.assert_array_equal(b.get_field(O.PHI), a.get_field(O.PHI))
    # refine the level-2 box (1, 0, 1): its child (2, 1, 3) (octant (0, 1, 1))
    # takes the stencil of its parent's cells
    bl2 = refine_boxes_explicit(2, [(2, 1, 0, 1)])
    c = O.OracleTree(bl2.level, bl2.ijk, bl2.tree)
    c.transfer_from(a)
    lv, ij = c.index(O.IDX_LEVEL), c.index(O.IDX_IJK)
    q = [n for n in range(len(lv)) if lv[n] == 3 and tuple(ij[n]) == (2, 1, 3)][0]
    lva, ija = a.index(O.IDX_LEVEL), a.index(O.IDX_IJK)
    p = [n for n in range(len(lva)) if lva[n] == 2 and tuple(ija[n]) == (1, 0, 1)][0]
    P = a.get_field(O.PHI)[p]                     # [k][j][i], interior of the parent
    got = c.get_field(O.PHI)[q]
    for (i, j, k) in [(1, 1, 1), (2, 5, 3), (6, 2, 4)]:   # stencils inside the parent
        cx, cy, cz = 0 + i // 2, 4 + j // 2, 4 + k // 2
        sx, sy, sz = (1 if i & 1 else -1), (1 if j & 1 else -1), (1 if k & 1 else -1)
        want = 0.25 * P[cz, cy, cx] + 0.25 * (P[cz, cy, cx + sx] + P[cz, cy + sy, cx] + P[cz + sz, cy, cx])
        assert abs(got[k, j, i] - want) <= 1e-15 * abs(want) + 1e-300, (i, j, k)


# --------------------------------------------------------------------- GPU

@pytest.mark.gpu
def test_gpu_scores_match_numpy():
    w = streamer_small()
    g = M.Tree.from_workload(w)
    g.set_rhs_from(w)
    sc = g.refine_scores()
    lv, ij = g.index(M.MG_IDX_LEVEL), g.index(M.MG_IDX_IJK)
    want = numpy_scores(lv, ij, g.get_field(M.MG_FIELD_RHS))
    print("scores", g.n, "boxes, max", want.max(), flush=True)
    assert np.array_equal(sc, want)


@pytest.mark.gpu
@pytest.mark.parametrize("case", ["streamer_small", "forest"])
def test_gpu_near_values_match_the_host_rule(case):
    """mg_refine_near on the GPU against the rule's per-box values computed
    here from the GPU's own scores (the same bits), and the plans from the
    two paths (identical lists); on the small streamer tree and on a forest
    of two trees with a seeded random charge."""
    if case == "streamer_small":
        w = streamer_small()
        g = M.Tree.from_workload(w)
        g.set_rhs_from(w)
    else:
        bl = forest_boxes()
        g = M.Tree(bl.level, bl.ijk, bl.tree, bc_type=(0,) * 6)
        g.set_field(M.MG_FIELD_RHS, np.random.default_rng(5).lognormal(0.0, 2.0, (g.n, 8, 8, 8)))
    sc = g.refine_scores()
    near = g.refine_near()
    lv, ij, tr = g.index(M.MG_IDX_LEVEL), g.index(M.MG_IDX_IJK), g.index(M.MG_IDX_TREE)
    want = near_of(lv, ij, tr, sc)
    print("near", g.n, "boxes, max", want.max(), flush=True)
    assert np.array_equal(near, want)
    c3 = 0.1 * float(want.max())
    a = M.mg_regrid_plan_near(g.h, near, c3, 0.125, g.nlev + 1)
    b = M.mg_regrid_plan(g.h, sc, c3, 0.125, g.nlev + 1)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    new = {(int(t), int(l), *map(int, c)) for l, c, t in zip(a[0], a[1], a[2])}
    old = {(int(t), int(l), *map(int, c)) for l, c, t in zip(lv, ij, tr)}
    assert new != old                            # the step changes the tree


@pytest.mark.gpu
def test_gpu_regrid_step_matches_the_oracle():
    """Solve on the small streamer tree, plan a new tree from the GPU scores
    with a threshold that both refines and derefines it, transfer phi (GPU vs
    oracle), then warm-started V-cycles on the new tree (GPU vs oracle)."""
    w = streamer_small()
    g = M.Tree.from_workload(w)
    o = O.OracleTree.from_workload(w)
    g.set_rhs_from(w)
    o.set_rhs_from(w)
    g.fmg_solve()
    o.fmg_solve()
    lv, ij = g.index(M.MG_IDX_LEVEL), g.index(M.MG_IDX_IJK)
    b = w.rhs(lv, ij)
    g.set_field(M.MG_FIELD_RHS, b)                 # leaf b again (the solve overwrote covered boxes)
    c3 = float(np.quantile(g.refine_scores()[:, 13][g.leaf_mask()], 0.5))
    # the charge has changed: the half x < 1/2 is gone, so that half is
    # derefined while the threshold refines around the rest (at this maximum
    # level a finer level would block every removal by 2:1 nesting)
    cen = (ij + 0.5) / (2.0 ** (lv - 1))[:, None]
    b[cen[:, 0] < 0.5] = 0.0
    g.set_field(M.MG_FIELD_RHS, b)
    sc = g.refine_scores()
    nl, nij, ntr = M.mg_regrid_plan(g.h, sc, c3, 0.125, g.nlev)
    old = {(int(l), *map(int, c)) for l, c in zip(lv, ij)}
    new = {(int(l), *map(int, c)) for l, c in zip(nl, nij)}
    assert new - old and old - new                 # both refined and derefined
    g2 = M.Tree(nl, nij, ntr, w.lo, w.length, w.bc_type, w.bc_val)
    o2 = O.OracleTree(nl, nij, ntr, w.lo, w.length, w.bc_type, w.bc_val)
    assert np.array_equal(g2.index(M.MG_IDX_ORDER), o2.index(O.IDX_ORDER))
    M.mg_transfer(g.h, g2.h)
    o.set_field(O.PHI, g.get_field(M.MG_FIELD_PHI))  # the same old potential on both sides
    o2.transfer_from(o)
    pg, po = g2.get_field(M.MG_FIELD_PHI), o2.get_field(O.PHI)
    print("regrid:", g.n, "->", g2.n, "boxes; transfer max diff", np.abs(pg - po).max(), flush=True)
    assert np.abs(pg - po).max() <= 1e-13 * np.abs(po).max()
    lv2, ij2 = g2.index(M.MG_IDX_LEVEL), g2.index(M.MG_IDX_IJK)
    b2 = w.rhs(lv2, ij2)
    g2.set_field(M.MG_FIELD_RHS, b2)
    o2.set_field(O.RHS, b2)
    sg, so = g2.vcycles(2), o2.vcycles(2)
    leaf = o2.leaf_mask()
    pg, po = g2.get_field(M.MG_FIELD_PHI), o2.get_field(O.PHI)
    err = np.linalg.norm((pg - po)[leaf]) / np.linalg.norm(po[leaf])
    print("after 2 V-cycles: rel", sg["rel"], so["rel"], "phi err", err, flush=True)
    np.testing.assert_allclose(sg["hist"], so["hist"], rtol=1e-5)
    assert err <= 1e-10


@pytest.mark.gpu
def test_gpu_regrid_full_size_matches_the_oracle():
    """The benchmark tree (10,825 boxes) with its streamer head moved down by
    0.01: GPU scores equal numpy's, the plan (c3 = 0.3 of the largest leaf
    score, one level deeper allowed) both refines and derefines, the GPU
    transfer equals the oracle's, and two warm-started V-cycles on the new
    tree agree with the oracle's."""
    from workloads import c2, c2_head_sequence
    w = c2()
    g = M.Tree.from_workload(w)
    o = O.OracleTree.from_workload(w)
    g.set_rhs_from(w)
    o.set_rhs_from(w)
    g.fmg_solve()
    o.fmg_solve()
    lv, ij = g.index(M.MG_IDX_LEVEL), g.index(M.MG_IDX_IJK)
    b = c2_head_sequence(lv, ij, 1, 0.0, z_head=0.61)[0]
    g.set_field(M.MG_FIELD_RHS, b)
    sc = g.refine_scores()
    assert np.array_equal(sc, numpy_scores(lv, ij, b))
    leaf = g.leaf_mask()
    nl, nij, ntr = M.mg_regrid_plan(g.h, sc, 0.3 * float(sc[leaf, 13].max()), 0.125, g.nlev + 1)
    old = {(int(l), *map(int, c)) for l, c in zip(lv, ij)}
    new = {(int(l), *map(int, c)) for l, c in zip(nl, nij)}
    assert new - old and old - new
    g2 = M.Tree(nl, nij, ntr, w.lo, w.length, w.bc_type, w.bc_val)
    o2 = O.OracleTree(nl, nij, ntr, w.lo, w.length, w.bc_type, w.bc_val)
    assert np.array_equal(g2.index(M.MG_IDX_ORDER), o2.index(O.IDX_ORDER))
    M.mg_transfer(g.h, g2.h)
    o.set_field(O.PHI, g.get_field(M.MG_FIELD_PHI))
    o2.transfer_from(o)
    pg, po = g2.get_field(M.MG_FIELD_PHI), o2.get_field(O.PHI)
    print("regrid:", g.n, "->", g2.n, "boxes; transfer max diff", np.abs(pg - po).max(), flush=True)
    assert np.abs(pg - po).max() <= 1e-13 * np.abs(po).max()
    lv2, ij2 = g2.index(M.MG_IDX_LEVEL), g2.index(M.MG_IDX_IJK)
    b2 = c2_head_sequence(lv2, ij2, 1, 0.0, z_head=0.61)[0]
    g2.set_field(M.MG_FIELD_RHS, b2)
    o2.set_field(O.RHS, b2)
    sg, so = g2.vcycles(2), o2.vcycles(2)
    leaf = o2.leaf_mask()
    pg, po = g2.get_field(M.MG_FIELD_PHI), o2.get_field(O.PHI)
    err = np.linalg.norm((pg - po)[leaf]) / np.linalg.norm(po[leaf])
    print("after 2 V-cycles: rel", sg["rel"], so["rel"], "phi err", err, flush=True)
    np.testing.assert_allclose(sg["hist"], so["hist"], rtol=1e-5)
    assert err <= 1e-10
