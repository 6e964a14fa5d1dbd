"""Host-side checks of libmg.so that need no GPU: symbol exports, the tree
builder's tables (bit-exact against the oracle and against a brute-force
search), and input validation."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_1708_08434_amd import mg as M
from paper_1708_08434_amd import nn as NN
from workloads import uniform_boxes, refine_boxes_explicit, streamer_small
from workloads.octree import BoxList
from tests.test_oracle_pins import amr_tree, brute_tables

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in sorted(os.listdir(inc)):
        if fn.endswith(".h"):
            src = re.sub(r"/\*.*?\*/", "", open(os.path.join(inc, fn)).read(), flags=re.S)
            names |= set(re.findall(r"\b(mg_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = M.lib()
    names = declared_functions()
    assert len(names) >= 28
    for name in names:
        assert hasattr(L, name), name
    assert set(M.EXPORTS) | set(NN.EXPORTS) <= set(names)
    assert set(NN.EXPORTS) - set(M.EXPORTS) >= {"mg_learned_solve", "mg_nn_forward"}


def test_learned_host_side_sizes_and_errors():
    """Sizes and argument checks of the learned-step ABI that need no GPU."""
    L = NN.lib()
    assert NN.mg_nn_state_bytes() >= 4 * 4 * NN.MG_NN_PARAMS + 2 * 8192
    assert NN.mg_nn_train_bytes(10) > NN.mg_nn_train_bytes(1) > 0
    bl = uniform_boxes(2)
    h = M.mg_tree_create(M.make_domain(), bl.level, bl.ijk)
    try:
        need = NN.mg_learned_bytes(h)
        assert need >= 8 * (1000 + 512 + 3 * 512) * 4
        # unbound tree / null network are rejected before any device work
        rc = L.mg_learned_step(h, None, None, 0, None)
        assert rc == M.MG_ESTATE
    finally:
        M.mg_tree_destroy(h)
    out = ctypes.c_void_p()
    assert L.mg_nn_create(ctypes.byref(out), None, 0, None) == M.MG_EINVAL
    assert L.mg_nn_create(ctypes.byref(out), ctypes.c_void_p(256), 16, None) == M.MG_ENOMEM


def forest():
    a = amr_tree()
    b = refine_boxes_explicit(2, [(2, 1, 1, 1)], tree=1)
    c = uniform_boxes(2, tree=2)
    return BoxList.concat([a, b, c])


@pytest.mark.parametrize("name", ["amr", "streamer", "forest"])
def test_tables_match_oracle(name):
    bl = {"amr": amr_tree, "streamer": lambda: streamer_small().boxes, "forest": forest}[name]()
    bl = bl.shuffled(11)
    g = M.Tree(bl.level, bl.ijk, bl.tree, bind=False)
    o = O.OracleTree(bl.level, bl.ijk, bl.tree)
    for what in range(8):
        assert np.array_equal(g.index(what), o.index(what)), what
    assert g.info.n_leaf_boxes == o.n_leaf_boxes
    ls = np.array(g.info.level_start[:g.nlev + 1])
    assert np.array_equal(ls, o.level_start)


@pytest.mark.parametrize("order", ["shuffled", "canonical"])
def test_tables_match_oracle_on_a_large_tree(order):
    """41,545 boxes (uniform level 6 plus a refined 8^3 block of it): the
    table loops run on several host threads at this size, and canonical
    input skips the sort."""
    bl = refine_boxes_explicit(6, [(6, i, j, k) for i in range(12, 20) for j in range(20, 28)
                                   for k in range(8, 16)])
    if order == "shuffled":
        bl = bl.shuffled(5)
    else:
        h = M.mg_tree_create(M.make_domain(), bl.level, bl.ijk, bl.tree)
        try:
            perm = M.mg_tree_index(h, M.MG_IDX_ORDER, len(bl.level)).reshape(-1)
        finally:
            M.mg_tree_destroy(h)
        bl = BoxList(bl.level[perm], bl.ijk[perm], bl.tree[perm])
    g = M.Tree(bl.level, bl.ijk, bl.tree, bind=False)
    assert g.n == 41545
    o = O.OracleTree(bl.level, bl.ijk, bl.tree)
    for what in range(8):
        assert np.array_equal(g.index(what), o.index(what)), what
    if order == "canonical":
        assert np.array_equal(g.index(M.MG_IDX_ORDER).reshape(-1), np.arange(g.n))


def test_tables_match_brute_force():
    bl = forest().shuffled(5)
    g = M.Tree(bl.level, bl.ijk, bl.tree, bind=False)
    order = g.index(M.MG_IDX_ORDER)
    inv = np.empty(bl.n, int)
    inv[order] = np.arange(bl.n)
    # brute force per tree (coordinates only make sense within one tree)
    par = np.full(bl.n, -1); nbr = np.full((bl.n, 6), -9); cfq = np.full((bl.n, 6), -1)
    for tr in np.unique(bl.tree):
        idx = np.where(bl.tree == tr)[0]
        sub = BoxList(bl.level[idx], bl.ijk[idx])
        p, nb, cq = brute_tables(sub)
        par[idx] = np.where(p >= 0, idx[np.maximum(p, 0)], p)
        nbr[idx] = np.where(nb >= 0, idx[np.maximum(nb, 0)], nb)
        cfq[idx] = np.where(cq >= 0, idx[np.maximum(cq, 0)], cq)

    def canon(a):
        return np.where(a >= 0, inv[np.maximum(a, 0)], a)
    assert np.array_equal(g.index(M.MG_IDX_PARENT), canon(par[order]))
    assert np.array_equal(g.index(M.MG_IDX_NBR), canon(nbr[order]))
    assert np.array_equal(g.index(M.MG_IDX_CFQ), canon(cfq[order]))


def _names(bl, **kw):
    out = []
    for make in (lambda: M.Tree(bl.level, bl.ijk, bl.tree, bind=False, **kw),
                 lambda: O.OracleTree(bl.level, bl.ijk, bl.tree, **kw)):
        try:
            make()
            out.append("OK")
        except (M.MGError, O.OracleError) as e:
            out.append(e.name)
    return out


def test_validation_agrees_with_oracle():
    good = amr_tree()
    oct8 = np.array([[a, b, c] for c in (0, 1) for b in (0, 1) for a in (0, 1)])
    cases = {
        "good": (good, "OK"),
        "no_root": (BoxList(good.level[good.level != 1], good.ijk[good.level != 1]), "ETOPO"),
        "sibling": (BoxList(np.delete(good.level, np.where(good.level == 5)[0][0]),
                            np.delete(good.ijk, np.where(good.level == 5)[0][0], axis=0)), "ETOPO"),
        "parent": (BoxList(np.append(good.level, 4), np.vstack([good.ijk, [[7, 7, 7]]])), "ETOPO"),
        "dup": (BoxList(np.append(good.level, good.level[3]), np.vstack([good.ijk, good.ijk[3:4]])),
                "EINVAL"),
        "range": (BoxList(np.append(good.level, 2), np.vstack([good.ijk, [[2, 0, 0]]])), "EINVAL"),
        "nesting": (BoxList.concat([uniform_boxes(2), BoxList(np.full(8, 3), oct8),
                                    BoxList(np.full(8, 4), 2 + oct8)]), "ENESTING"),
        "tree_gap": (BoxList.concat([good, BoxList([1], [[0, 0, 0]], [2])]), "ETOPO"),
    }
    for name, (bl, want) in cases.items():
        assert _names(bl) == [want, want], name
    assert _names(good, bc_type=(1,) * 6) == ["EINVAL", "EINVAL"]


def test_workspace_size_is_reported():
    w = streamer_small()
    g = M.Tree.from_workload(w, bind=False)
    n = g.n
    # phi, rhs, old and the fused sweeps' second buffer (FP64), plus the FP32 fields
    assert g.info.workspace_bytes >= 4 * 512 * 8 * n + 3 * 512 * 4 * n
    assert g.info.n_leaf_cells == w.n_leaf


def _no_gpu():
    import torch
    return torch.cuda.device_count() == 0


@pytest.mark.skipif(not _no_gpu(), reason="needs a machine without a GPU: the bind must fail in the runtime")
def test_a_failed_bind_leaves_the_tree_unbound():
    """Without a device, mg_tree_bind fails in the HIP runtime (MG_EHIP); the
    tree must then count as unbound, so the next call that needs a
    workspace is refused (MG_ESTATE) instead of running on tables that were
    never uploaded."""
    b = uniform_boxes(2)
    h = M.mg_tree_create(M.make_domain(), b.level, b.ijk, b.tree)
    try:
        nbytes = int(M.mg_tree_info(h).workspace_bytes)
        with pytest.raises(M.MGError) as e:
            M.mg_tree_bind(h, 1 << 20, nbytes, 0)
        assert e.value.code == M.MG_EHIP
        with pytest.raises(M.MGError) as e:
            M.mg_field_set(h, M.MG_FIELD_RHS, 1 << 20)
        assert e.value.code == M.MG_ESTATE
    finally:
        M.mg_tree_destroy(h)


def test_schedule_entries_are_validated():
    """mg_set_schedule takes one entry per level in 0..MG_GSRB_VARIANTS-1
    (host state only, no GPU); mg_autotune needs a bound workspace."""
    hdr = open(os.path.join(ROOT, "include", "mg.h")).read()
    assert int(re.search(r"#define MG_GSRB_VARIANTS (\d+)", hdr).group(1)) == M.MG_GSRB_VARIANTS
    bl = uniform_boxes(3)
    h = M.mg_tree_create(M.make_domain(), bl.level, bl.ijk)
    try:
        L = M.lib()
        for prec in (M.MG_FP64, M.MG_MIXED):
            for v in range(M.MG_GSRB_VARIANTS):
                M.mg_set_schedule(h, prec, [v, v, v])
            for bad in (-1, M.MG_GSRB_VARIANTS):
                sch = np.array([3, bad, 3], dtype=np.int32)
                assert L.mg_set_schedule(h, prec, sch.ctypes.data) == M.MG_EINVAL
        sch = np.zeros(3, dtype=np.int32)
        assert L.mg_set_schedule(h, 7, sch.ctypes.data) == M.MG_EINVAL
        assert L.mg_autotune(h, M.MG_FP64, 4, sch.ctypes.data) == M.MG_ESTATE
    finally:
        M.mg_tree_destroy(h)


def test_workload_leaf_counts_match_the_tables():
    """The generators' leaf count (used for neutrality and for cells/s) equals
    the leaf count of the library's and the oracle's own tables on a deep
    tree (coordinates beyond 2^7, where a too-narrow packed key collides)."""
    from workloads import c2
    w = c2()
    h = M.mg_tree_create(M.make_domain(), w.boxes.level, w.boxes.ijk, w.boxes.tree)
    try:
        info = M.mg_tree_info(h)
        assert int(info.n_leaf_cells) == w.n_leaf == 4849664
    finally:
        M.mg_tree_destroy(h)
    o = O.OracleTree.from_workload(w)
    assert int(o.leaf_mask().sum()) * 512 == w.n_leaf


def test_mesh_adaptation_and_fluid_argument_checks():
    """Argument and state checks of the mesh-adaptation and fluid entry
    points that need no GPU: the plan rejects bad thresholds and levels and
    reports the size it needs; the fluid workspace size grows with the table
    and the tree; an unbound tree is refused before any device work."""
    bl = refine_boxes_explicit(2, [(2, 0, 0, 0)])
    h = M.mg_tree_create(M.make_domain(), bl.level, bl.ijk)
    try:
        L = M.lib()
        n = len(bl.level)
        sc = np.ones((n, 27))
        lv = np.zeros(4 * n, dtype=np.int32)
        ij = np.zeros((4 * n, 3), dtype=np.int32)
        tr = np.zeros(4 * n, dtype=np.int32)
        need = ctypes.c_int64()
        P = lambda a: a.ctypes.data

        def plan(c3, deref, h_deref, max_level, cap):
            return L.mg_regrid_plan(h, P(sc), c3, deref, h_deref, max_level, cap, P(lv), P(ij), P(tr),
                                    ctypes.byref(need))
        for bad in [(0.0, 0.1, 1.0, 5), (-1.0, 0.1, 1.0, 5), (1.0, -0.1, 1.0, 5), (1.0, 0.1, 0.0, 5),
                    (1.0, 0.1, 1.0, 0), (1.0, 0.1, 1.0, 16)]:
            assert plan(*bad, 4 * n) == M.MG_EINVAL, bad
        # scores of 1 everywhere, c3 = 0.5: every leaf below level 4 is refined
        assert plan(0.5, 0.1, float("inf"), 4, 0) == M.MG_ENOMEM
        assert need.value > n
        m = need.value                              # room for the whole plan
        lv, ij, tr = (np.zeros(m, dtype=np.int32), np.zeros((m, 3), dtype=np.int32),
                      np.zeros(m, dtype=np.int32))
        assert plan(0.5, 0.1, float("inf"), 4, m) == M.MG_OK
        assert plan(0.5, 0.1, float("inf"), 4, m - 1) == M.MG_ENOMEM and need.value == m
        a = M.mg_fluid_workspace_bytes(h, 2)
        b = M.mg_fluid_workspace_bytes(h, 1000)
        assert b > a >= n * 8 * (4 * 512 + 1728 + 512)
        assert L.mg_fluid_workspace_bytes(h, 1) == -1
        tab = np.ones((4, 3))
        assert L.mg_fluid_bind(h, ctypes.c_void_p(256), 1 << 30, P(tab), 4, 1.0) == M.MG_ESTATE
        x = ctypes.c_void_p(256)
        assert L.mg_fluid_step(h, x, x, ctypes.c_double(1e-12), 2, None) == M.MG_ESTATE
        assert L.mg_fluid_stage(h, x, x, x, x, x, x, ctypes.c_double(0.0), ctypes.c_double(0.0),
                                ctypes.c_double(1.0), x, x, None) == M.MG_ESTATE
        assert L.mg_refine_scores(h, x) == M.MG_ESTATE
    finally:
        M.mg_tree_destroy(h)


def test_bench_schedule_option_and_gpu_count():
    """bench.py --schedule: one or two lists (FP64, then FP32) of one launch
    variant per level; anything else is refused.  --gpus above 1 is refused
    with a message, before any GPU work."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import bench
    assert bench.parse_schedule("3,7,7,11", 4, 14) == [[3, 7, 7, 11]]
    assert bench.parse_schedule("3,7,7,11/3,7,7,9", 4, 14) == [[3, 7, 7, 11], [3, 7, 7, 9]]
    for bad in ("3,7,7", "3,7,7,14", "3,7,7,-1", "3,7,x,1", "1,1,1,1/1,1,1,1/1,1,1,1", ""):
        with pytest.raises(SystemExit):
            bench.parse_schedule(bad, 4, 14)
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in (r.stdout + r.stderr), (r.returncode, r.stdout, r.stderr)
