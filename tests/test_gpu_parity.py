"""GPU parity: every step of the cycle and whole solves, through the C ABI,
against the oracle on the same seeded inputs.

Tolerances: single steps 1e-12 of the field's largest magnitude (the two
sides differ only by FMA contraction and summation order); whole solves a
relative L2 difference of 1e-10 on the leaf potential with the same V-cycle
count (the FP64 parity bar of the method's scope)."""
import numpy as np
import pytest

import oracle as O
from paper_1708_08434_amd import mg as M
from workloads import c1, c2, c3, c5, forest, streamer_small, uniform_boxes, refine_boxes_explicit
from tests import _geom as G

pytestmark = pytest.mark.gpu

STEP_TOL = 1e-12
SOLVE_TOL = 1e-10


def say(*a):
    print(*a, flush=True)


def pair(w, per_cell_bc=False):
    g = M.Tree.from_workload(w, per_cell_bc=per_cell_bc)
    o = O.OracleTree.from_workload(w)
    assert np.array_equal(g.index(M.MG_IDX_ORDER), o.index(O.IDX_ORDER))
    return g, o


def relmax(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def seed_fields(g, o, seed):
    rng = np.random.default_rng(seed)
    n = g.n
    phi = rng.standard_normal((n, 8, 8, 8))
    rhs = rng.standard_normal((n, 8, 8, 8)) * 100.0
    old = phi + 0.1 * rng.standard_normal((n, 8, 8, 8))
    for which_g, which_o, a in ((M.MG_FIELD_PHI, O.PHI, phi), (M.MG_FIELD_RHS, O.RHS, rhs),
                                (M.MG_FIELD_OLD, O.OLD, old)):
        g.set_field(which_g, a)
        o.set_field(which_o, a)


def old_mask(g, below):
    """Boxes whose old values are defined after a step that ran the down-leg
    from levels < `below`: on those coarse levels only where a prolongation
    reads them (the library copies phi into old nowhere else), everywhere on
    the other levels (untouched by both sides)."""
    lv = g.index(M.MG_IDX_LEVEL)
    if not below:
        return np.ones(g.n, dtype=bool)
    read = G.old_read_mask(lv, g.index(M.MG_IDX_IJK), g.index(M.MG_IDX_TREE), g.index(M.MG_IDX_CHILD))
    return np.where(lv < below, read, True)


def compare_fields(g, o, what, old_below=0):
    mask = old_mask(g, old_below) if old_below else np.ones(g.n, dtype=bool)
    for which_g, which_o, name in ((M.MG_FIELD_PHI, O.PHI, "phi"), (M.MG_FIELD_RHS, O.RHS, "rhs"),
                                   (M.MG_FIELD_OLD, O.OLD, "old")):
        a, b = g.get_field(which_g), o.get_field(which_o)
        if name == "old":
            a, b = a[mask], b[mask]
        e = relmax(a, b)
        assert e <= STEP_TOL, (what, name, e)


STEPS = [("smooth", M.MG_OP_SMOOTH, O.OP_SMOOTH, "top", 1),
         ("smooth2", M.MG_OP_SMOOTH, O.OP_SMOOTH, "mid", 2),
         ("fas_down", M.MG_OP_FAS_DOWN, O.OP_FAS_DOWN, "top", 0),
         ("fas_down_mid", M.MG_OP_FAS_DOWN, O.OP_FAS_DOWN, "mid", 0),
         ("prolong", M.MG_OP_PROLONG, O.OP_PROLONG, "top", 0),
         ("prolong_2", M.MG_OP_PROLONG, O.OP_PROLONG, 2, 0),
         ("coarse", M.MG_OP_COARSE, O.OP_COARSE, 1, 0),
         ("restrict_all", M.MG_OP_RESTRICT_ALL, O.OP_RESTRICT_ALL, 1, 0),
         ("vcycle", M.MG_OP_VCYCLE, O.OP_VCYCLE, "top", 2)]


@pytest.mark.parametrize("wname", ["uniform", "streamer"])
@pytest.mark.parametrize("step", STEPS, ids=[s[0] for s in STEPS])
def test_step_parity(wname, step):
    name, gop, oop, lev, arg = step
    w = c1() if wname == "uniform" else streamer_small()
    g, o = pair(w)
    level = {"top": o.nlev, "mid": o.nlev - 1}.get(lev, lev)
    say("step", wname, name, "level", level, "boxes", g.n)
    seed_fields(g, o, 17)
    g.step(gop, level, arg)
    o.step(oop, level, arg)
    # the down-legs write old on the levels below the step's level
    compare_fields(g, o, name, old_below=level if gop in (M.MG_OP_FAS_DOWN, M.MG_OP_VCYCLE) else 0)


def test_step_parity_per_cell_dirichlet():
    """Per-face-cell Dirichlet data through every ghost type and the root solve."""
    bl = refine_boxes_explicit(2, [(2, 0, 0, 0), (3, 1, 1, 1), (3, 0, 1, 0), (4, 2, 2, 2)])
    from workloads.configs import Workload, rhs_zero
    w = Workload("amr_bcval", bl, rhs_zero, bc_type=(0, 0, 1, 0, 0, 0))
    g, o = pair(w, per_cell_bc=True)
    lv, ij = o.index(O.IDX_LEVEL), o.index(O.IDX_IJK)
    bc = G.face_values(lv, ij, lambda x, y, z: np.sin(3 * x) + y * z)
    g.set_field(M.MG_FIELD_BCVAL, bc)
    o.set_bcval(bc)
    for op_g, op_o, lev in ((M.MG_OP_VCYCLE, O.OP_VCYCLE, o.nlev), (M.MG_OP_COARSE, O.OP_COARSE, 1)):
        seed_fields(g, o, 3)
        g.step(op_g, lev, 2)
        o.step(op_o, lev, 2)
        compare_fields(g, o, "bcval", old_below=lev if op_g == M.MG_OP_VCYCLE else 0)


def solve_pair(w, tol=1e-8):
    g, o = pair(w)
    g.set_rhs_from(w)
    o.set_rhs_from(w)
    sg = g.fmg_solve(rel_tol=tol)
    so = o.fmg_solve(tol=tol)
    leaf = o.leaf_mask()
    pg, po = g.get_field(M.MG_FIELD_PHI), o.get_field(O.PHI)
    err = np.linalg.norm((pg - po)[leaf]) / np.linalg.norm(po[leaf])
    return g, o, sg, so, err


@pytest.mark.parametrize("wname", ["uniform64", "streamer_small"])
def test_fmg_solve_parity(wname):
    w = c1() if wname == "uniform64" else streamer_small()
    say("fmg parity", wname, w.boxes.n, "boxes")
    g, o, sg, so, err = solve_pair(w)
    assert sg["n_vcycles"] == so["n_vcycles"], (sg["hist"], so["hist"])
    assert err <= SOLVE_TOL, err
    np.testing.assert_allclose(sg["hist"], so["hist"], rtol=1e-5)
    assert sg["rel"] <= 1e-8


@pytest.mark.timeout(600)
@pytest.mark.parametrize("wname", ["streamer", "branched", "forest", "two_streamers"])
def test_fmg_solve_parity_full_size(wname):
    """Full-size trees in the launch sequence the benchmark times: the
    benchmark streamer (base 64^3 + 4 refinement levels, 4.8e6 leaf cells),
    the branched streamer (base 64^3 + 6 levels, 2.9e7 leaf cells), the
    forest of 128 uneven trees (7.1e7 leaf cells; its largest trees span
    several chunks of the per-tree norm reduction) and the two streamers
    with background ionisation (base 64^3 + 7 levels, 1.2e8 leaf cells)."""
    w = {"streamer": c2, "branched": c3, "forest": forest, "two_streamers": c5}[wname]()
    say("fmg parity full size", wname, w.boxes.n, "boxes", w.n_leaf, "leaf cells")
    g, o, sg, so, err = solve_pair(w)
    say("  gpu", sg["n_vcycles"], sg["rel"], "oracle", so["n_vcycles"], so["rel"], "err", err)
    assert sg["n_vcycles"] == so["n_vcycles"]
    assert err <= SOLVE_TOL, err
    if wname == "forest":
        nleaf_tree = np.bincount(g.index(M.MG_IDX_TREE)[g.leaf_mask()])
        say("  leaf boxes per tree: max", nleaf_tree.max(), "min", nleaf_tree.min())
        assert nleaf_tree.max() > 2048  # a tree spans more than one reduction chunk
        np.testing.assert_allclose(g.tree_rel(), o.tree_rel(), rtol=1e-5)


def test_warm_vcycles_parity():
    w = streamer_small()
    g, o = pair(w)
    g.set_rhs_from(w)
    o.set_rhs_from(w)
    g.fmg_solve(rel_tol=1e-6)
    o.fmg_solve(tol=1e-6)
    b = o.get_field(O.RHS)
    leaf = o.leaf_mask()
    b[leaf] *= 1.01
    g.set_field(M.MG_FIELD_RHS, b)
    o.set_field(O.RHS, b)
    sg = g.vcycles(2)
    so = o.vcycles(2)
    np.testing.assert_allclose(sg["hist"], so["hist"], rtol=1e-5)
    pg, po = g.get_field(M.MG_FIELD_PHI), o.get_field(O.PHI)
    assert np.linalg.norm((pg - po)[leaf]) / np.linalg.norm(po[leaf]) <= SOLVE_TOL


@pytest.mark.parametrize("wname", ["streamer_small", "forest"])
def test_final_check_only_gives_the_same_bits(wname):
    """mg_vcycle with the residual check only after the last cycle, and with
    no statistics at all (no residual norm): the same phi bits, final
    residual and cycle count as with a check around every cycle; the skipped
    entries of the history are NaN.  Twice in a row, so the recorded graphs
    are replayed."""
    w = streamer_small() if wname == "streamer_small" else small_forest()
    g = M.Tree.from_workload(w)
    lv, ij = g.index(M.MG_IDX_LEVEL), g.index(M.MG_IDX_IJK)
    rhs0 = w.rhs(lv, ij, g.index(M.MG_IDX_TREE))
    g.set_field(M.MG_FIELD_RHS, rhs0)
    g.fmg_solve()
    phi0 = g.get_field(M.MG_FIELD_PHI)
    rhs1 = rhs0 * 1.05 + np.random.default_rng(5).standard_normal(rhs0.shape) * np.abs(rhs0).max() * 1e-3
    for rep in range(2):
        out = []
        for fco in (0, 1):
            g.set_field(M.MG_FIELD_PHI, phi0)
            g.set_field(M.MG_FIELD_RHS, rhs1)
            st = g.vcycles(2, final_check_only=fco)
            out.append((st, g.get_field(M.MG_FIELD_PHI)))
        (sa, pa), (sb, pb) = out
        g.set_field(M.MG_FIELD_PHI, phi0)
        g.set_field(M.MG_FIELD_RHS, rhs1)
        assert M.mg_vcycle(g.h, g.opts(), 2, stats=False) is None   # no statistics: no norms
        assert np.array_equal(g.get_field(M.MG_FIELD_PHI), pa)
        say("final check only", wname, rep, sa["hist"], sb["hist"])
        assert sa["n_vcycles"] == sb["n_vcycles"] == 2
        assert np.array_equal(pa, pb)
        assert sa["rel"] == sb["rel"] and sb["hist"][2] == sa["hist"][2]
        assert np.isnan(sb["hist"][0]) and np.isnan(sb["hist"][1]) and not np.isnan(sa["hist"][1])


@pytest.mark.parametrize("wname", ["streamer_small", "forest", "streamer"])
def test_residual_matches_oracle(wname):
    """Norms of the residual of a random field whose covered cells are not the
    means of their children: the library restricts, before a stopping test,
    only the covered cells next to leaf cells of their own level; the oracle
    restricts every level.  On a forest and on the full-size benchmark tree
    too."""
    w = {"streamer_small": streamer_small, "forest": small_forest, "streamer": c2}[wname]()
    g, o = pair(w)
    seed_fields(g, o, 5)
    rg, ro = g.residual(), o.residual()
    for k in ("rel", "l2", "linf"):
        assert abs(rg[k] - ro[k]) <= 1e-12 * abs(ro[k]), (k, rg[k], ro[k])


def test_bitwise_repeatable():
    w = streamer_small()
    g = M.Tree.from_workload(w)
    g.set_rhs_from(w)
    g.fmg_solve()
    a = g.get_field(M.MG_FIELD_PHI)
    g.fmg_solve()
    b = g.get_field(M.MG_FIELD_PHI)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("variant", [3, 7], ids=["half_sweeps", "fused"])
def test_linear_exact_on_gpu(variant):
    """Section 3.1 boundary setup on an AMR tree: the GPU solution is the
    linear potential at every leaf cell."""
    bl = refine_boxes_explicit(2, [(2, 0, 0, 0), (3, 1, 1, 1), (3, 0, 1, 0), (4, 2, 2, 2)])
    g = M.Tree(bl.level, bl.ijk, None, bc_type=(1, 1, 1, 1, 0, 0), bc_val=(0, 0, 0, 0, 0, 1.0))
    M.mg_set_schedule(g.h, M.MG_FP64, [variant] * g.nlev)
    g.set_field(M.MG_FIELD_RHS, np.zeros((g.n, 8, 8, 8)))
    g.fmg_solve(rel_tol=1e-13)
    x, y, z, h = G.cell_centres(g.index(M.MG_IDX_LEVEL), g.index(M.MG_IDX_IJK))
    leaf = g.leaf_mask()
    assert np.abs(g.get_field(M.MG_FIELD_PHI)[leaf] - z[leaf]).max() < 1e-11


def test_errors_are_reported():
    w = streamer_small()
    g = M.Tree.from_workload(w)
    b = w.rhs(g.index(M.MG_IDX_LEVEL), g.index(M.MG_IDX_IJK))
    b[g.leaf_mask().nonzero()[0][0], 0, 0, 0] = np.nan
    g.set_field(M.MG_FIELD_RHS, b)
    st = M.mg_fmg_solve(g.h, g.opts(), raise_on_error=False)
    assert st.status == M.MG_ENOCONV
    g.set_rhs_from(w)
    st = M.mg_fmg_solve(g.h, g.opts(max_cycles=1), raise_on_error=False)
    assert st.status == M.MG_ENOCONV
    with pytest.raises(M.MGError):
        g.step(M.MG_OP_SMOOTH, 99, 1)


def test_graph_replay_matches_direct_launches():
    """Recorded-graph replay and kernel-by-kernel launches run the same
    kernels in the same order: identical bits."""
    w = streamer_small()
    g = M.Tree.from_workload(w)
    g.set_rhs_from(w)
    a = g.fmg_solve(graphs=0)
    pa = g.get_field(M.MG_FIELD_PHI)
    b = g.fmg_solve(graphs=1)
    pb = g.get_field(M.MG_FIELD_PHI)
    c = g.fmg_solve(graphs=1)  # replay of the recorded graphs
    pc = g.get_field(M.MG_FIELD_PHI)
    assert a["n_vcycles"] == b["n_vcycles"] == c["n_vcycles"]
    assert np.array_equal(pa, pb) and np.array_equal(pb, pc)
    np.testing.assert_array_equal(a["hist"], c["hist"])


def test_kernel_timing_probes():
    w = streamer_small()
    g = M.Tree.from_workload(w)
    g.set_rhs_from(w)
    for graphs in (0, 1):
        M.mg_timing_read(g.h)
        M.mg_timing_enable(g.h, True)
        st = g.fmg_solve(graphs=graphs)
        M.mg_timing_enable(g.h, False)
        kt = M.mg_timing_read(g.h)
        say("timing", graphs, kt, st["n_vcycles"])
        assert kt["launches"] > 0 and kt["total_ms"] > 0
        # every half-sweep launch covers whole levels: bytes = 6144 per box
        assert kt["alg_bytes"] % 6144.0 == 0


# ------------------------------------------------------------- mixed precision

F32_STEP_TOL = 2e-5


def homog_pair(w):
    """GPU tree (whose FP32 fields carry the homogeneous correction problem)
    and an oracle tree with the same boundary types and zero boundary data."""
    g = M.Tree.from_workload(w)
    o = O.OracleTree(w.boxes.level, w.boxes.ijk, w.boxes.tree, w.lo, w.length, w.bc_type,
                     (0.0,) * 6)
    return g, o


@pytest.mark.parametrize("step", STEPS, ids=[s[0] for s in STEPS])
def test_fp32_step_parity(step):
    """Every cycle step on the FP32 correction fields agrees with the FP64
    oracle (homogeneous boundary data) to FP32 rounding."""
    name, gop, oop, lev, arg = step
    w = streamer_small()
    g, o = homog_pair(w)
    level = {"top": o.nlev, "mid": o.nlev - 1}.get(lev, lev)
    say("fp32 step", name, "level", level)
    rng = np.random.default_rng(23)
    n = g.n
    fields = [rng.standard_normal((n, 8, 8, 8)), rng.standard_normal((n, 8, 8, 8)) * 100.0]
    fields.append(fields[0] + 0.1 * rng.standard_normal((n, 8, 8, 8)))
    fields = [f.astype(np.float32).astype(np.float64) for f in fields]
    for which_g, which_o, a in zip((M.MG_FIELD_E32, M.MG_FIELD_R32, M.MG_FIELD_OLD32),
                                   (O.PHI, O.RHS, O.OLD), fields):
        g.set_field(which_g, a)
        o.set_field(which_o, a)
    g.step(gop | M.MG_OP_F32, level, arg)
    o.step(oop, level, arg)
    mask = old_mask(g, level if gop in (M.MG_OP_FAS_DOWN, M.MG_OP_VCYCLE) else 0)
    for which_g, which_o, nm in ((M.MG_FIELD_E32, O.PHI, "e"), (M.MG_FIELD_R32, O.RHS, "r"),
                                 (M.MG_FIELD_OLD32, O.OLD, "old")):
        a, b = g.get_field(which_g), o.get_field(which_o)
        if nm == "old":
            a, b = a[mask], b[mask]
        e = relmax(a, b)
        assert e <= F32_STEP_TOL, (name, nm, e)


MIXED_TOL = 1e-8


@pytest.mark.timeout(600)
@pytest.mark.parametrize("wname", ["uniform64", "streamer_small", "streamer_full", "branched",
                                   "forest"])
def test_mixed_solve_accuracy(wname):
    """FP32 cycles inside FP64 refinement.  At the 1e-8 residual tolerance the
    potential is as close to the fully converged discrete solution (oracle,
    1e-12) as the FP64 path's at the same tolerance (both carry an algebraic
    error of order conditioning x residual, ~1e-7 here); with a tighter
    tolerance the refinement keeps converging past FP32 rounding and the
    potential matches the oracle to a relative L2 of 1e-8."""
    w = {"uniform64": c1, "streamer_small": streamer_small, "streamer_full": c2,
         "branched": c3, "forest": forest}[wname]()
    g, o = pair(w)
    g.set_rhs_from(w)
    o.set_rhs_from(w)
    so = o.fmg_solve(tol=1e-12)
    leaf = o.leaf_mask()
    po = o.get_field(O.PHI)

    def err():
        pg = g.get_field(M.MG_FIELD_PHI)
        return np.linalg.norm((pg - po)[leaf]) / np.linalg.norm(po[leaf])
    sd = g.fmg_solve()
    e64 = err()
    sm = g.fmg_solve(precision=M.MG_MIXED)
    emx = err()
    st = g.fmg_solve(precision=M.MG_MIXED, rel_tol=1e-11)
    etight = err()
    say("mixed", wname, "| fp64:", sd["n_vcycles"], "cycles, err", e64, "| mixed 1e-8:",
        sm["n_vcycles"], "steps, err", emx, "| mixed 1e-11:", st["n_vcycles"], "steps, err", etight)
    assert sm["rel"] <= 1e-8 and st["rel"] <= 1e-11
    assert emx <= 2.0 * e64 + 1e-12, (emx, e64)
    assert etight <= MIXED_TOL, etight


def test_mixed_warm_vcycles():
    w = streamer_small()
    g = M.Tree.from_workload(w)
    g.set_rhs_from(w)
    g.fmg_solve(precision=M.MG_MIXED, rel_tol=1e-6)
    st = g.vcycles(0, precision=M.MG_MIXED)
    assert st["rel"] <= 1e-8 and st["n_vcycles"] >= 1


# ------------------------------------------------------------------- forests

def small_forest():
    from workloads import forest
    return forest(n_trees=6, refinements=2, base=2, lo_cells=2e4, hi_cells=1.5e5)


def test_forest_parity():
    """A forest of uneven trees solved together (one launch per level over all
    trees) matches the oracle's forest solve: same refinement-step count, same
    per-tree relative residuals, potential within 1e-10."""
    w = small_forest()
    say("forest", w.boxes.n, "boxes", w.n_leaf, "leaf cells", int(w.boxes.tree.max()) + 1, "trees")
    for prec in (M.MG_FP64, M.MG_MIXED):
        g, o, sg, so, err = None, None, None, None, None
        g, o = pair(w)
        g.set_rhs_from(w)
        o.set_rhs_from(w)
        sg = g.fmg_solve(precision=prec)
        if prec == M.MG_FP64:
            so = o.fmg_solve()
            assert sg["n_vcycles"] == so["n_vcycles"]
            np.testing.assert_allclose(g.tree_rel(), o.tree_rel(), rtol=1e-5)
            leaf = o.leaf_mask()
            pg, po = g.get_field(M.MG_FIELD_PHI), o.get_field(O.PHI)
            err = np.linalg.norm((pg - po)[leaf]) / np.linalg.norm(po[leaf])
            assert err <= SOLVE_TOL, err
        assert sg["rel"] <= 1e-8 and np.all(g.tree_rel() <= 1e-8)


def test_forest_trees_match_standalone_solves():
    """Every tree of the forest solution agrees with that tree solved alone by
    the oracle to 1e-12, to the accuracy a 1e-8 residual allows."""
    w = small_forest()
    g = M.Tree.from_workload(w)
    g.set_rhs_from(w)
    g.fmg_solve()
    phi = g.get_field(M.MG_FIELD_PHI)
    tid, leaf = g.index(M.MG_IDX_TREE), g.leaf_mask()
    lv, ij = g.index(M.MG_IDX_LEVEL), g.index(M.MG_IDX_IJK)
    for t in np.unique(tid):
        m = tid == t
        o = O.OracleTree(lv[m], ij[m], None, w.lo, w.length, w.bc_type, w.bc_val)
        o.set_field(O.RHS, w.rhs(o.index(O.IDX_LEVEL), o.index(O.IDX_IJK),
                                 np.full(o.n, t)))
        o.fmg_solve(tol=1e-12)
        po = o.get_field(O.PHI)
        # the oracle's canonical order of a single tree equals the forest's
        # order restricted to that tree (level, then Morton)
        pg = phi[m]
        lo = o.leaf_mask()
        err = np.linalg.norm((pg - po)[lo]) / np.linalg.norm(po[lo])
        say("tree", t, "boxes", o.n, "err vs standalone", err)
        assert err <= 1e-6, (t, err)


# ----------------------------------------------------------------- autotuner

def bcval_tree():
    """AMR tree with refinement boundaries, a Neumann face (-y) and per-cell
    Dirichlet data on the other faces."""
    bl = refine_boxes_explicit(2, [(2, 0, 0, 0), (3, 1, 1, 1), (3, 0, 1, 0), (4, 2, 2, 2)])
    from workloads.configs import Workload, rhs_zero
    w = Workload("amr_bcval", bl, rhs_zero, bc_type=(0, 0, 1, 0, 0, 0))
    g, o = pair(w, per_cell_bc=True)
    lv, ij = o.index(O.IDX_LEVEL), o.index(O.IDX_IJK)
    bc = G.face_values(lv, ij, lambda x, y, z: np.sin(3 * x) + y * z)
    g.set_field(M.MG_FIELD_BCVAL, bc)
    o.set_bcval(bc)
    return g, o


@pytest.mark.parametrize("tree", ["streamer_small", "bcval"])
@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_every_gsrb_variant_gives_the_same_bits(tree, fp32):
    """Half-sweep variants and fused sweeps (both colours in one launch, the
    neighbours' red face layers recomputed) give identical bits: V-cycles
    (pairs of sweeps) and an odd number of sweeps (a fused pair, then a
    half-sweep pair)."""
    if tree == "bcval":
        g, _ = bcval_tree()
    else:
        w = streamer_small()
        g = M.Tree.from_workload(w)
    rng = np.random.default_rng(9)
    phi0 = rng.standard_normal((g.n, 8, 8, 8))
    rhs0 = rng.standard_normal((g.n, 8, 8, 8)) * 100.0
    if fp32:
        phi0, rhs0 = (a.astype(np.float32).astype(np.float64) for a in (phi0, rhs0))
    fphi, frhs = (M.MG_FIELD_E32, M.MG_FIELD_R32) if fp32 else (M.MG_FIELD_PHI, M.MG_FIELD_RHS)
    prec, opf = (M.MG_MIXED, M.MG_OP_F32) if fp32 else (M.MG_FP64, 0)
    g.set_field(frhs, rhs0)
    ref = {}
    for v in range(M.MG_GSRB_VARIANTS):
        M.mg_set_schedule(g.h, prec, [v] * g.nlev)
        for name, op, lev, arg in (("vcycle", M.MG_OP_VCYCLE, g.nlev, 2),
                                   ("smooth3", M.MG_OP_SMOOTH, g.nlev, 3),
                                   ("smooth2_mid", M.MG_OP_SMOOTH, g.nlev - 1, 2)):
            g.set_field(fphi, phi0)
            g.set_field(frhs, rhs0)
            g.step(op | opf, lev, arg)
            out = g.get_field(fphi)
            if name not in ref:
                ref[name] = out
            assert np.array_equal(out, ref[name]), (tree, v, name)
    say("variants", tree, "fp32" if fp32 else "fp64", "all", M.MG_GSRB_VARIANTS, "identical")


@pytest.mark.parametrize("fp32", [False, True])
def test_persistent_sweeps_walk_several_boxes_on_the_benchmark_tree(fp32):
    """The persistent half-sweeps give a workgroup several boxes only on
    levels with more boxes than workgroups (2048 or 4096): on the benchmark
    tree's finest level (6784 boxes) they give the same bits as the one-box
    half-sweeps."""
    w = c2()
    g = M.Tree.from_workload(w)
    rng = np.random.default_rng(17)
    phi0 = rng.standard_normal((g.n, 8, 8, 8))
    rhs0 = rng.standard_normal((g.n, 8, 8, 8)) * 100.0
    if fp32:
        phi0, rhs0 = (a.astype(np.float32).astype(np.float64) for a in (phi0, rhs0))
    fphi, frhs = (M.MG_FIELD_E32, M.MG_FIELD_R32) if fp32 else (M.MG_FIELD_PHI, M.MG_FIELD_RHS)
    prec, opf = (M.MG_MIXED, M.MG_OP_F32) if fp32 else (M.MG_FP64, 0)
    ref = None
    for v in (3,) + M.MG_GSRB_PERSISTENT:
        M.mg_set_schedule(g.h, prec, [v] * g.nlev)
        g.set_field(fphi, phi0)
        g.set_field(frhs, rhs0)
        g.step(M.MG_OP_SMOOTH | opf, g.nlev, 3)
        out = g.get_field(fphi)
        if ref is None:
            ref = out
        assert np.array_equal(out, ref), v
    say("persistent variants on", g.n, "boxes:", "identical")


@pytest.mark.parametrize("v", M.MG_GSRB_FUSED + M.MG_GSRB_OCTET)
def test_fused_and_octet_sweeps_match_the_oracle(v):
    """Fused sweeps and octet half-sweeps against the oracle's sweep-by-sweep
    smoothing: per-cell Dirichlet data, a Neumann face and refinement
    boundaries."""
    g, o = bcval_tree()
    M.mg_set_schedule(g.h, M.MG_FP64, [v] * g.nlev)
    for op_g, op_o, lev, arg in ((M.MG_OP_SMOOTH, O.OP_SMOOTH, o.nlev, 2),
                                 (M.MG_OP_SMOOTH, O.OP_SMOOTH, o.nlev - 1, 4),
                                 (M.MG_OP_VCYCLE, O.OP_VCYCLE, o.nlev, 2)):
        seed_fields(g, o, 41)
        g.step(op_g, lev, arg)
        o.step(op_o, lev, arg)
        compare_fields(g, o, f"fused {v} op {op_g} level {lev}",
                       old_below=lev if op_g == M.MG_OP_VCYCLE else 0)


@pytest.mark.parametrize("wname", ["uniform64", "streamer_small", "forest"])
def test_fused_schedule_solve_parity(wname):
    """A whole FMG solve with fused sweeps on every level matches the oracle
    and the half-sweep solve bit for bit (on a forest too, where the fused
    down-sweep forms the coarse right-hand side of every tree's refined
    boxes in one launch)."""
    w = {"uniform64": c1, "streamer_small": streamer_small, "forest": small_forest}[wname]()
    g, o = pair(w)
    g.set_rhs_from(w)
    o.set_rhs_from(w)
    sh = g.fmg_solve()
    ph = g.get_field(M.MG_FIELD_PHI)
    M.mg_set_schedule(g.h, M.MG_FP64, [M.MG_GSRB_FUSED[1]] * g.nlev)
    sf = g.fmg_solve()
    pf = g.get_field(M.MG_FIELD_PHI)
    so = o.fmg_solve()
    leaf = o.leaf_mask()
    po = o.get_field(O.PHI)
    err = np.linalg.norm((pf - po)[leaf]) / np.linalg.norm(po[leaf])
    say("fused solve", wname, sf["n_vcycles"], "cycles, err vs oracle", err)
    assert sf["n_vcycles"] == so["n_vcycles"] == sh["n_vcycles"]
    assert err <= SOLVE_TOL
    assert np.array_equal(pf, ph)


@pytest.mark.parametrize("wname", ["streamer_small", "forest"])
def test_fused_schedule_mixed_solve_bits(wname):
    """Mixed precision: the FP32 correction cycles with fused sweeps on every
    level give the same refinement steps and the same FP64 potential, bit for
    bit, as with half-sweeps."""
    w = streamer_small() if wname == "streamer_small" else small_forest()
    g = M.Tree.from_workload(w, device="cuda:0")
    g.set_rhs_from(w)
    M.mg_set_schedule(g.h, M.MG_MIXED, [1] * g.nlev)  # one-box half-sweeps
    sh = g.fmg_solve(precision=M.MG_MIXED)
    ph = g.get_field(M.MG_FIELD_PHI)
    M.mg_set_schedule(g.h, M.MG_MIXED, [M.MG_GSRB_FUSED[1]] * g.nlev)
    sf = g.fmg_solve(precision=M.MG_MIXED)
    pf = g.get_field(M.MG_FIELD_PHI)
    say("mixed fused", wname, sh["n_vcycles"], sf["n_vcycles"], sf["rel"])
    assert sf["n_vcycles"] == sh["n_vcycles"]
    assert sf["rel"] <= 1e-8
    assert np.array_equal(pf, ph)


def test_autotune_keeps_the_solution(tmp_path, monkeypatch):
    from paper_1708_08434_amd import autotune
    monkeypatch.setenv("MG_TUNE_CACHE", str(tmp_path / "tune.json"))
    w = streamer_small()
    g = M.Tree.from_workload(w)
    g.set_rhs_from(w)
    s0 = g.fmg_solve()
    p0 = g.get_field(M.MG_FIELD_PHI)
    for prec in (M.MG_FP64, M.MG_MIXED):
        sched, cached = autotune.tune(g, prec, reps=4)
        assert not cached and len(sched) == g.nlev and all(0 <= v < M.MG_GSRB_VARIANTS for v in sched)
        say("autotuned", prec, sched)
    # the tuner leaves the solution in place
    assert np.array_equal(g.get_field(M.MG_FIELD_PHI), p0)
    s1 = g.fmg_solve()
    assert s1["n_vcycles"] == s0["n_vcycles"]
    assert np.array_equal(g.get_field(M.MG_FIELD_PHI), p0)
    sched2, cached = autotune.tune(g, M.MG_FP64, reps=4)
    assert cached


# ------------------------------------------------- bottom of the V-cycle

def mixed_forest_boxes():
    """Three trees: an AMR tree, a single root box (a leaf root), and a
    uniform two-level tree."""
    from workloads.octree import BoxList, uniform_boxes
    a = refine_boxes_explicit(2, [(2, 0, 0, 0), (3, 1, 1, 1), (3, 0, 1, 0), (4, 2, 2, 2)], tree=0)
    b = BoxList([1], [[0, 0, 0]], [1])
    c = uniform_boxes(2, tree=2)
    return BoxList.concat([a, b, c])


@pytest.mark.parametrize("top", [1, 2])
@pytest.mark.parametrize("prec", [M.MG_FP64, M.MG_MIXED], ids=["fp64", "mixed"])
def test_degenerate_trees_solve_like_the_oracle(top, prec):
    """The smallest trees: a single root box (the FMG pass is the exact root
    solve) and a uniform two-level tree (levels 1-2 only, one launch per
    cycle), with Dirichlet data on five faces and a Neumann face."""
    from workloads.octree import uniform_boxes
    bl = uniform_boxes(top)
    bct, bcv = (0, 0, 1, 0, 0, 0), (0.3, -0.2, 0.0, 0.1, 0.0, 1.0)
    g = M.Tree(bl.level, bl.ijk, bl.tree, bc_type=bct, bc_val=bcv)
    o = O.OracleTree(bl.level, bl.ijk, bl.tree, bc_type=bct, bc_val=bcv)
    rhs = np.random.default_rng(17 + top).standard_normal((g.n, 8, 8, 8)) * 50.0
    g.set_field(M.MG_FIELD_RHS, rhs)
    o.set_field(O.RHS, rhs)
    sg = g.fmg_solve(precision=prec)
    so = o.fmg_solve()
    leaf = o.leaf_mask()
    pg, po = g.get_field(M.MG_FIELD_PHI), o.get_field(O.PHI)
    err = np.linalg.norm((pg - po)[leaf]) / np.linalg.norm(po[leaf])
    say("degenerate", top, "levels", g.n, "boxes", sg["n_vcycles"], so["n_vcycles"], sg["rel"], "err", err)
    assert sg["rel"] <= 1e-8
    if prec == M.MG_FP64:
        assert sg["n_vcycles"] == so["n_vcycles"]
    assert err <= SOLVE_TOL, err


def run_both(g, fn):
    """fn(g) with levels 1-2 stepped level by level (schedule entry 0) and as
    one launch per tree; returns both results."""
    out = []
    for bot in (0, 1):
        for prec in (M.MG_FP64, M.MG_MIXED):
            M.mg_set_schedule(g.h, prec, [bot] + [3] * (g.nlev - 1))
        out.append(fn(g))
    return out


@pytest.mark.parametrize("tree", ["uniform64", "streamer_small", "bcval", "forest3"])
def test_bottom_kernel_gives_the_same_bits(tree):
    """One workgroup per tree for levels 1-2 (smoothing, residual,
    restriction, FAS right-hand side, root solve, prolongation) against the
    same steps as separate launches: V-cycles in FP64 and FP32, and a whole
    FMG solve."""
    if tree == "bcval":
        g, _ = bcval_tree()
        rhs0 = np.random.default_rng(2).standard_normal((g.n, 8, 8, 8)) * 100.0
    elif tree == "forest3":
        bl = mixed_forest_boxes()
        g = M.Tree(bl.level, bl.ijk, bl.tree, bc_type=(0, 0, 1, 0, 0, 0), bc_val=(0, 0, 0, 0, 0, 1.0))
        rhs0 = np.random.default_rng(3).standard_normal((g.n, 8, 8, 8)) * 100.0
    else:
        w = c1() if tree == "uniform64" else streamer_small()
        g = M.Tree.from_workload(w)
        rhs0 = w.rhs(g.index(M.MG_IDX_LEVEL), g.index(M.MG_IDX_IJK))
    rng = np.random.default_rng(11)
    phi0 = rng.standard_normal((g.n, 8, 8, 8))
    say("bottom", tree, g.n, "boxes", g.nlev, "levels")

    def vcyc(g):
        res = []
        for f_phi, f_rhs, opf, conv in ((M.MG_FIELD_PHI, M.MG_FIELD_RHS, 0, lambda a: a),
                                        (M.MG_FIELD_E32, M.MG_FIELD_R32, M.MG_OP_F32,
                                         lambda a: a.astype(np.float32).astype(np.float64))):
            g.set_field(f_phi, conv(phi0))
            g.set_field(f_rhs, conv(rhs0))
            g.step(M.MG_OP_VCYCLE | opf, g.nlev, 2)
            res.append(g.get_field(f_phi))
            g.set_field(f_phi, conv(phi0))
            g.set_field(f_rhs, conv(rhs0))
            g.step(M.MG_OP_VCYCLE | opf, 2, 3)  # V-cycle with level 2 on top, 3 sweeps
            res.append(g.get_field(f_phi))
        g.set_field(M.MG_FIELD_RHS, rhs0)
        st = g.fmg_solve()
        res.append(g.get_field(M.MG_FIELD_PHI))
        st2 = g.fmg_solve(precision=M.MG_MIXED)
        res.append(g.get_field(M.MG_FIELD_PHI))
        return res, (st["n_vcycles"], st2["n_vcycles"])
    (r0, c0), (r1, c1_) = run_both(g, vcyc)
    assert c0 == c1_, (c0, c1_)
    for q, (a, b) in enumerate(zip(r0, r1)):
        assert np.array_equal(a, b), (tree, q, np.abs(a - b).max())


def test_bottom_kernel_forest_matches_the_oracle():
    """The mixed forest (AMR tree, leaf root, uniform tree) solved with the
    one-launch bottom, against the oracle's forest solve."""
    bl = mixed_forest_boxes()
    kw = dict(bc_type=(0, 0, 1, 0, 0, 0), bc_val=(0, 0, 0, 0, 0, 1.0))
    g = M.Tree(bl.level, bl.ijk, bl.tree, **kw)
    o = O.OracleTree(bl.level, bl.ijk, bl.tree, (0.0, 0.0, 0.0), 1.0, kw["bc_type"], kw["bc_val"])
    assert np.array_equal(g.index(M.MG_IDX_ORDER), o.index(O.IDX_ORDER))
    lv, ij = o.index(O.IDX_LEVEL), o.index(O.IDX_IJK)
    x, y, z, h = G.cell_centres(lv, ij)
    rhs = -50.0 * np.exp(-((x - 0.4) ** 2 + (y - 0.5) ** 2 + (z - 0.6) ** 2) / 0.02)
    g.set_field(M.MG_FIELD_RHS, rhs)
    o.set_field(O.RHS, rhs)
    sg, so = g.fmg_solve(), o.fmg_solve()
    leaf = o.leaf_mask()
    pg, po = g.get_field(M.MG_FIELD_PHI), o.get_field(O.PHI)
    err = np.linalg.norm((pg - po)[leaf]) / np.linalg.norm(po[leaf])
    say("bottom forest", sg["n_vcycles"], so["n_vcycles"], err)
    assert sg["n_vcycles"] == so["n_vcycles"] and err <= SOLVE_TOL


def cs_order():
    """Natural cell index (k*8 + j)*8 + i of each colour-split position."""
    i, j, k = np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij")
    cs = ((i + j + k) & 1) * 256 + (k * 8 + j) * 4 + (i >> 1)
    nat = (k * 8 + j) * 8 + i
    out = np.empty(512, dtype=np.int64)
    out[cs.reshape(-1)] = nat.reshape(-1)
    return out


def test_borrowed_field_pointers():
    """mg_field lends the fields' own storage: its contents are the
    colour-split order of what mg_field_get copies out (FP64 and FP32), the
    level offsets are the tree's, a write through the pointer (announced by
    calling mg_field again) is what the next solve starts from, and a wrong
    dtype is refused."""
    import torch
    w = streamer_small()
    g = M.Tree.from_workload(w)
    g.set_rhs_from(w)
    g.fmg_solve(rel_tol=1e-6)
    g.fmg_solve(precision=M.MG_MIXED, rel_tol=1e-6)
    perm = cs_order()
    for which, dtype, tdt in ((M.MG_FIELD_PHI, M.MG_DTYPE_F64, torch.float64),
                              (M.MG_FIELD_RHS, M.MG_DTYPE_F64, torch.float64),
                              (M.MG_FIELD_E32, M.MG_DTYPE_F32, torch.float32)):
        ptr, n, lo = M.mg_field(g.h, which, dtype, g.nlev)
        assert n == 512 * g.n
        assert lo == [int(v) for v in g.info.level_start[:g.nlev + 1]]
        raw = torch.empty(n, dtype=tdt, device="cuda")
        M.mg_stream_copy(raw.data_ptr(), ptr, n * raw.element_size(), 0, g.stream.cuda_stream)
        g.stream.synchronize()
        nat = np.empty((g.n, 512))
        nat[:, perm] = raw.cpu().numpy().astype(np.float64).reshape(g.n, 512)
        assert np.array_equal(nat.reshape(g.n, 8, 8, 8), g.get_field(which)), which
    with pytest.raises(M.MGError) as e:
        M.mg_field(g.h, M.MG_FIELD_PHI, M.MG_DTYPE_F32)
    assert e.value.code == M.MG_EINVAL
    # write a converged potential through the pointer: warm V-cycles start from it
    g.fmg_solve(rel_tol=1e-10)
    conv = g.get_field(M.MG_FIELD_PHI, to_numpy=False)
    g.fmg_solve(rel_tol=1e-2)
    ptr, n, _ = M.mg_field(g.h, M.MG_FIELD_PHI, M.MG_DTYPE_F64)
    src = torch.empty(n, dtype=torch.float64, device="cuda")
    src[:] = conv.reshape(g.n, 512)[:, torch.from_numpy(perm).cuda()].reshape(-1)
    torch.cuda.synchronize()
    M.mg_stream_copy(ptr, src.data_ptr(), n * 8, 0, g.stream.cuda_stream)
    M.mg_field(g.h, M.MG_FIELD_PHI, M.MG_DTYPE_F64)
    st = g.vcycles(1)
    assert st["hist"][0] <= 1e-10, st["hist"]
