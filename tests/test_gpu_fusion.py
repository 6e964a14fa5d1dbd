"""Fused launch sequences (include/mg.h mg_set_fusion) against the unfused
ones, through the C ABI: every flag combination must give the same bits.

The unfused sequence is the one the oracle parity tests pin, step by step
and for whole solves; a fused sequence does the same arithmetic in the same
order on every value it produces, so the bar is bitwise equality of the
potential, the same cycle counts and the same residual histories, in FP64,
in the FP32 cycles of the mixed solve and for whole FMG solves.  The trees
cover every ghost type a fused kernel forms on the fly: same-level faces,
Dirichlet faces with constant and per-cell data, Neumann faces, refinement
boundaries, a forest with a leaf root, and the persistent, octet and fused
Gauss-Seidel schedules next to the plain half-sweeps."""
import numpy as np
import pytest

from paper_1708_08434_amd import mg as M
from workloads import c1, streamer_small, refine_boxes_explicit
from tests import _geom as G

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def make_tree(name):
    if name == "bcval":
        from workloads.configs import Workload, rhs_zero
        bl = refine_boxes_explicit(2, [(2, 0, 0, 0), (3, 1, 1, 1), (3, 0, 1, 0), (4, 2, 2, 2)])
        w = Workload("amr_bcval", bl, rhs_zero, bc_type=(0, 0, 1, 0, 0, 0))
        g = M.Tree.from_workload(w, per_cell_bc=True)
        lv, ij = g.index(M.MG_IDX_LEVEL), g.index(M.MG_IDX_IJK)
        g.set_field(M.MG_FIELD_BCVAL, G.face_values(lv, ij, lambda x, y, z: np.sin(3 * x) + y * z))
        rhs = np.random.default_rng(2).standard_normal((g.n, 8, 8, 8)) * 100.0
    elif name == "forest3":
        from workloads.octree import BoxList, uniform_boxes
        a = refine_boxes_explicit(2, [(2, 0, 0, 0), (3, 1, 1, 1), (3, 0, 1, 0), (4, 2, 2, 2)], tree=0)
        bl = BoxList.concat([a, BoxList([1], [[0, 0, 0]], [1]), uniform_boxes(2, tree=2)])
        g = M.Tree(bl.level, bl.ijk, bl.tree, bc_type=(0, 0, 1, 0, 0, 0), bc_val=(0, 0, 0, 0, 0, 1.0))
        rhs = np.random.default_rng(3).standard_normal((g.n, 8, 8, 8)) * 100.0
    elif name == "neumann_sides":
        # the paper's setup: Dirichlet bottom and top, Neumann sides (section 3.1)
        w = streamer_small()
        b = w.boxes
        g = M.Tree(b.level, b.ijk, b.tree, bc_type=(1, 1, 1, 1, 0, 0), bc_val=(0, 0, 0, 0, 0, 1.0))
        rhs = w.rhs(g.index(M.MG_IDX_LEVEL), g.index(M.MG_IDX_IJK))
    else:
        w = c1() if name == "uniform64" else streamer_small()
        g = M.Tree.from_workload(w)
        rhs = w.rhs(g.index(M.MG_IDX_LEVEL), g.index(M.MG_IDX_IJK))
    return g, rhs


SCHEDULES = {"half": 3, "persistent": 11, "octet": 9, "half_no_bottom": 3, "mixed_fused": None}


def schedule(g, kind):
    if SCHEDULES[kind] is not None:
        # level-1 entry: 0 = levels 1-2 step by step, else the one-launch bottom
        return [0 if kind == "half_no_bottom" else 3] + [SCHEDULES[kind]] * (g.nlev - 1)
    # fused sweeps on the middle levels, half-sweeps elsewhere (the tuner's
    # usual choice), the step-by-step bottom of the cycle
    return [0] + [7 if 2 <= l < g.nlev - 1 else 3 for l in range(2, g.nlev + 1)]


def run(g, rhs, phi0):
    out = []
    for f_phi, f_rhs, opf, conv in ((M.MG_FIELD_PHI, M.MG_FIELD_RHS, 0, lambda a: a),
                                    (M.MG_FIELD_E32, M.MG_FIELD_R32, M.MG_OP_F32,
                                     lambda a: a.astype(np.float32).astype(np.float64))):
        g.set_field(f_phi, conv(phi0))
        g.set_field(f_rhs, conv(rhs))
        g.step(M.MG_OP_VCYCLE | opf, g.nlev, 2)
        out.append(g.get_field(f_phi))
        g.set_field(f_phi, conv(phi0))
        g.set_field(f_rhs, conv(rhs))
        g.step(M.MG_OP_VCYCLE | opf, g.nlev, 1)
        out.append(g.get_field(f_phi))
    g.set_field(M.MG_FIELD_RHS, rhs)
    stats = []
    for prec in (M.MG_FP64, M.MG_MIXED):
        st = g.fmg_solve(precision=prec)
        out.append(g.get_field(M.MG_FIELD_PHI))
        stats.append((st["n_vcycles"], tuple(st["hist"])))
    return out, stats


@pytest.mark.parametrize("kind", list(SCHEDULES))
@pytest.mark.parametrize("name", ["uniform64", "streamer_small", "bcval", "forest3", "neumann_sides"])
def test_fusion_gives_the_same_bits(name, kind):
    g, rhs = make_tree(name)
    phi0 = np.random.default_rng(11).standard_normal((g.n, 8, 8, 8))
    sch = schedule(g, kind)
    for prec in (M.MG_FP64, M.MG_MIXED):
        M.mg_set_schedule(g.h, prec, sch)
    say("fusion", name, kind, g.n, "boxes", g.nlev, "levels, schedule", sch)
    M.mg_set_fusion(g.h, 0)
    ref, st_ref = run(g, rhs, phi0)
    M.mg_set_fusion(g.h, M.MG_FUSE_ALL)
    got, st_got = run(g, rhs, phi0)
    assert st_got == st_ref, (st_got, st_ref)
    for q, (a, b) in enumerate(zip(got, ref)):
        assert np.array_equal(a, b), (name, kind, q, np.abs(a - b).max())


def test_fusion_flags_are_checked():
    g, _ = make_tree("streamer_small")
    with pytest.raises(M.MGError) as e:
        M.mg_set_fusion(g.h, 1 << 20)
    assert e.value.code == M.MG_EINVAL


@pytest.mark.timeout(300)
def test_fusion_full_size_streamer_gives_the_same_bits():
    """The benchmark streamer tree (10,825 boxes, 9,472 leaf boxes): long
    enough that the persistent norm workgroups each walk several leaf boxes
    and the fused prolongation runs on levels of thousands of boxes; FP64 and
    mixed FMG solves with every flag against none."""
    from workloads import c2
    w = c2()
    g = M.Tree.from_workload(w)
    rhs = w.rhs(g.index(M.MG_IDX_LEVEL), g.index(M.MG_IDX_IJK))
    say("fusion full size", g.n, "boxes", int(g.info.n_leaf_boxes), "leaf boxes")
    out = {}
    for flags in (0, M.MG_FUSE_ALL):
        M.mg_set_fusion(g.h, flags)
        g.set_field(M.MG_FIELD_RHS, rhs)
        res = []
        for prec in (M.MG_FP64, M.MG_MIXED):
            st = g.fmg_solve(precision=prec)
            res.append((st["n_vcycles"], tuple(st["hist"]), g.get_field(M.MG_FIELD_PHI)))
        out[flags] = res
    for (na, ha, pa), (nb, hb, pb) in zip(out[0], out[M.MG_FUSE_ALL]):
        assert na == nb and ha == hb, (ha, hb)
        assert np.array_equal(pa, pb), np.abs(pa - pb).max()


def test_solve_statistics_count_the_recorded_launches():
    """The solve statistics report the kernel launches of the recorded FMG
    and per-cycle sequences; the fused sequences launch no more kernels than
    the unfused ones, in FP64 and in the mixed-precision solve."""
    g, rhs = make_tree("streamer_small")
    g.set_field(M.MG_FIELD_RHS, rhs)
    got = {}
    for flags in (0, M.MG_FUSE_ALL):
        M.mg_set_fusion(g.h, flags)
        for prec in (M.MG_FP64, M.MG_MIXED):
            st = g.fmg_solve(precision=prec)
            assert st["n_vcycles"] >= 2
            got[flags, prec] = (st["launches_fmg"], st["launches_cycle"])
            say("launches", flags, prec, got[flags, prec])
    for prec in (M.MG_FP64, M.MG_MIXED):
        f0, c0 = got[0, prec]
        f1, c1 = got[M.MG_FUSE_ALL, prec]
        assert 0 < c1 <= c0 and 0 < f1 <= f0
        assert f0 > c0 and f1 > c1

