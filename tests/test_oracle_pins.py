"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test targets a plausible mistake: a wrong ghost weight or sign breaks
linear exactness; a wrong stencil breaks the quadratic test; a wrong
transfer or cycle step breaks convergence to the dense solution; a first-order
boundary or interface treatment breaks the convergence orders.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as O
from workloads import uniform_boxes, refine_boxes_explicit, c1, streamer_small
from workloads.octree import BoxList
from tests import _geom as G

HERE = os.path.dirname(os.path.abspath(__file__))


def amr_tree():
    return refine_boxes_explicit(2, [(2, 0, 0, 0), (3, 1, 1, 1), (3, 0, 1, 0), (4, 2, 2, 2)])


def make(bl, bc_type=(0,) * 6, bc_val=(0.0,) * 6):
    return O.OracleTree(bl.level, bl.ijk, bl.tree, (0, 0, 0), 1.0, bc_type, bc_val)


def geometry(t):
    return G.cell_centres(t.index(O.IDX_LEVEL), t.index(O.IDX_IJK))


# ------------------------------------------------------------ paper facts

def test_golden_mesh_geometry():
    """Section 3.1 and section 2.5 mesh facts follow from the convention that
    a tree's root is one 8^3 box and level l has spacing len / (8 2^(l-1))."""
    with open(os.path.join(HERE, "golden", "paper_mesh_facts.json")) as f:
        g = json.load(f)
    for case in g["cases"]:
        L = case["domain_mm"]
        h = lambda l: L / (8 * 2 ** (l - 1))
        if "coarse_dx_mm" in case:
            lc = [l for l in range(1, 20) if abs(h(l) - case["coarse_dx_mm"]) < 1e-12]
            assert lc and 8 * 2 ** (lc[0] - 1) == case["expect_coarse_cells_per_dim"]
        if case["rule"] == "nearest":
            lf = min(range(1, 30), key=lambda l: abs(np.log(h(l) / case["fine_dx_mm"])))
        else:  # the coarsest spacing not above the requested one
            lf = min(l for l in range(1, 30) if h(l) <= case["fine_dx_mm"] * (1 + 1e-9))
        assert abs(h(lf) - case["expect_fine_dx_mm"]) / case["expect_fine_dx_mm"] < 0.01
        if "expect_uniform_cells" in case:
            n = (8 * 2 ** (lf - 1)) ** 3
            assert abs(np.log10(n) - np.log10(case["expect_uniform_cells"])) < 0.1
        if "coarse_dx_mm" in case:
            assert lf - lc[0] == case["expect_refinement_levels"]


# ------------------------------------------------------------ validation

def _err(bl, **kw):
    with pytest.raises(O.OracleError) as e:
        make(bl, **kw)
    return e.value.name


def test_validation_rejects_bad_trees():
    good = amr_tree()
    make(good)  # accepted
    # missing root
    m = good.level != 1
    assert _err(BoxList(good.level[m], good.ijk[m])) == "ETOPO"
    # incomplete siblings: drop one level-5 box
    idx = np.where(good.level == 5)[0][0]
    m = np.ones(good.n, bool); m[idx] = False
    assert _err(BoxList(good.level[m], good.ijk[m])) == "ETOPO"
    # missing parent: a level-5 box whose parent is absent
    bl = BoxList(np.append(good.level, 4), np.vstack([good.ijk, [[7, 7, 7]]]))
    assert _err(bl) in ("ETOPO",)
    # duplicates
    bl = BoxList(np.append(good.level, good.level[3]), np.vstack([good.ijk, good.ijk[3:4]]))
    assert _err(bl) == "EINVAL"
    # out of range
    bl = BoxList(np.append(good.level, 2), np.vstack([good.ijk, [[2, 0, 0]]]))
    assert _err(bl) == "EINVAL"
    # 2:1 violation: refine the level-3 box (1,1,1) next to unrefined level-2
    # boxes, so level-4 boxes touch level-2 leaves
    u = uniform_boxes(2)
    oct8 = np.array([[a, b, c] for c in (0, 1) for b in (0, 1) for a in (0, 1)])
    bad = BoxList.concat([u, BoxList(np.full(8, 3), oct8), BoxList(np.full(8, 4), 2 + oct8)])
    assert _err(bad) == "ENESTING"
    # all-Neumann
    assert _err(good, bc_type=(1,) * 6) == "EINVAL"


def brute_tables(bl):
    """O(n^2) neighbour search straight from coordinates."""
    n = bl.n
    L, P = bl.level.astype(int), bl.ijk.astype(int)
    nbr = np.full((n, 6), -9)
    cfq = np.full((n, 6), -1)
    par = np.full(n, -1)
    for b in range(n):
        for c in range(n):
            if L[c] == L[b] - 1 and np.all(P[c] == P[b] // 2):
                par[b] = c
        for d in range(6):
            a, s = d // 2, d % 2
            q = P[b].copy(); q[a] += 1 if s else -1
            if q[a] < 0 or q[a] >= 2 ** (L[b] - 1):
                nbr[b, d] = -2
                continue
            hit = [c for c in range(n) if L[c] == L[b] and np.all(P[c] == q)]
            if hit:
                nbr[b, d] = hit[0]
            else:
                nbr[b, d] = -1
                cfq[b, d] = [c for c in range(n) if L[c] == L[b] - 1 and np.all(P[c] == q // 2)][0]
    return par, nbr, cfq


def test_index_tables_match_brute_force():
    bl = amr_tree().shuffled(7)
    t = make(bl)
    order = t.index(O.IDX_ORDER)
    par, nbr, cfq = brute_tables(bl)
    inv = np.empty(bl.n, int); inv[order] = np.arange(bl.n)  # caller index -> canonical

    def to_canon(a):
        return np.where(a >= 0, inv[np.maximum(a, 0)], a)
    assert np.array_equal(t.index(O.IDX_PARENT), to_canon(par[order]))
    assert np.array_equal(t.index(O.IDX_NBR), to_canon(nbr[order]))
    assert np.array_equal(t.index(O.IDX_CFQ), to_canon(cfq[order]))
    lv = t.index(O.IDX_LEVEL)
    assert np.all(np.diff(lv) >= 0)


# ------------------------------------------------------- operator pins

@pytest.mark.parametrize("axis", [0, 1, 2])
def test_linear_exact_paper_bc(axis):
    """Section 3.1 boundary setup: Dirichlet 0 / 1 on two opposite faces,
    Neumann zero on the others, no charge: the potential is linear, and the
    discrete solution must equal it at every leaf cell on any AMR tree."""
    bct = [1] * 6; bct[2 * axis] = 0; bct[2 * axis + 1] = 0
    bcv = [0.0] * 6; bcv[2 * axis + 1] = 1.0
    t = make(amr_tree(), bct, bcv)
    t.set_field(O.RHS, np.zeros((t.n, 8, 8, 8)))
    t.fmg_solve(tol=1e-13)
    x = geometry(t)
    leaf = t.leaf_mask()
    phi = t.get_field(O.PHI)
    assert np.abs(phi[leaf] - x[axis][leaf]).max() < 1e-11


def test_linear_exact_per_cell_dirichlet():
    """Dirichlet data g = a + bx + cy + dz on all faces: the solution is that
    linear function (exercises per-face-cell boundary data, refinement
    boundaries in all directions and the root solve)."""
    lin = lambda x, y, z: 0.3 + 1.1 * x - 0.7 * y + 2.0 * z
    bl = amr_tree()
    t = make(bl)
    t.set_bcval(G.face_values(t.index(O.IDX_LEVEL), t.index(O.IDX_IJK), lin))
    t.set_field(O.RHS, np.zeros((t.n, 8, 8, 8)))
    t.fmg_solve(tol=1e-13)
    x, y, z, h = geometry(t)
    leaf = t.leaf_mask()
    assert np.abs(t.get_field(O.PHI)[leaf] - lin(x, y, z)[leaf]).max() < 1e-11


def test_quadratic_interior_stencil():
    """phi = x^2 + y^2 + z^2 has a 7-point Laplacian of exactly 6 at every cell
    whose stencil stays inside the domain (box faces included)."""
    t = make(uniform_boxes(3))
    lv, ij = t.index(O.IDX_LEVEL), t.index(O.IDX_IJK)
    x, y, z, h = G.cell_centres(lv, ij)
    leaf = t.leaf_mask()
    q = (x * x + y * y + z * z)[leaf].reshape(-1)
    Lq = t.apply(q, homog=True).reshape(-1, 8, 8, 8)
    xl, yl, zl = x[leaf], y[leaf], z[leaf]
    hh = h[leaf][0]
    inner = np.ones(xl.shape, bool)
    for c in (xl, yl, zl):
        inner &= (c > hh) & (c < 1 - hh)
    assert inner.sum() > 10000
    assert np.abs(Lq[inner] - 6.0).max() < 1e-9


def test_root_operator_matches_kronecker_solve():
    """The exact coarsest solve equals a dense solve of the operator built as a
    Kronecker sum of 1-D second-difference matrices (independent assembly)."""
    bct = (0, 1, 0, 0, 1, 0)
    bcv = (0.5, 0.0, -0.25, 1.0, 0.0, 2.0)
    t = make(uniform_boxes(1), bct, bcv)
    rng = np.random.default_rng(3)
    b = rng.standard_normal((1, 8, 8, 8))
    t.set_field(O.RHS, b)
    t.step(O.OP_COARSE)
    phi = t.get_field(O.PHI)[0]
    h = 1.0 / 8

    def T1(lo_type, hi_type):
        T = -2 * np.eye(8) + np.eye(8, k=1) + np.eye(8, k=-1)
        T[0, 0] += -1 if lo_type == 0 else 1
        T[7, 7] += -1 if hi_type == 0 else 1
        return T
    I = np.eye(8)
    Tx, Ty, Tz = T1(bct[0], bct[1]), T1(bct[2], bct[3]), T1(bct[4], bct[5])
    # natural layout index (k, j, i): i fastest -> kron(z, y, x)
    A = (np.kron(I, np.kron(I, Tx)) + np.kron(I, np.kron(Ty, I)) + np.kron(Tz, np.kron(I, I))) / h ** 2
    rhs = b[0].copy()
    for d in range(6):
        if bct[d] != 0:
            continue
        a, s = d // 2, d % 2
        sl = [slice(None)] * 3
        sl[2 - a] = 7 if s else 0
        rhs[tuple(sl)] -= 2 * bcv[d] / h ** 2
    ref = np.linalg.solve(A, rhs.reshape(-1)).reshape(8, 8, 8)
    assert np.abs(phi - ref).max() <= 1e-12 * np.abs(ref).max()


# ------------------------------------------------ multigrid vs direct

def _dense_check(bl, rhs_seed):
    t = make(bl, (0,) * 6, (0.1, 0.2, 0.0, 0.4, 0.0, 1.0))
    leaf = t.leaf_mask()
    nl = int(leaf.sum()) * 512
    rng = np.random.default_rng(rhs_seed)
    b_all = np.zeros((t.n, 8, 8, 8))
    b_all[leaf] = rng.standard_normal((int(leaf.sum()), 8, 8, 8)) * 10
    # operator by probing unit vectors: column j = L e_j (homogeneous data)
    rows, cols, vals = [], [], []
    e = np.zeros(nl)
    for j in range(nl):
        e[j] = 1.0
        col = t.apply(e, homog=True)
        e[j] = 0.0
        nz = np.nonzero(col)[0]
        rows.append(nz); cols.append(np.full(len(nz), j)); vals.append(col[nz])
    A = sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(nl, nl))
    affine = t.apply(np.zeros(nl), homog=False)
    x = spla.spsolve(A, b_all[leaf].reshape(-1) - affine)
    t.set_field(O.RHS, b_all)
    st = t.fmg_solve(tol=1e-12)
    phi = t.get_field(O.PHI)[leaf].reshape(-1)
    return np.linalg.norm(phi - x) / np.linalg.norm(x), st


def test_mg_converges_to_direct_solution_uniform():
    err, st = _dense_check(uniform_boxes(2), 1)
    assert err < 1e-10, err


@pytest.mark.slow
def test_mg_converges_to_direct_solution_refined():
    """16^3 plus one refined box (7,680 unknowns): covers the refinement
    boundary ghosts, FAS transfers and prolongation across levels."""
    bl = refine_boxes_explicit(2, [(2, 1, 0, 1)])
    assert bl.n_leaf_cells() == 7680
    err, st = _dense_check(bl, 2)
    assert err < 1e-10, err


# ------------------------------------------------ discretisation order

def _sine_error(top):
    t = make(uniform_boxes(top))
    x, y, z, h = geometry(t)
    ex = np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)
    t.set_field(O.RHS, -3 * np.pi ** 2 * ex)
    t.fmg_solve(tol=1e-11)
    return G.leaf_errors(t.get_field(O.PHI), ex, t.leaf_mask(), h)


def test_second_order_uniform():
    """Section 2.3: the discretisation is second-order accurate."""
    errs = [_sine_error(l) for l in (2, 3, 4, 5)]
    for (a2, ai), (b2, bi) in zip(errs[1:], errs[2:]):
        assert np.log2(a2 / b2) >= 1.9
        assert np.log2(ai / bi) >= 1.9


def gaussian_amr(base, amp=100.0, sigma=0.08, centre=(0.3, 0.3, 0.3)):
    """Tree refined twice (the octant [0, 1/2]^3 at the base level, then
    [0, 1/4]^3), the same geometric regions at every base level, with a
    Gaussian charge that straddles both refinement boundaries and exact
    Dirichlet data from its free-space potential."""
    ref = []
    for m, ext in ((0, 0.5), (1, 0.25)):
        l = base + m
        nn = 2 ** (l - 1)
        k = int(round(ext * nn))
        ref += [(l, i, j, q) for q in range(k) for j in range(k) for i in range(k)]
    bl = refine_boxes_explicit(base, ref, max_level=base + 2)
    t = make(bl)
    lv, ij = t.index(O.IDX_LEVEL), t.index(O.IDX_IJK)
    pot = lambda x, y, z: G.gaussian_potential(x, y, z, amp, sigma, centre)
    t.set_bcval(G.face_values(lv, ij, pot))
    x, y, z, h = G.cell_centres(lv, ij)
    t.set_field(O.RHS, -G.gaussian_charge(x, y, z, amp, sigma, centre))
    return t, pot(x, y, z), h


def _amr_orders(centre, sigma):
    errs = []
    for base in (2, 3, 4):
        t, ex, h = gaussian_amr(base, sigma=sigma, centre=centre)
        t.fmg_solve(tol=1e-11)
        errs.append(G.leaf_errors(t.get_field(O.PHI), ex, t.leaf_mask(), h))
    l2 = [np.log2(a[0] / b[0]) for a, b in zip(errs, errs[1:])]
    li = [np.log2(a[1] / b[1]) for a, b in zip(errs, errs[1:])]
    return l2, li


@pytest.mark.slow
def test_second_order_amr_charge_refined():
    """Refinement around the charge, as the criterion of section 2.5 places it
    (the charge lies inside the finest region): second order in L2 and max."""
    l2, li = _amr_orders((0.125, 0.125, 0.125), 0.03)
    assert min(l2) >= 1.8 and min(li) >= 1.8, (l2, li)


@pytest.mark.slow
def test_amr_order_charge_across_refinement_boundary():
    """With charge straddling both refinement boundaries, the coarse cell next
    to a refined box sees the mean of the 8 children, which differs from the
    point value by H^2/32 lap(phi): an O(1) local error along the interface,
    proportional to rho there, so the L2 order falls towards one.  This
    property of the non-conservative coarse side is reported, and pinned from
    both sides so that a change of the interface treatment is noticed."""
    l2, li = _amr_orders((0.5, 0.5, 0.5), 0.08)
    assert 0.8 <= l2[-1] <= 1.5, l2


def test_fmg_reaches_discretisation_error():
    """Section 2.1.2: one FMG cycle gives a solution within (here: at most twice)
    the discretisation error."""
    for top in (3, 4):
        t = make(uniform_boxes(top))
        x, y, z, h = geometry(t)
        ex = np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)
        t.set_field(O.RHS, -3 * np.pi ** 2 * ex)
        t.fmg_solve(tol=1e30)  # FMG pass only
        e_fmg = G.leaf_errors(t.get_field(O.PHI), ex, t.leaf_mask(), h)[0]
        t.fmg_solve(tol=1e-12)
        e_conv = G.leaf_errors(t.get_field(O.PHI), ex, t.leaf_mask(), h)[0]
        assert e_fmg <= 2.0 * e_conv, (e_fmg, e_conv)


def test_vcycle_reduction_factor():
    """V(2,2) red-black Gauss-Seidel on 3-D Poisson: textbook-level
    convergence, mean reduction over cycles 2-6 on uniform 64^3 below 0.2."""
    w = c1()
    t = O.OracleTree.from_workload(w)
    t.set_rhs_from(w)
    t.set_field(O.PHI, np.zeros((t.n, 8, 8, 8)))
    st = t.vcycles(6)
    hist = st["hist"]
    factor = (hist[6] / hist[1]) ** (1 / 5)
    assert factor < 0.2, hist


# ------------------------------------------------------- invariants

def test_symmetry():
    """Section 3.3: a deterministic model keeps mirror symmetry.  A centred blob
    with the applied potential on the top face is invariant under x <-> 1-x,
    y <-> 1-y and x <-> y, so the solution must be too."""
    w = c1(noise_rel=0.0)
    t = O.OracleTree.from_workload(w)
    t.set_rhs_from(w)
    t.fmg_solve(tol=1e-10)
    lv, ij = t.index(O.IDX_LEVEL), t.index(O.IDX_IJK)
    leaf = t.leaf_mask()
    # rebuild a dense 64^3 array from the level-4 boxes
    phi = t.get_field(O.PHI)
    U = np.zeros((64, 64, 64))
    for b in np.where(leaf)[0]:
        i, j, k = ij[b]
        U[8 * k:8 * k + 8, 8 * j:8 * j + 8, 8 * i:8 * i + 8] = phi[b]
    scale = np.abs(U).max()
    assert np.abs(U - U[:, :, ::-1]).max() <= 1e-9 * scale
    assert np.abs(U - U[:, ::-1, :]).max() <= 1e-9 * scale
    assert np.abs(U - U.transpose(0, 2, 1)).max() <= 1e-9 * scale


def test_gauss_law_uniform():
    """Discrete divergence theorem on a uniform tree (section 3.4 relies on the
    neutrality of streamers): the boundary flux 2 (g - phi_in) h summed over
    boundary faces equals the volume sum of (b - r) h^3."""
    w = c1()
    t = O.OracleTree.from_workload(w)
    t.set_rhs_from(w)
    t.fmg_solve(tol=1e-6)
    lv, ij = t.index(O.IDX_LEVEL), t.index(O.IDX_IJK)
    leaf = t.leaf_mask()
    phi = t.get_field(O.PHI)
    U = np.zeros((64, 64, 64)); B = np.zeros((64, 64, 64))
    b = t.get_field(O.RHS)
    for q in np.where(leaf)[0]:
        i, j, k = ij[q]
        U[8 * k:8 * k + 8, 8 * j:8 * j + 8, 8 * i:8 * i + 8] = phi[q]
        B[8 * k:8 * k + 8, 8 * j:8 * j + 8, 8 * i:8 * i + 8] = b[q]
    h = 1 / 64
    g = w.bc_val
    flux = 0.0
    for a in range(3):
        lo_face = np.take(U, 0, axis=2 - a)
        hi_face = np.take(U, 63, axis=2 - a)
        flux += (2 * (g[2 * a] - lo_face)).sum() * h + (2 * (g[2 * a + 1] - hi_face)).sum() * h
    # residual r = b - L phi, so sum L phi h^3 = sum (b - r) h^3
    t.step(O.OP_RESIDUAL, 4)
    r = t.get_field(O.RES)
    R = np.zeros((64, 64, 64))
    for q in np.where(leaf)[0]:
        i, j, k = ij[q]
        R[8 * k:8 * k + 8, 8 * j:8 * j + 8, 8 * i:8 * i + 8] = r[q]
    vol = ((B - R) * h ** 3).sum()
    assert abs(flux - vol) <= 1e-10 * (np.abs(B).sum() * h ** 3)


def test_superposition():
    w = c1()
    base = O.OracleTree.from_workload(w)
    base.set_rhs_from(w)
    base.fmg_solve(tol=1e-11)
    t_rho = O.OracleTree(w.boxes.level, w.boxes.ijk, None, w.lo, 1.0, w.bc_type, (0.0,) * 6)
    t_rho.set_rhs_from(w)
    t_rho.fmg_solve(tol=1e-11)
    t_g = O.OracleTree.from_workload(w)
    t_g.set_field(O.RHS, np.zeros((t_g.n, 8, 8, 8)))
    t_g.fmg_solve(tol=1e-11)
    s = t_rho.get_field(O.PHI) + t_g.get_field(O.PHI)
    p = base.get_field(O.PHI)
    leaf = base.leaf_mask()
    assert np.abs(s[leaf] - p[leaf]).max() <= 1e-8 * np.abs(p[leaf]).max()


def test_warm_start_two_vcycles():
    """Section 2.1.2: after a change of the charge density, two V-cycles from
    the previous potential suffice; here a 1% change of b warm-started with two
    V-cycles ends below the residual of a cold FMG followed by two V-cycles."""
    w = streamer_small()
    t = O.OracleTree.from_workload(w)
    t.set_rhs_from(w)
    t.fmg_solve(tol=1e-8)
    b = t.get_field(O.RHS)
    leaf = t.leaf_mask()
    b2 = b.copy()
    b2[leaf] *= 1.01
    t.set_field(O.RHS, b2)
    warm = t.vcycles(2)["rel"]
    cold = O.OracleTree.from_workload(w)
    cold.set_field(O.RHS, b2)
    cst = cold.fmg_solve(tol=1e30)
    cold_rel = cold.vcycles(2)["rel"]
    assert warm <= cold_rel, (warm, cold_rel)
