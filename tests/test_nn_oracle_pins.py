"""Pins of the learned-smoother oracle (oracle/nn_oracle.py).

The network, its gradient and the optimiser are checked against library
routines that share none of the oracle's code (torch's BF16 conversion,
conv3d and autograd in FP64, torch.optim.Adam), against brute-force loops
and against central finite differences.  The learned step on a tree is
checked against the composite residual computed independently by the C
oracle, against linearity, and against least-squares optimality.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle as O
from oracle import nn_oracle as N
from workloads import uniform_boxes, refine_boxes_explicit
from tests import _geom as G


def _rand_params(seed, scale=1.0):
    p = N.init_params(seed) * scale
    rng = np.random.default_rng(seed + 1)
    W1, b1, W2, b2, W3, b3 = N.unpack(p)
    b1 = rng.standard_normal(16) * 0.1
    b2 = rng.standard_normal(16) * 0.1
    b3 = rng.standard_normal(1) * 0.1
    return N.pack(W1, b1, W2, b2, W3, b3).astype(np.float32).astype(np.float64)


def _rand_x(seed, B):
    return np.random.default_rng(seed).standard_normal((B, 10, 10, 10)).astype(np.float32) \
        .astype(np.float64)


def _torch_forward(p, x, round_bf16):
    W1, b1, W2, b2, W3, b3 = (torch.tensor(a) for a in N.unpack(p))
    xt = torch.tensor(x)[:, None]

    def rd(t):
        return t.to(torch.float32).to(torch.bfloat16).to(torch.float64) if round_bf16 else t

    h = F.conv3d(rd(xt), rd(W1).reshape(16, 1, 3, 3, 3), b1)
    h = rd(torch.relu(h))
    h = F.conv3d(h, rd(W2).reshape(16, 16, 3, 3, 3), b2, padding=1)
    h = rd(torch.relu(h))
    y = F.conv3d(h, rd(W3).reshape(1, 16, 3, 3, 3), b3, padding=1)
    return y[:, 0].numpy()


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(3)
    v = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38, 1e-40, -1e-40],
                        # exact ties between two BF16 values (round to even)
                        np.float32(1.0) + np.float32(2.0 ** -8) * np.array([1.0, 3.0, 5.0])])
    v = v.astype(np.float32)
    ref = torch.tensor(v).to(torch.bfloat16).to(torch.float64).numpy()
    got = N.bf16(v)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("round_bf16", [False, True])
def test_forward_matches_torch_conv3d(round_bf16):
    p = _rand_params(5)
    x = _rand_x(6, 3)
    y, _ = N.forward(p, x, round_bf16)
    ref = _torch_forward(p, x, round_bf16)
    err = np.abs(y - ref).max() / np.abs(ref).max()
    # FP64 summation order differs between einsum and conv3d; with BF16 the
    # rounding points coincide, so ties aside the results agree to FP64 level
    assert err < (1e-12 if not round_bf16 else 1e-6), err


def test_forward_bruteforce_cells():
    """Three output cells by plain loops over the definition."""
    p = _rand_params(7)
    x = _rand_x(8, 1)
    W1, b1, W2, b2, W3, b3 = N.unpack(p)
    y, _ = N.forward(p, x, round_bf16=False)

    def a1(o, i, j, k):
        if not (0 <= i < 8 and 0 <= j < 8 and 0 <= k < 8):
            return 0.0
        s = b1[o]
        for dk in range(3):
            for dj in range(3):
                for di in range(3):
                    s += W1[o, (dk * 3 + dj) * 3 + di] * x[0, k + dk, j + dj, i + di]
        return max(s, 0.0)

    A1 = {}

    def a1c(c, i, j, k):
        key = (c, i, j, k)
        if key not in A1:
            A1[key] = a1(c, i, j, k)
        return A1[key]

    def a2(o, i, j, k):
        if not (0 <= i < 8 and 0 <= j < 8 and 0 <= k < 8):
            return 0.0
        s = b2[o]
        for c in range(16):
            for dk in range(3):
                for dj in range(3):
                    for di in range(3):
                        s += W2[o, c, (dk * 3 + dj) * 3 + di] * a1c(c, i + di - 1, j + dj - 1,
                                                                    k + dk - 1)
        return max(s, 0.0)

    for (i, j, k) in [(0, 0, 0), (7, 3, 5), (4, 7, 1)]:
        s = b3[0]
        for c in range(16):
            for dk in range(3):
                for dj in range(3):
                    for di in range(3):
                        s += W3[c, (dk * 3 + dj) * 3 + di] * a2(c, i + di - 1, j + dj - 1,
                                                                k + dk - 1)
        assert abs(s - y[0, k, j, i]) <= 1e-12 * max(1.0, abs(s))


def test_gradients_match_torch_autograd():
    p = _rand_params(9)
    x = _rand_x(10, 2)
    tgt = np.random.default_rng(11).standard_normal((2, 8, 8, 8))
    L, g = N.gradients(p, x, tgt, round_bf16=False)
    pt = torch.tensor(p, requires_grad=True)
    o = 0
    parts = []
    for n in (N.N_W1, 16, N.N_W2, 16, N.N_W3, 1):
        parts.append(pt[o:o + n])
        o += n
    W1, b1, W2, b2, W3, b3 = parts
    h = torch.relu(F.conv3d(torch.tensor(x)[:, None], W1.reshape(16, 1, 3, 3, 3), b1))
    h = torch.relu(F.conv3d(h, W2.reshape(16, 16, 3, 3, 3), b2, padding=1))
    y = F.conv3d(h, W3.reshape(1, 16, 3, 3, 3), b3, padding=1)[:, 0]
    loss = torch.mean((y - torch.tensor(tgt)) ** 2)
    loss.backward()
    assert abs(L - loss.item()) <= 1e-13 * abs(L)
    ref = pt.grad.numpy()
    for lo, n in ((0, N.N_W1), (N.N_W1, 16), (N.N_W1 + 16, N.N_W2),
                  (N.N_W1 + 16 + N.N_W2, 16), (N.N_W1 + 32 + N.N_W2, N.N_W3),
                  (N.N_PARAMS - 1, 1)):
        seg, rs = g[lo:lo + n], ref[lo:lo + n]
        assert np.abs(seg - rs).max() <= 1e-11 * np.abs(rs).max()


def test_gradients_central_differences():
    p = _rand_params(12)
    x = _rand_x(13, 2)
    tgt = np.random.default_rng(14).standard_normal((2, 8, 8, 8))
    _, g = N.gradients(p, x, tgt, round_bf16=False)
    rng = np.random.default_rng(15)
    segs = [(0, N.N_W1), (N.N_W1, 16), (N.N_W1 + 16, N.N_W2), (N.N_W1 + 16 + N.N_W2, 16),
            (N.N_W1 + 32 + N.N_W2, N.N_W3), (N.N_PARAMS - 1, 1)]
    idx = np.concatenate([lo + rng.choice(n, min(n, 6), replace=False) for lo, n in segs])
    eps = 1e-6
    for q in idx:
        e = np.zeros_like(p)
        e[q] = eps
        fd = (N.loss(p + e, x, tgt, False) - N.loss(p - e, x, tgt, False)) / (2 * eps)
        assert abs(fd - g[q]) <= 1e-6 * max(1e-3, abs(g[q])) + 1e-9, (q, fd, g[q])


def test_adam_matches_torch():
    rng = np.random.default_rng(16)
    p0 = rng.standard_normal(50)
    grads = [rng.standard_normal(50) for _ in range(4)]
    pt = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([pt], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for k, g in enumerate(grads, start=1):
        opt.zero_grad()
        pt.grad = torch.tensor(g)
        opt.step()
        p, m, v = N.adam_step(p, g, m, v, k, lr=3e-3)
    assert np.abs(p - pt.detach().numpy()).max() <= 1e-14


# ------------------------------------------------------------ learned step

def _tree(bl):
    return O.OracleTree(bl.level, bl.ijk, bl.tree, (0, 0, 0), 1.0, (0,) * 6, (0.0,) * 6)


def test_gather_face_layers_linear_field():
    """A residual that is linear in the level's global cell index continues
    across same-level leaf faces; other ghosts and the block edges are 0."""
    bl = refine_boxes_explicit(2, [(2, 0, 0, 0)])  # level 2 (16^3) with one refined box
    t = _tree(bl)
    lv = t.index(O.IDX_LEVEL)
    ij = t.index(O.IDX_IJK)
    nbr = t.index(O.IDX_NBR)
    leaf = t.leaf_mask()
    loc = np.arange(8)
    gi = 8 * ij[:, 0][:, None, None, None] + loc[None, None, None, :]
    gj = 8 * ij[:, 1][:, None, None, None] + loc[None, None, :, None]
    gk = 8 * ij[:, 2][:, None, None, None] + loc[None, :, None, None]
    f = lambda i, j, k: 1.0 + 0.02 * i + 0.03 * j + 0.05 * k  # noqa: E731
    h = 1.0 / (8.0 * 2.0 ** (lv - 1))
    r = f(gi, gj, gk) / (h ** 2)[:, None, None, None]
    X, scale = N.gather_inputs(r, lv, nbr, leaf, 1.0)
    ids = np.nonzero(leaf)[0]
    assert len(ids) == 7 + 8
    for q, b in enumerate(ids):
        G_ = np.arange(10) - 1
        I = 8 * ij[b, 0] + G_[None, None, :]
        J = 8 * ij[b, 1] + G_[None, :, None]
        K = 8 * ij[b, 2] + G_[:, None, None]
        want = np.broadcast_to(f(I, J, K), (10, 10, 10)).copy()
        interior = want[1:9, 1:9, 1:9]
        assert abs(scale[q] - np.sqrt(np.mean(interior ** 2))) <= 1e-14 * scale[q]
        want /= scale[q]
        ghost = np.zeros((10, 10, 10), dtype=bool)
        for fc, dst, _ in N.face_ghost_layers():
            nb = nbr[b, fc]
            if nb >= 0 and leaf[nb]:
                ghost[dst] = True
        ghost[1:9, 1:9, 1:9] = True
        assert np.allclose(X[q][ghost], want[ghost], rtol=1e-14, atol=0)
        assert np.all(X[q][~ghost] == 0.0)
        if lv[b] == 2 and tuple(ij[b]) == (1, 0, 0):
            # its -x neighbour (0,0,0) is refined: that ghost layer is zero
            assert np.all(X[q][1:9, 1:9, 0] == 0.0)


def _poisson_tree():
    bl = refine_boxes_explicit(2, [(2, 1, 1, 1)])
    t = _tree(bl)
    x, y, z, _ = G.cell_centres(t.index(O.IDX_LEVEL), t.index(O.IDX_IJK))
    t.set_field(O.RHS, np.exp(-((x - 0.6) ** 2 + (y - 0.55) ** 2 + (z - 0.7) ** 2) / 0.02) * 50)
    return t


def test_residual_leaf_matches_oracle_norm():
    t = _poisson_tree()
    t.fmg_solve(tol=1e30)
    phi = t.get_field(O.PHI)
    st = t.residual()
    r = N.residual_leaf(t, phi)
    lv = t.index(O.IDX_LEVEL)
    vol = (1.0 / (8.0 * 2.0 ** (lv - 1))) ** 3
    l2 = np.sqrt(np.sum(vol[:, None, None, None] * r * r))
    assert abs(l2 - st["l2"]) <= 1e-12 * st["l2"]


def test_learned_step_linearity_and_optimality():
    t = _poisson_tree()
    t.fmg_solve(tol=1e30)
    p = _rand_params(20, scale=0.5)
    out = N.learned_step(t, p)
    r_new = N.residual_leaf(t, t.get_field(O.PHI))
    lv = t.index(O.IDX_LEVEL)
    leaf = t.leaf_mask()
    assert len(out["levels"]) == 2
    pred = out["r"].copy()
    for l in out["levels"]:
        pred -= out["s"][0, l] * out["q"][int(l)]
    assert np.abs(r_new[leaf] - pred[leaf]).max() <= 1e-9 * np.abs(out["r"]).max()
    # the recomputed residual is orthogonal to every level's column (the
    # normal equations of the least-squares step), and the step helps
    vol = (1.0 / (8.0 * 2.0 ** (lv - 1))) ** 3
    w = vol[leaf, None, None, None]
    nr = np.sqrt(np.sum(w * out["r"][leaf] ** 2))
    for l in out["levels"]:
        ql = out["q"][int(l)][leaf]
        ip = np.sum(w * r_new[leaf] * ql)
        assert abs(ip) <= 1e-9 * np.sqrt(np.sum(w * ql * ql)) * nr
        assert out["s"][0, l] != 0.0
    assert np.sum(w * r_new[leaf] ** 2) < nr ** 2


def test_learned_step_single_level_minimises():
    """On a tree whose leaves share one level, s is the exact minimiser of the
    true residual norm along c."""
    t = _tree(uniform_boxes(3))
    x, y, z, _ = G.cell_centres(t.index(O.IDX_LEVEL), t.index(O.IDX_IJK))
    t.set_field(O.RHS, np.sin(3 * x) * np.cos(2 * y) * z * 40)
    t.fmg_solve(tol=1e30)
    phi0 = t.get_field(O.PHI)
    p = _rand_params(21, scale=0.5)
    out = N.learned_step(t, p)
    lv = t.index(O.IDX_LEVEL)
    leaf = t.leaf_mask()
    vol = (1.0 / (8.0 * 2.0 ** (lv - 1))) ** 3

    def norm_at(s):
        r = N.residual_leaf(t, phi0 + s * out["c"])
        return np.sum(vol[leaf, None, None, None] * r[leaf] ** 2)

    s = out["s"][0, 3]
    f0 = norm_at(s)
    for d in (1e-3, -1e-3, 0.05, -0.05):
        assert norm_at(s + d * max(1.0, abs(s))) >= f0
    assert f0 <= norm_at(0.0)


def test_learned_step_zero_network_is_identity():
    t = _poisson_tree()
    t.fmg_solve(tol=1e30)
    phi = t.get_field(O.PHI)
    out = N.learned_step(t, np.zeros(N.N_PARAMS))
    assert np.all(out["c"] == 0) and np.all(out["s"] == 0)
    leaf = t.leaf_mask()
    assert np.array_equal(t.get_field(O.PHI)[leaf], phi[leaf])


def test_learned_step_scale_invariance():
    """Scaling b (homogeneous boundary data) and phi by 2^k leaves the inputs
    and the steps unchanged and scales the correction exactly."""
    p = _rand_params(22, scale=0.5)
    outs = []
    for a in (1.0, 1024.0):
        t = _poisson_tree()
        t.set_field(O.RHS, t.get_field(O.RHS) * a)
        t.fmg_solve(tol=1e30)
        outs.append(N.learned_step(t, p))
    assert np.allclose(outs[0]["X"], outs[1]["X"], rtol=1e-12, atol=1e-14)
    assert np.allclose(outs[0]["s"], outs[1]["s"], rtol=1e-9)
    assert np.allclose(outs[0]["c"] * 1024.0, outs[1]["c"], rtol=1e-12, atol=1e-300)


# ----------------------------------------------------- per-level placement

def _amr_state(seed):
    """The AMR pin tree (levels 2-5, refinement boundaries, refined same-level
    neighbours) with a random potential and right-hand side."""
    from tests.test_oracle_pins import amr_tree
    t = _tree(amr_tree())
    rng = np.random.default_rng(seed)
    t.set_field(O.RHS, rng.standard_normal((t.n, 8, 8, 8)) * 50.0)
    t.set_field(O.PHI, rng.standard_normal((t.n, 8, 8, 8)))
    return t


@pytest.mark.parametrize("level", [3, 4, 5])
def test_level_step_residual_orthogonal_to_its_column(level):
    """After the per-level step the level's residual (recomputed by the C
    oracle's residual step) equals r - s q, is orthogonal to q = A0 c over the
    level's leaf cells (the one-column normal equation) and is smaller."""
    t = _amr_state(40 + level)
    lv, leaf = t.index(O.IDX_LEVEL), t.leaf_mask()
    on = leaf & (lv == level)
    assert on.any()
    t.step(O.OP_RESIDUAL, level)
    r = t.get_field(O.RES)
    phi0 = t.get_field(O.PHI)
    p = _rand_params(30, scale=0.5)
    out = N.learned_step_level(t, p, level)
    if out["s"][0] == 0.0:
        # a correction against the residual gets no step; negating the last
        # layer negates the network's output, so the same state gets one
        W1, b1, W2, b2, W3, b3 = N.unpack(p)
        p = N.pack(W1, b1, W2, b2, -W3, -b3)
        t.set_field(O.PHI, phi0)
        out = N.learned_step_level(t, p, level)
    s = out["s"][0]
    assert s > 0.0
    t.step(O.OP_RESIDUAL, level)
    r_new = t.get_field(O.RES)
    # q from the composite operator on c alone (homogeneous), an independent path
    saved = t.get_field(O.PHI)
    q = np.zeros_like(phi0)
    q[leaf] = t.apply(out["c"][leaf].ravel(), homog=True).reshape(-1, 8, 8, 8)
    t.set_field(O.PHI, saved)
    assert np.abs((r_new - (r - s * q))[on]).max() <= 1e-10 * np.abs(r[on]).max()
    ip = np.sum(r_new[on] * q[on])
    assert abs(ip) <= 1e-10 * np.sqrt(np.sum(q[on] ** 2) * np.sum(r[on] ** 2))
    assert np.sum(r_new[on] ** 2) < np.sum(r[on] ** 2)
    # only the level's leaf boxes moved
    assert np.array_equal(saved[~on], phi0[~on])


def test_level_step_equals_the_composite_step_on_a_restricted_state():
    """With covered cells restricted, the level's residual is the composite
    residual on its leaf boxes, so the per-level correction is the composite
    step's correction on those boxes."""
    t = _amr_state(50)
    t.step(O.OP_RESTRICT_ALL)
    phi = t.get_field(O.PHI)
    p = _rand_params(31, scale=0.5)
    comp = N.learned_step(t, p)
    t.set_field(O.PHI, phi)
    lv, leaf = t.index(O.IDX_LEVEL), t.leaf_mask()
    for level in (3, 4, 5):
        t.set_field(O.PHI, phi)
        out = N.learned_step_level(t, p, level)
        on = leaf & (lv == level)
        assert np.allclose(out["c"][on], comp["c"][on], rtol=1e-10, atol=1e-12 * np.abs(comp["c"]).max())
        assert np.all(out["c"][~on] == 0.0)


def test_levels_vcycle_with_zero_network_is_the_plain_vcycle():
    """The per-level V-cycle, built from the oracle's single steps, with a
    zero network (zero correction, zero step) is bit for bit the oracle's
    own V-cycle."""
    a, b = _amr_state(60), _amr_state(60)
    N.vcycle_levels(a, np.zeros(N.N_PARAMS), a.nlev)
    b.step(O.OP_VCYCLE, b.nlev, 2)
    assert np.array_equal(a.get_field(O.PHI), b.get_field(O.PHI))
