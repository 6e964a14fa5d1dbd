"""Oracle of the learned correction smoother: a 3-layer 3-D convolutional
network that maps a box's residual to an error correction.

TEST INFRASTRUCTURE ONLY (imported by tests; shares no code with the GPU
library).  Plain NumPy in FP64.  Where the GPU stores BF16 (the input, the
weights, and the two hidden activations) the value is rounded to BF16 here
too (round to nearest even on the FP32 bit pattern), so both sides round at
the same points; all accumulation is exact FP64 here and FP32 on the GPU.

Network (one box, no batch coupling):
  x  : 10^3 input (the residual on the box and its face-ghost layer, scaled)
  z1 = conv(x, W1) + b1   valid 3^3, 1 -> 16 channels, 8^3 output
  a1 = bf16(relu(z1))
  z2 = conv(a1, W2) + b2  3^3 with zero padding ("same"), 16 -> 16
  a2 = bf16(relu(z2))
  y  = conv(a2, W3) + b3  3^3 "same", 16 -> 1
Layout: x[b, k, j, i] (10^3), activations a[b, c, k, j, i] (8^3), weights
W1[16][27], W2[16 out][16 in][27], W3[16 in][27], tap index
t = (dk*3 + dj)*3 + di for offsets (di, dj, dk) in {0,1,2}^3 (cell + tap - 1
in "same" layers, cell + tap in the valid layer).
Loss: mean over boxes and cells of (y - target)^2.
"""
import numpy as np

N_W1, N_W2, N_W3 = 16 * 27, 16 * 16 * 27, 16 * 27
N_PARAMS = N_W1 + 16 + N_W2 + 16 + N_W3 + 1  # 7776 weights + 33 biases


def bf16(a):
    """Round to BF16 (nearest, ties to even) and return as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounded = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    nan = np.isnan(f)
    out = rounded.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(nan, np.nan, out)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + N_W1].reshape(16, 27); o += N_W1
    b1 = p[o:o + 16]; o += 16
    W2 = p[o:o + N_W2].reshape(16, 16, 27); o += N_W2
    b2 = p[o:o + 16]; o += 16
    W3 = p[o:o + N_W3].reshape(16, 27); o += N_W3
    b3 = p[o:o + 1]
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])


def _taps():
    return [(t % 3, (t // 3) % 3, t // 9) for t in range(27)]


def _patches_valid(x):
    """x [B,10,10,10] -> [B, 27, 8,8,8] with patch[t] = x[cell + tap]."""
    return np.stack([x[:, dk:dk + 8, dj:dj + 8, di:di + 8] for di, dj, dk in _taps()], axis=1)


def _patches_same(a):
    """a [B,C,8,8,8] -> [B,C,27,8,8,8] with patch[t] = a[cell + tap - 1] (0 outside)."""
    p = np.pad(a, ((0, 0), (0, 0), (1, 1), (1, 1), (1, 1)))
    return np.stack([p[:, :, dk:dk + 8, dj:dj + 8, di:di + 8] for di, dj, dk in _taps()], axis=2)


def forward(params, x, round_bf16=True):
    """Returns y [B,8,8,8] and the intermediates needed by backward."""
    rd = bf16 if round_bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(params)
    W1, W2, W3 = rd(W1), rd(W2), rd(W3)
    xr = rd(x)
    P1 = _patches_valid(xr)                                    # [B,27,8,8,8]
    z1 = np.einsum("ot,btkji->bokji", W1, P1) + b1[None, :, None, None, None]
    a1 = rd(np.maximum(z1, 0.0))
    P2 = _patches_same(a1)                                     # [B,16,27,8,8,8]
    z2 = np.einsum("oct,bctkji->bokji", W2, P2) + b2[None, :, None, None, None]
    a2 = rd(np.maximum(z2, 0.0))
    P3 = _patches_same(a2)
    y = np.einsum("ct,bctkji->bkji", W3, P3) + b3[0]
    return y, dict(xr=xr, P1=P1, z1=z1, a1=a1, P2=P2, z2=z2, a2=a2, P3=P3, W1=W1, W2=W2, W3=W3)


def loss(params, x, target, round_bf16=True):
    y, _ = forward(params, x, round_bf16)
    return float(np.mean((y - target) ** 2))


def _conv_same_transpose(g, W):
    """Adjoint of the "same" convolution: g [B,O,8,8,8], W [O,I,27] ->
    [B,I,8,8,8] with out[cell] = sum_t sum_o W[o,i,t] g[o, cell - tap + 1]."""
    B = g.shape[0]
    I = W.shape[1]
    out = np.zeros((B, I, 8, 8, 8))
    gp = np.pad(g, ((0, 0), (0, 0), (1, 1), (1, 1), (1, 1)))
    for t, (di, dj, dk) in enumerate(_taps()):
        # cell' = cell + tap - 1  ->  cell = cell' - tap + 1
        sl = gp[:, :, 2 - dk:10 - dk, 2 - dj:10 - dj, 2 - di:10 - di]
        out += np.einsum("oc,bokji->bckji", W[:, :, t], sl)
    return out


def gradients(params, x, target, round_bf16=True):
    """Loss and its gradient w.r.t. the FP32 master parameters (the BF16
    rounding of the weights is treated as identity in the backward pass)."""
    y, c = forward(params, x, round_bf16)
    B = x.shape[0]
    n = B * 512
    gy = 2.0 * (y - target) / n                                  # [B,8,8,8]
    dW3 = np.einsum("bkji,bctkji->ct", gy, c["P3"])
    db3 = np.array([gy.sum()])
    ga2 = _conv_same_transpose(gy[:, None], c["W3"][None])      # [B,16,...]
    gz2 = ga2 * (c["a2"] > 0)
    dW2 = np.einsum("bokji,bctkji->oct", gz2, c["P2"])
    db2 = gz2.sum(axis=(0, 2, 3, 4))
    ga1 = _conv_same_transpose(gz2, c["W2"])
    gz1 = ga1 * (c["a1"] > 0)
    dW1 = np.einsum("bokji,btkji->ot", gz1, c["P1"])
    db1 = gz1.sum(axis=(0, 2, 3, 4))
    L = float(np.mean((y - target) ** 2))
    return L, pack(dW1, db1, dW2, db2, dW3, db3)


def adam_step(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) of FP32 master parameters."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# The learned correction step on an octree (applied after a V-cycle).
#
# Reading of the method's learned-smoother extension: the network sees, per
# leaf box, the residual scaled by h^2 on the box and on its six face-ghost
# layers (the residual of the adjacent same-level leaf box; zero where the
# face neighbour is coarser, refined, or outside the domain; zero on the
# edges and corners of the 10^3 block), normalised by the box's RMS of
# h^2 r (1 where that is zero).  Its output times the same scale is the
# correction c on the box.  With q = A c (the composite operator with
# homogeneous boundary data) of c_l, the correction restricted to the leaf
# boxes of level l, each tree takes the step sizes s_l that minimise the
# volume-weighted L2 norm of r - sum_l s_l q_l over its leaf cells (a linear
# least-squares problem; a level whose column vanishes or is not finite gets
# 0), and phi += sum_l s_l c_l on the boxes whose step is not 0.
# ---------------------------------------------------------------------------

def face_ghost_layers():
    """(face, ghost slice of the 10^3 block, source slice of the neighbour's 8^3 box)."""
    full = slice(1, 9)
    return [
        (0, (full, full, 0), (slice(None), slice(None), 7)),
        (1, (full, full, 9), (slice(None), slice(None), 0)),
        (2, (full, 0, full), (slice(None), 7, slice(None))),
        (3, (full, 9, full), (slice(None), 0, slice(None))),
        (4, (0, full, full), (7, slice(None), slice(None))),
        (5, (9, full, full), (0, slice(None), slice(None))),
    ]


def gather_inputs(r, level, nbr, leaf, length):
    """Network inputs of every leaf box (canonical order).

    r: [n,8,8,8] residual (read on leaf boxes only); level: [n]; nbr: [n,6]
    same-level face neighbour or negative; leaf: [n] bool.
    Returns X [nleaf,10,10,10] and the per-box scales [nleaf]."""
    ids = np.nonzero(leaf)[0]
    h = length / (8.0 * 2.0 ** (np.asarray(level) - 1))
    X = np.zeros((len(ids), 10, 10, 10))
    scale = np.ones(len(ids))
    for q, b in enumerate(ids):
        s = h[b] ** 2 * r[b]
        rms = np.sqrt(np.mean(s * s))
        if rms > 0:
            scale[q] = rms
        X[q, 1:9, 1:9, 1:9] = s
        for f, dst, src in face_ghost_layers():
            nb = nbr[b, f]
            if nb >= 0 and leaf[nb]:
                X[q][dst] = h[nb] ** 2 * r[nb][src]
        X[q] /= scale[q]
    return X, scale


def residual_leaf(tree, phi):
    """b - A phi on the leaf boxes ([n,8,8,8], zero elsewhere); leaves the
    tree's phi field at phi with covered cells restricted."""
    from . import RHS
    leaf = tree.leaf_mask()
    lap = tree.apply(phi[leaf].ravel(), homog=False).reshape(-1, 8, 8, 8)
    r = np.zeros_like(phi)
    r[leaf] = tree.get_field(RHS)[leaf] - lap
    return r


def learned_step(tree, params, round_bf16=True):
    """One learned correction of the tree's phi field.  Returns a dict with
    the correction c [n,8,8,8], the steps s [ntree, nlev+1] and the
    residual before the step."""
    from . import PHI, IDX_LEVEL, IDX_NBR, IDX_TREE
    phi = tree.get_field(PHI)
    leaf = tree.leaf_mask()
    level = tree.index(IDX_LEVEL)
    tid = tree.index(IDX_TREE)
    nbr = tree.index(IDX_NBR)
    r = residual_leaf(tree, phi)
    X, scale = gather_inputs(r, level, nbr, leaf, tree.length)
    y, _ = forward(params, X, round_bf16)
    c = np.zeros_like(phi)
    c[leaf] = scale[:, None, None, None] * y
    h = tree.length / (8.0 * 2.0 ** (level - 1))
    w = np.sqrt(h ** 3)
    levels = np.unique(level[leaf])
    q = {}
    for l in levels:
        cl = np.where((leaf & (level == l))[:, None, None, None], c, 0.0)
        ql = np.zeros_like(phi)
        ql[leaf] = tree.apply(cl[leaf].ravel(), homog=True).reshape(-1, 8, 8, 8)
        q[int(l)] = ql
    s = np.zeros((tree.ntree, tree.nlev + 1))
    for tr in range(tree.ntree):
        m = leaf & (tid == tr)
        wm = w[m][:, None, None, None]
        cols = [(wm * q[int(l)][m]).ravel() for l in levels]
        # a column that is not finite counts as vanishing (its level gets 0)
        ok = [bool(np.all(np.isfinite(col))) for col in cols]
        if any(ok):
            A = np.stack([col for col, k in zip(cols, ok) if k], axis=1)
            sol = np.linalg.lstsq(A, (wm * r[m]).ravel(), rcond=None)[0]
            s[tr, [l for l, k in zip(levels, ok) if k]] = sol
    new = phi.copy()
    sl = s[tid[leaf], level[leaf]]
    upd = sl != 0  # boxes whose step is 0 keep phi (also where c is not finite)
    new[np.nonzero(leaf)[0][upd]] += sl[upd][:, None, None, None] * c[leaf][upd]
    tree.set_field(PHI, new)
    return dict(c=c, s=s, r=r, q=q, X=X, scale=scale, levels=levels)


# Fallback rule (a reading): a learned step is kept while it lowers the
# relative residual to at most KEEP times its value after the V-cycle; the
# first time it does not, phi is restored and the solve continues with plain
# V-cycles.
KEEP = 0.99


def learned_solve(tree, params, tol=1e-8, max_cycles=50, n_down=2, n_up=2):
    """FMG, then V-cycles each followed by a learned step, with the stopping
    test of the plain solve.  Returns dict(rel, n_vcycles, hist, accepted,
    fallback)."""
    from . import PHI
    st = tree.fmg_solve(tol=1e300, max_cycles=0, n_down=n_down, n_up=n_up)
    rel = st["rel"]
    hist = [rel]
    use, accepted, fallback, stall, k = True, 0, 0, 0, 0
    while rel > tol:
        k += 1
        if k > max_cycles:
            raise O_error("no convergence within max_cycles")
        prev = rel
        rel = tree.vcycles(1, tol=0.0, n_down=n_down, n_up=n_up)["rel"]
        if rel > tol and use:
            saved = tree.get_field(PHI)
            learned_step(tree, params)
            rl = tree.residual()["rel"]
            if rl <= KEEP * rel:
                rel = rl
                accepted += 1
            else:
                tree.set_field(PHI, saved)
                tree.step(5)  # restriction pass: covered cells as before
                use, fallback = False, k
        hist.append(rel)
        if not np.isfinite(rel):
            raise O_error("non-finite residual")
        stall = stall + 1 if rel >= prev else 0
        if stall >= 3:
            raise O_error("residual stagnates")
    return dict(rel=rel, n_vcycles=k, hist=np.array(hist), accepted=accepted, fallback=fallback)


# ---------------------------------------------------------------------------
# Per-level placement (a learned step after the up-sweeps of each level;
# the paper has no learned component, so this is a reading).  Inside a V-cycle, right
# after the up-sweeps of a level l >= 3 that has leaf boxes:
#   r   = b - L_l phi on the level-l boxes, with the ghosts of the cycle (no
#         restriction of covered cells: the level's own cycle state);
#   x   = network inputs of the level-l leaf boxes, built from r exactly as for
#         the composite step (same-level leaf neighbours fill the ghost layer);
#   c   = scale * network(x) on those boxes, zero elsewhere;
#   q   = A0 c (the composite operator with homogeneous boundary data) on the
#         level-l leaf boxes;
#   s   = per tree, <r, q> / <q, q> over the tree's level-l leaf cells (the
#         one-column least-squares step; 0 when <q, q> is 0 or not finite, or
#         when s <= 0);
#   phi += s c on those boxes.
# The solve: the FMG pass, one plain V-cycle (its residual factor is the
# plain factor), then V-cycles with the per-level steps while each such
# cycle's factor does not exceed the plain one; the first that does makes
# the rest plain (no restore: the cycle still lowered the residual).
# ---------------------------------------------------------------------------

def learned_step_level(tree, params, level, round_bf16=True):
    """The per-level step on `level` of the tree's current cycle state.
    Returns dict(s [ntree], c)."""
    from . import PHI, RES, IDX_LEVEL, IDX_NBR, IDX_TREE, OP_RESIDUAL
    phi = tree.get_field(PHI)
    lv = tree.index(IDX_LEVEL)
    tid = tree.index(IDX_TREE)
    nbr = tree.index(IDX_NBR)
    leaf = tree.leaf_mask()
    on = leaf & (lv == level)
    if not on.any():
        return dict(s=np.zeros(tree.ntree), c=np.zeros_like(phi))
    tree.step(OP_RESIDUAL, level)
    r = np.where((lv == level)[:, None, None, None], tree.get_field(RES), 0.0)
    X, scale = gather_inputs(r, lv, nbr, on, tree.length)
    y, _ = forward(params, X, round_bf16)
    c = np.zeros_like(phi)
    c[on] = scale[:, None, None, None] * y
    q = np.zeros_like(phi)
    q[leaf] = tree.apply(c[leaf].ravel(), homog=True).reshape(-1, 8, 8, 8)
    s = np.zeros(tree.ntree)
    for tr in range(tree.ntree):
        m = on & (tid == tr)
        if not m.any():
            continue
        rq, qq = float(np.sum(r[m] * q[m])), float(np.sum(q[m] * q[m]))
        if qq > 0 and np.isfinite(qq) and np.isfinite(rq) and rq / qq > 0:
            s[tr] = rq / qq
    new = phi.copy()
    st = s[tid[on]]
    upd = st != 0
    ids = np.nonzero(on)[0][upd]
    new[ids] += st[upd][:, None, None, None] * c[ids]
    tree.set_field(PHI, new)  # also undoes the restriction the operator application made
    return dict(s=s, c=c)


def vcycle_levels(tree, params, top, n_down=2, n_up=2, low_step=3):
    """One V-cycle with the per-level learned step after the up-sweeps of every
    level >= low_step, from the single steps of the C oracle."""
    from . import OP_SMOOTH, OP_FAS_DOWN, OP_PROLONG, OP_COARSE
    for l in range(top, 1, -1):
        tree.step(OP_SMOOTH, l, n_down)
        tree.step(OP_FAS_DOWN, l)
    tree.step(OP_COARSE, 1)
    for l in range(2, top + 1):
        tree.step(OP_PROLONG, l)
        tree.step(OP_SMOOTH, l, n_up)
        if l >= low_step:
            learned_step_level(tree, params, l)


def learned_solve_levels(tree, params, tol=1e-8, max_cycles=50, n_down=2, n_up=2):
    """The per-level learned solve (see above).  Returns dict(rel, n_vcycles,
    hist, accepted, fallback)."""
    st = tree.fmg_solve(tol=1e300, max_cycles=0, n_down=n_down, n_up=n_up)
    rel = st["rel"]
    hist, plain, use, accepted, fallback, stall, k = [rel], None, True, 0, 0, 0, 0
    while rel > tol:
        k += 1
        if k > max_cycles:
            raise O_error("no convergence within max_cycles")
        prev = rel
        if k == 1 or not use:
            rel = tree.vcycles(1, tol=0.0, n_down=n_down, n_up=n_up)["rel"]
            if k == 1:
                plain = rel / prev
        else:
            vcycle_levels(tree, params, tree.nlev, n_down, n_up)
            rel = tree.residual()["rel"]
            if rel / prev > plain:
                use, fallback = False, k
            else:
                accepted += 1
        hist.append(rel)
        if not np.isfinite(rel):
            raise O_error("non-finite residual")
        stall = stall + 1 if rel >= prev else 0
        if stall >= 3:
            raise O_error("residual stagnates")
    return dict(rel=rel, n_vcycles=k, hist=np.array(hist), accepted=accepted, fallback=fallback)


def O_error(msg):
    from . import OracleError
    return OracleError(-5, msg)


def init_params(seed):
    """He-style initialisation, seeded (input generation only)."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((16, 27)) * np.sqrt(2.0 / 27)
    W2 = rng.standard_normal((16, 16, 27)) * np.sqrt(2.0 / 432)
    W3 = rng.standard_normal((16, 27)) * np.sqrt(1.0 / 432)
    return pack(W1, np.zeros(16), W2, np.zeros(16), W3, np.zeros(1))
