"""Seeded synthetic workloads: an octree box list plus a right-hand side.

Each workload is a stand-in for the paper's streamer runs (section 3): the
unit cube plays the (40 mm)^3 domain, level 4 (64^3 cells) is the 625 um base
grid, the applied potential is 1 on the top face and 0 on the other faces, and
refinement follows the space-charge criterion of section 2.5 (refine where
|rho| h^2 exceeds a constant c3), here extended with a gradient term and a
three-cell buffer, with 2:1 nesting over all 26 neighbours.  The constant c3 is
tuned by log-bisection to hit a target leaf-cell count, and the tuned values
are cached in ``c3_cache.json`` next to this file.
"""
import json
import math
import os

import numpy as np

from . import charges
from .octree import BoxList, refine_by_score, uniform_boxes, pack

DIRICHLET, NEUMANN = 0, 1
_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_cache.json")


def _pmap(fn, items):
    """fn over items on a thread pool (NumPy releases the GIL in the array
    work), results in item order, so sums taken over them keep their order."""
    items = list(items)
    if len(items) <= 1:
        return [fn(it) for it in items]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(fn, items))


class Workload:
    """A tree (BoxList), a cubic domain with per-face boundary conditions, and
    a function giving b = -rho/eps0 at the cells of any set of boxes."""

    def __init__(self, name, boxes, rhs_fn, lo=(0.0, 0.0, 0.0), length=1.0,
                 bc_type=(DIRICHLET,) * 6, bc_val=(0, 0, 0, 0, 0, 1.0), meta=None):
        self.name = name
        self.boxes = boxes
        self._rhs_fn = rhs_fn
        self.lo = tuple(float(v) for v in lo)
        self.length = float(length)
        self.bc_type = tuple(int(v) for v in bc_type)
        self.bc_val = tuple(float(v) for v in bc_val)
        self.meta = dict(meta or {})

    def rhs(self, level, ijk, tree=None):
        """b at the cells of the given boxes, shape [n, 8, 8, 8] ([box][k][j][i])."""
        level = np.asarray(level).reshape(-1)
        ijk = np.asarray(ijk).reshape(-1, 3)
        tree = np.zeros(len(level), dtype=np.int32) if tree is None else np.asarray(tree).reshape(-1)
        out = np.zeros((len(level), 8, 8, 8))
        jobs = []
        for l in np.unique(level):
            idx = np.nonzero(level == l)[0]
            jobs += [(int(l), idx[s:s + 1024]) for s in range(0, len(idx), 1024)]

        def run(job):
            l, idx = job
            if getattr(self, "_rhs_tree_fn", None) is not None:
                out[idx] = self._rhs_tree_fn(l, ijk[idx], tree[idx])
            else:
                out[idx] = self._rhs_fn(l, ijk[idx])
        _pmap(run, jobs)
        return out

    @property
    def n_leaf(self):
        return self.boxes.n_leaf_cells()


# --------------------------------------------------------------------- small


def rhs_zero(level, ijk):
    return np.zeros((len(ijk), 8, 8, 8))


def c1(seed=1, top_level=4, amp=400.0, sigma=0.05, noise_rel=1e-3):
    """Uniform 64^3 grid (levels 1-4, 585 boxes): a Gaussian charge blob at the
    centre plus seeded uniform noise of relative amplitude 1e-3."""
    def fn(level, ijk):
        x, y, z, I, J, K = charges.cell_centres(level, ijk, (0.0, 0.0, 0.0), 1.0)
        rho = charges.gaussian_blob(x, y, z, amp, sigma, (0.5, 0.5, 0.5))
        rho = rho + noise_rel * amp * charges.noise(seed, level, I, J, K)
        return -rho
    return Workload("uniform64_blob", uniform_boxes(top_level), fn,
                    meta=dict(seed=seed, amp=amp, sigma=sigma, noise=noise_rel))


# ------------------------------------------------------------- streamers


class _Channels:
    """Streamer channels (top point, head centre) with head amplitude A_h and
    side amplitude A_s; sum of all channels."""

    def __init__(self, chans, radius, delta, amp_head, heads=None):
        self.chans = [(np.asarray(a, float), np.asarray(b, float)) for a, b in chans]
        self.heads = [True] * len(self.chans) if heads is None else list(heads)
        self.radius, self.delta, self.amp_head = radius, delta, amp_head
        body = sum(np.linalg.norm(b - a) for a, b in self.chans)
        # continuum estimate of neutrality: hemisphere area vs channel side area
        self.amp_side = amp_head * sum(self.heads) * radius / body

    def parts(self, x, y, z):
        head = np.zeros_like(x)
        side = np.zeros_like(x)
        for (p0, p1), has_head in zip(self.chans, self.heads):
            h, s = charges.channel_parts(x, y, z, p0, p1, self.radius, self.delta)
            if has_head:
                head += h
            side += s
        return head, side

    def rho(self, x, y, z):
        head, side = self.parts(x, y, z)
        return self.amp_head * head - self.amp_side * side

    def far(self, level, ijk, lo=(0.0, 0.0, 0.0), length=1.0, pad_cells=4, tails=8.0):
        """True for boxes whose region padded by pad_cells lies further than
        tails*delta from every channel surface (no charge to sample)."""
        ijk = np.asarray(ijk, dtype=np.float64).reshape(-1, 3)
        h = length / (8 * 2 ** (level - 1))
        c = np.asarray(lo) + (8 * ijk + 4) * h
        reach = np.sqrt(3.0) * (4 + pad_cells) * h + tails * self.delta
        near = np.zeros(len(c), dtype=bool)
        for p0, p1 in self.chans:
            ax = p1 - p0
            L = np.linalg.norm(ax)
            u = ax / L
            tpar = np.clip((c - p0) @ u, 0.0, L)
            dseg = np.linalg.norm(c - (p0 + tpar[:, None] * u), axis=1)
            dhead = np.linalg.norm(c - p1, axis=1)
            dsurf = np.minimum(np.abs(dseg - self.radius), np.abs(dhead - self.radius))
            near |= dsurf <= reach
        return ~near

    def neutralise(self, boxes, lo, length):
        """Set A_s so that the sum of rho*h^3 over the leaf cells vanishes."""
        leaf = boxes.leaf_mask()
        jobs = []
        for l in np.unique(boxes.level[leaf]):
            m = leaf & (boxes.level == l)
            ijk = boxes.ijk[m]
            jobs += [(int(l), ijk[s:s + 512]) for s in range(0, len(ijk), 512)]

        def part(job):
            l, ijk = job
            h = length / (8 * 2 ** (l - 1))
            x, y, z, *_ = charges.cell_centres(l, ijk, lo, length)
            a, b = self.parts(x, y, z)
            return a.sum() * h ** 3, b.sum() * h ** 3
        sh, ss = 0.0, 0.0
        for a, b in _pmap(part, jobs):
            sh += a
            ss += b
        if ss > 0:
            self.amp_side = self.amp_head * sh / ss


def _score_fn(rho_fn, lo, length, memo, far_fn=None):
    """max over a box and a 3-cell buffer of max(|rho| h^2, |grad rho| h^3).
    far_fn(level, ijk) -> bool marks boxes whose padded region holds no
    charge at all (score 0 without sampling)."""
    def score(level, ijk):
        keys = pack(ijk)
        d = memo.setdefault(level, {})
        out = np.empty(len(ijk))
        miss = [n for n, k in enumerate(keys.tolist()) if k not in d]
        if far_fn is not None and miss:
            far = far_fn(level, ijk[np.array(miss)])
            for n in np.array(miss)[far].tolist():
                d[int(keys[n])] = 0.0
            miss = [n for n in miss if int(keys[n]) not in d]
        h = length / (8 * 2 ** (level - 1))

        def chunk(idx):
            x, y, z, *_ = charges.cell_centres(level, ijk[idx], lo, length, pad=4)
            r = rho_fn(x, y, z)
            c = r[:, 1:-1, 1:-1, 1:-1]
            gx = (r[:, 1:-1, 1:-1, 2:] - r[:, 1:-1, 1:-1, :-2]) / (2 * h)
            gy = (r[:, 1:-1, 2:, 1:-1] - r[:, 1:-1, :-2, 1:-1]) / (2 * h)
            gz = (r[:, 2:, 1:-1, 1:-1] - r[:, :-2, 1:-1, 1:-1]) / (2 * h)
            crit = np.maximum(np.abs(c) * h * h, np.sqrt(gx * gx + gy * gy + gz * gz) * h ** 3)
            return crit.reshape(len(idx), -1).max(axis=1)
        parts = [np.array(miss[s:s + 256]) for s in range(0, len(miss), 256)]
        for idx, mx in zip(parts, _pmap(chunk, parts)):
            for n, v in zip(idx.tolist(), mx.tolist()):
                d[int(keys[n])] = v
        for n, k in enumerate(keys.tolist()):
            out[n] = d[k]
        return out
    return score


def _load_cache():
    if os.path.exists(_CACHE):
        with open(_CACHE) as f:
            return json.load(f)
    return {}


def tuned_tree(tag, rho_fn, base_level, max_level, target, lo=(0, 0, 0), length=1.0,
               tree=0, tol=0.1, use_cache=True, far_fn=None):
    """Balanced tree whose leaf-cell count is within ``tol`` of ``target``.
    c3 is found by log-bisection (and cached per ``tag``)."""
    memo = {}
    score = _score_fn(rho_fn, lo, length, memo, far_fn)
    cache = _load_cache() if use_cache else {}
    if tag in cache:
        c3 = cache[tag]
        return refine_by_score(base_level, max_level, score, c3, tree), c3
    lo_c, hi_c = -12.0, 6.0  # log10 bounds
    best = None
    for _ in range(40):
        mid = 0.5 * (lo_c + hi_c)
        bl = refine_by_score(base_level, max_level, score, 10 ** mid, tree)
        n = bl.n_leaf_cells()
        if best is None or abs(np.log(n / target)) < abs(np.log(best[0].n_leaf_cells() / target)):
            best = (bl, 10 ** mid)
        if abs(n - target) <= tol * target or hi_c - lo_c < 1e-3:
            break
        if n > target:
            lo_c = mid
        else:
            hi_c = mid
    return best


def save_c3(tag, c3):
    cache = _load_cache()
    cache[tag] = c3
    with open(_CACHE, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)


def c2(seed=2, refinements=4, target=5.0e6, amp_head=1e4, radius=0.02, delta=2e-3,
       z_head=0.62, use_cache=True):
    """Static AMR tree: base 64^3 (level 4) plus ``refinements`` levels, around
    one streamer along the z axis from z = 1 down to a hemispherical head
    centred at z = 0.62 (tip at 0.60), radius 0.02, head layer thickness 2e-3.
    The seed only fixes the tag; the shape is deterministic."""
    ch = _Channels([((0.5, 0.5, 1.0), (0.5, 0.5, z_head))], radius, delta, amp_head)
    base = 4
    tag = f"c2_s{seed}_r{refinements}_t{target:.3g}"
    bl, c3 = tuned_tree(tag, ch.rho, base, base + refinements, target, use_cache=use_cache)
    ch.neutralise(bl, (0.0, 0.0, 0.0), 1.0)

    def fn(level, ijk):
        x, y, z, *_ = charges.cell_centres(level, ijk, (0.0, 0.0, 0.0), 1.0)
        return -ch.rho(x, y, z)
    return Workload(f"streamer_L{base}+{refinements}", bl, fn,
                    meta=dict(seed=seed, c3=c3, amp_head=amp_head, amp_side=ch.amp_side,
                              radius=radius, delta=delta, target=target))


def c2_head_sequence(level, ijk, steps, dz, amp_head=1e4, radius=0.02, delta=2e-3, z_head=0.62):
    """Right-hand sides b = -rho of the C2 streamer on the unchanged C2 tree
    with its head centre moved down by s * dz, s = 0 .. steps-1 (the slow
    change of the charge between field solves of a time-stepped run), each
    neutralised on the C2 tree's leaf cells.  Returns [steps, n, 8, 8, 8] for
    the given boxes."""
    bl = c2().boxes
    level = np.asarray(level).reshape(-1)
    ijk = np.asarray(ijk).reshape(-1, 3)
    out = np.zeros((steps, len(level), 8, 8, 8))
    for s in range(steps):
        ch = _Channels([((0.5, 0.5, 1.0), (0.5, 0.5, z_head - s * dz))], radius, delta, amp_head)
        ch.neutralise(bl, (0.0, 0.0, 0.0), 1.0)

        def fn(lv, ij, ch=ch):
            x, y, z, *_ = charges.cell_centres(lv, ij, (0.0, 0.0, 0.0), 1.0)
            return -ch.rho(x, y, z)
        out[s] = Workload("c2_head_step", bl, fn).rhs(level, ijk)
    return out


E_CHARGE = 1.602176634e-19   # C
EPS0 = 8.8541878128e-12      # F/m


def paper_setup(n_head=1e19, length=0.04, volts=80e3):
    """The paper's field configuration in SI units (section 3.1): a (40 mm)^3
    domain with the base grid at 625 um (level 4 = 64^3), the bottom face
    grounded, 80 kV on the top face (a 2 MV/m background field along -z) and
    Neumann-zero sides.  The tree and the streamer are the C2 ones scaled to
    the domain; the charge density is e times a net ion-minus-electron density
    whose head layer peaks at n_head per m^3 (the channel sides neutralise
    it; 1e19 puts the head field near 10x the background, about what positive
    streamers reach in nitrogen at 1 bar), and the right-hand side is
    b = -rho / eps0 in V/m^2."""
    w = c2()
    scale = E_CHARGE * n_head / w.meta["amp_head"] / EPS0
    base_fn = w._rhs_fn

    def fn(level, ijk):
        return scale * base_fn(level, ijk)
    meta = dict(w.meta, n_head=n_head, length=length, volts=volts, e0=volts / length)
    return Workload("paper_setup_40mm", w.boxes, fn, length=length,
                    bc_type=(NEUMANN, NEUMANN, NEUMANN, NEUMANN, DIRICHLET, DIRICHLET),
                    bc_val=(0.0, 0.0, 0.0, 0.0, 0.0, volts), meta=meta)


def streamer_small(refinements=2, target=3.0e5, use_cache=True):
    """A reduced C2-shaped tree (base 32^3 + ``refinements`` levels) small enough
    for the CPU oracle to solve in a second or two."""
    ch = _Channels([((0.5, 0.5, 1.0), (0.5, 0.5, 0.62))], 0.04, 8e-3, 1e3)
    tag = f"small_r{refinements}_t{target:.3g}"
    bl, c3 = tuned_tree(tag, ch.rho, 3, 3 + refinements, target, use_cache=use_cache)
    ch.neutralise(bl, (0.0, 0.0, 0.0), 1.0)

    def fn(level, ijk):
        x, y, z, *_ = charges.cell_centres(level, ijk, (0.0, 0.0, 0.0), 1.0)
        return -ch.rho(x, y, z)
    return Workload(f"streamer_small_L3+{refinements}", bl, fn, meta=dict(c3=c3))


def c3(seed=3, refinements=6, target=3.0e7, amp_head=1e4, radius=0.015, delta=2e-3,
       use_cache=True):
    """Static AMR tree, base 64^3 plus ``refinements`` levels (effective
    4096^3), around a branched streamer: a trunk from (1/2, 1/2, 1) down to
    (1/2, 1/2, 0.8) and three seeded branches of length 0.25 from there, each
    at a polar angle U(10, 40) degrees from -z and azimuth 2 pi k / 3 +
    U(-0.3, 0.3), with a head at every branch tip (none at the fork);
    radius 0.015, head layer thickness 2e-3, neutralised."""
    rng = np.random.default_rng(seed)
    fork = np.array([0.5, 0.5, 0.8])
    chans, heads = [((0.5, 0.5, 1.0), tuple(fork))], [False]
    for k in range(3):
        pol = np.radians(rng.uniform(10.0, 40.0))
        az = 2.0 * np.pi * k / 3.0 + rng.uniform(-0.3, 0.3)
        d = np.array([np.sin(pol) * np.cos(az), np.sin(pol) * np.sin(az), -np.cos(pol)])
        chans.append((tuple(fork), tuple(fork + 0.25 * d)))
        heads.append(True)
    ch = _Channels(chans, radius, delta, amp_head, heads)
    base = 4
    tag = f"c3_s{seed}_r{refinements}_t{target:.3g}"
    bl, c3v = tuned_tree(tag, ch.rho, base, base + refinements, target, use_cache=use_cache,
                         far_fn=ch.far)
    ch.neutralise(bl, (0.0, 0.0, 0.0), 1.0)

    def fn(level, ijk):
        x, y, z, *_ = charges.cell_centres(level, ijk, (0.0, 0.0, 0.0), 1.0)
        return -ch.rho(x, y, z)
    return Workload(f"branched_L{base}+{refinements}", bl, fn,
                    meta=dict(seed=seed, c3=c3v, amp_head=amp_head, amp_side=ch.amp_side,
                              radius=radius, delta=delta, target=target,
                              branches=[list(map(float, b)) for _, b in chans[1:]]))


def _poisson_background(seed, base_level=4, lam=100.0):
    """(N_i - N_e) / lam per base-level cell, N ~ Poisson(lam) drawn by the
    inverse CDF of two counter-based uniforms per cell, [k][j][i]."""
    from scipy.stats import poisson
    from .rng import uniform01
    n = 8 << (base_level - 1)
    g = np.arange(n, dtype=np.int64)
    K, J, I = np.meshgrid(g, g, g, indexing="ij")
    u_i = uniform01(2 * seed, base_level, I, J, K)
    u_e = uniform01(2 * seed + 1, base_level, I, J, K)
    return (poisson.ppf(u_i, lam) - poisson.ppf(u_e, lam)) / lam


def _trilinear(grid, x, y, z):
    """Trilinear interpolation of cell-centred values on the unit cube
    (n^3 cells, [k][j][i]), clamped to the outermost cell centres."""
    n = grid.shape[0]
    def split(c):
        u = np.clip(c * n - 0.5, 0.0, n - 1.0)
        i0 = np.minimum(np.floor(u).astype(np.int64), n - 2)
        return i0, u - i0
    i0, fx = split(x)
    j0, fy = split(y)
    k0, fz = split(z)
    out = np.zeros_like(x)
    for dk in (0, 1):
        wz = fz if dk else 1.0 - fz
        for dj in (0, 1):
            wy = fy if dj else 1.0 - fy
            for di in (0, 1):
                wx = fx if di else 1.0 - fx
                out += wx * wy * wz * grid[k0 + dk, j0 + dj, i0 + di]
    return out


def c5(seed=5, refinements=7, target=1.0e8, amp_head=1e4, radius=0.02, delta=2e-3,
       use_cache=True):
    """Static AMR tree, base 64^3 plus ``refinements`` levels (effective
    8192^3), around two interacting streamers (axes x = 0.45 and 0.55 at
    y = 1/2, tips at z = 0.60 and 0.50; radius 0.02, head layer 2e-3,
    neutralised) plus a background ionisation 1e-3 A_h (N_i - N_e) / 100 with
    N ~ Poisson(100) per base 64^3 cell, interpolated trilinearly to the cell
    centres.  Refinement uses the channels' charge only (the background's
    |rho| h^2 is four orders of magnitude below the threshold)."""
    chans = [((0.45, 0.5, 1.0), (0.45, 0.5, 0.60 + radius)),
             ((0.55, 0.5, 1.0), (0.55, 0.5, 0.50 + radius))]
    ch = _Channels(chans, radius, delta, amp_head)
    base = 4
    tag = f"c5_s{seed}_r{refinements}_t{target:.3g}"
    bl, c3v = tuned_tree(tag, ch.rho, base, base + refinements, target, use_cache=use_cache,
                         far_fn=ch.far)
    ch.neutralise(bl, (0.0, 0.0, 0.0), 1.0)
    bg = 1e-3 * amp_head * _poisson_background(seed, base)

    def fn(level, ijk):
        x, y, z, *_ = charges.cell_centres(level, ijk, (0.0, 0.0, 0.0), 1.0)
        return -(ch.rho(x, y, z) + _trilinear(bg, x, y, z))
    return Workload(f"two_streamers_L{base}+{refinements}", bl, fn,
                    meta=dict(seed=seed, c3=c3v, amp_head=amp_head, amp_side=ch.amp_side,
                              radius=radius, delta=delta, target=target, background=1e-3))


def _forest_tree(t, refinements=5, base=3, lo_cells=1e5, hi_cells=2e6, use_cache=True):
    """Tree t of the forest: a seeded streamer, and the number of refinement
    levels (at most ``refinements``) and c3 that bring the leaf-cell count
    closest to a log-uniform target."""
    rng = np.random.default_rng(4000 + t)
    target = float(np.exp(rng.uniform(np.log(lo_cells), np.log(hi_cells))))
    tip = rng.uniform(0.55, 0.8)
    radius = rng.uniform(0.015, 0.03)
    delta = 0.1 * radius
    head = tip + radius
    ch = _Channels([((0.5, 0.5, 1.0), (0.5, 0.5, head))], radius, delta, 1e4)
    tag = f"forest_t{t}_r{refinements}_b{base}_t{target:.4g}"
    cache = _load_cache() if use_cache else {}
    if tag in cache:
        r, c3 = cache[tag]
        memo = {}
        bl = refine_by_score(base, base + int(r), _score_fn(ch.rho, (0, 0, 0), 1.0, memo, ch.far),
                             c3, t)
    else:
        best = None
        for r in range(1, refinements + 1):
            bl, c3 = tuned_tree(tag, ch.rho, base, base + r, target, tree=t, use_cache=False,
                                far_fn=ch.far)
            err = abs(np.log(bl.n_leaf_cells() / target))
            if best is None or err < best[0]:
                best = (err, bl, r, c3)
        _, bl, r, c3 = best
        if use_cache:
            save_c3(tag, [r, c3])
    ch.neutralise(bl, (0.0, 0.0, 0.0), 1.0)
    return bl, ch, (r, c3), target


def forest(n_trees=128, refinements=5, base=3, lo_cells=1e5, hi_cells=2e6, use_cache=True):
    """Forest of independent trees of uneven size (leaf cells log-uniform in
    [lo_cells, hi_cells]), each with one seeded streamer (tip height in
    [0.55, 0.8], radius in [0.015, 0.03], head layer thickness 0.1 R); tree t
    uses seed 4000 + t.  All trees share the unit-cube domain and boundary
    data, and differ in their charge."""
    parts = [_forest_tree(t, refinements, base, lo_cells, hi_cells, use_cache)
             for t in range(n_trees)]
    boxes = BoxList.concat([p[0] for p in parts])
    chans = [p[1] for p in parts]

    def fn_tree(level, ijk, tree):
        out = np.zeros((len(ijk), 8, 8, 8))
        for t in np.unique(tree):
            m = tree == t
            x, y, z, *_ = charges.cell_centres(level, ijk[m], (0.0, 0.0, 0.0), 1.0)
            out[m] = -chans[int(t)].rho(x, y, z)
        return out
    w = Workload(f"forest{n_trees}_L{base}+{refinements}", boxes, None,
                 meta=dict(c3=[p[2] for p in parts], targets=[p[3] for p in parts]))
    w._rhs_tree_fn = fn_tree
    return w
