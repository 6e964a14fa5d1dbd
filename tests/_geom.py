"""Geometry helpers shared by the tests (cell centres, boundary-face data,
closed-form solutions).  Pure input/expectation construction: none of the
solver's arithmetic lives here."""
import numpy as np
from scipy.special import erf


def cell_centres(level, ijk, length=1.0, lo=(0.0, 0.0, 0.0)):
    lv = np.asarray(level, dtype=np.float64)
    ij = np.asarray(ijk, dtype=np.float64).reshape(-1, 3)
    h = length / (8.0 * 2.0 ** (lv - 1))
    loc = np.arange(8) + 0.5
    H = h[:, None, None, None]
    x = lo[0] + (8 * ij[:, 0])[:, None, None, None] * H + loc[None, None, None, :] * H
    y = lo[1] + (8 * ij[:, 1])[:, None, None, None] * H + loc[None, None, :, None] * H
    z = lo[2] + (8 * ij[:, 2])[:, None, None, None] * H + loc[None, :, None, None] * H
    shape = (len(lv), 8, 8, 8)
    return (np.broadcast_to(x, shape).copy(), np.broadcast_to(y, shape).copy(),
            np.broadcast_to(z, shape).copy(), h)


def face_values(level, ijk, fn, length=1.0, lo=(0.0, 0.0, 0.0)):
    """[n][6][64] values of fn at the centres of the 64 face cells of each box
    face (faces -x,+x,-y,+y,-z,+z; tangential axes in increasing order, the
    first one fastest)."""
    lv = np.asarray(level, dtype=np.float64)
    ij = np.asarray(ijk, dtype=np.float64).reshape(-1, 3)
    n = len(lv)
    h = length / (8.0 * 2.0 ** (lv - 1))
    out = np.zeros((n, 6, 64))
    u = np.arange(8) + 0.5
    for d in range(6):
        a, s = d // 2, d % 2
        t1, t2 = (1, 2) if a == 0 else ((0, 2) if a == 1 else (0, 1))
        pos = [None, None, None]
        pos[a] = (lo[a] + (8 * ij[:, a] + (8 if s else 0)) * h)[:, None, None] * np.ones((1, 8, 8))
        pos[t1] = lo[t1] + (8 * ij[:, t1])[:, None, None] * h[:, None, None] \
            + u[None, None, :] * h[:, None, None]
        pos[t2] = lo[t2] + (8 * ij[:, t2])[:, None, None] * h[:, None, None] \
            + u[None, :, None] * h[:, None, None]
        pos = [np.broadcast_to(p, (n, 8, 8)) for p in pos]
        out[:, d, :] = fn(pos[0], pos[1], pos[2]).reshape(n, 64)
    return out


def gaussian_potential(x, y, z, amp, sigma, c=(0.5, 0.5, 0.5)):
    """Free-space potential of rho = amp exp(-r^2/2 sigma^2) with lap phi = -rho."""
    r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    small = r < 1e-12
    rs = np.where(small, 1.0, r)
    v = amp * sigma ** 3 * np.sqrt(np.pi / 2) * erf(rs / (np.sqrt(2) * sigma)) / rs
    return np.where(small, amp * sigma ** 2, v)


def gaussian_charge(x, y, z, amp, sigma, c=(0.5, 0.5, 0.5)):
    r2 = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2
    return amp * np.exp(-r2 / (2 * sigma ** 2))


def leaf_errors(phi, exact, leaf, h):
    """Volume-weighted L2 and max error over leaf cells."""
    e = (phi - exact)[leaf]
    vol = (h[leaf] ** 3)[:, None, None, None]
    l2 = np.sqrt((e * e * vol).sum())
    return l2, np.abs(e).max()


def old_read_mask(level, ijk, tree, child):
    """Per box: True where the multigrid's old copy of a coarse level is read
    by the prolongation of the correction into the next finer level, i.e. the
    box has children (its cells are covered and get the restricted value) or
    a same-level face or edge neighbour (same tree) has children.  Elsewhere
    the old field is scratch that the solver need not write."""
    lv = np.asarray(level).reshape(-1)
    ij = np.asarray(ijk).reshape(-1, 3)
    tr = np.zeros(len(lv), dtype=np.int64) if tree is None else np.asarray(tree).reshape(-1)
    refined = np.asarray(child).reshape(len(lv), -1)[:, 0] >= 0
    keys = {(int(tr[q]), int(lv[q]), int(ij[q, 0]), int(ij[q, 1]), int(ij[q, 2])) for q in np.nonzero(refined)[0]}
    offs = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)
            if 0 < abs(a) + abs(b) + abs(c) <= 2]
    out = refined.copy()
    for q in np.nonzero(~refined)[0]:
        t, l, i, j, k = int(tr[q]), int(lv[q]), int(ij[q, 0]), int(ij[q, 1]), int(ij[q, 2])
        out[q] = any((t, l, i + a, j + b, k + c) in keys for a, b, c in offs)
    return out
