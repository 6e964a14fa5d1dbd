"""Synthetic charge densities shaped like the paper's streamer runs.

All quantities are non-dimensional: the domain is the unit cube and eps0 = 1,
so the right-hand side handed to the solvers is b = -rho/eps0 = -rho
(the field equation of section 2.2, Poisson's equation with the space charge
e(n_i - n_e)).  Shapes follow section 3: a streamer is a charged channel whose
hemispherical head carries a thin positive surface-charge layer and whose sides
carry weak negative charge, the whole being electrically neutral.
"""
import numpy as np

from .rng import uniform01


def cell_centres(level, ijk, lo, length, pad=0):
    """Cell-centre coordinates of boxes at one level, optionally padded by
    ``pad`` cells on every side.  Returns x, y, z of shape [n, m, m, m]
    indexed [box][k][j][i] with m = 8 + 2*pad, plus the global cell indices."""
    ijk = np.asarray(ijk, dtype=np.int64).reshape(-1, 3)
    h = length / (8 * 2 ** (level - 1))
    loc = np.arange(-pad, 8 + pad, dtype=np.int64)
    I = (8 * ijk[:, 0])[:, None, None, None] + loc[None, None, None, :]
    J = (8 * ijk[:, 1])[:, None, None, None] + loc[None, None, :, None]
    K = (8 * ijk[:, 2])[:, None, None, None] + loc[None, :, None, None]
    shape = (len(ijk), len(loc), len(loc), len(loc))
    I, J, K = (np.broadcast_to(a, shape) for a in (I, J, K))
    x = lo[0] + (I + 0.5) * h
    y = lo[1] + (J + 0.5) * h
    z = lo[2] + (K + 0.5) * h
    return x, y, z, I, J, K


def gaussian_blob(x, y, z, amp, sigma, centre):
    r2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2
    return amp * np.exp(-r2 / (2.0 * sigma * sigma))


def channel_parts(x, y, z, p_top, p_head, radius, delta):
    """Unit-amplitude charge layers of one straight channel from ``p_top`` to
    the centre of its hemispherical head ``p_head``.

    Returns (head, side): head = exp(-(d-R)^2/2 delta^2) for points beyond the
    head centre (d = distance to p_head); side = exp(-(r_perp-R)^2/2 delta^2)
    for points whose projection falls on the channel body."""
    p0 = np.asarray(p_top, dtype=np.float64)
    p1 = np.asarray(p_head, dtype=np.float64)
    axis = p1 - p0
    length = np.linalg.norm(axis)
    u = axis / length
    dx, dy, dz = x - p0[0], y - p0[1], z - p0[2]
    t = dx * u[0] + dy * u[1] + dz * u[2]
    px, py, pz = dx - t * u[0], dy - t * u[1], dz - t * u[2]
    rperp = np.sqrt(px * px + py * py + pz * pz)
    d = np.sqrt((x - p1[0]) ** 2 + (y - p1[1]) ** 2 + (z - p1[2]) ** 2)
    inv = 1.0 / (2.0 * delta * delta)
    head = np.where(t > length, np.exp(-((d - radius) ** 2) * inv), 0.0)
    side = np.where((t >= 0) & (t <= length), np.exp(-((rperp - radius) ** 2) * inv), 0.0)
    return head, side


def noise(seed, level, I, J, K):
    """Uniform noise in [-1, 1) keyed by the global cell index."""
    return 2.0 * uniform01(seed, level, I, J, K) - 1.0
