"""Diagnostics of a rising bubble (Sec. III.D) and of a head-on droplet
collision (Sec. III) from the fields read back.

The bubble is the light fluid (phi < 1/2).  With its indicator weight
b = 1 - clamp(phi, 0, 1):
    centroid       x_c = sum b x / sum b
    rise velocity  v_c = sum b u / sum b
    circularity    perimeter of the circle of the bubble's area divided by
                   the perimeter of the phi = 1/2 contour (1 for a circle,
                   below 1 as the bubble deforms), with the contour traced by
                   marching squares on the node values.
Head-on collision (heavy fluid, phi >= 1/2, is water):
    droplets       connected pieces of phi >= 1/2 (faces connect; periodic
                   wrap joins pieces across the box edges)
    extent         largest distance of a water node from the collision axis
                   (the disc radius) and the water's length along the axis
    air speed      largest |u| where phi < 0.1, against the approach speed
Host-side numpy on arrays already copied back; not part of the time step.
"""
from __future__ import annotations

import math

import numpy as np


def _weights(phi):
    return 1.0 - np.clip(phi, 0.0, 1.0)


def centroid(phi):
    """(x, y[, z]) of the light-fluid indicator; phi indexed [z, y, x]."""
    b = _weights(phi)
    tot = b.sum()
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in phi.shape], indexing="ij")
    return tuple(float((b * g).sum() / tot) for g in reversed(grids))


def rise_velocity(phi, u):
    """Indicator-weighted mean velocity of the bubble, components (x, y[, z])."""
    b = _weights(phi)
    tot = b.sum()
    return tuple(float((b * u[a]).sum() / tot) for a in range(u.shape[0]))


def _contour_length(f, level=0.5):
    """Length of the level contour of a 2D field by marching squares: corners
    are classified by f >= level, an edge whose ends differ holds a crossing
    at the linear interpolation point, and the crossings of a cell are joined
    in edge order (two, or four in a saddle cell)."""
    a = f[:-1, :-1]
    b = f[:-1, 1:]
    c = f[1:, 1:]
    d = f[1:, :-1]
    # edges in order around the cell: (start, end, point at fraction t)
    edges = [(a, b, lambda t: (t, 0.0)), (b, c, lambda t: (1.0, t)), (c, d, lambda t: (1.0 - t, 1.0)),
             (d, a, lambda t: (0.0, 1.0 - t))]
    xs, ys, ms = [], [], []
    for p, q, place in edges:
        m = (p >= level) != (q >= level)
        t = np.where(m, (level - p) / np.where(m, q - p, 1.0), 0.0)
        x, y = place(t)
        xs.append(np.broadcast_to(x, p.shape))
        ys.append(np.broadcast_to(y, p.shape))
        ms.append(m)
    ms = np.stack(ms)
    xs = np.stack(xs)
    ys = np.stack(ys)
    n = ms.sum(axis=0)
    rank = np.cumsum(ms, axis=0) * ms  # 1, 2, ... for the crossing edges of a cell

    def kth(k):
        hit = rank == k
        return (xs * hit).sum(axis=0), (ys * hit).sum(axis=0)

    p1, p2, p3, p4 = kth(1), kth(2), kth(3), kth(4)
    seg1 = np.hypot(p1[0] - p2[0], p1[1] - p2[1])
    seg2 = np.hypot(p3[0] - p4[0], p3[1] - p4[1])
    return float(seg1[n >= 2].sum() + seg2[n == 4].sum())


def circularity(phi2d):
    """Circle perimeter of the bubble's area over its contour length (2D)."""
    area = float(_weights(phi2d).sum())
    return 2.0 * math.sqrt(math.pi * area) / _contour_length(phi2d)


def droplet_count(phi, level=0.5):
    """Number of connected water pieces (phi >= level) of a periodic 3D box,
    6-neighbour connectivity."""
    from scipy import ndimage

    lab, n = ndimage.label(phi >= level)
    if n == 0:
        return 0
    parent = list(range(n + 1))

    def root(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for ax in range(phi.ndim):
        lo = np.take(lab, 0, axis=ax)
        hi = np.take(lab, -1, axis=ax)
        for a, b in zip(lo[(lo > 0) & (hi > 0)], hi[(lo > 0) & (hi > 0)]):
            ra, rb = root(int(a)), root(int(b))
            if ra != rb:
                parent[ra] = rb
    return len({root(k) for k in range(1, n + 1)})


def collision_extent(phi, axis_yz=None, level=0.5):
    """(disc radius, length along x) of the water, phi indexed [z, y, x],
    collision axis along x through (y, z) = axis_yz (default: box centre)."""
    nz, ny, nx = phi.shape
    if axis_yz is None:
        axis_yz = (ny / 2.0, nz / 2.0)
    w = phi >= level
    if not w.any():
        return 0.0, 0.0
    z, y, x = np.nonzero(w)
    r = np.sqrt((y - axis_yz[0]) ** 2 + (z - axis_yz[1]) ** 2)
    return float(r.max()), float(x.max() - x.min() + 1)


def max_air_speed(phi, u, level=0.1):
    """Largest |u| over the air nodes (phi < level)."""
    air = phi < level
    if not air.any():
        return 0.0
    sp = np.sqrt((u ** 2).sum(axis=0))
    return float(sp[air].max())

