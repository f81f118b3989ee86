"""Reference values at sampled nodes of a large case, from the CPU reference
run on a window around each sample.

One step of the method reads neighbours at most four hops away (the streamed
populations come from x - c; the stencils of the collision read phi and u at
x +- c; u needs the new pressure at x +- c; the pressure needs u* and the
previous pressure at x +- c).  After s steps (plus the read, which is the
moment stage once more) a node therefore depends only on nodes within
4 s + 6 hops along each axis.  A window of half-width larger than that, cut
out of the initial fields, reproduces the node's values exactly: the window
edge (periodic wrap of the window, or a wall where the window is cut inside
a walled axis) lies outside the dependency cone.  Windows at a real wall keep
that wall where it is, windows reaching an open end keep it open, and the
part of a solid block inside a window stays a block there (a sliver of it
thinner than two nodes at a cut window edge is left out: it lies outside
the cone).
"""
from __future__ import annotations

import numpy as np

import oracle


def cone(steps: int) -> int:
    return 4 * steps + 6


def window_axes(cfg, center, half):
    """Index ranges of the window along each axis and the window's flags."""
    dims = [cfg["nx"], cfg["ny"], cfg["nz"]]
    walls = list(cfg.get("wall", (0, 0, 0))) + [0, 0, 0]
    idx, wall, pos = [], [], []
    for a in range(3 if cfg["dim"] == 3 else 2):
        n, c = dims[a], int(center[a])
        if 2 * half + 1 >= n:  # the whole axis
            idx.append(np.arange(n))
            wall.append(walls[a])
            pos.append(c)
        elif walls[a]:
            lo, hi = max(0, c - half), min(n, c + half + 1)
            idx.append(np.arange(lo, hi))
            wall.append(2 if walls[a] == 2 and hi == n else 1)
            pos.append(c - lo)
        else:
            idx.append(np.arange(c - half, c + half + 1) % n)
            wall.append(0)
            pos.append(half)
    if cfg["dim"] == 2:
        idx.append(np.arange(1))
        wall.append(0)
        pos.append(0)
    return idx, wall, pos


def window_reference(cfg, fields, center, steps, half=None):
    """Oracle fields (phi, P, u) of the window after ``steps`` steps and the
    window's index arrays: values at window position p correspond to the
    full-grid node (ix[p_x], iy[p_y], iz[p_z])."""
    if half is None:
        half = cone(steps) + 2
    idx, wall, pos = window_axes(cfg, center, half)
    ix, iy, iz = idx
    phi, P, u = fields
    sel = np.ix_(iz, iy, ix)
    wphi = phi[sel]
    wP = P[sel]
    wu = np.stack([u[a][sel] for a in range(cfg["dim"])])
    wcfg = dict(cfg, nx=len(ix), ny=len(iy), nz=len(iz), wall=tuple(wall), store="fp64")
    if cfg.get("block"):
        blo, bhi = cfg["block"]
        lo_w, hi_w = [], []
        for a, arr in enumerate(idx):
            if np.any(np.diff(arr) != 1):
                raise ValueError("a block in a window that wraps a periodic axis")
            lo_w.append(int(np.clip(blo[a] - arr[0], 0, len(arr))))
            hi_w.append(int(np.clip(bhi[a] - arr[0], 0, len(arr))))
        keep = all(h > l for l, h in zip(lo_w, hi_w))
        for a, arr in enumerate(idx):
            full = lo_w[a] == 0 and hi_w[a] == len(arr)
            if not full and hi_w[a] - lo_w[a] < 2:
                keep = False
        wcfg["block"] = (tuple(lo_w), tuple(hi_w)) if keep else None
    o = oracle.OracleCase(wcfg)
    o.init_fields(wphi, wP, wu)
    o.step(steps)
    return o.read_fields(), (ix, iy, iz), pos


def _block(axes, pos, radius):
    sl = []
    for a, arr in enumerate(axes):
        p = pos[a]
        sl.append((max(0, p - radius), min(len(arr), p + radius + 1)))
    return sl


def ref_block(ref, axes, pos, radius):
    """The window reference's block of +-radius around pos."""
    (xl, xh), (yl, yh), (zl, zh) = _block(axes, pos, radius)
    rphi, rP, ru = ref
    return rphi[zl:zh, yl:yh, xl:xh], rP[zl:zh, yl:yh, xl:xh], ru[:, zl:zh, yl:yh, xl:xh]


def inner_block(fields_full, ref, axes, pos, radius):
    """The window's block of +-radius around pos, from the full-grid fields
    and from the window reference."""
    ix, iy, iz = axes
    (xl, xh), (yl, yh), (zl, zh) = _block(axes, pos, radius)
    sel_full = np.ix_(iz[zl:zh], iy[yl:yh], ix[xl:xh])
    phi, P, u = fields_full
    got = (phi[sel_full], P[sel_full], np.stack([u[a][sel_full] for a in range(u.shape[0])]))
    return got, ref_block(ref, axes, pos, radius)


def sample_centers(cfg, fields, count, seed):
    """Seeded sample nodes: half near the interface (0.05 < phi < 0.95), a
    quarter in the bulk, a quarter next to the walls or the grid corners."""
    rng = np.random.Generator(np.random.PCG64(seed))
    phi = fields[0]
    nz, ny, nx = phi.shape
    out = []
    iface = np.argwhere((phi > 0.05) & (phi < 0.95))
    bulk = np.argwhere((phi <= 0.05) | (phi >= 0.95))
    for k in range(count):
        if k % 4 in (0, 1) and len(iface):
            z, y, x = iface[rng.integers(len(iface))]
        elif k % 4 == 2 and len(bulk):
            z, y, x = bulk[rng.integers(len(bulk))]
        else:
            x = rng.choice([0, nx - 1, rng.integers(nx)])
            y = rng.choice([0, ny - 1, rng.integers(ny)])
            z = rng.choice([0, nz - 1, rng.integers(nz)])
        out.append((int(x), int(y), int(z)))
    return out
