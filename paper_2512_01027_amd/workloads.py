"""Seeded synthetic inputs shaped like the paper's benchmark cases.

This module holds initial fields and case parameters only -- none of the
method's arithmetic -- so that the HIP path and the CPU reference can both be
fed from it.  Arrays are float64, node layout (nz, ny, nx) with x fastest;
velocity is (dim, nz, ny, nx).  Node i sits at coordinate i; a halfway wall
lies half a node outside the first and last node.

The interface profile is phi = 1/2 + 1/2 tanh(2 d / W), d the signed distance
into the heavy fluid (phi = 1), which is the stationary profile of the
conservative Allen-Cahn model (Sec. II) with interface width W.
"""
from __future__ import annotations

import math

import numpy as np

# Model constants used in every validation case of the paper (Sec. III):
# M = 0.166, W = 4, lambda_b = 1/6.
PAPER_M = 0.166
LAMBDA_B = 1.0 / 6.0


def base_case(dim: int, nx: int, ny: int, nz: int = 1, **kw) -> dict:
    cfg = {
        "dim": dim, "nx": nx, "ny": ny, "nz": nz if dim == 3 else 1,
        "q_hydro": 9 if dim == 2 else 27, "q_phase": 9 if dim == 2 else 19,
        "wall": (0, 0, 0), "delta_theta": 1,
        "rho_heavy": 1000.0, "rho_light": 1.0,
        "nu_heavy": 0.1, "nu_light": 0.1,
        "sigma": 0.01, "W": 4.0, "M": PAPER_M, "lambda_bulk": LAMBDA_B,
        "gravity": (0.0, 0.0, 0.0), "store": "fp64",
    }
    cfg.update(kw)
    return cfg


def _grid(cfg):
    nz, ny, nx = cfg["nz"], cfg["ny"], cfg["nx"]
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y, z


def tanh_profile(d, W):
    return 0.5 + 0.5 * np.tanh(2.0 * d / W)


def _zero_fields(cfg):
    shape = (cfg["nz"], cfg["ny"], cfg["nx"])
    return np.zeros(shape), np.zeros((cfg["dim"],) + shape)


def droplet(cfg, R, center=None, u0=None, P0=0.0, heavy_inside=True):
    """A sphere (3D) or disc (2D) of radius R; heavy fluid inside unless
    ``heavy_inside`` is False (a bubble)."""
    x, y, z = _grid(cfg)
    if center is None:
        center = (cfg["nx"] / 2.0, cfg["ny"] / 2.0, cfg["nz"] / 2.0)
    r2 = (x - center[0]) ** 2 + (y - center[1]) ** 2
    if cfg["dim"] == 3:
        r2 = r2 + (z - center[2]) ** 2
    d = R - np.sqrt(r2)
    phi = tanh_profile(d if heavy_inside else -d, cfg["W"])
    P, u = _zero_fields(cfg)
    P += P0
    if u0 is not None:
        for a in range(cfg["dim"]):
            u[a] += u0[a]
    return phi, P, u


def droplet_periodic(cfg, R, center, u0=None):
    """A heavy droplet of radius R centred anywhere in a periodic box: the
    distance is taken to the nearest periodic image, so the interface may
    cross the box's faces.  Built by broadcasting (one full-size temporary at
    a time), for grids of hundreds of millions of nodes."""
    nz, ny, nx = cfg["nz"], cfg["ny"], cfg["nx"]

    def axis(n, c):
        t = np.arange(n, dtype=np.float64) - c
        return t - n * np.round(t / n)

    dx = axis(nx, center[0])[None, None, :]
    dy = axis(ny, center[1])[None, :, None]
    dz = axis(nz, center[2])[:, None, None] if cfg["dim"] == 3 else np.zeros((1, 1, 1))
    r = dz * dz + (dx * dx + dy * dy)
    np.sqrt(r, out=r)
    np.subtract(R, r, out=r)
    np.multiply(r, 2.0 / cfg["W"], out=r)
    np.tanh(r, out=r)
    np.multiply(r, 0.5, out=r)
    np.add(r, 0.5, out=r)
    P, u = _zero_fields(cfg)
    if u0 is not None:
        for a in range(cfg["dim"]):
            u[a] += u0[a]
    return r, P, u


def config_droplet_max_grid(store="fp32", shape=(1024, 1024, 511), R=40.0):
    """The largest 3D grid the library accepts in 4-byte storage:
    1024 x 1024 x 511 (one field of 4-byte values is just under 2^31 bytes).
    Periodic; a droplet of radius R whose interface crosses all three pairs
    of faces (centre 0.6 R short of the high x face, 0.75 R past the low y
    face and 0.525 R short of the high z face), translated with
    u = (0.05, 0.02, 0.01); parameters of the 128^3 translated droplet."""
    nx, ny, nz = shape
    cfg = base_case(3, nx, ny, nz, sigma=0.005, nu_heavy=0.05, nu_light=0.05, W=4.0, store=store)
    center = (nx - 0.6 * R, 0.75 * R, nz - 0.525 * R)
    return cfg, droplet_periodic(cfg, R, center, u0=(0.05, 0.02, 0.01)), center


def slab(cfg, lo, hi, axis=0):
    """Heavy layer between two flat interfaces at coordinates lo < hi."""
    x, y, z = _grid(cfg)
    s = (x, y, z)[axis]
    d = np.minimum(s - lo, hi - s)
    phi = tanh_profile(d, cfg["W"])
    P, u = _zero_fields(cfg)
    return phi, P, u


def dam_block(cfg, bx, bz):
    """Heavy block x < bx, z < bz (all y) in the corner of a walled box."""
    x, y, z = _grid(cfg)
    dx = (bx - 0.5) - x
    dz = (bz - 0.5) - z
    d = np.minimum(dx, dz)
    corner = (dx < 0) & (dz < 0)
    d = np.where(corner, -np.sqrt(dx * dx + dz * dz), d)
    phi = tanh_profile(d, cfg["W"])
    P, u = _zero_fields(cfg)
    return phi, P, u


def add_noise(phi, amp, seed):
    """phi + U(-amp, amp) from NumPy PCG64(seed), clipped to [0, 1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.clip(phi + rng.uniform(-amp, amp, size=phi.shape), 0.0, 1.0)


def random_smooth(cfg, seed, amp=0.05, modes=3):
    """Random smooth periodic perturbations (sum of low Fourier modes)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x, y, z = _grid(cfg)
    out = np.zeros(x.shape)
    for _ in range(modes):
        kx, ky = rng.integers(1, 3, size=2)
        kz = rng.integers(1, 3) if cfg["dim"] == 3 else 0
        ph = rng.uniform(0, 2 * math.pi)
        a = rng.uniform(-amp, amp)
        out += a * np.sin(2 * math.pi * (kx * x / cfg["nx"] + ky * y / cfg["ny"] +
                                         kz * z / cfg["nz"]) + ph)
    return out


def shear_wave(cfg, amp=1e-4, heavy=False):
    """Single-phase u_x = amp sin(2 pi y / ny)."""
    x, y, z = _grid(cfg)
    phi = np.full(x.shape, 1.0 if heavy else 0.0)
    P, u = _zero_fields(cfg)
    u[0] = amp * np.sin(2 * math.pi * y / cfg["ny"])
    return phi, P, u


# ----------------------------------------------------------------- named cases

def config_static_droplet_2d():
    """2D 64x64 periodic static droplet R = 16 (rho ratio 1000, sigma 0.01,
    nu 0.1 both, W 4), D2Q9 / D2Q9, FP64."""
    cfg = base_case(2, 64, 64, sigma=0.01, nu_heavy=0.1, nu_light=0.1, W=4.0, store="fp64")
    phi, P, u = droplet(cfg, 16.0, center=(32.0, 32.0, 0.0))
    return cfg, (phi, P, u), 2000


def config_galilean_droplet_3d(n=128):
    """3D n^3 periodic droplet R = 24 translated with u = (0.05, 0.02, 0);
    D3Q27 hydro + D3Q19 phase field, FP32 store / FP32 compute."""
    cfg = base_case(3, n, n, n, sigma=0.005, nu_heavy=0.05, nu_light=0.05, W=4.0, store="fp32")
    R = 24.0 * n / 128.0
    phi, P, u = droplet(cfg, R, center=(n / 2, n / 2, n / 2), u0=(0.05, 0.02, 0.0))
    return cfg, (phi, P, u), 5000


def config_rising_bubble_3d(n=256, store="fp32", seed=1):
    """3D n^3 with walls in z and gravity -1e-6 z: air bubble R = 32 at a
    quarter height in water; phi + U(-1e-3, 1e-3) (seed 1)."""
    cfg = base_case(3, n, n, n, wall=(0, 0, 1), gravity=(0.0, 0.0, -1e-6), sigma=0.01,
                    nu_heavy=0.02, nu_light=0.2, W=5.0, store=store)
    R = 32.0 * n / 256.0
    phi, P, u = droplet(cfg, R, center=(n / 2, n / 2, n / 4), heavy_inside=False)
    phi = add_noise(phi, 1e-3, seed)
    return cfg, (phi, P, u), 4000


def config_dam_break_3d(nx=512, ny=256, nz=256, store="fp16", nu_light=0.15):
    """3D nx x ny x nz, walls on all faces, gravity -2e-6 z: water block
    (nx/4) x ny x (nz/2) in the corner; nu 0.01 (water) and nu_light (air)."""
    cfg = base_case(3, nx, ny, nz, wall=(1, 1, 1), gravity=(0.0, 0.0, -2e-6), sigma=0.005,
                    nu_heavy=0.01, nu_light=nu_light, W=4.0, store=store)
    phi, P, u = dam_block(cfg, nx // 4, nz // 2)
    return cfg, (phi, P, u), 20000


def config_dam_break_2d(nx=512, ny=256, store="fp32", nu_light=0.05):
    """The x-z slice of the all-walls dam break as a 2D case (y vertical):
    walls on all sides, gravity -2e-6 y, water block (nx/4) x (ny/2) in the
    corner; nu 0.01 (water) and nu_light (air)."""
    cfg = base_case(2, nx, ny, wall=(1, 1, 0), gravity=(0.0, -2e-6, 0.0), sigma=0.005,
                    nu_heavy=0.01, nu_light=nu_light, W=4.0, store=store)
    x, y, _ = _grid(cfg)
    dx = (nx // 4 - 0.5) - x
    dy = (ny // 2 - 0.5) - y
    d = np.minimum(dx, dy)
    corner = (dx < 0) & (dy < 0)
    d = np.where(corner, -np.sqrt(dx * dx + dy * dy), d)
    phi = tanh_profile(d, cfg["W"])
    P, u = _zero_fields(cfg)
    return cfg, (phi, P, u)


# Dam break against a block (Sec. III): container 3.22 x 1 x 1 m at 5.5 mm
# per node, water column H = 0.55 m high, block 0.161 x 0.403 x 0.161 m with
# its near face 0.744 m from the left end, centred across; water 999.10 and
# air 1.225 kg/m^3, nu 1.139e-6 and 1.461e-5 m^2/s, sigma 0.072 N/m; the
# characteristic velocity sqrt(2 g H) is 0.0289 in lattice units.  Only the
# geometry and the fluid parameters are used: the experiment's sensor records
# are not part of this workload.
DAM = {"L": 3.22, "B": 1.0, "Hbox": 1.0, "dx": 5.5e-3, "H": 0.55, "block": (0.161, 0.403, 0.161),
       "block_x": 0.744, "rho_w": 999.10, "rho_a": 1.225, "nu_w": 1.139e-6, "nu_a": 1.461e-5,
       "sigma": 0.072, "U": 0.0289}


def config_dam_break_block(store="fp16", nu_water=2e-3, column=0.25, q_hydro=27):
    """The dam break against a block (MARIN geometry of Sec. III) in lattice
    units: 585 x 182 x 182 nodes; walls on the sides and the floor, the top
    open at P = 0; gravity from sqrt(2 g H) = 0.0289 with H = 100 nodes;
    density ratio 815.6, air / water viscosity ratio 12.8 and sigma from the
    physical values at the time step that velocity fixes.  The water's
    physical viscosity would put tau within 1e-5 of 1/2, beyond what the
    step is stable at, so nu_water is a parameter (2e-3: tau = 0.506).  The
    paper does not give the water column's length: it is column x the
    container length, at the end away from the block.
    Returns cfg, fields and a dict with the block's position and the steps
    of one physical second."""
    d = DAM
    dx = d["dx"]
    nx, ny, nz = (int(round(v / dx)) for v in (d["L"], d["B"], d["Hbox"]))
    H = int(round(d["H"] / dx))
    g = d["U"] ** 2 / (2.0 * H)
    dt = dx * d["U"] / math.sqrt(2.0 * 9.81 * d["H"])
    sigma = d["sigma"] * dt * dt / (d["rho_a"] * dx ** 3)
    bx, by, bz = (int(round(v / dx)) for v in d["block"])
    x0 = int(round(d["block_x"] / dx))
    y0 = (ny - by) // 2
    cfg = base_case(3, nx, ny, nz, q_hydro=q_hydro, wall=(1, 1, 2), gravity=(0.0, 0.0, -g), p_top=0.0,
                    rho_heavy=d["rho_w"] / d["rho_a"], rho_light=1.0, nu_heavy=nu_water,
                    nu_light=nu_water * d["nu_a"] / d["nu_w"], sigma=sigma, W=4.0, store=store,
                    block=((x0, y0, 0), (x0 + bx, y0 + by, bz)))
    x, y, z = _grid(cfg)
    xc = nx - int(round(column * nx))
    dxw = x - (xc - 0.5)
    dzw = (H - 0.5) - z
    dist = np.minimum(dxw, dzw)
    corner = (dxw < 0) & (dzw < 0)
    dist = np.where(corner, -np.sqrt(dxw * dxw + dzw * dzw), dist)
    phi = tanh_profile(dist, cfg["W"])
    # hydrostatic pressure of the column, P = 0 above it (the open top's level)
    rho = cfg["rho_light"] + phi * (cfg["rho_heavy"] - cfg["rho_light"])
    P = np.zeros_like(phi)
    P[nz - 1] = 0.5 * g * rho[nz - 1]
    for k in range(nz - 2, -1, -1):
        P[k] = P[k + 1] + 0.5 * g * (rho[k] + rho[k + 1])
    u = np.zeros((3,) + phi.shape)
    blk = (slice(0, bz), slice(y0, y0 + by), slice(x0, x0 + bx))
    phi[blk] = 0.0
    P[blk] = 0.0
    info = {"block_face_x": x0 + bx, "column_start_x": xc, "steps_per_second": 1.0 / dt, "g": g}
    return cfg, (phi, P, u), info


# Table I of Sec. III.D: surrounding fluid density, dynamic viscosities of
# the surrounding fluid (1) and the bubble (2), surface tension.
TABLE1 = {1: {"rho1": 2.2, "mu1": 7.3e-3, "mu2": 7.3e-4, "sigma": 3.0e-5},
          2: {"rho1": 220.0, "mu1": 7.3e-1, "mu2": 7.3e-3, "sigma": 2.4e-4}}


def config_table1_bubble(case, store="fp64"):
    """2D rising bubble of Sec. III.D, Table I: 200 x 400, bubble R = 50 at
    (100, 100), g = 1.36e-8 along -y, bubble density 0.22; no-slip walls on
    all sides (the paper names no boundary conditions; the benchmark's box is
    closed).  Returns cfg, fields and the steps of one time unit
    sqrt(2R / g)."""
    t = TABLE1[case]
    rho2 = 0.22
    cfg = base_case(2, 200, 400, wall=(1, 1, 0), gravity=(0.0, -1.36e-8, 0.0), rho_heavy=t["rho1"],
                    rho_light=rho2, nu_heavy=t["mu1"] / t["rho1"], nu_light=t["mu2"] / rho2,
                    sigma=t["sigma"], W=4.0, store=store)
    phi, P, u = droplet(cfg, 50.0, center=(100.0, 100.0, 0.0), heavy_inside=False)
    unit = math.sqrt(2.0 * 50.0 / 1.36e-8)
    return cfg, (phi, P, u), unit


# Head-on binary collision of water droplets in air (Sec. III): relative
# velocity 2.45 m/s, radius 0.35 mm, surface tension 0.072 N/m, kinematic
# viscosities 1.51e-5 (air) and 1.00e-6 m^2/s (water), densities 1 and
# 1000 kg/m^3, so Re = U D / nu_water = 1715 and We = rho_water U^2 D / sigma
# = 58.4.
HEAD_ON = {"Re": 1715.0, "We": 58.4, "nu_air_over_water": 15.1}


def config_head_on_collision(D=64.0, U=0.06, grid=(256, 192, 192), gap=8.0, store="fp32", q_hydro=19,
                             offset=(0.0, 0.0, 0.0)):
    """Two water droplets of diameter D (nodes) in air approaching along x
    with relative velocity U (lattice units), periodic box.  The lattice
    units keep the paper's Re, We and air / water viscosity ratio:
    nu_water = U D / Re, nu_air = 15.1 nu_water, sigma = rho_water U^2 D / We.
    U D must keep nu_water near 2e-3 or above: at nu_water = 1.1e-3 the
    collision diverges (on the CPU reference as on the GPU), at 2.2e-3 it
    runs (U D = 3.84, the default D = 64, U = 0.06).
    D3Q19 for both lattices (the paper's 3D lattice) unless q_hydro = 27.
    Each droplet moves at U / 2 (weighted by its own phi) and holds the
    Laplace pressure 2 sigma / R; the droplets start gap nodes apart.
    offset moves the pair off the grid's mirror planes (on them, grad phi
    vanishes exactly at nodes where theta is not small, and the interface
    normal follows rounding).
    Returns cfg, fields and the steps of one time unit D / U."""
    nx, ny, nz = grid
    h = HEAD_ON
    nu_w = U * D / h["Re"]
    cfg = base_case(3, nx, ny, nz, q_hydro=q_hydro, sigma=1000.0 * U * U * D / h["We"], nu_heavy=nu_w,
                    nu_light=h["nu_air_over_water"] * nu_w, W=4.0, store=store)
    x, y, z = _grid(cfg)
    R = D / 2.0
    c1 = nx / 2.0 - R - gap / 2.0 + offset[0]
    c2 = nx / 2.0 + R + gap / 2.0 + offset[0]
    rr = (y - ny / 2.0 - offset[1]) ** 2 + (z - nz / 2.0 - offset[2]) ** 2
    p1 = tanh_profile(R - np.sqrt((x - c1) ** 2 + rr), cfg["W"])
    p2 = tanh_profile(R - np.sqrt((x - c2) ** 2 + rr), cfg["W"])
    # the sum, not the max: smooth across the gap (a kink there puts zeros of
    # lap(phi) where the delta-theta switch is active); p1 + p2 < 1 since the
    # profiles are logistic in 4 d / W and the droplets are gap apart
    phi = p1 + p2
    P, u = _zero_fields(cfg)
    P += 2.0 * cfg["sigma"] / R * phi
    u[0] = 0.5 * U * (p1 - p2)
    return cfg, (phi, P, u), int(round(D / U))


def serving_case(rng, store="fp16", max_nodes=None):
    """One request of the serving stream: 75% 3D (n log-uniform in [32, 192]),
    25% 2D (n log-uniform in [128, 1024]); static droplet or rising bubble;
    density ratio in {10, 100, 1000}; R = n/6; 1000..10000 steps.  With
    max_nodes, a request of more nodes is drawn but not built (None)."""
    is3d = rng.uniform() < 0.75
    if is3d:
        n = int(round(math.exp(rng.uniform(math.log(32), math.log(192)))))
    else:
        n = int(round(math.exp(rng.uniform(math.log(128), math.log(1024)))))
    kind = "droplet" if rng.uniform() < 0.5 else "bubble"
    ratio = float(rng.choice([10.0, 100.0, 1000.0]))
    steps = int(rng.integers(1000, 10001))
    dim = 3 if is3d else 2
    if max_nodes is not None and n ** dim > max_nodes:
        return None
    R = n / 6.0
    if kind == "droplet":
        cfg = base_case(dim, n, n, n, rho_heavy=ratio, rho_light=1.0, sigma=0.005 if is3d else 0.01,
                        nu_heavy=0.05, nu_light=0.05, W=4.0, store=store)
        phi, P, u = droplet(cfg, R)
    else:
        g = (0.0, -1e-6, 0.0) if dim == 2 else (0.0, 0.0, -1e-6)
        wall = (0, 1, 0) if dim == 2 else (0, 0, 1)
        cfg = base_case(dim, n, n, n, rho_heavy=ratio, rho_light=1.0, sigma=0.01, nu_heavy=0.02,
                        nu_light=0.2, W=5.0, wall=wall, gravity=g, store=store)
        c = (n / 2, n / 4, 0.0) if dim == 2 else (n / 2, n / 2, n / 4)
        phi, P, u = droplet(cfg, R, center=c, heavy_inside=False)
    return cfg, (phi, P, u), steps, kind
