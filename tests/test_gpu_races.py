"""Race checks of the tile-parallel kernels and the in-place AA pattern.

- Tile order: the same case run with its tiles taken in reverse order
  (pulbm_set_tile_order) must give bitwise the same fields.  Each tile then
  runs on another workgroup, XCD and time, so a kernel that read in one
  launch what another workgroup writes in the same launch (a missing step
  boundary, a population slot shared between tiles, an LDS buffer reused
  across tiles) would change the result.
- Repeatability: two runs of the same case are bitwise equal.
- In place against two buffers: the CPU reference streams into a second
  buffer (an A/B scheme); the FP64 parity tests (test_gpu_parity and the
  others) compare the in-place AA kernels with it at 1e-10 over up to 2000
  steps, which a race between the in-place reads and writes would break at
  the size of the populations.

Cases cover the interior and boundary paths (walls, open top, block), both
3D hydro lattices (D3Q27 and D3Q19 with the velocity rebuilt in collide),
2D, ragged tiles in every axis, the three storage widths, and odd and even
step counts.
"""
import numpy as np
import pytest

from paper_2512_01027_amd import binding as B
from paper_2512_01027_amd import workloads as W

pytestmark = pytest.mark.gpu


def _fields(cfg, seed=3):
    dim = cfg["dim"]
    R = 0.3 * min(cfg["nx"], cfg["ny"], cfg["nz"] if dim == 3 else 10 ** 9)
    phi, P, u = W.droplet(cfg, R, center=(cfg["nx"] * 0.45, cfg["ny"] * 0.55, cfg["nz"] * 0.5))
    phi = np.clip(phi + W.random_smooth(cfg, seed, amp=0.02), 0, 1)
    for a in range(dim):
        u[a] += W.random_smooth(cfg, seed + 1 + a, amp=0.01)
    return phi, P, u


CASES = {
    "3d_walls_block_open_top": lambda st: W.base_case(3, 150, 14, 12, wall=(1, 1, 2), gravity=(0, 0, -1e-5),
                                                       p_top=0.01, block=((60, 4, 0), (70, 10, 5)), store=st),
    "3d_periodic_d3q19": lambda st: W.base_case(3, 131, 10, 9, q_hydro=19, store=st),
    "3d_periodic_d3q27": lambda st: W.base_case(3, 140, 11, 7, store=st),
    "2d_walls_gravity": lambda st: W.base_case(2, 200, 75, wall=(1, 1, 0), gravity=(0, -1e-5, 0), store=st),
}


def _run(cfg, fields, steps, order):
    c = B.Case(cfg)
    c.set_tile_order(order)
    c.init_fields(*fields)
    c.step(steps)
    out = c.read_fields()
    c.close()
    return out


@pytest.mark.parametrize("store", ["fp64", "fp32", "fp16"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_reversed_tile_order_is_bitwise_equal(name, store):
    cfg = CASES[name](store)
    f = _fields(cfg)
    for steps in (7, 12):
        a = _run(cfg, f, steps, 0)
        b = _run(cfg, f, steps, 1)
        for fa, fb, nm in zip(a, b, ("phi", "P", "u")):
            assert np.isfinite(fa).all()
            assert np.array_equal(fa, fb), f"{name} {store} {steps} steps: {nm} depends on the tile order"


@pytest.mark.parametrize("store", ["fp32", "fp16"])
def test_runs_repeat_bitwise(store):
    cfg = CASES["3d_walls_block_open_top"](store)
    f = _fields(cfg, seed=8)
    a = _run(cfg, f, 9, 0)
    b = _run(cfg, f, 9, 0)
    for fa, fb in zip(a, b):
        assert np.array_equal(fa, fb)


def test_tile_order_switches_back():
    cfg = CASES["3d_periodic_d3q27"]("fp32")
    f = _fields(cfg)
    c = B.Case(cfg)
    c.init_fields(*f)
    c.step(3)
    c.set_tile_order(1)
    c.step(3)
    c.set_tile_order(0)
    c.step(3)
    mixed = c.read_fields()
    c.close()
    ref = _run(cfg, f, 9, 0)
    for fa, fb in zip(mixed, ref):
        assert np.array_equal(fa, fb)
    with pytest.raises(B.PulbmError):
        c2 = B.Case(cfg)
        try:
            c2.set_tile_order(2)
        finally:
            c2.close()
