"""The windowed reference used for full-size sampled parity: a window cut out
around a node reproduces the full-grid reference at that node (and its
neighbourhood) after a few steps, for periodic and walled axes, with gravity.
This pins the dependency-cone bound that the full-size GPU tests rely on.
"""
import numpy as np
import pytest

import oracle
from paper_2512_01027_amd import workloads as W

from _window import cone, inner_block, sample_centers, window_reference


def _case():
    cfg = W.base_case(3, 44, 40, 36, wall=(0, 0, 1), gravity=(0.0, 0.0, -1e-5), sigma=0.01,
                      nu_heavy=0.02, nu_light=0.2, W=5.0)
    phi, P, u = W.droplet(cfg, 9.0, center=(20.0, 22.0, 12.0), heavy_inside=False)
    phi = np.clip(phi + W.random_smooth(cfg, 3, amp=0.02), 0, 1)
    for a in range(3):
        u[a] += W.random_smooth(cfg, 4 + a, amp=0.01)
    return cfg, (phi, P, u)


@pytest.mark.parametrize("steps", [1, 2])
def test_window_reproduces_full_grid(steps):
    cfg, f = _case()
    o = oracle.OracleCase(cfg)
    o.init_fields(*f)
    o.step(steps)
    full = o.read_fields()
    half = cone(steps) + 2
    centers = [(20, 22, 0), (3, 38, 35), (20, 22, 12), (43, 0, 18)]
    for c in centers:
        ref, axes, pos = window_reference(cfg, f, c, steps, half)
        got, want = inner_block(full, ref, axes, pos, 2)
        for a, b in zip(got, want):
            assert np.abs(a - b).max() <= 1e-13 * max(np.abs(b).max(), 1e-300), c


def test_window_too_small_is_detected():
    """A window narrower than the cone differs: the bound is not vacuous."""
    cfg, f = _case()
    o = oracle.OracleCase(cfg)
    o.init_fields(*f)
    o.step(2)
    full = o.read_fields()
    ref, axes, pos = window_reference(cfg, f, (20, 22, 12), 2, half=3)
    got, want = inner_block(full, ref, axes, pos, 0)
    assert max(np.abs(a - b).max() for a, b in zip(got, want)) > 1e-9


def test_sample_centers_cover_walls_and_interface():
    cfg, f = _case()
    cs = sample_centers(cfg, f, 16, 1)
    assert len(cs) == 16
    assert any(z in (0, cfg["nz"] - 1) for _, _, z in cs)
    assert any(0.05 < f[0][z, y, x] < 0.95 for x, y, z in cs)


def test_window_with_block_and_open_top():
    """Windows cut out of a case with a block and an open top keep the part
    of the block inside them and the open end when they reach it."""
    cfg = W.base_case(3, 60, 40, 44, wall=(1, 1, 2), gravity=(0.0, 0.0, -1e-5), p_top=0.01, nu_heavy=0.05,
                      nu_light=0.15, sigma=0.01, block=((20, 10, 0), (28, 30, 9)))
    phi, P, u = W.droplet(cfg, 6.0, center=(35.3, 20.2, 12.4))
    phi[0:9, 10:30, 20:28] = 0.0
    P[0:9, 10:30, 20:28] = 0.0
    o = oracle.OracleCase(cfg)
    o.init_fields(phi, P, u)
    o.step(2)
    full = o.read_fields()
    # block face, top edge, corner, floor beside it, open top
    for c in [(28, 20, 4), (27, 29, 9), (19, 9, 9), (21, 12, 0), (40, 20, 43)]:
        ref, axes, pos = window_reference(cfg, (phi, P, u), c, 2)
        got, want = inner_block(full, ref, axes, pos, 2)
        for a, b in zip(got, want):
            assert np.abs(a - b).max() <= 1e-13 * max(np.abs(b).max(), 1e-300), c
