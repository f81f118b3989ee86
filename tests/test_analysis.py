"""Bubble diagnostics (centroid, rise velocity, circularity) against closed
forms: straight-line chords, the circle's 2 pi R, Ramanujan's ellipse
perimeter (accurate to ~1e-10 relative at this aspect ratio), exact centroids
and uniform velocities."""
import math

import numpy as np
import pytest

from paper_2512_01027_amd import analysis as A
from paper_2512_01027_amd import workloads as W


@pytest.mark.parametrize("th", [0.0, 0.3, 1.2, 2.5])
def test_contour_of_a_line_is_its_chord(th):
    y, x = np.mgrid[0:50, 0:50].astype(float)
    f = (x - 24.5) * math.cos(th) + (y - 24.5) * math.sin(th)
    c, s = abs(math.cos(th)), abs(math.sin(th))
    assert A._contour_length(f, 0.0) == pytest.approx(49.0 / max(c, s), rel=1e-12)


def test_contour_through_nodes_is_kept():
    """A line of slope -1 through nodes: every cell on it contributes."""
    y, x = np.mgrid[0:50, 0:50].astype(float)
    assert A._contour_length(x + y - 50.0, 0.0) == pytest.approx(48 * math.sqrt(2.0), rel=1e-12)


@pytest.mark.parametrize("R", [20.0, 50.0])
def test_circle(R):
    cfg = W.base_case(2, 200, 400)
    phi, _, _ = W.droplet(cfg, R, center=(100.3, 150.7, 0.0), heavy_inside=False)
    assert A._contour_length(phi[0]) == pytest.approx(2 * math.pi * R, rel=2e-3 if R < 30 else 1e-4)
    assert A.circularity(phi[0]) == pytest.approx(1.0, abs=5e-3)
    cx, cy = A.centroid(phi[0])
    assert cx == pytest.approx(100.3, abs=1e-6) and cy == pytest.approx(150.7, abs=1e-6)


def test_ellipse_perimeter_and_circularity():
    y, x = np.mgrid[0:400, 0:200].astype(float)
    a, b = 60.0, 30.0
    r = np.sqrt(((x - 100) / a) ** 2 + ((y - 200) / b) ** 2)
    phi = 0.5 + 0.5 * np.tanh(2 * (r - 1) * min(a, b) / 4)
    h = ((a - b) / (a + b)) ** 2
    per = math.pi * (a + b) * (1 + 3 * h / (10 + math.sqrt(4 - 3 * h)))
    assert A._contour_length(phi) == pytest.approx(per, rel=2e-4)
    # circle of the same area over the perimeter; the indicator area of the
    # diffuse profile is pi a b to about the interface width's curvature term
    assert A.circularity(phi) == pytest.approx(2 * math.pi * math.sqrt(a * b) / per, rel=5e-3)


def test_rise_velocity_of_uniform_flow():
    cfg = W.base_case(2, 64, 80)
    phi, _, u = W.droplet(cfg, 10.0, heavy_inside=False, u0=(0.01, -0.02))
    assert A.rise_velocity(phi[0], u[:, 0]) == pytest.approx((0.01, -0.02), rel=1e-12)
