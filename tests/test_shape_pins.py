"""Pins of the shape diagnostics (oracle/shape.py) on closed forms: the
perimeter, centroid and Taylor deformation of circles and ellipses drawn
with the interface profile of Eq. (7)."""
import math

import numpy as np
import pytest

import shape
from paper_2408_15654_amd import workloads as W


def ellipse_phi(n, a, b, cx, cy, theta, walls=False):
    y, x = np.mgrid[0:n, 0:n].astype(float)
    dx = x - cx
    dx -= n * np.round(dx / n)
    dy = y - cy
    if not walls:
        dy -= n * np.round(dy / n)
    u = dx * math.cos(theta) + dy * math.sin(theta)
    v = -dx * math.sin(theta) + dy * math.cos(theta)
    r = np.sqrt((u / a) ** 2 + (v / b) ** 2)
    # distance to the ellipse along the ray, to first order in (1 - r)
    d = (1 - r) * a * b * r / np.sqrt((b * u / a) ** 2 + (a * v / b) ** 2 + 1e-12)
    return W.tanh_profile(d, 4.0)


def test_circle():
    phi, _ = W.single_drop(128, 128, 30.0, W=4.0)
    s = shape.shape(phi, {})
    assert abs(s["length"] / (2 * math.pi * 30.0) - 1) < 5e-3
    assert s["taylor_D"] < 1e-10
    assert abs(s["cx"] - 64.0) < 1e-9 and abs(s["cy"] - 64.0) < 1e-9
    assert abs(s["Ixx"] - s["Iyy"]) < 1e-9 and abs(s["Ixy"]) < 1e-9


@pytest.mark.parametrize("theta_deg", [0.0, 30.0, -55.0])
def test_ellipse_across_the_periodic_corner(theta_deg):
    a, b = 40.0, 20.0
    th = math.radians(theta_deg)
    s = shape.shape(ellipse_phi(160, a, b, 2.0, 150.0, th), {})
    assert abs(s["cx"] - 2.0) < 1e-6 and abs(s["cy"] - 150.0) < 1e-6
    assert abs(s["angle"] - th) < 1e-3
    assert abs(s["taylor_D"] / ((a - b) / (a + b)) - 1) < 0.03
    ramanujan = math.pi * (3 * (a + b) - math.sqrt((3 * a + b) * (a + 3 * b)))
    assert abs(s["length"] / ramanujan - 1) < 0.02


def test_centroid_between_walls_is_the_plain_mean():
    """Off-centre drop in a channel: the plain mean of c along y (the tail of
    the profile over the larger part of the channel above the drop pulls it
    up by ~1e-4)."""
    phi = ellipse_phi(96, 12.0, 12.0, 48.0, 20.0, 0.0, walls=True)
    s = shape.shape(phi, {"walls_y": 1})
    assert abs(s["cy"] - 20.0) < 1e-3 and abs(s["cx"] - 48.0) < 1e-6
