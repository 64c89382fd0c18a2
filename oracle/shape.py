"""Shape diagnostics of one time level, in plain float64 numpy (TEST
INFRASTRUCTURE ONLY, like the rest of oracle/).

The paper follows a sheared drop through the length C of its interface
(Sec. 4.4) and, in the usual way for drops in shear, through the Taylor
deformation D = (L - B)/(L + B) of its half-axes L >= B.  Definitions used
here (the paper gives no formula for either):

  fluid-A fraction   c = (phi - phiB) / (phiA - phiB)
  area               A = sum c
  centroid           along a periodic direction the circular mean of the
                     site index weighted by c; along the wall direction the
                     plain mean
  second moments     I_ab = sum c d_a d_b / A with d the minimum-image
                     displacement from the centroid
  half-axes          L, B = 2 sqrt(eigenvalues of I) (a uniform ellipse of
                     half-axes a, b has eigenvalues a^2/4, b^2/4)
  orientation        angle of the eigenvector of the larger eigenvalue,
                     folded into (-pi/2, pi/2]
  interface length   C = sum |grad phi| / (phiA - phiB), grad phi from the
                     isotropic D2Q9 stencil (a flat tanh profile integrates
                     to exactly phiA - phiB across the interface)
"""
from __future__ import annotations

import math

import numpy as np

W9 = [(1, 0, 1 / 9), (0, 1, 1 / 9), (-1, 0, 1 / 9), (0, -1, 1 / 9),
      (1, 1, 1 / 36), (-1, 1, 1 / 36), (-1, -1, 1 / 36), (1, -1, 1 / 36)]


def _neighbour(a, dx, dy, walls):
    """a at (x + dx, y + dy): periodic in x; in y periodic or, between
    walls, the nearest row inside (mirror ghost)."""
    b = np.roll(a, -dx, axis=1)
    if not walls:
        return np.roll(b, -dy, axis=0)
    ny = a.shape[0]
    idx = np.clip(np.arange(ny) + dy, 0, ny - 1)
    return b[idx, :]


def grad(a, walls):
    gx = np.zeros_like(a)
    gy = np.zeros_like(a)
    for cx, cy, w in W9:
        v = _neighbour(a, cx, cy, walls)
        gx += w * cx * v
        gy += w * cy * v
    return 3.0 * gx, 3.0 * gy


def _circular_mean(idx, weight, n):
    ang = 2 * math.pi * idx / n
    z = (weight * np.exp(1j * ang)).sum()
    return (math.atan2(z.imag, z.real) * n / (2 * math.pi)) % n


def _min_image(d, n):
    return d - n * np.round(d / n)


def shape(phi: np.ndarray, params: dict) -> dict:
    phiA, phiB = float(params.get("phiA", 1.0)), float(params.get("phiB", 0.0))
    walls = bool(params.get("walls_y", 0))
    ny, nx = phi.shape
    c = (phi - phiB) / (phiA - phiB)
    area = float(c.sum())
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    cx = _circular_mean(x, c, nx)
    cy = float((c * y).sum() / area) if walls else _circular_mean(y, c, ny)
    dx = _min_image(x - cx, nx)
    dy = (y - cy) if walls else _min_image(y - cy, ny)
    ixx = float((c * dx * dx).sum() / area)
    ixy = float((c * dx * dy).sum() / area)
    iyy = float((c * dy * dy).sum() / area)
    tr, det = ixx + iyy, ixx * iyy - ixy * ixy
    disc = math.sqrt(max(tr * tr / 4 - det, 0.0))
    l1, l2 = tr / 2 + disc, max(tr / 2 - disc, 0.0)
    L, B = 2 * math.sqrt(l1), 2 * math.sqrt(l2)
    angle = 0.5 * math.atan2(2 * ixy, ixx - iyy)
    gx, gy = grad(phi, walls)
    length = float(np.hypot(gx, gy).sum() / (phiA - phiB))
    return {"area": area, "cx": cx, "cy": cy, "Ixx": ixx, "Ixy": ixy, "Iyy": iyy,
            "length": length, "taylor_D": (L - B) / (L + B), "angle": angle}
