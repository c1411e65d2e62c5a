"""Parallel-beam geometry (oracle; test infrastructure only).

The paper's experiment (Section 4.1) uses equally spaced angles in [0, pi) and,
per angle, parallel rays at a fixed spacing; the image is an l x c array of
square pixels whose (i, j) entry is vector component c(i-1)+j (Section 3.1).
Readings fixed here:

G1  pixel (i, j), 0-based, has centre x_j = (j - (c-1)/2) d, y_i = ((l-1)/2 - i) d
    (image centred at the origin, row 0 at the top, d = pixel size);
G2  theta_a = theta0 + a * dtheta (default theta0 = 0, dtheta = pi / A);
G3  ray (a, k) is the line x cos(theta_a) + y sin(theta_a) = s_k with
    s_k = (k - (B-1)/2) ds + offset;
G4  the data vector is angle-major: component a*B + k;
G7  cos/sin are exact at multiples of pi/4 (0, +-1, +-sqrt(2)/2), libm otherwise.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Geometry:
    rows: int
    cols: int
    n_angles: int
    n_bins: int
    pixel: float = 1.0
    theta0: float = 0.0
    dtheta: float | None = None          # None -> pi / n_angles
    bin_spacing: float = 1.0
    bin_offset: float = 0.0

    @property
    def n(self) -> int:
        return self.rows * self.cols

    @property
    def m(self) -> int:
        return self.n_angles * self.n_bins

    @property
    def step(self) -> float:
        return math.pi / self.n_angles if self.dtheta is None else self.dtheta


_SQRT_HALF = math.sqrt(0.5)
# (cos, sin) of m * pi / 4 for m = 0..7, exact.
_OCTANT = [(1.0, 0.0), (_SQRT_HALF, _SQRT_HALF), (0.0, 1.0), (-_SQRT_HALF, _SQRT_HALF),
           (-1.0, 0.0), (-_SQRT_HALF, -_SQRT_HALF), (0.0, -1.0), (_SQRT_HALF, -_SQRT_HALF)]


def angle_cos_sin(g: Geometry, a: int):
    """(theta, cos, sin) of angle index a, snapped at multiples of pi/4 (G7)."""
    theta = g.theta0 + a * g.step
    q = theta / (math.pi / 4.0)
    m = round(q)
    if abs(q - m) < 1e-12:
        c, s = _OCTANT[m % 8]
    else:
        c, s = math.cos(theta), math.sin(theta)
    return theta, c, s


def angle_table(g: Geometry):
    """Arrays (theta[A], cos[A], sin[A]) in float64."""
    rows = [angle_cos_sin(g, a) for a in range(g.n_angles)]
    t = np.array([r[0] for r in rows])
    c = np.array([r[1] for r in rows])
    s = np.array([r[2] for r in rows])
    return t, c, s


def pixel_centres(g: Geometry):
    """(x[cols], y[rows]) pixel-centre coordinates (G1)."""
    x = (np.arange(g.cols, dtype=np.float64) - (g.cols - 1) / 2.0) * g.pixel
    y = ((g.rows - 1) / 2.0 - np.arange(g.rows, dtype=np.float64)) * g.pixel
    return x, y


def bin_positions(g: Geometry):
    """s[B]: signed distance of each ray from the origin (G3)."""
    return (np.arange(g.n_bins, dtype=np.float64) - (g.n_bins - 1) / 2.0) * g.bin_spacing + g.bin_offset
