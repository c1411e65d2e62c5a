"""Projection matrix entries as line-in-pixel intersection lengths, one ray at a
time, by merging the ray's crossings with the pixel grid (oracle; test
infrastructure only).

The paper's data model is Rx = b with R the m x n projection ("Radon") matrix
(Section 2); its experiment samples parallel rays at equally spaced angles
(Section 4.1).  Entry R[(a, k), (i, j)] is read as the length of ray (a, k)
inside pixel (i, j) (reading G5).  For a ray that is not parallel to an axis
the lengths come from the sorted parameters at which the ray crosses the
vertical and horizontal grid lines: each gap between consecutive crossings lies
in one pixel (found from the gap's midpoint) and contributes the gap's length.

A ray parallel to an axis that runs exactly along a grid line (shared edge or
outer border) gives each adjacent pixel half a pixel length per pixel crossed
(reading G6).
"""
from __future__ import annotations

import math

import numpy as np

from .geometry import Geometry, angle_cos_sin, bin_positions


def ray_weights(g: Geometry, a: int, k: int):
    """(pixel indices, lengths) of ray (a, k); pixel index = i * cols + j."""
    _, c, s = angle_cos_sin(g, a)
    sk = float(bin_positions(g)[k])
    d = g.pixel
    hw = g.cols * d / 2.0
    hh = g.rows * d / 2.0
    if s == 0.0 or c == 0.0:
        return _axis_ray(g, c, s, sk)
    # Points on the ray: P(tau) = sk * (c, s) + tau * (-s, c)  (unit speed).
    # Parameter interval inside the image rectangle [-hw, hw] x [-hh, hh].
    tx = sorted(((sk * c - hw) / s, (sk * c + hw) / s))
    ty = sorted(((-hh - sk * s) / c, (hh - sk * s) / c))
    lo, hi = max(tx[0], ty[0]), min(tx[1], ty[1])
    if not hi > lo:
        return np.zeros(0, dtype=np.int64), np.zeros(0)
    X = -hw + np.arange(g.cols + 1) * d          # vertical grid lines
    Y = -hh + np.arange(g.rows + 1) * d          # horizontal grid lines
    tau_x = (sk * c - X) / s
    tau_y = (Y - sk * s) / c
    taus = np.concatenate(([lo, hi], tau_x[(tau_x > lo) & (tau_x < hi)],
                           tau_y[(tau_y > lo) & (tau_y < hi)]))
    taus = np.unique(taus)
    lens = np.diff(taus)
    mids = 0.5 * (taus[:-1] + taus[1:])
    xm = sk * c - mids * s
    ym = sk * s + mids * c
    j = np.clip(np.floor((xm + hw) / d).astype(np.int64), 0, g.cols - 1)
    i = np.clip(np.floor((hh - ym) / d).astype(np.int64), 0, g.rows - 1)
    keep = lens > 0
    idx = i[keep] * g.cols + j[keep]
    # merge any repeated pixel (cannot happen for a straight line, kept for safety)
    uniq, inv = np.unique(idx, return_inverse=True)
    return uniq, np.bincount(inv, weights=lens[keep])


def _axis_ray(g: Geometry, c: float, s: float, sk: float):
    d = g.pixel
    if s == 0.0:
        # x * c = sk with c = +-1: a vertical line x = sk / c crossing every row.
        pos = sk / c
        centres = (np.arange(g.cols) - (g.cols - 1) / 2.0) * d
        dist = np.abs(centres - pos)
        w_col = np.where(dist < d / 2.0, d, np.where(dist == d / 2.0, d / 2.0, 0.0))
        cols = np.nonzero(w_col)[0]
        idx = (np.arange(g.rows)[:, None] * g.cols + cols[None, :]).ravel()
        w = np.broadcast_to(w_col[cols][None, :], (g.rows, cols.size)).ravel()
    else:
        # y * s = sk with s = +-1: a horizontal line y = sk / s crossing every column.
        pos = sk / s
        centres = ((g.rows - 1) / 2.0 - np.arange(g.rows)) * d
        dist = np.abs(centres - pos)
        w_row = np.where(dist < d / 2.0, d, np.where(dist == d / 2.0, d / 2.0, 0.0))
        rows = np.nonzero(w_row)[0]
        idx = (rows[:, None] * g.cols + np.arange(g.cols)[None, :]).ravel()
        w = np.broadcast_to(w_row[rows][:, None], (rows.size, g.cols)).ravel()
    order = np.argsort(idx)
    return idx[order].astype(np.int64), np.asarray(w, dtype=np.float64)[order]


def ray_sum(g: Geometry, x_flat, a: int, k: int) -> float:
    """(R x) for the single ray (a, k)."""
    idx, w = ray_weights(g, a, k)
    return float(np.dot(w, np.asarray(x_flat, dtype=np.float64)[idx]))


def chord_length_rectangle(g: Geometry, a: int, k: int) -> float:
    """Length of ray (a, k) inside the whole image rectangle, by clipping the
    line against the four sides (Liang-Barsky).  Independent of the grid; used
    to pin the all-ones image."""
    _, c, s = angle_cos_sin(g, a)
    sk = float(bin_positions(g)[k])
    hw = g.cols * g.pixel / 2.0
    hh = g.rows * g.pixel / 2.0
    # P(tau) = (sk c - tau s, sk s + tau c); constraints -hw <= x <= hw, -hh <= y <= hh.
    lo, hi = -math.inf, math.inf
    for p, q in ((-s, hw - sk * c), (s, hw + sk * c), (c, hh - sk * s), (-c, hh + sk * s)):
        # constraint written as p * tau <= q
        if p == 0.0:
            if q < 0.0:
                return 0.0
            continue
        t = q / p
        if p > 0.0:
            hi = min(hi, t)
        else:
            lo = max(lo, t)
    return max(0.0, hi - lo)
