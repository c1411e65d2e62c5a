"""Line-in-pixel intersection lengths from a closed form (oracle; test
infrastructure only).

For a square pixel of side p and a line at signed distance d from the pixel
centre, with direction normal (cos t, sin t), c = |cos t|, s = |sin t|, the
chord length is the projection of the square's indicator: the convolution of
two boxes of widths p*c and p*s divided by c*s, i.e. a trapezoid of area p^2
(reading G8):

    w(d) = min(p / max(c, s), max(0, (p (c + s) / 2 - |d|) / (c s)))    if c s > 0,
    w(d) = p if |d| < p/2,  p/2 if |d| = p/2,  0 otherwise              if c s = 0.

The axis case follows reading G6 (a line on a shared edge gives each pixel half).
This is a second, independent definition of R: the tests pin it to the
per-ray crossing merge in ``siddon``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .geometry import Geometry, angle_cos_sin, bin_positions, pixel_centres


def chord_weight(d, c: float, s: float, pixel: float):
    """Chord length through a pixel for offsets d (array) at |cos|=c, |sin|=s."""
    d = np.abs(np.asarray(d, dtype=np.float64))
    c, s = abs(c), abs(s)
    if c * s > 0.0:
        return np.minimum(pixel / max(c, s), np.maximum(0.0, (pixel * (c + s) / 2.0 - d) / (c * s)))
    half = pixel / 2.0
    return np.where(d < half, pixel, np.where(d == half, half, 0.0))


def angle_block(g: Geometry, a: int):
    """Sparse (B x n) block of R for angle a, built pixel by pixel."""
    _, c, s = angle_cos_sin(g, a)
    xs, ys = pixel_centres(g)
    X, Y = np.meshgrid(xs, ys)                       # [rows, cols]
    t = (X * c + Y * s).ravel()                       # projection of each pixel centre
    e = g.pixel * (abs(c) + abs(s)) / 2.0             # half-width of the trapezoid
    ds = g.bin_spacing
    s0 = float(bin_positions(g)[0])
    kbase = np.floor((t - e - s0) / ds).astype(np.int64)
    q_count = int(np.floor(2.0 * e / ds)) + 3
    rows, cols, vals = [], [], []
    pix = np.arange(g.n, dtype=np.int64)
    sk_all = bin_positions(g)
    for q in range(q_count):
        k = kbase + q
        ok = (k >= 0) & (k < g.n_bins)
        kk = k[ok]
        w = chord_weight(sk_all[kk] - t[ok], c, s, g.pixel)
        nz = w > 0.0
        rows.append(kk[nz])
        cols.append(pix[ok][nz])
        vals.append(w[nz])
    r = np.concatenate(rows)
    cc = np.concatenate(cols)
    v = np.concatenate(vals)
    return sp.csr_matrix((v, (r, cc)), shape=(g.n_bins, g.n))


def system_matrix(g: Geometry):
    """R (m x n, CSR) from the closed form, angle block by angle block."""
    blocks = [angle_block(g, a) for a in range(g.n_angles)]
    return sp.vstack(blocks, format="csr")


def column(g: Geometry, i: int, j: int):
    """(ray indices, weights) of column (i, j) of R: every ray through pixel (i, j)."""
    xs, ys = pixel_centres(g)
    sk_all = bin_positions(g)
    out_r, out_w = [], []
    for a in range(g.n_angles):
        _, c, s = angle_cos_sin(g, a)
        w = chord_weight(sk_all - (xs[j] * c + ys[i] * s), c, s, g.pixel)
        nz = np.nonzero(w > 0.0)[0]
        out_r.append(a * g.n_bins + nz)
        out_w.append(w[nz])
    return np.concatenate(out_r), np.concatenate(out_w)
