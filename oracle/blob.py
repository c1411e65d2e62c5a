"""BlobART of Section 3.4: ART with blob basis functions (oracle; test
infrastructure only).

The image is x(r) = sum_j c_j b(|r - r_j|) with generalised Kaiser-Bessel
blobs b centred on the pixel centres r_j; the data of ray i is the line
integral of x, so the system matrix entry (i, j) is the blob's projection
p(d) at the distance d of centre r_j from ray i; ART (oracle/art.py) then
runs on the coefficients c.  The paper fixes none of the blob's parameters;
readings:

B1  blob b(r) = w^m I_m(alpha w) / I_m(alpha), w = sqrt(1 - (r/a)^2) for
    r < a, 0 beyond; m = 2, alpha = 10.4, radius a = 2 pixels (the values
    usually taken for this basis); centres on the pixel grid;
B2  its projection is p(d) = (a / I_m(alpha)) sqrt(2 pi / alpha)
    w^(m + 1/2) I_(m + 1/2)(alpha w), w = sqrt(1 - (d/a)^2), for |d| < a
    (the line integral of b written out; pinned against quadrature);
B3  the Bayesian criterion of eq. (2.3) acts on c, with mu the uniform
    coefficient vector whose image is the mean gray level of reading R2:
    c_mu = mu / S, S = sum over grid offsets o of b(|o|) (the image of a
    constant coefficient field away from the border);
B4  rays of one angle are visited in phases q = floor(2 a / ds + 1e-9) + 1
    apart (rays farther apart than the blob's diameter meet disjoint blobs);
B5  the reconstructed image is x sampled at the pixel centres.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sps
from scipy.special import iv

from .geometry import Geometry, angle_cos_sin, bin_positions, pixel_centres

M_ORDER = 2
ALPHA = 10.4
RADIUS = 2.0


def blob(r, a=RADIUS, alpha=ALPHA, m=M_ORDER):
    """b(r) of reading B1 (r in pixel units)."""
    r = np.asarray(r, dtype=np.float64)
    t = 1.0 - (r / a) ** 2
    w = np.sqrt(np.clip(t, 0.0, None))
    val = w ** m * iv(m, alpha * w) / iv(m, alpha)
    return np.where(t > 0.0, val, 0.0)


def blob_projection(d, a=RADIUS, alpha=ALPHA, m=M_ORDER):
    """p(d) of reading B2: the integral of b along a line at distance d."""
    d = np.asarray(d, dtype=np.float64)
    t = 1.0 - (d / a) ** 2
    w = np.sqrt(np.clip(t, 0.0, None))
    val = (a / iv(m, alpha)) * math.sqrt(2.0 * math.pi / alpha) * w ** (m + 0.5) * iv(m + 0.5, alpha * w)
    return np.where(t > 0.0, val, 0.0)


def grid_sum(a=RADIUS):
    """S of reading B3: sum of b over the integer offsets within the radius."""
    k = int(math.ceil(a))
    o = np.arange(-k, k + 1)
    X, Y = np.meshgrid(o, o)
    return float(blob(np.hypot(X, Y), a).sum())


def system_matrix(g: Geometry, a=RADIUS):
    """R_blob (m x n, CSR): entry (ray, blob) = p(distance in pixel units) *
    pixel (lengths in the geometry's unit)."""
    xs, ys = pixel_centres(g)
    X, Y = np.meshgrid(xs, ys)
    sk = bin_positions(g)
    rows, cols, vals = [], [], []
    pix = np.arange(g.n)
    for ai in range(g.n_angles):
        _, c, s = angle_cos_sin(g, ai)
        t = (X * c + Y * s).ravel()
        for k in range(g.n_bins):
            d = (sk[k] - t) / g.pixel
            sel = np.abs(d) < a
            v = blob_projection(d[sel], a) * g.pixel
            nz = v > 0.0
            rows.append(np.full(int(nz.sum()), ai * g.n_bins + k))
            cols.append(pix[sel][nz])
            vals.append(v[nz])
    return sps.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(g.m, g.n))


def synthesize(g: Geometry, c, a=RADIUS):
    """x at the pixel centres from the coefficients c (reading B5)."""
    c = np.asarray(c, dtype=np.float64).reshape(g.rows, g.cols)
    k = int(math.ceil(a))
    out = np.zeros_like(c)
    for di in range(-k, k + 1):
        for dj in range(-k, k + 1):
            wgt = float(blob(math.hypot(di, dj), a))
            if wgt == 0.0:
                continue
            # out[i, j] += wgt * c[i + di, j + dj] where inside
            src = c[max(di, 0):g.rows + min(di, 0), max(dj, 0):g.cols + min(dj, 0)]
            out[max(-di, 0):g.rows + min(-di, 0), max(-dj, 0):g.cols + min(-dj, 0)] += wgt * src
    return out


def phases(g: Geometry, a=RADIUS) -> int:
    """q of reading B4 (the same for every angle)."""
    return int(math.floor(2.0 * a * g.pixel / g.bin_spacing + 1e-9)) + 1


def ray_order(g: Geometry, a=RADIUS):
    q = phases(g, a)
    out = []
    for ai in range(g.n_angles):
        for ph in range(q):
            out.extend(ai * g.n_bins + k for k in range(ph, g.n_bins, q))
    return out


def blob_art(g: Geometry, Rb, b, r: float, lam: float, n_iter: int, record: bool = False):
    """n_iter cycles of BlobART; returns (coefficients, image, trace)."""
    from .art import art_sweep, mean_gray
    b = np.asarray(b, dtype=np.float64).ravel()
    mu = mean_gray(g, b)
    c = np.full(g.n, mu / grid_sum())
    u = np.zeros(g.m)
    order = ray_order(g)
    tr = {"mu": mu, "c_mu": mu / grid_sum(), "images": []}
    for _ in range(n_iter):
        c, u = art_sweep(Rb, b, c, u, r, lam, order)
        if record:
            tr["images"].append(synthesize(g, c).ravel())
    return c, synthesize(g, c).ravel(), tr
