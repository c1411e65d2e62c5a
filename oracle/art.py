"""ART and SupART of Section 3.4 (oracle; test infrastructure only).

ART here is the row-action method for the Bayesian criterion of eq. (2.3),
r^2 ||R x - b||^2 + ||x - mu||^2: with y = x - mu and an auxiliary vector u
(one entry per ray) the minimiser is the minimum-norm solution of the
consistent system  r R y + u = r (b - R mu), and one ART step projects the
current (y, u) toward the hyperplane of one ray, scaled by the relaxation
lambda:

    c   = lambda (r (b_i - <R_i, x>) - u_i) / (1 + r^2 ||R_i||^2)
    u_i = u_i + c
    x   = x + r c R_i^T

One iteration is a full cycle through the rays.  SupART perturbs x with
Algorithm 1 (S_TV) before each cycle (the superiorized step of Section 3.1,
with u as the auxiliary vector carried by the basic algorithm).  Readings:

R1  rays are visited angle by angle in increasing angle index, and within an
    angle in q phases: rays k = ph, ph + q, ph + 2q, ... for ph = 0 .. q-1,
    with q = floor(2 e / ds + 1e-9) + 1 (e = half-width of a pixel's footprint
    on the detector for that angle, ds = bin spacing), so rays of one phase touch
    disjoint pixels (the paper fixes no order); the ratio 2e/ds gets 1e-9
    added before the floor so that one that rounds to just below an integer
    keeps a margin;
R2  mu is the uniform image whose value is the mean gray level estimated
    from the data: for parallel beams each angle's data sums to the image
    integral divided by ds, so mu = ds * sum(b) / (A * n * pixel^2);
R3  x starts at mu and u at 0 (the start that makes the limit the minimiser);
R4  rays whose R_i is zero are skipped.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .geometry import Geometry, angle_cos_sin
from .suppcg import TVParams, s_tv


def phases(g: Geometry, a: int) -> int:
    """q of reading R1 for angle a."""
    _, c, s = angle_cos_sin(g, a)
    e = g.pixel * (abs(c) + abs(s)) / 2.0
    return int(math.floor(2.0 * e / g.bin_spacing + 1e-9)) + 1


def ray_order(g: Geometry):
    """Ray indices a * B + k in the order of reading R1."""
    out = []
    for a in range(g.n_angles):
        q = phases(g, a)
        for ph in range(q):
            out.extend(a * g.n_bins + k for k in range(ph, g.n_bins, q))
    return out


def mean_gray(g: Geometry, b) -> float:
    """mu of reading R2."""
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(g.bin_spacing * b.sum() / (g.n_angles * g.n * g.pixel ** 2))


@dataclass
class ARTResult:
    x: np.ndarray
    u: np.ndarray
    trace: dict = field(default_factory=dict)


def art_sweep(R, b, x, u, r: float, lam: float, order):
    """One ART cycle through the rays in `order`; x (n) and u (m) are updated in
    place and returned."""
    R = R.tocsr()
    b = np.asarray(b, dtype=np.float64).ravel()
    for i in order:
        lo, hi = R.indptr[i], R.indptr[i + 1]
        if lo == hi:
            continue
        cols = R.indices[lo:hi]
        w = R.data[lo:hi]
        nrm2 = float(w @ w)
        if nrm2 == 0.0:
            continue
        c = lam * (r * (b[i] - float(w @ x[cols])) - u[i]) / (1.0 + r * r * nrm2)
        u[i] += c
        x[cols] += (r * c) * w
    return x, u


def supart(g: Geometry, R, b, r: float, lam: float, n_iter: int, tvp: TVParams | None = None,
           x0=None, record: bool = False) -> ARTResult:
    """n_iter cycles of ART (tvp None or K = 0) or SupART from x0 (default mu)."""
    b = np.asarray(b, dtype=np.float64).ravel()
    mu = mean_gray(g, b)
    x = np.full(g.n, mu) if x0 is None else np.asarray(x0, dtype=np.float64).ravel().copy()
    u = np.zeros(g.m)
    order = ray_order(g)
    ell = 0
    tr = {"mu": mu, "ell": [], "x": []}
    for _ in range(n_iter):
        if tvp is not None and tvp.K > 0:
            st = s_tv(x.reshape(g.rows, g.cols), ell, tvp)
            x = x + st.s.ravel()
            ell = st.ell
            tr["ell"].append(ell)
        x, u = art_sweep(R, b, x, u, r, lam, order)
        if record:
            tr["x"].append(x.copy())
    return ARTResult(x, u, tr)


def bayes_minimiser(R, b, r: float, mu: float):
    """Dense minimiser of r^2 ||R x - b||^2 + ||x - mu||^2: (r^2 R^T R + I) x =
    r^2 R^T b + mu (tiny grids only)."""
    Rd = R.toarray() if hasattr(R, "toarray") else np.asarray(R)
    n = Rd.shape[1]
    lhs = r * r * (Rd.T @ Rd) + np.eye(n)
    rhs = r * r * (Rd.T @ np.asarray(b, dtype=np.float64).ravel()) + mu
    return np.linalg.solve(lhs, rhs)
