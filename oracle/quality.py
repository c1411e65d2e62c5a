"""The selective error of Section 4.2, eq. (4.1) (oracle; test infrastructure only).

SE(x) = C * sqrt( sum over (i, j) in S of ([x]_ij - [x_ref]_ij)^2 ), where S is
the set of pixels inside a centred ellipse and x_ref is the phantom.  The paper
places the ellipse just inside the skull of its 243 x 243 phantom, with a 5 cm
horizontal and a 7 cm vertical semi-axis on 0.0752 cm pixels.  Readings fixed
here:

Q1  pixel (i, j) belongs to S when its centre (reading G1) lies in the closed
    ellipse: (x_j / a_h)^2 + (y_i / a_v)^2 <= 1, with a_h the horizontal (along a
    row, i.e. across columns) and a_v the vertical semi-axis, in the
    geometry's length unit;
Q2  the paper leaves C as a constant depending on the phantom; C <= 0 selects
    C = 1 / sqrt(sum over S of [x_ref]_ij^2), so SE(0) = 1 and SE is the
    relative error inside S;
Q3  on images other than the paper's, the ellipse keeps its size relative to
    the image width: a_h = 5 / (243 * 0.0752) * width, a_v = 7 / (243 * 0.0752)
    * width, width = cols * pixel.
"""
from __future__ import annotations

import numpy as np

from .geometry import Geometry

# The paper's phantom: 243 pixels of 0.0752 cm; ellipse semi-axes 5 cm, 7 cm.
PAPER_WIDTH_CM = 243 * 0.0752
PAPER_AXES_CM = (5.0, 7.0)


def paper_axes(g: Geometry):
    """(a_h, a_v) of reading Q3 for geometry g."""
    w = g.cols * g.pixel
    return (PAPER_AXES_CM[0] / PAPER_WIDTH_CM * w, PAPER_AXES_CM[1] / PAPER_WIDTH_CM * w)


def ellipse_mask(g: Geometry, axes) -> np.ndarray:
    """Boolean [rows, cols]: the set S of reading Q1."""
    ah, av = float(axes[0]), float(axes[1])
    mask = np.zeros((g.rows, g.cols), dtype=bool)
    for i in range(g.rows):
        y = ((g.rows - 1) / 2.0 - i) * g.pixel
        for j in range(g.cols):
            x = (j - (g.cols - 1) / 2.0) * g.pixel
            mask[i, j] = (x / ah) ** 2 + (y / av) ** 2 <= 1.0
    return mask


def selective_error(g: Geometry, x, x_ref, axes, C: float = 0.0) -> float:
    """SE(x) of eq. (4.1) with S from reading Q1 and C from reading Q2."""
    mask = ellipse_mask(g, axes)
    x = np.asarray(x, dtype=np.float64).reshape(g.rows, g.cols)
    ref = np.asarray(x_ref, dtype=np.float64).reshape(g.rows, g.cols)
    if C <= 0.0:
        C = 1.0 / np.sqrt(np.sum(ref[mask] ** 2))
    d = (x - ref)[mask]
    return float(C * np.sqrt(np.sum(d * d)))


def se_curve(g: Geometry, prob, x0, tvp, n_iter: int, x_ref, axes, C: float = 0.0):
    """SE of every iterate of Algorithm 3: [SE(x_0), SE(x_1), ..., SE(x_{N+1})]
    for N = n_iter loop bodies (fewer if the run stops), with prob and tvp as
    for ``suppcg.suppcg`` (tvp None or K = 0: PCG; an identity preconditioner
    in prob: CG and SupCG)."""
    from .suppcg import suppcg
    res = suppcg(prob, x0, tvp, n_iter, record_vectors=True)
    its = [np.asarray(x0, dtype=np.float64).ravel()] + list(res.trace["x"])
    return [selective_error(g, v, x_ref, axes, C) for v in its], res
