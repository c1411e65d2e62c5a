"""Total variation and its nonascending vector (oracle; test infrastructure only).

Section 3.1 defines, for an image [y] with l rows and c columns,

    TV(y) = sum_{i=1}^{l-1} sum_{j=1}^{c-1}
            sqrt(([y]_{i,j} - [y]_{i+1,j})^2 + ([y]_{i,j} - [y]_{i,j+1})^2),

and the nonascending vector t: t_bar is, componentwise, minus the partial
derivative of TV where that partial derivative is well defined and 0
otherwise; t = t_bar / ||t_bar|| if t_bar != 0, else the zero vector.

Reading A8: pixel (i, j) enters up to three square-root terms, T_{i,j},
T_{i-1,j} and T_{i,j-1} (T_{p,q} being the (p, q) summand above).  The partial
derivative with respect to [y]_{i,j} is well defined iff none of the terms it
enters has both differences exactly zero (a square root of zero is not
differentiable there); then it is the sum of

    (2 y_{i,j} - y_{i+1,j} - y_{i,j+1}) / T_{i,j}      if i < l,  j < c,
    (y_{i,j} - y_{i-1,j}) / T_{i-1,j}                  if i > 1,  j < c,
    (y_{i,j} - y_{i,j-1}) / T_{i,j-1}                  if i < l,  j > 1.
"""
from __future__ import annotations

import numpy as np


def total_variation(y) -> float:
    """TV(y) for an l x c image."""
    y = np.asarray(y, dtype=np.float64)
    dv = y[:-1, :-1] - y[1:, :-1]      # [y]_{i,j} - [y]_{i+1,j}
    dh = y[:-1, :-1] - y[:-1, 1:]      # [y]_{i,j} - [y]_{i,j+1}
    return float(np.sum(np.sqrt(dv * dv + dh * dh)))


def neg_gradient(y):
    """t_bar: minus the partial derivatives of TV, 0 where not well defined."""
    y = np.asarray(y, dtype=np.float64)
    l, c = y.shape
    dv = y[:-1, :-1] - y[1:, :-1]
    dh = y[:-1, :-1] - y[:-1, 1:]
    T = np.sqrt(dv * dv + dh * dh)             # T[p, q] for p < l-1, q < c-1 (0-based)
    zero = (dv == 0.0) & (dh == 0.0)           # non-differentiable summands
    grad = np.zeros((l, c))
    bad = np.zeros((l, c), dtype=bool)
    Ts = np.where(zero, 1.0, T)                # safe divisor; masked entries are discarded
    # term of T_{i,j}: pixel (i, j) itself, i < l-1, j < c-1
    grad[:-1, :-1] += (dv + dh) / Ts
    bad[:-1, :-1] |= zero
    # term of T_{i-1,j} at pixel (i, j): its vertical difference is y_{i-1,j} - y_{i,j}
    grad[1:, :-1] += -dv / Ts
    bad[1:, :-1] |= zero
    # term of T_{i,j-1} at pixel (i, j): its horizontal difference is y_{i,j-1} - y_{i,j}
    grad[:-1, 1:] += -dh / Ts
    bad[:-1, 1:] |= zero
    grad[bad] = 0.0
    return -grad


def nonascending(y):
    """(t, ||t_bar||): t = t_bar / ||t_bar|| or zeros."""
    tb = neg_gradient(y)
    nrm = float(np.sqrt(np.sum(tb * tb)))
    if nrm == 0.0:
        return np.zeros_like(tb), 0.0
    return tb / nrm, nrm
