"""R and R^T as explicit sparse matrices (oracle; test infrastructure only).

The paper poses reconstruction as least squares, min ||R y - b||^2 (eq. 2.1),
solved through the normal equations R^T R x = R^T b (eq. 2.2).  Here R is
assembled as a CSR matrix and R^T is its exact transpose, so the adjoint is
exact by construction.

Two assemblies exist: ``"siddon"`` (ray by ray crossing merge, the primary
definition, for small images) and ``"closed"`` (closed-form chord lengths, any
size).  The tests pin one against the other.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import closed_form, siddon
from .geometry import Geometry

_CACHE: dict = {}


def siddon_matrix(g: Geometry):
    """R (m x n, CSR) assembled ray by ray from ``siddon.ray_weights``."""
    indptr = [0]
    indices, data = [], []
    for a in range(g.n_angles):
        for k in range(g.n_bins):
            idx, w = siddon.ray_weights(g, a, k)
            indices.append(idx)
            data.append(w)
            indptr.append(indptr[-1] + idx.size)
    return sp.csr_matrix((np.concatenate(data), np.concatenate(indices).astype(np.int64),
                          np.asarray(indptr, dtype=np.int64)), shape=(g.m, g.n))


def matrix(g: Geometry, method: str | None = None):
    """Cached R for geometry g.  Default method: Siddon up to 128x128, else closed form."""
    if method is None:
        method = "siddon" if g.n <= 128 * 128 and g.m <= 200_000 else "closed"
    key = (g, method)
    if key not in _CACHE:
        if method == "siddon":
            R = siddon_matrix(g)
        elif method == "closed":
            R = closed_form.system_matrix(g)
        else:
            raise ValueError(method)
        R.sum_duplicates()
        R.sort_indices()
        _CACHE[key] = (R, R.T.tocsr())
    return _CACHE[key]


def project(g: Geometry, x, method: str | None = None):
    """R x for an image x (any shape with n entries, row-major); returns [A*B]."""
    R, _ = matrix(g, method)
    return R @ np.asarray(x, dtype=np.float64).ravel()


def backproject(g: Geometry, y, method: str | None = None):
    """R^T y for data y (any shape with m entries, angle-major); returns [n]."""
    _, RT = matrix(g, method)
    return RT @ np.asarray(y, dtype=np.float64).ravel()


def clear_cache():
    _CACHE.clear()
