"""The paper's preconditioner M = F^-1 D F (oracle; test infrastructure only).

Section 3.2 uses M = F^-1 D F with F the discrete Fourier transform and D the
diagonal of a ramp filter combined with a generalised Hamming window,
h(w) = (|w| + mu) (rho + (1 - rho) cos w) for -pi <= w <= pi (eq. 3.2).

Readings (the paper gives the 1-D filter only):

A5  the image is zero-embedded in the top-left corner of a P x P array with
    P = 2^ceil(log2(2 max(l, c))) (so the product is a linear, not circular,
    convolution), transformed by the 2-D DFT, multiplied by
    D[u, v] = h(sqrt(w_u^2 + w_v^2)) with w_u = 2 pi u' / P, u' in [-P/2, P/2)
    (radial frequency, not clamped), inverse transformed and cropped back.
    M = E^T F^-1 D F E is symmetric; it is positive definite iff h > 0 on
    [0, pi sqrt 2], i.e. iff mu > 0 and rho > 1/2 (A6).
A7  scaling D by c > 0 leaves every PCG iterate unchanged.
"""
from __future__ import annotations

import math

import numpy as np


def pad_size(rows: int, cols: int) -> int:
    return 1 << int(math.ceil(math.log2(2 * max(rows, cols))))


def window(w, mu: float, rho: float):
    """h(w) = (|w| + mu) * (rho + (1 - rho) cos w), eq. (3.2)."""
    w = np.asarray(w, dtype=np.float64)
    return (np.abs(w) + mu) * (rho + (1.0 - rho) * np.cos(w))


def diagonal(P: int, mu: float, rho: float):
    """D[u, v] on the P x P DFT grid (numpy.fft ordering)."""
    wf = 2.0 * math.pi * np.fft.fftfreq(P)        # u' / P in [-1/2, 1/2), times 2 pi
    W = np.sqrt(wf[:, None] ** 2 + wf[None, :] ** 2)
    return window(W, mu, rho)


def apply(g_img, mu: float, rho: float, P: int | None = None):
    """z = E^T Re(F^-1 D F E g) for an l x c image g."""
    g_img = np.asarray(g_img, dtype=np.float64)
    rows, cols = g_img.shape
    if P is None:
        P = pad_size(rows, cols)
    E = np.zeros((P, P))
    E[:rows, :cols] = g_img
    Z = np.fft.ifft2(diagonal(P, mu, rho) * np.fft.fft2(E))
    return Z.real[:rows, :cols].copy()


def dense(rows: int, cols: int, mu: float, rho: float):
    """M as a dense n x n matrix (tiny grids only), column by column."""
    n = rows * cols
    out = np.zeros((n, n))
    for q in range(n):
        e = np.zeros(n)
        e[q] = 1.0
        out[:, q] = apply(e.reshape(rows, cols), mu, rho).ravel()
    return out
