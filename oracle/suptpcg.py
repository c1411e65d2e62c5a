"""Algorithms 4 and 5: transformed PCG and its superiorized form (oracle; test
infrastructure only; dense matrices, tiny grids).

Section 5: with M = N^T N (N invertible), one step of CG on N A N^T x_hat = N y
is U_TPCG (Algorithm 4), and SupTPCG (Algorithm 5) perturbs x_hat_k by
N^-T s_k with s_k from S_TV applied to N^T x_hat_k.  Table 2 states that
SupPCG(x0) and SupTPCG(N^-T x0) are equivalent through x_i = N^T x_hat_i,
p_k = N^T p_hat_k, h_hat_k = N h_k.  The tests use this as an invariant of the
SupPCG oracle.
"""
from __future__ import annotations

import numpy as np

from . import tv as tvmod
from .suppcg import TVParams, s_tv


def sqrt_spd(M):
    """Symmetric square root N of an SPD matrix, so that M = N^T N = N N."""
    lam, V = np.linalg.eigh(0.5 * (M + M.T))
    if lam.min() <= 0.0:
        raise ValueError("M is not positive definite")
    return (V * np.sqrt(lam)) @ V.T


def suptpcg(R, b, N, shape, xhat0, tvp: TVParams | None, n_iter: int, eps: float = 0.0):
    """Algorithm 5 with dense R (m x n) and N (n x n).  Returns per-iteration
    x_hat_{k}, x_hat_{k+1/2}, p_hat_k and l_k, plus the final k."""
    R = np.asarray(R, dtype=np.float64)
    A = R.T @ R
    y = R.T @ b
    NANt = N @ A @ N.T
    Ny = N @ y
    NinvT = np.linalg.inv(N.T)

    def f(xhat):
        r = R @ (N.T @ xhat) - b
        return float(r @ r)

    xhat_half = xhat0.copy()                        # step 1
    g = NANt @ xhat0 - Ny                           # step 2
    z = g                                           # step 3
    p = -z                                          # step 4
    h = NANt @ p                                    # step 5
    alpha = -float(g @ p) / float(p @ h)            # step 6
    xhat = xhat0 + alpha * p                        # step 7
    k, ell = 1, 0                                   # steps 8-9
    hist = {"x": [xhat.copy()], "x_half": [xhat_half.copy()], "p": [p.copy()], "ell": [ell]}
    done = 0
    while f(xhat_half) > eps and done < n_iter:     # step 10
        if tvp is not None and tvp.K > 0:
            st = s_tv((N.T @ xhat).reshape(shape), ell, tvp)        # step 11
            s, ell = st.s.ravel(), st.ell
        else:
            s = np.zeros_like(xhat)
        xhat_half = xhat + NinvT @ s                # step 12
        # step 13: Algorithm 4, U_TPCG(x_hat, p_hat, h_hat)
        g = NANt @ xhat_half - Ny
        z = g
        beta = float(z @ h) / float(p @ h)
        p = -z + beta * p
        h = NANt @ p
        alpha = -float(g @ p) / float(p @ h)
        xhat = xhat_half + alpha * p
        k += 1                                      # step 14
        done += 1
        hist["x"].append(xhat.copy())
        hist["x_half"].append(xhat_half.copy())
        hist["p"].append(p.copy())
        hist["ell"].append(ell)
    return k, hist


__all__ = ["sqrt_spd", "suptpcg", "tvmod"]
