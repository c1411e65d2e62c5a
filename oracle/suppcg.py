"""Algorithms 1-3 of the paper: S_TV, U_PCG and SupPCG (oracle; test
infrastructure only).

Written in the paper's order and notation: f(x) = ||Rx - b||^2, A = R^T R,
y = R^T b (Section 3.3).  Readings:

A9   Algorithm 1's repeat-loop is capped at ``max_trials`` trials per inner
     step; if none is accepted the inner step leaves y unchanged, keeps every
     increment of l, and is reported as exhausted.
A11  "N iterations" are N executions of the loop body (steps 11-14) with the
     termination test disabled (eps = 0 never stops a run with noisy data);
     after them k = N + 1 and the outputs are x_{N+1/2} (the paper's return
     value x_{k-1/2}) and x_{N+1}.
A13  if p^T h = 0 the step cannot be formed; the run stops and reports a
     breakdown (p = 0 means g is orthogonal to the range of M: solved).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import tv as tvmod


@dataclass
class TVParams:
    K: int
    a: float
    gamma: float
    max_trials: int = 100


@dataclass
class STVResult:
    s: np.ndarray            # y - x
    ell: int
    trials: list             # trials used by each inner step
    exhausted: bool
    tv_after: float          # TV(y) at return


def s_tv(x_img, ell: int, p: TVParams, replay=None) -> STVResult:
    """Algorithm 1, S_TV(x, l, a, gamma, K): returns (y - x, l).

    ``replay`` (optional list): trials to use in each inner step, taken from a
    previous run; the acceptance test is then not evaluated.
    """
    x_img = np.asarray(x_img, dtype=np.float64)
    y = x_img.copy()
    trials_used = []
    exhausted = False
    tv_y = tvmod.total_variation(y)
    for i in range(p.K):
        t, _ = tvmod.nonascending(y)
        tv_y = tvmod.total_variation(y)
        n_tr = 0
        accepted = False
        while True:
            g_tilde = p.gamma * p.a ** ell
            y_tilde = y + g_tilde * t
            ell += 1
            n_tr += 1
            if replay is not None:
                ok = n_tr == replay[i]          # replay[i] > max_trials: never accepted
            else:
                tv_new = tvmod.total_variation(y_tilde)
                ok = tv_new <= tv_y
            if ok:
                y = y_tilde
                tv_y = tvmod.total_variation(y) if replay is not None else tv_new
                accepted = True
                break
            if n_tr >= p.max_trials:
                break
        if not accepted:
            exhausted = True
        trials_used.append(n_tr if accepted else p.max_trials + 1)
    return STVResult(y - x_img, ell, trials_used, exhausted, tv_y)


class Problem:
    """The least-squares problem of eq. (2.1): R (sparse, m x n), b, image shape."""

    def __init__(self, R, b, shape, precond=None):
        self.R = R
        self.RT = R.T.tocsr()
        self.b = np.asarray(b, dtype=np.float64).ravel()
        self.shape = tuple(shape)
        self.y = self.RT @ self.b                       # y = R^T b
        # precond: callable on an image (l x c) -> image; None = identity (plain CG)
        self.M = precond if precond is not None else (lambda v: v)

    def A(self, v):
        return self.RT @ (self.R @ v)

    def f(self, x):
        r = self.R @ x - self.b
        return float(r @ r)

    def apply_M(self, g):
        return np.asarray(self.M(g.reshape(self.shape)), dtype=np.float64).ravel()


def u_pcg(prob: Problem, x, p, h, pth_prev):
    """Algorithm 2, U_PCG(x, p, h).  Returns (x, p, h, alpha, beta, p^T h, f(x_in))."""
    Rx = prob.R @ x
    f_in = float((Rx - prob.b) @ (Rx - prob.b))
    g = prob.RT @ Rx - prob.y            # g = A x - y
    z = prob.apply_M(g)                  # z = M g
    beta = float(z @ h) / pth_prev       # beta = z^T h / p^T h
    p = -z + beta * p
    h = prob.A(p)                        # h = A p
    pth = float(p @ h)
    if pth == 0.0:
        return x, p, h, None, beta, pth, f_in
    alpha = -float(g @ p) / pth          # alpha = -g^T p / p^T h
    x = x + alpha * p
    return x, p, h, alpha, beta, pth, f_in


@dataclass
class SupPCGResult:
    k: int
    x_half: np.ndarray          # x_{k-1/2}: the paper's output
    x_last: np.ndarray          # x_k
    status: str                 # "ok" | "converged" (f <= eps) | "breakdown"
    trace: dict = field(default_factory=dict)


def suppcg(prob: Problem, x0, tvp: TVParams | None, n_iter: int, eps: float = 0.0,
           replay=None, record_vectors: bool = False) -> SupPCGResult:
    """Algorithm 3, SupPCG(x0, a, gamma, K, eps); ``tvp=None`` or K = 0 is plain PCG.

    Runs at most ``n_iter`` loop bodies (A11).  The trace holds, per loop body
    k: f(x_{k+1/2}) (computed in U_PCG's first step), TV(x_{k+1/2}), l_{k+1},
    the trials of each inner step, alpha_k, beta_k and ||s_k||.  With
    ``record_vectors`` it also keeps x_k, x_{k+1/2}, p_k and h_k (tiny problems).
    """
    x0 = np.asarray(x0, dtype=np.float64).ravel()
    tr = {"f_half": [], "tv_half": [], "ell": [], "trials": [], "alpha": [], "beta": [],
          "s_norm": [], "exhausted": []}
    # steps 1-9
    x_half = x0.copy()
    Rx0 = prob.R @ x0
    f_cur = float((Rx0 - prob.b) @ (Rx0 - prob.b))       # f(x_{1/2})
    g = prob.RT @ Rx0 - prob.y
    z = prob.apply_M(g)
    p = -z
    h = prob.A(p)
    pth = float(p @ h)
    tr["f0"] = f_cur
    if pth == 0.0:
        return SupPCGResult(1, x_half, x0.copy(), "breakdown", tr)
    alpha = -float(g @ p) / pth
    x = x0 + alpha * p
    tr["alpha0"] = alpha
    if record_vectors:
        tr["x"] = [x.copy()]
        tr["x_half_v"] = [x_half.copy()]
        tr["p"] = [p.copy()]
        tr["h"] = [h.copy()]
    k = 1
    ell = 0
    status = "ok"
    done = 0
    while f_cur > eps and done < n_iter:                  # step 10
        if tvp is not None and tvp.K > 0:                 # step 11
            rep = None if replay is None else replay[done]
            st = s_tv(x.reshape(prob.shape), ell, tvp, rep)
            s = st.s.ravel()
            ell = st.ell
            tr["trials"].append(st.trials)
            tr["exhausted"].append(st.exhausted)
        else:
            s = np.zeros_like(x)
            tr["trials"].append([])
            tr["exhausted"].append(False)
        x_half = x + s                                    # step 12
        tr["s_norm"].append(float(np.sqrt(s @ s)))
        tr["tv_half"].append(tvmod.total_variation(x_half.reshape(prob.shape)))
        tr["ell"].append(ell)
        x_new, p, h, alpha, beta, pth_new, f_half = u_pcg(prob, x_half, p, h, pth)   # step 13
        tr["f_half"].append(f_half)
        tr["beta"].append(beta)
        tr["alpha"].append(alpha)
        k += 1                                            # step 14
        done += 1
        f_cur = f_half
        if alpha is None:
            x = x_new
            status = "breakdown"
            break
        x = x_new
        pth = pth_new
        if record_vectors:
            tr["x"].append(x.copy())
            tr["x_half_v"].append(x_half.copy())
            tr["p"].append(p.copy())
            tr["h"].append(h.copy())
    if status == "ok" and not f_cur > eps:
        status = "converged"
    return SupPCGResult(k, x_half, x, status, tr)
