"""Learned SPD preconditioner M = C^T diag(softplus(d)) C (oracle; test
infrastructure only; float64).

Not in the paper: the paper's preconditioner is the Fourier ramp-Hamming
filter of Section 3.2; this is a learned alternative used in the same place in
Algorithm 2 (step 2, z = M g).  Reading A18:

* C is a stack of L linear 3x3 convolutions without bias (cross-correlation
  with zero "same" padding): 1 -> F channels, then F -> F channels.
* d has one entry per channel of the last layer; softplus(d) > 0.
* C^T is the exact adjoint of C: each layer's adjoint is the correlation with
  the spatially flipped kernel and swapped channel roles, applied in reverse
  layer order.  M is symmetric positive semi-definite by construction.
* Training loss over probe pairs (v, A v): mean over the batch of
  ||M(A v) - v||^2 / ||v||^2, gradient by hand-written backpropagation, Adam.

Weights are stored as W[l] of shape (F_out, F_in, 3, 3); tap (ky, kx) reads
the input at offset (ky - 1, kx - 1).

Parity of trained weights against a GPU training run is unpinned (training in
float32 is not bit-reproducible against float64); the pieces (C, C^T, M, the
loss gradient, one Adam step) are pinned by the tests.
"""
from __future__ import annotations

import math

import numpy as np


def softplus(d):
    d = np.asarray(d, dtype=np.float64)
    return np.where(d > 20.0, d, np.log1p(np.exp(np.minimum(d, 20.0))))


def sigmoid(d):
    return 1.0 / (1.0 + np.exp(-np.asarray(d, dtype=np.float64)))


def shift(x, dy, dx):
    """s[..., i, j] = x[..., i + dy, j + dx], zero outside."""
    out = np.zeros_like(x)
    H, W = x.shape[-2:]
    ys, ye = max(0, -dy), min(H, H - dy)
    xs, xe = max(0, -dx), min(W, W - dx)
    if ys < ye and xs < xe:
        out[..., ys:ye, xs:xe] = x[..., ys + dy:ye + dy, xs + dx:xe + dx]
    return out


def conv(x, W):
    """Cross-correlation with zero padding.  x: (B, Fi, H, W); W: (Fo, Fi, 3, 3)."""
    B, Fi, H, Wd = x.shape
    Fo = W.shape[0]
    y = np.zeros((B, Fo, H, Wd))
    for ky in range(3):
        for kx in range(3):
            xs = shift(x, ky - 1, kx - 1)                       # (B, Fi, H, W)
            y += np.einsum("oi,bihw->bohw", W[:, :, ky, kx], xs)
    return y


def conv_t(y, W):
    """Adjoint of conv: (B, Fo, H, W) -> (B, Fi, H, W)."""
    B, Fo, H, Wd = y.shape
    Fi = W.shape[1]
    x = np.zeros((B, Fi, H, Wd))
    for ky in range(3):
        for kx in range(3):
            ys = shift(y, -(ky - 1), -(kx - 1))
            x += np.einsum("oi,bohw->bihw", W[:, :, ky, kx], ys)
    return x


def wgrad(G, X):
    """d<G, conv(X, W)>/dW: (B, Fo, H, W), (B, Fi, H, W) -> (Fo, Fi, 3, 3)."""
    out = np.zeros((G.shape[1], X.shape[1], 3, 3))
    for ky in range(3):
        for kx in range(3):
            out[:, :, ky, kx] = np.einsum("bohw,bihw->oi", G, shift(X, ky - 1, kx - 1))
    return out


def wgrad_t(H, Y):
    """d<H, conv_t(Y, W)>/dW: (B, Fi, H, W), (B, Fo, H, W) -> (Fo, Fi, 3, 3)."""
    out = np.zeros((Y.shape[1], H.shape[1], 3, 3))
    for ky in range(3):
        for kx in range(3):
            out[:, :, ky, kx] = np.einsum("bihw,bohw->oi", H, shift(Y, -(ky - 1), -(kx - 1)))
    return out


def init_params(layers=4, channels=16, seed=0):
    """He-normal weights, d = softplus^-1(1)."""
    rng = np.random.default_rng(seed)
    Ws = []
    fin = 1
    for _ in range(layers):
        std = math.sqrt(2.0 / (9 * fin))
        Ws.append(rng.standard_normal((channels, fin, 3, 3)) * std)
        fin = channels
    d = np.full(channels, math.log(math.e - 1.0))
    return Ws, d


def apply(Ws, d, u):
    """M u for u of shape (B, H, W) or (H, W)."""
    u = np.asarray(u, dtype=np.float64)
    single = u.ndim == 2
    a = u[None, None] if single else u[:, None]
    for W in Ws:
        a = conv(a, W)
    b = a * softplus(d)[None, :, None, None]
    for W in reversed(Ws):
        b = conv_t(b, W)
    return b[0, 0] if single else b[:, 0]


def interior(shape, margin: int):
    """1 on pixels at least `margin` away from every image edge, else 0."""
    H, W = shape[-2], shape[-1]
    m = np.zeros((H, W))
    m[margin:H - margin, margin:W - margin] = 1.0
    return m


def loss_and_grad(Ws, d, Av, v, margin: int = 0):
    """Loss mean_b ||P (M(Av_b) - v_b)||^2 / ||P v_b||^2 and its gradient, with
    P the restriction to the interior pixels (margin 0: the whole image).

    Returns (loss, [dL/dW_l], dL/dd)."""
    Av = np.asarray(Av, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    B = Av.shape[0]
    P = interior(v.shape, margin)
    sig = softplus(d)
    acts = [Av[:, None]]                       # a_0 .. a_L (forward chain)
    for W in Ws:
        acts.append(conv(acts[-1], W))
    back = [acts[-1] * sig[None, :, None, None]]   # b_L = D a_L, then b_{l-1} = conv_t(b_l, W_l)
    for W in reversed(Ws):
        back.append(conv_t(back[-1], W))
    back = back[::-1]                          # back[l] = b_l, l = 0..L
    z = back[0][:, 0]
    nv = np.sum((P * v) ** 2, axis=(1, 2))
    r = P * (z - v)
    loss = float(np.mean(np.sum(r * r, axis=(1, 2)) / nv))
    L = len(Ws)
    gW = [np.zeros_like(W) for W in Ws]
    # dloss/dz
    e = (2.0 / B) * (r / nv[:, None, None])[:, None]
    # back through the adjoint chain: b_{l-1} = conv_t(b_l, W_l)
    for l in range(1, L + 1):
        W = Ws[l - 1]
        gW[l - 1] += wgrad_t(e, back[l])
        e = conv(e, W)
    # e = dloss/db_L ; b_L = sig * a_L
    gd = np.sum(e * acts[L], axis=(0, 2, 3)) * sigmoid(d)
    f = e * sig[None, :, None, None]
    for l in range(L, 0, -1):
        W = Ws[l - 1]
        gW[l - 1] += wgrad(f, acts[l - 1])
        f = conv_t(f, W)
    return loss, gW, gd


class Adam:
    """Adam (beta1, beta2, eps) on a list of arrays."""

    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [np.zeros_like(p) for p in params]
        self.v = [np.zeros_like(p) for p in params]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        out = []
        for i, (p, g) in enumerate(zip(params, grads)):
            self.m[i] = self.b1 * self.m[i] + (1 - self.b1) * g
            self.v[i] = self.b2 * self.v[i] + (1 - self.b2) * g * g
            mh = self.m[i] / (1 - self.b1 ** self.t)
            vh = self.v[i] / (1 - self.b2 ** self.t)
            out.append(p - self.lr * mh / (np.sqrt(vh) + self.eps))
        return out


def flatten(Ws, d):
    return np.concatenate([W.ravel() for W in Ws] + [np.asarray(d).ravel()])


def unflatten(theta, layers=4, channels=16):
    Ws = []
    o = 0
    fin = 1
    for _ in range(layers):
        sz = channels * fin * 9
        Ws.append(theta[o:o + sz].reshape(channels, fin, 3, 3))
        o += sz
        fin = channels
    return Ws, theta[o:o + channels]
