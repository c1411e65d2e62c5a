"""Pins of the oracle's total variation, nonascending vector and preconditioner
(CPU only)."""
import math

import numpy as np
import pytest

from oracle import precond, tv


# ---- total variation (Section 3.1) -------------------------------------------------

def test_tv_hand_built_images():
    # P11
    assert tv.total_variation(np.full((7, 9), 3.25)) == 0.0
    step = np.zeros((7, 9))
    step[:, 5:] = 1.0                         # vertical edge between columns 4 and 5
    assert tv.total_variation(step) == pytest.approx(6.0, abs=1e-14)   # l - 1 terms
    spike = np.zeros((7, 9))
    spike[3, 4] = 2.5
    assert tv.total_variation(spike) == pytest.approx(2.5 * (2 + math.sqrt(2)), abs=1e-13)
    rng = np.random.default_rng(0)
    y = rng.standard_normal((10, 8))
    assert tv.total_variation(-3.0 * y + 7.0) == pytest.approx(3.0 * tv.total_variation(y), rel=1e-13)


def test_tv_brute_force_loop():
    rng = np.random.default_rng(1)
    y = rng.standard_normal((5, 6))
    want = 0.0
    for i in range(4):
        for j in range(5):
            want += math.sqrt((y[i, j] - y[i + 1, j]) ** 2 + (y[i, j] - y[i, j + 1]) ** 2)
    assert tv.total_variation(y) == pytest.approx(want, rel=1e-14)


def test_neg_gradient_spike_and_zero_rule():
    # P12: spike pixel gets -(2 + sqrt 2); pixels touching a flat term get 0
    spike = np.zeros((7, 9))
    spike[3, 4] = 1.0
    tb = tv.neg_gradient(spike)
    assert tb[3, 4] == pytest.approx(-(2 + math.sqrt(2)), abs=1e-14)
    assert tb[3, 3] == 0.0 and tb[2, 4] == 0.0        # enter a flat term -> undefined -> 0
    assert tb[0, 0] == 0.0
    t, nrm = tv.nonascending(np.full((4, 4), 2.0))
    assert nrm == 0.0 and not t.any()


def test_neg_gradient_matches_finite_differences():
    rng = np.random.default_rng(7)
    y = rng.standard_normal((9, 11))
    tb = tv.neg_gradient(y)
    h = 1e-6
    fd = np.zeros_like(y)
    for i in range(9):
        for j in range(11):
            e = np.zeros_like(y)
            e[i, j] = h
            fd[i, j] = (tv.total_variation(y + e) - tv.total_variation(y - e)) / (2 * h)
    assert np.max(np.abs(-tb - fd)) <= 1e-6 * max(1.0, np.max(np.abs(fd)))


def test_nonascending_vector_is_nonascending():
    rng = np.random.default_rng(8)
    y = rng.standard_normal((12, 12))
    t, nrm = tv.nonascending(y)
    assert np.linalg.norm(t) == pytest.approx(1.0, abs=1e-14)
    base = tv.total_variation(y)
    for d in (1e-2, 1e-4, 1e-6):
        assert tv.total_variation(y + d * t) <= base
    # directional derivative along t is -||t_bar||
    d = 1e-7
    assert (tv.total_variation(y + d * t) - base) / d == pytest.approx(-nrm, rel=1e-4)


# ---- preconditioner (Section 3.2, eq. 3.2) ----------------------------------------

def test_window_values():
    assert precond.window(0.0, 1e-3, 0.6) == pytest.approx(1e-3)
    assert precond.window(math.pi, 0.0, 0.8) == pytest.approx(math.pi * 0.6)
    assert precond.window(-1.0, 0.1, 0.5) == pytest.approx(1.1 * (0.5 + 0.5 * math.cos(1.0)))


def test_pad_size():
    assert precond.pad_size(64, 64) == 128
    assert precond.pad_size(512, 512) == 1024
    assert precond.pad_size(243, 243) == 512
    assert precond.pad_size(2048, 2048) == 4096
    assert precond.pad_size(100, 30) == 256


@pytest.mark.parametrize("u,v", [(0, 0), (1, 0), (3, 5), (8, 8), (15, 2), (16, 0)])
def test_fourier_modes_are_eigenvectors(u, v):
    # P9: with no padding (P = side) a cosine mode is scaled by h(|omega|)
    P = 32
    i = np.arange(P)[:, None]
    j = np.arange(P)[None, :]
    mode = np.cos(2 * math.pi * (u * i + v * j) / P + 0.3)
    mu, rho = 1e-3, 0.7
    ou = 2 * math.pi * (u if u < P / 2 else u - P) / P
    ov = 2 * math.pi * (v if v < P / 2 else v - P) / P
    lam = (math.hypot(ou, ov) + mu) * (rho + (1 - rho) * math.cos(math.hypot(ou, ov)))
    out = precond.apply(mode, mu, rho, P=P)
    assert np.max(np.abs(out - lam * mode)) <= 1e-12


def test_precond_symmetric():
    rng = np.random.default_rng(4)
    u = rng.standard_normal((20, 13))
    v = rng.standard_normal((20, 13))
    a = np.sum(precond.apply(u, 1e-5, 0.8) * v)
    b = np.sum(u * precond.apply(v, 1e-5, 0.8))
    assert a == pytest.approx(b, rel=1e-12)


def test_precond_embedding_is_linear_convolution():
    # the zero-embedded product equals a direct (non-circular) convolution with the
    # kernel K = ifft2(D); check one output pixel by brute force
    rng = np.random.default_rng(9)
    g = rng.standard_normal((6, 5))
    mu, rho = 1e-3, 0.6
    P = precond.pad_size(6, 5)
    K = np.real(np.fft.ifft2(precond.diagonal(P, mu, rho)))
    z = precond.apply(g, mu, rho)
    for (i, j) in ((0, 0), (3, 2), (5, 4)):
        want = sum(g[a, b] * K[(i - a) % P, (j - b) % P] for a in range(6) for b in range(5))
        assert z[i, j] == pytest.approx(want, rel=1e-12, abs=1e-13)


def test_precond_definiteness_threshold():
    # P10: dense M on an 8 x 8 image is positive definite for rho > 1/2 and has a
    # negative eigenvalue for rho = 0.4 (the paper's grid value, A6)
    lam_ok = np.linalg.eigvalsh(precond.dense(8, 8, 1e-5, 0.6))
    assert lam_ok.min() > 0
    lam_ok2 = np.linalg.eigvalsh(precond.dense(8, 8, 1e-3, 0.8))
    assert lam_ok2.min() > 0
    lam_bad = np.linalg.eigvalsh(precond.dense(8, 8, 1e-5, 0.4))
    assert lam_bad.min() < 0
