"""Pins of the learned-preconditioner oracle (CPU only)."""
import numpy as np
import pytest
import scipy.signal

from oracle import learned as ol


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 7, 9))
    W = rng.standard_normal((4, 3, 3, 3))
    y = ol.conv(x, W)
    for b in range(2):
        for o in range(4):
            want = sum(scipy.signal.correlate2d(x[b, i], W[o, i], mode="same", boundary="fill")
                       for i in range(3))
            assert np.max(np.abs(y[b, o] - want)) <= 1e-12


def _dense(fn, shape_in):
    n = int(np.prod(shape_in))
    cols = []
    for q in range(n):
        e = np.zeros(n)
        e[q] = 1.0
        cols.append(fn(e.reshape(shape_in)).ravel())
    return np.stack(cols, axis=1)


def test_conv_t_is_dense_transpose():
    rng = np.random.default_rng(1)
    W = rng.standard_normal((3, 2, 3, 3))
    C = _dense(lambda x: ol.conv(x, W), (1, 2, 4, 5))
    CT = _dense(lambda y: ol.conv_t(y, W), (1, 3, 4, 5))
    assert np.max(np.abs(C.T - CT)) <= 1e-12


def test_m_symmetric_psd():
    Ws, d = ol.init_params(layers=3, channels=4, seed=2)
    rng = np.random.default_rng(3)
    d = rng.standard_normal(4)
    M = _dense(lambda u: ol.apply(Ws, d, u), (6, 5))
    assert np.max(np.abs(M - M.T)) <= 1e-12 * np.max(np.abs(M))
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() >= -1e-10 * np.max(np.abs(M))


def test_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(4)
    Ws, d = ol.init_params(layers=3, channels=3, seed=5)
    d = d + 0.3 * rng.standard_normal(3)
    Av = rng.standard_normal((2, 6, 7))
    v = rng.standard_normal((2, 6, 7))
    loss, gW, gd = ol.loss_and_grad(Ws, d, Av, v)
    theta = ol.flatten(Ws, d)
    g = ol.flatten(gW, gd)
    h = 1e-6
    idx = rng.choice(theta.size, 40, replace=False)
    for q in idx:
        tp = theta.copy()
        tm = theta.copy()
        tp[q] += h
        tm[q] -= h
        lp = ol.loss_and_grad(*ol.unflatten(tp, 3, 3), Av, v)[0]
        lm = ol.loss_and_grad(*ol.unflatten(tm, 3, 3), Av, v)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[q]) <= 1e-6 * max(1.0, abs(fd)), (q, fd, g[q])
    # the loss is the documented quantity
    z = ol.apply(Ws, d, Av)
    want = np.mean([np.sum((z[b] - v[b]) ** 2) / np.sum(v[b] ** 2) for b in range(2)])
    assert loss == pytest.approx(want, rel=1e-13)


def test_margin_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(14)
    Ws, d = ol.init_params(layers=2, channels=3, seed=15)
    Av = rng.standard_normal((2, 9, 10))
    v = rng.standard_normal((2, 9, 10))
    loss, gW, gd = ol.loss_and_grad(Ws, d, Av, v, margin=2)
    g = ol.flatten(gW, gd)
    theta = ol.flatten(Ws, d)
    h = 1e-6
    for q in rng.choice(theta.size, 30, replace=False):
        tp = theta.copy()
        tm = theta.copy()
        tp[q] += h
        tm[q] -= h
        fd = (ol.loss_and_grad(*ol.unflatten(tp, 2, 3), Av, v, margin=2)[0] -
              ol.loss_and_grad(*ol.unflatten(tm, 2, 3), Av, v, margin=2)[0]) / (2 * h)
        assert abs(fd - g[q]) <= 1e-6 * max(1.0, abs(fd)), (q, fd, g[q])
    z = ol.apply(Ws, d, Av)
    want = np.mean([np.sum((z[b] - v[b])[2:7, 2:8] ** 2) / np.sum(v[b][2:7, 2:8] ** 2) for b in range(2)])
    assert loss == pytest.approx(want, rel=1e-13)


def test_crop_interior_equals_full_image():
    # M = C^T D C with L 3x3 layers reaches L pixels each way through C and L
    # through C^T: 2L in all.  On a crop whose interior keeps 2L pixels from the
    # crop's edges, M(crop) equals M(full image) on that interior, so the
    # margin-2L loss on crops is the full-size loss on those pixels.
    rng = np.random.default_rng(16)
    L = 3
    Ws, d = ol.init_params(layers=L, channels=4, seed=17)
    u = rng.standard_normal((40, 44))
    full = ol.apply(Ws, d, u)
    r0, c0, h, w = 9, 11, 20, 22
    crop = ol.apply(Ws, d, u[r0:r0 + h, c0:c0 + w])
    m = 2 * L
    np.testing.assert_allclose(crop[m:h - m, m:w - m], full[r0 + m:r0 + h - m, c0 + m:c0 + w - m],
                               rtol=0, atol=1e-12)
    # one pixel less of margin and the zero padding shows
    assert np.max(np.abs(crop[m - 1, m:w - m] - full[r0 + m - 1, c0 + m:c0 + w - m])) > 1e-6


def test_adam_first_step_is_signed_lr():
    p = [np.array([1.0, -2.0, 3.0])]
    g = [np.array([0.5, -4.0, 1e-3])]
    opt = ol.Adam(p, lr=1e-2)
    out = opt.step(p, g)
    np.testing.assert_allclose(out[0], p[0] - 1e-2 * np.sign(g[0]), rtol=0, atol=1e-7)


def test_softplus_and_init():
    assert ol.softplus(np.log(np.e - 1.0)) == pytest.approx(1.0, rel=1e-14)
    assert ol.softplus(50.0) == 50.0
    Ws, d = ol.init_params(4, 16, 0)
    assert [W.shape for W in Ws] == [(16, 1, 3, 3)] + [(16, 16, 3, 3)] * 3
    assert np.allclose(ol.softplus(d), 1.0)
