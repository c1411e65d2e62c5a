"""Pins of the ART / SupART oracle (Section 3.4, eq. (2.3)).

ART is pinned to the dense minimiser of the Bayesian criterion it is built
for, to the single-row projection property, to its ray order (rays of one
phase touch disjoint pixels, every ray once per cycle) and to the mean-gray
estimate on data whose integral is known; SupART to ART when its steps are 0
and to Algorithm 1's step schedule."""
import numpy as np
import pytest

from oracle import art, projector
from oracle.geometry import Geometry, angle_cos_sin
from oracle.suppcg import TVParams


def tiny(rows=6, cols=6, A=12, B=11, seed=0, **kw):
    g = Geometry(rows, cols, A, B, **kw)
    R, _ = projector.matrix(g)
    rng = np.random.default_rng(seed)
    x_true = rng.uniform(0.2, 1.0, g.n)
    b = R @ x_true + 0.05 * rng.standard_normal(g.m)
    return g, R, b


@pytest.mark.parametrize("r,lam", [(1.0, 1.0), (2.0, 0.5), (0.3, 1.5)])
def test_art_converges_to_the_bayesian_minimiser(r, lam):
    g, R, b = tiny()
    res = art.supart(g, R, b, r, lam, 3000)
    want = art.bayes_minimiser(R, b, r, res.trace["mu"])
    assert np.linalg.norm(res.x - want) <= 1e-7 * np.linalg.norm(want)


def test_art_limit_does_not_depend_on_the_order_of_phases():
    g, R, b = tiny(seed=3)
    mu = art.mean_gray(g, b)
    x1, u1 = np.full(g.n, mu), np.zeros(g.m)
    order = art.ray_order(g)
    rev = order[::-1]
    x2, u2 = x1.copy(), u1.copy()
    for _ in range(4000):
        art.art_sweep(R, b, x1, u1, 2.0, 1.0, order)
        art.art_sweep(R, b, x2, u2, 2.0, 1.0, rev)
    assert np.linalg.norm(x1 - x2) <= 1e-7 * np.linalg.norm(x1)


def test_one_step_with_unit_relaxation_solves_its_row():
    g, R, b = tiny(seed=1)
    R = R.tocsr()
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, g.n)
    u = rng.uniform(-1, 1, g.m)
    r = 3.0
    i = int(np.argmax(np.diff(R.indptr)))
    art.art_sweep(R, b, x, u, r, 1.0, [i])
    row = R.getrow(i)
    assert abs(r * (b[i] - float((row @ x)[0])) - u[i]) <= 1e-12 * (1 + abs(u[i]))


@pytest.mark.parametrize("geom", [dict(rows=16, cols=16, A=20, B=25),
                                  dict(rows=12, cols=20, A=9, B=40, bin_spacing=0.4),
                                  dict(rows=10, cols=10, A=7, B=17, pixel=0.7, bin_spacing=0.6, theta0=0.2)])
def test_ray_order_phases_touch_disjoint_pixels(geom):
    A, B = geom.pop("A"), geom.pop("B")
    g = Geometry(geom.pop("rows"), geom.pop("cols"), A, B, **geom)
    R, _ = projector.matrix(g)
    R = R.tocsr()
    order = art.ray_order(g)
    assert sorted(order) == list(range(g.m))        # every ray once
    for a in range(g.n_angles):
        q = art.phases(g, a)
        for ph in range(q):
            seen = set()
            for k in range(ph, g.n_bins, q):
                cols = set(R.indices[R.indptr[a * B + k]:R.indptr[a * B + k + 1]].tolist())
                assert not (cols & seen), (a, ph, k)
                seen |= cols
        # with one phase fewer, some angle of these geometries would overlap
        if q > 1:
            _, co, si = angle_cos_sin(g, a)
            e = g.pixel * 0.5 * (abs(co) + abs(si))
            assert (q - 1) * g.bin_spacing <= 2 * e + 1e-12


def test_phase_counts_by_hand():
    # unit pixels and bins: at 0 degrees e = 1/2 -> q = 2; at 45 degrees
    # e = sqrt(2)/2 -> 2e = 1.414 -> q = 2; bins of 0.4: q = floor(1/0.4) + 1 = 3
    # at 0 degrees and floor(1.414/0.4) + 1 = 4 at 45 degrees
    g = Geometry(8, 8, 4, 12)
    assert [art.phases(g, a) for a in range(4)] == [2, 2, 2, 2]
    h = Geometry(8, 8, 4, 30, bin_spacing=0.4)
    assert [art.phases(h, a) for a in range(4)] == [3, 4, 3, 4]


def test_mean_gray_of_a_centred_disk():
    # a disk of radius 20 and density 1 in a 64 x 64 image.  At 0 and 90
    # degrees every pixel's weights sum to pixel^2 / ds over the bins (a pixel
    # is one bin wide, split in halves on bin edges), so the data of each
    # angle integrate the image exactly and mu = disk area / n; at oblique
    # angles the sampled trapezoids sum to the area only on average
    ys, xs = np.mgrid[0:64, 0:64]
    img = (((xs - 31.5) ** 2 + (ys - 31.5) ** 2) <= 20.0 ** 2).astype(float)
    g = Geometry(64, 64, 2, 91)
    R, _ = projector.matrix(g)
    assert art.mean_gray(g, R @ img.ravel()) == pytest.approx(img.sum() / g.n, rel=1e-12)
    g = Geometry(64, 64, 16, 91)
    R, _ = projector.matrix(g)
    assert art.mean_gray(g, R @ img.ravel()) == pytest.approx(img.sum() / g.n, rel=1e-3)


def test_supart_with_zero_steps_is_art():
    g, R, b = tiny(seed=4)
    plain = art.supart(g, R, b, 5.0, 0.05, 6)
    # gamma = 0: every trial step is zero and is accepted (TV equal)
    sup0 = art.supart(g, R, b, 5.0, 0.05, 6, TVParams(3, 0.5, 0.0))
    assert np.array_equal(plain.x, sup0.x)
    assert sup0.trace["ell"] == [3 * (k + 1) for k in range(6)]


def test_supart_lowers_tv_against_art():
    from oracle import tv
    g, R, b = tiny(rows=16, cols=16, A=20, B=25, seed=5)
    plain = art.supart(g, R, b, 5.0, 0.05, 10)
    sup = art.supart(g, R, b, 5.0, 0.05, 10, TVParams(10, 1 - 1e-5, 1e-2))
    assert tv.total_variation(sup.x.reshape(16, 16)) < tv.total_variation(plain.x.reshape(16, 16))
