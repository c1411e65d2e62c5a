"""Pins of the oracle's projector R and its transpose (CPU only).

Each check compares the oracle against something other than itself: clipping a
line against a square, the whole-image chord, column sums at theta = 0, the
disk's analytic projection, and the two independent assemblies of R.
"""
import math

import numpy as np
import pytest

from oracle import closed_form, projector, siddon
from oracle.geometry import Geometry, angle_cos_sin, bin_positions, pixel_centres
from oracle.geometry import angle_table as angle_table_arrays


def clip_length(c, s, sk, x0, x1, y0, y1):
    """Length of the line x c + y s = sk inside [x0,x1] x [y0,y1], by clipping the
    parametric line P(tau) = sk (c, s) + tau (-s, c) against the four sides."""
    lo, hi = -math.inf, math.inf
    px, py = sk * c, sk * s
    for dirc, start, a, b in ((-s, px, x0, x1), (c, py, y0, y1)):
        if dirc == 0.0:
            if not (a <= start <= b):
                return 0.0
            continue
        t0, t1 = (a - start) / dirc, (b - start) / dirc
        lo, hi = max(lo, min(t0, t1)), min(hi, max(t0, t1))
    return max(0.0, hi - lo)


TINY = [Geometry(4, 5, 7, 9), Geometry(6, 6, 12, 11), Geometry(5, 3, 8, 8, pixel=0.7, bin_spacing=0.6),
        Geometry(6, 6, 10, 9, theta0=0.3, dtheta=0.29, bin_offset=0.21)]


def test_chord_weight_matches_square_clip():
    # P1: the closed-form chord equals clipping the line against one pixel square
    rng = np.random.default_rng(11)
    for _ in range(2000):
        th = rng.uniform(0, math.pi)
        c, s = math.cos(th), math.sin(th)
        p = rng.uniform(0.3, 2.0)
        d = rng.uniform(-1.2 * p, 1.2 * p)
        # pixel centred at (0.4, -0.3): line at signed distance d from the centre
        cx, cy = 0.4, -0.3
        sk = d + cx * c + cy * s
        want = clip_length(c, s, sk, cx - p / 2, cx + p / 2, cy - p / 2, cy + p / 2)
        got = float(closed_form.chord_weight(np.array([d]), c, s, p)[0])
        assert abs(got - want) <= 1e-12 * max(1.0, p)


def test_chord_weight_area_and_axis_ties():
    # the trapezoid integrates to the pixel area; axis lines on an edge give half
    for th in (0.1, 0.7, math.pi / 4, 1.3):
        c, s = abs(math.cos(th)), abs(math.sin(th))
        dd = np.linspace(-2, 2, 400001)
        area = np.trapezoid(closed_form.chord_weight(dd, c, s, 1.0), dd)
        assert abs(area - 1.0) < 1e-8
    w = closed_form.chord_weight(np.array([0.0, 0.5, -0.5, 0.5000001, 0.49]), 1.0, 0.0, 1.0)
    assert list(w) == [1.0, 0.5, 0.5, 0.0, 1.0]


@pytest.mark.parametrize("g", TINY)
def test_siddon_equals_closed_form_tiny(g):
    # P5: the two independent assemblies of R agree entry by entry
    Rs, _ = projector.matrix(g, "siddon")
    Rc, _ = projector.matrix(g, "closed")
    diff = abs(Rs - Rc)
    assert diff.max() <= 1e-12


def test_siddon_equals_closed_form_small64():
    g = Geometry(64, 64, 90, 91)
    Rs, _ = projector.matrix(g, "siddon")
    Rc, _ = projector.matrix(g, "closed")
    # lines through pixel corners leave rounding-level (1e-14) entries in one
    # assembly and none in the other; the entries above that level agree
    assert (Rs.data > 1e-12).sum() == (Rc.data > 1e-12).sum() == 477_832
    assert abs(Rs - Rc).max() <= 1e-12


def test_siddon_sampled_rays_ct512_match_closed_form():
    g = Geometry(512, 512, 720, 725)
    rng = np.random.default_rng(5)
    xs, ys = pixel_centres(g)
    sk = bin_positions(g)
    for _ in range(40):
        a, k = int(rng.integers(720)), int(rng.integers(725))
        idx, w = siddon.ray_weights(g, a, k)
        _, c, s = angle_cos_sin(g, a)
        i, j = idx // g.cols, idx % g.cols
        wc = closed_form.chord_weight(sk[k] - (xs[j] * c + ys[i] * s), c, s, 1.0)
        assert np.all(np.abs(wc - w) <= 1e-11)
        # and no pixel outside the Siddon set has a nonzero closed-form weight
        X, Y = np.meshgrid(xs, ys)
        wall = closed_form.chord_weight(sk[k] - (X * c + Y * s), c, s, 1.0).ravel()
        assert set(np.nonzero(wall > 1e-12)[0]) <= set(idx.tolist())


@pytest.mark.parametrize("g", TINY + [Geometry(64, 64, 90, 91)])
def test_all_ones_image_gives_rectangle_chords(g):
    # P2: every ray sum of the all-ones image is the chord through the image rectangle
    # (a line along the outer border counts half, reading G6)
    q = projector.project(g, np.ones(g.n))
    sk = bin_positions(g)
    want = []
    for a in range(g.n_angles):
        _, c, s = angle_cos_sin(g, a)
        for k in range(g.n_bins):
            w = siddon.chord_length_rectangle(g, a, k)
            if (s == 0.0 and abs(sk[k]) == g.cols * g.pixel / 2) or \
               (c == 0.0 and abs(sk[k]) == g.rows * g.pixel / 2):
                w *= 0.5
            want.append(w)
    assert np.max(np.abs(q - np.array(want))) <= 1e-12 * max(g.rows, g.cols)


def test_all_ones_chord_independent_clip():
    g = Geometry(7, 5, 13, 12, bin_offset=0.13)
    q = projector.project(g, np.ones(g.n))
    sk = bin_positions(g)
    for a in range(g.n_angles):
        _, c, s = angle_cos_sin(g, a)
        for k in range(g.n_bins):
            want = clip_length(c, s, sk[k], -2.5, 2.5, -3.5, 3.5)
            assert abs(q[a * g.n_bins + k] - want) <= 1e-12


def test_theta_zero_gives_column_sums_and_half_ties():
    # P3: at theta = 0 a ray between columns is a column sum; on a grid line the mean
    g = Geometry(6, 8, 4, 17, bin_spacing=0.5)
    rng = np.random.default_rng(2)
    img = rng.standard_normal((6, 8))
    q = projector.project(g, img).reshape(4, 17)
    xs, _ = pixel_centres(g)
    colsum = img.sum(axis=0)
    for k, s in enumerate(bin_positions(g)):
        on_line = abs((s + 4.0) - round(s + 4.0)) < 1e-12
        if abs(s) > 4.0:
            want = 0.0
        elif abs(s) == 4.0:
            want = 0.5 * colsum[0 if s < 0 else 7]
        elif on_line:
            jl = int(round(s + 4.0)) - 1
            want = 0.5 * (colsum[jl] + colsum[jl + 1])
        else:
            want = colsum[int(math.floor(s + 4.0))]
        assert abs(q[0, k] - want) <= 1e-12


def _disk_image(side, r, sub=8):
    off = (np.arange(sub) + 0.5) / sub - 0.5
    c = np.arange(side) - (side - 1) / 2.0
    X = c[None, :, None, None] + off[None, None, None, :]
    Y = ((side - 1) / 2.0 - np.arange(side))[:, None, None, None] + off[None, None, :, None]
    return ((X * X + Y * Y) <= r * r).mean(axis=(2, 3))


def test_centred_disk_matches_analytic_chord():
    # P4: R(disk) against 2 sqrt(r^2 - s^2); the pixelised disk is a discretisation,
    # so the error falls roughly as 1/r
    errs = []
    for r in (10, 20, 40):
        side = 2 * r + 8
        g = Geometry(side, side, 36, 2 * r + 11)
        q = projector.project(g, _disk_image(side, r), method="closed").reshape(36, -1)
        s = bin_positions(g)
        want = 2.0 * np.sqrt(np.maximum(0.0, r * r - s * s))
        err = np.linalg.norm(q - want[None, :]) / np.linalg.norm(np.broadcast_to(want, q.shape))
        errs.append(err)
        assert err <= 0.6 / r
    assert errs[1] < 0.7 * errs[0] and errs[2] < 0.7 * errs[1]


def test_adjoint_identity():
    # P7: <R x, y> = <x, R^T y>
    g = Geometry(64, 64, 90, 91)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(g.n)
    y = rng.standard_normal(g.m)
    lhs = projector.project(g, x) @ y
    rhs = x @ projector.backproject(g, y)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs) + 1e-9


def test_column_matches_matrix():
    g = Geometry(16, 12, 20, 21)
    R, _ = projector.matrix(g, "siddon")
    for (i, j) in ((0, 0), (7, 5), (15, 11)):
        rows, w = closed_form.column(g, i, j)
        col = R[:, i * g.cols + j].toarray().ravel()
        dense = np.zeros(g.m)
        dense[rows] = w
        assert np.max(np.abs(dense - col)) <= 1e-12


# ---- literal geometry (Section 4.1: equally spaced angles in [0, pi), parallel
# rays at a fixed spacing, centred on the rotation axis) ----

def test_angle_table_literal():
    _, c, s = angle_table_arrays(Geometry(3, 3, 4, 3))
    h = math.sqrt(0.5)
    assert list(c) == [1.0, h, 0.0, -h] and list(s) == [0.0, h, 1.0, h]
    th = [angle_cos_sin(Geometry(3, 3, 6, 3), a)[0] for a in range(6)]
    assert th[0] == 0.0
    assert np.allclose(np.diff(th), math.pi / 6, rtol=0, atol=1e-15)
    assert th[-1] + math.pi / 6 == pytest.approx(math.pi, abs=1e-15)     # [0, pi), pi excluded
    _, c6, s6 = angle_cos_sin(Geometry(3, 3, 6, 3), 1)
    assert c6 == pytest.approx(math.sqrt(3) / 2, abs=3e-16) and s6 == pytest.approx(0.5, abs=3e-16)


def test_bin_positions_literal():
    assert list(bin_positions(Geometry(2, 2, 1, 5))) == [-2.0, -1.0, 0.0, 1.0, 2.0]
    assert list(bin_positions(Geometry(2, 2, 1, 4))) == [-1.5, -0.5, 0.5, 1.5]
    s = bin_positions(Geometry(2, 2, 1, 4, bin_spacing=0.5, bin_offset=0.1))
    assert np.allclose(s, [-0.65, -0.15, 0.35, 0.85], rtol=0, atol=1e-16)
    # the paper's detector: 345 rays 0.0752 apart, the middle one through the axis
    s = bin_positions(Geometry(243, 243, 360, 345, pixel=0.0752, bin_spacing=0.0752))
    assert s[172] == 0.0 and s[0] == pytest.approx(-172 * 0.0752, abs=1e-13)


def test_tiny_matrix_literal():
    # 2 x 2 unit pixels (row 0 on top), angles 0 and pi/2, three bins at -1, 0, 1.
    # theta = 0: the lines x = -1, 0, 1 run along the left border, the middle
    # edge and the right border (each adjacent pixel gets half a pixel, G6);
    # theta = pi/2: y = -1, 0, 1 along the bottom border, the middle edge, the top.
    R, _ = projector.matrix(Geometry(2, 2, 2, 3), "siddon")
    want = np.array([
        [0.5, 0.0, 0.5, 0.0],     # x = -1: left column
        [0.5, 0.5, 0.5, 0.5],     # x = 0
        [0.0, 0.5, 0.0, 0.5],     # x = 1: right column
        [0.0, 0.0, 0.5, 0.5],     # y = -1: bottom row (row 1)
        [0.5, 0.5, 0.5, 0.5],     # y = 0
        [0.5, 0.5, 0.0, 0.0],     # y = 1: top row (row 0)
    ])
    assert np.array_equal(R.toarray(), want)
    # even bin count, even column count: the lines x = -1/2, 1/2 run through
    # the pixel centres and take each pixel of their column whole
    R, _ = projector.matrix(Geometry(3, 2, 1, 2), "siddon")
    assert np.array_equal(R.toarray(), [[1.0, 0.0, 1.0, 0.0, 1.0, 0.0],
                                        [0.0, 1.0, 0.0, 1.0, 0.0, 1.0]])
    # odd column count: the same lines now lie on the edges around the centre column
    R, _ = projector.matrix(Geometry(2, 3, 1, 2), "siddon")
    assert np.array_equal(R.toarray(), [[0.5, 0.5, 0.0, 0.5, 0.5, 0.0],
                                        [0.0, 0.5, 0.5, 0.0, 0.5, 0.5]])
    # 45 degrees through the centre of a single pixel: its diagonal
    R, _ = projector.matrix(Geometry(1, 1, 4, 1), "siddon")
    assert R.toarray()[1, 0] == pytest.approx(math.sqrt(2), abs=1e-15)
    assert R.toarray()[3, 0] == pytest.approx(math.sqrt(2), abs=1e-15)
