"""Pins of the selective error (Section 4.2, eq. (4.1)) in the oracle.

The ellipse set S is checked against lattice-point counts that do not come from
the oracle's formula (Gauss's circle problem, hand counts on half-integer
lattices), its orientation against a hand-drawn ellipse, and SE against
invariants that fix C, the mask and the square root."""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import quality
from oracle.geometry import Geometry


# Number of integer points (x, y) with x^2 + y^2 <= r^2 (Gauss's circle
# problem; OEIS A000328), r = 0 .. 10.
GAUSS_CIRCLE = [1, 5, 13, 29, 49, 81, 113, 149, 197, 253, 317]


@pytest.mark.parametrize("r", range(1, 11))
def test_circle_on_odd_grid_counts_lattice_points(r):
    # odd image: pixel centres are the integer lattice around the origin
    g = Geometry(25, 25, 1, 1)
    assert int(quality.ellipse_mask(g, (r, r)).sum()) == GAUSS_CIRCLE[r]


def test_circle_on_even_grid_counts_half_integer_points():
    # even image: centres at (+-1/2, +-1/2), (+-1/2, +-3/2), ...
    g = Geometry(8, 8, 1, 1)
    assert int(quality.ellipse_mask(g, (1.0, 1.0)).sum()) == 4      # only the four (+-1/2, +-1/2)
    # r = 2: 1/2^2+1/2^2 = 0.5, 1/2^2+3/2^2 = 2.5 (8 points), 3/2^2+3/2^2 = 4.5 > 4
    assert int(quality.ellipse_mask(g, (2.0, 2.0)).sum()) == 12


def test_horizontal_axis_runs_along_a_row():
    g = Geometry(9, 11, 1, 1)
    m = quality.ellipse_mask(g, (3.0, 1.0))        # wide, flat ellipse
    want = np.zeros((9, 11), dtype=bool)
    want[4, 2:9] = True                             # centre row: x = -3 .. 3
    want[3, 5] = want[5, 5] = True                  # y = +-1 at x = 0 only
    np.testing.assert_array_equal(m, want)
    mt = quality.ellipse_mask(g, (1.0, 3.0))        # tall ellipse
    assert mt[:, 5].sum() == 7 and mt[4].sum() == 3


def test_pixel_size_scales_the_set():
    a = quality.ellipse_mask(Geometry(31, 31, 1, 1), (7.0, 11.0))
    b = quality.ellipse_mask(Geometry(31, 31, 1, 1, pixel=0.5), (3.5, 5.5))
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("ah,av", [(40.0, 56.0), (93.1, 66.5), (120.0, 120.0)])
def test_area_within_perimeter_bound(ah, av):
    g = Geometry(257, 257, 1, 1)
    cnt = int(quality.ellipse_mask(g, (ah, av)).sum())
    # a unit cell whose centre is counted but which crosses the boundary lies
    # within a band of width sqrt(2) around the boundary
    perim = math.pi * (3 * (ah + av) - math.sqrt((3 * ah + av) * (ah + 3 * av)))
    assert abs(cnt - math.pi * ah * av) <= math.sqrt(2) * perim


def test_se_invariants():
    rng = np.random.default_rng(5)
    g = Geometry(21, 17, 1, 1)
    ref = rng.uniform(0.1, 1.0, (21, 17))
    axes = (6.0, 8.0)
    m = quality.ellipse_mask(g, axes)
    assert quality.selective_error(g, ref, ref, axes) == 0.0
    # default C makes SE(0) = 1
    assert abs(quality.selective_error(g, np.zeros_like(ref), ref, axes) - 1.0) < 1e-14
    # a constant offset c inside S: SE = C |c| sqrt(|S|)
    c = 0.3
    x = ref + c
    assert abs(quality.selective_error(g, x, ref, axes, C=2.0) - 2.0 * c * math.sqrt(m.sum())) < 1e-12
    # changes outside S do not count
    y = ref.copy()
    y[~m] += 5.0
    assert quality.selective_error(g, y, ref, axes, C=1.0) == 0.0
    # one pixel inside S off by d: SE = C |d|
    z = ref.copy()
    z[10, 8] -= 0.25
    assert m[10, 8]
    assert abs(quality.selective_error(g, z, ref, axes, C=3.0) - 0.75) < 1e-15


def test_paper_axes_reproduce_the_paper_ellipse():
    # on the paper's own grid (243 pixels of 0.0752 cm) the axes are 5 and 7 cm
    g = Geometry(243, 243, 1, 1, pixel=0.0752)
    ah, av = quality.paper_axes(g)
    assert abs(ah - 5.0) < 1e-12 and abs(av - 7.0) < 1e-12
    # ... and on a 512 grid of unit pixels they keep their share of the width
    ah, av = quality.paper_axes(Geometry(512, 512, 1, 1))
    assert abs(ah / 512 - 5.0 / (243 * 0.0752)) < 1e-15
    assert abs(av / ah - 1.4) < 1e-12


def test_se_curve_of_cg_on_exact_data_reaches_zero():
    # consistent data of a full-rank tiny system: CG on the normal equations
    # recovers the phantom, so the curve starts at SE(0) = 1 and ends near 0
    from oracle import projector, suppcg
    g = Geometry(6, 6, 24, 12)
    R, _ = projector.matrix(g)
    rng = np.random.default_rng(3)
    ref = rng.uniform(0.2, 1.0, (6, 6))
    b = R @ ref.ravel()
    prob = suppcg.Problem(R, b, (6, 6), None)
    axes = (2.5, 2.5)
    curve, res = quality.se_curve(g, prob, np.zeros(36), None, 80, ref, axes)
    assert curve[0] == pytest.approx(1.0, abs=1e-15)
    assert len(curve) == len(res.trace["x"]) + 1
    assert curve[-1] < 1e-6
