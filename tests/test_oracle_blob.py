"""Pins of the BlobART oracle (Section 3.4, blob basis).

The blob's projection is checked against numerical quadrature of the blob
along lines (scipy.integrate.quad, an independent route to the same line
integral) and against the blob's volume; the synthesis against the blob's
values; BlobART against the dense minimiser of the Bayesian criterion in
coefficient space; its ray phases against the matrix's supports."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import art, blob
from oracle.geometry import Geometry


@pytest.mark.parametrize("d", [0.0, 0.3, 1.0, 1.7, 1.99, -1.2])
def test_projection_is_the_line_integral(d):
    a = blob.RADIUS
    L = math.sqrt(max(a * a - d * d, 0.0))
    want, err = quad(lambda t: float(blob.blob(math.hypot(d, t))), -L, L, epsabs=1e-13, epsrel=1e-12, limit=200)
    assert float(blob.blob_projection(d)) == pytest.approx(want, rel=1e-9, abs=1e-12)


def test_projection_integrates_to_the_blob_volume():
    a = blob.RADIUS
    vol, _ = quad(lambda r: 2 * math.pi * r * float(blob.blob(r)), 0, a, epsabs=1e-13, epsrel=1e-12)
    tot, _ = quad(lambda d: float(blob.blob_projection(d)), -a, a, epsabs=1e-13, epsrel=1e-12)
    assert tot == pytest.approx(vol, rel=1e-9)


def test_blob_values_at_centre_and_edge():
    assert float(blob.blob(0.0)) == pytest.approx(1.0, abs=1e-15)
    assert float(blob.blob(blob.RADIUS)) == 0.0 and float(blob.blob(2.5)) == 0.0
    assert float(blob.blob_projection(blob.RADIUS)) == 0.0
    assert float(blob.blob_projection(0.7)) == float(blob.blob_projection(-0.7))


def test_synthesis_of_an_impulse_and_a_constant_field():
    g = Geometry(11, 13, 1, 1)
    c = np.zeros(g.n)
    c[5 * 13 + 6] = 1.0
    img = blob.synthesize(g, c).reshape(11, 13)
    for di in range(-2, 3):
        for dj in range(-2, 3):
            assert img[5 + di, 6 + dj] == pytest.approx(float(blob.blob(math.hypot(di, dj))), abs=1e-15)
    assert img.sum() == pytest.approx(blob.grid_sum(), rel=1e-14)
    const = blob.synthesize(g, np.full(g.n, 0.5)).reshape(11, 13)
    assert np.allclose(const[2:-2, 2:-2], 0.5 * blob.grid_sum(), rtol=1e-14)


def test_blob_art_converges_to_the_bayesian_minimiser():
    g = Geometry(6, 6, 12, 13)
    Rb = blob.system_matrix(g)
    rng = np.random.default_rng(0)
    b = Rb @ rng.uniform(0.2, 1.0, g.n) + 0.02 * rng.standard_normal(g.m)
    c, img, tr = blob.blob_art(g, Rb, b, 1.0, 1.0, 3000)
    want = art.bayes_minimiser(Rb, b, 1.0, tr["c_mu"])
    assert np.linalg.norm(c - want) <= 1e-7 * np.linalg.norm(want)


@pytest.mark.parametrize("geom", [dict(rows=12, cols=12, A=9, B=25),
                                  dict(rows=10, cols=14, A=5, B=40, bin_spacing=0.6, pixel=0.8)])
def test_blob_phases_touch_disjoint_blobs(geom):
    A, B = geom.pop("A"), geom.pop("B")
    g = Geometry(geom.pop("rows"), geom.pop("cols"), A, B, **geom)
    Rb = blob.system_matrix(g).tocsr()
    q = blob.phases(g)
    assert sorted(blob.ray_order(g)) == list(range(g.m))
    for ai in range(A):
        for ph in range(q):
            seen = set()
            for k in range(ph, B, q):
                i = ai * B + k
                cols = set(Rb.indices[Rb.indptr[i]:Rb.indptr[i + 1]].tolist())
                assert not (cols & seen)
                seen |= cols


def test_blob_matrix_matches_its_definition():
    # one ray through the middle of a 7 x 7 grid at 0 degrees: blobs on the
    # central column are at distance 0, the neighbours at 1 and 2 (no weight)
    g = Geometry(7, 7, 1, 3)
    Rb = blob.system_matrix(g).toarray()
    row = Rb[1].reshape(7, 7)
    assert np.allclose(row[:, 3], float(blob.blob_projection(0.0)), rtol=1e-15)
    assert np.allclose(row[:, 2], float(blob.blob_projection(1.0)), rtol=1e-15)
    assert np.all(row[:, [0, 1, 5, 6]] == 0.0)
