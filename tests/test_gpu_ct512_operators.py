"""Whole-vector parity of R, R^T and the solvers' gradient R^T (R x - b) at
512x512, 720 angles, 725 bins (tests/golden/ct512_operators.npz, written by
tests/golden/make_ct512_operators.py from the oracle only), and on a ragged
geometry whose backprojection takes four pixels per lane with partial tiles.

Bar: 1e-5 relative L2 over the whole output vector."""
import os
import sys

import numpy as np
import pytest

from oracle import projector as oproj
from oracle.geometry import Geometry as OG
from tests._problems import rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "ct512_operators.npz")


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1807_10151_amd as sp_mod
    return sp_mod


@pytest.fixture(scope="module")
def gold():
    sys.path.insert(0, os.path.join(HERE, "golden"))
    from make_ct512_operators import inputs
    d = dict(np.load(GOLD))
    d["x_ell"], d["x_gauss"], d["y_gauss"] = inputs()
    d["b"] = np.load(os.path.join(HERE, "golden", "ct512_oracle.npz"))["b"]
    return d


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def test_ct512_project_whole_vector(sp, gold):
    g = sp.Geometry(512, 512, 720, 725)
    for name in ("ell", "gauss"):
        got = sp.sp_project(g, cuda(gold[f"x_{name}"])).cpu().numpy().ravel()
        e = rel_l2(got, gold[f"Rx_{name}"])
        print(f"R x_{name}: rel_l2 {e:.3e}", flush=True)
        assert e <= 1e-5


def test_ct512_backproject_whole_vector(sp, gold):
    g = sp.Geometry(512, 512, 720, 725)
    got = sp.sp_backproject(g, cuda(gold["y_gauss"])).cpu().numpy().ravel()
    e = rel_l2(got, gold["RTy_gauss"])
    print(f"R^T y_gauss: rel_l2 {e:.3e}", flush=True)
    assert e <= 1e-5


def test_ct512_gradient_float64_residual(sp, gold):
    # the solvers' form: R x - b kept in float64, R^T of the float64 sinogram
    g = sp.Geometry(512, 512, 720, 725)
    b = cuda(gold["b"])
    for name in ("ell", "gauss"):
        grad, f = sp.sp_gradient(g, cuda(gold[f"x_{name}"]), b)
        e = rel_l2(grad.cpu().numpy().ravel(), gold[f"grad_{name}"])
        print(f"R^T (R x_{name} - b): rel_l2 {e:.3e}", flush=True)
        assert e <= 1e-5
        r = gold[f"Rx_{name}"].astype(np.float64) - gold["b"].astype(np.float64).ravel()
        assert float(f.item()) == pytest.approx(float(r @ r), rel=1e-5)


# 522 x 520: 17 x 66 four-pixel tiles (4,488 waves, so R^T takes four pixels
# per lane); 520 = 16 * 32 + 8 leaves partial tiles on the right and 522 = 65 *
# 8 + 2 at the bottom.
RAGGED4 = OG(522, 520, 90, 741)


@pytest.fixture(scope="module")
def ragged_matrix():
    return oproj.matrix(RAGGED4, "closed")


def test_ragged_four_pixel_backprojection(sp, ragged_matrix):
    R, RT = ragged_matrix
    og = RAGGED4
    g = sp.Geometry(og.rows, og.cols, og.n_angles, og.n_bins)
    rng = np.random.default_rng(522)
    y = rng.standard_normal((og.n_angles, og.n_bins)).astype(np.float32)
    got = sp.sp_backproject(g, cuda(y)).cpu().numpy().ravel()
    want = RT @ y.astype(np.float64).ravel()
    e = rel_l2(got, want)
    print(f"ragged 522x520 R^T: rel_l2 {e:.3e}", flush=True)
    assert e <= 1e-5
    # the edge columns and rows that partial tiles cover
    got2 = got.reshape(og.rows, og.cols)
    want2 = want.reshape(og.rows, og.cols)
    assert rel_l2(got2[:, 512:], want2[:, 512:]) <= 1e-5
    assert rel_l2(got2[520:, :], want2[520:, :]) <= 1e-5
    x = rng.standard_normal((og.rows, og.cols)).astype(np.float32)
    gotR = sp.sp_project(g, cuda(x)).cpu().numpy().ravel()
    assert rel_l2(gotR, R @ x.astype(np.float64).ravel()) <= 1e-5
    # h^T p: adjoint identity through the GPU pair
    lhs = float(np.dot(gotR.astype(np.float64), y.astype(np.float64).ravel()))
    rhs = float(np.dot(x.astype(np.float64).ravel(), got.astype(np.float64)))
    assert abs(lhs - rhs) <= 1e-6 * abs(lhs)


def test_ragged_four_pixel_gradient(sp, ragged_matrix):
    R, RT = ragged_matrix
    og = RAGGED4
    g = sp.Geometry(og.rows, og.cols, og.n_angles, og.n_bins)
    from synth import random_ellipses
    img, rng = random_ellipses(og.rows, og.cols, 20, 4)
    b = (R @ img.ravel() + 0.01 * rng.standard_normal(og.m)).astype(np.float32)
    x = (0.9 * img).astype(np.float32)
    grad, _ = sp.sp_gradient(g, cuda(x), cuda(b.reshape(og.n_angles, og.n_bins)))
    want = RT @ (R @ x.astype(np.float64).ravel() - b.astype(np.float64))
    assert rel_l2(grad.cpu().numpy().ravel(), want) <= 1e-5
