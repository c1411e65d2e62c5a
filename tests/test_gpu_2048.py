"""The 2048 x 2048, 2048-angle, 2899-bin geometry on the GPU: R and R^T on
rays and pixels the oracle computes one by one, the preconditioner (P = 4096)
against the oracle's FFT form, and a batch of 2048^2 slices against single
solves (bitwise)."""
import numpy as np
import pytest

from oracle import closed_form, siddon
from oracle import precond as oprecond
from oracle.geometry import Geometry as OG
from tests._problems import MU, RHO, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
SIDE, ANGLES, BINS = 2048, 2048, 2899


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1807_10151_amd as sp_mod
    return sp_mod


@pytest.fixture(scope="module")
def phantom():
    from synth import random_ellipses
    img, rng = random_ellipses(SIDE, SIDE, 50, 5000)
    return img.astype(np.float32), rng


def test_project_2048_sampled_rays(sp, phantom):
    img32, _ = phantom
    og = OG(SIDE, SIDE, ANGLES, BINS)
    got = sp.sp_project(sp.Geometry(SIDE, SIDE, ANGLES, BINS), torch.from_numpy(img32).cuda()).cpu().numpy()
    rng = np.random.default_rng(31)
    aa = rng.integers(0, ANGLES, 160)
    kk = rng.integers(BINS // 6, BINS - BINS // 6, 160)
    aa[:4] = [0, 512, 1024, 1536]          # axis and diagonal angles
    xv = img32.astype(np.float64).ravel()
    want = np.array([siddon.ray_sum(og, xv, int(a), int(k)) for a, k in zip(aa, kk)])
    assert rel_l2(got[aa, kk], want) <= 1e-5


def test_backproject_2048_sampled_pixels(sp):
    og = OG(SIDE, SIDE, ANGLES, BINS)
    rng = np.random.default_rng(37)
    y = rng.standard_normal((ANGLES, BINS)).astype(np.float32)
    got = sp.sp_backproject(sp.Geometry(SIDE, SIDE, ANGLES, BINS), torch.from_numpy(y).cuda()).cpu().numpy()
    pix = [(0, 0), (2047, 2047), (1023, 1024), (0, 2047)] + \
          [tuple(rng.integers(0, SIDE, 2)) for _ in range(12)]
    yv = y.astype(np.float64).ravel()
    want = []
    for i, j in pix:
        idx, w = closed_form.column(og, int(i), int(j))
        want.append(np.dot(w, yv[idx]))
    gv = np.array([got[i, j] for i, j in pix])
    assert rel_l2(gv, np.array(want)) <= 1e-5


def test_precond_2048(sp):
    rng = np.random.default_rng(41)
    gimg = rng.standard_normal((SIDE, SIDE)).astype(np.float32)
    want = oprecond.apply(gimg.astype(np.float64), MU, RHO)
    got = sp.sp_precond_apply(sp.Geometry(SIDE, SIDE, 4, 5), torch.from_numpy(gimg).cuda(), MU, RHO)
    assert rel_l2(got.cpu().numpy(), want) <= 1e-5


def test_batch_2048_equals_single(sp, phantom):
    img32, rng0 = phantom
    geoms = [sp.Geometry(SIDE, SIDE, ANGLES, BINS), sp.Geometry(SIDE, SIDE, ANGLES, BINS),
             sp.Geometry(512, 512, 720, 725)]
    bs = []
    for i, g in enumerate(geoms):
        if i == 0:
            x = torch.from_numpy(img32).cuda()
        else:
            x = torch.from_numpy(np.ascontiguousarray(img32[::4, ::4] if g.rows == 512 else img32.T)).cuda()
        b = sp.sp_project(g, x)
        noise = torch.from_numpy(np.random.default_rng(50 + i).standard_normal(g.m).astype(np.float32)).cuda()
        bs.append((b + 0.005 * float(b.max()) * noise.reshape(b.shape)).contiguous())
    kw = dict(K=1, a=0.5, gamma=0.5, mu=MU, rho=RHO, max_iter=3)
    got = sp.sp_suppcg_solve_batched(geoms, bs, graph=True, **kw)
    for i, g in enumerate(geoms):
        rs = sp.sp_suppcg_solve(g, bs[i], None, graph=True, **kw)
        assert got[i].k == rs.k == 4
        np.testing.assert_array_equal(got[i].x_half.cpu().numpy(), rs.x_half.cpu().numpy())
        np.testing.assert_array_equal(got[i].trace["f_half"], rs.trace["f_half"])
        np.testing.assert_array_equal(got[i].trace["ell"], rs.trace["ell"])
