"""GPU parity of the operators (R, R^T, M, TV, S_TV) against the CPU oracle.

Tolerance for R and R^T: 1e-5 relative L2 over the output (float32 data and
outputs against the float64 oracle).  Inputs are seeded; expected values come from the oracle.
"""
import math

import numpy as np
import pytest

from oracle import closed_form, siddon
from oracle import precond as oprecond
from oracle import projector as oproj
from oracle import suppcg as osup
from oracle import tv as otv
from oracle.geometry import Geometry as OG
from tests._problems import rel_l2, workload_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1807_10151_amd as sp_mod
    return sp_mod


def G(og):
    import paper_1807_10151_amd as spm
    return spm.Geometry(og.rows, og.cols, og.n_angles, og.n_bins, og.pixel, og.theta0, og.dtheta,
                        og.bin_spacing, og.bin_offset)


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


RAGGED = [
    OG(64, 64, 90, 91),                      # the small workload's geometry
    OG(37, 53, 45, 61),                      # ragged sizes, odd bins
    OG(50, 30, 24, 60),                      # even bins (half-integer rays)
    OG(16, 16, 8, 24, pixel=0.7, bin_spacing=0.5, bin_offset=0.13),
    OG(20, 24, 7, 33, theta0=0.1, dtheta=0.45),
    OG(1, 1, 4, 3),                          # single pixel
    OG(3, 70, 1, 5),                         # one angle, wide image
    OG(33, 33, 360, 47),                     # includes 45 and 135 degrees
    OG(200, 150, 30, 251),                   # larger, few angles
    OG(9, 300, 12, 301, theta0=0.3),         # thin, wide image
    OG(260, 240, 16, 360, dtheta=0.19),      # coarse angle steps
]


@pytest.mark.parametrize("og", RAGGED, ids=lambda g: f"{g.rows}x{g.cols}_{g.n_angles}x{g.n_bins}")
def test_project_matches_oracle(sp, og):
    rng = np.random.default_rng(og.rows * 1000 + og.n_angles)
    for x in (rng.standard_normal((og.rows, og.cols)), rng.uniform(0, 1, (og.rows, og.cols))):
        x32 = x.astype(np.float32)
        want = oproj.project(og, x32.astype(np.float64))
        got = sp.sp_project(G(og), cuda(x32)).cpu().numpy().ravel()
        assert rel_l2(got, want) <= 1e-5, rel_l2(got, want)


@pytest.mark.parametrize("og", RAGGED, ids=lambda g: f"{g.rows}x{g.cols}_{g.n_angles}x{g.n_bins}")
def test_backproject_matches_oracle(sp, og):
    rng = np.random.default_rng(og.cols * 7 + og.n_bins)
    y = rng.standard_normal((og.n_angles, og.n_bins)).astype(np.float32)
    want = oproj.backproject(og, y.astype(np.float64))
    got = sp.sp_backproject(G(og), cuda(y)).cpu().numpy().ravel()
    assert rel_l2(got, want) <= 1e-5, rel_l2(got, want)


def test_adjoint_identity_gpu(sp):
    og = OG(64, 64, 90, 91)
    rng = np.random.default_rng(1)
    x = cuda(rng.standard_normal((64, 64)))
    y = cuda(rng.standard_normal((90, 91)))
    Rx = sp.sp_project(G(og), x)
    RTy = sp.sp_backproject(G(og), y)
    lhs = float((Rx.double() * y.double()).sum())
    rhs = float((x.double() * RTy.double()).sum())
    assert abs(lhs - rhs) <= 1e-6 * abs(lhs)


def test_project_small64_phantom(sp):
    og, img, b = workload_problem("small64")
    want = oproj.project(og, img.astype(np.float64))
    got = sp.sp_project(G(og), cuda(img)).cpu().numpy().ravel()
    assert rel_l2(got, want) <= 1e-5


def test_project_ct512_sampled_rays(sp):
    # full-size 512^2 x 720 x 725 projection, checked on 400 rays computed one by
    # one by the oracle's crossing merge
    og = OG(512, 512, 720, 725)
    from synth import random_ellipses
    img, _ = random_ellipses(512, 512, 20, 1)
    img32 = img.astype(np.float32)
    got = sp.sp_project(G(og), cuda(img32)).cpu().numpy()
    rng = np.random.default_rng(17)
    aa = rng.integers(0, 720, 400)
    kk = rng.integers(0, 725, 400)
    aa[:4] = [0, 180, 360, 540]            # axis and diagonal angles
    want = np.array([siddon.ray_sum(og, img32.astype(np.float64).ravel(), int(a), int(k))
                     for a, k in zip(aa, kk)])
    assert rel_l2(got[aa, kk], want) <= 1e-5


@pytest.mark.parametrize("side,n_angles,n_bins", [(256, 360, 364), (384, 536, 545), (1536, 2152, 2174)])
def test_project_split_rays_sampled(sp, side, n_angles, n_bins):
    # geometries whose rays R sums in 4, 2 and 8 parts (an underfilled grid,
    # a nearly full one, an image of more than 2^21 pixels), on 300 rays
    # computed one by one by the oracle's crossing merge
    og = OG(side, side, n_angles, n_bins)
    from synth import random_ellipses
    img, _ = random_ellipses(side, side, 20, 3)
    img32 = img.astype(np.float32)
    got = sp.sp_project(G(og), cuda(img32)).cpu().numpy()
    rng = np.random.default_rng(side)
    aa = rng.integers(0, n_angles, 300)
    kk = rng.integers(0, n_bins, 300)
    aa[:2] = [0, n_angles // 2]
    kk[:2] = [n_bins // 2, n_bins // 2]
    want = np.array([siddon.ray_sum(og, img32.astype(np.float64).ravel(), int(a), int(k))
                     for a, k in zip(aa, kk)])
    assert rel_l2(got[aa, kk], want) <= 1e-5


def test_backproject_ct512_sampled_pixels(sp):
    og = OG(512, 512, 720, 725)
    rng = np.random.default_rng(23)
    y = rng.standard_normal((720, 725)).astype(np.float32)
    got = sp.sp_backproject(G(og), cuda(y)).cpu().numpy()
    pix = [(0, 0), (511, 511), (255, 256), (0, 511), (100, 37)] + \
          [tuple(rng.integers(0, 512, 2)) for _ in range(40)]
    yv = y.astype(np.float64).ravel()
    want = np.array([np.dot(closed_form.column(og, int(i), int(j))[1],
                            yv[closed_form.column(og, int(i), int(j))[0]]) for i, j in pix])
    gv = np.array([got[i, j] for i, j in pix])
    assert rel_l2(gv, want) <= 1e-5


@pytest.mark.parametrize("shape", [(64, 64), (37, 53), (5, 3), (128, 100)])
def test_precond_matches_oracle(sp, shape):
    og = OG(shape[0], shape[1], 4, 5)
    rng = np.random.default_rng(shape[0])
    gimg = rng.standard_normal(shape).astype(np.float32)
    for mu, rho in ((1e-5, 0.8), (1e-3, 0.6)):
        want = oprecond.apply(gimg.astype(np.float64), mu, rho)
        got = sp.sp_precond_apply(G(og), cuda(gimg), mu, rho).cpu().numpy()
        assert rel_l2(got, want) <= 1e-5, rel_l2(got, want)


def test_precond_rejects_indefinite(sp):
    og = OG(8, 8, 4, 5)
    with pytest.raises(sp.SupPCGError) as e:
        sp.sp_precond_apply(G(og), cuda(np.zeros((8, 8))), 1e-5, 0.4)
    assert e.value.code == 2


@pytest.mark.parametrize("shape", [(64, 64), (37, 53), (2, 2), (1, 9)])
def test_tv_value_and_gradient(sp, shape):
    og = OG(shape[0], shape[1], 4, 5)
    rng = np.random.default_rng(5)
    y = rng.standard_normal(shape).astype(np.float32)
    y[0, :2] = 1.0                                       # a flat spot (zero rule)
    if shape[0] > 1:
        y[1, 0] = 1.0
    tv = float(sp.sp_tv(G(og), cuda(y)).item())
    assert tv == pytest.approx(otv.total_variation(y.astype(np.float64)), rel=1e-12, abs=1e-12)
    tb, n2 = sp.sp_tv_grad(G(og), cuda(y))
    want = otv.neg_gradient(y.astype(np.float64))
    assert rel_l2(tb.cpu().numpy(), want) <= 1e-6 or np.linalg.norm(want) == 0
    assert (tb.cpu().numpy() == 0)[want == 0].all()


def test_tv_perturb_matches_algorithm1(sp):
    og, img, _ = workload_problem("small64")
    rng = np.random.default_rng(3)
    x = (img + 0.05 * rng.standard_normal(img.shape)).astype(np.float32)
    for K, a, gam, ell in ((1, 0.5, 0.5, 0), (3, 0.5, 8.0, 2), (4, 0.9, 3.0, 5)):
        p = osup.TVParams(K, a, gam)
        ref = osup.s_tv(x.astype(np.float64), ell, p)
        xh, ell_out, tvh, trials = sp.sp_tv_perturb(G(og), cuda(x), ell, K, a, gam)
        assert ell_out == ref.ell and trials == ref.trials
        want = x.astype(np.float64) + ref.s
        assert rel_l2(xh.cpu().numpy(), want) <= 1e-6
        assert tvh == pytest.approx(ref.tv_after, rel=1e-6)


def test_tv_perturb_trial_cap(sp):
    og = OG(8, 8, 4, 5)
    x = np.random.default_rng(2).standard_normal((8, 8)).astype(np.float32)
    xh, ell, tvh, trials = sp.sp_tv_perturb(G(og), cuda(x), 0, 1, 1 - 1e-12, 1e6, max_trials=20)
    assert ell == 20 and trials == [21]
    assert np.array_equal(xh.cpu().numpy(), x)


def test_invalid_geometry_rejected(sp):
    og = OG(0, 4, 4, 5)
    with pytest.raises(sp.SupPCGError) as e:
        sp.sp_project(G(og), cuda(np.zeros(0)), cuda(np.zeros((4, 5))))
    assert e.value.code == 1
