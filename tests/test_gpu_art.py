"""GPU parity of ART and SupART (Section 3.4, eq. (2.3)) against the oracle.

Bars: the image after a fixed number of cycles within 1e-5 relative L2 of
the float64 oracle (both iterate in float64; the sums differ in order and the
weights in rounding only), identical l and trials traces for SupART, and the
per-iterate selective error within C 1e-5 ||x_k||.  The GPU projects the
rays of one phase of an angle concurrently; the oracle takes them one after
another in the same order, which the phases make equivalent."""
import numpy as np
import pytest

from oracle import art as oart
from oracle import projector as oproj
from oracle import quality as oq
from oracle.geometry import Geometry as OG
from oracle.suppcg import TVParams
from tests._problems import rel_l2, workload_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1807_10151_amd as sp_mod
    return sp_mod


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def sp_geom(sp, og):
    return sp.Geometry(og.rows, og.cols, og.n_angles, og.n_bins, pixel=og.pixel, theta0=og.theta0,
                       dtheta=og.dtheta, bin_spacing=og.bin_spacing, bin_offset=og.bin_offset)


@pytest.fixture(scope="module")
def small():
    og, img, b = workload_problem("small64")
    R, _ = oproj.matrix(og)
    return og, img, b, R


def test_art_table1_matches_oracle(sp, small):
    og, img, b, R = small
    print("ART 64x64x90x91 r=5 lambda=0.01, 4 cycles", flush=True)
    want = oart.supart(og, R, b.astype(np.float64), 5.0, 1e-2, 4)
    got = sp.sp_supart_solve(sp_geom(sp, og), cuda(b), K=0, r=5.0, lam=1e-2, max_iter=4)
    e = rel_l2(got.x.cpu().numpy(), want.x)
    print(f"ART rel_l2 {e:.3e}", flush=True)
    assert e <= 1e-5


def test_supart_table1_matches_oracle(sp, small):
    og, img, b, R = small
    print("SupART 64x64x90x91 (10, 1-1e-5, 1e-2, 5, 5e-2), 3 cycles", flush=True)
    tvp = TVParams(10, 1 - 1e-5, 1e-2)
    want = oart.supart(og, R, b.astype(np.float64), 5.0, 5e-2, 3, tvp)
    got = sp.sp_supart_solve(sp_geom(sp, og), cuda(b), K=10, a=1 - 1e-5, gamma=1e-2, r=5.0, lam=5e-2, max_iter=3)
    assert list(got.trace["ell"]) == want.trace["ell"]
    e = rel_l2(got.x.cpu().numpy(), want.x)
    print(f"SupART rel_l2 {e:.3e}", flush=True)
    assert e <= 1e-5


@pytest.fixture(scope="module")
def paper243():
    """The paper's shape (Section 4.1: 243^2 pixels, 360 angles, 345 bins):
    20 random ellipses (seed 3), 1% noise, the oracle's closed-form R."""
    from synth import noisy_data, random_ellipses, unit_noise
    og = OG(243, 243, 360, 345)
    img, rng = random_ellipses(243, 243, 20, 3)
    R, _ = oproj.matrix(og)
    b = noisy_data(R @ img.astype(np.float64).ravel(), unit_noise(rng, og.m), 0.01).astype(np.float32)
    return og, img, b.reshape(og.n_angles, og.n_bins), R


def test_art_and_supart_paper_shape(sp, paper243):
    og, img, b, R = paper243
    g = sp_geom(sp, og)
    print("ART 243x243x360x345 r=5 lambda=0.01, 2 cycles", flush=True)
    want = oart.supart(og, R, b.astype(np.float64), 5.0, 1e-2, 2)
    got = sp.sp_supart_solve(g, cuda(b), K=0, r=5.0, lam=1e-2, max_iter=2)
    e = rel_l2(got.x.cpu().numpy(), want.x)
    print(f"ART rel_l2 {e:.3e}", flush=True)
    assert e <= 1e-5
    print("SupART 243x243x360x345 (10, 1-1e-5, 1e-2, 5, 5e-2), 2 cycles", flush=True)
    tvp = TVParams(10, 1 - 1e-5, 1e-2)
    want = oart.supart(og, R, b.astype(np.float64), 5.0, 5e-2, 2, tvp)
    got = sp.sp_supart_solve(g, cuda(b), K=10, a=1 - 1e-5, gamma=1e-2, r=5.0, lam=5e-2, max_iter=2)
    assert list(got.trace["ell"]) == want.trace["ell"]
    e = rel_l2(got.x.cpu().numpy(), want.x)
    print(f"SupART rel_l2 {e:.3e}", flush=True)
    assert e <= 1e-5


@pytest.mark.parametrize("og", [OG(37, 53, 45, 61, bin_spacing=0.45),
                                OG(20, 24, 7, 33, pixel=0.7, theta0=0.1, dtheta=0.45, bin_spacing=0.6,
                                   bin_offset=0.13),
                                OG(41, 57, 4, 75, theta0=1e-7, dtheta=np.pi / 2)],
                         ids=["37x53-ds0.45", "20x24-pixel0.7", "41x57-near-axis"])
def test_art_ragged_geometries(sp, og):
    print(f"ART {og}", flush=True)
    R, _ = oproj.matrix(og)
    rng = np.random.default_rng(og.n)
    x_true = rng.uniform(0.1, 1.0, og.n)
    b = (R @ x_true + 0.02 * rng.standard_normal(og.m)).astype(np.float32)
    want = oart.supart(og, R, b.astype(np.float64), 2.0, 0.5, 3)
    got = sp.sp_supart_solve(sp_geom(sp, og), cuda(b.reshape(og.n_angles, og.n_bins)), K=0, r=2.0, lam=0.5,
                             max_iter=3)
    assert rel_l2(got.x.cpu().numpy(), want.x) <= 1e-5


def test_art_graph_equals_eager_and_x0(sp, small):
    og, img, b, R = small
    g = sp_geom(sp, og)
    kw = dict(K=2, a=0.5, gamma=0.5, r=5.0, lam=0.05, max_iter=3)
    a = sp.sp_supart_solve(g, cuda(b), graph=True, **kw)
    e = sp.sp_supart_solve(g, cuda(b), graph=False, **kw)
    assert torch.equal(a.x, e.x)
    assert list(a.trace["ell"]) == list(e.trace["ell"])
    x0 = np.full((og.rows, og.cols), 0.3, dtype=np.float32)
    got = sp.sp_supart_solve(g, cuda(b), cuda(x0), K=0, r=5.0, lam=0.05, max_iter=2)
    want = oart.supart(og, R, b.astype(np.float64), 5.0, 0.05, 2, x0=x0.ravel())
    assert rel_l2(got.x.cpu().numpy(), want.x) <= 1e-5


def test_art_se_curve(sp, small):
    og, img, b, R = small
    axes = oq.paper_axes(og)
    want = oart.supart(og, R, b.astype(np.float64), 5.0, 1e-2, 3, record=True)
    got = sp.sp_supart_solve(sp_geom(sp, og), cuda(b), K=0, r=5.0, lam=1e-2, max_iter=3, se_ref=cuda(img),
                             timing=True)
    mu = want.trace["mu"]
    iterates = [np.full(og.n, mu)] + want.trace["x"]
    C = 1.0 / np.sqrt(np.sum(img.astype(np.float64)[oq.ellipse_mask(og, axes)] ** 2))
    se = got.trace["se"]
    assert len(se) == 4
    for k, xk in enumerate(iterates):
        assert abs(se[k] - oq.selective_error(og, xk, img, axes)) <= C * 1e-5 * np.linalg.norm(xk)
    t = got.trace["t_ms"]
    assert t[0] == 0.0 and np.all(np.diff(t) > 0.0)


def test_art_rejects_bad_parameters(sp, small):
    og, img, b, R = small
    g = sp_geom(sp, og)
    for kw in (dict(lam=2.0), dict(lam=0.0), dict(r=0.0), dict(r=float("nan"))):
        with pytest.raises(sp.SupPCGError):
            sp.sp_supart_solve(g, cuda(b), max_iter=1, **kw)
